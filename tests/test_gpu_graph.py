"""A single-mesh voxelize call and the grid consumers enqueue kernels only,
so they can be captured in a HIP graph (through torch's graph capture) and
replayed: every replay, with eager work and synchronizations in between,
must give the eager result."""
import numpy as np
import pytest

from paper_2106_01326_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("strict", [False, True])
def test_voxelize_graph_replays(oracle_mod, strict):
    import torch

    import paper_2106_01326_amd as tv

    m = synth.make_mesh(24, 0.4, 128, "ellipsoids", 4, 8001)
    want = oracle_mod.voxelize_mesh(m, mode=oracle_mod.STRICT if strict else oracle_mod.HALF_OPEN)
    v = torch.from_numpy(m.verts).cuda()
    t = torch.from_numpy(m.tets).cuda()
    grid = tv.alloc_grid(m.dims)
    ws = tv.alloc_workspace(tv.workspace_bytes(m.nv, m.nt, m.dims))
    tv.voxelize(v, t, m.dims, m.bbox, strict=strict, grid=grid, workspace=ws)  # eager warm-up
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        tv.voxelize(v, t, m.dims, m.bbox, strict=strict, grid=grid, workspace=ws)
    for r in range(4):
        grid.fill_(-1)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(grid.cpu().numpy().view(np.uint32), want), f"replay {r}"
        assert tv.fetch_status(ws) == tv.TV_OK


def test_unpack_graph_replays():
    import torch

    import oracle.grids as G
    import paper_2106_01326_amd as tv

    dims = (16, 16, 64)
    rng = np.random.default_rng(8002)
    words = G.pack(rng.random(dims) < 0.3)
    grid = torch.from_numpy(words.view(np.int32)).cuda()
    out = torch.empty(dims, dtype=torch.uint8, device="cuda")
    tv.unpack(grid, dims, out=out)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        tv.unpack(grid, dims, out=out)
    for r in range(4):
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), G.unpack(words, dims)), f"replay {r}"


def test_prepared_batch_graph_replays(oracle_mod):
    """tv_batch_run enqueues kernels only: a captured run replays to the
    oracle's grids for every mesh, with eager work between replays."""
    import torch

    import paper_2106_01326_amd as tv

    ms = synth.workload_batch(first=16, workers=1)
    ms.append(synth.make_mesh(24, 0.3, 128, "ellipsoids", 3, 8003))
    want = [oracle_mod.voxelize_mesh(m) for m in ms]
    items = [(torch.from_numpy(m.verts).cuda(), torch.from_numpy(m.tets).cuda(), m.dims, m.bbox, False)
             for m in ms]
    b = tv.Batch(items)
    b.prepare()
    b.run_prepared()  # eager warm-up
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run_prepared()
    for r in range(4):
        for grid in b.grids:
            grid.fill_(-1)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, grid in enumerate(b.grids):
            assert np.array_equal(grid.cpu().numpy().view(np.uint32), want[i]), f"replay {r} mesh {i}"
            assert b.status(i) == tv.TV_OK
