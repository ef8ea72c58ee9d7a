"""Parity of the grid consumers (tv_unpack, tv_pool, tv_bricks) with the
numpy oracle, bit for bit / value for value, through the C ABI."""
import numpy as np
import pytest

from paper_2106_01326_amd import synth

pytestmark = pytest.mark.gpu


def banner(msg):
    print(f"[case] {msg}", flush=True)


def rand_words(rng, dims, density):
    """Random grid words with zero padding bits."""
    import oracle.grids as G

    return G.pack(rng.random(dims) < density)


def dev_words(w):
    import torch

    return torch.from_numpy(np.ascontiguousarray(w).view(np.int32)).cuda()


DIMS = [(1, 1, 1), (2, 4, 8), (4, 2, 16), (8, 8, 32), (4, 8, 64), (16, 8, 128), (2, 2, 1024),
        (64, 32, 4), (32, 64, 2)]


@pytest.mark.parametrize("dims", DIMS)
def test_unpack(dims):
    import torch

    import oracle.grids as G
    import paper_2106_01326_amd as tv

    banner(f"unpack {dims}")
    rng = np.random.default_rng(sum(dims))
    w = rand_words(rng, dims, 0.4)
    want = G.unpack(w, dims)
    g = dev_words(w)
    u8 = tv.unpack(g, dims)
    f32 = tv.unpack(g, dims, dtype=torch.float32)
    torch.cuda.synchronize()
    assert np.array_equal(u8.cpu().numpy(), want)
    assert np.array_equal(f32.cpu().numpy(), want.astype(np.float32))
    # an output that is not 16-byte aligned takes the per-voxel path
    n = int(np.prod(dims))
    raw = torch.zeros(n + 1, dtype=torch.uint8, device="cuda")
    tv.unpack(g, dims, out=raw[1:])
    assert np.array_equal(raw[1:].cpu().numpy().reshape(dims), want) and int(raw[0]) == 0


def test_unpack_voxelized_mesh(oracle_mod):
    import torch

    import oracle.grids as G
    import paper_2106_01326_amd as tv

    m = synth.make_mesh(16, 0.3, 64, "ellipsoids", 3, 2001)
    banner("unpack of a voxelized mesh")
    v = torch.from_numpy(m.verts).cuda()
    t = torch.from_numpy(m.tets).cuda()
    grid, _ = tv.voxelize(v, t, m.dims, m.bbox)
    dense = tv.unpack(grid, m.dims, dtype=torch.float32)
    want = G.unpack(oracle_mod.voxelize_mesh(m), m.dims)
    assert np.array_equal(dense.cpu().numpy(), want.astype(np.float32))


POOL = [((8, 8, 32), 2), ((8, 8, 32), 8), ((16, 16, 64), 4), ((4, 4, 8), 2), ((32, 32, 32), 32),
        ((64, 32, 16), 16), ((8, 16, 1024), 2), ((8, 8, 2048), 8), ((4, 4, 4), 4)]


@pytest.mark.parametrize("dims,f", POOL)
def test_pool(dims, f):
    import torch

    import oracle.grids as G
    import paper_2106_01326_amd as tv

    banner(f"pool {dims} / {f}")
    rng = np.random.default_rng(f + sum(dims))
    for density in (0.02, 0.5):
        w = rand_words(rng, dims, density)
        g = dev_words(w)
        frac = tv.pool(g, dims, f, tv.POOL_FRACTION)
        anyg = tv.pool(g, dims, f, tv.POOL_ANY)
        torch.cuda.synchronize()
        assert np.array_equal(frac.cpu().numpy().astype(np.float64), G.pool_fraction(w, dims, f))
        assert np.array_equal(anyg.cpu().numpy().view(np.uint32), G.pool_any(w, dims, f))


def test_pool_rejects_bad_factor():
    import paper_2106_01326_amd as tv

    g = dev_words(np.zeros(8 * 8, dtype=np.uint32))
    for f in (1, 3, 64, 16):
        with pytest.raises(tv.TVError):
            tv.pool(g, (8, 8, 8), f)


BRICKS = [(8, 8, 32), (16, 8, 64), (32, 16, 128), (8, 32, 32)]


@pytest.mark.parametrize("dims", BRICKS)
def test_bricks(dims):
    import oracle.grids as G
    import paper_2106_01326_amd as tv

    banner(f"bricks {dims}")
    rng = np.random.default_rng(7 + sum(dims))
    for density in (0.0, 0.0005, 0.01, 0.5):
        w = rand_words(rng, dims, density)
        want_ids, want_words = G.bricks(w, dims)
        ids, bw, n = tv.bricks(dev_words(w), dims)
        assert n == len(want_ids)
        assert np.array_equal(ids.cpu().numpy().view(np.uint32), want_ids)
        assert np.array_equal(bw.cpu().numpy().view(np.uint32), want_words)
        if n > 1:
            # a capacity below the count keeps the first bricks and still counts all
            ids2, bw2, n2 = tv.bricks(dev_words(w), dims, capacity=n // 2)
            assert n2 == n and len(ids2) == n // 2
            assert np.array_equal(ids2.cpu().numpy().view(np.uint32), want_ids[: n // 2])
            assert np.array_equal(bw2.cpu().numpy().view(np.uint32), want_words[: n // 2])


def test_bricks_of_large_mesh_grid(oracle_mod):
    """Bricks of a voxelized 256^3 mesh reproduce the grid exactly."""
    import torch

    import oracle.grids as G
    import paper_2106_01326_amd as tv

    m = synth.make_mesh(32, 0.3, 256, "ellipsoids", 3, 2002)
    banner("bricks of a 256^3 mesh grid")
    grid, _ = tv.voxelize(torch.from_numpy(m.verts).cuda(), torch.from_numpy(m.tets).cuda(), m.dims, m.bbox)
    words = grid.cpu().numpy().view(np.uint32)
    ids, bw, n = tv.bricks(grid, m.dims)
    want_ids, want_words = G.bricks(words, m.dims)
    assert 0 < n < tv.load_library().tv_brick_count_max(tv._dims(m.dims))
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), want_ids)
    assert np.array_equal(bw.cpu().numpy().view(np.uint32), want_words)


def test_bricks_rejects_unsupported_dims():
    import paper_2106_01326_amd as tv

    g = dev_words(np.zeros(4 * 8, dtype=np.uint32))
    with pytest.raises(tv.TVError):
        tv.bricks(g, (4, 8, 32))


# ----------------------------------------------------------- batch export

EXPORT_DIMS = [(32, 32, 32), (64, 64, 64), (8, 32, 64), (1, 2, 1024), (16, 16, 16), (128, 4, 32)]


@pytest.mark.parametrize("res", [1, 8, 32, 64])
def test_export_batch_random_grids(res):
    import torch

    import oracle.grids as G
    import paper_2106_01326_amd as tv

    banner(f"export batch res={res}")
    rng = np.random.default_rng(res + 11)
    ws = [rand_words(rng, d, 0.35) for d in EXPORT_DIMS]
    items = [(dev_words(w), d) for w, d in zip(ws, EXPORT_DIMS)]
    frac = tv.export_batch(items, res, "fraction")
    anyv = tv.export_batch(items, res, "any")
    torch.cuda.synchronize()
    want_f = G.export_batch(list(zip(ws, EXPORT_DIMS)), res, 0).astype(np.float32)
    want_a = G.export_batch(list(zip(ws, EXPORT_DIMS)), res, 1)
    assert frac.dtype == torch.float32 and anyv.dtype == torch.uint8
    assert np.array_equal(frac.cpu().numpy(), want_f)
    assert np.array_equal(anyv.cpu().numpy(), want_a)


def test_export_batch_of_a_voxelized_batch(oracle_mod):
    """Uneven meshes voxelized in one batch call, exported at 32^3 and 16^3,
    against the oracle's grids exported by the numpy oracle."""
    import torch

    import oracle.grids as G
    import paper_2106_01326_amd as tv

    meshes = synth.workload_batch(24, seed=31, workers=1)
    banner(f"export of a voxelized batch of {len(meshes)} meshes")
    items = [(torch.from_numpy(m.verts).cuda(), torch.from_numpy(m.tets).cuda(), m.dims, m.bbox, False)
             for m in meshes]
    grids, _ = tv.voxelize_batch(items)
    refs = [(g, m.dims) for g, m in zip(grids, meshes)]
    want_grids = [(oracle_mod.voxelize_mesh(m), m.dims) for m in meshes]
    for res in (32, 16):
        got = tv.export_batch(refs, res, "fraction")
        torch.cuda.synchronize()
        want = G.export_batch(want_grids, res, 0).astype(np.float32)
        assert np.array_equal(got.cpu().numpy(), want), f"res {res}"


def test_export_batch_unaligned_output():
    """An output that is not aligned for the 4-cells-per-thread stores takes
    the one-cell path; the values are the same."""
    import torch

    import oracle.grids as G
    import paper_2106_01326_amd as tv

    banner("export unaligned output")
    rng = np.random.default_rng(5)
    dims = [(32, 32, 32), (64, 16, 8)]
    ws = [rand_words(rng, d, 0.5) for d in dims]
    items = [(dev_words(w), d) for w, d in zip(ws, dims)]
    res = 16
    n = len(dims) * res ** 3
    for mode, dt, code in (("fraction", torch.float32, 0), ("any", torch.uint8, 1)):
        raw = torch.zeros(n + 1, dtype=dt, device="cuda")
        tv.export_batch(items, res, mode, out=raw[1:])
        torch.cuda.synchronize()
        want = G.export_batch(list(zip(ws, dims)), res, code)
        want = want.astype(np.float32) if code == 0 else want
        assert np.array_equal(raw[1:].cpu().numpy().reshape(want.shape), want), mode
        assert float(raw[0]) == 0
