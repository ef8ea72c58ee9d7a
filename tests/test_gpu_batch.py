"""Batched voxelization: every mesh of a batch equals, bit for bit, its
own single-mesh result and the oracle; a bad mesh does not affect the
others."""
import numpy as np
import pytest

from helpers import to_numpy_words
from paper_2106_01326_amd import synth

pytestmark = pytest.mark.gpu


def banner(msg):
    print(f"[case] {msg}", flush=True)


def to_item(m):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(m.tets)).cuda()
    if m.verts is not None:
        return (torch.from_numpy(m.verts).cuda(), t, m.dims, m.bbox, False)
    return (torch.from_numpy(m.qverts).cuda(), t, m.dims, None, True)


@pytest.fixture(scope="module")
def uneven():
    ms = synth.workload_batch(first=40, workers=8)
    # extra variety: int32 lattice input, odd dims, an empty mesh, a 256^3 grid
    ms.append(synth.make_mesh(16, 0.3, 32, "ellipsoids", 2, 2001, fmt="q32"))
    odd = synth.make_mesh(7, 0.25, 32, "sphere", 0, 2002)
    odd.dims = (16, 64, 8)
    ms.append(odd)
    ms.append(synth.Mesh(tets=np.zeros((0, 4), np.int32), dims=(32, 32, 32),
                         bbox=(np.zeros(3, np.float32), np.ones(3, np.float32)),
                         verts=np.zeros((1, 3), np.float32)))
    ms.append(synth.make_mesh(24, 0.3, 256, "ellipsoids", 3, 2003))
    return ms


@pytest.mark.parametrize("per_tet", [False, True])
def test_batch_matches_oracle_and_solo(oracle_mod, uneven, per_tet):
    import paper_2106_01326_amd as tv

    banner(f"batch of {len(uneven)} meshes per_tet={per_tet}")
    b = tv.Batch([to_item(m) for m in uneven])
    for g in b.grids:
        g.fill_(-1)  # stale contents must be overwritten
    grids = b.run(per_tet=per_tet)
    for i, (m, g) in enumerate(zip(uneven, grids)):
        got = to_numpy_words(g)
        want = oracle_mod.voxelize_mesh(m)
        assert np.array_equal(got, want), f"mesh {i} ({m.nt} tets, dims {m.dims})"
        assert b.status(i) == tv.TV_OK
    # single-mesh calls agree
    for i in (0, 5, len(uneven) - 1):
        v, t, dims, bbox, q = to_item(uneven[i])
        g, _ = tv.voxelize(v, t, dims, bbox, qverts=q)
        assert np.array_equal(to_numpy_words(g), to_numpy_words(grids[i]))


def test_full_batch_workload_every_mesh(oracle_mod):
    """The whole uneven batch workload (1024 meshes, 32^3 and 64^3 grids,
    fp32 input) in one batched call: every mesh's grid against the oracle."""
    import paper_2106_01326_amd as tv

    ms = synth.workload_batch(count=1024, workers=8)
    banner(f"full batch workload: {len(ms)} meshes, {sum(m.nt for m in ms)} tets")
    b = tv.Batch([to_item(m) for m in ms])
    for g in b.grids:
        g.fill_(-1)
    grids = b.run()
    bad = []
    for i, (m, g) in enumerate(zip(ms, grids)):
        if b.status(i) != tv.TV_OK or not np.array_equal(to_numpy_words(g), oracle_mod.voxelize_mesh(m)):
            bad.append(i)
    assert not bad, f"{len(bad)} meshes differ, first {bad[:5]}"


def test_batch_rerun_and_strict(oracle_mod, uneven):
    import paper_2106_01326_amd as tv

    b = tv.Batch([to_item(m) for m in uneven[:12]])
    first = [to_numpy_words(g).copy() for g in b.run()]
    strict = [to_numpy_words(g).copy() for g in b.run(strict=True)]
    again = [to_numpy_words(g).copy() for g in b.run()]
    for i, m in enumerate(uneven[:12]):
        assert np.array_equal(first[i], again[i])
        assert np.array_equal(strict[i], oracle_mod.voxelize_mesh(m, mode=oracle_mod.STRICT))


def test_bad_mesh_is_isolated(oracle_mod):
    import paper_2106_01326_amd as tv

    ms = synth.workload_batch(first=6, workers=1)
    bad = ms[2]
    bad_tets = np.concatenate([bad.tets, np.array([[0, 1, 2, bad.nv + 7]], np.int32)])
    nanv = ms[4].verts.copy()
    nanv[0, 0] = np.nan
    items = [to_item(m) for m in ms]
    import torch

    items[2] = (items[2][0], torch.from_numpy(bad_tets).cuda(), bad.dims, bad.bbox, False)
    items[4] = (torch.from_numpy(nanv).cuda(), items[4][1], ms[4].dims, ms[4].bbox, False)
    b = tv.Batch(items)
    grids = b.run()
    st = [b.status(i) for i in range(len(ms))]
    assert st[2] == tv.TV_ERR_INDEX and st[4] == tv.TV_ERR_RANGE
    assert all(s == tv.TV_OK for i, s in enumerate(st) if i not in (2, 4))
    for i, m in enumerate(ms):
        want = oracle_mod.voxelize_mesh(m)
        if i == 4:  # tets that use vertex 0 are skipped
            keep = ~np.any(m.tets == 0, axis=1)
            q = oracle_mod.snap(np.where(np.isnan(nanv), 0, nanv), *m.bbox)
            want = oracle_mod.voxelize_q(q, m.tets[keep], m.dims)
        assert np.array_equal(to_numpy_words(grids[i]), want), f"mesh {i}"
    assert b.status(len(ms)) == tv.TV_ERR_INVALID_ARG


def test_whole_grid_meshes_check_their_tets(oracle_mod):
    """Meshes whose grid is a single tile (32^3 in a batch), one of them with
    many chunks: a bad index flags its mesh, a vertex that fails the snap
    drops the tets using it, and every other mesh is untouched."""
    import torch

    import paper_2106_01326_amd as tv

    ms = [synth.make_mesh(8, 0.2, 32, "sphere", 0, 7100 + i) for i in range(3)]
    ms.append(synth.make_mesh(12, 0.3, 64, "ellipsoids", 2, 7103))  # binned, 4 tiles
    ms.append(synth.make_mesh(40, 0.3, 32, "all", 0, 7104))  # one tile, many chunks
    bad_tets = np.concatenate([ms[0].tets, np.array([[0, 1, 2, ms[0].nv + 7], [-3, 1, 2, 3]], np.int32)])
    nanv = ms[1].verts.copy()
    nanv[5, 2] = np.nan
    items = [to_item(m) for m in ms]
    items[0] = (items[0][0], torch.from_numpy(bad_tets).cuda(), ms[0].dims, ms[0].bbox, False)
    items[1] = (torch.from_numpy(nanv).cuda(), items[1][1], ms[1].dims, ms[1].bbox, False)
    b = tv.Batch(items)
    grids = b.run()
    assert [b.status(i) for i in range(len(ms))] == [tv.TV_ERR_INDEX, tv.TV_ERR_RANGE, tv.TV_OK, tv.TV_OK,
                                                    tv.TV_OK]
    for i, m in enumerate(ms):
        want = oracle_mod.voxelize_mesh(m)
        if i == 1:
            keep = ~np.any(m.tets == 5, axis=1)
            q = oracle_mod.snap(np.where(np.isnan(nanv), 0, nanv), *m.bbox)
            want = oracle_mod.voxelize_q(q, m.tets[keep], m.dims)
        assert np.array_equal(to_numpy_words(grids[i]), want), f"mesh {i}"


def test_single_mesh_batch(oracle_mod):
    """A batch of one mesh keeps its descriptor in the workspace table like
    any batch; the grid equals the oracle's and the single-mesh call's."""
    import paper_2106_01326_amd as tv

    m = synth.make_mesh(20, 0.35, 64, "ellipsoids", 3, 7201)
    banner("batch of one mesh")
    b = tv.Batch([to_item(m)])
    b.grids[0].fill_(-1)
    want = oracle_mod.voxelize_mesh(m)
    assert np.array_equal(to_numpy_words(b.run()[0]), want)
    b.prepare()
    b.grids[0].fill_(-1)
    assert np.array_equal(to_numpy_words(b.run_prepared()[0]), want)
    assert b.status(0) == tv.TV_OK


def test_prepared_batch_runs(oracle_mod, uneven):
    """tv_batch_prepare once, tv_batch_run many times: every run equals the
    oracle; a run sees the buffers' current contents; the plan only works
    with its own workspace."""
    import ctypes

    import torch

    import paper_2106_01326_amd as tv

    ms = uneven[:20] + uneven[-4:]
    banner(f"prepared batch of {len(ms)} meshes")
    items = [to_item(m) for m in ms]
    b = tv.Batch(items)
    b.prepare()
    for r in range(2):
        for g in b.grids:
            g.fill_(-1)
        grids = b.run_prepared()
        for i, (m, g) in enumerate(zip(ms, grids)):
            assert np.array_equal(to_numpy_words(g), oracle_mod.voxelize_mesh(m)), f"run {r} mesh {i}"
            assert b.status(i) == tv.TV_OK
    # strict mode through its own plan
    b.prepare(strict=True)
    for i, (m, g) in enumerate(zip(ms, b.run_prepared())):
        assert np.array_equal(to_numpy_words(g), oracle_mod.voxelize_mesh(m, mode=oracle_mod.STRICT)), f"mesh {i}"
    # new vertex contents in place (same topology): the next run uses them
    b.prepare()
    k = 3
    m = ms[k]
    moved = synth.Mesh(tets=m.tets, dims=m.dims, bbox=m.bbox,
                       verts=(0.5 + 0.8 * (m.verts - 0.5)).astype(np.float32))
    items[k][0].copy_(torch.from_numpy(moved.verts).cuda())
    grids = b.run_prepared()
    assert np.array_equal(to_numpy_words(grids[k]), oracle_mod.voxelize_mesh(moved))
    assert np.array_equal(to_numpy_words(grids[0]), oracle_mod.voxelize_mesh(ms[0]))
    # the plan names its workspace: another one is refused before anything runs
    other = tv.alloc_workspace(b.workspace.numel())
    lib = tv.load_library()
    st = lib.tv_batch_run(ctypes.byref(b.plan), ctypes.c_void_p(other.data_ptr()), other.numel(), None)
    assert st == tv.TV_ERR_INVALID_ARG and b"another workspace" in lib.tv_last_error()


def test_prepared_batch_accumulates(oracle_mod):
    """A batch prepared with TV_ACCUMULATE ORs each run into the grids: two
    runs over the two halves of every mesh's tets (swapped in place between
    the runs) give the whole mesh's grid."""
    import torch

    import paper_2106_01326_amd as tv

    ms = synth.workload_batch(first=8, workers=1)
    banner(f"accumulating prepared batch of {len(ms)} meshes")
    halves = []
    items = []
    for m in ms:
        h = m.nt // 2
        a, b = np.ascontiguousarray(m.tets[:h]), np.ascontiguousarray(m.tets[h:2 * h])
        halves.append((a, b))
        items.append((torch.from_numpy(m.verts).cuda(), torch.from_numpy(a).cuda(), m.dims, m.bbox, False))
    b = tv.Batch(items)
    for g in b.grids:
        g.zero_()
    b.prepare(accumulate=True)
    b.run_prepared()
    for (a, bb), it in zip(halves, items):
        it[1].copy_(torch.from_numpy(bb).cuda())
    grids = b.run_prepared()
    for i, m in enumerate(ms):
        h = m.nt // 2
        even = synth.Mesh(tets=m.tets[:2 * h], dims=m.dims, bbox=m.bbox, verts=m.verts)
        assert np.array_equal(to_numpy_words(grids[i]), oracle_mod.voxelize_mesh(even)), f"mesh {i}"
        assert b.status(i) == tv.TV_OK
