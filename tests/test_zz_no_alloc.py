"""The allocation-free entry point (tv_voxelize_noalloc) against the
workspace entry point (tv_voxelize) on the same inputs, bit for bit: two
calls in a row, the second on a smaller mesh (the shared scratch array keeps
the first call's contents), then a call with a data error and a clean call
after it.  The outputs and the grids start filled with ones, so any word the
path fails to write shows up."""
import numpy as np
import pytest

from helpers import first_mismatch
from paper_2106_01326_amd import synth

pytestmark = pytest.mark.gpu


def banner(msg):
    print(f"[case] {msg}", flush=True)


def run_both(tv, torch, m, strict=False):
    v = torch.from_numpy(np.ascontiguousarray(m.verts)).cuda()
    t = torch.from_numpy(np.ascontiguousarray(m.tets)).cuda()
    g_ws = tv.alloc_grid(m.dims).fill_(-1)
    g_ws, ws = tv.voxelize(v, t, m.dims, m.bbox, strict=strict, grid=g_ws)
    want_status = tv.fetch_status(ws)
    g_na = tv.alloc_grid(m.dims).fill_(-1)
    status = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    g_na, status = tv.voxelize_noalloc(v, t, m.dims, m.bbox, strict=strict, grid=g_na, status=status)
    torch.cuda.synchronize()
    return (g_na.cpu().numpy().view(np.uint32), int(status.item()),
            g_ws.cpu().numpy().view(np.uint32), want_status)


def assert_same(got, want, what):
    mm = first_mismatch(got, want)
    assert mm is None, f"{what}: first differing word {mm[0]} ({mm[1]} words differ)"


def test_noalloc_matches_workspace_call_twice_in_a_row():
    import torch

    import paper_2106_01326_amd as tv

    big = synth.medium_shape_fp32(41)
    small = synth.make_mesh(12, 0.3, 64, "ellipsoids", 2, 42)
    need_big = tv.workspace_bytes(big.nv, big.nt, big.dims)
    assert need_big <= tv.NOALLOC_MAX_BYTES
    assert tv.workspace_bytes(small.nv, small.nt, small.dims) < need_big
    for name, m in (("medium shape", big), ("small after it", small)):
        banner(f"noalloc {name}: nt={m.nt} dims={m.dims}")
        got, st, want, want_st = run_both(tv, torch, m)
        assert want_st == tv.TV_OK and st == tv.TV_OK
        assert_same(got, want, name)
        assert int(np.unpackbits(got.view(np.uint8)).sum()) > 0


def test_noalloc_strict_and_data_errors():
    import torch

    import paper_2106_01326_amd as tv

    m = synth.workload_small()
    banner("noalloc strict small")
    got, st, want, want_st = run_both(tv, torch, m, strict=True)
    assert st == want_st == tv.TV_OK
    assert_same(got, want, "strict")

    bad = synth.workload_small()
    bad.tets = bad.tets.copy()
    bad.tets[len(bad.tets) // 2, 2] = bad.nv + 7  # an index outside [0, nv)
    banner("noalloc bad index")
    got, st, want, want_st = run_both(tv, torch, bad)
    assert want_st == tv.TV_ERR_INDEX and st == tv.TV_ERR_INDEX
    assert_same(got, want, "bad index")

    # the status words are cleared per call: a clean mesh reports TV_OK again
    banner("noalloc clean after error")
    got, st, want, want_st = run_both(tv, torch, m)
    assert st == want_st == tv.TV_OK
    assert_same(got, want, "clean after error")


def test_noalloc_refuses_meshes_beyond_the_scratch():
    import torch

    import paper_2106_01326_amd as tv

    # sizes alone decide: tets of this count need more than the fixed array
    nt = tv.NOALLOC_MAX_BYTES // 40
    v = torch.zeros((4, 3), dtype=torch.float32, device="cuda")
    t = torch.zeros((nt, 4), dtype=torch.int32, device="cuda")
    dims = (32, 32, 32)
    assert tv.workspace_bytes(4, nt, dims) > tv.NOALLOC_MAX_BYTES
    grid = tv.alloc_grid(dims).fill_(-1)
    banner(f"noalloc refuses nt={nt}")
    with pytest.raises(tv.TVError) as e:
        tv.voxelize_noalloc(v, t, dims, ((0, 0, 0), (1, 1, 1)), grid=grid)
    assert e.value.code == tv.TV_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert (grid.cpu().numpy().view(np.uint32) == 0xFFFFFFFF).all()  # nothing was enqueued
