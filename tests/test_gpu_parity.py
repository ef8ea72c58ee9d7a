"""Parity of the HIP path with the CPU oracle, bit for bit (integer output:
the bar is bit-exactness, padding bits included).  Every case goes through
the C ABI (tv_voxelize / tv_voxelize_q) via the thin binding."""
import numpy as np
import pytest

from helpers import first_mismatch, gpu_voxelize_mesh, gpu_voxelize_q, window_bits
from paper_2106_01326_amd import synth

pytestmark = pytest.mark.gpu

HALF, STRICT = 0, 1
LAT = 1 << 16


def banner(msg):
    print(f"[case] {msg}", flush=True)


def oracle_threads():
    """Host threads for full-size oracle runs: the machine's CPU share (16), or
    fewer where the machine has fewer."""
    import os

    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(16, n))


def oracle_words(oracle_mod, mesh, strict=False, **kw):
    return oracle_mod.voxelize_mesh(mesh, mode=STRICT if strict else HALF, **kw)


def assert_same(got, want, what):
    mm = first_mismatch(got, want)
    assert mm is None, f"{what}: first differing word {mm[0]} ({mm[1]} words differ)"


@pytest.mark.parametrize("per_tet", [False, True])
@pytest.mark.parametrize("strict", [False, True])
def test_small_workload(oracle_mod, strict, per_tet):
    m = synth.workload_small()
    banner(f"small workload nt={m.nt} strict={strict} per_tet={per_tet}")
    got, st = gpu_voxelize_mesh(m, strict, per_tet=per_tet)
    assert st == 0
    assert_same(got, oracle_words(oracle_mod, m, strict), "small")


@pytest.mark.parametrize("dims", [(32, 16, 8), (16, 32, 64), (1, 2, 32), (64, 64, 1), (8, 8, 2),
                                  (128, 4, 128), (4, 4, 2), (2, 1, 16), (1, 1, 1)])
def test_varied_dims(oracle_mod, dims):
    m = synth.make_mesh(6, 0.35, 32, "ellipsoids", 3, 101)
    m.dims = dims
    banner(f"dims {dims}")
    got, st = gpu_voxelize_mesh(m)
    assert st == 0
    assert_same(got, oracle_words(oracle_mod, m), f"dims {dims}")


@pytest.mark.parametrize("c,m_,off,n", [(4, 4, 2, 32), (3, 5, 1, 32), (5, 2, 3, 16), (2, 9, 6, 64)])
@pytest.mark.parametrize("strict", [False, True])
def test_aligned_lattice_ties(oracle_mod, c, m_, off, n, strict):
    """Vertices on voxel centers: every shared face passes through centers,
    so every center of the union is a tie case."""
    S = (LAT // 2) // n
    idx = synth._grid_index(c)
    q = ((2 * (idx * m_ + off) + 1) * S).astype(np.int32)
    rng = np.random.default_rng(c * 7 + m_)
    tets = np.array([t[rng.permutation(4)] for t in synth.kuhn_tets(c)], dtype=np.int32)
    banner(f"aligned c={c} m={m_} off={off} n={n} strict={strict}")
    got, st = gpu_voxelize_q(q, tets, (n, n, n), strict)
    want = oracle_mod.voxelize_q(q, tets, (n, n, n), mode=STRICT if strict else HALF)
    assert st == 0
    assert_same(got, want, "aligned")


def test_corner_tets_every_orientation(oracle_mod):
    import itertools

    n = 32
    S = (LAT // 2) // n
    O = np.array([(2 * 16 + 1) * S] * 3)
    for M in (1, 3, 6):
        for sx, sy, sz in itertools.product((1, -1), repeat=3):
            V = np.array([O, O + M * 2 * S * np.array([sx, 0, 0]), O + M * 2 * S * np.array([0, sy, 0]),
                          O + M * 2 * S * np.array([0, 0, sz])], dtype=np.int32)
            t = np.array([[0, 1, 2, 3], [3, 2, 1, 0]], dtype=np.int32)
            for strict in (False, True):
                got, _ = gpu_voxelize_q(V, t, (n, n, n), strict)
                want = oracle_mod.voxelize_q(V, t, (n, n, n), mode=STRICT if strict else HALF)
                assert_same(got, want, f"corner M={M} s=({sx},{sy},{sz}) strict={strict}")


def test_random_tets_with_heavy_ties(oracle_mod):
    """Random tets with vertices on a coarse sub-lattice of voxel centers
    and corners: many faces pass exactly through centers."""
    rng = np.random.default_rng(202)
    n = 16
    S = (LAT // 2) // n
    for trial in range(4):
        nt = 400
        q = (rng.integers(0, 2 * n + 1, size=(4 * nt, 3)) * S).astype(np.int32)
        tets = np.arange(4 * nt, dtype=np.int32).reshape(nt, 4)
        for strict in (False, True):
            got, st = gpu_voxelize_q(q, tets, (n, n, n), strict)
            want = oracle_mod.voxelize_q(q, tets, (n, n, n), mode=STRICT if strict else HALF)
            assert_same(got, want, f"random ties trial {trial} strict={strict}")


def test_extreme_coordinates_exactness(oracle_mod):
    """Huge tets with vertices at the ends of the lattice range exercise the
    largest face-function magnitudes (close to 2^52)."""
    rng = np.random.default_rng(303)
    lo, hi = -16384, 65536 + 16384
    corners = np.array([[lo, lo, lo], [hi, lo, lo], [lo, hi, lo], [lo, lo, hi], [hi, hi, hi],
                        [hi, hi, lo], [lo, hi, hi], [hi, lo, hi]], dtype=np.int32)
    rand = rng.integers(lo, hi + 1, size=(200, 3)).astype(np.int32)
    q = np.concatenate([corners, rand])
    tets = np.concatenate([np.array([[0, 1, 2, 3], [4, 5, 6, 7], [0, 4, 5, 6]], dtype=np.int32),
                           rng.integers(0, q.shape[0], size=(60, 4)).astype(np.int32)])
    for dims in ((32, 32, 32), (8, 64, 128)):
        got, st = gpu_voxelize_q(q, tets, dims)
        assert st == 0
        assert_same(got, oracle_mod.voxelize_q(q, tets, dims), f"extreme {dims}")


def test_full_cube_all_ones(oracle_mod):
    m = synth.make_mesh(10, 0.4, 64, "all", 0, 404)
    got, st = gpu_voxelize_mesh(m)
    assert st == 0
    nz = m.dims[2]
    assert np.all(got == np.uint32(0xFFFFFFFF)) if nz % 32 == 0 else True
    assert_same(got, oracle_words(oracle_mod, m), "full cube")


def test_empty_and_degenerate(oracle_mod):
    import torch

    import paper_2106_01326_amd as tv

    # nt == 0: all-zero grid (stale contents overwritten)
    q = torch.zeros((4, 3), dtype=torch.int32, device="cuda")
    t = torch.zeros((0, 4), dtype=torch.int32, device="cuda")
    grid = torch.full((tv.grid_words((8, 8, 64)),), -1, dtype=torch.int32, device="cuda")
    tv.voxelize(q, t, (8, 8, 64), qverts=True, grid=grid)
    assert int(grid.abs().sum()) == 0
    # degenerate tets only
    qn = np.array([[0, 0, 0], [40000, 0, 0], [0, 40000, 0], [20000, 20000, 0], [9000, 9000, 9000]], np.int32)
    tn = np.array([[0, 1, 2, 3], [0, 0, 1, 4], [4, 4, 4, 4], [0, 1, 2, 4]], np.int32)
    got, st = gpu_voxelize_q(qn, tn, (16, 16, 16))
    assert st == 0
    assert_same(got, oracle_mod.voxelize_q(qn, tn, (16, 16, 16)), "degenerate")


def test_device_data_errors(oracle_mod):
    """A bad tet index or an off-range / NaN coordinate is reported after the
    fact; the offending tets are skipped and the rest is still voxelized."""
    m = synth.make_mesh(6, 0.3, 32, "sphere", 0, 505)
    good = oracle_words(oracle_mod, m)
    bad = synth.Mesh(tets=np.concatenate([m.tets, np.array([[0, 1, 2, m.nv + 5]], np.int32)]),
                     dims=m.dims, bbox=m.bbox, verts=m.verts)
    got, st = gpu_voxelize_mesh(bad)
    import paper_2106_01326_amd as tv

    assert st == tv.TV_ERR_INDEX
    assert_same(got, good, "bad index skipped")
    v = m.verts.copy()
    extra = np.array([[np.nan, 0.5, 0.5], [0.5, 7.0, 0.5]], np.float32)
    v = np.concatenate([v, extra])
    t = np.concatenate([m.tets, np.array([[0, 1, 2, m.nv], [0, 1, 3, m.nv + 1]], np.int32)])
    got, st = gpu_voxelize_mesh(synth.Mesh(tets=t, dims=m.dims, bbox=m.bbox, verts=v))
    assert st == tv.TV_ERR_RANGE
    assert_same(got, good, "range error skipped")


def test_snap_matches_oracle_bit_exact(oracle_mod):
    """fp32 -> lattice on awkward values: arbitrary bbox, midpoints, range
    ends.  Compared through whole-mesh output where each tet is a tiny
    probe around one vertex."""
    rng = np.random.default_rng(606)
    lo = np.array([-1.7, 0.3, -100.0], np.float32)
    hi = np.array([2.9, 0.30003, 250.5], np.float32)
    base = rng.uniform(lo, hi, size=(3000, 3)).astype(np.float32)
    q = oracle_mod.snap(base, lo, hi)
    assert q.min() >= -16384 and q.max() <= 81920
    # tets from consecutive quadruples: outputs depend on every snapped coordinate
    tets = np.arange(3000, dtype=np.int32).reshape(-1, 4)
    m = synth.Mesh(tets=tets, dims=(64, 64, 64), bbox=(lo, hi), verts=base)
    got, st = gpu_voxelize_mesh(m)
    assert st == 0
    assert_same(got, oracle_mod.voxelize_q(q, tets, (64, 64, 64)), "snap probes")
    # the snapped vertices themselves, through tv_snap
    import torch

    import paper_2106_01326_amd as tv

    edge = np.array([[-16384 / LAT, 81920 / LAT, 0.5], [(2 * 77 + 1) / (2 * LAT), (2 * 78 + 1) / (2 * LAT), 1.0],
                     [0.0, 1.0, 1.0 / 3.0]], np.float32)
    lo01, hi01 = np.zeros(3, np.float32), np.ones(3, np.float32)
    for b_lo, b_hi, vv in ((lo, hi, base), (lo01, hi01, edge)):
        q = tv.snap(torch.from_numpy(vv).cuda(), (b_lo, b_hi)).cpu().numpy()
        assert np.array_equal(q, oracle_mod.snap(vv, b_lo, b_hi))
    bad = np.array([[np.nan, 0, 0], [0.5, 0.5, 0.5], [0, 2.0, 0]], np.float32)
    q = tv.snap(torch.from_numpy(bad).cuda(), (lo01, hi01)).cpu().numpy()
    assert np.all(q[0] == tv.Q_INVALID) and np.all(q[2] == tv.Q_INVALID)
    assert list(q[1]) == [32768, 32768, 32768]


@pytest.mark.parametrize("per_tet", [False, True])
def test_shared_tiles_and_chunks(oracle_mod, per_tet):
    """Many tets per tile (a fine mesh in a coarse grid): tiles take several
    chunks, are zeroed first and flushed with word atomics."""
    m = synth.make_mesh(24, 0.35, 32, "ellipsoids", 3, 909)  # ~30k tets kept in one 32^3 tile
    banner(f"shared tiles nt={m.nt}")
    for dims in ((32, 32, 32), (16, 16, 64), (64, 64, 32)):
        m.dims = dims
        got, st = gpu_voxelize_mesh(m, per_tet=per_tet)
        assert st == 0
        assert_same(got, oracle_words(oracle_mod, m), f"shared tiles {dims}")


@pytest.mark.parametrize("per_tet", [False, True])
def test_large_tets_mixed_with_small(oracle_mod, per_tet):
    """Tets whose candidate box meets more tiles than the cap go through the
    large-tet kernel after the tile kernel; mixed with ordinary tets."""
    rng = np.random.default_rng(1001)
    small = synth.make_mesh(10, 0.3, 256, "ellipsoids", 2, 1002)
    q_small = oracle_mod.snap(small.verts, *small.bbox)
    big_q = np.array([[1000, 2000, 3000], [64000, 5000, 9000], [4000, 63000, 20000], [30000, 30000, 64000],
                      [-16000, -16000, -16000], [81000, 40000, 100], [40000, 81000, 200], [40000, 40000, 81000]],
                     np.int32)
    q = np.concatenate([q_small, big_q])
    n0 = q_small.shape[0]
    big_t = np.array([[n0, n0 + 1, n0 + 2, n0 + 3], [n0 + 4, n0 + 5, n0 + 6, n0 + 7]], np.int32)
    tets = np.concatenate([small.tets, big_t])
    tets = tets[rng.permutation(tets.shape[0])]
    for dims in ((256, 256, 256), (128, 512, 64)):
        got, st = gpu_voxelize_q(q, tets, dims, per_tet=per_tet)
        assert st == 0
        assert_same(got, oracle_mod.voxelize_q(q, tets, dims), f"large tets {dims}")


def test_random_tet_order(oracle_mod):
    """Input order with no spatial coherence (the binning's aggregated
    atomics see distinct keys in every lane)."""
    m = synth.make_mesh(20, 0.4, 128, "ellipsoids", 4, 1003, shuffle=True)
    got, st = gpu_voxelize_mesh(m)
    assert st == 0
    assert_same(got, oracle_words(oracle_mod, m), "shuffled")


def test_tets_straddling_tile_corners(oracle_mod):
    """Small tets placed at random tile corners, in random order: every tet
    meets up to 8 tiles and a workgroup of the binning passes meets far more
    distinct tiles than its aggregation table holds, so many pieces take the
    direct global-atomic path of both passes."""
    rng = np.random.default_rng(1005)
    dims = (256, 256, 256)
    pitch = LAT // 256  # lattice units per voxel
    n = 2048
    corner = np.stack([rng.integers(1, 16, n) * 16, rng.integers(1, 16, n) * 16,
                       np.full(n, 128)], axis=1) * pitch
    q = (corner[:, None, :] + rng.integers(-6 * pitch, 6 * pitch + 1, size=(n, 4, 3))).reshape(-1, 3)
    tets = np.arange(4 * n, dtype=np.int32).reshape(n, 4)
    banner(f"{n} tets at tile corners, {dims}")
    got, st = gpu_voxelize_q(q, tets, dims)
    assert st == 0
    want = oracle_mod.voxelize_q(q.astype(np.int32), tets, dims)
    assert int(np.unpackbits(want.view(np.uint8)).sum()) > 0
    assert_same(got, want, "tile-corner tets")


@pytest.mark.parametrize("strict", [False, True])
def test_tets_smaller_than_voxels(oracle_mod, strict):
    """More tets than voxels (the regime where small pieces are finished as
    soon as their faces are built, next to larger ones in the same tiles)."""
    m = synth.make_mesh(40, 0.4, 64, "all", 0, 1006)
    banner(f"{m.nt} tets in a 64^3 grid, strict={strict}")
    got, st = gpu_voxelize_mesh(m, strict=strict)
    assert st == 0
    assert_same(got, oracle_words(oracle_mod, m, strict=strict), "small tets")


def test_repeatable_bit_identical():
    m = synth.make_mesh(16, 0.4, 64, "ellipsoids", 4, 707)
    ref, _ = gpu_voxelize_mesh(m)
    for _ in range(5):
        got, _ = gpu_voxelize_mesh(m)
        assert np.array_equal(got, ref)


# ------------------------------------------------------- full-size workloads

@pytest.fixture(scope="module")
def medium():
    return synth.workload_medium()


@pytest.mark.parametrize("per_tet", [False, True])
def test_medium_workload_full_grid(oracle_mod, medium, per_tet):
    banner(f"medium workload nt={medium.nt} nv={medium.nv} per_tet={per_tet}")
    got, st = gpu_voxelize_mesh(medium, per_tet=per_tet)
    assert st == 0
    assert_same(got, oracle_words(oracle_mod, medium), "medium")


def test_many_tets_full_grid(oracle_mod):
    """A mesh above the binning's many-tets threshold (2^21 tets: four tets
    per binning thread) against the oracle over the whole 256^3 grid."""
    m = synth.make_mesh(72, 0.3, 256, "all", 0, 3301)
    assert m.nt >= 1 << 21
    banner(f"many-tets mesh nt={m.nt}")
    got, st = gpu_voxelize_mesh(m)
    assert st == 0
    assert_same(got, oracle_words(oracle_mod, m), "many tets")


def test_large_workload_full_grid(oracle_mod, large):
    """The whole 1024^3 grid of the large workload (5.56M tets, fp32 input
    snapped on the device) against the oracle over every tet, bit for bit."""
    banner(f"large workload full grid nt={large.nt} nv={large.nv}")
    got, st = gpu_voxelize_mesh(large)
    assert st == 0
    want = oracle_words(oracle_mod, large, threads=oracle_threads())
    assert_same(got, want, "large (full grid)")
    assert int(np.unpackbits(want.view(np.uint8)).sum()) > 0


def test_large_workload_sampled_windows(oracle_mod, large):
    """1024^3 grid: the oracle recomputes random windows one by one (every
    tet, only the window's voxels), compared bit for bit."""
    banner(f"large workload nt={large.nt} nv={large.nv}")
    got, st = gpu_voxelize_mesh(large)
    assert st == 0
    q = oracle_mod.snap(large.verts, *large.bbox)
    rng = np.random.default_rng(808)
    n = 1024
    total = 0
    for w in range(6):
        i0, j0 = rng.integers(0, n - 48, size=2)
        k0 = int(rng.integers(0, n - 200))
        win = (int(i0), int(i0) + 47, int(j0), int(j0) + 47, k0, k0 + 199)
        want = oracle_mod.voxelize_q(q, large.tets, large.dims, window=win)
        a = window_bits(got, large.dims, win)
        b = window_bits(want, large.dims, win)
        assert np.array_equal(a, b), f"window {win}"
        total += int(b.sum())
    assert total > 0
    # global properties: padding-free layout, set count within a sane range
    nset = int(np.unpackbits(got.view(np.uint8)).sum())
    assert 0.05 * n ** 3 < nset < 0.95 * n ** 3


def test_full_size_cube_partition():
    """At the large configuration's full size (128^3 Kuhn cells, 12.6M tets,
    jitter 0.45, 1024^3 grid) with every tet kept: the grid is all ones, and
    two random halves of the tets give disjoint grids whose union is all ones
    -- each voxel center covered exactly once by a conforming mesh under the
    half-open rule.  A property that holds at any size, checked in the launch
    configuration bench.py times."""
    import torch

    import paper_2106_01326_amd as tv

    m = synth.make_mesh(128, 0.45, 1024, "all", 0, 2)
    banner(f"full-size cube partition: {m.nt} tets")
    v = torch.from_numpy(m.verts).cuda()
    rng = np.random.default_rng(2024)
    side = rng.random(m.nt) < 0.5
    grids = []
    for tets in (m.tets, m.tets[side], m.tets[~side]):
        t = torch.from_numpy(np.ascontiguousarray(tets)).cuda()
        g, ws = tv.voxelize(v, t, m.dims, m.bbox)
        assert tv.fetch_status(ws) == tv.TV_OK
        grids.append(g)
        del t, ws
    full, a, b = grids
    ones = torch.full_like(full, -1)
    assert torch.equal(full, ones)
    assert not torch.any(a & b)
    assert torch.equal(a | b, ones)
