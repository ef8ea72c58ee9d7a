"""Accumulating voxelization (TV_ACCUMULATE) and the pipelined call from
host inputs (tv_voxelize_pipelined): the grid of a mesh voxelized in tet
slices equals the oracle's grid of the whole mesh, bit for bit."""
import numpy as np
import pytest

from paper_2106_01326_amd import synth

pytestmark = pytest.mark.gpu


def banner(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def mesh():
    return synth.make_mesh(20, 0.4, 128, "ellipsoids", 4, 6001)


def words(grid):
    return grid.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("per_tet", [False, True])
def test_accumulate_two_halves(oracle_mod, mesh, per_tet):
    import torch

    import paper_2106_01326_amd as tv

    m = mesh
    banner(f"accumulate halves per_tet={per_tet}")
    v = torch.from_numpy(m.verts).cuda()
    h = m.nt // 2
    a = torch.from_numpy(np.ascontiguousarray(m.tets[:h])).cuda()
    b = torch.from_numpy(np.ascontiguousarray(m.tets[h:])).cuda()
    grid = tv.alloc_grid(m.dims)
    grid.fill_(-1)  # stale content: the first call overwrites it
    tv.voxelize(v, a, m.dims, m.bbox, grid=grid, per_tet=per_tet)
    tv.voxelize(v, b, m.dims, m.bbox, grid=grid, per_tet=per_tet, accumulate=True)
    assert np.array_equal(words(grid), oracle_mod.voxelize_mesh(m))
    # accumulating onto ones keeps them
    ones = tv.alloc_grid(m.dims)
    ones.fill_(-1)
    tv.voxelize(v, a, m.dims, m.bbox, grid=ones, per_tet=per_tet, accumulate=True)
    assert np.all(words(ones) == 0xFFFFFFFF)


def test_accumulate_keeps_status(mesh):
    import torch

    import paper_2106_01326_amd as tv

    m = mesh
    v = torch.from_numpy(m.verts).cuda()
    bad = torch.from_numpy(np.array([[0, 1, 2, m.nv + 7]], np.int32)).cuda()
    good = torch.from_numpy(np.ascontiguousarray(m.tets[:100])).cuda()
    grid = tv.alloc_grid(m.dims)
    need = tv.workspace_bytes(m.nv, 100, m.dims)
    ws = tv.alloc_workspace(need)
    tv.voxelize(v, bad, m.dims, m.bbox, grid=grid, workspace=ws)
    tv.voxelize(v, good, m.dims, m.bbox, grid=grid, workspace=ws, accumulate=True)
    assert tv.fetch_status(ws) == tv.TV_ERR_INDEX
    tv.voxelize(v, good, m.dims, m.bbox, grid=grid, workspace=ws)  # a plain call clears it
    assert tv.fetch_status(ws) == tv.TV_OK


@pytest.mark.parametrize("chunks", [1, 3, 8, 64, 1000])
def test_pipelined_matches_oracle(oracle_mod, mesh, chunks):
    import torch

    import paper_2106_01326_amd as tv

    m = mesh
    banner(f"pipelined chunks={chunks}")
    vh = torch.from_numpy(m.verts).pin_memory()
    th = torch.from_numpy(m.tets).pin_memory()
    grid, ws, vd, td = tv.voxelize_pipelined(vh, th, m.dims, m.bbox, chunks=chunks)
    torch.cuda.synchronize()
    assert tv.fetch_status(ws) == tv.TV_OK
    assert np.array_equal(words(grid), oracle_mod.voxelize_mesh(m))
    assert np.array_equal(td.cpu().numpy(), m.tets)


def test_pipelined_strict_pageable_and_empty(oracle_mod, mesh):
    import torch

    import paper_2106_01326_amd as tv

    m = mesh
    vh = torch.from_numpy(m.verts)  # pageable: correct, only not overlapped
    th = torch.from_numpy(m.tets)
    grid, _, _, _ = tv.voxelize_pipelined(vh, th, m.dims, m.bbox, chunks=5, strict=True)
    assert np.array_equal(words(grid), oracle_mod.voxelize_mesh(m, mode=oracle_mod.STRICT))
    empty = torch.zeros((0, 4), dtype=torch.int32)
    g0 = tv.alloc_grid(m.dims)
    g0.fill_(-1)
    tv.voxelize_pipelined(vh, empty, m.dims, m.bbox, chunks=4, grid=g0)
    assert not np.any(words(g0))


def test_pipelined_bad_slice_reports(mesh):
    import torch

    import paper_2106_01326_amd as tv

    m = mesh
    tets = m.tets.copy()
    tets[len(tets) // 2, 3] = m.nv + 3  # a bad index in a middle slice
    grid, ws, _, _ = tv.voxelize_pipelined(torch.from_numpy(m.verts).pin_memory(),
                                          torch.from_numpy(tets).pin_memory(), m.dims, m.bbox, chunks=6)
    assert tv.fetch_status(ws) == tv.TV_ERR_INDEX
