"""CPU-side checks of the C-ABI library: it loads without a GPU and exports
every function declared in include/*.h; host-side argument checks return
their documented codes without touching the device."""
import ctypes
import os

import pytest

import paper_2106_01326_amd as tv
from helpers import header_symbols


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(tv.library_path()):
        import __graft_entry__

        __graft_entry__.build()
    return tv.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = header_symbols()
    assert "tv_voxelize" in names and "tv_voxelize_q" in names
    for n in names:
        assert hasattr(lib, n), f"{n} declared in include/ but not exported"
    assert set(tv.EXPORTED) <= set(names)


def test_grid_words_and_dims(lib):
    assert tv.grid_words((256, 256, 256)) == 256 * 256 * 8
    assert tv.grid_words((1, 2, 1)) == 2
    assert tv.grid_words((8, 8, 48)) == 0  # not a power of two
    assert tv.grid_words((1, 1, 65536)) == 0


def test_workspace_grows_with_vertices(lib):
    a = tv.workspace_bytes(10, 10, (32, 32, 32))
    b = tv.workspace_bytes(10000, 10, (32, 32, 32))
    assert a >= 256 and b > a and b % 256 == 0


def call_q(lib, nv=4, nt=1, dims=(8, 8, 8), grid=256, ws=256, ws_bytes=1 << 20, flags=0, tets=256, q=256):
    d = tv.Dims(*dims)
    P = ctypes.c_void_p
    return lib.tv_voxelize_q(P(q), nv, P(tets), nt, d, P(grid), P(ws), ws_bytes, None, flags)


def test_host_argument_errors(lib):
    # pointers are never dereferenced on these paths: the checks fail first
    assert call_q(lib, dims=(8, 12, 8)) == tv.TV_ERR_UNSUPPORTED_DIMS
    assert call_q(lib, dims=(0, 8, 8)) == tv.TV_ERR_UNSUPPORTED_DIMS
    assert call_q(lib, nv=-1) == tv.TV_ERR_INVALID_ARG
    assert call_q(lib, grid=0) == tv.TV_ERR_INVALID_ARG
    assert call_q(lib, tets=0) == tv.TV_ERR_INVALID_ARG
    assert call_q(lib, flags=4) == tv.TV_ERR_INVALID_ARG
    assert call_q(lib, tets=264) == tv.TV_ERR_INVALID_ARG  # tets not 16-byte aligned
    assert call_q(lib, ws=0) == tv.TV_ERR_WORKSPACE
    assert call_q(lib, ws=260) == tv.TV_ERR_WORKSPACE
    assert call_q(lib, ws_bytes=16) == tv.TV_ERR_WORKSPACE
    assert b"workspace" in lib.tv_last_error()
    d = tv.Dims(8, 8, 8)
    bad = tv.BBox((ctypes.c_float * 3)(0, 0, 0), (ctypes.c_float * 3)(1, 0, 1))
    P = ctypes.c_void_p
    assert lib.tv_voxelize(P(256), 4, P(256), 1, d, bad, P(256), P(256), 1 << 20, None, 0) == tv.TV_ERR_INVALID_ARG
    assert lib.tv_snap(P(256), 4, bad, P(256), None) == tv.TV_ERR_INVALID_ARG
    assert lib.tv_status_string(tv.TV_ERR_INDEX) == b"TV_ERR_INDEX"


def test_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(tv, "_lib", None)
    monkeypatch.setattr(tv, "LIB_PATH", "/nonexistent/libtetvox.so")
    with pytest.raises(RuntimeError, match="missing"):
        tv.load_library()


def test_batch_host_errors_name_the_mesh(lib):
    P = ctypes.c_void_p
    good = tv.MeshC(256, tv.VERTS_F32, 4, 256, 1, tv.Dims(8, 8, 8),
                    tv.BBox((ctypes.c_float * 3)(0, 0, 0), (ctypes.c_float * 3)(1, 1, 1)), 256)
    bad = tv.MeshC(256, tv.VERTS_F32, 4, 256, 1, tv.Dims(8, 6, 8),
                   tv.BBox((ctypes.c_float * 3)(0, 0, 0), (ctypes.c_float * 3)(1, 1, 1)), 256)
    arr = (tv.MeshC * 3)(good, good, bad)
    assert lib.tv_batch_workspace_bytes(ctypes.cast(arr, P), 3, 0) == 0
    assert lib.tv_voxelize_batch(ctypes.cast(arr, P), 3, P(256), 1 << 30, None, 0) == tv.TV_ERR_UNSUPPORTED_DIMS
    assert b"mesh 2" in lib.tv_last_error()
    arr2 = (tv.MeshC * 2)(good, good)
    need = lib.tv_batch_workspace_bytes(ctypes.cast(arr2, P), 2, 0)
    assert need > 0
    assert lib.tv_voxelize_batch(ctypes.cast(arr2, P), 2, P(256), need - 256, None, 0) == tv.TV_ERR_WORKSPACE
    assert lib.tv_voxelize_batch(ctypes.cast(arr2, P), 0, P(256), need, None, 0) == tv.TV_ERR_INVALID_ARG


def test_batch_prepare_and_run_host_errors(lib):
    """tv_batch_prepare / tv_batch_run: every argument error is caught on the
    host before anything is enqueued."""
    P = ctypes.c_void_p
    box = tv.BBox((ctypes.c_float * 3)(0, 0, 0), (ctypes.c_float * 3)(1, 1, 1))
    good = tv.MeshC(256, tv.VERTS_F32, 4, 256, 1, tv.Dims(8, 8, 8), box, 256)
    bad = tv.MeshC(256, tv.VERTS_F32, 4, 256, 1, tv.Dims(8, 8, 24), box, 256)
    arr = (tv.MeshC * 2)(good, good)
    need = lib.tv_batch_workspace_bytes(ctypes.cast(arr, P), 2, 0)
    plan = tv.BatchPlanC()
    prep = lambda a, n, ws, nbytes, flags, pl: lib.tv_batch_prepare(ctypes.cast(a, P), n, P(ws), nbytes, None,
                                                                    flags, pl)
    assert prep(arr, 2, 256, need, 0, None) == tv.TV_ERR_INVALID_ARG  # no plan
    assert prep(arr, 0, 256, need, 0, ctypes.byref(plan)) == tv.TV_ERR_INVALID_ARG
    assert prep(arr, 2, 256, need, tv.PATH_PER_TET, ctypes.byref(plan)) == tv.TV_ERR_INVALID_ARG
    assert b"per-tet" in lib.tv_last_error()
    assert prep(arr, 2, 256, need - 256, 0, ctypes.byref(plan)) == tv.TV_ERR_WORKSPACE
    assert prep(arr, 2, 0, need, 0, ctypes.byref(plan)) == tv.TV_ERR_WORKSPACE
    assert prep((tv.MeshC * 2)(good, bad), 2, 256, need, 0, ctypes.byref(plan)) == tv.TV_ERR_UNSUPPORTED_DIMS
    assert b"mesh 1" in lib.tv_last_error()
    assert plan.check == 0  # a failed prepare leaves no usable plan
    # a plan that tv_batch_prepare did not fill (or that was edited) is refused
    assert lib.tv_batch_run(ctypes.byref(plan), P(256), need, None) == tv.TV_ERR_INVALID_ARG
    forged = tv.BatchPlanC(meshes=2, nv=8, nt=2, ntiles=2, ws=256, flags=0, check=12345)
    assert lib.tv_batch_run(ctypes.byref(forged), P(256), need, None) == tv.TV_ERR_INVALID_ARG
    assert b"tv_batch_prepare" in lib.tv_last_error()
    assert lib.tv_batch_run(None, P(256), need, None) == tv.TV_ERR_INVALID_ARG


def test_launch_parameters(lib):
    """tv_params: defaults, validation (nothing changes on an error), reset,
    and workspace sizes that follow the tile fields."""
    assert tv.default_params("single") == {"tile_cols_log2": 5, "min_tiles": 512, "chunk_pieces": 0,
                                           "strip_columns": 6, "piece_cap": 8, "wgs_per_cu": 2,
                                           "cull_columns": 3}
    assert tv.default_params("batch")["cull_columns"] == 6
    assert tv.default_params("batch")["min_tiles"] == 1
    try:
        base = tv.workspace_bytes(1000, 1000, (256, 256, 256))
        tv.set_params("single", strip_columns=3, chunk_pieces=64, piece_cap=1, wgs_per_cu=8)
        assert tv.get_params("single")["strip_columns"] == 3
        assert tv.workspace_bytes(1000, 1000, (256, 256, 256)) == base  # no tile field changed
        tv.set_params("single", tile_cols_log2=3)  # 8x8-column tiles: more tile counters
        assert tv.workspace_bytes(1000, 1000, (256, 256, 256)) > base
        before = tv.get_params("single")
        for bad in ({"tile_cols_log2": 6}, {"tile_cols_log2": 2}, {"min_tiles": 0}, {"chunk_pieces": 63},
                    {"chunk_pieces": -1}, {"strip_columns": 0}, {"strip_columns": 65}, {"piece_cap": 9},
                    {"wgs_per_cu": 0}, {"cull_columns": -1}, {"cull_columns": 1025}):
            with pytest.raises(tv.TVError):
                tv.set_params("single", **bad)
            assert tv.get_params("single") == before
        assert tv.get_params("batch") == tv.default_params("batch")  # the other set is untouched
        P = tv.ParamsC()
        assert lib.tv_get_params(2, ctypes.byref(P)) == tv.TV_ERR_INVALID_ARG
        assert lib.tv_set_params(-1, None) == tv.TV_ERR_INVALID_ARG
    finally:
        tv.set_params("single", None)
    assert tv.get_params("single") == tv.default_params("single")


def test_tune_cache_roundtrip(tmp_path):
    """The tuner's JSON cache: entries stored by key are applied by key; a
    missing key changes nothing."""
    from paper_2106_01326_amd import tune

    path = str(tmp_path / "tune.json")
    params = dict(tv.default_params("batch"), strip_columns=12, chunk_pieces=2048)
    tune._store(path, "gfx950:batch:n2^10:nt2^25", {"params": params, "ms_default": 3.7, "ms_best": 3.5})
    assert tune.cached("gfx950:batch:n2^10:nt2^25", path)["params"] == params
    try:
        assert not tune.apply_cached("batch", "gfx950:batch:other", path)
        assert tv.get_params("batch") == tv.default_params("batch")
        assert tune.apply_cached("batch", "gfx950:batch:n2^10:nt2^25", path)
        assert tv.get_params("batch") == params
    finally:
        tv.set_params("batch", None)
    assert tune.size_class_single(5_557_093, (1024, 1024, 1024)) == "nt2^22:dims1024x1024x1024"
    assert tune.size_class_batch(1024, 42_800_000) == "n2^10:nt2^25"


def test_noalloc_host_checks(lib):
    """tv_voxelize_noalloc refuses what the host can see before touching the
    device: sizes beyond its fixed scratch array and flags it does not take."""
    import re

    from helpers import ROOT

    text = open(os.path.join(ROOT, "include", "tv.h")).read()
    m = re.search(r"#define TV_NOALLOC_MAX_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == tv.NOALLOC_MAX_BYTES
    P = ctypes.c_void_p
    d = tv.Dims(32, 32, 32)
    box = tv._bbox(((0, 0, 0), (1, 1, 1)))
    big = tv.NOALLOC_MAX_BYTES // 40
    assert tv.workspace_bytes(4, big, (32, 32, 32)) > tv.NOALLOC_MAX_BYTES
    call = lib.tv_voxelize_noalloc
    assert call(P(256), 4, P(256), big, d, box, P(256), None, None, 0) == tv.TV_ERR_WORKSPACE
    assert call(P(256), 4, P(256), 1, d, box, P(256), None, None, tv.ACCUMULATE) == tv.TV_ERR_INVALID_ARG
    assert call(P(256), 4, P(256), 1, d, box, P(256), None, None, tv.PATH_PER_TET) == tv.TV_ERR_INVALID_ARG
    assert call(P(256), 4, P(256), 1, d, box, None, None, None, 0) == tv.TV_ERR_INVALID_ARG
    assert call(P(256), 4, P(256), 1, tv.Dims(32, 24, 32), box, P(256), None, None, 0) == \
        tv.TV_ERR_UNSUPPORTED_DIMS
    bad = tv._bbox(((0, 0, 0), (1, 0, 1)))
    assert call(P(256), 4, P(256), 1, d, bad, P(256), None, None, 0) == tv.TV_ERR_INVALID_ARG


def test_export_host_checks(lib):
    """tv_export_batch refuses bad arguments before touching the device."""
    P = ctypes.c_void_p
    ref = (tv.GridRefC * 1)(tv.GridRefC(P(256), tv.Dims(32, 32, 32)))
    call = lib.tv_export_batch
    ws_n = lib.tv_export_workspace_bytes(1)
    assert ws_n >= 256 and ws_n % 256 == 0 and lib.tv_export_workspace_bytes(0) == 0
    a = ctypes.cast(ref, P)
    assert call(a, 1, 12, 0, P(256), P(256), ws_n, None) == tv.TV_ERR_INVALID_ARG  # res not a power of two
    assert call(a, 1, 2048, 0, P(256), P(256), ws_n, None) == tv.TV_ERR_INVALID_ARG
    assert call(a, 1, 32, 5, P(256), P(256), ws_n, None) == tv.TV_ERR_INVALID_ARG  # mode
    assert call(a, 0, 32, 0, P(256), P(256), ws_n, None) == tv.TV_ERR_INVALID_ARG
    assert call(a, 1, 32, 0, None, P(256), ws_n, None) == tv.TV_ERR_INVALID_ARG
    assert call(a, 1, 32, 0, P(256), P(260), ws_n, None) == tv.TV_ERR_WORKSPACE
    assert call(a, 1, 32, 0, P(256), P(256), 16, None) == tv.TV_ERR_WORKSPACE
    bad = (tv.GridRefC * 1)(tv.GridRefC(P(256), tv.Dims(32, 24, 32)))
    assert call(ctypes.cast(bad, P), 1, 32, 0, P(256), P(256), ws_n, None) == tv.TV_ERR_UNSUPPORTED_DIMS
    # pooling 1024^3 to one cell would count 2^30 voxels in a float
    big = (tv.GridRefC * 1)(tv.GridRefC(P(256), tv.Dims(1024, 1024, 1024)))
    assert call(ctypes.cast(big, P), 1, 1, 0, P(256), P(256), ws_n, None) == tv.TV_ERR_INVALID_ARG


def test_bricks_voxelize_host_checks(lib):
    """tv_voxelize_bricks refuses what the host can see: dims below one brick
    or not powers of two, null outputs, capacity, flags, workspace."""
    P = ctypes.c_void_p
    box = tv._bbox(((0, 0, 0), (1, 1, 1)))
    ws_n = lib.tv_voxelize_bricks_workspace_bytes(4, 1, tv.Dims(64, 64, 64))
    assert ws_n > tv.workspace_bytes(4, 1, (64, 64, 64)) - 1 and ws_n % 256 == 0

    def call(dims=(64, 64, 64), index=256, pool=256, ids=256, cap=16, count=256, ws=256, ws_bytes=None, flags=0):
        return lib.tv_voxelize_bricks(P(256), 4, P(256), 1, tv.Dims(*dims), box, P(index), P(pool), P(ids), cap,
                                      P(count), P(ws), ws_n if ws_bytes is None else ws_bytes, None, flags)

    assert call(dims=(4, 64, 64)) == tv.TV_ERR_UNSUPPORTED_DIMS   # below 8 columns
    assert call(dims=(64, 64, 16)) == tv.TV_ERR_UNSUPPORTED_DIMS  # below one word
    assert call(dims=(64, 48, 64)) == tv.TV_ERR_UNSUPPORTED_DIMS
    assert call(index=0) == tv.TV_ERR_INVALID_ARG
    assert call(count=0) == tv.TV_ERR_INVALID_ARG
    assert call(pool=0) == tv.TV_ERR_INVALID_ARG
    assert call(cap=-1) == tv.TV_ERR_INVALID_ARG
    assert call(flags=tv.ACCUMULATE) == tv.TV_ERR_INVALID_ARG
    assert call(ws=0) == tv.TV_ERR_WORKSPACE
    assert call(ws_bytes=ws_n - 256) == tv.TV_ERR_WORKSPACE
