"""gfx950 tetrahedral-mesh voxelizer: thin Python binding over the C ABI.

Every function here only marshals arguments (torch tensors -> device
pointers, the current HIP stream) and calls ``libtetvox.so``; all work runs in
the library's HIP kernels.  Importing works without a GPU; calling a compute
function requires the built library and a GPU, and raises otherwise -- there
is no CPU fallback.

Grids are returned as torch.int32 tensors holding the uint32 words of the
layout in include/tv.h: voxel (i,j,k) is bit k%32 of word
(i*ny + j)*ceil(nz/32) + k//32.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "_lib", "libtetvox.so")

TV_OK = 0
TV_ERR_INVALID_ARG = -1
TV_ERR_UNSUPPORTED_DIMS = -2
TV_ERR_INDEX = -3
TV_ERR_RANGE = -4
TV_ERR_WORKSPACE = -5
TV_ERR_HIP = -7
TV_ERR_TOO_LARGE = -8
TV_ERR_TIMEOUT = -9
TV_ERR_NOT_FOUND = -10
TV_ERR_IO = -11

TIE_HALF_OPEN = 0
TIE_STRICT = 1
ACCUMULATE = 8
PATH_PER_TET = 2
Q_INVALID = -(1 << 31)

VERTS_F32 = 0
VERTS_Q32 = 1

EXPORTED = ("tv_grid_words", "tv_workspace_bytes", "tv_voxelize", "tv_voxelize_q", "tv_snap",
            "tv_batch_workspace_bytes", "tv_voxelize_batch", "tv_batch_prepare", "tv_batch_run",
            "tv_default_params", "tv_get_params", "tv_set_params",
            "tv_fetch_status", "tv_status_string", "tv_last_error", "tv_profile_enable",
            "tv_profile_read", "tv_profile_stage_name", "tv_server_create", "tv_server_submit",
            "tv_server_poll", "tv_server_wait", "tv_server_result", "tv_server_copy_grid",
            "tv_server_release", "tv_server_get_stats", "tv_server_destroy", "tv_unpack", "tv_pool",
            "tv_brick_count_max", "tv_bricks_workspace_bytes", "tv_bricks", "tv_read_mesh",
            "tv_free_host_mesh", "tv_quality_workspace_bytes", "tv_mesh_quality",
            "tv_voxelize_pipelined", "tv_voxelize_noalloc", "tv_export_workspace_bytes", "tv_export_batch",
            "tv_voxelize_bricks", "tv_voxelize_bricks_workspace_bytes")

BRICK_FULL = 0xFFFFFFFF
BRICK_UNUSED = 0xFFFFFFFF
EXPORT_FRACTION = 0
EXPORT_ANY = 1
UNPACK_U8 = 0
UNPACK_F32 = 1
POOL_FRACTION = 0
POOL_ANY = 1

REQ_HOST_INPUTS = 0
REQ_PINNED_INPUTS = 4
REQ_DEVICE_INPUTS = 8
REQ_DONE = 2


class Dims(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32)]


class BBox(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_float * 3), ("hi", ctypes.c_float * 3)]


class MeshC(ctypes.Structure):
    _fields_ = [("verts", ctypes.c_void_p), ("vert_format", ctypes.c_uint32), ("nv", ctypes.c_int64),
                ("tets", ctypes.c_void_p), ("nt", ctypes.c_int64), ("dims", Dims), ("bbox", BBox),
                ("grid", ctypes.c_void_p)]


class BatchPlanC(ctypes.Structure):
    _fields_ = [("meshes", ctypes.c_int64), ("nv", ctypes.c_int64), ("nt", ctypes.c_int64),
                ("ntiles", ctypes.c_int64), ("ws", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("launch", ctypes.c_int32 * 5), ("check", ctypes.c_uint32)]


PARAM_FIELDS = ("tile_cols_log2", "min_tiles", "chunk_pieces", "strip_columns", "piece_cap", "wgs_per_cu",
                "cull_columns")
PARAMS_SINGLE = 0
PARAMS_BATCH = 1


class ParamsC(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in PARAM_FIELDS]


class HostMeshC(ctypes.Structure):
    _fields_ = [("verts", ctypes.c_void_p), ("nv", ctypes.c_int64), ("tets", ctypes.c_void_p),
                ("nt", ctypes.c_int64), ("bbox", BBox), ("skipped_elements", ctypes.c_int64)]


class GridRefC(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_void_p), ("dims", Dims)]


class QualityC(ctypes.Structure):
    _fields_ = [("tets", ctypes.c_int64), ("invalid", ctypes.c_int64), ("degenerate", ctypes.c_int64),
                ("inverted", ctypes.c_int64), ("min_dihedral_below", ctypes.c_int64 * 4),
                ("min_dihedral_deg", ctypes.c_double), ("mean_min_dihedral_deg", ctypes.c_double),
                ("volume_mean", ctypes.c_double), ("volume_cv", ctypes.c_double),
                ("covered_voxels", ctypes.c_int64), ("occupied_voxels", ctypes.c_int64)]


class RequestC(ctypes.Structure):
    _fields_ = [("verts", ctypes.c_void_p), ("vert_format", ctypes.c_uint32), ("nv", ctypes.c_int64),
                ("tets", ctypes.c_void_p), ("nt", ctypes.c_int64), ("dims", Dims), ("bbox", BBox),
                ("flags", ctypes.c_uint32)]


class ServerConfigC(ctypes.Structure):
    _fields_ = [("device_bytes", ctypes.c_size_t), ("pinned_bytes", ctypes.c_size_t),
                ("streams", ctypes.c_int32), ("max_wave_meshes", ctypes.c_int32)]


class ServerStatsC(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("released", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("waves", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("running", ctypes.c_int64), ("inflight_waves", ctypes.c_int64),
                ("device_in_use", ctypes.c_size_t), ("device_peak", ctypes.c_size_t),
                ("pinned_in_use", ctypes.c_size_t), ("inflight_peak", ctypes.c_int64)]


class TVError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"{status_name(code)}: {msg}" if msg else status_name(code))
        self.code = code


_lib = None


def library_path() -> str:
    return LIB_PATH


def load_library():
    """Load libtetvox.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2106_01326_amd.build` (no CPU fallback exists)")
    # torch ships its own HIP runtime and loads it under a file name that the
    # loader does not match against an already loaded /opt/rocm runtime;
    # loading torch first makes this library bind to torch's runtime, so the
    # process has exactly one.
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    u32 = ctypes.c_uint32
    st = ctypes.c_int32
    lib.tv_grid_words.argtypes = [Dims]
    lib.tv_grid_words.restype = ctypes.c_size_t
    lib.tv_workspace_bytes.argtypes = [i64, i64, Dims, u32]
    lib.tv_workspace_bytes.restype = ctypes.c_size_t
    lib.tv_voxelize.argtypes = [P, i64, P, i64, Dims, BBox, P, P, ctypes.c_size_t, P, u32]
    lib.tv_voxelize.restype = st
    lib.tv_voxelize_q.argtypes = [P, i64, P, i64, Dims, P, P, ctypes.c_size_t, P, u32]
    lib.tv_voxelize_q.restype = st
    lib.tv_voxelize_noalloc.argtypes = [P, i64, P, i64, Dims, BBox, P, P, P, u32]
    lib.tv_voxelize_noalloc.restype = st
    lib.tv_voxelize_bricks.argtypes = [P, i64, P, i64, Dims, BBox, P, P, P, i64, P, P, ctypes.c_size_t, P, u32]
    lib.tv_voxelize_bricks.restype = st
    lib.tv_voxelize_bricks_workspace_bytes.argtypes = [i64, i64, Dims]
    lib.tv_voxelize_bricks_workspace_bytes.restype = ctypes.c_size_t
    lib.tv_batch_workspace_bytes.argtypes = [P, ctypes.c_int32, u32]
    lib.tv_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.tv_voxelize_batch.argtypes = [P, ctypes.c_int32, P, ctypes.c_size_t, P, u32]
    lib.tv_voxelize_batch.restype = st
    lib.tv_batch_prepare.argtypes = [P, ctypes.c_int32, P, ctypes.c_size_t, P, u32,
                                     ctypes.POINTER(BatchPlanC)]
    lib.tv_batch_prepare.restype = st
    lib.tv_batch_run.argtypes = [ctypes.POINTER(BatchPlanC), P, ctypes.c_size_t, P]
    lib.tv_batch_run.restype = st
    for name in ("tv_default_params", "tv_get_params", "tv_set_params"):
        getattr(lib, name).argtypes = [ctypes.c_int32, ctypes.POINTER(ParamsC)]
        getattr(lib, name).restype = st
    lib.tv_snap.argtypes = [P, i64, BBox, P, P]
    lib.tv_snap.restype = st
    lib.tv_fetch_status.argtypes = [P, ctypes.c_int32, P]
    lib.tv_fetch_status.restype = st
    lib.tv_status_string.argtypes = [st]
    lib.tv_status_string.restype = ctypes.c_char_p
    lib.tv_last_error.argtypes = []
    lib.tv_last_error.restype = ctypes.c_char_p
    lib.tv_server_create.argtypes = [P, P]
    lib.tv_server_create.restype = st
    lib.tv_server_submit.argtypes = [P, P, P]
    lib.tv_server_submit.restype = st
    lib.tv_server_poll.argtypes = [P, i64, P]
    lib.tv_server_poll.restype = st
    lib.tv_server_wait.argtypes = [P, i64, ctypes.c_double]
    lib.tv_server_wait.restype = st
    lib.tv_server_result.argtypes = [P, i64, P, P, P, P]
    lib.tv_server_result.restype = st
    lib.tv_server_copy_grid.argtypes = [P, i64, P, ctypes.c_size_t]
    lib.tv_server_copy_grid.restype = st
    lib.tv_server_release.argtypes = [P, i64]
    lib.tv_server_release.restype = st
    lib.tv_server_get_stats.argtypes = [P, P]
    lib.tv_server_get_stats.restype = st
    lib.tv_server_destroy.argtypes = [P]
    lib.tv_server_destroy.restype = st
    lib.tv_profile_enable.argtypes = [ctypes.c_int32]
    lib.tv_profile_enable.restype = st
    lib.tv_profile_read.argtypes = [P, ctypes.c_int32, P, P]
    lib.tv_profile_read.restype = st
    lib.tv_profile_stage_name.argtypes = [ctypes.c_int32]
    lib.tv_profile_stage_name.restype = ctypes.c_char_p
    lib.tv_read_mesh.argtypes = [ctypes.c_char_p, P]
    lib.tv_read_mesh.restype = st
    lib.tv_free_host_mesh.argtypes = [P]
    lib.tv_free_host_mesh.restype = None
    lib.tv_voxelize_pipelined.argtypes = [P, i64, P, i64, Dims, BBox, P, P, P, P, ctypes.c_size_t, P, P,
                                          ctypes.c_int32, u32]
    lib.tv_voxelize_pipelined.restype = st
    lib.tv_quality_workspace_bytes.argtypes = [i64]
    lib.tv_quality_workspace_bytes.restype = ctypes.c_size_t
    lib.tv_mesh_quality.argtypes = [P, u32, i64, P, i64, Dims, BBox, P, u32, P, ctypes.c_size_t, P, P]
    lib.tv_mesh_quality.restype = st
    lib.tv_unpack.argtypes = [P, Dims, P, u32, P]
    lib.tv_unpack.restype = st
    lib.tv_pool.argtypes = [P, Dims, ctypes.c_int32, u32, P, P]
    lib.tv_pool.restype = st
    lib.tv_brick_count_max.argtypes = [Dims]
    lib.tv_brick_count_max.restype = i64
    lib.tv_bricks_workspace_bytes.argtypes = [Dims]
    lib.tv_bricks_workspace_bytes.restype = ctypes.c_size_t
    lib.tv_bricks.argtypes = [P, Dims, P, P, i64, P, P, ctypes.c_size_t, P]
    lib.tv_bricks.restype = st
    lib.tv_export_workspace_bytes.argtypes = [ctypes.c_int32]
    lib.tv_export_workspace_bytes.restype = ctypes.c_size_t
    lib.tv_export_batch.argtypes = [P, ctypes.c_int32, ctypes.c_int32, u32, P, P, ctypes.c_size_t, P]
    lib.tv_export_batch.restype = st
    _lib = lib
    return lib


def status_name(code: int) -> str:
    try:
        return load_library().tv_status_string(code).decode()
    except RuntimeError:
        return f"status {code}"


def _check(code: int):
    if code != TV_OK:
        raise TVError(code, load_library().tv_last_error().decode())


def _dims(dims) -> Dims:
    nx, ny, nz = (int(d) for d in dims)
    return Dims(nx, ny, nz)


def grid_words(dims) -> int:
    return int(load_library().tv_grid_words(_dims(dims)))


def workspace_bytes(nv: int, nt: int, dims, flags: int = 0) -> int:
    return int(load_library().tv_workspace_bytes(int(nv), int(nt), _dims(dims), int(flags)))


def _torch():
    import torch

    return torch


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t, dtype, shape_tail, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if shape_tail is not None and (t.dim() != 2 or t.shape[1] != shape_tail):
        raise ValueError(f"{name} must have shape [n, {shape_tail}]")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr()), int(t.shape[0])


def alloc_workspace(nbytes: int, device=None):
    torch = _torch()
    # torch's caching allocator returns 512-byte aligned blocks
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8,
                       device=device if device is not None else "cuda")


def alloc_grid(dims, device=None):
    torch = _torch()
    return torch.empty(grid_words(dims), dtype=torch.int32,
                       device=device if device is not None else "cuda")


def _bbox(bbox) -> BBox:
    lo, hi = bbox
    return BBox((ctypes.c_float * 3)(*[float(x) for x in lo]), (ctypes.c_float * 3)(*[float(x) for x in hi]))


def voxelize(verts, tets, dims, bbox=None, *, qverts=False, strict=False, per_tet=False, grid=None,
             workspace=None, stream=None, accumulate=False):
    """Voxelize one mesh on the GPU (asynchronous on ``stream``).

    verts: [nv,3] float32 world coordinates (``qverts=False``, needs ``bbox``
    = (lo[3], hi[3])) or [nv,3] int32 lattice coordinates (``qverts=True``).
    tets: [nt,4] int32.  ``per_tet`` selects the reference path.
    ``accumulate`` ORs into ``grid`` instead of overwriting it.  Returns
    (grid, workspace); call ``fetch_status`` on the workspace to read
    device-side data errors.
    """
    lib = load_library()
    torch = _torch()
    d = _dims(dims)
    flags = (TIE_STRICT if strict else TIE_HALF_OPEN) | (PATH_PER_TET if per_tet else 0) | \
        (ACCUMULATE if accumulate else 0)
    if accumulate and grid is None:
        raise ValueError("accumulate needs the grid to add to")
    vptr, nv = _dev_ptr(verts, torch.int32 if qverts else torch.float32, 3, "verts")
    tptr, nt = _dev_ptr(tets, torch.int32, 4, "tets")
    if grid is None:
        grid = alloc_grid(dims, verts.device)
    gptr, _ = _dev_ptr(grid, torch.int32, None, "grid")
    if grid.numel() < grid_words(dims):
        raise ValueError("grid tensor too small")
    need = workspace_bytes(nv, nt, dims, flags)
    if workspace is None:
        workspace = alloc_workspace(need, verts.device)
        if accumulate:
            workspace.zero_()  # an accumulating call keeps the status words it finds
    wptr, _ = _dev_ptr(workspace, torch.uint8, None, "workspace")
    s = _stream_handle(stream)
    if qverts:
        rc = lib.tv_voxelize_q(vptr, nv, tptr, nt, d, gptr, wptr, workspace.numel(), s, flags)
    else:
        if bbox is None:
            raise ValueError("fp32 vertices need a bbox")
        rc = lib.tv_voxelize(vptr, nv, tptr, nt, d, _bbox(bbox), gptr, wptr, workspace.numel(), s, flags)
    _check(rc)
    return grid, workspace


NOALLOC_MAX_BYTES = 64 << 20  # TV_NOALLOC_MAX_BYTES


def voxelize_noalloc(verts, tets, dims, bbox, *, strict=False, grid=None, status=None, stream=None):
    """Voxelize one mesh (fp32 world coordinates) with the library's fixed
    per-GPU scratch array instead of a workspace (tv_voxelize_noalloc).
    ``grid`` and ``status`` (a one-element int32 device tensor receiving the
    data-error status) are allocated here when not given; pass them to keep
    the call free of allocations.  Returns (grid, status)."""
    lib = load_library()
    torch = _torch()
    d = _dims(dims)
    vptr, nv = _dev_ptr(verts, torch.float32, 3, "verts")
    tptr, nt = _dev_ptr(tets, torch.int32, 4, "tets")
    if grid is None:
        grid = alloc_grid(dims, verts.device)
    gptr, _ = _dev_ptr(grid, torch.int32, None, "grid")
    if grid.numel() < grid_words(dims):
        raise ValueError("grid tensor too small")
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=verts.device)
    sptr, _ = _dev_ptr(status, torch.int32, None, "status")
    rc = lib.tv_voxelize_noalloc(vptr, nv, tptr, nt, d, _bbox(bbox), gptr, sptr, _stream_handle(stream),
                                 TIE_STRICT if strict else TIE_HALF_OPEN)
    _check(rc)
    return grid, status


class Export:
    """The (grid, dims) list of a batch export, marshalled once
    (tv_export_batch takes it as a host array); ``run`` exports the grids'
    current contents.  ``grids``: list of (grid tensor, dims)."""

    def __init__(self, grids):
        torch = _torch()
        self.n = len(grids)
        if self.n == 0:
            raise ValueError("no grids")
        self.grids = list(grids)  # keeps the tensors alive
        self.array = (GridRefC * self.n)()
        for i, (g, dims) in enumerate(self.grids):
            gptr, _ = _dev_ptr(g, torch.int32, None, f"grids[{i}]")
            if g.numel() < grid_words(dims):
                raise ValueError(f"grids[{i}] tensor too small for dims {dims}")
            self.array[i] = GridRefC(gptr, _dims(dims))
        self.device = self.grids[0][0].device

    def run(self, res, mode="fraction", *, out=None, workspace=None, stream=None):
        """One dense [n, res, res, res] tensor: float32 fractions
        (``mode="fraction"``) or uint8 occupancy (``mode="any"``)."""
        lib = load_library()
        torch = _torch()
        code = {"fraction": EXPORT_FRACTION, "any": EXPORT_ANY}[mode]
        dt = torch.float32 if code == EXPORT_FRACTION else torch.uint8
        if out is None:
            out = torch.empty((self.n, res, res, res), dtype=dt, device=self.device)
        optr, _ = _dev_ptr(out, dt, None, "out")
        if out.numel() < self.n * res ** 3:
            raise ValueError("out too small")
        if workspace is None:
            workspace = alloc_workspace(int(lib.tv_export_workspace_bytes(self.n)), self.device)
        wptr, _ = _dev_ptr(workspace, torch.uint8, None, "workspace")
        _check(lib.tv_export_batch(ctypes.cast(self.array, ctypes.c_void_p), self.n, int(res), code, optr, wptr,
                                   workspace.numel(), _stream_handle(stream)))
        return out


def export_batch(grids, res, mode="fraction", *, out=None, workspace=None, stream=None):
    """Many grids of any dims -> one dense [n, res, res, res] tensor in one
    launch (tv_export_batch); see ``Export`` to marshal the list once."""
    return Export(grids).run(res, mode, out=out, workspace=workspace, stream=stream)


def bricks_workspace_bytes(nv: int, nt: int, dims) -> int:
    return int(load_library().tv_voxelize_bricks_workspace_bytes(int(nv), int(nt), _dims(dims)))


def brick_count_max(dims) -> int:
    return int(load_library().tv_brick_count_max(_dims(dims)))


def voxelize_bricks(verts, tets, dims, bbox, capacity, *, strict=False, index=None, pool=None, ids=None,
                    count=None, workspace=None, stream=None):
    """Voxelize one mesh (fp32 world coordinates) straight into sparse bricks
    (tv_voxelize_bricks).  Returns (index, pool, ids, count, workspace): int32
    tensors holding the uint32 outputs (index [bricks], pool [capacity, 64],
    ids [capacity], count [1]); read data errors and pool overflow with
    ``fetch_status(workspace)``."""
    lib = load_library()
    torch = _torch()
    vptr, nv = _dev_ptr(verts, torch.float32, 3, "verts")
    tptr, nt = _dev_ptr(tets, torch.int32, 4, "tets")
    dev = verts.device
    nb = brick_count_max(dims)
    capacity = int(capacity)
    if index is None:
        index = torch.empty(max(nb, 1), dtype=torch.int32, device=dev)
    if pool is None:
        pool = torch.empty((max(capacity, 1), 64), dtype=torch.int32, device=dev)
    if ids is None:
        ids = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
    if count is None:
        count = torch.empty(1, dtype=torch.int32, device=dev)
    if index.numel() < nb or pool.numel() < 64 * capacity or ids.numel() < capacity:
        raise ValueError("index, pool or ids too small")
    iptr, _ = _dev_ptr(index, torch.int32, None, "index")
    pptr, _ = _dev_ptr(pool, torch.int32, None, "pool")
    dptr, _ = _dev_ptr(ids, torch.int32, None, "ids")
    cptr, _ = _dev_ptr(count, torch.int32, None, "count")
    flags = TIE_STRICT if strict else TIE_HALF_OPEN
    need = bricks_workspace_bytes(nv, nt, dims)
    if workspace is None:
        workspace = alloc_workspace(need, dev)
    wptr, _ = _dev_ptr(workspace, torch.uint8, None, "workspace")
    _check(lib.tv_voxelize_bricks(vptr, nv, tptr, nt, _dims(dims), _bbox(bbox), iptr, pptr, dptr, capacity, cptr,
                                  wptr, workspace.numel(), _stream_handle(stream), flags))
    return index, pool, ids, count, workspace


def voxelize_pipelined(verts_host, tets_host, dims, bbox, chunks=8, *, strict=False, per_tet=False,
                       verts_dev=None, tets_dev=None, grid=None, workspace=None, stream=None,
                       copy_stream=None):
    """Voxelize host inputs (pinned CPU tensors for overlap) with the copies
    of tet slices overlapped with the voxelization of earlier slices; returns
    (grid, workspace, verts_dev, tets_dev).  ``copy_stream`` defaults to a
    new torch stream."""
    lib = load_library()
    torch = _torch()
    for t, dt, w, name in ((verts_host, torch.float32, 3, "verts_host"), (tets_host, torch.int32, 4, "tets_host")):
        if not isinstance(t, torch.Tensor) or t.is_cuda or t.dtype != dt or t.dim() != 2 or t.shape[1] != w \
                or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous host {dt} tensor of shape [n, {w}]")
    nv, nt = int(verts_host.shape[0]), int(tets_host.shape[0])
    dev = torch.device("cuda", torch.cuda.current_device())
    verts_dev = torch.empty((nv, 3), dtype=torch.float32, device=dev) if verts_dev is None else verts_dev
    tets_dev = torch.empty((nt, 4), dtype=torch.int32, device=dev) if tets_dev is None else tets_dev
    grid = alloc_grid(dims, dev) if grid is None else grid
    k = max(1, min(int(chunks), 64))
    per = (nt + k - 1) // k if nt else 0
    flags = (TIE_STRICT if strict else TIE_HALF_OPEN) | (PATH_PER_TET if per_tet else 0)
    if workspace is None:
        workspace = alloc_workspace(workspace_bytes(nv, per, dims, flags), dev)
    copy_stream = copy_stream if copy_stream is not None else torch.cuda.Stream()
    _check(lib.tv_voxelize_pipelined(
        ctypes.c_void_p(verts_host.data_ptr()), nv, ctypes.c_void_p(tets_host.data_ptr()), nt, _dims(dims),
        _bbox(bbox), ctypes.c_void_p(verts_dev.data_ptr()), ctypes.c_void_p(tets_dev.data_ptr()),
        ctypes.c_void_p(grid.data_ptr()), ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
        _stream_handle(stream), ctypes.c_void_p(copy_stream.cuda_stream), k, flags))
    return grid, workspace, verts_dev, tets_dev


def snap(verts, bbox, out=None, stream=None):
    """fp32 world coordinates [nv,3] -> int32 lattice coordinates [nv,3] on
    the device (bad vertices come back as Q_INVALID)."""
    lib = load_library()
    torch = _torch()
    vptr, nv = _dev_ptr(verts, torch.float32, 3, "verts")
    if out is None:
        out = torch.empty((nv, 3), dtype=torch.int32, device=verts.device)
    optr, _ = _dev_ptr(out, torch.int32, 3, "out")
    _check(lib.tv_snap(vptr, nv, _bbox(bbox), optr, _stream_handle(stream)))
    return out


def fetch_status(workspace, mesh_index: int = 0, stream=None) -> int:
    """Device-side data-error status of a finished call (synchronizes)."""
    lib = load_library()
    torch = _torch()
    wptr, _ = _dev_ptr(workspace, torch.uint8, None, "workspace")
    return int(lib.tv_fetch_status(wptr, int(mesh_index), _stream_handle(stream)))


def read_mesh(path):
    """Read a MEDIT .mesh or Gmsh .msh (ASCII) tet mesh with the native reader:
    (verts float32 [nv, 3], tets int32 [nt, 4] 0-based, bbox ((lo), (hi)),
    skipped non-tet elements), as host numpy arrays."""
    import numpy as np

    lib = load_library()
    m = HostMeshC()
    _check(lib.tv_read_mesh(os.fsencode(path), ctypes.byref(m)))
    try:
        verts = np.ctypeslib.as_array(ctypes.cast(m.verts, ctypes.POINTER(ctypes.c_float)),
                                      shape=(m.nv * 3,)).reshape(m.nv, 3).copy() if m.nv else \
            np.zeros((0, 3), np.float32)
        tets = np.ctypeslib.as_array(ctypes.cast(m.tets, ctypes.POINTER(ctypes.c_int32)),
                                     shape=(m.nt * 4,)).reshape(m.nt, 4).copy() if m.nt else \
            np.zeros((0, 4), np.int32)
        bbox = (tuple(m.bbox.lo), tuple(m.bbox.hi))
        return verts, tets, bbox, int(m.skipped_elements)
    finally:
        lib.tv_free_host_mesh(ctypes.byref(m))


def quality(verts, tets, dims, bbox, grid, *, qverts=False, strict=False, workspace=None, stream=None):
    """Mesh quality report (see tv_mesh_quality): a dict of the counts,
    dihedral-angle and volume statistics, and covered vs occupied voxels of
    ``grid`` (the grid of these tets at ``dims``).  Synchronizes."""
    lib = load_library()
    torch = _torch()
    vptr, nv = _dev_ptr(verts, torch.int32 if qverts else torch.float32, 3, "verts")
    tptr, nt = _dev_ptr(tets, torch.int32, 4, "tets")
    need = int(lib.tv_quality_workspace_bytes(nv))
    if workspace is None:
        workspace = alloc_workspace(need, verts.device)
    wptr, _ = _dev_ptr(workspace, torch.uint8, None, "workspace")
    out = QualityC()
    _check(lib.tv_mesh_quality(vptr, VERTS_Q32 if qverts else VERTS_F32, nv, tptr, nt, _dims(dims),
                               _bbox(bbox), _grid_ptr(grid, dims), TIE_STRICT if strict else 0, wptr,
                               workspace.numel(), _stream_handle(stream), ctypes.byref(out)))
    r = {k: getattr(out, k) for k, _ in QualityC._fields_}
    r["min_dihedral_below"] = list(out.min_dihedral_below)
    return r


def _grid_ptr(grid, dims):
    torch = _torch()
    if not isinstance(grid, torch.Tensor) or not grid.is_cuda or grid.dtype not in (torch.int32, torch.uint32):
        raise TypeError("grid must be a device int32/uint32 tensor")
    if not grid.is_contiguous() or grid.numel() < grid_words(dims):
        raise ValueError("grid must be contiguous with tv_grid_words(dims) words")
    return ctypes.c_void_p(grid.data_ptr())


def unpack(grid, dims, dtype=None, out=None, stream=None):
    """Dense [nx, ny, nz] tensor of a packed grid (1 = set): uint8 by
    default, or float32."""
    lib = load_library()
    torch = _torch()
    dtype = dtype or torch.uint8
    if dtype not in (torch.uint8, torch.float32):
        raise TypeError("dtype must be uint8 or float32")
    nx, ny, nz = (int(d) for d in dims)
    if out is None:
        out = torch.empty((nx, ny, nz), dtype=dtype, device=grid.device)
    elif out.dtype != dtype or not out.is_contiguous() or out.numel() != nx * ny * nz:
        raise ValueError("out must be a contiguous tensor of nx*ny*nz elements of dtype")
    fmt = UNPACK_U8 if dtype == torch.uint8 else UNPACK_F32
    _check(lib.tv_unpack(_grid_ptr(grid, dims), _dims(dims), ctypes.c_void_p(out.data_ptr()), fmt,
                         _stream_handle(stream)))
    return out


def pool(grid, dims, factor, mode=POOL_FRACTION, out=None, stream=None):
    """Coarser level by ``factor``: float32 [nx/f, ny/f, nz/f] occupancy
    fractions (POOL_FRACTION) or the packed any-grid of dims/f (POOL_ANY)."""
    lib = load_library()
    torch = _torch()
    f = int(factor)
    nx, ny, nz = (int(d) for d in dims)
    if out is None:
        if mode == POOL_FRACTION:
            out = torch.empty((nx // f, ny // f, nz // f), dtype=torch.float32, device=grid.device)
        else:
            out = torch.empty(grid_words((max(nx // f, 1), max(ny // f, 1), max(nz // f, 1))),
                              dtype=torch.int32, device=grid.device)
    _check(lib.tv_pool(_grid_ptr(grid, dims), _dims(dims), f, int(mode), ctypes.c_void_p(out.data_ptr()),
                       _stream_handle(stream)))
    return out


def bricks(grid, dims, capacity=None, stream=None):
    """Non-empty 8x8x32 bricks of a grid in increasing id: (ids uint32 [n],
    words uint32 [n, 64]) as device tensors (synchronizes to read n)."""
    lib = load_library()
    torch = _torch()
    nmax = int(lib.tv_brick_count_max(_dims(dims)))
    cap = nmax if capacity is None else int(capacity)
    dev = grid.device
    ids = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    words = torch.empty((max(cap, 1), 64), dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    wsb = int(lib.tv_bricks_workspace_bytes(_dims(dims)))
    ws = alloc_workspace(wsb, dev)
    _check(lib.tv_bricks(_grid_ptr(grid, dims), _dims(dims), ctypes.c_void_p(ids.data_ptr()),
                         ctypes.c_void_p(words.data_ptr()), cap, ctypes.c_void_p(count.data_ptr()),
                         ctypes.c_void_p(ws.data_ptr()), wsb, _stream_handle(stream)))
    n = int(count.item())
    k = min(n, cap)
    return ids[:k], words[:k], n


def profile_enable(on: bool = True):
    """Enable/disable per-stage HIP-event timing of subsequent calls."""
    _check(load_library().tv_profile_enable(1 if on else 0))


def profile_read() -> tuple[dict, int]:
    """Summed milliseconds per stage since the last read, and the call count
    (waits for the recorded events)."""
    lib = load_library()
    ms = (ctypes.c_double * 16)()
    n = ctypes.c_int32(0)
    calls = ctypes.c_int64(0)
    _check(lib.tv_profile_read(ctypes.cast(ms, ctypes.c_void_p), 16, ctypes.cast(ctypes.pointer(n), ctypes.c_void_p),
                               ctypes.cast(ctypes.pointer(calls), ctypes.c_void_p)))
    out = {lib.tv_profile_stage_name(i).decode(): ms[i] for i in range(n.value)}
    return out, int(calls.value)


def _mesh_struct(verts, tets, dims, bbox, grid, qverts):
    torch = _torch()
    vptr, nv = _dev_ptr(verts, torch.int32 if qverts else torch.float32, 3, "verts")
    tptr, nt = _dev_ptr(tets, torch.int32, 4, "tets")
    gptr, _ = _dev_ptr(grid, torch.int32, None, "grid")
    if grid.numel() < grid_words(dims):
        raise ValueError("grid tensor too small")
    if bbox is None:
        bbox = ((0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    return MeshC(vptr.value, VERTS_Q32 if qverts else VERTS_F32, nv, tptr.value, nt, _dims(dims),
                 _bbox(bbox), gptr.value)


def _params_which(which):
    if which in ("single", PARAMS_SINGLE):
        return PARAMS_SINGLE
    if which in ("batch", PARAMS_BATCH):
        return PARAMS_BATCH
    raise ValueError(f"params set {which!r}: 'single' or 'batch'")


def default_params(which="single"):
    """The library's default launch parameters (tv_default_params) as a dict."""
    p = ParamsC()
    _check(load_library().tv_default_params(_params_which(which), ctypes.byref(p)))
    return {f: int(getattr(p, f)) for f in PARAM_FIELDS}


def get_params(which="single"):
    """Launch parameters in force (tv_get_params) as a dict."""
    p = ParamsC()
    _check(load_library().tv_get_params(_params_which(which), ctypes.byref(p)))
    return {f: int(getattr(p, f)) for f in PARAM_FIELDS}


def set_params(which="single", params=None, **fields):
    """Sets launch parameters (tv_set_params): ``params`` (a dict) updated by
    ``fields``, over the current values; ``set_params(which, None)`` with no
    fields restores the defaults.  Returns the previous setting."""
    lib = load_library()
    w = _params_which(which)
    old = get_params(which)
    if params is None and not fields:
        _check(lib.tv_set_params(w, None))
        return old
    new = dict(old)
    new.update(params or {})
    new.update(fields)
    unknown = set(new) - set(PARAM_FIELDS)
    if unknown:
        raise ValueError(f"unknown parameters {sorted(unknown)}")
    _check(lib.tv_set_params(w, ctypes.byref(ParamsC(*[int(new[f]) for f in PARAM_FIELDS]))))
    return old


class Batch:
    """A prepared batch: device tensors of many meshes and their descriptor
    array, reusable across calls (the grids are overwritten each call)."""

    def __init__(self, items, device=None):
        """items: iterable of (verts, tets, dims, bbox, qverts) with device
        tensors; a grid is allocated per mesh."""
        torch = _torch()
        self.items = list(items)
        self.grids = [alloc_grid(it[2], it[0].device) for it in self.items]
        n = len(self.items)
        self.array = (MeshC * n)()
        for i, ((v, t, dims, bbox, q), g) in enumerate(zip(self.items, self.grids)):
            self.array[i] = _mesh_struct(v, t, dims, bbox, g, q)
        self.n = n
        need = int(load_library().tv_batch_workspace_bytes(ctypes.cast(self.array, ctypes.c_void_p), n, 0))
        if need == 0:
            _check(TV_ERR_INVALID_ARG)
        self.workspace = alloc_workspace(need, self.items[0][0].device if n else device)
        del torch

    def run(self, strict=False, per_tet=False, stream=None):
        flags = (TIE_STRICT if strict else TIE_HALF_OPEN) | (PATH_PER_TET if per_tet else 0)
        lib = load_library()
        _check(lib.tv_voxelize_batch(ctypes.cast(self.array, ctypes.c_void_p), self.n,
                                     ctypes.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
                                     _stream_handle(stream), flags))
        return self.grids

    def resize_workspace(self):
        """Grows the workspace if the batch parameters in force need more."""
        need = int(load_library().tv_batch_workspace_bytes(ctypes.cast(self.array, ctypes.c_void_p), self.n, 0))
        if need == 0:
            _check(TV_ERR_INVALID_ARG)
        if self.workspace.numel() < need:
            self.workspace = alloc_workspace(need, self.workspace.device)
            self.plan = None
        return self.workspace

    def prepare(self, strict=False, accumulate=False, stream=None):
        """Uploads the descriptor table into the workspace (tv_batch_prepare);
        afterwards ``run_prepared`` enqueues kernels only and may be captured
        in a HIP graph.  Any other call on this batch's workspace (``run``)
        overwrites the table, so prepare again after one."""
        flags = (TIE_STRICT if strict else TIE_HALF_OPEN) | (ACCUMULATE if accumulate else 0)
        self.plan = BatchPlanC()
        _check(load_library().tv_batch_prepare(ctypes.cast(self.array, ctypes.c_void_p), self.n,
                                               ctypes.c_void_p(self.workspace.data_ptr()),
                                               self.workspace.numel(), _stream_handle(stream), flags,
                                               ctypes.byref(self.plan)))
        return self.plan

    def run_prepared(self, stream=None):
        """One run of the prepared batch (tv_batch_run)."""
        if getattr(self, "plan", None) is None:
            raise TVError(TV_ERR_INVALID_ARG, "prepare() the batch first")
        _check(load_library().tv_batch_run(ctypes.byref(self.plan), ctypes.c_void_p(self.workspace.data_ptr()),
                                           self.workspace.numel(), _stream_handle(stream)))
        return self.grids

    def status(self, i, stream=None):
        return fetch_status(self.workspace, i, stream)


def voxelize_batch(items, strict=False, per_tet=False, stream=None):
    """Voxelize many meshes in one launch sequence.  items: list of
    (verts, tets, dims, bbox, qverts).  Returns (grids, Batch)."""
    b = Batch(items)
    return b.run(strict=strict, per_tet=per_tet, stream=stream), b


class Server:
    """Continuous-batching voxelization server (tv_server_* in the C ABI).

    Requests carry numpy arrays (pageable or pinned host memory) or device
    tensors; the caller keeps them alive until the request is done.  Grids
    stay on the device until ``release``."""

    def __init__(self, device_bytes=8 << 30, pinned_bytes=1 << 30, streams=2, max_wave_meshes=1024):
        lib = load_library()
        cfg = ServerConfigC(int(device_bytes), int(pinned_bytes), int(streams), int(max_wave_meshes))
        h = ctypes.c_void_p()
        _check(lib.tv_server_create(ctypes.cast(ctypes.pointer(cfg), ctypes.c_void_p),
                                    ctypes.cast(ctypes.pointer(h), ctypes.c_void_p)))
        self._h = h
        self._keep = {}

    def submit(self, verts, tets, dims, bbox=None, *, qverts=False, strict=False, inputs="host"):
        """Queue one request; returns its ticket.  ``inputs`` is "host"
        (numpy, staged through pinned memory), "pinned" (pinned torch CPU
        tensors, copied directly) or "device" (device tensors)."""
        lib = load_library()
        if inputs == "device" or inputs == "pinned":
            vptr, nv = verts.data_ptr(), int(verts.shape[0])
            tptr, nt = tets.data_ptr(), int(tets.shape[0])
        else:
            import numpy as np

            verts = np.ascontiguousarray(verts, dtype=np.int32 if qverts else np.float32)
            tets = np.ascontiguousarray(tets, dtype=np.int32)
            vptr, nv = verts.ctypes.data, int(verts.shape[0])
            tptr, nt = tets.ctypes.data, int(tets.shape[0])
        flags = {"host": REQ_HOST_INPUTS, "pinned": REQ_PINNED_INPUTS, "device": REQ_DEVICE_INPUTS}[inputs]
        if strict:
            flags |= TIE_STRICT
        if bbox is None:
            bbox = ((0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
        req = RequestC(vptr, VERTS_Q32 if qverts else VERTS_F32, nv, tptr, nt, _dims(dims), _bbox(bbox), flags)
        t = ctypes.c_int64()
        _check(lib.tv_server_submit(self._h, ctypes.cast(ctypes.pointer(req), ctypes.c_void_p),
                                    ctypes.cast(ctypes.pointer(t), ctypes.c_void_p)))
        self._keep[t.value] = (verts, tets)
        return t.value

    def poll(self, ticket):
        st = ctypes.c_int32()
        _check(load_library().tv_server_poll(self._h, ticket, ctypes.cast(ctypes.pointer(st), ctypes.c_void_p)))
        return st.value

    def wait(self, ticket, timeout=0.0):
        _check(load_library().tv_server_wait(self._h, ticket, float(timeout)))

    def result(self, ticket):
        """(device grid address, words, data status, latency seconds)."""
        g = ctypes.c_void_p()
        n = ctypes.c_size_t()
        ds = ctypes.c_int32()
        lat = ctypes.c_double()
        P = ctypes.c_void_p
        _check(load_library().tv_server_result(self._h, ticket, ctypes.cast(ctypes.pointer(g), P),
                                               ctypes.cast(ctypes.pointer(n), P),
                                               ctypes.cast(ctypes.pointer(ds), P),
                                               ctypes.cast(ctypes.pointer(lat), P)))
        return g.value, n.value, ds.value, lat.value

    def copy_grid(self, ticket, out):
        """Copy a done request's grid into ``out`` (numpy uint32 or a torch
        int32 tensor, host or device)."""
        ptr = out.ctypes.data if hasattr(out, "ctypes") else out.data_ptr()
        _check(load_library().tv_server_copy_grid(self._h, ticket, ctypes.c_void_p(ptr), int(out.size if hasattr(out, "ctypes") else out.numel())))
        return out

    def release(self, ticket):
        _check(load_library().tv_server_release(self._h, ticket))
        self._keep.pop(ticket, None)

    def stats(self):
        st = ServerStatsC()
        _check(load_library().tv_server_get_stats(self._h, ctypes.cast(ctypes.pointer(st), ctypes.c_void_p)))
        return {k: getattr(st, k) for k, _ in ServerStatsC._fields_}

    def close(self):
        if self._h:
            _check(load_library().tv_server_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
