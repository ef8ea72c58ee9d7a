"""CPU oracle for the tetrahedral voxelizer.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The product
path (the HIP library and its binding) never imports, loads or calls it.

``tv_oracle.c`` is the plain C voxelizer (Theorem 1 per candidate center);
``micro.py`` is an exact-rational barycentric test used to pin it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tv_oracle.c")
LIB = os.path.join(HERE, "_build", "libtv_oracle.so")

HALF_OPEN = 0
STRICT = 1

_lib = None


def build(src: str = SRC, out: str = LIB) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, no FMA contraction)."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-ffp-contract=off",
           "-fno-fast-math", "-fPIC", "-shared", "-pthread", src, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build()
    _lib = _bind(ctypes.CDLL(LIB))
    return _lib


def use_library(path):
    """Point this module at another build of the oracle source (the mutation
    tests build deliberately broken copies); ``None`` restores the default.
    Returns the previously bound library handle."""
    global _lib
    prev = _lib
    _lib = None if path is None else _bind(ctypes.CDLL(path))
    return prev


def _bind(lib):
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.oracle_snap.argtypes = [P, i64, P, P, P]
    lib.oracle_snap.restype = ctypes.c_int
    lib.oracle_point_in_tet.argtypes = [P, P, P, P, P, ctypes.c_int]
    lib.oracle_point_in_tet.restype = ctypes.c_int
    lib.oracle_theorem1_dets.argtypes = [P, P, P, P, P, P]
    lib.oracle_theorem1_dets.restype = None
    lib.oracle_six_volume.argtypes = [P, P, P, P]
    lib.oracle_six_volume.restype = i64
    lib.oracle_voxelize.argtypes = [P, i64, P, i64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P]
    lib.oracle_voxelize.restype = ctypes.c_int
    return lib


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code}")
        self.code = code


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def snap(verts, lo, hi) -> np.ndarray:
    """fp32 world coordinates [nv,3] -> int32 lattice coordinates [nv,3]."""
    v = np.ascontiguousarray(verts, dtype=np.float32)
    lo = np.ascontiguousarray(lo, dtype=np.float32)
    hi = np.ascontiguousarray(hi, dtype=np.float32)
    q = np.empty(v.shape, dtype=np.int32)
    rc = _load().oracle_snap(_ptr(v), v.shape[0], _ptr(lo), _ptr(hi), _ptr(q))
    if rc:
        raise OracleError(rc)
    return q


def _i64(v):
    return np.ascontiguousarray(np.asarray(v, dtype=np.int64).reshape(3))


def point_in_tet(P, A, B, C, D, mode=HALF_OPEN) -> bool:
    a = [_i64(x) for x in (P, A, B, C, D)]
    return bool(_load().oracle_point_in_tet(*[_ptr(x) for x in a], mode))


def theorem1_dets(P, A, B, C, D):
    a = [_i64(x) for x in (P, A, B, C, D)]
    out = np.zeros(4, dtype=np.int64)
    _load().oracle_theorem1_dets(*[_ptr(x) for x in a], _ptr(out))
    return out


def six_volume(A, B, C, D) -> int:
    a = [_i64(x) for x in (A, B, C, D)]
    return int(_load().oracle_six_volume(*[_ptr(x) for x in a]))


def grid_words(dims) -> int:
    nx, ny, nz = dims
    return nx * ny * ((nz + 31) // 32)


def voxelize_q(q, tets, dims, mode=HALF_OPEN, window=None, brute=False, threads=None,
               coverage=False):
    """Lattice verts q[nv,3] + tets[nt,4] -> uint32 words (and optionally the
    uint8 coverage count [nx,ny,nz]).  ``window`` = (i0,i1,j0,j1,k0,k1)
    inclusive restricts which voxels are computed."""
    q = np.ascontiguousarray(q, dtype=np.int32)
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    nx, ny, nz = (int(d) for d in dims)
    words = np.zeros(grid_words(dims), dtype=np.uint32)
    cover = np.zeros((nx, ny, nz), dtype=np.uint8) if coverage else None
    win = None if window is None else np.ascontiguousarray(window, dtype=np.int64)
    if threads is None:
        threads = os.cpu_count() or 1
    rc = _load().oracle_voxelize(_ptr(q), q.shape[0], _ptr(tets), tets.shape[0], nx, ny, nz,
                                 _ptr(win), int(mode), int(bool(brute)), int(threads),
                                 _ptr(words), _ptr(cover))
    if rc:
        raise OracleError(rc)
    return (words, cover) if coverage else words


def voxelize_mesh(mesh, mode=HALF_OPEN, **kw):
    """Voxelize a ``synth.Mesh`` (snapping fp32 vertices first)."""
    if mesh.verts is not None:
        q = snap(mesh.verts, mesh.bbox[0], mesh.bbox[1])
    else:
        q = mesh.qverts
    return voxelize_q(q, mesh.tets, mesh.dims, mode=mode, **kw)


def unpack(words, dims) -> np.ndarray:
    """uint32 words -> uint8 [nx, ny, nz] occupancy."""
    nx, ny, nz = dims
    w = (nz + 31) // 32
    bits = np.unpackbits(np.ascontiguousarray(words, dtype=np.uint32).view(np.uint8),
                         bitorder="little")
    return bits.reshape(nx, ny, w * 32)[..., :nz]
