"""Shared helpers of the test suite (no method arithmetic here)."""
from __future__ import annotations

import re
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    """Function names declared in include/*.h."""
    names = []
    inc = os.path.join(ROOT, "include")
    for fn in sorted(os.listdir(inc)):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(inc, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(tv_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def gpu_available() -> bool:
    try:
        import torch

        return torch.cuda.is_available()
    except Exception:
        return False


def to_numpy_words(grid) -> np.ndarray:
    return grid.cpu().numpy().view(np.uint32)


def gpu_voxelize_mesh(mesh, strict=False, stream=None, per_tet=False, stale=True):
    """Run the HIP path on a synth.Mesh; returns (uint32 words, status).
    With ``stale`` the output grid starts filled with ones, so every word the
    path fails to write shows up."""
    import torch

    import paper_2106_01326_amd as tv

    tets = torch.from_numpy(np.ascontiguousarray(mesh.tets)).cuda()
    grid = tv.alloc_grid(mesh.dims)
    if stale:
        grid.fill_(-1)
    if mesh.verts is not None:
        v = torch.from_numpy(np.ascontiguousarray(mesh.verts)).cuda()
        grid, ws = tv.voxelize(v, tets, mesh.dims, mesh.bbox, strict=strict, per_tet=per_tet,
                               grid=grid, stream=stream)
    else:
        v = torch.from_numpy(np.ascontiguousarray(mesh.qverts)).cuda()
        grid, ws = tv.voxelize(v, tets, mesh.dims, qverts=True, strict=strict, per_tet=per_tet,
                               grid=grid, stream=stream)
    status = tv.fetch_status(ws, 0, stream)
    return to_numpy_words(grid), status


def gpu_voxelize_q(q, tets, dims, strict=False, per_tet=False):
    import torch

    import paper_2106_01326_amd as tv

    qt = torch.from_numpy(np.ascontiguousarray(q, dtype=np.int32)).cuda()
    tt = torch.from_numpy(np.ascontiguousarray(tets, dtype=np.int32)).cuda()
    grid = tv.alloc_grid(dims)
    grid.fill_(-1)
    grid, ws = tv.voxelize(qt, tt, dims, qverts=True, strict=strict, per_tet=per_tet, grid=grid)
    return to_numpy_words(grid), tv.fetch_status(ws)


def window_bits(words, dims, win):
    """Occupancy bits of the inclusive voxel window (i0,i1,j0,j1,k0,k1)."""
    nx, ny, nz = dims
    W = (nz + 31) // 32
    i0, i1, j0, j1, k0, k1 = win
    sub = np.ascontiguousarray(words.reshape(nx, ny, W)[i0:i1 + 1, j0:j1 + 1, :])
    bits = np.unpackbits(sub.view(np.uint8), bitorder="little").reshape(i1 - i0 + 1, j1 - j0 + 1, W * 32)
    return bits[..., k0:k1 + 1]


def first_mismatch(a, b):
    d = np.nonzero(a != b)[0]
    return None if d.size == 0 else (int(d[0]), int(d.size))
