"""Oracle for the grid consumers: dense unpacking, coarser levels and sparse
bricks of a packed occupancy grid.

TEST INFRASTRUCTURE ONLY (see the package docstring): plain numpy on the
CPU, sharing nothing with the HIP path.

The paper motivates solid grids by 3D CNN inputs (Section 1; the 3D CNN
connection is left to future work in Section 6) and notes that sparse voxel
data is usually stored sparsely (Octrees paragraph, Section 5).  The grid
layout is the library's: W = ceil(nz/32) little-endian uint32 words per
(i, j) column, voxel (i, j, k) at bit k & 31 of word (i*ny + j)*W + k//32.
"""
from __future__ import annotations

import numpy as np

from . import unpack as _unpack


def unpack(words, dims) -> np.ndarray:
    """uint8 [nx, ny, nz], 1 where the voxel is set."""
    nx, ny, nz = (int(d) for d in dims)
    return np.ascontiguousarray(_unpack(words, (nx, ny, nz)))


def pack(bits) -> np.ndarray:
    """Inverse of unpack: uint8/bool [nx, ny, nz] -> uint32 words, padding 0."""
    b = np.asarray(bits).astype(bool)
    nx, ny, nz = b.shape
    W = (nz + 31) // 32
    full = np.zeros((nx, ny, 32 * W), dtype=bool)
    full[..., :nz] = b
    return np.packbits(full, axis=-1, bitorder="little").view(np.uint32).reshape(-1).copy()


def pool_fraction(words, dims, f) -> np.ndarray:
    """float64 [nx/f, ny/f, nz/f]: fraction of set voxels per f^3 block."""
    nx, ny, nz = (int(d) for d in dims)
    b = unpack(words, dims).astype(np.int64)
    blocks = b.reshape(nx // f, f, ny // f, f, nz // f, f)
    return blocks.sum(axis=(1, 3, 5)) / float(f ** 3)


def pool_any(words, dims, f) -> np.ndarray:
    """Packed grid of dims / f: a voxel is set iff any voxel of its block is."""
    nx, ny, nz = (int(d) for d in dims)
    b = unpack(words, dims).astype(bool)
    anyb = b.reshape(nx // f, f, ny // f, f, nz // f, f).any(axis=(1, 3, 5))
    return pack(anyb)


def bricks(words, dims):
    """Non-empty 8 x 8 x 32 bricks in increasing id: (ids uint32 [n],
    brick words uint32 [n, 64]).  Brick (bx, by, bz) has id
    (bx*(ny/8) + by)*(nz/32) + bz and holds word bz of columns
    (8bx+u, 8by+v), u-major."""
    nx, ny, nz = (int(d) for d in dims)
    W = nz // 32
    w = np.ascontiguousarray(words, dtype=np.uint32).reshape(nx // 8, 8, ny // 8, 8, W)
    # -> [bx, by, bz, u, v]
    per = w.transpose(0, 2, 4, 1, 3).reshape(nx // 8, ny // 8, W, 64)
    flat = per.reshape(-1, 64)
    ids = np.nonzero(flat.any(axis=1))[0].astype(np.uint32)
    return ids, flat[ids].copy()


def export_batch(grids, res, mode):
    """One dense [n, res, res, res] tensor from n packed grids of any dims:
    per axis a grid finer than res is pooled by n_a/res and a coarser one
    repeated res/n_a times.  mode 0: float64 fraction of set voxels in each
    cell's source block; mode 1: uint8, 1 when any voxel of the block is set.
    ``grids``: list of (words, dims)."""
    out = []
    for words, dims in grids:
        b = unpack(words, dims).astype(np.int64)
        block = 1
        for axis, n in enumerate(int(d) for d in dims):
            if n > res:
                f = n // res
                shape = list(b.shape)
                shape[axis:axis + 1] = [res, f]
                b = b.reshape(shape).sum(axis=axis + 1)
                block *= f
        for axis, n in enumerate(int(d) for d in dims):
            if n < res:
                b = np.repeat(b, res // n, axis=axis)
        out.append(b / float(block) if mode == 0 else (b > 0).astype(np.uint8))
    return np.stack(out) if out else np.zeros((0, res, res, res))
