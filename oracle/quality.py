"""Oracle for the mesh quality report: the assumptions the paper's voxelizer
makes about its input (Section 3, "Voxelization": a large minimum angle, no
overlapping tets, small variance), computed with plain numpy on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).  It shares nothing
with the HIP path; the voxel coverage comes from the C oracle's own
per-voxel coverage count.
"""
from __future__ import annotations

import numpy as np

Q_MIN, Q_MAX = -16384, 65536 + 16384
BELOW_DEG = (1.0, 5.0, 10.0, 20.0)

# the six edges (a, b) of a tet and the two other vertices (c, d)
_EDGES = ((0, 1, 2, 3), (0, 2, 1, 3), (0, 3, 1, 2), (1, 2, 0, 3), (1, 3, 0, 2), (2, 3, 0, 1))


def six_volume(P) -> np.ndarray:
    """6V = det(B-A, C-A, D-A) per tet, exact in int64 (P: int [n, 4, 3])."""
    P = np.asarray(P, dtype=np.int64)
    b, c, d = P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]
    return (b[:, 0] * (c[:, 1] * d[:, 2] - c[:, 2] * d[:, 1])
            - b[:, 1] * (c[:, 0] * d[:, 2] - c[:, 2] * d[:, 0])
            + b[:, 2] * (c[:, 0] * d[:, 1] - c[:, 1] * d[:, 0]))


def min_dihedral_deg(W) -> np.ndarray:
    """Smallest of the six dihedral angles (degrees) per tet (W: float [n, 4, 3]).
    The dihedral angle at edge ab is the angle between the normals of the
    faces abc and abd, both formed with the edge first."""
    W = np.asarray(W, dtype=np.float64)
    out = np.full(W.shape[0], 180.0)
    for a, b, c, d in _EDGES:
        e = W[:, b] - W[:, a]
        n1 = np.cross(e, W[:, c] - W[:, a])
        n2 = np.cross(e, W[:, d] - W[:, a])
        cs = (n1 * n2).sum(axis=1) / np.sqrt((n1 * n1).sum(axis=1) * (n2 * n2).sum(axis=1))
        out = np.minimum(out, np.degrees(np.arccos(np.clip(cs, -1.0, 1.0))))
    return out


def quality(oracle_mod, q, tets, dims, ext, mode=0) -> dict:
    """Report for lattice vertices q [nv, 3] (int32; a failed snap is
    outside the lattice range), tets [nt, 4], grid dims and the bbox extent
    per axis (world units per 2^16 lattice units)."""
    q = np.asarray(q, dtype=np.int64)
    tets = np.asarray(tets, dtype=np.int64)
    nv = q.shape[0]
    idx_ok = np.all((tets >= 0) & (tets < nv), axis=1)
    valid = idx_ok.copy()
    P = np.zeros((tets.shape[0], 4, 3), np.int64)
    P[idx_ok] = q[tets[idx_ok]]
    valid &= np.all((P >= Q_MIN) & (P <= Q_MAX), axis=(1, 2))
    Pv = P[valid]
    six = six_volume(Pv)
    nondeg = six != 0
    scale = np.asarray(ext, dtype=np.float64) / 65536.0
    W = Pv[nondeg].astype(np.float64) * scale
    md = min_dihedral_deg(W)
    vol = np.abs(six[nondeg]).astype(np.float64) * float(np.prod(scale)) / 6.0
    # voxel coverage by the C oracle (per-voxel count of containing tets)
    # (vertices off the lattice range are used by invalid tets only; the C
    # oracle checks every vertex, so they are replaced before the call)
    vert_ok = np.all((q >= Q_MIN) & (q <= Q_MAX), axis=1)
    q_clean = np.where(vert_ok[:, None], q, 0).astype(np.int32)
    words, cover = oracle_mod.voxelize_q(q_clean, tets[valid].astype(np.int32), dims, mode=mode,
                                         coverage=True)
    n = int(nondeg.sum())
    mean_v = float(vol.mean()) if n else 0.0
    return {"tets": int(valid.sum()), "invalid": int((~valid).sum()), "degenerate": int((~nondeg).sum()),
            "inverted": int((six < 0).sum()),
            "min_dihedral_below": [int((md < t).sum()) for t in BELOW_DEG],
            "min_dihedral_deg": float(md.min()) if n else 0.0,
            "mean_min_dihedral_deg": float(md.mean()) if n else 0.0,
            "volume_mean": mean_v, "volume_cv": float(vol.std() / mean_v) if n and mean_v > 0 else 0.0,
            "covered_voxels": int(cover.astype(np.int64).sum()),
            "occupied_voxels": int((cover > 0).sum()),
            "min_dihedral_all": md, "words": words}
