"""Exact-rational point-in-tetrahedron test (micro-oracle).

TEST INFRASTRUCTURE ONLY: used by the tests to pin the C oracle; never on
the product path.

This is the textbook formulation, independent of Theorem 1 (Section 4) and
of the C oracle's determinant code: solve the 4x4 barycentric system

    lA*A + lB*B + lC*C + lD*D = P',   lA + lB + lC + lD = 1

exactly with Fractions (Gauss-Jordan elimination, partial pivoting on
non-zero entries) and call P' inside when every l > 0.

P' is the voxel center pushed by the fixed tie-break perturbation,
P' = P + eps*ez + eps^2*ey + eps^3*ex with eps = 2^-64, in "half_open" mode,
and P' = P in "strict" mode (Theorem 1 taken literally: points on a face are
outside).  For integer inputs with |coordinate| <= 2^18 every face function
has integer gradient components below 2^40, so eps = 2^-64 already decides
every sign exactly as the limit eps -> 0+ does.
"""
from __future__ import annotations

from fractions import Fraction

EPS = Fraction(1, 1 << 64)


def _solve(mat, rhs):
    """Solve mat @ x = rhs exactly; None when mat is singular."""
    n = len(rhs)
    a = [[Fraction(v) for v in row] + [Fraction(r)] for row, r in zip(mat, rhs)]
    for col in range(n):
        piv = next((r for r in range(col, n) if a[r][col] != 0), None)
        if piv is None:
            return None
        a[col], a[piv] = a[piv], a[col]
        pv = a[col][col]
        a[col] = [v / pv for v in a[col]]
        for r in range(n):
            if r != col and a[r][col] != 0:
                f = a[r][col]
                a[r] = [x - f * y for x, y in zip(a[r], a[col])]
    return [a[r][n] for r in range(n)]


def barycentric(P, A, B, C, D, mode="half_open"):
    """Exact barycentric coordinates of the (perturbed) point, or None if the
    tet is degenerate."""
    px, py, pz = (Fraction(v) for v in P)
    if mode == "half_open":
        pz += EPS
        py += EPS ** 2
        px += EPS ** 3
    elif mode != "strict":
        raise ValueError(mode)
    mat = [
        [A[0], B[0], C[0], D[0]],
        [A[1], B[1], C[1], D[1]],
        [A[2], B[2], C[2], D[2]],
        [1, 1, 1, 1],
    ]
    return _solve(mat, [px, py, pz, 1])


def inside(P, A, B, C, D, mode="half_open") -> bool:
    lam = barycentric(P, A, B, C, D, mode)
    return lam is not None and all(v > 0 for v in lam)


def voxelize_bruteforce(q, tets, dims, mode="half_open"):
    """Every voxel center against every tet, exactly.  Tiny inputs only.
    Returns a uint8 array [nx, ny, nz] of 0/1."""
    import numpy as np

    nx, ny, nz = dims
    s = [(1 << 15) // n for n in dims]
    out = np.zeros((nx, ny, nz), dtype=np.uint8)
    tv = [[tuple(int(c) for c in q[v]) for v in t] for t in tets]
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                P = ((2 * i + 1) * s[0], (2 * j + 1) * s[1], (2 * k + 1) * s[2])
                for A, B, C, D in tv:
                    if inside(P, A, B, C, D, mode):
                        out[i, j, k] = 1
                        break
    return out
