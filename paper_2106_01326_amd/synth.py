"""Seeded synthetic tetrahedral meshes that stand in for mesher output.

The paper voxelizes tetrahedral meshes produced from Thingi10k / ModelNet
models (Table 1, Section 5); those datasets are not available here, so every
workload is a jittered Kuhn subdivision of the unit cube:

* ``n`` cubes per axis, each cut into the 6 Kuhn tetrahedra that share the
  cube's main diagonal (one per axis permutation), which gives a conforming
  mesh of ``6 n^3`` tets of good quality (the paper's voxelizer assumes large
  minimum angles and no overlaps, Section 3 "Voxelization");
* vertices strictly inside the cube are jittered by ``U[-delta, delta]`` cell
  widths per axis; vertices on the cube's boundary stay put, so the union of
  all tets is always exactly the cube;
* a tet whose orientation could turn non-positive after the vertices are
  placed on the 2^16 fixed-point lattice gets its interior vertices redrawn
  (repeatedly, from a seeded sub-stream) until every tet is safely positive;
  together with the fixed boundary this keeps the mesh conforming;
* tets are kept by centroid (a sphere, or a union of random ellipsoids) and
  the vertex array is compacted to the vertices still referenced.

This module holds only input generation.  It contains no part of the
voxelization arithmetic: no snapping to the lattice and no point-in-tet
predicate.  The validity guard below is a floating-point determinant with a
safety margin, i.e. a mesh-quality check on the generator's side.

Tet order is cube-major (x slowest, z fastest), 6 consecutive tets per cube,
like the spatially coherent order of a mesher's output; ``shuffle`` permutes
it for robustness tests.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

LATTICE = 1 << 16  # lattice units per bbox extent (fixed-point resolution)

# The 6 axis permutations and their parities: the Kuhn tet built from the
# path corner -> +e[p0] -> +e[p1] -> +e[p2] has orientation sign = parity.
_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))
_PARITY = (1, -1, -1, 1, 1, -1)


@dataclass
class Mesh:
    """One synthetic mesh, in the form the voxelizer consumes.

    ``verts`` is float32 [nv, 3] world coordinates (fp32 input path) or None;
    ``qverts`` is int32 [nv, 3] lattice coordinates (int32 input path) or None.
    ``tets`` is int32 [nt, 4].  ``dims`` is (nx, ny, nz); ``bbox`` is
    (lo[3], hi[3]) as float32 values.
    """

    tets: np.ndarray
    dims: tuple
    bbox: tuple
    verts: np.ndarray | None = None
    qverts: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def nt(self) -> int:
        return int(self.tets.shape[0])

    @property
    def nv(self) -> int:
        v = self.verts if self.verts is not None else self.qverts
        return int(v.shape[0])

    @property
    def fmt(self) -> str:
        return "f32" if self.verts is not None else "q32"


def kuhn_tets(n: int) -> np.ndarray:
    """Connectivity of the Kuhn subdivision of an n^3 cube grid.

    Vertex (x, y, z) has index (x*(n+1) + y)*(n+1) + z.  Cubes are listed
    x-major with z fastest and every tet is positively oriented (odd
    permutations get their last two vertices swapped).
    """
    m = n + 1
    cx, cy, cz = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    corner = ((cx * m + cy) * m + cz).reshape(-1).astype(np.int64)
    step = np.array([m * m, m, 1], dtype=np.int64)
    out = np.empty((corner.size, 6, 4), dtype=np.int32)
    for t, (perm, par) in enumerate(zip(_PERMS, _PARITY)):
        v0 = corner
        v1 = v0 + step[perm[0]]
        v2 = v1 + step[perm[1]]
        v3 = corner + step.sum()
        if par > 0:
            out[:, t] = np.stack([v0, v1, v2, v3], axis=1)
        else:
            out[:, t] = np.stack([v0, v1, v3, v2], axis=1)
    return out.reshape(-1, 4)


def _grid_index(n: int) -> np.ndarray:
    m = n + 1
    g = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), axis=-1)
    return g.reshape(-1, 3)


def _interior_mask(idx: np.ndarray, n: int) -> np.ndarray:
    return np.all((idx > 0) & (idx < n), axis=1)


def _orient_with_margin(p: np.ndarray, tets: np.ndarray, margin: bool) -> np.ndarray:
    """Float64 orientation of tets (in lattice units) minus a safety margin.

    ``p`` holds vertex positions in lattice units.  With ``margin`` the result
    is a lower bound on the orientation after every coordinate moves by up to
    half a lattice unit (rows move by up to sqrt(3) each; Hadamard's bound on
    the multilinear expansion), plus one unit for float64 evaluation error.
    """
    a = p[tets[:, 0]]
    e1 = p[tets[:, 1]] - a
    e2 = p[tets[:, 2]] - a
    e3 = p[tets[:, 3]] - a
    det = np.einsum("ij,ij->i", e1, np.cross(e2, e3))
    if not margin:
        return det - 0.5
    n1 = np.linalg.norm(e1, axis=1)
    n2 = np.linalg.norm(e2, axis=1)
    n3 = np.linalg.norm(e3, axis=1)
    r3 = math.sqrt(3.0)
    bound = r3 * (n2 * n3 + n1 * n3 + n1 * n2) + 3.0 * (n1 + n2 + n3) + 3.0 * r3 + 1.0
    return det - bound


def jittered_kuhn(n: int, delta: float, rng: np.random.Generator, fmt: str = "f32",
                  max_rounds: int = 200):
    """Jittered Kuhn mesh of the unit cube, repaired to be safely conforming.

    Returns (positions, tets, rounds).  For ``fmt == "f32"`` positions are
    float32 in [0, 1]; for ``fmt == "q32"`` they are int32 lattice coordinates
    in [0, 2^16] drawn directly on the lattice (integer jitter of up to
    floor(delta * cell) units).
    """
    idx = _grid_index(n)
    tets = kuhn_tets(n)
    interior = _interior_mask(idx, n)
    nvtx = idx.shape[0]
    jit_rng = np.random.Generator(np.random.PCG64(rng.integers(0, 2**63)))

    if fmt == "q32":
        if LATTICE % n:
            raise ValueError("integer lattice meshes need n dividing 2^16")
        cell = LATTICE // n
        amp = int(math.floor(delta * cell))

        def draw(count):
            return jit_rng.integers(-amp, amp + 1, size=(count, 3)).astype(np.int64)

        base = idx.astype(np.int64) * cell
        jit = np.zeros((nvtx, 3), dtype=np.int64)
        jit[interior] = draw(int(interior.sum()))

        def place(j):
            return base + j

        def lattice_pos(pos):
            return pos.astype(np.float64)

        margin = False
    else:
        def draw(count):
            return jit_rng.uniform(-delta, delta, size=(count, 3))

        base = idx.astype(np.float64)
        jit = np.zeros((nvtx, 3), dtype=np.float64)
        jit[interior] = draw(int(interior.sum()))

        def place(j):
            return ((base + j) / n).astype(np.float32)

        def lattice_pos(pos):
            return pos.astype(np.float64) * LATTICE

        margin = True

    pos = place(jit)
    check = np.arange(tets.shape[0])
    rounds = 0
    while True:
        o = _orient_with_margin(lattice_pos(pos), tets[check], margin)
        bad = check[o <= 0]
        if bad.size == 0:
            break
        rounds += 1
        if rounds > max_rounds:
            raise RuntimeError("jitter repair did not converge")
        redo = np.zeros(nvtx, dtype=bool)
        redo[tets[bad].reshape(-1)] = True
        redo &= interior
        if not redo.any():
            raise RuntimeError("an unjittered tet is not safely positive")
        jit[redo] = draw(int(redo.sum()))
        pos = place(jit)
        touched = redo[tets].any(axis=1)
        check = np.nonzero(touched)[0]
    if fmt == "q32":
        pos = pos.astype(np.int32)
    return pos, tets, rounds


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation from a normalised Gaussian quaternion."""
    q = rng.normal(size=4)
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def random_ellipsoids(k: int, rng: np.random.Generator):
    out = []
    for _ in range(k):
        c = rng.uniform(0.2, 0.8, size=3)
        ax = rng.uniform(0.15, 0.45, size=3)
        r = random_rotation(rng)
        out.append((c, ax, r))
    return out


def centroids_unit(pos: np.ndarray, tets: np.ndarray, fmt: str) -> np.ndarray:
    p = pos.astype(np.float64)
    if fmt == "q32":
        p = p / LATTICE
    return p[tets].mean(axis=1)


def keep_union_ellipsoids(cent: np.ndarray, ellipsoids) -> np.ndarray:
    keep = np.zeros(cent.shape[0], dtype=bool)
    for c, ax, r in ellipsoids:
        local = (cent - c) @ r  # coordinates in the ellipsoid's frame
        keep |= np.sum((local / ax) ** 2, axis=1) <= 1.0
    return keep


def keep_sphere(cent: np.ndarray, center, radius: float) -> np.ndarray:
    return np.sum((cent - np.asarray(center)) ** 2, axis=1) <= radius * radius


def compact(pos: np.ndarray, tets: np.ndarray):
    used = np.unique(tets.reshape(-1))
    remap = np.full(pos.shape[0], -1, dtype=np.int64)
    remap[used] = np.arange(used.size)
    return pos[used].copy(), remap[tets].astype(np.int32)


def make_mesh(n: int, delta: float, grid: int, keep: str, k: int, seed, fmt: str = "f32",
              shuffle: bool = False) -> Mesh:
    """One seeded mesh.  ``keep`` is "all", "sphere" or "ellipsoids" (k of them)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos, tets, rounds = jittered_kuhn(n, delta, rng, fmt)
    ntot = tets.shape[0]
    ell = None
    if keep == "all":
        sel = np.ones(ntot, dtype=bool)
    elif keep == "sphere":
        sel = keep_sphere(centroids_unit(pos, tets, fmt), (0.5, 0.5, 0.5), 0.45)
    elif keep == "ellipsoids":
        ell = random_ellipsoids(k, rng)
        sel = keep_union_ellipsoids(centroids_unit(pos, tets, fmt), ell)
    else:
        raise ValueError(keep)
    tets = tets[sel]
    if shuffle:
        tets = tets[rng.permutation(tets.shape[0])]
    pos, tets = compact(pos, tets)
    lo = np.zeros(3, dtype=np.float32)
    hi = np.ones(3, dtype=np.float32)
    meta = dict(n=n, delta=delta, grid=grid, keep=keep, k=k, fmt=fmt, repair_rounds=rounds,
                tets_before_keep=int(ntot), tets_kept=int(tets.shape[0]))
    m = Mesh(tets=tets, dims=(grid, grid, grid), bbox=(lo, hi), meta=meta)
    if fmt == "q32":
        m.qverts = pos
    else:
        m.verts = pos
    return m


# ---------------------------------------------------------------------------
# The five named workloads.  Seeds: 0..4 by workload index.

def workload_small(seed: int = 0) -> Mesh:
    """8^3 cubes (3072 tets), jitter 0.2 cell, sphere r=0.45 keep, 32^3 grid, fp32."""
    return make_mesh(8, 0.2, 32, "sphere", 0, seed, "f32")


def workload_medium(seed: int = 1) -> Mesh:
    """64^3 cubes (1.57M tets), jitter 0.3, 3 ellipsoids, 256^3 grid, int32 lattice verts."""
    return make_mesh(64, 0.3, 256, "ellipsoids", 3, seed, "q32")


def workload_large(seed: int = 2) -> Mesh:
    """128^3 cubes (12.6M tets), jitter 0.45, 6 ellipsoids, 1024^3 grid, fp32."""
    return make_mesh(128, 0.45, 1024, "ellipsoids", 6, seed, "f32")


def batch_params(count: int = 1024, seed: int = 3):
    """Per-mesh parameters of the uneven batch: n~U{4..48}, delta~U[0,0.4],
    k~U{1..4} ellipsoids, grid 32^3 or 64^3 with probability 1/2 each."""
    ss = np.random.SeedSequence(seed)
    children = ss.spawn(count)
    out = []
    for child in children:
        r = np.random.Generator(np.random.PCG64(child))
        n = int(r.integers(4, 49))
        delta = float(r.uniform(0.0, 0.4))
        k = int(r.integers(1, 5))
        grid = 32 if r.random() < 0.5 else 64
        out.append(dict(n=n, delta=delta, k=k, grid=grid, seed=child.spawn(1)[0]))
    return out


def batch_mesh(p) -> Mesh:
    return make_mesh(p["n"], p["delta"], p["grid"], "ellipsoids", p["k"], p["seed"], "f32")


def workload_batch(count: int = 1024, seed: int = 3, first: int | None = None,
                   workers: int | None = None):
    """The uneven batch (1024 meshes by default); ``first`` truncates it.
    Meshes are generated in ``workers`` processes (each mesh is seeded on its
    own, so the result does not depend on the worker count)."""
    ps = batch_params(count, seed)
    if first is not None:
        ps = ps[:first]
    if workers is None:
        import os

        workers = min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 1)
    if workers <= 1 or len(ps) < 8:
        return [batch_mesh(p) for p in ps]
    return pool_map(batch_mesh, ps, workers, chunksize=4)


def pool_map(fn, items, workers: int, chunksize: int = 1):
    """``map`` over worker processes started fresh ("spawn"): a caller that
    has already initialised the GPU never forks its own state into them.
    The pool is closed and joined, so its workers end normally."""
    import multiprocessing as mp

    pool = mp.get_context("spawn").Pool(workers)
    try:
        out = pool.map(fn, items, chunksize=chunksize)
        pool.close()
    except BaseException:
        pool.terminate()
        raise
    finally:
        pool.join()
    return out


def medium_shape_fp32(seed) -> Mesh:
    """The medium workload's shape (64^3 cubes, jitter 0.3, 3 ellipsoids,
    256^3 grid) with fp32 vertices, as used in the serving mix."""
    return make_mesh(64, 0.3, 256, "ellipsoids", 3, seed, "f32")
