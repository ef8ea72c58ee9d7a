"""Pins of the quality-report oracle (oracle/quality.py) by closed forms:
dihedral angles of the Kuhn orthoscheme and of the regular tetrahedron,
orientations of the Kuhn tets (the sign of the axis permutation), volumes,
and the coverage identity of a conforming mesh (every voxel exactly once)
against a duplicated tet (extra coverage = that tet's voxels)."""
import math

import numpy as np

LAT = 1 << 16


def cube_kuhn(n):
    """n^3 unit cells, each split into its 6 Kuhn tets, on the lattice."""
    import itertools

    step = LAT // n
    idx = lambda i, j, k: (i * (n + 1) + j) * (n + 1) + k
    q = np.array([[i * step, j * step, k * step] for i in range(n + 1) for j in range(n + 1)
                  for k in range(n + 1)], np.int32)
    tets = []
    for i, j, k in itertools.product(range(n), repeat=3):
        for perm in itertools.permutations(range(3)):
            p = [0, 0, 0]
            path = [idx(i, j, k)]
            for ax in perm:
                p[ax] += 1
                path.append(idx(i + p[0], j + p[1], k + p[2]))
            tets.append(path)
    return q, np.array(tets, np.int32)


def test_kuhn_cube_closed_forms(oracle_mod):
    import oracle.quality as Q

    q, tets = cube_kuhn(2)
    r = Q.quality(oracle_mod, q, tets, (16, 16, 16), (1.0, 1.0, 1.0))
    assert r["tets"] == 48 and r["invalid"] == 0 and r["degenerate"] == 0
    # half of each cell's 6 tets follow an odd permutation of the axes
    assert r["inverted"] == 24
    # the Kuhn orthoscheme's dihedral angles are 45, 60 and 90 degrees
    assert abs(r["min_dihedral_deg"] - 45.0) < 1e-9 and abs(r["mean_min_dihedral_deg"] - 45.0) < 1e-9
    assert r["min_dihedral_below"] == [0, 0, 0, 0]
    assert abs(r["volume_mean"] - 1.0 / (6 * 8)) < 1e-15 and r["volume_cv"] < 1e-12
    # conforming: every voxel center of the cube exactly once
    assert r["covered_voxels"] == r["occupied_voxels"] == 16 ** 3


def test_regular_tet_and_overlap(oracle_mod):
    import oracle.quality as Q

    # a (nearly) regular tet, lattice-rounded, and a copy of it: overlap
    s = 20000
    V = np.array([[0, 0, 0], [2 * s, 0, 0], [s, round(s * math.sqrt(3)), 0],
                  [s, round(s / math.sqrt(3)), round(s * math.sqrt(8.0 / 3.0))]], np.float64)
    q = (V + 8000).astype(np.int32)
    one = Q.quality(oracle_mod, q, np.array([[0, 1, 2, 3]], np.int32), (32, 32, 32), (1.0, 1.0, 1.0))
    assert abs(one["min_dihedral_deg"] - math.degrees(math.acos(1.0 / 3.0))) < 1e-3
    assert one["covered_voxels"] == one["occupied_voxels"] > 0
    two = Q.quality(oracle_mod, q, np.array([[0, 1, 2, 3], [3, 2, 1, 0]], np.int32), (32, 32, 32),
                    (1.0, 1.0, 1.0))
    assert two["covered_voxels"] - two["occupied_voxels"] == one["occupied_voxels"]
    assert two["inverted"] == 0 or two["inverted"] == 1


def test_degenerate_invalid_and_thresholds(oracle_mod):
    import oracle.quality as Q

    q = np.array([[0, 0, 0], [40000, 0, 0], [0, 40000, 0], [20000, 20000, 0],  # 4 coplanar points
                  [0, 0, 40000], [40000, 0, 300], [100000, 0, 0]], np.int32)   # a sliver, an off-lattice point
    tets = np.array([[0, 1, 2, 3],   # degenerate
                     [0, 1, 2, 5],   # flat sliver: small dihedral angle
                     [0, 1, 2, 4],   # right corner
                     [0, 1, 2, 6],   # off-lattice vertex: invalid
                     [0, 1, 2, 9]],  # index out of range: invalid
                    np.int32)
    r = Q.quality(oracle_mod, q, tets, (16, 16, 16), (1.0, 1.0, 1.0))
    assert r["invalid"] == 2 and r["tets"] == 3 and r["degenerate"] == 1
    assert r["min_dihedral_below"][0] == 1  # the sliver is flatter than 1 degree
    # the trirectangular corner tet: 90 degrees at the origin's edges, and
    # arccos(1/sqrt(3)) between the slanted face and each coordinate plane
    corner = math.degrees(math.acos(1.0 / math.sqrt(3.0)))
    assert abs(float(np.sort(r["min_dihedral_all"])[1]) - corner) < 1e-9
