"""Writers of tet-mesh files for the reader tests (MEDIT .mesh, Gmsh 2.2 and
4.1 ASCII).  Coordinates are written as the shortest decimal of their
float32 value, so reading them back as double and rounding to float32
returns them exactly."""
import numpy as np


def _num(x) -> str:
    return repr(float(np.float32(x)))


def write_medit(path, verts, tets):
    with open(path, "w") as f:
        f.write("MeshVersionFormatted 2\nDimension 3\n")
        f.write(f"Vertices\n{len(verts)}\n")
        for v in verts:
            f.write(f"{_num(v[0])} {_num(v[1])} {_num(v[2])} 0\n")
        f.write(f"Tetrahedra\n{len(tets)}\n")
        for t in tets:
            f.write(f"{t[0] + 1} {t[1] + 1} {t[2] + 1} {t[3] + 1} 1\n")
        f.write("End\n")


def write_gmsh22(path, verts, tets, tag0=1):
    with open(path, "w") as f:
        f.write("$MeshFormat\n2.2 0 8\n$EndMeshFormat\n")
        f.write(f"$Nodes\n{len(verts)}\n")
        for i, v in enumerate(verts):
            f.write(f"{tag0 + i} {_num(v[0])} {_num(v[1])} {_num(v[2])}\n")
        f.write("$EndNodes\n")
        f.write(f"$Elements\n{len(tets) + 1}\n1 15 2 0 0 {tag0}\n")  # a point element first
        for k, t in enumerate(tets):
            f.write(f"{k + 2} 4 2 1 1 {tag0 + t[0]} {tag0 + t[1]} {tag0 + t[2]} {tag0 + t[3]}\n")
        f.write("$EndElements\n")


def write_gmsh41(path, verts, tets, block=1000):
    """Nodes and tets in blocks of at most ``block`` entries."""
    nv, nt = len(verts), len(tets)
    with open(path, "w") as f:
        f.write("$MeshFormat\n4.1 0 8\n$EndMeshFormat\n")
        nb = (nv + block - 1) // block
        f.write(f"$Nodes\n{nb} {nv} 1 {nv}\n")
        for b in range(nb):
            lo, hi = b * block, min(nv, (b + 1) * block)
            f.write(f"3 1 0 {hi - lo}\n")
            for i in range(lo, hi):
                f.write(f"{i + 1}\n")
            for i in range(lo, hi):
                v = verts[i]
                f.write(f"{_num(v[0])} {_num(v[1])} {_num(v[2])}\n")
        f.write("$EndNodes\n")
        eb = (nt + block - 1) // block
        f.write(f"$Elements\n{eb} {nt} 1 {nt}\n")
        for b in range(eb):
            lo, hi = b * block, min(nt, (b + 1) * block)
            f.write(f"3 1 4 {hi - lo}\n")
            for k in range(lo, hi):
                t = tets[k]
                f.write(f"{k + 1} {t[0] + 1} {t[1] + 1} {t[2] + 1} {t[3] + 1}\n")
        f.write("$EndElements\n")
