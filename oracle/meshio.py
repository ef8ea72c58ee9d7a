"""Oracle reader for tet-mesh files: MEDIT ".mesh" (ASCII) and Gmsh ".msh"
2.2 / 4.1 (ASCII), written in plain Python.

TEST INFRASTRUCTURE ONLY (see the package docstring).  It shares nothing
with the library's native reader.  Both sides follow one definition:
coordinates are parsed as double and rounded to float32; tet indices become
0-based; elements that are not 4-node tetrahedra are counted as skipped.
The paper voxelizes the tetrahedral meshes its mesher writes (Section 3).
"""
from __future__ import annotations

import numpy as np

# MEDIT sections other than Vertices/Tetrahedra: tokens per entry, and
# whether the entries are mesh elements
_MEDIT_SKIP = {"Edges": (3, True), "Triangles": (4, True), "Quadrilaterals": (5, True),
               "Hexahedra": (9, True), "Prisms": (7, True), "Corners": (1, False),
               "Ridges": (1, False), "RequiredVertices": (1, False), "RequiredEdges": (1, False),
               "RequiredTriangles": (1, False), "Normals": (3, False), "Tangents": (3, False),
               "NormalAtVertices": (2, False), "TangentAtEdges": (3, False)}

# Gmsh element type -> node count (4 is the 4-node tetrahedron)
_GMSH_NODES = {1: 2, 2: 3, 3: 4, 4: 4, 5: 8, 6: 6, 7: 5, 8: 3, 9: 6, 10: 9, 11: 10, 15: 1}


class MeshFileError(ValueError):
    pass


def _f32(tok: str) -> np.float32:
    return np.float32(float(tok))


def _medit(text: str):
    toks = []
    for line in text.splitlines():
        toks.extend(line.split("#", 1)[0].split())
    it = iter(toks)
    verts, tets, skipped = None, None, 0
    for kw in it:
        if kw == "End":
            break
        if kw == "MeshVersionFormatted":
            if int(next(it)) not in (1, 2):
                raise MeshFileError("version")
        elif kw == "Dimension":
            if int(next(it)) != 3:
                raise MeshFileError("dimension")
        elif kw == "Vertices":
            n = int(next(it))
            verts = np.zeros((n, 3), np.float32)
            for i in range(n):
                verts[i] = [_f32(next(it)) for _ in range(3)]
                int(next(it))  # reference tag
        elif kw == "Tetrahedra":
            n = int(next(it))
            tets = np.zeros((n, 4), np.int32)
            for i in range(n):
                idx = [int(next(it)) for _ in range(4)]
                int(next(it))
                if min(idx) < 1:
                    raise MeshFileError("index")
                tets[i] = [v - 1 for v in idx]
        elif kw in _MEDIT_SKIP:
            per, element = _MEDIT_SKIP[kw]
            n = int(next(it))
            for _ in range(n * per):
                next(it)
            skipped += n if element else 0
        else:
            raise MeshFileError(f"keyword {kw}")
    if verts is None or tets is None:
        raise MeshFileError("sections")
    return verts, tets, skipped


def _gmsh(text: str):
    lines = [ln.split() for ln in text.splitlines()]
    lines = [ln for ln in lines if ln]
    version = float(lines[1][0])
    if lines[1][1] != "0":
        raise MeshFileError("binary")
    v4 = version >= 4.0
    pos = 3  # after $MeshFormat, the version line and $EndMeshFormat
    tag_index: dict[int, int] = {}
    coords: list[list[np.float32]] = []
    tet_tags: list[int] = []
    skipped = 0
    while pos < len(lines):
        sec = lines[pos][0]
        pos += 1
        if sec == "$Nodes":
            if not v4:
                n = int(lines[pos][0])
                pos += 1
                for k in range(n):
                    tag, x, y, z = lines[pos + k][:4]
                    tag_index[int(tag)] = len(coords)
                    coords.append([_f32(x), _f32(y), _f32(z)])
                pos += n
            else:
                nblocks = int(lines[pos][0])
                pos += 1
                for _ in range(nblocks):
                    m = int(lines[pos][3])
                    pos += 1
                    tags = [int(lines[pos + k][0]) for k in range(m)]
                    pos += m
                    for k in range(m):
                        tag_index[tags[k]] = len(coords)
                        coords.append([_f32(t) for t in lines[pos + k][:3]])
                    pos += m
        elif sec == "$Elements":
            if not v4:
                n = int(lines[pos][0])
                pos += 1
                for k in range(n):
                    ln = [int(t) for t in lines[pos + k]]
                    etype, ntags = ln[1], ln[2]
                    nodes = ln[3 + ntags: 3 + ntags + _GMSH_NODES[etype]]
                    if etype == 4:
                        tet_tags.extend(nodes)
                    else:
                        skipped += 1
                pos += n
            else:
                nblocks = int(lines[pos][0])
                pos += 1
                for _ in range(nblocks):
                    etype, m = int(lines[pos][2]), int(lines[pos][3])
                    pos += 1
                    for k in range(m):
                        ln = [int(t) for t in lines[pos + k]]
                        if etype == 4:
                            tet_tags.extend(ln[1:5])
                    if etype != 4:
                        skipped += m
                    pos += m
        # skip to this section's end marker
        end = "$End" + sec[1:]
        while lines[pos][0] != end:
            pos += 1
        pos += 1
    verts = np.array(coords, np.float32).reshape(-1, 3)
    tets = np.array([tag_index[t] for t in tet_tags], np.int32).reshape(-1, 4)
    return verts, tets, skipped


def read_mesh(path):
    """(verts float32 [nv, 3], tets int32 [nt, 4] 0-based, skipped count)."""
    with open(path) as f:
        text = f.read()
    body = "\n".join(line.split("#", 1)[0] for line in text.splitlines())
    first = body.split(None, 1)[0] if body.split() else ""
    if first == "MeshVersionFormatted":
        return _medit(text)
    if first == "$MeshFormat":
        return _gmsh(text)
    raise MeshFileError("format")
