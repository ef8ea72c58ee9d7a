// Tet-mesh file readers (host code): the step before voxelization, reading
// the tetrahedral meshes a mesher writes (the paper's pipeline generates them
// with a TetWild-style mesher, Section 3 "Tetrahedral Mesh generating").
// Formats: MEDIT ".mesh" (ASCII) and Gmsh ".msh" 2.2 and 4.1 (ASCII).
// Coordinates are parsed as double and rounded to float (the voxelizer's
// input type); indices become 0-based.
#include <ctype.h>
#include <errno.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <exception>
#include <string>
#include <unordered_map>
#include <vector>

#include "tv.h"
#include "tv_internal.h"

namespace {

// Whole-file tokenizer over whitespace; '#' starts a comment in MEDIT files
// (Gmsh files have none).
struct Reader {
    std::vector<char> buf;
    size_t pos = 0;
    bool hash_comments = false;

    bool load(const char *path) {
        FILE *f = fopen(path, "rb");
        if (!f) return false;
        if (fseek(f, 0, SEEK_END) != 0) {
            fclose(f);
            return false;
        }
        const long n = ftell(f);
        if (n < 0 || fseek(f, 0, SEEK_SET) != 0) {
            fclose(f);
            return false;
        }
        buf.resize((size_t)n + 1);
        const size_t got = fread(buf.data(), 1, (size_t)n, f);
        fclose(f);
        if (got != (size_t)n) return false;
        buf[(size_t)n] = '\0';
        return true;
    }
    void skip_space() {
        for (;;) {
            while (pos + 1 < buf.size() && isspace((unsigned char)buf[pos])) ++pos;
            if (hash_comments && pos + 1 < buf.size() && buf[pos] == '#') {
                while (pos + 1 < buf.size() && buf[pos] != '\n') ++pos;
                continue;
            }
            return;
        }
    }
    bool at_end() {
        skip_space();
        return pos + 1 >= buf.size();
    }
    // Could the rest of the file hold n entries of `tokens` tokens each?
    // Every token takes at least one byte, so a count above the bytes left
    // (a corrupt or hostile header) is refused before anything is sized
    // from it.
    bool can_hold(int64_t n, int64_t tokens) const {
        if (n < 0) return false;
        const int64_t left = (int64_t)(buf.size() - pos);
        return n <= left / tokens;
    }
    // next whitespace-delimited token (empty at the end)
    std::string token() {
        skip_space();
        const size_t b = pos;
        while (pos + 1 < buf.size() && !isspace((unsigned char)buf[pos])) ++pos;
        return std::string(buf.data() + b, pos - b);
    }
    bool integer(int64_t &v) {
        skip_space();
        char *end = nullptr;
        errno = 0;
        const long long x = strtoll(buf.data() + pos, &end, 10);
        if (end == buf.data() + pos || errno) return false;
        if (*end && !isspace((unsigned char)*end)) return false;
        pos = (size_t)(end - buf.data());
        v = x;
        return true;
    }
    bool real(double &v) {
        skip_space();
        char *end = nullptr;
        errno = 0;
        const double x = strtod(buf.data() + pos, &end);
        if (end == buf.data() + pos) return false;
        if (*end && !isspace((unsigned char)*end)) return false;
        pos = (size_t)(end - buf.data());
        v = x;
        return true;
    }
};

struct Parsed {
    std::vector<float> verts;
    std::vector<int32_t> tets;
    int64_t skipped = 0;
};

tv_status io_error(const char *path, const char *what) {
    return tv::set_error(TV_ERR_IO, "%s: %s", path, what);
}

// MEDIT: keyword sections; entries of a section have a fixed token count.
int medit_entry_tokens(const std::string &kw) {
    static const std::unordered_map<std::string, int> n = {
        {"Edges", 3},         {"Triangles", 4},        {"Quadrilaterals", 5},
        {"Hexahedra", 9},     {"Prisms", 7},           {"Corners", 1},
        {"Ridges", 1},        {"RequiredVertices", 1}, {"RequiredEdges", 1},
        {"RequiredTriangles", 1}, {"Normals", 3},      {"Tangents", 3},
        {"NormalAtVertices", 2},  {"TangentAtEdges", 3}};
    const auto it = n.find(kw);
    return it == n.end() ? -1 : it->second;
}

tv_status read_medit(Reader &r, const char *path, Parsed &out) {
    r.hash_comments = true;
    bool have_v = false, have_t = false;
    while (!r.at_end()) {
        const std::string kw = r.token();
        int64_t n = 0;
        if (kw == "End") break;
        if (kw == "MeshVersionFormatted") {
            if (!r.integer(n) || (n != 1 && n != 2)) return io_error(path, "bad MeshVersionFormatted");
        } else if (kw == "Dimension") {
            if (!r.integer(n) || n != 3) return io_error(path, "only Dimension 3 is supported");
        } else if (kw == "Vertices") {
            if (!r.integer(n) || !r.can_hold(n, 4)) return io_error(path, "bad Vertices count");
            out.verts.resize((size_t)n * 3);
            for (int64_t i = 0; i < n; ++i) {
                double x[3];
                int64_t ref;
                if (!r.real(x[0]) || !r.real(x[1]) || !r.real(x[2]) || !r.integer(ref))
                    return io_error(path, "truncated Vertices section");
                for (int a = 0; a < 3; ++a) out.verts[(size_t)(3 * i + a)] = (float)x[a];
            }
            have_v = true;
        } else if (kw == "Tetrahedra") {
            if (!r.integer(n) || !r.can_hold(n, 5)) return io_error(path, "bad Tetrahedra count");
            out.tets.resize((size_t)n * 4);
            for (int64_t i = 0; i < n; ++i) {
                int64_t v[5];
                for (int a = 0; a < 5; ++a)
                    if (!r.integer(v[a])) return io_error(path, "truncated Tetrahedra section");
                for (int a = 0; a < 4; ++a) {
                    if (v[a] < 1 || v[a] > INT32_MAX) return io_error(path, "tet index out of range");
                    out.tets[(size_t)(4 * i + a)] = (int32_t)(v[a] - 1);
                }
            }
            have_t = true;
        } else {
            const int per = medit_entry_tokens(kw);
            if (per < 0) return tv::set_error(TV_ERR_IO, "%s: unknown keyword '%s'", path, kw.c_str());
            if (!r.integer(n) || !r.can_hold(n, per)) return io_error(path, "bad section count");
            for (int64_t i = 0; i < n * per; ++i)
                if (r.token().empty()) return io_error(path, "truncated section");
            // other element kinds are counted as skipped; tags and normals are not elements
            if (kw == "Edges" || kw == "Triangles" || kw == "Quadrilaterals" || kw == "Hexahedra" ||
                kw == "Prisms")
                out.skipped += n;
        }
    }
    if (!have_v || !have_t) return io_error(path, "no Vertices or no Tetrahedra section");
    return TV_OK;
}

// Gmsh: "$Section ... $EndSection" blocks, line-structured.
bool skip_to_end(Reader &r, const std::string &name) {
    const std::string end = "$End" + name.substr(1);
    while (!r.at_end())
        if (r.token() == end) return true;
    return false;
}

int gmsh_nodes_of_type(int64_t type) {
    switch (type) {
        case 1: return 2;   case 2: return 3;   case 3: return 4;   case 4: return 4;
        case 5: return 8;   case 6: return 6;   case 7: return 5;   case 8: return 3;
        case 9: return 6;   case 10: return 9;  case 11: return 10; case 15: return 1;
        default: return -1;
    }
}

tv_status read_gmsh(Reader &r, const char *path, Parsed &out) {
    double version = 0.0;
    int64_t ftype = 0, dsize = 0;
    if (!r.real(version) || !r.integer(ftype) || !r.integer(dsize))
        return io_error(path, "bad $MeshFormat line");
    if (ftype != 0) return io_error(path, "binary Gmsh files are not supported");
    const bool v2 = version >= 2.0 && version < 3.0, v4 = version >= 4.0 && version < 5.0;
    if (!v2 && !v4) return io_error(path, "Gmsh version must be 2.x or 4.x");
    if (r.token() != "$EndMeshFormat") return io_error(path, "missing $EndMeshFormat");
    std::unordered_map<int64_t, int32_t> index;  // node tag -> vertex index
    std::vector<int64_t> tet_tags;               // 4 node tags per tet
    bool have_n = false, have_e = false;
    while (!r.at_end()) {
        const std::string sec = r.token();
        if (sec.empty() || sec[0] != '$') return io_error(path, "expected a $Section");
        if (sec == "$Nodes") {
            if (v2) {
                int64_t n;
                if (!r.integer(n) || !r.can_hold(n, 4)) return io_error(path, "bad $Nodes count");
                out.verts.reserve((size_t)n * 3);
                for (int64_t i = 0; i < n; ++i) {
                    int64_t tag;
                    double x[3];
                    if (!r.integer(tag) || !r.real(x[0]) || !r.real(x[1]) || !r.real(x[2]))
                        return io_error(path, "truncated $Nodes");
                    if (!index.emplace(tag, (int32_t)(out.verts.size() / 3)).second)
                        return io_error(path, "duplicate node tag");
                    for (int a = 0; a < 3; ++a) out.verts.push_back((float)x[a]);
                }
            } else {
                int64_t blocks, n, mn, mx;
                if (!r.integer(blocks) || !r.integer(n) || !r.integer(mn) || !r.integer(mx) ||
                    !r.can_hold(blocks, 4) || !r.can_hold(n, 4))
                    return io_error(path, "bad $Nodes header");
                out.verts.reserve((size_t)n * 3);
                for (int64_t b = 0; b < blocks; ++b) {
                    int64_t edim, etag, param, m;
                    if (!r.integer(edim) || !r.integer(etag) || !r.integer(param) || !r.integer(m))
                        return io_error(path, "bad node block header");
                    if (param) return io_error(path, "parametric nodes are not supported");
                    if (!r.can_hold(m, 4)) return io_error(path, "bad node block size");
                    std::vector<int64_t> tags((size_t)m);
                    for (int64_t i = 0; i < m; ++i)
                        if (!r.integer(tags[(size_t)i])) return io_error(path, "truncated node tags");
                    for (int64_t i = 0; i < m; ++i) {
                        double x[3];
                        if (!r.real(x[0]) || !r.real(x[1]) || !r.real(x[2]))
                            return io_error(path, "truncated node coordinates");
                        if (!index.emplace(tags[(size_t)i], (int32_t)(out.verts.size() / 3)).second)
                            return io_error(path, "duplicate node tag");
                        for (int a = 0; a < 3; ++a) out.verts.push_back((float)x[a]);
                    }
                }
            }
            if (r.token() != "$EndNodes") return io_error(path, "missing $EndNodes");
            have_n = true;
        } else if (sec == "$Elements") {
            if (v2) {
                int64_t n;
                if (!r.integer(n) || !r.can_hold(n, 4)) return io_error(path, "bad $Elements count");
                for (int64_t i = 0; i < n; ++i) {
                    int64_t tag, type, ntags;
                    if (!r.integer(tag) || !r.integer(type) || !r.integer(ntags) || ntags < 0)
                        return io_error(path, "bad element line");
                    for (int64_t k = 0; k < ntags; ++k)
                        if (r.token().empty()) return io_error(path, "truncated element tags");
                    const int nn = gmsh_nodes_of_type(type);
                    if (nn < 0) return io_error(path, "unknown element type");
                    for (int k = 0; k < nn; ++k) {
                        int64_t v;
                        if (!r.integer(v)) return io_error(path, "truncated element nodes");
                        if (type == 4) tet_tags.push_back(v);
                    }
                    if (type != 4) ++out.skipped;
                }
            } else {
                int64_t blocks, n, mn, mx;
                if (!r.integer(blocks) || !r.integer(n) || !r.integer(mn) || !r.integer(mx) ||
                    !r.can_hold(blocks, 4) || !r.can_hold(n, 2))
                    return io_error(path, "bad $Elements header");
                for (int64_t b = 0; b < blocks; ++b) {
                    int64_t edim, etag, type, m;
                    if (!r.integer(edim) || !r.integer(etag) || !r.integer(type) || !r.integer(m))
                        return io_error(path, "bad element block header");
                    const int nn = gmsh_nodes_of_type(type);
                    if (nn < 0) return io_error(path, "unknown element type");
                    if (!r.can_hold(m, 1 + nn)) return io_error(path, "bad element block size");
                    for (int64_t i = 0; i < m; ++i) {
                        int64_t tag;
                        if (!r.integer(tag)) return io_error(path, "truncated element block");
                        for (int k = 0; k < nn; ++k) {
                            int64_t v;
                            if (!r.integer(v)) return io_error(path, "truncated element nodes");
                            if (type == 4) tet_tags.push_back(v);
                        }
                    }
                    if (type != 4) out.skipped += m;
                }
            }
            if (r.token() != "$EndElements") return io_error(path, "missing $EndElements");
            have_e = true;
        } else if (!skip_to_end(r, sec)) {
            return io_error(path, "unterminated section");
        }
    }
    if (!have_n || !have_e) return io_error(path, "no $Nodes or no $Elements section");
    out.tets.resize(tet_tags.size());
    for (size_t i = 0; i < tet_tags.size(); ++i) {
        const auto it = index.find(tet_tags[i]);
        if (it == index.end()) return io_error(path, "element refers to an unknown node");
        out.tets[i] = it->second;
    }
    return TV_OK;
}

tv_status read_mesh(const char *path, tv_host_mesh *out) {
    Reader r;
    if (!r.load(path)) return tv::set_error(TV_ERR_IO, "%s: cannot read", path);
    Parsed p;
    r.hash_comments = true;  // a MEDIT file may open with comments; Gmsh files have none
    const std::string first = r.token();
    r.hash_comments = false;
    tv_status st;
    if (first == "MeshVersionFormatted") {
        r.pos = 0;
        st = read_medit(r, path, p);
    } else if (first == "$MeshFormat") {
        st = read_gmsh(r, path, p);
    } else {
        return io_error(path, "not a MEDIT .mesh or Gmsh .msh ASCII file");
    }
    if (st) return st;
    const int64_t nv = (int64_t)(p.verts.size() / 3), nt = (int64_t)(p.tets.size() / 4);
    for (int32_t v : p.tets)
        if (v < 0 || v >= nv) return io_error(path, "tet index out of range");
    out->verts = static_cast<float *>(malloc(sizeof(float) * (size_t)(3 * nv + 1)));
    out->tets = static_cast<int32_t *>(malloc(sizeof(int32_t) * (size_t)(4 * nt + 1)));
    if (!out->verts || !out->tets) {
        tv_free_host_mesh(out);
        return tv::set_error(TV_ERR_IO, "%s: out of host memory", path);
    }
    memcpy(out->verts, p.verts.data(), sizeof(float) * (size_t)(3 * nv));
    memcpy(out->tets, p.tets.data(), sizeof(int32_t) * (size_t)(4 * nt));
    out->nv = nv;
    out->nt = nt;
    out->skipped_elements = p.skipped;
    for (int a = 0; a < 3; ++a) {
        float lo = nv ? p.verts[(size_t)a] : 0.0f, hi = lo;
        for (int64_t i = 1; i < nv; ++i) {
            const float x = p.verts[(size_t)(3 * i + a)];
            lo = x < lo ? x : lo;
            hi = x > hi ? x : hi;
        }
        out->bbox.lo[a] = lo;
        out->bbox.hi[a] = hi;
    }
    return TV_OK;
}

}  // namespace

extern "C" {

tv_status tv_read_mesh(const char *path, tv_host_mesh *out) {
    if (!path || !out) return tv::set_error(TV_ERR_INVALID_ARG, "null path or output");
    memset(out, 0, sizeof *out);
    // no exception may cross the C ABI: a file too large for host memory is
    // an I/O error like any other unreadable file
    try {
        const tv_status st = read_mesh(path, out);
        if (st) tv_free_host_mesh(out);
        return st;
    } catch (const std::exception &e) {
        tv_free_host_mesh(out);
        return tv::set_error(TV_ERR_IO, "%s: %s", path, e.what());
    } catch (...) {
        tv_free_host_mesh(out);
        return tv::set_error(TV_ERR_IO, "%s: cannot read", path);
    }
}

void tv_free_host_mesh(tv_host_mesh *m) {
    if (!m) return;
    free(m->verts);
    free(m->tets);
    m->verts = nullptr;
    m->tets = nullptr;
    m->nv = m->nt = 0;
}

}  // extern "C"
