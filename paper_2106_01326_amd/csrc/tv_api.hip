// C ABI of the voxelizer: argument checks, workspace carving and the launch
// sequence shared by the single-mesh and batch calls.  Declarations and the
// contract are in include/tv.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "tv.h"
#include "tv_internal.h"
#include "tv_kernels.h"
#include "tv_profile.h"
#include "tv_workspace.h"

namespace {

thread_local char g_last_error[256] = "";

// Launch parameters in force for single-mesh calls ([0]) and batch calls
// ([1]); each call takes a copy when it starts.  (They do not depend on the
// device, so neither do workspace sizes.)
std::mutex g_params_mu;
tv::Params g_params[2] = {tv::kDefaultSingle, tv::kDefaultBatch};

tv::Params current_params(int which) {
    std::lock_guard<std::mutex> lk(g_params_mu);
    return g_params[which];
}

tv_status fail(tv_status code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
    return code;
}

tv_status check_hip(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(TV_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return TV_OK;
}

bool pow2_dim(int32_t n) { return n >= 1 && n <= 32768 && (n & (n - 1)) == 0; }

tv::GridGeom make_geom(tv_dims d) {
    tv::GridGeom g;
    const int32_t n[3] = {d.nx, d.ny, d.nz};
    for (int a = 0; a < 3; ++a) {
        g.n[a] = n[a];
        g.shift[a] = tv::kLatticeBits - tv::ilog2(n[a]);
        g.half[a] = (1 << (tv::kLatticeBits - 1)) / n[a];
    }
    g.words = (d.nz + 31) / 32;
    return g;
}

// Compute units of the current device (cached per device id).
int device_cus() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            n <= 0)
            n = 256;
        cached[dev] = n;
    }
    return cached[dev];
}

constexpr uint32_t kKnownFlags = TV_TIE_STRICT | TV_PATH_PER_TET | TV_ACCUMULATE;
constexpr int64_t kMaxTets = (int64_t)1 << 28;  // piece slots stay below 2^32

// Host-visible checks of one mesh; `which` prefixes messages of batch entries.
tv_status check_mesh_impl(const void *verts, uint32_t fmt, int64_t nv, const int32_t *tets, int64_t nt,
                     tv_dims dims, const tv_bbox *bbox, const uint32_t *grid, const char *which) {
    if (!pow2_dim(dims.nx) || !pow2_dim(dims.ny) || !pow2_dim(dims.nz))
        return fail(TV_ERR_UNSUPPORTED_DIMS,
                    "%sdims (%d,%d,%d): each must be a power of two in [1,32768]", which, dims.nx,
                    dims.ny, dims.nz);
    if (nv < 0 || nt < 0 || nv > INT32_MAX || nt > kMaxTets)
        return fail(TV_ERR_INVALID_ARG, "%ssizes nv=%lld nt=%lld out of range", which,
                    (long long)nv, (long long)nt);
    if (!grid) return fail(TV_ERR_INVALID_ARG, "%sgrid is null", which);
    if (nt > 0 && (!tets || !verts || nv == 0))
        return fail(TV_ERR_INVALID_ARG, "%snull vertex/tet array with nt > 0", which);
    if (((uintptr_t)tets & 15u) || ((uintptr_t)verts & 3u) || ((uintptr_t)grid & 3u))
        return fail(TV_ERR_INVALID_ARG, "%stets must be 16-byte, verts and grid 4-byte aligned",
                    which);
    if (fmt != TV_VERTS_F32 && fmt != TV_VERTS_Q32)
        return fail(TV_ERR_INVALID_ARG, "%sunknown vertex format %u", which, fmt);
    if (fmt == TV_VERTS_F32) {
        for (int a = 0; a < 3; ++a)
            if (!isfinite(bbox->lo[a]) || !isfinite(bbox->hi[a]) || !(bbox->hi[a] > bbox->lo[a]))
                return fail(TV_ERR_INVALID_ARG, "%sbbox axis %d: need finite lo < hi", which, a);
    }
    return TV_OK;
}

tv::MeshDesc make_desc_impl(const void *verts, uint32_t fmt, int64_t nv, const int32_t *tets,
                       int64_t nt, tv_dims dims, const tv_bbox *bbox, uint32_t *grid,
                       const tv::Params &P) {
    tv::MeshDesc d;
    memset(&d, 0, sizeof d);
    d.verts = verts;
    d.tets = reinterpret_cast<const int4 *>(tets);
    d.grid = grid;
    d.nv = nv;
    d.nt = nt;
    d.g = make_geom(dims);
    d.p = tv::plan_tiles(dims, P.min_tiles, P.tile_cols_log2);
    d.fmt = fmt == TV_VERTS_F32 ? tv::kFmtF32 : tv::kFmtQ32;
    d.direct = d.p.ntiles == 1 ? 1 : 0;
    if (fmt == TV_VERTS_F32) {
        for (int a = 0; a < 3; ++a) {
            d.box.lo[a] = (double)bbox->lo[a];
            d.box.ext[a] = (double)bbox->hi[a] - (double)bbox->lo[a];
        }
    }
    return d;
}

// Fills the bases of the descriptors and the call totals.  `table`: the
// descriptors go into a device table in the workspace (batch calls).
tv::CallSizes assign_bases_impl(std::vector<tv::MeshDesc> &descs, bool table) {
    tv::CallSizes c = {(int64_t)descs.size(), 0, 0, 0, table};
    for (size_t i = 0; i < descs.size(); ++i) {
        tv::MeshDesc &d = descs[i];
        d.mesh = (int32_t)i;
        d.vert_base = c.nv;
        d.tet_base = c.nt;
        d.tile_base = c.ntiles;
        c.nv += d.nv;
        c.nt += d.nt;
        c.ntiles += d.p.ntiles;
    }
    return c;
}

// Copies the descriptor table and its prefix sums (vertex, tet and tile
// bases, each with a final total) into the workspace, on `s`.
tv_status upload_table(const std::vector<tv::MeshDesc> &descs, const tv::CallSizes &c, uint8_t *ws,
                       hipStream_t s) {
    const tv::WorkspaceLayout L = tv::layout(c);
    std::vector<uint8_t> host(L.descs_bytes);
    memcpy(host.data(), descs.data(), sizeof(tv::MeshDesc) * descs.size());
    int64_t *pre = reinterpret_cast<int64_t *>(host.data() + sizeof(tv::MeshDesc) * descs.size());
    const size_t n = descs.size();
    for (size_t i = 0; i <= n; ++i) {
        pre[i] = i < n ? descs[i].vert_base : c.nv;
        pre[n + 1 + i] = i < n ? descs[i].tet_base : c.nt;
        pre[2 * (n + 1) + i] = i < n ? descs[i].tile_base : c.ntiles;
    }
    if (hipMemcpyAsync(ws + L.descs, host.data(), L.descs_bytes, hipMemcpyHostToDevice, s) !=
        hipSuccess)
        return fail(TV_ERR_HIP, "descriptor upload failed");
    return TV_OK;
}

// Kernel-side view of a call: the descriptor table in the workspace, or the
// single descriptor `one` passed by value.
tv::MeshTable make_table(const tv::CallSizes &c, uint8_t *ws, const tv::MeshDesc *one,
                         uint32_t flags, const tv::Params &P) {
    const tv::WorkspaceLayout L = tv::layout(c);
    tv::MeshTable T;
    memset(&T, 0, sizeof T);
    T.n = (int32_t)c.meshes;
    T.chunk = P.chunk ? P.chunk : tv::auto_chunk(c.nt, c.ntiles, c.table);
    T.strip = P.strip;
    T.piece_cap = P.piece_cap;
    T.nocull = P.cull;
    T.accumulate = (flags & TV_ACCUMULATE) ? 1 : 0;
    T.nv_total = c.nv;
    T.nt_total = c.nt;
    T.ntiles_total = c.ntiles;
    if (c.table) {
        uint8_t *dev = ws + L.descs;
        const size_t n = (size_t)c.meshes;
        T.descs = reinterpret_cast<const tv::MeshDesc *>(dev);
        const int64_t *dpre = reinterpret_cast<const int64_t *>(dev + sizeof(tv::MeshDesc) * n);
        T.vert_pre = dpre;
        T.tet_pre = dpre + (n + 1);
        T.tile_pre = dpre + 2 * (n + 1);
    } else {
        T.one = *one;
    }
    return T;
}

// The launch sequence: kernels only (no host copies, memsets or
// allocations).  The host descriptors `descs[0, ndescs)` are needed by the
// per-tet reference path only.
tv_status enqueue(const tv::MeshTable &T, const tv::CallSizes &c, uint8_t *ws, hipStream_t s,
                  uint32_t flags, const tv::MeshDesc *descs, size_t ndescs, int wgs_per_cu) {
    const tv::WorkspaceLayout L = tv::layout(c);
    const tv::BinBuffers b = tv::bin_buffers(ws, L);
    const bool strict = (flags & TV_TIE_STRICT) != 0;
    const bool accumulate = (flags & TV_ACCUMULATE) != 0;
    tv::profile_count_call();
    {
        tv::StageScope sc(tv::kStageClear, s);
        if (!accumulate) {
            tv::launch_clear(b.meta, (int64_t)L.clear_end / 4, s);
        } else {
            // keep the status words: data errors of earlier accumulated calls stay visible
            tv::launch_clear(b.meta, tv::kMetaWords, s);
            tv::launch_clear(b.tile_count, (int64_t)(L.clear_end - L.tile_count) / 4, s);
        }
        tv::launch_set_word(b.meta + tv::kMetaMeshes, (uint32_t)c.meshes, s);
    }
    {
        tv::StageScope sc(tv::kStageIngest, s);
        tv::launch_ingest(T, b, s);
    }
    tv_status st = check_hip("ingest launch");
    if (st) return st;
    if (flags & TV_PATH_PER_TET) {
        if (!descs) return fail(TV_ERR_INVALID_ARG, "the per-tet path needs host descriptors");
        tv::StageScope sc(tv::kStageVoxelize, s);
        for (size_t i = 0; i < ndescs; ++i) {
            const tv::MeshDesc &d = descs[i];
            if (!accumulate) tv::launch_clear(d.grid, (int64_t)d.g.n[0] * d.g.n[1] * d.g.words, s);
            tv::launch_voxelize_per_tet(d, b, strict, s);
        }
        return check_hip("per-tet voxelize launch");
    }
    {
        tv::StageScope sc(tv::kStageBin, s);
        tv::launch_bin_count(T, b, s);
        tv::launch_scan_tiles(T, b, s);
        tv::launch_bin_scatter(T, b, s);
        if (!accumulate && !T.bricks.index) tv::launch_zero_shared_tiles(T, b, s);
    }
    if ((st = check_hip("binning launch"))) return st;
    const int cus = device_cus();
    {
        tv::StageScope sc(tv::kStageVoxelize, s);
        tv::launch_tile_voxelize(T, b, strict, wgs_per_cu * cus, s);
    }
    {
        tv::StageScope sc(tv::kStageLarge, s);
        tv::launch_large_tets(T, b, strict, cus, s);
        if (T.bricks.index) tv::launch_bricks_canonical(T, b, 4 * cus, s);
    }
    return check_hip("voxelize launch");
}

// The whole call for final descriptors: table upload (batch calls), then
// the launch sequence.
tv_status run_impl(std::vector<tv::MeshDesc> &descs, const tv::CallSizes &c, uint8_t *ws,
                   hipStream_t s, uint32_t flags, const tv::Params &P) {
    if (c.table) {
        const tv_status st = upload_table(descs, c, ws, s);
        if (st) return st;
    }
    const tv::MeshTable T = make_table(c, ws, descs.data(), flags, P);
    return enqueue(T, c, ws, s, flags, descs.data(), descs.size(), P.wgs_per_cu);
}

// Workspace bytes of a single-mesh call under parameters P.
size_t single_ws_bytes(int64_t nv, int64_t nt, tv_dims dims, const tv::Params &P) {
    tv::CallSizes c = {1, nv, nt, tv::plan_tiles(dims, P.min_tiles, P.tile_cols_log2).ntiles};
    return tv::layout(c).total;
}

// Consistency tag of a batch plan (catches plans not made by
// tv_batch_prepare, or edited since).
uint32_t plan_check(const tv_batch_plan &p) {
    uint64_t h = 0x9e3779b97f4a7c15ull;
    const uint64_t v[9] = {(uint64_t)p.meshes,
                           (uint64_t)p.nv,
                           (uint64_t)p.nt,
                           (uint64_t)p.ntiles,
                           p.ws,
                           (uint64_t)p.flags,
                           (uint64_t)(uint32_t)p.launch[0] << 32 | (uint32_t)p.launch[1],
                           (uint64_t)(uint32_t)p.launch[2] << 32 | (uint32_t)p.launch[3],
                           (uint64_t)(uint32_t)p.launch[4]};
    for (uint64_t x : v) {
        h ^= x + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
        h *= 0xff51afd7ed558ccdull;
    }
    return (uint32_t)(h ^ (h >> 32)) | 1u;
}

tv_status check_ws(void *ws, size_t ws_bytes, size_t need, uint32_t flags) {
    if (flags & ~kKnownFlags) return fail(TV_ERR_INVALID_ARG, "unknown flag bits 0x%x", flags);
    if (!ws || ((uintptr_t)ws & 255u))
        return fail(TV_ERR_WORKSPACE, "workspace null or not 256-byte aligned");
    if (ws_bytes < need)
        return fail(TV_ERR_WORKSPACE, "workspace of %zu bytes, need %zu", ws_bytes, need);
    return TV_OK;
}

tv_status voxelize_one(const void *verts, uint32_t fmt, int64_t nv, const int32_t *tets, int64_t nt,
                       tv_dims dims, const tv_bbox *bbox, uint32_t *grid, void *ws, size_t ws_bytes,
                       void *stream, uint32_t flags) {
    tv_status st = check_mesh_impl(verts, fmt, nv, tets, nt, dims, bbox, grid, "");
    if (st) return st;
    const tv::Params P = current_params(0);
    if ((st = check_ws(ws, ws_bytes, single_ws_bytes(nv, nt, dims, P), flags))) return st;
    std::vector<tv::MeshDesc> descs(1, make_desc_impl(verts, fmt, nv, tets, nt, dims, bbox, grid, P));
    const tv::CallSizes c = assign_bases_impl(descs, false);
    return run_impl(descs, c, static_cast<uint8_t *>(ws), reinterpret_cast<hipStream_t>(stream), flags,
                    P);
}

bool batch_descs(const tv_mesh *meshes, int32_t n, const tv::Params &P,
                 std::vector<tv::MeshDesc> &descs, tv_status &st) {
    descs.clear();
    descs.reserve((size_t)n);
    char which[48];
    for (int32_t i = 0; i < n; ++i) {
        const tv_mesh &m = meshes[i];
        snprintf(which, sizeof which, "mesh %d: ", i);
        st = check_mesh_impl(m.verts, m.vert_format, m.nv, m.tets, m.nt, m.dims, &m.bbox, m.grid, which);
        if (st) return false;
        descs.push_back(make_desc_impl(m.verts, m.vert_format, m.nv, m.tets, m.nt, m.dims, &m.bbox,
                                       m.grid, P));
    }
    st = TV_OK;
    return true;
}

}  // namespace

namespace tv {

tv_status check_mesh(const void *verts, uint32_t fmt, int64_t nv, const int32_t *tets, int64_t nt,
                     tv_dims dims, const tv_bbox *bbox, const uint32_t *grid, const char *which) {
    return check_mesh_impl(verts, fmt, nv, tets, nt, dims, bbox, grid, which);
}

MeshDesc make_batch_desc(const void *verts, uint32_t fmt, int64_t nv, const int32_t *tets,
                         int64_t nt, tv_dims dims, const tv_bbox *bbox, uint32_t *grid) {
    return make_desc_impl(verts, fmt, nv, tets, nt, dims, bbox, grid, kDefaultBatch);
}

CallSizes assign_bases(std::vector<MeshDesc> &descs) {
    return assign_bases_impl(descs, descs.size() > 1);
}

tv_status run_meshes(std::vector<MeshDesc> &descs, const CallSizes &c, uint8_t *ws, hipStream_t s,
                     uint32_t flags) {
    return run_impl(descs, c, ws, s, flags, kDefaultBatch);
}

tv_status set_error(tv_status code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
    return code;
}

}  // namespace tv

// ------------------------------------------------ allocation-free call
//
// tv_voxelize_noalloc takes its workspace from a fixed device array instead
// of the caller.  Host code must never pass `scratch` itself to a kernel or a
// copy: in host code the name is only a stand-in for the symbol, so the
// device address of each GPU's copy is fetched once per device with
// hipGetSymbolAddress and cached.
constexpr size_t kStaticScratchBytes = TV_NOALLOC_MAX_BYTES;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array.
tv_status static_scratch(uint8_t **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(TV_ERR_HIP, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(TV_ERR_HIP, "device %d beyond the %d the scratch table holds", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(TV_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<uint8_t *>(p);
    }
    *out = g_scratch_ptr[dev];
    return TV_OK;
}

// The call's data-error status word -> a tv_status, in device memory.
__global__ void k_status_code(const uint32_t *word, int32_t *out) {
    const uint32_t w = *word;
    *out = (w & tv::kStatusIndex) ? TV_ERR_INDEX : (w & tv::kStatusRange) ? TV_ERR_RANGE : TV_OK;
}

}  // namespace

extern "C" {

size_t tv_grid_words(tv_dims d) {
    if (!pow2_dim(d.nx) || !pow2_dim(d.ny) || !pow2_dim(d.nz)) return 0;
    return (size_t)d.nx * (size_t)d.ny * (size_t)((d.nz + 31) / 32);
}

size_t tv_workspace_bytes(int64_t nv, int64_t nt, tv_dims dims, uint32_t flags) {
    (void)flags;
    if (nv < 0 || nt < 0 || !tv_grid_words(dims)) return 0;
    return single_ws_bytes(nv, nt, dims, current_params(0));
}

tv_status tv_voxelize(const float *verts, int64_t nv, const int32_t *tets, int64_t nt,
                      tv_dims dims, tv_bbox bbox, uint32_t *grid, void *ws, size_t ws_bytes,
                      void *stream, uint32_t flags) {
    return voxelize_one(verts, TV_VERTS_F32, nv, tets, nt, dims, &bbox, grid, ws, ws_bytes, stream,
                        flags);
}

tv_status tv_voxelize_q(const int32_t *qverts, int64_t nv, const int32_t *tets, int64_t nt,
                        tv_dims dims, uint32_t *grid, void *ws, size_t ws_bytes, void *stream,
                        uint32_t flags) {
    return voxelize_one(qverts, TV_VERTS_Q32, nv, tets, nt, dims, nullptr, grid, ws, ws_bytes,
                        stream, flags);
}

size_t tv_voxelize_bricks_workspace_bytes(int64_t nv, int64_t nt, tv_dims dims) {
    if (nv < 0 || nt < 0 || !tv_grid_words(dims)) return 0;
    const tv::Params P = current_params(0);
    tv::CallSizes c = {1, nv, nt, tv::plan_tiles(dims, P.min_tiles, P.tile_cols_log2).ntiles};
    c.piece_slots = tv::kPieceCapSparse;
    return tv::layout(c).total;
}

tv_status tv_voxelize_bricks(const float *verts, int64_t nv, const int32_t *tets, int64_t nt,
                             tv_dims dims, tv_bbox bbox, uint32_t *index, uint32_t *pool,
                             uint32_t *pool_ids, int64_t capacity, uint32_t *pool_count, void *ws,
                             size_t ws_bytes, void *stream, uint32_t flags) {
    if (!pow2_dim(dims.nx) || !pow2_dim(dims.ny) || !pow2_dim(dims.nz) || dims.nx < 8 || dims.ny < 8 ||
        dims.nz < 32)
        return fail(TV_ERR_UNSUPPORTED_DIMS,
                    "bricks: dims (%d,%d,%d) must be powers of two with nx, ny >= 8 and nz >= 32",
                    dims.nx, dims.ny, dims.nz);
    const int64_t nbx = dims.nx / 8, nby = dims.ny / 8, nbz = dims.nz / 32;
    const int64_t nbricks = nbx * nby * nbz;
    if (nbricks > (int64_t)0xfffffffe)
        return fail(TV_ERR_UNSUPPORTED_DIMS, "bricks: %lld bricks do not fit 32-bit ids", (long long)nbricks);
    if (!index || !pool_count || capacity < 0 || (capacity > 0 && (!pool || !pool_ids)) ||
        capacity > ((int64_t)1 << 32) - 2)
        return fail(TV_ERR_INVALID_ARG, "bricks: null output or bad capacity %lld", (long long)capacity);
    if (flags & ~(uint32_t)TV_TIE_STRICT)
        return fail(TV_ERR_INVALID_ARG, "bricks: takes TV_TIE_STRICT only (flags 0x%x)", flags);
    if (nt > ((int64_t)1 << 32) / tv::kPieceCapSparse)
        return fail(TV_ERR_INVALID_ARG, "bricks: %lld tets exceed the piece slots", (long long)nt);
    // the index stands in for the grid in the shared checks (only its
    // presence and alignment are looked at)
    tv_status st = check_mesh_impl(verts, TV_VERTS_F32, nv, tets, nt, dims, &bbox, index, "");
    if (st) return st;
    const tv::Params P = current_params(0);
    if ((st = check_ws(ws, ws_bytes, tv_voxelize_bricks_workspace_bytes(nv, nt, dims), flags))) return st;
    tv::MeshDesc d = make_desc_impl(verts, TV_VERTS_F32, nv, tets, nt, dims, &bbox, nullptr, P);
    tv::CallSizes c = {1, nv, nt, d.p.ntiles, false};
    c.piece_slots = tv::kPieceCapSparse;
    tv::MeshTable T = make_table(c, static_cast<uint8_t *>(ws), &d, flags, P);
    // one task per tile, so that a brick has one writer (large tets aside)
    // and the pool holds no slots given up in races between tasks; tets
    // meeting up to 27 tiles go through the tile pipeline
    T.chunk = 1 << 30;
    T.piece_cap = tv::kPieceCapSparse;
    T.bricks.index = index;
    T.bricks.pool = pool;
    T.bricks.ids = pool_ids;
    T.bricks.count = pool_count;
    T.bricks.capacity = capacity;
    T.bricks.nby = (int32_t)nby;
    T.bricks.nbz = (int32_t)nbz;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    tv::launch_clear(index, nbricks, s);
    tv::launch_set_word(pool_count, 0u, s);
    return enqueue(T, c, static_cast<uint8_t *>(ws), s, flags, &d, 1, P.wgs_per_cu);
}

size_t tv_batch_workspace_bytes(const tv_mesh *meshes, int32_t n, uint32_t flags) {
    (void)flags;
    if (!meshes || n <= 0) return 0;
    std::vector<tv::MeshDesc> descs;
    tv_status st;
    if (!batch_descs(meshes, n, current_params(1), descs, st)) return 0;
    return tv::layout(assign_bases_impl(descs, true)).total;
}

tv_status tv_voxelize_batch(const tv_mesh *meshes, int32_t n, void *ws, size_t ws_bytes,
                            void *stream, uint32_t flags) {
    if (!meshes || n <= 0) return fail(TV_ERR_INVALID_ARG, "empty batch");
    const tv::Params P = current_params(1);
    std::vector<tv::MeshDesc> descs;
    tv_status st;
    if (!batch_descs(meshes, n, P, descs, st)) return st;
    const tv::CallSizes c = assign_bases_impl(descs, true);
    if (c.nt > kMaxTets) return fail(TV_ERR_INVALID_ARG, "batch has more than 2^28 tets");
    if ((st = check_ws(ws, ws_bytes, tv::layout(c).total, flags))) return st;
    return run_impl(descs, c, static_cast<uint8_t *>(ws), reinterpret_cast<hipStream_t>(stream), flags,
                    P);
}

tv_status tv_default_params(int32_t which, tv_params *out) {
    if (!out || (which != TV_PARAMS_SINGLE && which != TV_PARAMS_BATCH))
        return fail(TV_ERR_INVALID_ARG, "params: need TV_PARAMS_SINGLE or TV_PARAMS_BATCH and an output");
    const tv::Params &P = which == TV_PARAMS_SINGLE ? tv::kDefaultSingle : tv::kDefaultBatch;
    *out = {P.tile_cols_log2, P.min_tiles, P.chunk, P.strip, P.piece_cap, P.wgs_per_cu, P.cull};
    return TV_OK;
}

tv_status tv_get_params(int32_t which, tv_params *out) {
    if (!out || (which != TV_PARAMS_SINGLE && which != TV_PARAMS_BATCH))
        return fail(TV_ERR_INVALID_ARG, "params: need TV_PARAMS_SINGLE or TV_PARAMS_BATCH and an output");
    const tv::Params P = current_params(which);
    *out = {P.tile_cols_log2, P.min_tiles, P.chunk, P.strip, P.piece_cap, P.wgs_per_cu, P.cull};
    return TV_OK;
}

tv_status tv_set_params(int32_t which, const tv_params *p) {
    if (which != TV_PARAMS_SINGLE && which != TV_PARAMS_BATCH)
        return fail(TV_ERR_INVALID_ARG, "params: need TV_PARAMS_SINGLE or TV_PARAMS_BATCH");
    tv::Params P = which == TV_PARAMS_SINGLE ? tv::kDefaultSingle : tv::kDefaultBatch;
    if (p) {
        if (p->tile_cols_log2 < 3 || p->tile_cols_log2 > 5)
            return fail(TV_ERR_INVALID_ARG, "params: tile_cols_log2 %d not in [3,5]", p->tile_cols_log2);
        if (p->min_tiles < 1 || p->min_tiles > (1 << 20))
            return fail(TV_ERR_INVALID_ARG, "params: min_tiles %d not in [1,2^20]", p->min_tiles);
        if (p->chunk_pieces != 0 && (p->chunk_pieces < 64 || p->chunk_pieces > 65536))
            return fail(TV_ERR_INVALID_ARG, "params: chunk_pieces %d neither 0 nor in [64,65536]",
                        p->chunk_pieces);
        if (p->strip_columns < 1 || p->strip_columns > 64)
            return fail(TV_ERR_INVALID_ARG, "params: strip_columns %d not in [1,64]", p->strip_columns);
        if (p->piece_cap < 1 || p->piece_cap > tv::kPieceCap)
            return fail(TV_ERR_INVALID_ARG, "params: piece_cap %d not in [1,%d]", p->piece_cap, tv::kPieceCap);
        if (p->wgs_per_cu < 1 || p->wgs_per_cu > 8)
            return fail(TV_ERR_INVALID_ARG, "params: wgs_per_cu %d not in [1,8]", p->wgs_per_cu);
        if (p->cull_columns < 0 || p->cull_columns > 1024)
            return fail(TV_ERR_INVALID_ARG, "params: cull_columns %d not in [0,1024]", p->cull_columns);
        P = {p->tile_cols_log2, p->min_tiles, p->chunk_pieces, p->strip_columns, p->piece_cap,
             p->wgs_per_cu, p->cull_columns};
    }
    std::lock_guard<std::mutex> lk(g_params_mu);
    g_params[which] = P;
    return TV_OK;
}

tv_status tv_batch_prepare(const tv_mesh *meshes, int32_t n, void *ws, size_t ws_bytes,
                           void *stream, uint32_t flags, tv_batch_plan *plan) {
    if (!plan) return fail(TV_ERR_INVALID_ARG, "plan is null");
    memset(plan, 0, sizeof *plan);
    if (!meshes || n <= 0) return fail(TV_ERR_INVALID_ARG, "empty batch");
    if (flags & TV_PATH_PER_TET)
        return fail(TV_ERR_INVALID_ARG, "the per-tet path is not available for a prepared batch");
    const tv::Params P = current_params(1);
    std::vector<tv::MeshDesc> descs;
    tv_status st;
    if (!batch_descs(meshes, n, P, descs, st)) return st;
    const tv::CallSizes c = assign_bases_impl(descs, true);
    if (c.nt > kMaxTets) return fail(TV_ERR_INVALID_ARG, "batch has more than 2^28 tets");
    if ((st = check_ws(ws, ws_bytes, tv::layout(c).total, flags))) return st;
    if ((st = upload_table(descs, c, static_cast<uint8_t *>(ws), reinterpret_cast<hipStream_t>(stream))))
        return st;
    // runs with TV_ACCUMULATE keep the status words: start them clear
    const tv::WorkspaceLayout L = tv::layout(c);
    if (hipMemsetAsync(static_cast<uint8_t *>(ws) + L.status, 0, 4 * (size_t)tv::status_words(c.meshes),
                       reinterpret_cast<hipStream_t>(stream)) != hipSuccess)
        return fail(TV_ERR_HIP, "status clear failed");
    plan->meshes = c.meshes;
    plan->nv = c.nv;
    plan->nt = c.nt;
    plan->ntiles = c.ntiles;
    plan->ws = (uint64_t)(uintptr_t)ws;
    plan->flags = flags;
    plan->launch[0] = P.chunk;
    plan->launch[1] = P.strip;
    plan->launch[2] = P.piece_cap;
    plan->launch[3] = P.wgs_per_cu;
    plan->launch[4] = P.cull;
    plan->check = plan_check(*plan);
    return TV_OK;
}

tv_status tv_batch_run(const tv_batch_plan *plan, void *ws, size_t ws_bytes, void *stream) {
    if (!plan || plan->check != plan_check(*plan) || plan->meshes <= 0)
        return fail(TV_ERR_INVALID_ARG, "not a plan filled by tv_batch_prepare");
    if (plan->ws != (uint64_t)(uintptr_t)ws)
        return fail(TV_ERR_INVALID_ARG, "the plan belongs to another workspace");
    const tv::CallSizes c = {plan->meshes, plan->nv, plan->nt, plan->ntiles, true};
    tv_status st;
    if ((st = check_ws(ws, ws_bytes, tv::layout(c).total, plan->flags))) return st;
    uint8_t *w = static_cast<uint8_t *>(ws);
    tv::Params P = tv::kDefaultBatch;  // the tile plan is already in the table
    P.chunk = plan->launch[0];
    P.strip = plan->launch[1];
    P.piece_cap = plan->launch[2];
    P.wgs_per_cu = plan->launch[3];
    P.cull = plan->launch[4];
    const tv::MeshTable T = make_table(c, w, nullptr, plan->flags, P);
    return enqueue(T, c, w, reinterpret_cast<hipStream_t>(stream), plan->flags, nullptr, 0,
                   P.wgs_per_cu);
}

tv_status tv_voxelize_pipelined(const float *verts_host, int64_t nv, const int32_t *tets_host,
                                int64_t nt, tv_dims dims, tv_bbox bbox, float *verts_dev,
                                int32_t *tets_dev, uint32_t *grid, void *ws, size_t ws_bytes,
                                void *stream, void *copy_stream, int32_t chunks, uint32_t flags) {
    if ((flags & TV_ACCUMULATE) || (flags & ~kKnownFlags))
        return fail(TV_ERR_INVALID_ARG, "bad flags 0x%x for a pipelined call", flags);
    if (nv < 0 || nt < 0 || (nv && (!verts_host || !verts_dev)) || (nt && (!tets_host || !tets_dev)))
        return fail(TV_ERR_INVALID_ARG, "null or negative pipelined inputs");
    const int64_t k = chunks < 1 ? 1 : (chunks > 64 ? 64 : chunks);
    const int64_t per = nt ? (nt + k - 1) / k : 0;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const hipStream_t cs = reinterpret_cast<hipStream_t>(copy_stream);
    // host checks of the whole call before anything is enqueued
    tv_status st = check_mesh_impl(verts_dev, TV_VERTS_F32, nv, tets_dev, nt, dims, &bbox, grid, "");
    if (st) return st;
    if ((st = check_ws(ws, ws_bytes, tv_workspace_bytes(nv, per, dims, flags), flags))) return st;
    const int64_t nslices = per ? (nt + per - 1) / per : 1;
    if (nslices == 1) {
        // nothing to overlap: copy and voxelize in order on one stream
        bool ok = true;
        if (nv) ok = hipMemcpyAsync(verts_dev, verts_host, (size_t)12 * (size_t)nv, hipMemcpyHostToDevice, s) ==
                     hipSuccess;
        if (nt) ok = ok && hipMemcpyAsync(tets_dev, tets_host, (size_t)16 * (size_t)nt, hipMemcpyHostToDevice,
                                          s) == hipSuccess;
        if (!ok) return fail(TV_ERR_HIP, "pipelined copy failed");
        return voxelize_one(verts_dev, TV_VERTS_F32, nv, tets_dev, nt, dims, &bbox, grid, ws, ws_bytes, s,
                            flags);
    }
    // events come from a per-thread, per-device pool (recording an event again
    // does not disturb waits already enqueued on its earlier record)
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(TV_ERR_HIP, "no current device");
    thread_local std::vector<std::vector<hipEvent_t>> pool;
    if ((size_t)dev >= pool.size()) pool.resize((size_t)dev + 1);
    std::vector<hipEvent_t> &ev = pool[(size_t)dev];
    while (ev.size() < (size_t)nslices + 1) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return fail(TV_ERR_HIP, "event creation failed");
        ev.push_back(e);
    }
    bool ok = true;
    if (nv) ok = hipMemcpyAsync(verts_dev, verts_host, (size_t)12 * (size_t)nv, hipMemcpyHostToDevice, cs) ==
                 hipSuccess;
    ok = ok && hipEventRecord(ev[0], cs) == hipSuccess;
    for (int64_t i = 0; ok && i < nslices; ++i) {
        const int64_t t0 = i * per, n = per ? (nt - t0 < per ? nt - t0 : per) : 0;
        if (n) ok = hipMemcpyAsync(tets_dev + 4 * t0, tets_host + 4 * t0, (size_t)16 * (size_t)n,
                                   hipMemcpyHostToDevice, cs) == hipSuccess;
        ok = ok && hipEventRecord(ev[(size_t)i + 1], cs) == hipSuccess;
    }
    ok = ok && hipStreamWaitEvent(s, ev[0], 0) == hipSuccess;
    for (int64_t i = 0; ok && i < nslices; ++i) {
        const int64_t t0 = i * per, n = per ? (nt - t0 < per ? nt - t0 : per) : 0;
        ok = hipStreamWaitEvent(s, ev[(size_t)i + 1], 0) == hipSuccess;
        if (!ok) break;
        st = voxelize_one(verts_dev, TV_VERTS_F32, nv, tets_dev + 4 * t0, n, dims, &bbox, grid, ws, ws_bytes,
                          s, flags | (i ? TV_ACCUMULATE : 0u));
        if (st) break;
    }
    if (st) return st;
    if (!ok) return fail(TV_ERR_HIP, "pipelined copy or wait failed");
    return check_hip("pipelined voxelize");
}

tv_status tv_snap(const float *verts, int64_t nv, tv_bbox bbox, int32_t *q_out, void *stream) {
    if (nv < 0 || nv > INT32_MAX || (nv > 0 && (!verts || !q_out)))
        return fail(TV_ERR_INVALID_ARG, "bad snap arguments");
    tv::BoxD box;
    for (int a = 0; a < 3; ++a) {
        if (!isfinite(bbox.lo[a]) || !isfinite(bbox.hi[a]) || !(bbox.hi[a] > bbox.lo[a]))
            return fail(TV_ERR_INVALID_ARG, "bbox axis %d: need finite lo < hi", a);
        box.lo[a] = (double)bbox.lo[a];
        box.ext[a] = (double)bbox.hi[a] - (double)bbox.lo[a];
    }
    tv::launch_snap_only(verts, nv, box, q_out, reinterpret_cast<hipStream_t>(stream));
    return check_hip("snap launch");
}

tv_status tv_fetch_status(const void *ws, int32_t mesh_index, void *stream) {
    if (!ws || mesh_index < 0) return fail(TV_ERR_INVALID_ARG, "bad workspace or mesh index");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    uint32_t meshes = 0, word = 0;
    const uint8_t *w = static_cast<const uint8_t *>(ws);
    if (hipMemcpyAsync(&meshes, w + 4 * tv::kMetaMeshes, 4, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(TV_ERR_HIP, "reading the workspace header failed");
    if ((uint32_t)mesh_index >= meshes)
        return fail(TV_ERR_INVALID_ARG, "mesh index %d outside the last call's %u meshes",
                    mesh_index, meshes);
    if (hipMemcpyAsync(&word, w + 4 * tv::kMetaWords + 4 * (size_t)mesh_index, 4,
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(TV_ERR_HIP, "reading the status word failed");
    if (word & tv::kStatusIndex) return TV_ERR_INDEX;
    if (word & tv::kStatusRange) return TV_ERR_RANGE;
    if (word & tv::kStatusFull) return TV_ERR_TOO_LARGE;
    return TV_OK;
}

const char *tv_status_string(tv_status s) {
    switch (s) {
    case TV_OK: return "TV_OK";
    case TV_ERR_INVALID_ARG: return "TV_ERR_INVALID_ARG";
    case TV_ERR_UNSUPPORTED_DIMS: return "TV_ERR_UNSUPPORTED_DIMS";
    case TV_ERR_INDEX: return "TV_ERR_INDEX";
    case TV_ERR_RANGE: return "TV_ERR_RANGE";
    case TV_ERR_WORKSPACE: return "TV_ERR_WORKSPACE";
    case TV_ERR_HIP: return "TV_ERR_HIP";
    case TV_ERR_TOO_LARGE: return "TV_ERR_TOO_LARGE";
    case TV_ERR_TIMEOUT: return "TV_ERR_TIMEOUT";
    case TV_ERR_NOT_FOUND: return "TV_ERR_NOT_FOUND";
    case TV_ERR_IO: return "TV_ERR_IO";
    default: return "TV_ERR_UNKNOWN";
    }
}

const char *tv_last_error(void) { return g_last_error; }

tv_status tv_voxelize_noalloc(const float *verts, int64_t nv, const int32_t *tets, int64_t nt,
                              tv_dims dims, tv_bbox bbox, uint32_t *grid, int32_t *status_out,
                              void *stream, uint32_t flags) {
    tv_status st = check_mesh_impl(verts, TV_VERTS_F32, nv, tets, nt, dims, &bbox, grid, "");
    if (st) return st;
    if (flags & ~(uint32_t)TV_TIE_STRICT)
        return fail(TV_ERR_INVALID_ARG, "tv_voxelize_noalloc takes TV_TIE_STRICT only (flags 0x%x)",
                    flags);
    const tv::Params P = current_params(0);
    const size_t need = single_ws_bytes(nv, nt, dims, P);
    if (need > kStaticScratchBytes)
        return fail(TV_ERR_WORKSPACE,
                    "mesh needs %zu bytes of scratch; the allocation-free call holds %zu "
                    "(use tv_voxelize with a workspace)",
                    need, kStaticScratchBytes);
    uint8_t *ws = nullptr;
    if ((st = static_scratch(&ws))) return st;
    const tv::MeshDesc d = make_desc_impl(verts, TV_VERTS_F32, nv, tets, nt, dims, &bbox, grid, P);
    tv::MeshDesc one = d;
    one.mesh = 0;
    const tv::CallSizes c = {1, nv, nt, d.p.ntiles, false};
    const tv::MeshTable T = make_table(c, ws, &one, flags, P);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if ((st = enqueue(T, c, ws, s, flags, &one, 1, P.wgs_per_cu))) return st;
    if (status_out) {
        const tv::WorkspaceLayout L = tv::layout(c);
        k_status_code<<<1, 1, 0, s>>>(reinterpret_cast<const uint32_t *>(ws + L.status), status_out);
        return check_hip("status launch");
    }
    return TV_OK;
}

}  // extern "C"
