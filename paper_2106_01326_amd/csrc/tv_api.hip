// C ABI of the voxelizer: argument checks, workspace carving and the launch
// sequence of the single-mesh path.  Declarations and the contract are in
// include/tv.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "tv.h"
#include "tv_kernels.h"
#include "tv_profile.h"
#include "tv_workspace.h"

namespace {

thread_local char g_last_error[256] = "";

// Tiles wanted per grid before tiles are made smaller (independent of the
// device so that workspace sizes do not depend on it).
constexpr int64_t kMinTiles = 512;

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

constexpr uint32_t kKnownFlags = TV_TIE_STRICT | TV_PATH_PER_TET;
constexpr int64_t kMaxTets = (int64_t)1 << 28;  // piece slots stay below 2^32

tv_status check_common(int64_t nv, const int32_t *tets, int64_t nt, tv_dims dims, uint32_t *grid,
                       void *ws, size_t ws_bytes, uint32_t flags, const void *verts) {
    if (!pow2_dim(dims.nx) || !pow2_dim(dims.ny) || !pow2_dim(dims.nz))
        return fail(TV_ERR_UNSUPPORTED_DIMS,
                    "dims (%d,%d,%d): each must be a power of two in [1,32768]", dims.nx, dims.ny,
                    dims.nz);
    if (nv < 0 || nt < 0 || nv > INT32_MAX || nt > kMaxTets)
        return fail(TV_ERR_INVALID_ARG, "sizes nv=%lld nt=%lld out of range", (long long)nv,
                    (long long)nt);
    if (!grid) return fail(TV_ERR_INVALID_ARG, "grid is null");
    if (nt > 0 && (!tets || !verts || nv == 0))
        return fail(TV_ERR_INVALID_ARG, "null vertex/tet array with nt > 0");
    if (((uintptr_t)tets & 15u) || ((uintptr_t)verts & 3u))
        return fail(TV_ERR_INVALID_ARG, "tets must be 16-byte and verts 4-byte aligned");
    if (flags & ~kKnownFlags) return fail(TV_ERR_INVALID_ARG, "unknown flag bits 0x%x", flags);
    if (!ws || ((uintptr_t)ws & 255u))
        return fail(TV_ERR_WORKSPACE, "workspace null or not 256-byte aligned");
    const size_t need = tv_workspace_bytes(nv, nt, dims, flags);
    if (ws_bytes < need)
        return fail(TV_ERR_WORKSPACE, "workspace of %zu bytes, need %zu", ws_bytes, need);
    return TV_OK;
}

tv_status check_bbox(const tv_bbox &bbox, tv::BoxD &box) {
    for (int a = 0; a < 3; ++a) {
        if (!isfinite(bbox.lo[a]) || !isfinite(bbox.hi[a]) || !(bbox.hi[a] > bbox.lo[a]))
            return fail(TV_ERR_INVALID_ARG, "bbox axis %d: need finite lo < hi", a);
        box.lo[a] = (double)bbox.lo[a];
        box.ext[a] = (double)bbox.hi[a] - (double)bbox.lo[a];
    }
    return TV_OK;
}

// Everything after ingest: binning, tile voxelization, large tets (or the
// per-tet reference path).
tv_status run_single(const int4 *q4, int64_t nv, const int32_t *tets32, int64_t nt, tv_dims dims,
                     uint32_t *grid, const tv::TilePlan &p, const tv::WorkspaceLayout &L,
                     uint8_t *ws, hipStream_t s, uint32_t flags) {
    const tv::GridGeom g = make_geom(dims);
    const tv::BinBuffers b = tv::bin_buffers(ws, L);
    const int4 *tets = reinterpret_cast<const int4 *>(tets32);
    const bool strict = (flags & TV_TIE_STRICT) != 0;
    if (flags & TV_PATH_PER_TET) {
        tv::StageScope sc(tv::kStageVoxelize, s);
        tv::launch_clear(grid, (int64_t)tv_grid_words(dims), s);
        tv::launch_voxelize_per_tet(q4, nv, tets, nt, g, grid, b.status, strict, s);
        return check_hip("per-tet voxelize launch");
    }
    {
        tv::StageScope sc(tv::kStageBin, s);
        tv::launch_bin_count(q4, nv, tets, nt, g, p, b, s);
        tv::launch_scan_tiles(p, b, s);
        tv::launch_bin_scatter(q4, nv, tets, nt, g, p, b, s);
        tv::launch_zero_shared_tiles(g, p, b, grid, s);
    }
    tv_status st = check_hip("binning launch");
    if (st) return st;
    const int cus = device_cus();
    {
        tv::StageScope sc(tv::kStageVoxelize, s);
        int64_t wgs = 2 * (int64_t)cus;
        tv::launch_tile_voxelize(q4, tets, g, p, b, grid, strict, (int)wgs, s);
    }
    {
        tv::StageScope sc(tv::kStageLarge, s);
        tv::launch_large_tets(q4, tets, g, b, grid, strict, cus, s);
    }
    return check_hip("voxelize launch");
}

tv_status voxelize_common(const void *verts, bool fp32, const tv::BoxD *box, int64_t nv,
                          const int32_t *tets, int64_t nt, tv_dims dims, uint32_t *grid, void *ws,
                          hipStream_t s, uint32_t flags) {
    const tv::TilePlan p = tv::plan_tiles(dims, kMinTiles);
    const tv::WorkspaceLayout L = tv::single_layout(nv, nt, p);
    uint8_t *w = static_cast<uint8_t *>(ws);
    uint32_t *status = reinterpret_cast<uint32_t *>(w + L.status);
    int4 *q4 = reinterpret_cast<int4 *>(w + L.q4);
    tv::profile_count_call();
    {
        tv::StageScope sc(tv::kStageClear, s);
        tv::launch_clear(status, (int64_t)(L.clear_end - L.status) / 4, s);
    }
    {
        tv::StageScope sc(tv::kStageIngest, s);
        if (fp32)
            tv::launch_ingest_f32(static_cast<const float *>(verts), nv, *box, q4, status, s);
        else
            tv::launch_ingest_q32(static_cast<const int32_t *>(verts), nv, q4, status, s);
    }
    tv_status st = check_hip("ingest launch");
    if (st) return st;
    return run_single(q4, nv, tets, nt, dims, grid, p, L, w, s, flags);
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
    return tv::single_layout(nv, nt, tv::plan_tiles(dims, kMinTiles)).total;
}

tv_status tv_voxelize(const float *verts, int64_t nv, const int32_t *tets, int64_t nt,
                      tv_dims dims, tv_bbox bbox, uint32_t *grid, void *ws, size_t ws_bytes,
                      void *stream, uint32_t flags) {
    tv_status st = check_common(nv, tets, nt, dims, grid, ws, ws_bytes, flags, verts);
    if (st) return st;
    tv::BoxD box;
    if ((st = check_bbox(bbox, box))) return st;
    return voxelize_common(verts, true, &box, nv, tets, nt, dims, grid, ws,
                           reinterpret_cast<hipStream_t>(stream), flags);
}

tv_status tv_voxelize_q(const int32_t *qverts, int64_t nv, const int32_t *tets, int64_t nt,
                        tv_dims dims, uint32_t *grid, void *ws, size_t ws_bytes, void *stream,
                        uint32_t flags) {
    tv_status st = check_common(nv, tets, nt, dims, grid, ws, ws_bytes, flags, qverts);
    if (st) return st;
    return voxelize_common(qverts, false, nullptr, nv, tets, nt, dims, grid, ws,
                           reinterpret_cast<hipStream_t>(stream), flags);
}

tv_status tv_snap(const float *verts, int64_t nv, tv_bbox bbox, int32_t *q_out, void *stream) {
    if (nv < 0 || nv > INT32_MAX || (nv > 0 && (!verts || !q_out)))
        return fail(TV_ERR_INVALID_ARG, "bad snap arguments");
    tv::BoxD box;
    tv_status st = check_bbox(bbox, box);
    if (st) return st;
    tv::launch_snap_only(verts, nv, box, q_out, reinterpret_cast<hipStream_t>(stream));
    return check_hip("snap launch");
}

tv_status tv_fetch_status(const void *ws, int32_t mesh_index, void *stream) {
    if (!ws || mesh_index < 0 || mesh_index >= tv::kStatusWords)
        return fail(TV_ERR_INVALID_ARG, "bad workspace or mesh index %d", mesh_index);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    uint32_t word = 0;
    const uint8_t *w = static_cast<const uint8_t *>(ws);
    if (hipMemcpyAsync(&word, w + tv::kStatusOffset + 4 * (size_t)mesh_index, 4,
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(TV_ERR_HIP, "reading the status word failed");
    if (word & tv::kStatusIndex) return TV_ERR_INDEX;
    if (word & tv::kStatusRange) return TV_ERR_RANGE;
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
    default: return "TV_ERR_UNKNOWN";
    }
}

const char *tv_last_error(void) { return g_last_error; }

}  // extern "C"
