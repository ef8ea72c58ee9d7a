// Host-side launch wrappers and shared host/device structs of the kernels
// (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tv_common.h"

namespace tv {

// World bbox in double: lo and extent (hi - lo) per axis.
struct BoxD {
    double lo[3];
    double ext[3];
};

// Tiling of one grid: tiles of 2^lx x 2^ly columns and 2^lw words per column.
struct TilePlan {
    int32_t lx, ly, lw;
    int32_t ntx, nty, ntz;  // tiles per axis
    int64_t ntiles;
    int32_t chunk;      // pieces per chunk (one workgroup task)
    int32_t strip;      // columns per lane task
    int32_t piece_cap;  // tets meeting more tiles than this go to the large-tet kernel
};

// meta[] slots
constexpr int kMetaQueue = 0;   // next chunk to hand out
constexpr int kMetaBig = 1;     // number of large tets
constexpr int kMetaChunks = 2;  // total chunks

// Device buffers of the binned pipeline (all inside the caller's workspace).
struct BinBuffers {
    uint32_t *status;       // per-mesh status word
    uint32_t *meta;         // counters (kMeta*)
    uint32_t *tile_count;   // [ntiles] pieces per tile
    uint32_t *tile_cursor;  // [ntiles] fill cursor of the scatter pass
    uint32_t *tile_off;     // [ntiles + 1] first piece slot per tile
    uint32_t *chunk_off;    // [ntiles + 1] first chunk per tile
    uint32_t *pieces;       // [nt * piece_cap] tet ids sorted by tile
    uint32_t *big;          // [nt] large tets
};

void launch_ingest_f32(const float *v, int64_t nv, const BoxD &box, int4 *q4, uint32_t *status,
                       hipStream_t s);
void launch_ingest_q32(const int32_t *q, int64_t nv, int4 *q4, uint32_t *status, hipStream_t s);
void launch_snap_only(const float *v, int64_t nv, const BoxD &box, int32_t *q, hipStream_t s);
void launch_clear(uint32_t *p, int64_t nwords, hipStream_t s);
void launch_bin_count(const int4 *q4, int64_t nv, const int4 *tets, int64_t nt, const GridGeom &g,
                      const TilePlan &p, const BinBuffers &b, hipStream_t s);
void launch_scan_tiles(const TilePlan &p, const BinBuffers &b, hipStream_t s);
void launch_bin_scatter(const int4 *q4, int64_t nv, const int4 *tets, int64_t nt,
                        const GridGeom &g, const TilePlan &p, const BinBuffers &b, hipStream_t s);
void launch_zero_shared_tiles(const GridGeom &g, const TilePlan &p, const BinBuffers &b,
                              uint32_t *grid, hipStream_t s);
void launch_tile_voxelize(const int4 *q4, const int4 *tets, const GridGeom &g, const TilePlan &p,
                          const BinBuffers &b, uint32_t *grid, bool strict, int workgroups,
                          hipStream_t s);
void launch_large_tets(const int4 *q4, const int4 *tets, const GridGeom &g, const BinBuffers &b,
                       uint32_t *grid, bool strict, int workgroups, hipStream_t s);
void launch_voxelize_per_tet(const int4 *q4, int64_t nv, const int4 *tets, int64_t nt,
                             const GridGeom &g, uint32_t *grid, uint32_t *status, bool strict,
                             hipStream_t s);
int tile_max_words();

}  // namespace tv
