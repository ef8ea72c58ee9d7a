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
};

constexpr int32_t kFmtF32 = 0;
constexpr int32_t kFmtQ32 = 1;

// Everything the kernels need to know about one mesh of a call.
struct MeshDesc {
    const void *verts;   // fp32 or int32 [nv][3]
    const int4 *tets;    // [nt]
    uint32_t *grid;      // output words
    int64_t nv, nt;
    int64_t vert_base;   // first lattice record of the mesh in the call's q4 array
    int64_t tet_base;    // global index of tets[0] among the call's tets
    int64_t tile_base;   // global index of the mesh's first tile
    BoxD box;
    GridGeom g;
    TilePlan p;
    int32_t fmt;         // kFmtF32 / kFmtQ32
    int32_t mesh;        // index (status word)
    int32_t direct;      // the grid is a single tile: its pieces are the mesh's tets in
                         // order, never binned (the tile kernel checks their indices)
};

// Sparse output of a single-mesh call: bricks of 8 x 8 columns x 32 z
// voxels (one grid word per column).  index[brick id]: 0 empty, kBrickFull
// every voxel set, else 1 + the brick's slot; pool[slot][64] the brick's
// words (column (8bx+u, 8by+v) at word u*8 + v); ids[slot] the brick of a
// slot (kBrickUnused for a slot given up in a race); *count the slots taken.
constexpr uint32_t kBrickFull = 0xffffffffu;
constexpr uint32_t kBrickUnused = 0xffffffffu;
struct BrickOut {
    uint32_t *index;
    uint32_t *pool;
    uint32_t *ids;
    uint32_t *count;
    int64_t capacity;
    int32_t nby, nbz;  // bricks per y row (ny / 8) and per column (nz / 32)
};

// The meshes of one call.  A single mesh travels by value in `one`; a batch
// lives in device memory with prefix sums over vertices, tets and tiles
// (each [n + 1]) that map a global index to its mesh.
struct MeshTable {
    const MeshDesc *descs;
    const int64_t *vert_pre;
    const int64_t *tet_pre;
    const int64_t *tile_pre;
    int32_t n;
    int32_t chunk;      // pieces per chunk (one workgroup task)
    int32_t strip;      // kept columns per lane task
    int32_t piece_cap;  // tets meeting more tiles than this go to the large-tet kernel
    int32_t accumulate; // OR into the grids instead of overwriting them
    int32_t nocull;     // boxes of at most this many columns skip row culling
    int64_t nv_total, nt_total, ntiles_total;
    MeshDesc one;
    BrickOut bricks;    // sparse output (single-mesh calls), used when bricks.index != nullptr
};

// meta[] slots
constexpr int kMetaQueue = 0;   // next chunk to hand out
constexpr int kMetaBig = 1;     // number of large tets
constexpr int kMetaChunks = 2;  // total chunks
constexpr int kMetaMeshes = 3;  // meshes of the last call (status words in use)

// Device buffers of the binned pipeline (all inside the caller's workspace).
struct BinBuffers {
    uint32_t *meta;         // counters (kMeta*)
    uint32_t *status;       // one status word per mesh
    uint32_t *tile_count;   // [ntiles] pieces per tile
    uint32_t *tile_cursor;  // [ntiles] fill cursor of the scatter pass
    uint32_t *tile_off;     // [ntiles + 1] first piece slot per tile
    uint32_t *chunk_off;    // [ntiles + 1] first chunk of the tile of each rank
    uint32_t *tile_order;   // [ntiles] tile of each rank (largest tiles first)
    uint32_t *rank_mesh;    // [ntiles] mesh of the tile of each rank
    uint32_t *task_rank;    // [tasks] rank of the tile of each queue task
    uint32_t *pieces;       // [nt * piece_cap] global tet ids sorted by tile
    uint32_t *big;          // [nt] large tets (global ids)
    uint2 *trec;            // [nt] tile summary: (first tile key, shape code; 0 = no pieces)
    int4 *q4;               // [nv] lattice vertices (.w = invalid flag)
};

void launch_ingest(const MeshTable &T, const BinBuffers &b, hipStream_t s);
void launch_snap_only(const float *v, int64_t nv, const BoxD &box, int32_t *q, hipStream_t s);
void launch_clear(uint32_t *p, int64_t nwords, hipStream_t s);
void launch_set_word(uint32_t *p, uint32_t value, hipStream_t s);
void launch_bin_count(const MeshTable &T, const BinBuffers &b, hipStream_t s);
void launch_scan_tiles(const MeshTable &T, const BinBuffers &b, hipStream_t s);
void launch_bin_scatter(const MeshTable &T, const BinBuffers &b, hipStream_t s);
void launch_zero_shared_tiles(const MeshTable &T, const BinBuffers &b, hipStream_t s);
void launch_tile_voxelize(const MeshTable &T, const BinBuffers &b, bool strict, int workgroups,
                          hipStream_t s);
void launch_large_tets(const MeshTable &T, const BinBuffers &b, bool strict, int workgroups,
                       hipStream_t s);
void launch_voxelize_per_tet(const MeshDesc &d, const BinBuffers &b, bool strict, hipStream_t s);
void launch_bricks_canonical(const MeshTable &T, const BinBuffers &b, int workgroups, hipStream_t s);
int tile_max_words();

}  // namespace tv
