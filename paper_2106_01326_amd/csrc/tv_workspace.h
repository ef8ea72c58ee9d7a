// Tile planning and workspace layout (byte offsets into the caller's
// 256-byte aligned workspace), shared by the single-mesh and batch calls.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "tv.h"
#include "tv_kernels.h"

namespace tv {

constexpr int32_t kMetaWords = 64;
constexpr int32_t kMinStatusWords = 64;
constexpr int32_t kPieceCap = 8;  // piece slots reserved per tet (the largest piece_cap)
constexpr int32_t kPieceCapSparse = 27;  // the same for sparse-output calls

// Launch parameters of the tile pipeline (tv_params in the C ABI).
struct Params {
    int32_t tile_cols_log2;  // largest tile edge in columns, log2 (3..5)
    int32_t min_tiles;       // tiles are made smaller while a grid has fewer
    int32_t chunk;           // pieces per work-queue task
    int32_t strip;           // kept columns per lane task
    int32_t piece_cap;       // tets meeting more tiles go to the large-tet kernel
    int32_t wgs_per_cu;      // persistent tile workgroups per compute unit
    int32_t cull;            // boxes of at most this many columns skip row culling
};
// A lone grid wants >= 512 tiles to spread over the chip; batch meshes keep
// the largest tiles (their parallelism comes from the mesh count).  chunk 0
// sizes the queue tasks from the tet count (auto_chunk).  Values from the
// autotuner's searches on the large, medium and batch workloads.
constexpr Params kDefaultSingle = {5, 512, 0, 6, 8, 2, 3};
constexpr Params kDefaultBatch = {5, 1, 0, 6, 8, 2, 6};

// Pieces per work-queue task when Params::chunk is 0.  A single mesh: about
// 4096 tasks in all (pieces, about 2 per tet, / 4096 = nt / 2048), a power
// of two in [256, 16384]; a call that already has 4096 tiles or more keeps
// at least 4096 pieces per task: more tasks would only split its tiles into
// shares that are flushed with atomics.  A batch of meshes: about 1024 tasks
// (nt / 1024, a power of two in [256, 65536]): its many small tiles then
// mostly take one task each, written with plain stores, while a small batch
// (a serving wave of a few meshes) still spreads over the chip.
inline int32_t auto_chunk(int64_t nt, int64_t ntiles, bool batch) {
    int32_t c = 256;
    if (batch) {
        while (c < 65536 && (int64_t)c * 2 * 1024 <= nt) c *= 2;
        return c;
    }
    while (c < 16384 && (int64_t)c * 2 * 2048 <= nt) c *= 2;
    if (ntiles >= 4096 && c < 4096) c = 4096;
    return c;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

inline int ilog2(int64_t n) {
    int s = 0;
    while ((int64_t(1) << s) < n) ++s;
    return s;
}

// Tiles of at most 2^max_log2 x 2^max_log2 columns (max_log2 <= 5) x 4
// words (at most 16 KiB of LDS bitmap), made smaller (down to 8 x 8
// columns) while the grid has fewer than `min_tiles` of them, so that a lone
// small grid still spreads over the chip.
inline TilePlan plan_tiles(tv_dims d, int64_t min_tiles, int max_log2) {
    TilePlan p;
    const int W = (d.nz + 31) / 32;
    p.lw = ilog2(W) < 2 ? ilog2(W) : 2;
    p.lx = ilog2(d.nx) < max_log2 ? ilog2(d.nx) : max_log2;
    p.ly = ilog2(d.ny) < max_log2 ? ilog2(d.ny) : max_log2;
    auto count = [&]() {
        return (int64_t)(d.nx >> p.lx) * (int64_t)(d.ny >> p.ly) * (int64_t)(W >> p.lw);
    };
    while (count() < min_tiles && (p.lx > 3 || p.ly > 3)) {
        if (p.lx >= p.ly) --p.lx;
        else --p.ly;
    }
    p.ntx = d.nx >> p.lx;
    p.nty = d.ny >> p.ly;
    p.ntz = W >> p.lw;
    p.ntiles = count();
    return p;
}

// Sizes of one call (a single mesh or a batch).
struct CallSizes {
    int64_t meshes;
    int64_t nv, nt, ntiles;  // totals over the meshes
    // the descriptors live in a device table inside the workspace (batch
    // calls); otherwise a single mesh's descriptor is a kernel argument
    bool table = false;
    int32_t piece_slots = kPieceCap;  // piece slots per tet
};

struct WorkspaceLayout {
    size_t meta;         // kMetaWords uint32 (fixed at offset 0)
    size_t status;       // max(kMinStatusWords, meshes) uint32
    size_t tile_count;   // ntiles uint32
    size_t tile_cursor;  // ntiles uint32
    size_t clear_end;    // [0, clear_end) is zeroed at the start of a call
    size_t tile_off;     // ntiles + 1
    size_t chunk_off;    // ntiles + 1
    size_t tile_order;   // ntiles
    size_t rank_mesh;    // ntiles
    size_t task_rank;    // max_tasks(c)
    size_t descs;        // meshes MeshDesc, then 3 x (meshes + 1) int64 prefix sums
    size_t descs_bytes;
    size_t q4;           // nv int4 lattice vertices (.w = invalid flag)
    size_t pieces;       // nt * piece_slots uint32
    size_t big;          // nt uint32
    size_t trec;         // nt uint2: per-tet tile summary from the counting pass
    size_t total;
};

// Queue tasks of a call, at most: a tile has max(1, ceil(pieces / chunk))
// of them, pieces are at most piece_slots per tet and a task holds at least
// 64 pieces (the smallest chunk_pieces).
inline int64_t max_tasks(const CallSizes &c) {
    return c.ntiles + (c.nt * (int64_t)c.piece_slots + 63) / 64 + 1;
}

inline int64_t status_words(int64_t meshes) {
    return meshes > kMinStatusWords ? meshes : kMinStatusWords;
}

inline WorkspaceLayout layout(const CallSizes &c) {
    WorkspaceLayout L;
    size_t off = 0;
    L.meta = off;
    off += sizeof(uint32_t) * kMetaWords;
    L.status = off;
    off += sizeof(uint32_t) * (size_t)status_words(c.meshes);
    L.tile_count = off;
    off += 4 * (size_t)c.ntiles;
    L.tile_cursor = off;
    off += 4 * (size_t)c.ntiles;
    L.clear_end = off;
    off = align256(off);
    L.tile_off = off;
    off = align256(off + 4 * ((size_t)c.ntiles + 1));
    L.chunk_off = off;
    off = align256(off + 4 * ((size_t)c.ntiles + 1));
    L.tile_order = off;
    off = align256(off + 4 * (size_t)c.ntiles);
    L.rank_mesh = off;
    off = align256(off + 4 * (size_t)c.ntiles);
    L.task_rank = off;
    off = align256(off + 4 * (size_t)max_tasks(c));
    L.descs = off;
    L.descs_bytes = c.table ? sizeof(MeshDesc) * (size_t)c.meshes +
                                  3 * sizeof(int64_t) * ((size_t)c.meshes + 1)
                            : 0;
    off = align256(off + L.descs_bytes);
    L.q4 = off;
    off = align256(off + 16 * (size_t)c.nv);
    L.pieces = off;
    off = align256(off + 4 * (size_t)c.nt * (size_t)c.piece_slots);
    L.big = off;
    off = align256(off + 4 * (size_t)c.nt);
    L.trec = off;
    off = align256(off + 8 * (size_t)c.nt);
    L.total = off;
    return L;
}

inline BinBuffers bin_buffers(uint8_t *ws, const WorkspaceLayout &L) {
    BinBuffers b;
    b.meta = reinterpret_cast<uint32_t *>(ws + L.meta);
    b.status = reinterpret_cast<uint32_t *>(ws + L.status);
    b.tile_count = reinterpret_cast<uint32_t *>(ws + L.tile_count);
    b.tile_cursor = reinterpret_cast<uint32_t *>(ws + L.tile_cursor);
    b.tile_off = reinterpret_cast<uint32_t *>(ws + L.tile_off);
    b.chunk_off = reinterpret_cast<uint32_t *>(ws + L.chunk_off);
    b.tile_order = reinterpret_cast<uint32_t *>(ws + L.tile_order);
    b.rank_mesh = reinterpret_cast<uint32_t *>(ws + L.rank_mesh);
    b.task_rank = reinterpret_cast<uint32_t *>(ws + L.task_rank);
    b.pieces = reinterpret_cast<uint32_t *>(ws + L.pieces);
    b.big = reinterpret_cast<uint32_t *>(ws + L.big);
    b.trec = reinterpret_cast<uint2 *>(ws + L.trec);
    b.q4 = reinterpret_cast<int4 *>(ws + L.q4);
    return b;
}

}  // namespace tv
