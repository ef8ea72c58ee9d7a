// Tile planning and workspace layout of the single-mesh path (byte offsets
// into the caller's 256-byte aligned workspace).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "tv.h"
#include "tv_kernels.h"

namespace tv {

constexpr int32_t kStatusWords = 64;  // per-mesh device status words
constexpr size_t kStatusOffset = 0;
constexpr int32_t kMetaWords = 64;
constexpr int32_t kPieceCap = 8;
constexpr int32_t kChunkPieces = 4096;
constexpr int32_t kStripColumns = 8;

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

inline int ilog2(int64_t n) {
    int s = 0;
    while ((int64_t(1) << s) < n) ++s;
    return s;
}

// Tiles of at most 32 x 32 columns x 4 words (16 KiB of LDS bitmap), made
// smaller (down to 8 x 8 columns) while the grid has fewer than
// `min_tiles` of them, so that small grids still spread over the chip.
inline TilePlan plan_tiles(tv_dims d, int64_t min_tiles) {
    TilePlan p;
    const int W = (d.nz + 31) / 32;
    p.lw = ilog2(W) < 2 ? ilog2(W) : 2;
    p.lx = ilog2(d.nx) < 5 ? ilog2(d.nx) : 5;
    p.ly = ilog2(d.ny) < 5 ? ilog2(d.ny) : 5;
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
    p.chunk = kChunkPieces;
    p.strip = kStripColumns;
    p.piece_cap = kPieceCap;
    return p;
}

struct WorkspaceLayout {
    size_t status;       // kStatusWords uint32
    size_t meta;         // kMetaWords uint32
    size_t tile_count;   // ntiles uint32
    size_t tile_cursor;  // ntiles uint32
    size_t clear_end;    // [status, clear_end) is zeroed at the start of a call
    size_t tile_off;     // ntiles + 1
    size_t chunk_off;    // ntiles + 1
    size_t q4;           // nv int4 lattice vertices (.w = invalid flag)
    size_t pieces;       // nt * piece_cap uint32
    size_t big;          // nt uint32
    size_t total;
};

inline WorkspaceLayout single_layout(int64_t nv, int64_t nt, const TilePlan &p) {
    WorkspaceLayout L;
    size_t off = 0;
    L.status = off;
    off += sizeof(uint32_t) * kStatusWords;
    L.meta = off;
    off += sizeof(uint32_t) * kMetaWords;
    L.tile_count = off;
    off += 4 * (size_t)p.ntiles;
    L.tile_cursor = off;
    off += 4 * (size_t)p.ntiles;
    L.clear_end = off;
    off = align256(off);
    L.tile_off = off;
    off = align256(off + 4 * ((size_t)p.ntiles + 1));
    L.chunk_off = off;
    off = align256(off + 4 * ((size_t)p.ntiles + 1));
    L.q4 = off;
    off = align256(off + 16 * (size_t)nv);
    L.pieces = off;
    off = align256(off + 4 * (size_t)nt * (size_t)p.piece_cap);
    L.big = off;
    off = align256(off + 4 * (size_t)nt);
    L.total = off;
    return L;
}

inline BinBuffers bin_buffers(uint8_t *ws, const WorkspaceLayout &L) {
    BinBuffers b;
    b.status = reinterpret_cast<uint32_t *>(ws + L.status);
    b.meta = reinterpret_cast<uint32_t *>(ws + L.meta);
    b.tile_count = reinterpret_cast<uint32_t *>(ws + L.tile_count);
    b.tile_cursor = reinterpret_cast<uint32_t *>(ws + L.tile_cursor);
    b.tile_off = reinterpret_cast<uint32_t *>(ws + L.tile_off);
    b.chunk_off = reinterpret_cast<uint32_t *>(ws + L.chunk_off);
    b.pieces = reinterpret_cast<uint32_t *>(ws + L.pieces);
    b.big = reinterpret_cast<uint32_t *>(ws + L.big);
    return b;
}

}  // namespace tv
