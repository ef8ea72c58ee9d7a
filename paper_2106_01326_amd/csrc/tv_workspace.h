// Workspace layout of the single-mesh path (byte offsets into the caller's
// 256-byte aligned workspace).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "tv.h"

namespace tv {

constexpr int32_t kStatusWords = 64;  // per-mesh device status words
constexpr size_t kStatusOffset = 0;

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct WorkspaceLayout {
    size_t status;  // kStatusWords uint32
    size_t q4;      // nv int4 lattice vertices (.w = invalid flag)
    size_t total;
};

inline WorkspaceLayout single_layout(int64_t nv, int64_t nt, tv_dims dims) {
    (void)nt;
    (void)dims;
    WorkspaceLayout L;
    size_t off = 0;
    L.status = off;
    off += align256(sizeof(uint32_t) * kStatusWords);
    L.q4 = off;
    off += align256(16 * (size_t)nv);
    L.total = off;
    return L;
}

}  // namespace tv
