// Library-internal entry points shared by the C-ABI front end and the
// serving loop.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "tv.h"
#include "tv_kernels.h"
#include "tv_workspace.h"

namespace tv {

// Host-visible checks of one mesh; `which` prefixes error messages.
tv_status check_mesh(const void *verts, uint32_t fmt, int64_t nv, const int32_t *tets, int64_t nt,
                     tv_dims dims, const tv_bbox *bbox, const uint32_t *grid, const char *which);

// Descriptor of one mesh of a batch (device pointers; bases filled later).
MeshDesc make_batch_desc(const void *verts, uint32_t fmt, int64_t nv, const int32_t *tets,
                         int64_t nt, tv_dims dims, const tv_bbox *bbox, uint32_t *grid);

// Assigns vertex/tet/tile bases and returns the call totals.
CallSizes assign_bases(std::vector<MeshDesc> &descs);

// Enqueues the whole pipeline for final descriptors on `s`.
tv_status run_meshes(std::vector<MeshDesc> &descs, const CallSizes &c, uint8_t *ws, hipStream_t s,
                     uint32_t flags);

// Records an error message for tv_last_error() and returns `code`.
tv_status set_error(tv_status code, const char *fmt, ...);

}  // namespace tv
