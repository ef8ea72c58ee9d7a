// Host-side launch wrappers of the device kernels (internal to the library).
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

__device__ __forceinline__ bool index_ok(int32_t x, int64_t nv) { return x >= 0 && (int64_t)x < nv; }

void launch_ingest_f32(const float *v, int64_t nv, const BoxD &box, int4 *q4, uint32_t *status,
                       hipStream_t s);
void launch_ingest_q32(const int32_t *q, int64_t nv, int4 *q4, uint32_t *status, hipStream_t s);
void launch_clear(uint32_t *p, int64_t nwords, uint32_t *status, int32_t nstatus, hipStream_t s);
void launch_voxelize_per_tet(const int4 *q4, int64_t nv, const int4 *tets, int64_t nt,
                             const GridGeom &g, uint32_t *grid, uint32_t *status, bool strict,
                             hipStream_t s);

}  // namespace tv
