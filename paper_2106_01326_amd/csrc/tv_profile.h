// Per-stage HIP-event timing (diagnostics; see tv_profile_* in tv.h).
#pragma once

#include <hip/hip_runtime.h>

namespace tv {

enum Stage : int {
    kStageClear = 0,   // workspace counters (and, on the reference path, the grid)
    kStageIngest,      // snap / range check of the vertices
    kStageBin,         // tile binning: count, scan, scatter, shared-tile zeroing
    kStageVoxelize,    // column-span voxelization into tiles (or per tet)
    kStageLarge,       // tets meeting more tiles than the cap
    kStageCount
};

bool profile_on();
void profile_count_call();

// Records a start event on construction and an end event on destruction
// when profiling is enabled; no-op otherwise.
class StageScope {
  public:
    StageScope(int stage, hipStream_t s);
    ~StageScope();
    StageScope(const StageScope &) = delete;
    StageScope &operator=(const StageScope &) = delete;

  private:
    int stage_;
    hipStream_t s_;
    hipEvent_t start_ = nullptr;
};

}  // namespace tv
