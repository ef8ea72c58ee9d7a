// Host-side scheduling pieces of the serving loop, free of any HIP call so
// that they build and run on a CPU alone:
//   - Arena: first-fit sub-allocator over one preallocated region (byte
//     offsets, 256-byte granules, neighbouring free blocks coalesce);
//   - Admission: FIFO admission of requests into waves by memory footprint
//     and wave limits.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <deque>
#include <map>
#include <unordered_map>
#include <vector>

namespace tv {
namespace sched {

constexpr size_t kGranule = 256;

inline size_t round_up(size_t x) { return (x + kGranule - 1) & ~(kGranule - 1); }

class Arena {
  public:
    explicit Arena(size_t size = 0) { reset(size); }

    void reset(size_t size) {
        size_ = size & ~(kGranule - 1);
        free_.clear();
        used_.clear();
        in_use_ = 0;
        if (size_) free_[0] = size_;
    }

    // First fit; returns false (and leaves `off` alone) when no free block
    // is large enough.  Zero-byte requests take one granule.
    bool alloc(size_t bytes, size_t *off) {
        const size_t need = round_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            const size_t at = it->first, len = it->second;
            free_.erase(it);
            if (len > need) free_[at + need] = len - need;
            used_[at] = need;
            in_use_ += need;
            *off = at;
            return true;
        }
        return false;
    }

    // Returns false for an offset that is not an allocated block.
    bool release(size_t off) {
        auto u = used_.find(off);
        if (u == used_.end()) return false;
        size_t at = off, len = u->second;
        used_.erase(u);
        in_use_ -= len;
        auto next = free_.lower_bound(at);
        if (next != free_.end() && next->first == at + len) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == at) {
                at = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[at] = len;
        return true;
    }

    size_t size() const { return size_; }
    size_t in_use() const { return in_use_; }
    size_t largest_free() const {
        size_t m = 0;
        for (const auto &kv : free_) m = kv.second > m ? kv.second : m;
        return m;
    }
    size_t free_blocks() const { return free_.size(); }
    size_t used_blocks() const { return used_.size(); }

  private:
    size_t size_ = 0;
    size_t in_use_ = 0;
    std::map<size_t, size_t> free_;             // offset -> length
    std::unordered_map<size_t, size_t> used_;   // offset -> length
};

// Memory a request needs while it runs: device bytes for its inputs and its
// grid (the grid stays until the client releases it), pinned staging bytes
// for its host inputs, and its share of the wave's workspace.
struct Footprint {
    size_t inputs = 0, grid = 0, staging = 0, workspace = 0;
};

struct WaveLimits {
    int32_t max_meshes = 1024;   // meshes per wave
    int32_t max_inflight = 2;    // waves on the device at once
};

// FIFO admission of queued requests into one wave.  `try_take(i)` reserves
// request i's memory and returns false when it does not fit; the wave stops
// at the first request that does not fit (no overtaking, so a large request
// cannot starve) or at the mesh limit.  Returns the number taken from the
// front of the queue.
template <class TryTake>
int32_t admit_wave(size_t queued, const WaveLimits &lim, int32_t inflight, TryTake try_take) {
    if (inflight >= lim.max_inflight) return 0;
    int32_t taken = 0;
    while ((size_t)taken < queued && taken < lim.max_meshes) {
        if (!try_take((size_t)taken)) break;
        ++taken;
    }
    return taken;
}

}  // namespace sched
}  // namespace tv
