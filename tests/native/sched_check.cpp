// CPU-only checks of the serving loop's scheduling pieces (tv_sched.h):
// arena allocation, coalescing, exhaustion and FIFO admission limits.
// Built with g++ (host only) by tests/test_sched_native.py; prints one line
// per check and exits non-zero on the first failure.
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "tv_sched.h"

using tv::sched::Arena;

#define CHECK(cond)                                                    \
    do {                                                               \
        if (!(cond)) {                                                 \
            fprintf(stderr, "FAILED %s:%d %s\n", __FILE__, __LINE__, #cond); \
            return 1;                                                  \
        }                                                              \
    } while (0)

static int arena_basics() {
    Arena a(4096);
    size_t o1, o2, o3, o4;
    CHECK(a.alloc(100, &o1) && o1 == 0);
    CHECK(a.alloc(256, &o2) && o2 == 256);
    CHECK(a.alloc(1024, &o3) && o3 == 512);
    CHECK(a.in_use() == 256 + 256 + 1024);
    CHECK(!a.alloc(4096, &o4));           // does not fit
    CHECK(a.release(o2));
    CHECK(!a.release(o2));                // double free refused
    CHECK(!a.release(12345));             // unknown offset refused
    CHECK(a.alloc(200, &o4) && o4 == 256); // first fit reuses the hole
    CHECK(a.release(o1) && a.release(o3) && a.release(o4));
    CHECK(a.in_use() == 0 && a.free_blocks() == 1 && a.largest_free() == 4096);
    printf("ok arena_basics\n");
    return 0;
}

static int arena_random_stress() {
    // random alloc/free; invariants: no overlap, in_use bookkeeping, full
    // coalescing once everything is freed
    Arena a(1 << 20);
    std::mt19937 rng(7);
    std::vector<std::pair<size_t, size_t>> live;  // offset, bytes
    for (int step = 0; step < 20000; ++step) {
        if (!live.empty() && (rng() % 3 == 0 || a.largest_free() < 8192)) {
            const size_t k = rng() % live.size();
            CHECK(a.release(live[k].first));
            live.erase(live.begin() + (long)k);
        } else {
            const size_t bytes = 1 + rng() % 8192;
            size_t off;
            if (a.alloc(bytes, &off)) {
                for (auto &l : live)
                    CHECK(off + tv::sched::round_up(bytes) <= l.first ||
                          l.first + tv::sched::round_up(l.second) <= off);
                live.push_back({off, bytes});
            }
        }
        size_t sum = 0;
        for (auto &l : live) sum += tv::sched::round_up(l.second);
        CHECK(sum == a.in_use());
    }
    for (auto &l : live) CHECK(a.release(l.first));
    CHECK(a.in_use() == 0 && a.free_blocks() == 1 && a.largest_free() == (1u << 20));
    printf("ok arena_random_stress\n");
    return 0;
}

static int admission() {
    tv::sched::WaveLimits lim;
    lim.max_meshes = 3;
    lim.max_inflight = 2;
    // FIFO: stops at the first request that does not fit (no overtaking)
    std::vector<bool> fits = {true, true, false, true, true};
    std::vector<size_t> tried;
    int32_t n = tv::sched::admit_wave(fits.size(), lim, 0, [&](size_t i) {
        tried.push_back(i);
        return (bool)fits[i];
    });
    CHECK(n == 2 && tried.size() == 3);
    // mesh limit
    n = tv::sched::admit_wave(10, lim, 1, [&](size_t) { return true; });
    CHECK(n == 3);
    // in-flight limit
    n = tv::sched::admit_wave(10, lim, 2, [&](size_t) { return true; });
    CHECK(n == 0);
    // empty queue
    n = tv::sched::admit_wave(0, lim, 0, [&](size_t) { return true; });
    CHECK(n == 0);
    printf("ok admission\n");
    return 0;
}

static int pressure_simulation() {
    // A simulated server loop: requests of random footprints arrive; each
    // tick admits a FIFO wave into free memory, waves finish after a fixed
    // number of ticks and release inputs (grids are released one tick
    // later).  Every request completes, memory never over-commits, and a
    // request larger than the arena is refused at submission.
    const size_t cap = 64 * 1024;
    Arena a(cap);
    std::mt19937 rng(11);
    struct R { size_t bytes, off; bool in; };
    std::vector<R> reqs;
    for (int i = 0; i < 500; ++i) reqs.push_back({(size_t)(1 + rng() % 20000), 0, false});
    size_t too_big = cap + 1;
    CHECK(tv::sched::round_up(too_big) > a.size());  // refused up front
    std::vector<size_t> queue;
    for (size_t i = 0; i < reqs.size(); ++i) queue.push_back(i);
    std::vector<std::pair<int, std::vector<size_t>>> waves;  // finish tick, members
    tv::sched::WaveLimits lim;
    lim.max_meshes = 16;
    lim.max_inflight = 2;
    size_t done = 0;
    for (int tick = 0; tick < 100000 && done < reqs.size(); ++tick) {
        for (size_t w = 0; w < waves.size();) {
            if (waves[w].first <= tick) {
                for (size_t r : waves[w].second) {
                    CHECK(a.release(reqs[r].off));
                    ++done;
                }
                waves.erase(waves.begin() + (long)w);
            } else {
                ++w;
            }
        }
        std::vector<size_t> taken;
        int32_t n = tv::sched::admit_wave(queue.size(), lim, (int32_t)waves.size(), [&](size_t i) {
            R &r = reqs[queue[i]];
            if (!a.alloc(r.bytes, &r.off)) return false;
            taken.push_back(queue[i]);
            return true;
        });
        CHECK((size_t)n == taken.size());
        CHECK(a.in_use() <= cap);
        queue.erase(queue.begin(), queue.begin() + n);
        if (n) waves.push_back({tick + 3, taken});
    }
    CHECK(done == reqs.size() && a.in_use() == 0);
    printf("ok pressure_simulation\n");
    return 0;
}

int main() {
    if (arena_basics() || arena_random_stress() || admission() || pressure_simulation()) return 1;
    printf("all ok\n");
    return 0;
}
