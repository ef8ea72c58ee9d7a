// CPU-only checks of the serving loop's threads (tv_serve_core.h) behind a
// fake executor: admission by memory, overlap of waves on two streams,
// waiting without the lock when the front request only partly fits,
// staging on the launcher threads, launch failures, data statuses, client
// releases, shutdown with work queued, and a multi-client stress run.
// Built with g++ (host only) under ThreadSanitizer and under
// AddressSanitizer/UBSan by tests/test_sched_native.py; prints one line per
// check and exits non-zero on the first failure.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <atomic>
#include <future>
#include <mutex>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "tv_serve_core.h"

using tv::serve::Config;
using tv::serve::Core;
using tv::serve::Req;
using tv::serve::Wave;

#define CHECK(cond)                                                          \
    do {                                                                     \
        if (!(cond)) {                                                       \
            fprintf(stderr, "FAILED %s:%d %s\n", __FILE__, __LINE__, #cond); \
            fflush(stderr);                                                  \
            _exit(1);                                                        \
        }                                                                    \
    } while (0)

// Waves complete once their launch number is below `gate`; a request with
// nv == 13 fails to launch; one with nt == 7 reports an index error.  The
// workspace of a wave is 4096 bytes plus 4 per tet.
struct FakeExec final : tv::serve::Executor {
    std::atomic<uint64_t> gate{~0ull};
    std::atomic<int> launches{0};
    std::vector<uint8_t> pinned;
    std::mutex m;
    std::set<std::thread::id> launch_threads;
    std::atomic<int> staged_ok{0}, staged_bad{0};
    std::atomic<int> max_concurrent{0}, running{0};

    explicit FakeExec(size_t pinned_bytes) : pinned(pinned_bytes) {}

    size_t workspace_bytes(const std::vector<const Req *> &rs) override {
        size_t b = 4096;
        for (const Req *q : rs) b += 4 * (size_t)q->r.nt;
        return b;
    }
    tv_status launch(const Wave &, const std::vector<const Req *> &rs) override {
        {
            std::lock_guard<std::mutex> lk(m);
            launch_threads.insert(std::this_thread::get_id());
        }
        launches++;
        for (const Req *q : rs) {
            if (q->r.nv == 13) return TV_ERR_HIP;
            if (q->has_st) {
                // stage the vertices and check what arrived
                const size_t vb = 12 * (size_t)q->r.nv;
                memcpy(pinned.data() + q->st_off, q->r.verts, vb);
                if (memcmp(pinned.data() + q->st_off, q->r.verts, vb) == 0) staged_ok++;
                else staged_bad++;
            }
        }
        const int now = ++running;
        int prev = max_concurrent.load();
        while (now > prev && !max_concurrent.compare_exchange_weak(prev, now)) {
        }
        return TV_OK;
    }
    bool done(const Wave &w) override {
        const bool d = w.seq < gate.load();
        return d;
    }
    void finish(const Wave &w, std::vector<tv_status> &out) override {
        --running;
        out.assign(w.tickets.size(), TV_OK);
        (void)w;
    }
};

// Every arena region a wave's device work would touch (its workspace, its
// requests' input copies and grids) must be disjoint from the regions of
// every other wave in flight and from the grids that clients still hold.
// Regions are taken at launch and given back at finish (workspace, inputs)
// or by the client before it releases a request (grid).
struct RegionExec final : tv::serve::Executor {
    struct Region {
        size_t lo, hi;
        int64_t owner;  // wave sequence for workspace and inputs, -1 - ticket offset for grids
    };
    std::mutex m;
    std::vector<Region> live;
    std::atomic<int> overlaps{0}, launched{0};
    std::atomic<uint64_t> gate{~0ull};

    static size_t up(size_t b) { return tv::sched::round_up(b ? b : 1); }
    size_t workspace_bytes(const std::vector<const Req *> &rs) override {
        size_t b = 4096;
        for (const Req *q : rs) b += 8 * (size_t)q->r.nt;
        return b;
    }
    void take(size_t lo, size_t bytes, int64_t owner) {
        const size_t hi = lo + up(bytes);
        for (const Region &r : live)
            if (lo < r.hi && r.lo < hi) overlaps++;
        live.push_back({lo, hi, owner});
    }
    void drop_owner(int64_t owner) {
        std::vector<Region> keep;
        for (const Region &r : live)
            if (r.owner != owner) keep.push_back(r);
        live.swap(keep);
    }
    // the client gives a grid back before releasing its request
    void drop_grid(size_t off) {
        std::lock_guard<std::mutex> lk(m);
        std::vector<Region> keep;
        for (const Region &r : live)
            if (!(r.owner < 0 && r.lo == off)) keep.push_back(r);
        live.swap(keep);
    }
    tv_status launch(const Wave &w, const std::vector<const Req *> &rs) override {
        std::lock_guard<std::mutex> lk(m);
        take(w.ws_off, workspace_bytes(rs), (int64_t)w.seq);
        for (const Req *q : rs) {
            if (q->has_in) take(q->in_off, q->in_bytes, (int64_t)w.seq);
            take(q->grid_off, q->grid_words * 4, -1);
        }
        launched++;
        return TV_OK;
    }
    bool done(const Wave &w) override { return w.seq < gate.load(); }
    void finish(const Wave &w, std::vector<tv_status> &out) override {
        std::lock_guard<std::mutex> lk(m);
        drop_owner((int64_t)w.seq);
        out.assign(w.tickets.size(), TV_OK);
    }
};

// finish() above does not see the requests; the data status of nt == 7 is
// checked through this executor, which remembers each wave's tets.
struct StatusExec final : tv::serve::Executor {
    std::mutex m;
    std::vector<std::vector<int64_t>> nts;  // by wave sequence
    size_t workspace_bytes(const std::vector<const Req *> &rs) override { return 4096 + 64 * rs.size(); }
    tv_status launch(const Wave &w, const std::vector<const Req *> &rs) override {
        std::lock_guard<std::mutex> lk(m);
        if (nts.size() <= w.seq) nts.resize(w.seq + 1);
        for (const Req *q : rs) nts[w.seq].push_back(q->r.nt);
        return TV_OK;
    }
    bool done(const Wave &) override { return true; }
    void finish(const Wave &w, std::vector<tv_status> &out) override {
        std::lock_guard<std::mutex> lk(m);
        out.clear();
        for (int64_t nt : nts[w.seq]) out.push_back(nt == 7 ? TV_ERR_INDEX : TV_OK);
    }
};

static tv_request make_req(const void *verts, int64_t nv, int64_t nt, uint32_t flags) {
    tv_request r;
    memset(&r, 0, sizeof r);
    r.verts = verts;
    r.vert_format = TV_VERTS_F32;
    r.nv = nv;
    r.tets = reinterpret_cast<const int32_t *>(verts);
    r.nt = nt;
    r.dims.nx = r.dims.ny = r.dims.nz = 32;
    r.flags = flags;
    return r;
}

static void wait_done(Core &c, int64_t t) { CHECK(c.wait(t, 10.0) == TV_OK); }

// Runs fn on another thread and fails if it does not return within 2 s
// (a call that blocks on the server's lock would never return).
template <class F>
static void returns_promptly(F fn) {
    auto fut = std::async(std::launch::async, fn);
    if (fut.wait_for(std::chrono::seconds(2)) != std::future_status::ready) {
        fprintf(stderr, "FAILED: a server call did not return (lock held)\n");
        fflush(stderr);
        _exit(1);
    }
    fut.get();
}

static void sleep_ms(int ms) { std::this_thread::sleep_for(std::chrono::milliseconds(ms)); }

static void basic_and_overlap() {
    Config cfg;
    cfg.device_bytes = 1 << 20;
    cfg.pinned_bytes = 1 << 16;
    cfg.streams = 2;
    cfg.max_wave_meshes = 1;
    FakeExec ex(cfg.pinned_bytes);
    ex.gate = 0;  // nothing completes yet
    Core core(cfg, &ex);
    core.start();
    static const float dummy[64] = {0};
    std::vector<int64_t> t(6);
    for (auto &x : t) CHECK(core.submit(make_req(dummy, 4, 1, TV_REQ_DEVICE_INPUTS), 1024, 4096, &x) == TV_OK);
    // two waves (one per stream) in flight, the rest queued
    for (int i = 0; i < 200 && core.stats().inflight_waves < 2; ++i) sleep_ms(5);
    tv_server_stats s = core.stats();
    CHECK(s.inflight_waves == 2 && s.inflight_peak == 2);
    CHECK(s.queued == 4 && s.running == 2);
    ex.gate = ~0ull;
    for (int64_t x : t) wait_done(core, x);
    s = core.stats();
    CHECK(s.completed == 6 && s.waves == 6 && s.running == 0 && s.inflight_peak == 2);
    CHECK(ex.max_concurrent.load() == 2);
    for (int64_t x : t) {
        tv_status ds = -99;
        double lat = -1;
        size_t off = 0, words = 0;
        CHECK(core.result(x, &off, &words, &ds, &lat) == TV_OK);
        CHECK(ds == TV_OK && lat >= 0 && words == 1024);
        CHECK(core.release(x) == TV_OK);
        CHECK(core.release(x) == TV_ERR_NOT_FOUND);
    }
    CHECK(core.stats().device_in_use == 0);
    int32_t st = 0;
    CHECK(core.poll(12345, &st) == TV_ERR_NOT_FOUND);
    core.stop();
    printf("ok basic_and_overlap\n");
}

// The front request's grid fits while another wave is in flight, but its
// inputs do not: the scheduler must sleep with the lock released, and admit
// the request once the wave in flight retires.
static void front_partly_fits_inputs() {
    Config cfg;
    cfg.device_bytes = 64 * 1024;
    cfg.pinned_bytes = 64 * 1024;
    cfg.streams = 2;
    cfg.max_wave_meshes = 4;
    FakeExec ex(cfg.pinned_bytes);
    ex.gate = 0;
    Core core(cfg, &ex);
    core.start();
    static float verts[3 * 2000];
    for (int i = 0; i < 6000; ++i) verts[i] = (float)i;
    int64_t a = 0, b = 0;
    // A: device inputs, 16 KiB grid, ~4 KiB workspace
    CHECK(core.submit(make_req(verts, 4, 10, TV_REQ_DEVICE_INPUTS), 4096, 4136, &a) == TV_OK);
    for (int i = 0; i < 200 && core.stats().inflight_waves < 1; ++i) sleep_ms(5);
    // B: pinned inputs of ~40 KiB and a 16 KiB grid: its grid fits beside
    // A, its inputs do not
    CHECK(core.submit(make_req(verts, 2000, 1000, TV_REQ_PINNED_INPUTS), 4096, 8096, &b) == TV_OK);
    sleep_ms(50);
    for (int k = 0; k < 20; ++k) {
        returns_promptly([&] {
            tv_server_stats s = core.stats();
            CHECK(s.queued == 1 && s.running == 1);
            int32_t st = -1;
            CHECK(core.poll(b, &st) == TV_OK && st == TV_REQ_QUEUED);
        });
        sleep_ms(2);
    }
    ex.gate = 1;  // A retires; once its grid is released B must be admitted
    wait_done(core, a);
    CHECK(core.release(a) == TV_OK);
    for (int i = 0; i < 400 && core.stats().running == 0; ++i) sleep_ms(5);
    CHECK(core.stats().running == 1);
    ex.gate = ~0ull;
    wait_done(core, b);
    CHECK(core.stats().completed == 2);
    core.stop();
    printf("ok front_partly_fits_inputs\n");
}

// Same with the workspace: grid and inputs fit, the wave's workspace does not.
static void front_partly_fits_workspace() {
    Config cfg;
    cfg.device_bytes = 64 * 1024;
    cfg.pinned_bytes = 0;
    cfg.streams = 2;
    cfg.max_wave_meshes = 4;
    FakeExec ex(0);
    ex.gate = 0;
    Core core(cfg, &ex);
    core.start();
    static const float dummy[64] = {0};
    int64_t a = 0, b = 0;
    CHECK(core.submit(make_req(dummy, 4, 10, TV_REQ_DEVICE_INPUTS), 4096, 4136, &a) == TV_OK);
    for (int i = 0; i < 200 && core.stats().inflight_waves < 1; ++i) sleep_ms(5);
    CHECK(core.submit(make_req(dummy, 4, 8000, TV_REQ_DEVICE_INPUTS), 4096, 36096, &b) == TV_OK);
    sleep_ms(50);
    for (int k = 0; k < 20; ++k) {
        returns_promptly([&] { CHECK(core.stats().queued == 1); });
        sleep_ms(2);
    }
    ex.gate = ~0ull;
    wait_done(core, a);
    CHECK(core.release(a) == TV_OK);
    wait_done(core, b);
    CHECK(core.stats().completed == 2 && core.stats().waves == 2);
    core.stop();
    printf("ok front_partly_fits_workspace\n");
}

// Retained grids fill the arena; the queue waits (lock released) until the
// client releases one.
static void release_unblocks_queue() {
    Config cfg;
    cfg.device_bytes = 48 * 1024;
    cfg.pinned_bytes = 0;
    cfg.streams = 1;
    cfg.max_wave_meshes = 1;
    FakeExec ex(0);
    Core core(cfg, &ex);
    core.start();
    static const float dummy[64] = {0};
    int64_t t[3];
    // each request: 16 KiB grid + 4100-byte workspace
    for (int i = 0; i < 2; ++i) {
        CHECK(core.submit(make_req(dummy, 4, 1, TV_REQ_DEVICE_INPUTS), 4096, 4100, &t[i]) == TV_OK);
        wait_done(core, t[i]);
    }
    CHECK(core.submit(make_req(dummy, 4, 1, TV_REQ_DEVICE_INPUTS), 4096, 4100, &t[2]) == TV_OK);
    sleep_ms(50);
    int32_t st = -1;
    returns_promptly([&] { CHECK(core.poll(t[2], &st) == TV_OK && st == TV_REQ_QUEUED); });
    CHECK(core.release(t[0]) == TV_OK);
    wait_done(core, t[2]);
    CHECK(core.stats().completed == 3);
    core.stop();
    printf("ok release_unblocks_queue\n");
}

// Host inputs are staged on launcher threads, not on the scheduler's.
static void staging_on_launchers() {
    Config cfg;
    cfg.device_bytes = 1 << 20;
    cfg.pinned_bytes = 1 << 18;
    cfg.streams = 2;
    cfg.max_wave_meshes = 2;
    FakeExec ex(cfg.pinned_bytes);
    Core core(cfg, &ex);
    core.start();
    static float verts[3 * 300];
    for (int i = 0; i < 900; ++i) verts[i] = (float)(i * 7 % 13);
    std::vector<int64_t> t(20);
    for (auto &x : t) CHECK(core.submit(make_req(verts, 300, 10, TV_REQ_HOST_INPUTS), 1024, 4096, &x) == TV_OK);
    for (int64_t x : t) wait_done(core, x);
    CHECK(ex.staged_ok.load() == 20 && ex.staged_bad.load() == 0);
    CHECK(core.stats().pinned_in_use == 0);
    {
        std::lock_guard<std::mutex> lk(ex.m);
        CHECK(ex.launch_threads.size() >= 1 && ex.launch_threads.size() <= 2);
    }
    // pageable inputs need staging: a server without any is refused
    Config c0 = cfg;
    c0.pinned_bytes = 0;
    FakeExec ex0(0);
    Core core0(c0, &ex0);
    core0.start();
    int64_t x = 0;
    CHECK(core0.submit(make_req(verts, 300, 10, TV_REQ_HOST_INPUTS), 1024, 4096, &x) == TV_ERR_TOO_LARGE);
    CHECK(core0.stats().rejected == 1);
    core0.stop();
    core.stop();
    printf("ok staging_on_launchers\n");
}

// A wave that fails to launch finishes with the error; the server goes on.
static void launch_failure_and_status() {
    Config cfg;
    cfg.device_bytes = 1 << 20;
    cfg.pinned_bytes = 0;
    cfg.streams = 2;
    cfg.max_wave_meshes = 1;
    FakeExec ex(0);
    Core core(cfg, &ex);
    core.start();
    static const float dummy[64] = {0};
    int64_t bad = 0, good = 0;
    CHECK(core.submit(make_req(dummy, 13, 1, TV_REQ_DEVICE_INPUTS), 1024, 4096, &bad) == TV_OK);
    CHECK(core.submit(make_req(dummy, 4, 1, TV_REQ_DEVICE_INPUTS), 1024, 4096, &good) == TV_OK);
    wait_done(core, bad);
    wait_done(core, good);
    tv_status ds = 0;
    CHECK(core.result(bad, nullptr, nullptr, &ds, nullptr) == TV_OK && ds == TV_ERR_HIP);
    CHECK(core.result(good, nullptr, nullptr, &ds, nullptr) == TV_OK && ds == TV_OK);
    core.stop();

    StatusExec sx;
    Config c2 = cfg;
    c2.max_wave_meshes = 8;
    Core core2(c2, &sx);
    core2.start();
    std::vector<int64_t> t(16);
    for (size_t i = 0; i < t.size(); ++i)
        CHECK(core2.submit(make_req(dummy, 4, (i % 3 == 0) ? 7 : 9, TV_REQ_DEVICE_INPUTS), 1024, 4096, &t[i]) ==
              TV_OK);
    for (size_t i = 0; i < t.size(); ++i) {
        wait_done(core2, t[i]);
        CHECK(core2.result(t[i], nullptr, nullptr, &ds, nullptr) == TV_OK);
        CHECK(ds == ((i % 3 == 0) ? TV_ERR_INDEX : TV_OK));
    }
    core2.stop();
    printf("ok launch_failure_and_status\n");
}

// Requests of the other tie mode never share a wave; FIFO order holds.
static void tie_modes_split_waves() {
    Config cfg;
    cfg.device_bytes = 1 << 20;
    cfg.pinned_bytes = 0;
    cfg.streams = 1;
    cfg.max_wave_meshes = 16;
    FakeExec ex(0);
    ex.gate = 0;
    Core core(cfg, &ex);
    core.start();
    static const float dummy[64] = {0};
    int64_t first = 0;
    CHECK(core.submit(make_req(dummy, 4, 1, TV_REQ_DEVICE_INPUTS), 1024, 4096, &first) == TV_OK);
    for (int i = 0; i < 200 && core.stats().inflight_waves < 1; ++i) sleep_ms(5);
    std::vector<int64_t> t(6);
    const uint32_t fl[6] = {0, 0, TV_TIE_STRICT, TV_TIE_STRICT, 0, TV_TIE_STRICT};
    for (int i = 0; i < 6; ++i)
        CHECK(core.submit(make_req(dummy, 4, 1, TV_REQ_DEVICE_INPUTS | fl[i]), 1024, 4096, &t[i]) == TV_OK);
    ex.gate = ~0ull;
    for (int64_t x : t) wait_done(core, x);
    // waves: [first], [0,0], [S,S], [0], [S]
    CHECK(core.stats().waves == 5);
    core.stop();
    printf("ok tie_modes_split_waves\n");
}

// Stopping with a wave in flight and requests queued drains the wave and
// returns.
static void stop_with_work() {
    Config cfg;
    cfg.device_bytes = 1 << 20;
    cfg.pinned_bytes = 0;
    cfg.streams = 2;
    cfg.max_wave_meshes = 1;
    FakeExec ex(0);
    ex.gate = 0;
    Core core(cfg, &ex);
    core.start();
    static const float dummy[64] = {0};
    for (int i = 0; i < 8; ++i) {
        int64_t x = 0;
        CHECK(core.submit(make_req(dummy, 4, 1, TV_REQ_DEVICE_INPUTS), 1024, 4096, &x) == TV_OK);
    }
    for (int i = 0; i < 200 && core.stats().inflight_waves < 2; ++i) sleep_ms(5);
    std::thread opener([&] {
        sleep_ms(50);
        ex.gate = ~0ull;
    });
    core.stop();
    opener.join();
    CHECK(core.stats().completed == 2);
    printf("ok stop_with_work\n");
}

// Four clients submit, wait for, check and release 2000 requests of random
// size against a small arena, with waves finishing at random times.
static void stress() {
    Config cfg;
    cfg.device_bytes = 512 * 1024;
    cfg.pinned_bytes = 256 * 1024;
    cfg.streams = 3;
    cfg.max_wave_meshes = 8;
    FakeExec ex(cfg.pinned_bytes);
    Core core(cfg, &ex);
    core.start();
    std::atomic<bool> run{true};
    std::thread ticker([&] {
        // waves finish a few at a time
        std::mt19937 rng(5);
        uint64_t g = 0;
        while (run.load()) {
            g += 1 + rng() % 3;
            ex.gate = g;
            std::this_thread::sleep_for(std::chrono::microseconds(50 + rng() % 200));
        }
        ex.gate = ~0ull;
    });
    static float verts[3 * 1000];
    for (int i = 0; i < 3000; ++i) verts[i] = (float)i;
    std::atomic<int> ok{0}, refused{0}, timeouts{0}, bad{0};
    std::vector<std::thread> clients;
    for (int c = 0; c < 4; ++c) {
        clients.emplace_back([&, c] {
            std::mt19937 rng(100 + c);
            for (int i = 0; i < 500; ++i) {
                const int64_t nv = 14 + rng() % 986, nt = 1 + rng() % 2000;  // nv 13 fails on purpose elsewhere
                const uint32_t in = (rng() % 3 == 0)   ? TV_REQ_HOST_INPUTS
                                    : (rng() % 2 == 0) ? TV_REQ_PINNED_INPUTS
                                                       : TV_REQ_DEVICE_INPUTS;
                const size_t words = 256u << (rng() % 5);
                int64_t t = 0;
                if (core.submit(make_req(verts, nv, nt, in), words, 4096 + 4 * (size_t)nt, &t) != TV_OK) {
                    refused++;
                    continue;
                }
                if (core.wait(t, 60.0) != TV_OK) {
                    timeouts++;
                    continue;
                }
                tv_status ds = -99;
                size_t w = 0;
                if (core.result(t, nullptr, &w, &ds, nullptr) == TV_OK && ds == TV_OK && w == words) ok++;
                else bad++;
                core.release(t);
            }
        });
    }
    for (auto &t : clients) t.join();
    run = false;
    ticker.join();
    tv_server_stats s = core.stats();
    if (ok.load() != 2000)
        fprintf(stderr, "stress: ok %d refused %d timeouts %d bad %d\n", ok.load(), refused.load(),
                timeouts.load(), bad.load());
    CHECK(ok.load() == 2000);
    CHECK(s.completed == 2000 && s.released == 2000 && s.device_in_use == 0 && s.pinned_in_use == 0);
    CHECK(ex.staged_bad.load() == 0);
    core.stop();
    printf("ok stress (%lld waves, peak %lld in flight)\n", (long long)s.waves, (long long)s.inflight_peak);
}

// Clients in the shape of the serving benchmark (one thread submits at
// random times, another waits for, reads and releases each request in
// order) against a small arena on two streams, with waves finishing at
// random times: no region of a wave in flight or of a held grid is ever
// handed out twice.
static void regions_disjoint() {
    Config cfg;
    cfg.device_bytes = 768 * 1024;
    cfg.pinned_bytes = 0;
    cfg.streams = 2;
    cfg.max_wave_meshes = 16;
    RegionExec ex;
    Core core(cfg, &ex);
    core.start();
    std::atomic<bool> run{true};
    std::thread ticker([&] {
        std::mt19937 rng(9);
        uint64_t g = 0;
        while (run.load()) {
            g += 1 + rng() % 2;
            ex.gate = g;
            std::this_thread::sleep_for(std::chrono::microseconds(20 + rng() % 150));
        }
        ex.gate = ~0ull;
    });
    static float verts[3 * 2000];
    const int n = 4000;
    std::vector<std::atomic<int64_t>> tickets(n);
    for (auto &t : tickets) t = 0;
    std::atomic<int> ok{0};
    std::thread collector([&] {
        for (int i = 0; i < n; ++i) {
            while (tickets[i].load() == 0) std::this_thread::sleep_for(std::chrono::microseconds(20));
            const int64_t t = tickets[i].load();
            if (t < 0) continue;
            CHECK(core.wait(t, 60.0) == TV_OK);
            size_t off = 0, words = 0;
            tv_status ds = -99;
            CHECK(core.result(t, &off, &words, &ds, nullptr) == TV_OK && ds == TV_OK);
            ex.drop_grid(off);
            CHECK(core.release(t) == TV_OK);
            ok++;
        }
    });
    std::mt19937 rng(77);
    for (int i = 0; i < n; ++i) {
        const int64_t nv = 14 + rng() % 1986, nt = 1 + rng() % 4000;
        const uint32_t in = (rng() % 2) ? TV_REQ_PINNED_INPUTS : TV_REQ_DEVICE_INPUTS;
        const size_t words = 256u << (rng() % 6);
        int64_t t = 0;
        if (core.submit(make_req(verts, nv, nt, in), words, 4096 + 8 * (size_t)nt, &t) != TV_OK) t = -1;
        tickets[i] = t;
        if (rng() % 4 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 100));
    }
    collector.join();
    run = false;
    ticker.join();
    tv_server_stats s = core.stats();
    core.stop();
    if (ex.overlaps.load())
        fprintf(stderr, "regions_disjoint: %d overlaps over %d waves\n", ex.overlaps.load(), ex.launched.load());
    CHECK(ex.overlaps.load() == 0);
    CHECK(ok.load() == n && s.completed == n && s.device_in_use == 0);
    printf("ok regions_disjoint (%lld waves, peak %lld in flight)\n", (long long)s.waves,
           (long long)s.inflight_peak);
}

int main() {
    setvbuf(stdout, nullptr, _IONBF, 0);
    regions_disjoint();
    basic_and_overlap();
    front_partly_fits_inputs();
    front_partly_fits_workspace();
    release_unblocks_queue();
    staging_on_launchers();
    launch_failure_and_status();
    tie_modes_split_waves();
    stop_with_work();
    stress();
    printf("all ok\n");
    return 0;
}
