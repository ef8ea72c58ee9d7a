// Continuous-batching server (tv_server_* in tv.h): a scheduler thread
// admits queued requests into waves by memory footprint and launches each
// wave as one batched launch sequence on a free compute stream; a
// completion thread polls the waves' events, timestamps their requests and
// returns their input and workspace memory.  Grids stay in the device arena
// until the client releases them.
#include <hip/hip_runtime.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "tv.h"
#include "tv_internal.h"
#include "tv_sched.h"
#include "tv_workspace.h"

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr uint32_t kInputsMask = TV_REQ_PINNED_INPUTS | TV_REQ_DEVICE_INPUTS;

struct Req {
    tv_request r;
    size_t verts_bytes = 0;  // 12 * nv rounded up to 256
    size_t in_bytes = 0;     // device copy of the inputs (0 for device inputs)
    size_t in_off = 0, st_off = 0, grid_off = 0;
    bool has_in = false, has_st = false, has_grid = false;
    size_t grid_words = 0;
    double t_submit = 0.0, t_done = 0.0;
    int32_t state = TV_REQ_QUEUED;
    tv_status data_status = TV_OK;
};

struct Wave {
    std::vector<int64_t> tickets;
    size_t ws_off = 0;
    int32_t stream = 0;
    hipEvent_t done = nullptr;
};

}  // namespace

struct tv_server {
    int device = 0;
    uint8_t *dev = nullptr;
    uint8_t *pin = nullptr;
    tv::sched::Arena dev_arena, pin_arena;
    tv::sched::WaveLimits lim;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<bool> stream_busy;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::deque<int64_t> queue;
    std::unordered_map<int64_t, Req> reqs;
    std::vector<Wave> inflight;
    int64_t next_ticket = 1;
    uint64_t frees = 0;  // bumped whenever memory or a stream frees up
    tv_server_stats stats{};
    bool stop = false;
    std::thread sched_thread, done_thread;

    int free_stream() const {
        for (size_t i = 0; i < stream_busy.size(); ++i)
            if (!stream_busy[i]) return (int)i;
        return -1;
    }

    bool needs_staging(const Req &q) const {
        return (q.r.flags & kInputsMask) == TV_REQ_HOST_INPUTS && q.in_bytes > 0;
    }

    void release_regions(Req &q, bool grid_too) {
        if (q.has_in) dev_arena.release(q.in_off), q.has_in = false;
        if (q.has_st) pin_arena.release(q.st_off), q.has_st = false;
        if (grid_too && q.has_grid) dev_arena.release(q.grid_off), q.has_grid = false;
        stats.device_in_use = dev_arena.in_use();
        stats.pinned_in_use = pin_arena.in_use();
        ++frees;
    }

    bool reserve(Req &q) {
        if (!dev_arena.alloc(q.grid_words * 4, &q.grid_off)) return false;
        q.has_grid = true;
        if (q.in_bytes) {
            if (!dev_arena.alloc(q.in_bytes, &q.in_off)) {
                release_regions(q, true);
                return false;
            }
            q.has_in = true;
        }
        if (needs_staging(q)) {
            if (!pin_arena.alloc(q.in_bytes, &q.st_off)) {
                release_regions(q, true);
                return false;
            }
            q.has_st = true;
        }
        return true;
    }

    tv::MeshDesc desc_of(const Req &q) const {
        const void *verts = q.r.verts;
        const int32_t *tets = q.r.tets;
        if (q.in_bytes) {
            verts = dev + q.in_off;
            tets = reinterpret_cast<const int32_t *>(dev + q.in_off + q.verts_bytes);
        }
        return tv::make_batch_desc(verts, q.r.vert_format, q.r.nv, tets, q.r.nt, q.r.dims, &q.r.bbox,
                                   reinterpret_cast<uint32_t *>(dev + q.grid_off));
    }

    void scheduler();
    void completer();
    void launch(Wave &w, std::vector<Req *> &rs, std::unique_lock<std::mutex> &lk);
};

void tv_server::launch(Wave &w, std::vector<Req *> &rs, std::unique_lock<std::mutex> &lk) {
    // Called with the lock held; copies and launches without it.
    std::vector<tv::MeshDesc> descs;
    descs.reserve(rs.size());
    for (Req *q : rs) descs.push_back(desc_of(*q));
    const tv::CallSizes c = tv::assign_bases(descs);
    const uint32_t flags = rs[0]->r.flags & TV_TIE_STRICT;
    hipStream_t s = streams[w.stream];
    lk.unlock();
    tv_status st = TV_OK;
    for (Req *q : rs) {
        if (!q->in_bytes) continue;
        const size_t vb = 12 * (size_t)q->r.nv, tb = 16 * (size_t)q->r.nt;
        if (q->has_st) {
            memcpy(pin + q->st_off, q->r.verts, vb);
            memcpy(pin + q->st_off + q->verts_bytes, q->r.tets, tb);
            if (hipMemcpyAsync(dev + q->in_off, pin + q->st_off, q->verts_bytes + tb,
                               hipMemcpyHostToDevice, s) != hipSuccess)
                st = TV_ERR_HIP;
        } else {
            if (hipMemcpyAsync(dev + q->in_off, q->r.verts, vb, hipMemcpyHostToDevice, s) != hipSuccess ||
                hipMemcpyAsync(dev + q->in_off + q->verts_bytes, q->r.tets, tb, hipMemcpyHostToDevice,
                               s) != hipSuccess)
                st = TV_ERR_HIP;
        }
    }
    if (st == TV_OK) st = tv::run_meshes(descs, c, dev + w.ws_off, s, flags);
    if (st == TV_OK && hipEventRecord(w.done, s) != hipSuccess) st = TV_ERR_HIP;
    lk.lock();
    if (st != TV_OK) {
        // nothing will complete on the device: finish the wave here
        const double t = now_s();
        for (Req *q : rs) {
            q->data_status = st;
            q->state = TV_REQ_DONE;
            q->t_done = t;
            release_regions(*q, false);
        }
        dev_arena.release(w.ws_off);
        stream_busy[w.stream] = false;
        stats.running -= (int64_t)rs.size();
        stats.completed += (int64_t)rs.size();
        ++frees;
        cv_done.notify_all();
        return;
    }
    inflight.push_back(w);
    stats.inflight_waves = (int64_t)inflight.size();
    cv_done.notify_all();
}

void tv_server::scheduler() {
    hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    uint64_t seen_frees = frees;
    for (;;) {
        cv_sched.wait(lk, [&] { return stop || (!queue.empty() && free_stream() >= 0); });
        if (stop) break;
        const int si = free_stream();
        const uint32_t wflags = reqs[queue.front()].r.flags & TV_TIE_STRICT;
        std::vector<int64_t> taken;
        int32_t inflight_waves = (int32_t)inflight.size();
        tv::sched::WaveLimits lim1 = lim;
        lim1.max_inflight = (int32_t)streams.size();
        const int32_t n = tv::sched::admit_wave(queue.size(), lim1, inflight_waves, [&](size_t i) {
            Req &q = reqs[queue[i]];
            if ((q.r.flags & TV_TIE_STRICT) != wflags) return false;
            if (!reserve(q)) return false;
            taken.push_back(queue[i]);
            return true;
        });
        (void)n;
        // the wave's workspace; shrink the wave from its tail until it fits
        size_t ws_off = 0;
        while (!taken.empty()) {
            std::vector<tv::MeshDesc> descs;
            for (int64_t t : taken) descs.push_back(desc_of(reqs[t]));
            const size_t ws = tv::layout(tv::assign_bases(descs)).total;
            if (dev_arena.alloc(ws, &ws_off)) break;
            release_regions(reqs[taken.back()], true);
            taken.pop_back();
        }
        if (taken.empty()) {
            // nothing fits now: wait until memory or a stream frees up
            cv_sched.wait(lk, [&] { return stop || frees != seen_frees; });
            seen_frees = frees;
            continue;
        }
        for (size_t i = 0; i < taken.size(); ++i) queue.pop_front();
        Wave w;
        w.tickets = taken;
        w.ws_off = ws_off;
        w.stream = si;
        w.done = events[si];
        stream_busy[si] = true;
        std::vector<Req *> rs;
        for (int64_t t : taken) {
            Req &q = reqs[t];
            q.state = TV_REQ_RUNNING;
            rs.push_back(&q);
        }
        stats.queued = (int64_t)queue.size();
        stats.running += (int64_t)taken.size();
        stats.waves += 1;
        stats.device_in_use = dev_arena.in_use();
        if (stats.device_in_use > stats.device_peak) stats.device_peak = stats.device_in_use;
        stats.pinned_in_use = pin_arena.in_use();
        launch(w, rs, lk);
        seen_frees = frees;
    }
}

void tv_server::completer() {
    hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    std::vector<uint32_t> words;
    for (;;) {
        if (inflight.empty()) {
            if (stop) break;
            cv_done.wait(lk, [&] { return stop || !inflight.empty(); });
            continue;
        }
        bool progressed = false;
        for (size_t k = 0; k < inflight.size();) {
            if (hipEventQuery(inflight[k].done) != hipSuccess) {
                ++k;
                continue;
            }
            const double t = now_s();
            Wave w = inflight[k];
            inflight.erase(inflight.begin() + (long)k);
            // per-mesh status words (at offset 4 * kMetaWords of the workspace)
            const size_t n = w.tickets.size();
            words.assign(n, 0u);
            hipStream_t s = streams[w.stream];
            lk.unlock();
            const bool ok =
                hipMemcpyAsync(words.data(), dev + w.ws_off + 4 * tv::kMetaWords, 4 * n,
                               hipMemcpyDeviceToHost, s) == hipSuccess &&
                hipStreamSynchronize(s) == hipSuccess;
            lk.lock();
            for (size_t i = 0; i < n; ++i) {
                Req &q = reqs[w.tickets[i]];
                q.t_done = t;
                q.state = TV_REQ_DONE;
                q.data_status = !ok                               ? TV_ERR_HIP
                                : (words[i] & tv::kStatusIndex) ? TV_ERR_INDEX
                                : (words[i] & tv::kStatusRange) ? TV_ERR_RANGE
                                                                : TV_OK;
                release_regions(q, false);
            }
            dev_arena.release(w.ws_off);
            stream_busy[w.stream] = false;
            stats.running -= (int64_t)n;
            stats.completed += (int64_t)n;
            stats.inflight_waves = (int64_t)inflight.size();
            stats.device_in_use = dev_arena.in_use();
            ++frees;
            progressed = true;
            cv_done.notify_all();
            cv_sched.notify_all();
        }
        if (!progressed) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        }
    }
}

extern "C" {

tv_status tv_server_create(const tv_server_config *cfg, tv_server **out) {
    if (!cfg || !out || cfg->device_bytes < 4096 || cfg->streams < 1 || cfg->max_wave_meshes < 1)
        return tv::set_error(TV_ERR_INVALID_ARG, "bad server configuration");
    tv_server *s = new tv_server();
    if (hipGetDevice(&s->device) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&s->dev), cfg->device_bytes) != hipSuccess) {
        delete s;
        return tv::set_error(TV_ERR_HIP, "device arena allocation failed");
    }
    if (cfg->pinned_bytes &&
        hipHostMalloc(reinterpret_cast<void **>(&s->pin), cfg->pinned_bytes, hipHostMallocDefault) !=
            hipSuccess) {
        hipFree(s->dev);
        delete s;
        return tv::set_error(TV_ERR_HIP, "pinned staging allocation failed");
    }
    s->dev_arena.reset(cfg->device_bytes);
    s->pin_arena.reset(cfg->pinned_bytes);
    s->lim.max_meshes = cfg->max_wave_meshes;
    s->lim.max_inflight = cfg->streams;
    for (int i = 0; i < cfg->streams; ++i) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        // default priority; non-blocking with respect to the null stream
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            tv_server_destroy(s);
            return tv::set_error(TV_ERR_HIP, "stream creation failed");
        }
        s->streams.push_back(st);
        s->events.push_back(ev);
        s->stream_busy.push_back(false);
    }
    s->sched_thread = std::thread([s] { s->scheduler(); });
    s->done_thread = std::thread([s] { s->completer(); });
    *out = s;
    return TV_OK;
}

tv_status tv_server_submit(tv_server *s, const tv_request *req, int64_t *ticket) {
    if (!s || !req || !ticket) return tv::set_error(TV_ERR_INVALID_ARG, "null argument");
    const uint32_t inputs = req->flags & kInputsMask;
    if ((req->flags & ~(kInputsMask | TV_TIE_STRICT)) || inputs == kInputsMask)
        return tv::set_error(TV_ERR_INVALID_ARG, "bad request flags 0x%x", req->flags);
    // the grid pointer is checked against a stand-in (the server owns grids);
    // host inputs are checked for presence only (their device copies are
    // aligned by the arena)
    static const uint32_t kStandIn[4] = {0, 0, 0, 0};
    const bool dev_in = inputs == TV_REQ_DEVICE_INPUTS;
    const void *vcheck = dev_in ? req->verts : (req->verts ? (const void *)kStandIn : nullptr);
    const int32_t *tcheck =
        dev_in ? req->tets : (req->tets ? reinterpret_cast<const int32_t *>(kStandIn) : nullptr);
    tv_status st = tv::check_mesh(vcheck, req->vert_format, req->nv, tcheck, req->nt, req->dims,
                                  &req->bbox, kStandIn, "");
    if (st) return st;
    Req q;
    q.r = *req;
    q.grid_words = tv_grid_words(req->dims);
    q.verts_bytes = tv::sched::round_up(12 * (size_t)req->nv);
    q.in_bytes = inputs == TV_REQ_DEVICE_INPUTS ? 0 : q.verts_bytes + 16 * (size_t)req->nt;
    // could it ever fit alone?
    std::vector<tv::MeshDesc> one(1, tv::make_batch_desc(req->verts, req->vert_format, req->nv,
                                                         req->tets, req->nt, req->dims, &req->bbox,
                                                         nullptr));
    const size_t ws = tv::layout(tv::assign_bases(one)).total;
    std::unique_lock<std::mutex> lk(s->mu);
    const bool fits = tv::sched::round_up(q.grid_words * 4) + tv::sched::round_up(q.in_bytes) +
                          tv::sched::round_up(ws) <= s->dev_arena.size() &&
                      (!s->needs_staging(q) || tv::sched::round_up(q.in_bytes) <= s->pin_arena.size());
    if (!fits) {
        s->stats.rejected += 1;
        return tv::set_error(TV_ERR_TOO_LARGE, "request needs more memory than the server has");
    }
    q.t_submit = now_s();
    const int64_t t = s->next_ticket++;
    s->reqs.emplace(t, q);
    s->queue.push_back(t);
    s->stats.submitted += 1;
    s->stats.queued = (int64_t)s->queue.size();
    *ticket = t;
    s->cv_sched.notify_all();
    return TV_OK;
}

tv_status tv_server_poll(tv_server *s, int64_t ticket, int32_t *state) {
    if (!s || !state) return tv::set_error(TV_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return tv::set_error(TV_ERR_NOT_FOUND, "unknown ticket %lld", (long long)ticket);
    *state = it->second.state;
    return TV_OK;
}

tv_status tv_server_wait(tv_server *s, int64_t ticket, double timeout_s) {
    if (!s) return tv::set_error(TV_ERR_INVALID_ARG, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto done = [&] {
        auto it = s->reqs.find(ticket);
        return it == s->reqs.end() || it->second.state == TV_REQ_DONE;
    };
    if (timeout_s > 0) {
        if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done))
            return tv::set_error(TV_ERR_TIMEOUT, "request %lld not done", (long long)ticket);
    } else {
        s->cv_done.wait(lk, done);
    }
    if (s->reqs.find(ticket) == s->reqs.end())
        return tv::set_error(TV_ERR_NOT_FOUND, "unknown ticket %lld", (long long)ticket);
    return TV_OK;
}

tv_status tv_server_result(tv_server *s, int64_t ticket, const uint32_t **grid, size_t *words,
                           tv_status *data_status, double *latency_s) {
    if (!s) return tv::set_error(TV_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end() || it->second.state != TV_REQ_DONE)
        return tv::set_error(TV_ERR_NOT_FOUND, "ticket %lld unknown or not done", (long long)ticket);
    const Req &q = it->second;
    if (grid) *grid = reinterpret_cast<const uint32_t *>(s->dev + q.grid_off);
    if (words) *words = q.grid_words;
    if (data_status) *data_status = q.data_status;
    if (latency_s) *latency_s = q.t_done - q.t_submit;
    return TV_OK;
}

tv_status tv_server_copy_grid(tv_server *s, int64_t ticket, void *dst, size_t words) {
    const uint32_t *g = nullptr;
    size_t n = 0;
    tv_status st = tv_server_result(s, ticket, &g, &n, nullptr, nullptr);
    if (st) return st;
    if (!dst || words < n) return tv::set_error(TV_ERR_INVALID_ARG, "destination too small");
    if (hipMemcpy(dst, g, 4 * n, hipMemcpyDefault) != hipSuccess)
        return tv::set_error(TV_ERR_HIP, "grid copy failed");
    return TV_OK;
}

tv_status tv_server_release(tv_server *s, int64_t ticket) {
    if (!s) return tv::set_error(TV_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end() || it->second.state != TV_REQ_DONE)
        return tv::set_error(TV_ERR_NOT_FOUND, "ticket %lld unknown or not done", (long long)ticket);
    s->release_regions(it->second, true);
    s->reqs.erase(it);
    s->stats.released += 1;
    s->cv_sched.notify_all();
    return TV_OK;
}

tv_status tv_server_get_stats(tv_server *s, tv_server_stats *out) {
    if (!s || !out) return tv::set_error(TV_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->queued = (int64_t)s->queue.size();
    return TV_OK;
}

tv_status tv_server_destroy(tv_server *s) {
    if (!s) return tv::set_error(TV_ERR_INVALID_ARG, "null server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_sched.notify_all();
    s->cv_done.notify_all();
    if (s->sched_thread.joinable()) s->sched_thread.join();
    if (s->done_thread.joinable()) s->done_thread.join();  // drains in-flight waves
    for (hipStream_t st : s->streams) hipStreamDestroy(st);
    for (hipEvent_t ev : s->events) hipEventDestroy(ev);
    if (s->pin) hipHostFree(s->pin);
    if (s->dev) hipFree(s->dev);
    delete s;
    return TV_OK;
}

}  // extern "C"
