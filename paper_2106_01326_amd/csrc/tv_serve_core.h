// The serving loop's threads and bookkeeping, free of any HIP call: the
// device work goes through an Executor, so the same loop runs on the GPU
// (tv_server.hip) and, with a fake executor, on a CPU alone under the
// thread sanitizer (tests/native).
//
// Threads:
//   - the scheduler admits queued requests in FIFO order into a wave while
//     their memory (grid + inputs + staging, then the wave's workspace) fits
//     and a stream is free, and hands the wave to that stream's launcher;
//   - one launcher per stream stages the wave's host inputs, enqueues its
//     copies and kernels (Executor::launch) and puts it in flight, so
//     staging copies and launch overhead never hold up admission;
//   - the completer polls the in-flight waves, collects each finished
//     wave's per-request status and returns its inputs, staging and
//     workspace (grids stay until the client releases them).
//
// Waiting: the scheduler sleeps on a condition variable until a request is
// queued and a stream is free, and, when the front request does not fit,
// until memory or a stream is returned by someone else (`frees` counts only
// returns by the completer, a launcher's failure path or a client release,
// never the scheduler's own roll-backs, so that wait always releases the
// lock).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "tv.h"
#include "tv_sched.h"

namespace tv {
namespace serve {

inline double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr uint32_t kInputsMask = TV_REQ_PINNED_INPUTS | TV_REQ_DEVICE_INPUTS;

// One request and the arena regions it holds (offsets into the executor's
// device arena and pinned staging area).
struct Req {
    tv_request r{};
    size_t verts_bytes = 0;  // 12 * nv rounded up to 256
    size_t in_bytes = 0;     // device copy of the inputs (0 for device inputs)
    size_t in_off = 0, st_off = 0, grid_off = 0;
    bool has_in = false, has_st = false, has_grid = false;
    size_t grid_words = 0;
    double t_submit = 0.0, t_done = 0.0;
    int32_t state = TV_REQ_QUEUED;
    tv_status data_status = TV_OK;

    bool needs_staging() const { return (r.flags & kInputsMask) == TV_REQ_HOST_INPUTS && in_bytes > 0; }
};

struct Wave {
    uint64_t seq = 0;  // launch order, from 0
    std::vector<int64_t> tickets;
    size_t ws_off = 0;
    int32_t stream = 0;
};

// Device side of the server.  launch, done and finish are called without
// the server's lock; launch and finish of one stream's waves come from one
// thread at a time.
class Executor {
  public:
    virtual ~Executor() = default;
    // called once by every server thread before its first executor call
    virtual void thread_init() {}
    // workspace bytes a wave of these requests needs
    virtual size_t workspace_bytes(const std::vector<const Req *> &rs) = 0;
    // stages and copies the wave's inputs and enqueues its work on stream
    // w.stream, marking its completion; TV_OK or an error (then nothing
    // of the wave will complete on the device)
    virtual tv_status launch(const Wave &w, const std::vector<const Req *> &rs) = 0;
    // true once the wave's work has finished (must not block for long)
    virtual bool done(const Wave &w) = 0;
    // per-request data status of a finished wave, in ticket order
    virtual void finish(const Wave &w, std::vector<tv_status> &out) = 0;
};

struct Config {
    size_t device_bytes = 0, pinned_bytes = 0;
    int32_t streams = 1, max_wave_meshes = 1;
};

class Core {
  public:
    Core(const Config &cfg, Executor *ex) : ex_(ex) {
        dev_arena_.reset(cfg.device_bytes);
        pin_arena_.reset(cfg.pinned_bytes);
        lim_.max_meshes = cfg.max_wave_meshes;
        lim_.max_inflight = cfg.streams;
        stream_busy_.assign((size_t)cfg.streams, false);
        pending_.resize((size_t)cfg.streams);
        has_pending_.assign((size_t)cfg.streams, false);
    }
    Core(const Core &) = delete;
    Core &operator=(const Core &) = delete;
    ~Core() { stop(); }

    void start() {
        sched_ = std::thread([this] { scheduler(); });
        for (size_t i = 0; i < stream_busy_.size(); ++i)
            launchers_.emplace_back([this, i] { launcher((int32_t)i); });
        done_ = std::thread([this] { completer(); });
    }

    // Stops admission, launches the waves already handed to launchers,
    // waits for every wave in flight and joins the threads.  Requests still
    // queued are never run.
    void stop() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (stopped_) return;
            stop_ = true;
        }
        cv_sched_.notify_all();
        cv_launch_.notify_all();
        cv_done_.notify_all();
        if (sched_.joinable()) sched_.join();
        for (auto &t : launchers_)
            if (t.joinable()) t.join();
        if (done_.joinable()) done_.join();
        std::lock_guard<std::mutex> lk(mu_);
        stopped_ = true;
    }

    size_t device_size() const { return dev_arena_.size(); }
    size_t pinned_size() const { return pin_arena_.size(); }

    // Queues a request that has passed the argument checks.  ws_alone is
    // the workspace it would need alone; TV_ERR_TOO_LARGE when it could
    // never fit.
    tv_status submit(const tv_request &r, size_t grid_words, size_t ws_alone, int64_t *ticket) {
        Req q;
        q.r = r;
        q.grid_words = grid_words;
        q.verts_bytes = sched::round_up(12 * (size_t)r.nv);
        q.in_bytes = (r.flags & kInputsMask) == TV_REQ_DEVICE_INPUTS ? 0 : q.verts_bytes + 16 * (size_t)r.nt;
        std::lock_guard<std::mutex> lk(mu_);
        const bool fits = sched::round_up(q.grid_words * 4) + sched::round_up(q.in_bytes) +
                                  sched::round_up(ws_alone) <= dev_arena_.size() &&
                          (!q.needs_staging() || sched::round_up(q.in_bytes) <= pin_arena_.size());
        if (!fits) {
            stats_.rejected += 1;
            return TV_ERR_TOO_LARGE;
        }
        q.t_submit = now_s();
        const int64_t t = next_ticket_++;
        reqs_.emplace(t, q);
        queue_.push_back(t);
        stats_.submitted += 1;
        stats_.queued = (int64_t)queue_.size();
        *ticket = t;
        cv_sched_.notify_all();
        return TV_OK;
    }

    tv_status poll(int64_t ticket, int32_t *state) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end()) return TV_ERR_NOT_FOUND;
        *state = it->second.state;
        return TV_OK;
    }

    tv_status wait(int64_t ticket, double timeout_s) {
        std::unique_lock<std::mutex> lk(mu_);
        auto done = [&] {
            auto it = reqs_.find(ticket);
            return it == reqs_.end() || it->second.state == TV_REQ_DONE;
        };
        if (timeout_s > 0) {
            // deadline on the steady clock, waited for in steps of at most
            // 20 ms against the system clock (a timed wait on the system
            // clock is a plain pthread timed wait, which the thread
            // sanitizer understands; a clock jump moves one step at most)
            using std::chrono::microseconds;
            const auto end = std::chrono::steady_clock::now() +
                             microseconds((int64_t)std::min(timeout_s * 1e6, 1e15));
            while (!done()) {
                const auto now = std::chrono::steady_clock::now();
                if (now >= end) return TV_ERR_TIMEOUT;
                const microseconds left = std::chrono::duration_cast<microseconds>(end - now);
                cv_done_.wait_until(lk, std::chrono::system_clock::now() +
                                            std::min(left + microseconds(1), microseconds(20000)));
            }
        } else {
            cv_done_.wait(lk, done);
        }
        return reqs_.count(ticket) ? TV_OK : TV_ERR_NOT_FOUND;
    }

    // A done request's grid offset and size, data status and latency.
    tv_status result(int64_t ticket, size_t *grid_off, size_t *words, tv_status *data_status,
                     double *latency_s) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end() || it->second.state != TV_REQ_DONE) return TV_ERR_NOT_FOUND;
        const Req &q = it->second;
        if (grid_off) *grid_off = q.grid_off;
        if (words) *words = q.grid_words;
        if (data_status) *data_status = q.data_status;
        if (latency_s) *latency_s = q.t_done - q.t_submit;
        return TV_OK;
    }

    tv_status release(int64_t ticket) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end() || it->second.state != TV_REQ_DONE) return TV_ERR_NOT_FOUND;
        drop_regions(it->second, true);
        reqs_.erase(it);
        stats_.released += 1;
        ++frees_;
        cv_sched_.notify_all();
        return TV_OK;
    }

    tv_server_stats stats() {
        std::lock_guard<std::mutex> lk(mu_);
        tv_server_stats s = stats_;
        s.queued = (int64_t)queue_.size();
        return s;
    }

  private:
    Executor *ex_;
    sched::Arena dev_arena_, pin_arena_;
    sched::WaveLimits lim_;
    std::mutex mu_;
    std::condition_variable cv_sched_, cv_launch_, cv_done_;
    std::deque<int64_t> queue_;
    std::unordered_map<int64_t, Req> reqs_;  // element references stay valid on insert
    std::vector<bool> stream_busy_;
    std::vector<Wave> pending_;      // per stream: the wave its launcher takes next
    std::vector<bool> has_pending_;
    std::vector<Wave> inflight_;
    int32_t launching_ = 0;  // waves handed to launchers and not yet in flight
    uint64_t frees_ = 0;     // memory or a stream returned (never by the scheduler's roll-backs)
    uint64_t next_wave_ = 0;
    int64_t next_ticket_ = 1;
    tv_server_stats stats_{};
    bool stop_ = false, stopped_ = false;
    std::thread sched_, done_;
    std::vector<std::thread> launchers_;

    int free_stream() const {
        for (size_t i = 0; i < stream_busy_.size(); ++i)
            if (!stream_busy_[i]) return (int)i;
        return -1;
    }

    // Returns a request's inputs and staging (and its grid when grid_too).
    void drop_regions(Req &q, bool grid_too) {
        if (q.has_in) dev_arena_.release(q.in_off), q.has_in = false;
        if (q.has_st) pin_arena_.release(q.st_off), q.has_st = false;
        if (grid_too && q.has_grid) dev_arena_.release(q.grid_off), q.has_grid = false;
        stats_.device_in_use = dev_arena_.in_use();
        stats_.pinned_in_use = pin_arena_.in_use();
    }

    bool reserve(Req &q) {
        if (!dev_arena_.alloc(q.grid_words * 4, &q.grid_off)) return false;
        q.has_grid = true;
        if (q.in_bytes) {
            if (!dev_arena_.alloc(q.in_bytes, &q.in_off)) {
                drop_regions(q, true);
                return false;
            }
            q.has_in = true;
        }
        if (q.needs_staging()) {
            if (!pin_arena_.alloc(q.in_bytes, &q.st_off)) {
                drop_regions(q, true);
                return false;
            }
            q.has_st = true;
        }
        return true;
    }

    // Marks a wave's requests done with their statuses and returns its
    // inputs, staging, workspace and stream.  Lock held.
    void retire(const Wave &w, const std::vector<tv_status> &st) {
        const double t = now_s();
        for (size_t i = 0; i < w.tickets.size(); ++i) {
            Req &q = reqs_[w.tickets[i]];
            q.t_done = t;
            q.state = TV_REQ_DONE;
            q.data_status = i < st.size() ? st[i] : TV_ERR_HIP;
            drop_regions(q, false);
        }
        dev_arena_.release(w.ws_off);
        stream_busy_[(size_t)w.stream] = false;
        stats_.running -= (int64_t)w.tickets.size();
        stats_.completed += (int64_t)w.tickets.size();
        stats_.device_in_use = dev_arena_.in_use();
        ++frees_;
        cv_done_.notify_all();
        cv_sched_.notify_all();
    }

    void scheduler() {
        ex_->thread_init();
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            cv_sched_.wait(lk, [&] { return stop_ || (!queue_.empty() && free_stream() >= 0); });
            if (stop_) break;
            const uint64_t seen = frees_;
            const int si = free_stream();
            const uint32_t wflags = reqs_[queue_.front()].r.flags & TV_TIE_STRICT;
            std::vector<int64_t> taken;
            sched::WaveLimits lim1 = lim_;
            lim1.max_inflight = (int32_t)stream_busy_.size();
            const int32_t busy = (int32_t)stream_busy_.size() - 1;  // one stream is free
            sched::admit_wave(queue_.size(), lim1, busy, [&](size_t i) {
                Req &q = reqs_[queue_[i]];
                if ((q.r.flags & TV_TIE_STRICT) != wflags) return false;
                if (!reserve(q)) return false;
                taken.push_back(queue_[i]);
                return true;
            });
            // the wave's workspace; shrink the wave from its tail until it fits
            size_t ws_off = 0;
            while (!taken.empty()) {
                std::vector<const Req *> rs;
                for (int64_t t : taken) rs.push_back(&reqs_[t]);
                if (dev_arena_.alloc(ex_->workspace_bytes(rs), &ws_off)) break;
                drop_regions(reqs_[taken.back()], true);
                taken.pop_back();
            }
            if (taken.empty()) {
                // the front request does not fit now: sleep (lock released)
                // until someone returns memory or a stream
                cv_sched_.wait(lk, [&] { return stop_ || frees_ != seen; });
                continue;
            }
            for (size_t i = 0; i < taken.size(); ++i) queue_.pop_front();
            Wave w;
            w.seq = next_wave_++;
            w.tickets = std::move(taken);
            w.ws_off = ws_off;
            w.stream = si;
            for (int64_t t : w.tickets) reqs_[t].state = TV_REQ_RUNNING;
            stream_busy_[(size_t)si] = true;
            stats_.queued = (int64_t)queue_.size();
            stats_.running += (int64_t)w.tickets.size();
            stats_.waves += 1;
            stats_.device_in_use = dev_arena_.in_use();
            if (stats_.device_in_use > stats_.device_peak) stats_.device_peak = stats_.device_in_use;
            stats_.pinned_in_use = pin_arena_.in_use();
            pending_[(size_t)si] = std::move(w);
            has_pending_[(size_t)si] = true;
            ++launching_;
            cv_launch_.notify_all();
        }
    }

    void launcher(int32_t si) {
        ex_->thread_init();
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            cv_launch_.wait(lk, [&] { return stop_ || has_pending_[(size_t)si]; });
            if (!has_pending_[(size_t)si]) break;  // stopping, nothing left to launch
            Wave w = std::move(pending_[(size_t)si]);
            has_pending_[(size_t)si] = false;
            std::vector<const Req *> rs;
            for (int64_t t : w.tickets) rs.push_back(&reqs_[t]);
            lk.unlock();
            const tv_status st = ex_->launch(w, rs);
            lk.lock();
            --launching_;
            if (st != TV_OK) {
                // nothing of this wave will complete on the device
                retire(w, std::vector<tv_status>(w.tickets.size(), st));
                continue;
            }
            inflight_.push_back(std::move(w));
            stats_.inflight_waves = (int64_t)inflight_.size();
            if (stats_.inflight_waves > stats_.inflight_peak) stats_.inflight_peak = stats_.inflight_waves;
            cv_done_.notify_all();
        }
        cv_done_.notify_all();  // the completer may be waiting for the last launch
    }

    void completer() {
        ex_->thread_init();
        std::unique_lock<std::mutex> lk(mu_);
        std::vector<tv_status> st;
        for (;;) {
            if (inflight_.empty()) {
                if (stop_ && launching_ == 0) break;
                cv_done_.wait(lk, [&] { return (stop_ && launching_ == 0) || !inflight_.empty(); });
                continue;
            }
            bool progressed = false;
            for (size_t k = 0; k < inflight_.size();) {
                if (!ex_->done(inflight_[k])) {
                    ++k;
                    continue;
                }
                Wave w = std::move(inflight_[k]);
                inflight_.erase(inflight_.begin() + (long)k);
                stats_.inflight_waves = (int64_t)inflight_.size();
                lk.unlock();
                ex_->finish(w, st);
                lk.lock();
                retire(w, st);
                progressed = true;
            }
            if (!progressed) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            }
        }
    }
};

}  // namespace serve
}  // namespace tv
