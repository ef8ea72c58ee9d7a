// Continuous-batching server (tv_server_* in tv.h).  The threads and the
// admission bookkeeping live in tv_serve_core.h (HIP-free); this file is the
// device side: the arena and staging memory, one compute stream and
// completion event per stream, and the executor that stages inputs,
// enqueues a wave's copies and kernels and reads back its status words.
#include <hip/hip_runtime.h>
#include <string.h>

#include <memory>
#include <vector>

#include "tv.h"
#include "tv_internal.h"
#include "tv_serve_core.h"
#include "tv_workspace.h"

namespace {

using tv::serve::Req;
using tv::serve::Wave;

class HipExec final : public tv::serve::Executor {
  public:
    int device = 0;
    uint8_t *dev = nullptr;  // device arena
    uint8_t *pin = nullptr;  // pinned staging area
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;  // one wave per stream at a time

    void thread_init() override { hipSetDevice(device); }

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

    size_t workspace_bytes(const std::vector<const Req *> &rs) override {
        std::vector<tv::MeshDesc> descs;
        descs.reserve(rs.size());
        for (const Req *q : rs) descs.push_back(desc_of(*q));
        return tv::layout(tv::assign_bases(descs)).total;
    }

    tv_status launch(const Wave &w, const std::vector<const Req *> &rs) override {
        std::vector<tv::MeshDesc> descs;
        descs.reserve(rs.size());
        for (const Req *q : rs) descs.push_back(desc_of(*q));
        const tv::CallSizes c = tv::assign_bases(descs);
        const uint32_t flags = rs[0]->r.flags & TV_TIE_STRICT;
        hipStream_t s = streams[(size_t)w.stream];
        for (const Req *q : rs) {
            if (!q->in_bytes) continue;
            const size_t vb = 12 * (size_t)q->r.nv, tb = 16 * (size_t)q->r.nt;
            if (q->has_st) {
                // pageable inputs: through this wave's share of the staging area
                memcpy(pin + q->st_off, q->r.verts, vb);
                memcpy(pin + q->st_off + q->verts_bytes, q->r.tets, tb);
                if (hipMemcpyAsync(dev + q->in_off, pin + q->st_off, q->verts_bytes + tb,
                                   hipMemcpyHostToDevice, s) != hipSuccess)
                    return TV_ERR_HIP;
            } else if (hipMemcpyAsync(dev + q->in_off, q->r.verts, vb, hipMemcpyHostToDevice, s) != hipSuccess ||
                       hipMemcpyAsync(dev + q->in_off + q->verts_bytes, q->r.tets, tb,
                                      hipMemcpyHostToDevice, s) != hipSuccess) {
                return TV_ERR_HIP;
            }
        }
        tv_status st = tv::run_meshes(descs, c, dev + w.ws_off, s, flags);
        if (st == TV_OK && hipEventRecord(events[(size_t)w.stream], s) != hipSuccess) st = TV_ERR_HIP;
        if (st != TV_OK) hipStreamSynchronize(s);  // nothing may still read the wave's memory
        return st;
    }

    bool done(const Wave &w) override { return hipEventQuery(events[(size_t)w.stream]) == hipSuccess; }

    void finish(const Wave &w, std::vector<tv_status> &out) override {
        // per-mesh status words (at offset 4 * kMetaWords of the workspace)
        const size_t n = w.tickets.size();
        words_.assign(n, 0u);
        hipStream_t s = streams[(size_t)w.stream];
        const bool ok = hipMemcpyAsync(words_.data(), dev + w.ws_off + 4 * tv::kMetaWords, 4 * n,
                                       hipMemcpyDeviceToHost, s) == hipSuccess &&
                        hipStreamSynchronize(s) == hipSuccess;
        out.assign(n, TV_OK);
        for (size_t i = 0; i < n; ++i)
            out[i] = !ok                                ? TV_ERR_HIP
                     : (words_[i] & tv::kStatusIndex) ? TV_ERR_INDEX
                     : (words_[i] & tv::kStatusRange) ? TV_ERR_RANGE
                                                      : TV_OK;
    }

  private:
    std::vector<uint32_t> words_;  // used by the completer thread only
};

}  // namespace

struct tv_server {
    HipExec ex;
    std::unique_ptr<tv::serve::Core> core;
};

extern "C" {

tv_status tv_server_create(const tv_server_config *cfg, tv_server **out) {
    if (!cfg || !out || cfg->device_bytes < 4096 || cfg->streams < 1 || cfg->max_wave_meshes < 1)
        return tv::set_error(TV_ERR_INVALID_ARG, "bad server configuration");
    tv_server *s = new tv_server();
    HipExec &ex = s->ex;
    if (hipGetDevice(&ex.device) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&ex.dev), cfg->device_bytes) != hipSuccess) {
        delete s;
        return tv::set_error(TV_ERR_HIP, "device arena allocation failed");
    }
    if (cfg->pinned_bytes &&
        hipHostMalloc(reinterpret_cast<void **>(&ex.pin), cfg->pinned_bytes, hipHostMallocDefault) !=
            hipSuccess) {
        hipFree(ex.dev);
        delete s;
        return tv::set_error(TV_ERR_HIP, "pinned staging allocation failed");
    }
    for (int i = 0; i < cfg->streams; ++i) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        // default priority; non-blocking with respect to the null stream
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            if (st) hipStreamDestroy(st);
            tv_server_destroy(s);
            return tv::set_error(TV_ERR_HIP, "stream creation failed");
        }
        ex.streams.push_back(st);
        ex.events.push_back(ev);
    }
    tv::serve::Config c;
    c.device_bytes = cfg->device_bytes;
    c.pinned_bytes = cfg->pinned_bytes;
    c.streams = cfg->streams;
    c.max_wave_meshes = cfg->max_wave_meshes;
    s->core.reset(new tv::serve::Core(c, &s->ex));
    s->core->start();
    *out = s;
    return TV_OK;
}

tv_status tv_server_submit(tv_server *s, const tv_request *req, int64_t *ticket) {
    if (!s || !req || !ticket) return tv::set_error(TV_ERR_INVALID_ARG, "null argument");
    const uint32_t inputs = req->flags & tv::serve::kInputsMask;
    if ((req->flags & ~(tv::serve::kInputsMask | TV_TIE_STRICT)) || inputs == tv::serve::kInputsMask)
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
    // the workspace it would need alone (could it ever fit?)
    std::vector<tv::MeshDesc> one(1, tv::make_batch_desc(req->verts, req->vert_format, req->nv,
                                                         req->tets, req->nt, req->dims, &req->bbox,
                                                         nullptr));
    const size_t ws = tv::layout(tv::assign_bases(one)).total;
    st = s->core->submit(*req, tv_grid_words(req->dims), ws, ticket);
    if (st == TV_ERR_TOO_LARGE)
        return tv::set_error(TV_ERR_TOO_LARGE, "request needs more memory than the server has");
    return st;
}

tv_status tv_server_poll(tv_server *s, int64_t ticket, int32_t *state) {
    if (!s || !state) return tv::set_error(TV_ERR_INVALID_ARG, "null argument");
    if (s->core->poll(ticket, state) != TV_OK)
        return tv::set_error(TV_ERR_NOT_FOUND, "unknown ticket %lld", (long long)ticket);
    return TV_OK;
}

tv_status tv_server_wait(tv_server *s, int64_t ticket, double timeout_s) {
    if (!s) return tv::set_error(TV_ERR_INVALID_ARG, "null server");
    const tv_status st = s->core->wait(ticket, timeout_s);
    if (st == TV_ERR_TIMEOUT) return tv::set_error(TV_ERR_TIMEOUT, "request %lld not done", (long long)ticket);
    if (st != TV_OK) return tv::set_error(TV_ERR_NOT_FOUND, "unknown ticket %lld", (long long)ticket);
    return TV_OK;
}

tv_status tv_server_result(tv_server *s, int64_t ticket, const uint32_t **grid, size_t *words,
                           tv_status *data_status, double *latency_s) {
    if (!s) return tv::set_error(TV_ERR_INVALID_ARG, "null server");
    size_t off = 0;
    if (s->core->result(ticket, &off, words, data_status, latency_s) != TV_OK)
        return tv::set_error(TV_ERR_NOT_FOUND, "ticket %lld unknown or not done", (long long)ticket);
    if (grid) *grid = reinterpret_cast<const uint32_t *>(s->ex.dev + off);
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
    if (s->core->release(ticket) != TV_OK)
        return tv::set_error(TV_ERR_NOT_FOUND, "ticket %lld unknown or not done", (long long)ticket);
    return TV_OK;
}

tv_status tv_server_get_stats(tv_server *s, tv_server_stats *out) {
    if (!s || !out) return tv::set_error(TV_ERR_INVALID_ARG, "null argument");
    *out = s->core->stats();
    return TV_OK;
}

tv_status tv_server_destroy(tv_server *s) {
    if (!s) return tv::set_error(TV_ERR_INVALID_ARG, "null server");
    if (s->core) s->core->stop();  // drains in-flight waves, joins the threads
    s->core.reset();
    HipExec &ex = s->ex;
    for (hipStream_t st : ex.streams) hipStreamDestroy(st);
    for (hipEvent_t ev : ex.events) hipEventDestroy(ev);
    if (ex.pin) hipHostFree(ex.pin);
    if (ex.dev) hipFree(ex.dev);
    delete s;
    return TV_OK;
}

}  // extern "C"
