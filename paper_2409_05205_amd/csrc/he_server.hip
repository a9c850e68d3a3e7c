// Serving runtime: continuous batching of encrypted layer requests.
//
// Requests name a registered layer and device buffers that stay resident
// (the client's c0 and shares, an output buffer).  A load-generator thread
// submits a trace of requests at their scheduled arrival times; a dispatcher
// thread
//   * admits the oldest pending request as soon as a stream slot is free and
//     its transient memory (layer workspace, plus gather/scatter staging when
//     batched) fits in the HBM budget, carved first-fit from one preallocated
//     pool, so the loop never calls hipMalloc;
//   * batches up to max_batch pending requests of the same layer with it
//     (inputs gathered by device copies into staging, outputs scattered back);
//   * runs batches on several streams at once, so requests that arrive while
//     others are on the GPU overlap with them;
//   * polls completion events and records arrival / dispatch / completion
//     times per request.
// With one stream and max_batch = 1 it is the plain one-request-per-launch
// FCFS server.  Results do not depend on batching: a request's output words
// are those of a lone he_conv_layer / he_fc_layer call on its inputs.

#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/he.h"
#include "he_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct LayerReg {
    he_ctx *ctx;
    const he_layer *ly;
    he_layer_info info;
    size_t c0_words, sh_words, shn_words, out_words;   // per image
};

struct Req {
    uint32_t layer;
    int64_t after = -1;                // request this one waits for (-1: none)
    double arrival;                    // seconds after start (dependents: when their predecessor completed)
    const uint32_t *c0, *sh, *shn;
    uint32_t *out;
    double dispatch = -1, complete = -1;
    uint32_t batch = 0;
    int status = HE_OK;
};

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
    uint32_t *sync = nullptr;           // counter block of the one-launch layer form on this stream
    bool busy = false;
    std::vector<uint32_t> reqs;
    size_t off = 0, bytes = 0;          // pool allocation
};

// First-fit allocator over [0, size) with coalescing of freed ranges.
struct Pool {
    size_t size = 0;
    std::map<size_t, size_t> free_;     // offset -> length
    void init(size_t n) {
        size = n;
        free_.clear();
        if (n) free_[0] = n;
    }
    bool alloc(size_t n, size_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n;
                const size_t o = it->first + n;
                free_.erase(it);
                if (rest) free_[o] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n) {
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct he_server {
    he_server_config cfg;
    int device = 0;
    std::vector<LayerReg> layers;
    std::vector<Req> reqs;
    std::vector<double> sched;          // scheduled arrival of each request as added
    std::vector<std::vector<uint32_t>> dependents;
    std::vector<Slot> slots;
    void *pool_base = nullptr;
    Pool pool;
    // submission queue
    std::mutex mu;
    std::deque<uint32_t> inbox;
    std::atomic<bool> gen_done{false};
    Clock::time_point t0;
    int first_error = HE_OK;
    std::atomic<bool> aborted{false};
};

namespace {

double now_s(const he_server *s) { return std::chrono::duration<double>(Clock::now() - s->t0).count(); }

size_t batch_bytes(const LayerReg &L, uint32_t B) {
    size_t ws = he_layer_workspace_bytes(L.ly, B);
    if (B == 1) return a256(ws);
    return a256(ws) + a256(B * L.c0_words * 4) + a256(B * L.sh_words * 4) + a256(B * L.shn_words * 4) +
           a256(B * L.out_words * 4);
}

int launch_batch(he_server *s, Slot &sl, const std::vector<uint32_t> &ids) {
    const Req &h = s->reqs[ids[0]];
    const LayerReg &L = s->layers[h.layer];
    const uint32_t B = (uint32_t)ids.size();
    char *base = (char *)s->pool_base + sl.off;
    const size_t ws_bytes = a256(he_layer_workspace_bytes(L.ly, B));
    void *ws = base;
    const bool conv = L.info.kind == HE_LAYER_CONV;
    const bool has_sh = h.sh != nullptr, has_shn = h.shn != nullptr;
    int rc;
    if (B == 1) {
        rc = he_layer_call_sync(L.ctx, L.ly, 1, h.c0, h.sh, h.shn, h.out, ws, ws_bytes, sl.sync, sl.st);
    } else {
        uint32_t *c0 = (uint32_t *)(base + ws_bytes);
        uint32_t *sh = (uint32_t *)((char *)c0 + a256(B * L.c0_words * 4));
        uint32_t *shn = (uint32_t *)((char *)sh + a256(B * L.sh_words * 4));
        uint32_t *out = (uint32_t *)((char *)shn + a256(B * L.shn_words * 4));
        for (uint32_t i = 0; i < B; ++i) {
            const Req &r = s->reqs[ids[i]];
            if (hipMemcpyAsync(c0 + i * L.c0_words, r.c0, L.c0_words * 4, hipMemcpyDeviceToDevice, sl.st) !=
                hipSuccess)
                return HE_EDEVICE;
            if (has_sh && hipMemcpyAsync(sh + i * L.sh_words, r.sh, L.sh_words * 4, hipMemcpyDeviceToDevice,
                                         sl.st) != hipSuccess)
                return HE_EDEVICE;
            if (has_shn && hipMemcpyAsync(shn + i * L.shn_words, r.shn, L.shn_words * 4, hipMemcpyDeviceToDevice,
                                          sl.st) != hipSuccess)
                return HE_EDEVICE;
        }
        rc = he_layer_call_sync(L.ctx, L.ly, B, c0, has_sh ? sh : nullptr, has_shn ? shn : nullptr, out, ws,
                                ws_bytes, sl.sync, sl.st);
        if (rc == HE_OK) {
            for (uint32_t i = 0; i < B; ++i) {
                const Req &r = s->reqs[ids[i]];
                if (hipMemcpyAsync(r.out, out + i * L.out_words, L.out_words * 4, hipMemcpyDeviceToDevice,
                                   sl.st) != hipSuccess)
                    return HE_EDEVICE;
            }
        }
    }
    if (rc != HE_OK) return rc;
    return hipEventRecord(sl.done, sl.st) == hipSuccess ? HE_OK : HE_EDEVICE;
}

void generator(he_server *s) {
    hipSetDevice(s->device);
    for (uint32_t i = 0; i < s->reqs.size(); ++i) {
        if (s->reqs[i].after >= 0) continue;   // released by the dispatcher when its predecessor completes
        const double due = s->reqs[i].arrival;
        while (now_s(s) < due && !s->aborted) {
            const double left = due - now_s(s);
            if (left > 200e-6) std::this_thread::sleep_for(std::chrono::microseconds((int64_t)((left - 150e-6) * 1e6)));
        }
        std::lock_guard<std::mutex> lk(s->mu);
        s->inbox.push_back(i);
    }
    s->gen_done = true;
}

// A finished request lets its dependents arrive now; the dependents of a failed
// request fail with it (recursively).
void release_dependents(he_server *s, uint32_t id, double t, std::deque<uint32_t> &pending, size_t &done) {
    for (uint32_t d : s->dependents[id]) {
        Req &r = s->reqs[d];
        if (s->reqs[id].status != HE_OK) {
            r.status = s->reqs[id].status;
            r.arrival = r.dispatch = r.complete = t;
            ++done;
            release_dependents(s, d, t, pending, done);
        } else {
            if (r.arrival < t) r.arrival = t;
            pending.push_back(d);
        }
    }
}

void dispatcher(he_server *s) {
    hipSetDevice(s->device);
    std::deque<uint32_t> pending;          // arrival order
    size_t done = 0;
    const size_t total = s->reqs.size();
    while (done < total) {
        bool progressed = false;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            while (!s->inbox.empty()) {
                pending.push_back(s->inbox.front());
                s->inbox.pop_front();
                progressed = true;
            }
        }
        // completions
        for (Slot &sl : s->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q != hipErrorNotReady) {
                const double t = now_s(s);
                for (uint32_t id : sl.reqs) {
                    s->reqs[id].complete = t;
                    if (q != hipSuccess) s->reqs[id].status = HE_EDEVICE;
                }
                if (q != hipSuccess && s->first_error == HE_OK) s->first_error = HE_EDEVICE;
                for (uint32_t id : sl.reqs) release_dependents(s, id, t, pending, done);
                done += sl.reqs.size();
                s->pool.release(sl.off, sl.bytes);
                sl.busy = false;
                sl.reqs.clear();
                progressed = true;
            }
        }
        // admissions
        for (Slot &sl : s->slots) {
            if (sl.busy || pending.empty()) continue;
            const uint32_t head = pending.front();
            const uint32_t lay = s->reqs[head].layer;
            std::vector<uint32_t> ids{head};
            const bool h_sh = s->reqs[head].sh != nullptr, h_shn = s->reqs[head].shn != nullptr;
            for (auto it = std::next(pending.begin()); it != pending.end() && ids.size() < s->cfg.max_batch; ++it) {
                const Req &o = s->reqs[*it];
                if (o.layer == lay && (o.sh != nullptr) == h_sh && (o.shn != nullptr) == h_shn) ids.push_back(*it);
            }
            // shrink the batch until its memory fits the free budget
            size_t off = 0, need = 0;
            bool ok = false;
            while (!ids.empty()) {
                need = batch_bytes(s->layers[lay], (uint32_t)ids.size());
                if (s->pool.alloc(need, &off)) {
                    ok = true;
                    break;
                }
                ids.pop_back();
            }
            if (!ok) {
                bool any_busy = false;
                for (const Slot &o : s->slots) any_busy |= o.busy;
                if (!any_busy) {   // can never fit: fail this request rather than wait forever
                    s->reqs[head].status = HE_ENOMEM;
                    s->reqs[head].complete = s->reqs[head].dispatch = now_s(s);
                    pending.pop_front();
                    ++done;
                    release_dependents(s, head, s->reqs[head].complete, pending, done);
                    if (s->first_error == HE_OK) s->first_error = HE_ENOMEM;
                    progressed = true;
                }
                break;   // wait for memory to come back (oldest request first)
            }
            for (uint32_t id : ids)
                for (auto it = pending.begin(); it != pending.end(); ++it)
                    if (*it == id) {
                        pending.erase(it);
                        break;
                    }
            sl.off = off;
            sl.bytes = need;
            sl.reqs = ids;
            const double t = now_s(s);
            for (uint32_t id : ids) {
                s->reqs[id].dispatch = t;
                s->reqs[id].batch = (uint32_t)ids.size();
            }
            const int rc = launch_batch(s, sl, ids);
            if (rc != HE_OK) {
                for (uint32_t id : ids) {
                    s->reqs[id].status = rc;
                    s->reqs[id].complete = now_s(s);
                }
                for (uint32_t id : ids) release_dependents(s, id, now_s(s), pending, done);
                if (s->first_error == HE_OK) s->first_error = rc;
                done += ids.size();
                s->pool.release(off, need);
                sl.reqs.clear();
                hipStreamSynchronize(sl.st);
            } else {
                sl.busy = true;
            }
            progressed = true;
        }
        if (s->cfg.timeout_s > 0 && now_s(s) > s->cfg.timeout_s) {
            // give up: every request not yet completed is reported as failed
            for (Req &r : s->reqs)
                if (r.complete < 0) r.status = HE_EDEVICE;
            if (s->first_error == HE_OK) s->first_error = HE_EDEVICE;
            s->aborted = true;
            return;
        }
        if (!progressed) std::this_thread::yield();
    }
}

}  // namespace

extern "C" {

int he_server_create(const he_server_config *cfg, he_server **out) {
    if (!cfg || !out || cfg->streams == 0 || cfg->streams > 64 || cfg->max_batch == 0 || cfg->max_batch > 1024)
        return HE_EINVAL;
    he_server *s = new (std::nothrow) he_server();
    if (!s) return HE_ENOMEM;
    s->cfg = *cfg;
    hipGetDevice(&s->device);
    s->slots.resize(cfg->streams);
    for (Slot &sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess || !(sl.sync = he_sync_block_alloc())) {
            he_server_free(s);
            return HE_EDEVICE;
        }
    }
    if (cfg->hbm_budget_bytes) {
        if (hipMalloc(&s->pool_base, cfg->hbm_budget_bytes) != hipSuccess) {
            he_server_free(s);
            return HE_ENOMEM;
        }
    }
    s->pool.init(cfg->hbm_budget_bytes);
    *out = s;
    return HE_OK;
}

int he_server_add_layer(he_server *s, he_ctx *ctx, const he_layer *ly, uint32_t *layer_id) {
    if (!s || !ctx || !ly || !layer_id) return HE_EINVAL;
    LayerReg L;
    L.ctx = ctx;
    L.ly = ly;
    if (he_layer_info_get(ly, &L.info) != HE_OK) return HE_EINVAL;
    const size_t N = L.info.N, Lm = L.info.L;
    if (L.info.kind == HE_LAYER_CONV) {
        L.c0_words = (size_t)L.info.K_in * Lm * N;
        L.sh_words = (size_t)L.info.K_in * N;
        L.shn_words = (size_t)L.info.K_out * N;
        L.out_words = (size_t)L.info.K_out * Lm * N;
    } else {
        L.c0_words = Lm * N;
        L.sh_words = N;
        L.shn_words = (size_t)L.info.blocks * L.info.n_o_p;
        L.out_words = (size_t)L.info.blocks * Lm * L.info.n_o_p;
    }
    *layer_id = (uint32_t)s->layers.size();
    s->layers.push_back(L);
    return HE_OK;
}

int he_server_add_request_after(he_server *s, uint32_t layer_id, double arrival_s, int64_t after,
                                const uint32_t *d_c0, const uint32_t *d_sh, const uint32_t *d_sh_next,
                                uint32_t *d_out) {
    if (!s || layer_id >= s->layers.size() || !d_c0 || !d_out || arrival_s < 0) return HE_EINVAL;
    if (after >= (int64_t)s->reqs.size() || after < -1) return HE_EINVAL;
    if (after < 0) {   // independent requests form a time-ordered trace
        for (size_t i = s->reqs.size(); i-- > 0;)
            if (s->reqs[i].after < 0) {
                if (arrival_s < s->sched[i]) return HE_EINVAL;
                break;
            }
    }
    Req r;
    r.layer = layer_id;
    r.after = after;
    r.arrival = arrival_s;
    r.c0 = d_c0;
    r.sh = d_sh;
    r.shn = d_sh_next;
    r.out = d_out;
    s->reqs.push_back(r);
    s->sched.push_back(arrival_s);
    return HE_OK;
}

int he_server_add_request(he_server *s, uint32_t layer_id, double arrival_s, const uint32_t *d_c0,
                          const uint32_t *d_sh, const uint32_t *d_sh_next, uint32_t *d_out) {
    return he_server_add_request_after(s, layer_id, arrival_s, -1, d_c0, d_sh, d_sh_next, d_out);
}

int he_server_run(he_server *s) {
    if (!s) return HE_EINVAL;
    s->dependents.assign(s->reqs.size(), {});
    for (size_t i = 0; i < s->reqs.size(); ++i) {
        Req &r = s->reqs[i];
        r.arrival = s->sched[i];
        r.dispatch = r.complete = -1;
        r.batch = 0;
        r.status = HE_OK;
        if (r.after >= 0) s->dependents[r.after].push_back((uint32_t)i);
    }
    s->first_error = HE_OK;
    s->aborted = false;
    s->gen_done = false;
    s->inbox.clear();
    s->t0 = Clock::now();
    std::thread g(generator, s);
    std::thread d(dispatcher, s);
    g.join();
    d.join();
    if (!s->aborted)
        for (Slot &sl : s->slots) hipStreamSynchronize(sl.st);
    return s->first_error;
}

int he_server_results(const he_server *s, double *arrival, double *dispatch, double *complete, uint32_t *batch,
                      int32_t *status) {
    if (!s) return HE_EINVAL;
    for (size_t i = 0; i < s->reqs.size(); ++i) {
        const Req &r = s->reqs[i];
        if (arrival) arrival[i] = r.arrival;
        if (dispatch) dispatch[i] = r.dispatch;
        if (complete) complete[i] = r.complete;
        if (batch) batch[i] = r.batch;
        if (status) status[i] = r.status;
    }
    return HE_OK;
}

uint32_t he_server_requests(const he_server *s) { return s ? (uint32_t)s->reqs.size() : 0; }

void he_server_free(he_server *s) {
    if (!s) return;
    for (Slot &sl : s->slots) {
        if (sl.st) hipStreamSynchronize(sl.st);
        if (sl.done) hipEventDestroy(sl.done);
        if (sl.st) hipStreamDestroy(sl.st);
        if (sl.sync) hipFree(sl.sync);
    }
    if (s->pool_base) hipFree(s->pool_base);
    delete s;
}

}  // extern "C"
