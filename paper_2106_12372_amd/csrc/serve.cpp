// Serving loop: continuous batching of cache queries and training steps from
// several independent resident caches (each cache is the network of Sec. 3-5;
// queries per Sec. 3.5, training steps per Sec. 3.3 and 3.5 and Eq. 5).
//
// One scheduler thread owns the device work.  Clients submit requests from any
// thread; a request is admitted as soon as an in-flight slot is free and its
// scratch memory (training partials) fits in the arena's free space, so
// requests that arrive while others run are launched alongside them on a pool
// of HIP streams.  Queued queries of one cache that no training step of that
// cache separates are launched together, as one multi-segment kernel (up to
// kMaxSegs requests; FP16/BF16 caches).  Requests on one cache keep their
// submission order on the device through events: a query waits for the
// cache's last training step, a training step waits for that step and every
// query issued since.  Requests of different caches, and queries between two
// steps of one cache, overlap.  Kernels are deterministic, each record's result
// is independent of the other records of its launch, and caches share no
// state, so a request's result is the same alone and in any mix.
//
// While requests are on the device the scheduler polls their events (yielding
// the core between polls); when none are, it sleeps on a condition variable
// until a submission arrives.  Completion callbacks (host functions queued
// behind each launch) were measured as the wake-up instead: they doubled the
// median latency of the serving trace, and a callback that takes the
// scheduler's lock can deadlock against a HIP call made under that lock.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <list>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "nrc_api_internal.h"
#include "nrc_internal.h"

using namespace nrc;

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over a byte range, 256-byte granularity.
class Arena {
public:
    void init(size_t size) { free_.clear(); if (size) free_[0] = size; total_ = size; }
    size_t total() const { return total_; }
    bool alloc(size_t bytes, size_t* off) {
        bytes = (bytes + 255) & ~(size_t)255;
        if (bytes == 0) { *off = 0; return true; }
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
        if (bytes == 0) return;
        auto it = free_.emplace(off, bytes).first;
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

private:
    std::map<size_t, size_t> free_;
    size_t total_ = 0;
};

struct Request {
    uint64_t ticket;
    int cache;
    nrc_request req;
    size_t scratch_bytes;
    double t_submit;
};

struct Inflight {
    std::vector<Request> rs;   // one training step, or one or more queries of one cache
    int slot;
    int stream;
    size_t scratch_off;
    size_t scratch_bytes;
    double t_start;
    int status;                // NRC_OK, or the error of a launch that failed after queueing work
};

struct CacheDeps {
    uint64_t last_train = 0;               // ticket of the last training step (0: none)
    std::vector<uint64_t> reads;           // queries issued since that step
};

}  // namespace

struct nrc_server {
    nrc_serve_config cfg;
    std::vector<nrc_cache*> caches;
    char* scratch_base = nullptr;
    Arena arena;
    std::vector<hipStream_t> streams;
    std::vector<int> stream_load;
    std::vector<hipEvent_t> slot_event;     // completion event per in-flight slot
    std::vector<int> slot_free;
    struct HostOut { float loss; int32_t skipped; int32_t pad[2]; };
    static_assert(offsetof(HostOut, skipped) == 4, "one copy fills loss and skipped");
    HostOut* host_out = nullptr;            // pinned, one per slot

    std::mutex mu;
    std::condition_variable cv;
    std::list<Request> pending;             // erasing one entry leaves the others' iterators valid
    std::vector<Inflight> inflight;
    std::unordered_map<uint64_t, int> inflight_slot;   // ticket -> slot while on the device
    std::unordered_map<uint64_t, nrc_result> done;
    std::vector<CacheDeps> deps;
    uint64_t next_ticket = 1;
    size_t n_outstanding = 0;
    uint64_t wakeups = 0;                   // submissions, under mu
    bool stop = false;
    int device = 0;
    std::thread worker;
    std::string worker_error;

    void run();
    bool try_launch(std::vector<Request>& rs, std::unique_lock<std::mutex>& lk);
    void retire(std::unique_lock<std::mutex>& lk);
    void fail_group(const std::vector<Request>& rs, int rc, double t);
};

void nrc_server::fail_group(const std::vector<Request>& rs, int rc, double t) {
    for (const Request& r : rs) {
        nrc_result res{};
        res.status = rc;
        res.t_submit = r.t_submit;
        res.t_start = res.t_done = t;
        done[r.ticket] = res;
        --n_outstanding;
    }
    cv.notify_all();
}

// Launches a training step (rs.size() == 1) or one or more queries of one
// cache; false if no slot or no scratch is free.
bool nrc_server::try_launch(std::vector<Request>& rs, std::unique_lock<std::mutex>&) {
    int slot = -1;
    for (int i = 0; i < (int)slot_free.size(); ++i)
        if (slot_free[i]) { slot = i; break; }
    if (slot < 0) return false;
    const Request& r = rs[0];
    size_t off = 0;
    if (!arena.alloc(r.scratch_bytes, &off)) return false;
    int st = 0;
    for (int i = 1; i < (int)streams.size(); ++i)
        if (stream_load[i] < stream_load[st]) st = i;
    hipStream_t s = streams[st];
    CacheDeps& dp = deps[r.cache];
    auto wait_on = [&](uint64_t t) {
        auto it = inflight_slot.find(t);
        if (it != inflight_slot.end()) (void)hipStreamWaitEvent(s, slot_event[it->second], 0);
    };
    wait_on(dp.last_train);
    nrc_cache* c = caches[r.cache];
    int rc;
    bool enqueued = false;                // device work that may use the scratch is queued
    if (r.req.kind == NRC_REQ_TRAIN) {
        for (uint64_t t : dp.reads) wait_on(t);
        char* sc = scratch_base + off;
        const ScratchLayout sl = scratch_layout(c->cfg, r.req.n);
        rc = enqueue_train_step(c, r.req.enc, r.req.target, nullptr, r.req.n, sc, (float*)(sc + sl.loss),
                                (int32_t*)(sc + sl.skipped), s);
        enqueued = true;                  // even a failed enqueue may have queued the training kernel
        if (rc == NRC_OK) {
            // loss and skip flag are adjacent in the scratch and in HostOut
            if (hipMemcpyAsync(&host_out[slot].loss, sc + sl.loss, 8, hipMemcpyDeviceToHost, s) != hipSuccess)
                rc = NRC_EDEVICE;
        }
    } else if (rs.size() == 1) {
        rc = enqueue_forward(c, r.req.enc, r.req.n, r.req.rgb, s);
    } else {
        SegList segs{};
        segs.count = (int)rs.size();
        int64_t tiles = 0;
        for (int k = 0; k < segs.count; ++k) {
            tiles += (rs[k].req.n + 63) / 64;
            segs.tile_end[k] = tiles;
            segs.enc[k] = rs[k].req.enc;
            segs.rgb[k] = rs[k].req.rgb;
            segs.n[k] = rs[k].req.n;
        }
        Geo d(c->cfg.width, c->cfg.n_hidden);
        d.F = c->cfg.factorize ? albedo_col(c->cfg.enc_preset) : 0;
        const hipError_t e = launch_fwd_mfma_segs(c->cfg.precision, d, c->query_ffr(), segs, s);
        rc = e == hipSuccess ? NRC_OK : device_fail(e, "multi-segment forward launch");
    }
    if (r.req.kind != NRC_REQ_TRAIN) {
        host_out[slot].loss = 0.0f;
        host_out[slot].skipped = 0;
    } else if (rc != NRC_OK) {
        host_out[slot].loss = 0.0f;
        host_out[slot].skipped = 1;
    }
    const double t0 = now_s();
    const bool recorded = hipEventRecord(slot_event[slot], s) == hipSuccess;
    if (!recorded && rc == NRC_OK) rc = NRC_EDEVICE;
    if (rc != NRC_OK && !(enqueued && recorded)) {
        // nothing that uses the scratch is queued, or its end cannot be
        // observed: in the latter case the scratch is never reused
        if (!enqueued) arena.release(off, r.scratch_bytes);
        fail_group(rs, rc, t0);
        return true;
    }
    // later requests of this cache order after these (a failed step too: it
    // may have run its kernels)
    if (r.req.kind == NRC_REQ_TRAIN) {
        dp.last_train = r.ticket;
        dp.reads.clear();
    } else {
        for (const Request& q : rs) dp.reads.push_back(q.ticket);
    }
    slot_free[slot] = 0;
    ++stream_load[st];
    for (const Request& q : rs) inflight_slot[q.ticket] = slot;
    // a training step whose enqueue failed part-way retires like the others,
    // once its queued work has finished, and then reports the error
    inflight.push_back(Inflight{rs, slot, st, off, r.scratch_bytes, t0, rc});
    return true;
}

void nrc_server::retire(std::unique_lock<std::mutex>&) {
    for (size_t i = 0; i < inflight.size();) {
        Inflight& f = inflight[i];
        const hipError_t q = hipEventQuery(slot_event[f.slot]);
        if (q == hipErrorNotReady) { ++i; continue; }
        const double t_done = now_s();
        CacheDeps& dp = deps[f.rs[0].cache];
        for (const Request& r : f.rs) {
            nrc_result res{};
            res.status = f.status != NRC_OK ? f.status : q == hipSuccess ? NRC_OK : NRC_EDEVICE;
            res.loss = host_out[f.slot].loss;
            res.skipped = host_out[f.slot].skipped;
            res.t_submit = r.t_submit;
            res.t_start = f.t_start;
            res.t_done = t_done;
            done[r.ticket] = res;
            inflight_slot.erase(r.ticket);
            if (dp.last_train == r.ticket) dp.last_train = 0;
            for (size_t k = 0; k < dp.reads.size(); ++k)
                if (dp.reads[k] == r.ticket) { dp.reads.erase(dp.reads.begin() + k); break; }
            --n_outstanding;
        }
        arena.release(f.scratch_off, f.scratch_bytes);
        slot_free[f.slot] = 1;
        --stream_load[f.stream];
        inflight[i] = inflight.back();
        inflight.pop_back();
        cv.notify_all();
    }
}

void nrc_server::run() {
    (void)hipSetDevice(device);
    const bool segments = !fp32_form(cfg.cache_cfg.precision);   // multi-segment launches (matrix-core forms)
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
        if (stop && pending.empty() && inflight.empty()) break;
        const uint64_t seen = wakeups;
        // Admit in arrival order; a request that does not fit lets later
        // requests of other caches through, never later ones of its own cache.
        // A query takes along the queries of its cache queued after it, up to
        // the cache's next training step.
        std::vector<char> blocked(caches.size(), 0);
        for (auto it = pending.begin(); it != pending.end();) {
            if (blocked[it->cache]) { ++it; continue; }
            std::vector<Request> group{*it};
            std::vector<std::list<Request>::iterator> members{it};
            if (segments && it->req.kind == NRC_REQ_INFER) {
                for (auto jt = std::next(it); jt != pending.end() && (int)group.size() < kMaxSegs; ++jt) {
                    if (jt->cache != it->cache) continue;
                    if (jt->req.kind != NRC_REQ_INFER) break;
                    group.push_back(*jt);
                    members.push_back(jt);
                }
            }
            if (try_launch(group, lk)) {
                for (size_t k = 1; k < members.size(); ++k) pending.erase(members[k]);
                it = pending.erase(members[0]);
            } else {
                blocked[it->cache] = 1;
                ++it;
            }
        }
        retire(lk);
        if (stop && pending.empty() && inflight.empty()) break;
        if (inflight.empty() && pending.empty()) {
            // idle: sleep until a submission (or shutdown)
            cv.wait(lk, [&] { return stop || wakeups != seen; });
        } else if (inflight.empty()) {
            continue;                     // a slot or scratch was just retired: admit again
        } else {
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        }
    }
}

extern "C" {

int nrc_serve_create(const nrc_serve_config* cfg, nrc_server** out) {
    if (!out) return fail(NRC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cfg) return fail(NRC_EINVAL, "config is NULL");
    if (cfg->n_caches < 1 || cfg->n_caches > 64) return fail(NRC_EINVAL, "n_caches must be in 1..64");
    if (cfg->n_streams < 1 || cfg->n_streams > 16) return fail(NRC_EINVAL, "n_streams must be in 1..16");
    if (cfg->max_inflight < 1 || cfg->max_inflight > 1024) return fail(NRC_EINVAL, "max_inflight must be in 1..1024");
    int rc = validate_config(&cfg->cache_cfg);
    if (rc != NRC_OK) return rc;
    if (!cfg->arena || ((uintptr_t)cfg->arena & 255)) return fail(NRC_EINVAL, "arena must be non-NULL and 256-byte aligned");
    const size_t cache_bytes = (cache_layout(cfg->cache_cfg).total + 255) & ~(size_t)255;
    const size_t caches_total = cache_bytes * (size_t)cfg->n_caches;
    if (cfg->arena_bytes < caches_total)
        return fail(NRC_ENOMEM, "arena of %zu bytes cannot hold %d caches (%zu bytes)", cfg->arena_bytes,
                    cfg->n_caches, caches_total);
    nrc_server* s = new (std::nothrow) nrc_server();
    if (!s) return fail(NRC_ENOMEM, "host allocation failed");
    s->cfg = *cfg;
    hipError_t e = hipGetDevice(&s->device);
    char* base = (char*)cfg->arena;
    for (int i = 0; i < cfg->n_caches && e == hipSuccess; ++i) {
        nrc_cache* c = nullptr;
        rc = nrc_cache_create(&cfg->cache_cfg, base + (size_t)i * cache_bytes, cache_bytes, nullptr, &c);
        if (rc != NRC_OK) {
            for (nrc_cache* p : s->caches) nrc_cache_destroy(p);
            delete s;
            return rc;
        }
        s->caches.push_back(c);
    }
    s->deps.resize(cfg->n_caches);
    s->scratch_base = base + caches_total;
    s->arena.init(cfg->arena_bytes - caches_total);
    for (int i = 0; i < cfg->n_streams && e == hipSuccess; ++i) {
        hipStream_t st;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) s->streams.push_back(st);
    }
    s->stream_load.assign(s->streams.size(), 0);
    for (int i = 0; i < cfg->max_inflight && e == hipSuccess; ++i) {
        hipEvent_t ev;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) s->slot_event.push_back(ev);
    }
    s->slot_free.assign(s->slot_event.size(), 1);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&s->host_out, sizeof(nrc_server::HostOut) * cfg->max_inflight, hipHostMallocDefault);
    if (e != hipSuccess) {
        for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
        for (hipEvent_t ev : s->slot_event) (void)hipEventDestroy(ev);
        for (nrc_cache* p : s->caches) nrc_cache_destroy(p);
        delete s;
        return device_fail(e, "server set-up");
    }
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return ok();
}

int nrc_serve_set_weights(nrc_server* srv, int cache_id, const float* host_w, int64_t n) {
    if (!srv || !host_w) return fail(NRC_EINVAL, "NULL argument");
    if (cache_id < 0 || cache_id >= (int)srv->caches.size()) return fail(NRC_EINVAL, "bad cache id %d", cache_id);
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->n_outstanding) return fail(NRC_EBUSY, "requests are pending");
    return nrc_set_weights(srv->caches[cache_id], host_w, n, nullptr);
}

int nrc_serve_get_weights(nrc_server* srv, int cache_id, float* host_w, int64_t n) {
    if (!srv || !host_w) return fail(NRC_EINVAL, "NULL argument");
    if (cache_id < 0 || cache_id >= (int)srv->caches.size()) return fail(NRC_EINVAL, "bad cache id %d", cache_id);
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->n_outstanding) return fail(NRC_EBUSY, "requests are pending");
    return nrc_get_weights(srv->caches[cache_id], host_w, n, nullptr);
}

int nrc_serve_submit(nrc_server* srv, int cache_id, const nrc_request* req, uint64_t* ticket) {
    if (!srv || !req || !ticket) return fail(NRC_EINVAL, "NULL argument");
    if (cache_id < 0 || cache_id >= (int)srv->caches.size()) return fail(NRC_EINVAL, "bad cache id %d", cache_id);
    const nrc_config& cc = srv->cfg.cache_cfg;
    Request r{};
    r.cache = cache_id;
    r.req = *req;
    if (req->kind == NRC_REQ_INFER) {
        if (req->n < 0) return fail(NRC_EINVAL, "n must be >= 0");
        if (req->n > 0 && (!req->enc || !req->rgb)) return fail(NRC_EINVAL, "NULL buffer");
        if (!aligned16(req->enc) || ((uintptr_t)req->rgb & 3)) return fail(NRC_EINVAL, "misaligned buffer");
        r.scratch_bytes = 0;
    } else if (req->kind == NRC_REQ_TRAIN) {
        if (req->n < 1 || req->n > ((int64_t)1 << 31)) return fail(NRC_EINVAL, "bad training batch size");
        if (!req->enc || !req->target) return fail(NRC_EINVAL, "NULL buffer");
        if (!aligned16(req->enc) || ((uintptr_t)req->target & 3)) return fail(NRC_EINVAL, "misaligned buffer");
        r.scratch_bytes = scratch_layout(cc, req->n).total;
    } else {
        return fail(NRC_EINVAL, "unknown request kind %d", req->kind);
    }
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->stop) return fail(NRC_EINVAL, "server is shutting down");
    if (((r.scratch_bytes + 255) & ~(size_t)255) > srv->arena.total())
        return fail(NRC_ENOMEM, "request needs %zu bytes of scratch, the arena has %zu", r.scratch_bytes,
                    srv->arena.total());
    r.ticket = srv->next_ticket++;
    r.t_submit = now_s();
    if (req->kind == NRC_REQ_INFER && req->n == 0) {
        nrc_result res{};
        res.status = NRC_OK;
        res.t_submit = res.t_start = res.t_done = r.t_submit;
        srv->done[r.ticket] = res;
    } else {
        srv->pending.push_back(r);
        ++srv->n_outstanding;
        ++srv->wakeups;
        srv->cv.notify_all();
    }
    *ticket = r.ticket;
    return ok();
}

int nrc_serve_poll(nrc_server* srv, uint64_t ticket, nrc_result* res) {
    if (!srv || !res) return fail(NRC_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->done.find(ticket);
    if (it != srv->done.end()) {
        *res = it->second;
        srv->done.erase(it);
        ok();
        return res->status < 0 ? res->status : NRC_OK;
    }
    if (ticket == 0 || ticket >= srv->next_ticket) return fail(NRC_ENOTFOUND, "unknown ticket");
    if (srv->inflight_slot.count(ticket)) { res->status = NRC_PENDING; ok(); return NRC_PENDING; }
    for (const Request& r : srv->pending)
        if (r.ticket == ticket) { res->status = NRC_PENDING; ok(); return NRC_PENDING; }
    return fail(NRC_ENOTFOUND, "ticket already collected");
}

int nrc_serve_drain(nrc_server* srv) {
    if (!srv) return fail(NRC_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv.wait(lk, [&] { return srv->n_outstanding == 0; });
    return ok();
}

int nrc_serve_destroy(nrc_server* srv) {
    if (!srv) return fail(NRC_EINVAL, "NULL argument");
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        if (srv->n_outstanding) return fail(NRC_EBUSY, "requests are pending; call nrc_serve_drain first");
        srv->stop = true;
        srv->cv.notify_all();
    }
    srv->worker.join();
    for (hipStream_t st : srv->streams) (void)hipStreamSynchronize(st);
    for (hipStream_t st : srv->streams) (void)hipStreamDestroy(st);
    for (hipEvent_t ev : srv->slot_event) (void)hipEventDestroy(ev);
    if (srv->host_out) (void)hipHostFree(srv->host_out);
    for (nrc_cache* c : srv->caches) nrc_cache_destroy(c);
    delete srv;
    return ok();
}

}  // extern "C"
