// cc_serve.hip — continuous batching of connected-components requests.
//
// Requests arrive in host memory (cc_serve_submit) and wait in a FIFO queue.
// Admission moves a request to the ready list once it fits: a large request
// needs a block of the server's device arena (8m + 4n bytes, its edges and its
// labels-as-parent-array, plus the scratch its solve grows: the membership
// bitmap, the regrouped hook's buffers), a small one needs only a place in a
// batch. The scratch is lent to the worker's slot for that one solve, so no
// worker allocates or frees device memory while serving. Worker
// threads, one HIP stream each, take ready work as soon as they are free:
// a run of small requests is packed into one staging buffer and solved by one
// persistent batched launch; a large request runs the single-graph path on its
// own stream. Different workers' copies and kernels overlap on the device, and
// requests that arrive while others run are admitted as memory frees up.
// Head-of-line blocking is bounded: later requests may pass a request that does
// not fit yet at most kMaxBypass times.
#include <time.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cc_internal.h"

namespace {

using namespace ccm;

constexpr int kMaxBypass = 256;
constexpr uint64_t kAlign = 256;

uint64_t now_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

uint64_t align_up(uint64_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over byte offsets of one device block.
class Arena {
public:
    uint64_t size = 0;
    bool alloc(uint64_t bytes, uint64_t* off) {
        bytes = align_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const uint64_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = align_up(bytes ? bytes : 1);
        used_ -= bytes;
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
    void reset(uint64_t s) {
        size = s;
        free_.clear();
        if (s) free_[0] = s;
        used_ = 0;
    }
    uint64_t used() const { return used_; }

private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t used_ = 0;
};

struct Req {
    uint64_t ticket = 0, n = 0, m = 0;
    const uint32_t* eh = nullptr;
    uint32_t* Lh = nullptr;
    uint32_t flags = 0;
    uint64_t foot = 0;      // device bytes of the large path: edges, labels, scratch
    uint64_t scratch = 0;   // of which the solve's own scratch (lent to the slot)
    bool small = false;
    uint64_t off = 0;       // arena offset (large path)
    int status = CC_OK;
    bool done = false;
    uint32_t batched = 0;
    int bypassed = 0;
    uint64_t t_submit = 0, t_admit = 0, t_start = 0, t_done = 0;
};

struct Worker {
    std::thread th;
    hipStream_t stream = nullptr;
    Slot slot;
    char* dstage = nullptr;      // device staging for batches
    char* hstage = nullptr;      // pinned host staging for batches
};

}  // namespace

struct cc_server {
    int device = 0;
    cc_serve_opts opts{};
    ccm::Tuner* tuner = nullptr;   // the context's stored batch schedules
    uint64_t stage_cap = 0;      // bytes per worker staging buffer
    char* arena_base = nullptr;
    Arena arena;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req*> queue;
    std::deque<Req*> ready;
    std::unordered_map<uint64_t, Req*> reqs;
    uint64_t next_ticket = 1;
    uint32_t inflight = 0;
    uint32_t waiters = 0;     // threads inside cc_serve_wait
    bool closing = false;
    std::vector<Worker> workers;
};

namespace {

// Move queued requests that fit into the ready list (caller holds mu).
void admit(cc_server* s) {
    Req* blocked = nullptr;
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        if (s->inflight >= s->opts.max_inflight) break;
        Req* r = *it;
        bool ok = r->small || s->arena.alloc(r->foot, &r->off);
        if (ok) {
            r->t_admit = now_ns();
            s->ready.push_back(r);
            ++s->inflight;
            it = s->queue.erase(it);
            if (blocked) ++blocked->bypassed;
        } else {
            if (!blocked) blocked = r;
            if (r->bypassed >= kMaxBypass || blocked->bypassed >= kMaxBypass) break;
            ++it;
        }
    }
}

void finish(cc_server* s, Req* r, int status) {
    r->status = status;
    r->t_done = now_ns();
    r->done = true;
}

int run_large(cc_server* s, Worker& w, Req* r) {
    char* base = s->arena_base + r->off;
    uint32_t* d_edges = reinterpret_cast<uint32_t*>(base);
    uint32_t* d_L = reinterpret_cast<uint32_t*>(base + align_up(8 * r->m));
    char* d_scratch = base + align_up(8 * r->m) + align_up(4 * r->n);
    if (r->m)
        CCM_HIP(hipMemcpyAsync(d_edges, r->eh, 8 * r->m, hipMemcpyHostToDevice, w.stream));
    LentScratch own;
    slot_lend_scratch(&w.slot, d_scratch, r->n, r->m, r->flags, &own);
    int rc = run_solve(&w.slot, r->n, r->m, d_edges, d_L, r->flags, 0, w.stream);
    if (!rc) {
        const hipError_t e = hipMemcpyAsync(r->Lh, d_L, 4 * r->n, hipMemcpyDeviceToHost, w.stream);
        rc = e == hipSuccess ? slot_sync(&w.slot, w.stream) : hip_fail(e, "label download");
    }
    (void)hipStreamSynchronize(w.stream);     // the lent block is idle before it is returned
    slot_return_scratch(&w.slot, &own);
    return rc;
}

// Pack small requests into the worker's staging and solve them in one launch.
void run_small(cc_server* s, Worker& w, std::vector<Req*>& rs) {
    const uint32_t G = (uint32_t)rs.size();
    std::vector<uint64_t> eoff(G), loff(G);
    uint64_t at = 0;
    for (uint32_t i = 0; i < G; ++i) { eoff[i] = at; at += align_up(8 * rs[i]->m); }
    const uint64_t edge_bytes = at;
    for (uint32_t i = 0; i < G; ++i) { loff[i] = at; at += align_up(4 * rs[i]->n); }
    const uint64_t status_off = at;
    at += align_up(4ull * G);
    const uint64_t total = at;
    for (uint32_t i = 0; i < G; ++i)
        if (rs[i]->m) std::memcpy(w.hstage + eoff[i], rs[i]->eh, 8 * rs[i]->m);
    std::vector<GraphDesc> descs(G);
    for (uint32_t i = 0; i < G; ++i) {
        descs[i].edges = reinterpret_cast<const int32_t*>(w.dstage + eoff[i]);
        descs[i].L = reinterpret_cast<int32_t*>(w.dstage + loff[i]);
        descs[i].status = reinterpret_cast<int32_t*>(w.dstage + status_off) + i;
        descs[i].n = (uint32_t)rs[i]->n;
        descs[i].pad = 0;
        descs[i].m = (int64_t)rs[i]->m;
    }
    int rc = CC_OK;
    hipError_t e = hipSuccess;
    if (edge_bytes) e = hipMemcpyAsync(w.dstage, w.hstage, edge_bytes, hipMemcpyHostToDevice, w.stream);
    if (e != hipSuccess) rc = hip_fail(e, "batch upload");
    if (!rc) rc = launch_batch(&w.slot, G, descs.data(),
                               tuner_lookup(s->tuner, s->device, G, descs.data()), w.stream);
    if (!rc) {
        e = hipMemcpyAsync(w.hstage + edge_bytes, w.dstage + edge_bytes, total - edge_bytes,
                           hipMemcpyDeviceToHost, w.stream);
        if (e != hipSuccess) rc = hip_fail(e, "batch download");
    }
    e = hipStreamSynchronize(w.stream);
    if (!rc && e != hipSuccess) rc = hip_fail(e, "batch sync");
    for (uint32_t i = 0; i < G; ++i) {
        Req* r = rs[i];
        r->batched = 1;
        if (rc) { r->status = rc; continue; }
        std::memcpy(r->Lh, w.hstage + loff[i], 4 * r->n);
        r->status = reinterpret_cast<const int32_t*>(w.hstage + status_off)[i];
    }
}

void worker_main(cc_server* s, int wi) {
    Worker& w = s->workers[wi];
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        admit(s);
        if (s->ready.empty()) {
            if (s->closing && s->queue.empty()) break;
            s->cv_work.wait(lk);
            continue;
        }
        std::vector<Req*> take;
        // a ready large request, if any (the first in order)
        auto large = std::find_if(s->ready.begin(), s->ready.end(), [](Req* r) { return !r->small; });
        bool small_due = s->ready.front()->small;
        if (small_due && s->opts.coalesce_us && !s->closing) {
            // coalescing window: a batch of small requests waits until its oldest
            // has been ready for coalesce_us (or half a staging buffer has
            // gathered), so that requests arriving meanwhile join the same launch
            uint64_t bytes = 0, oldest = UINT64_MAX;
            for (Req* r : s->ready)
                if (r->small) {
                    bytes += align_up(8 * r->m) + align_up(4 * r->n) + 4;
                    oldest = std::min(oldest, r->t_admit);
                }
            const uint64_t due = oldest + 1000ull * s->opts.coalesce_us;
            const uint64_t now = now_ns();
            if (now < due && bytes < s->stage_cap / 2) {
                if (large == s->ready.end()) {
                    s->cv_work.wait_for(lk, std::chrono::nanoseconds(due - now));
                    continue;
                }
                small_due = false;       // meanwhile, a large request goes first
            }
        }
        if (small_due) {
            // the ready small requests, in order, up to the staging capacity
            uint64_t bytes = 0;
            for (auto it = s->ready.begin(); it != s->ready.end();) {
                Req* r = *it;
                if (!r->small) { ++it; continue; }
                uint64_t b = align_up(8 * r->m) + align_up(4 * r->n) + 4;
                if (!take.empty() && bytes + b + 256 > s->stage_cap) break;
                bytes += b;
                take.push_back(r);
                it = s->ready.erase(it);
            }
        } else {
            if (large == s->ready.end()) large = s->ready.begin();
            take.push_back(*large);
            s->ready.erase(large);
        }
        const uint64_t t_start = now_ns();
        for (Req* r : take) r->t_start = t_start;
        lk.unlock();
        if (take.size() == 1 && !take[0]->small) {
            int rc = run_large(s, w, take[0]);
            take[0]->status = rc;
        } else {
            run_small(s, w, take);
        }
        lk.lock();
        for (Req* r : take) {
            if (!r->small) s->arena.release(r->off, r->foot);
            --s->inflight;
            finish(s, r, r->status);
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
}

void server_free(cc_server* s) {
    for (auto& w : s->workers) {
        if (w.stream) (void)hipStreamDestroy(w.stream);
        slot_destroy(&w.slot);
        if (w.dstage) (void)hipFree(w.dstage);
        if (w.hstage) (void)hipHostFree(w.hstage);
    }
    if (s->arena_base) (void)hipFree(s->arena_base);
    for (auto& kv : s->reqs) delete kv.second;
    delete s;
}

}  // namespace

extern "C" int cc_serve_open(cc_ctx* ctx, const cc_serve_opts* opts, cc_server** out) {
    if (!ctx || !out) return fail(CC_EINVAL, "NULL argument");
    *out = nullptr;
    int dev = 0;
    uint64_t budget = 0;
    uint32_t samples = 0;
    int rc = ctx_info(ctx, &dev, &budget, &samples);
    if (rc) return rc;
    cc_server* s = new cc_server();
    s->device = dev;
    s->tuner = ctx_tuner(ctx);
    if (opts) s->opts = *opts;
    if (!s->opts.max_inflight) s->opts.max_inflight = 64;
    if (!s->opts.queue_capacity) s->opts.queue_capacity = 4096;
    if (!s->opts.streams) s->opts.streams = 4;
    if (s->opts.streams > 16) s->opts.streams = 16;
    if (!s->opts.small_n) s->opts.small_n = 65536;
    if (!s->opts.hbm_budget) s->opts.hbm_budget = std::min<uint64_t>(budget, 32ull << 30);
    const uint64_t W = s->opts.streams;
    s->stage_cap = std::min<uint64_t>(256ull << 20, s->opts.hbm_budget / (4 * W));
    s->stage_cap &= ~(kAlign - 1);
    const uint64_t stage_total = s->stage_cap * W;
    if (stage_total >= s->opts.hbm_budget) { delete s; return fail(CC_EINVAL, "hbm_budget too small"); }
    const uint64_t arena_bytes = (s->opts.hbm_budget - stage_total) & ~(kAlign - 1);
    if (hipSetDevice(dev) != hipSuccess) { delete s; return fail(CC_EDEVICE, "hipSetDevice"); }
    if (hipMalloc(&s->arena_base, arena_bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return fail(CC_ENOMEM, "server arena allocation failed");
    }
    s->arena.reset(arena_bytes);
    s->workers.resize(W);
    for (uint64_t i = 0; i < W; ++i) {
        Worker& w = s->workers[i];
        if (hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking) != hipSuccess ||
            hipMalloc(&w.dstage, s->stage_cap) != hipSuccess ||
            hipHostMalloc(&w.hstage, s->stage_cap, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            server_free(s);
            return fail(CC_ENOMEM, "server worker allocation failed");
        }
        rc = slot_create(&w.slot, dev, samples);
        if (!rc) rc = batch_reserve(&w.slot, std::max<uint32_t>(s->opts.max_inflight, 1024));
        if (rc) { server_free(s); return rc; }
    }
    for (uint64_t i = 0; i < W; ++i) s->workers[i].th = std::thread(worker_main, s, (int)i);
    *out = s;
    return CC_OK;
}

extern "C" int cc_serve_submit(cc_server* s, uint64_t n, uint64_t m, const uint32_t* edges_host,
                               uint32_t* L_host, uint32_t flags, uint64_t* ticket) {
    if (!s || !ticket) return fail(CC_EINVAL, "NULL argument");
    if (n > 0xFFFFFFFFull) return fail(CC_EINVAL, "n must be < 2^32");
    if (m && !edges_host) return fail(CC_EINVAL, "edges_host is NULL with m > 0");
    if (n && !L_host) return fail(CC_EINVAL, "L_host is NULL with n > 0");
    if (n == 0 && m) return fail(CC_ERANGE, "entries given for an empty vertex set");
    if (flags & ~(uint32_t)(CC_F_ZROOT | CC_F_ZROOT_EXACT | CC_F_NO_SPLIT | CC_F_NO_TILE |
                            CC_F_SYMMETRIC))
        return fail(CC_EINVAL, "flag not accepted by the server (CC_F_ZROOT_HINT, unknown)");
    Req* r = new Req();
    r->n = n; r->m = m; r->eh = edges_host; r->Lh = L_host; r->flags = flags;
    r->scratch = solve_scratch_bytes(n, m, flags);
    r->foot = align_up(8 * m) + align_up(4 * n) + r->scratch;
    const uint64_t stage_need = align_up(8 * m) + align_up(4 * n) + 512;
    r->small = n <= s->opts.small_n && n < (1ull << 31) && stage_need <= s->stage_cap;
    if (!r->small && r->foot > s->arena.size) {
        delete r;
        return fail(CC_ENOMEM, "request exceeds the server's HBM budget");
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->closing) { delete r; return fail(CC_ECANCELED, "server is closing"); }
    if (s->queue.size() >= s->opts.queue_capacity) { delete r; return fail(CC_EAGAIN, "queue full"); }
    r->ticket = s->next_ticket++;
    r->t_submit = now_ns();
    if (n == 0) {
        r->t_admit = r->t_submit;
        finish(s, r, CC_OK);
    } else {
        s->queue.push_back(r);
    }
    s->reqs[r->ticket] = r;
    *ticket = r->ticket;
    s->cv_work.notify_one();
    return CC_OK;
}

extern "C" int cc_serve_wait(cc_server* s, uint64_t ticket, int64_t timeout_us, cc_req_stats* stats) {
    if (!s) return fail(CC_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(CC_EINVAL, "unknown ticket");
    Req* r = it->second;
    auto pred = [r] { return r->done; };
    ++s->waiters;
    bool ok = true;
    if (timeout_us < 0) s->cv_done.wait(lk, pred);
    else ok = s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), pred);
    --s->waiters;
    if (s->closing) s->cv_done.notify_all();
    if (!ok) return CC_ETIMEDOUT;
    if (stats) {
        stats->status = r->status;
        stats->batched = r->batched;
        stats->t_submit_ns = r->t_submit;
        stats->t_admit_ns = r->t_admit;
        stats->t_start_ns = r->t_start ? r->t_start : r->t_admit;
        stats->t_done_ns = r->t_done;
    }
    const int st = r->status;
    s->reqs.erase(it);
    delete r;
    return st;
}

extern "C" int cc_serve_close(cc_server* s) {
    if (!s) return fail(CC_EINVAL, "NULL server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->closing = true;
        for (Req* r : s->queue) finish(s, r, CC_ECANCELED);
        s->queue.clear();
        s->cv_work.notify_all();
        s->cv_done.notify_all();
    }
    for (auto& w : s->workers)
        if (w.th.joinable()) w.th.join();
    {
        // every request is done now; let threads still inside cc_serve_wait leave
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.notify_all();
        s->cv_done.wait(lk, [s] { return s->waiters == 0; });
    }
    server_free(s);
    return CC_OK;
}
