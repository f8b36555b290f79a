// cc_api.hip — the C ABI of include/cc.h: contexts, argument checks, the
// single-graph entry points and the step entry points.
#include <time.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "cc_internal.h"

// One record of a context's per-call status ring (pinned host memory): the
// status bits the call's work produced, then the call's number, both written by
// the device at the end of the call's stream work.
struct StatusRec {
    uint32_t bits;
    uint32_t pad;
    uint64_t seq;
};

struct cc_ctx {
    int device = 0;
    ccm::Slot slot;
    uint64_t hbm_budget = 0;
    uint32_t samples = 0;
    // per-call status (cc_status_t): created on first use
    std::mutex st_mu;
    StatusRec* st_ring = nullptr;
    hipEvent_t st_ev[CC_STATUS_RING] = {};
    uint64_t st_seq = 0;
    // batch schedules: forced one, stored picks, the cache file
    ccm::Tuner tuner;
    // cc_hook_log_drain: the copy stream, per-launch events and pinned counter
    // snapshots (created on first use)
    std::mutex dr_mu;
    hipStream_t dr_stream = nullptr;
    hipEvent_t dr_ev[CC_DRAIN_MAX_CHUNKS] = {};
    uint64_t* dr_counts = nullptr;
};

namespace ccm {

static thread_local std::string t_detail;

int fail(int code, const std::string& detail) {
    t_detail = detail;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    t_detail = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
    return CC_EDEVICE;
}

int device_cu_count(int device) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 256;
    return cus > 0 ? cus : 256;
}

static uint32_t next_pow2(uint64_t x) {
    uint32_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

int slot_create(Slot* s, int device, uint32_t samples) {
    *s = Slot{};
    s->device = device;
    s->samples = samples;
    s->table = next_pow2(4ull * samples);
    if (s->table < 1024) s->table = 1024;
    CCM_HIP(hipSetDevice(device));
    size_t bytes = sizeof(DevState) + (2ull * s->table + 5ull * kGridCap + 2) * sizeof(uint32_t);
    char* base = nullptr;
    hipError_t e = hipMalloc(&base, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(CC_ENOMEM, "slot scratch allocation failed");
    }
    s->st = reinterpret_cast<DevState*>(base);
    s->hkeys = reinterpret_cast<uint32_t*>(base + sizeof(DevState));
    s->hcounts = s->hkeys + s->table;
    s->bmin = s->hcounts + s->table;
    s->xs = s->bmin + kGridCap;
    CCM_HIP(hipMemset(s->st, 0, sizeof(DevState)));
    // one 64-byte block: the status word, or a 64-bit value read back by an entry point
    e = hipHostMalloc(&s->host_status, 64, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(base);
        s->st = nullptr;
        return fail(CC_ENOMEM, "pinned host status allocation failed");
    }
    *s->host_status = 0;
    CCM_HIP(hipDeviceSynchronize());
    return CC_OK;
}

void slot_destroy(Slot* s) {
    if (!s) return;
    if (hipSetDevice(s->device) != hipSuccess) return;
    (void)hipDeviceSynchronize();
    if (s->st) (void)hipFree(s->st);
    if (s->deg) (void)hipFree(s->deg);
    if (s->zbits) (void)hipFree(s->zbits);
    if (s->csr_tiles) (void)hipFree(s->csr_tiles);
    tiled_free(&s->tiled);
    batch_scratch_free(&s->batch);
    if (s->host_status) (void)hipHostFree(s->host_status);
    *s = Slot{};
}

__global__ void k_status_take(DevState* st, uint32_t* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const uint32_t w = __hip_atomic_exchange(&st->status, 0u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(out, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// The status code of a word of kStatus* bits (the most severe one first).
int status_code(uint32_t w) {
    if (w & kStatusInternal) return fail(CC_EDEVICE, "internal scratch bound exceeded");
    if (w & kStatusRange) return fail(CC_ERANGE, "an endpoint is >= n");
    if (w & kStatusBadOffsets) return fail(CC_EINVAL, "CSR offsets are not a valid row index");
    if (w & kStatusLogFull) return fail(CC_ENOMEM, "update log capacity exceeded");
    return CC_OK;
}

int slot_sync(Slot* s, hipStream_t stream) {
    // read-and-clear in one kernel writing to pinned host memory
    k_status_take<<<1, 64, 0, stream>>>(s->st, s->host_status);
    CCM_HIP(hipGetLastError());
    CCM_HIP(hipStreamSynchronize(stream));
    const uint32_t w = __atomic_load_n(s->host_status, __ATOMIC_ACQUIRE);
    return status_code(w);
}

// Moves the status word into a per-call record: the bits, then the call's
// number (system-scope stores to pinned host memory).
__global__ void k_status_record(DevState* st, uint32_t* bits, uint64_t* seq_out, uint64_t seq) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const uint32_t w = __hip_atomic_exchange(&st->status, 0u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(bits, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(seq_out, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

}  // namespace ccm

using namespace ccm;

// ---- errors / version -------------------------------------------------------------------

extern "C" const char* cc_strerror(int code) {
    switch (code) {
        case CC_OK: return "CC_OK";
        case CC_EINVAL: return "CC_EINVAL: invalid argument";
        case CC_ERANGE: return "CC_ERANGE: vertex ID out of range";
        case CC_ENOMEM: return "CC_ENOMEM: out of device memory or budget";
        case CC_EDEVICE: return "CC_EDEVICE: HIP runtime error";
        case CC_EAGAIN: return "CC_EAGAIN: queue full";
        case CC_ECANCELED: return "CC_ECANCELED: cancelled";
        case CC_ETIMEDOUT: return "CC_ETIMEDOUT: timed out";
        default: return "unknown status";
    }
}

extern "C" const char* cc_last_error_detail(void) { return t_detail.c_str(); }

extern "C" int cc_version(void) { return 100; }

// ---- contexts -----------------------------------------------------------------------------

extern "C" int cc_create(cc_ctx** out, const cc_ctx_opts* opts) {
    if (!out) return fail(CC_EINVAL, "out is NULL");
    *out = nullptr;
    int dev = opts ? opts->device : -1;
    if (dev < 0) CCM_HIP(hipGetDevice(&dev));
    int ndev = 0;
    CCM_HIP(hipGetDeviceCount(&ndev));
    if (dev >= ndev) return fail(CC_EINVAL, "device ordinal out of range");
    uint32_t samples = (opts && opts->zroot_samples) ? opts->zroot_samples : 65536u;
    if (samples > (1u << 24)) return fail(CC_EINVAL, "zroot_samples above 2^24");
    cc_ctx* c = new cc_ctx();
    c->device = dev;
    c->samples = samples;
    int rc = slot_create(&c->slot, dev, samples);
    if (rc) { delete c; return rc; }
    if (opts && opts->reserved) {
        slot_destroy(&c->slot);
        delete c;
        return fail(CC_EINVAL, "cc_ctx_opts.reserved must be 0");
    }
    tuner_open(&c->tuner, opts ? opts->tune_cache : nullptr, opts && opts->batch_autotune);
    if (opts && opts->hbm_budget) c->hbm_budget = opts->hbm_budget;
    else {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess) c->hbm_budget = fr / 4 * 3;
        else c->hbm_budget = 1ull << 34;
    }
    *out = c;
    return CC_OK;
}

namespace ccm {
int ctx_info(cc_ctx* ctx, int* device, uint64_t* budget, uint32_t* samples) {
    if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
    *device = ctx->device;
    *budget = ctx->hbm_budget;
    *samples = ctx->samples;
    return CC_OK;
}
Tuner* ctx_tuner(cc_ctx* ctx) { return ctx ? &ctx->tuner : nullptr; }
}  // namespace ccm

extern "C" void cc_destroy(cc_ctx* ctx) {
    if (!ctx) return;
    slot_destroy(&ctx->slot);    // waits for the device
    for (auto& e : ctx->st_ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->st_ring) (void)hipHostFree(ctx->st_ring);
    for (auto& e : ctx->dr_ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->dr_counts) (void)hipHostFree(ctx->dr_counts);
    if (ctx->dr_stream) (void)hipStreamDestroy(ctx->dr_stream);
    delete ctx;
}

namespace {
std::mutex g_default_mu;
cc_ctx* g_default[64] = {};

int default_ctx(cc_ctx** out) {
    int dev = 0;
    CCM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(CC_EINVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_default_mu);
    if (!g_default[dev]) {
        cc_ctx_opts o{};
        o.device = dev;
        int rc = cc_create(&g_default[dev], &o);
        if (rc) return rc;
    }
    *out = g_default[dev];
    return CC_OK;
}

int check_graph(uint64_t n, uint64_t m, const void* edges, const void* L) {
    if (n > 0xFFFFFFFFull) return fail(CC_EINVAL, "n must be < 2^32");
    if (m && !edges) return fail(CC_EINVAL, "edge_list is NULL with m > 0");
    if (n && !L) return fail(CC_EINVAL, "L is NULL with n > 0");
    if (n == 0 && m) return fail(CC_ERANGE, "entries given for an empty vertex set");
    if (m > (1ull << 40)) return fail(CC_EINVAL, "m above 2^40");
    return CC_OK;
}

int set_dev(cc_ctx* ctx) {
    CCM_HIP(hipSetDevice(ctx->device));
    return CC_OK;
}

constexpr uint32_t kKnownFlags = CC_F_ZROOT | CC_F_ZROOT_EXACT | CC_F_ZROOT_HINT | CC_F_NO_SPLIT |
                                 CC_F_NO_TILE | CC_F_CANON | CC_F_SYMMETRIC;

int check_flags(uint32_t flags) {
    if (flags & ~kKnownFlags) return fail(CC_EINVAL, "unknown flag bits");
    return CC_OK;
}

// After a whole-path call's kernels: record its outcome in the next ring slot
// and fill *st (nothing when st is NULL: the outcome stays for cc_sync).
int finish_status(cc_ctx* ctx, hipStream_t stream, cc_status_t* st) {
    if (!st) return CC_OK;
    std::lock_guard<std::mutex> lk(ctx->st_mu);
    if (!ctx->st_ring) {
        StatusRec* ring = nullptr;
        if (hipHostMalloc(&ring, sizeof(StatusRec) * CC_STATUS_RING, hipHostMallocCoherent) !=
            hipSuccess) {
            (void)hipGetLastError();
            return fail(CC_ENOMEM, "status ring allocation failed");
        }
        std::memset(ring, 0, sizeof(StatusRec) * CC_STATUS_RING);
        for (auto& e : ctx->st_ev) {
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                return fail(CC_EDEVICE, "status event creation failed");
            }
        }
        ctx->st_ring = ring;
    }
    const uint64_t seq = ++ctx->st_seq;
    const uint32_t slot = (uint32_t)(seq % CC_STATUS_RING);
    StatusRec* r = &ctx->st_ring[slot];
    k_status_record<<<1, 64, 0, stream>>>(ctx->slot.st, &r->bits, &r->seq, seq);
    CCM_HIP(hipGetLastError());
    CCM_HIP(hipEventRecord(ctx->st_ev[slot], stream));
    st->ctx = ctx;
    st->seq = seq;
    st->slot = slot;
    st->pad = 0;
    return CC_OK;
}

uint64_t mono_us() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (uint64_t)ts.tv_sec * 1000000ull + (uint64_t)ts.tv_nsec / 1000;
}

}  // namespace

extern "C" int cc_status_wait(cc_status_t* st, int64_t timeout_us) {
    if (!st || !st->ctx || !st->seq || st->slot >= CC_STATUS_RING)
        return fail(CC_EINVAL, "status not filled by a call");
    cc_ctx* ctx = st->ctx;
    hipEvent_t ev = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->st_mu);
        if (!ctx->st_ring || st->seq > ctx->st_seq) return fail(CC_EINVAL, "unknown status");
        if (ctx->st_seq - st->seq >= CC_STATUS_RING)
            return fail(CC_EINVAL, "status record reused by later calls");
        ev = ctx->st_ev[st->slot];
    }
    int rc = set_dev(ctx);
    if (rc) return rc;
    if (timeout_us < 0) {
        CCM_HIP(hipEventSynchronize(ev));
    } else {
        const uint64_t t_end = mono_us() + (uint64_t)timeout_us;
        while (true) {
            const hipError_t e = hipEventQuery(ev);
            if (e == hipSuccess) break;
            if (e != hipErrorNotReady) return hip_fail(e, "hipEventQuery");
            if (mono_us() >= t_end) return CC_ETIMEDOUT;
            timespec ts{0, 20000};
            nanosleep(&ts, nullptr);
        }
    }
    const StatusRec* r = &ctx->st_ring[st->slot];
    const uint64_t seq = __atomic_load_n(&r->seq, __ATOMIC_ACQUIRE);
    const uint32_t bits = __atomic_load_n(&r->bits, __ATOMIC_RELAXED);
    if (seq != st->seq || __atomic_load_n(&r->seq, __ATOMIC_ACQUIRE) != seq)
        return fail(CC_EINVAL, "status record reused by later calls");
    return status_code(bits);
}

// ---- single graph ---------------------------------------------------------------------------

extern "C" int cc_solve(uint64_t n, uint64_t m, const uint32_t* edge_list, uint32_t* L) {
    int rc = check_graph(n, m, edge_list, L);
    if (rc) return rc;
    if (n == 0) return CC_OK;
    cc_ctx* ctx = nullptr;
    if ((rc = default_ctx(&ctx))) return rc;
    std::lock_guard<std::mutex> lk(g_default_mu);  // the default slot is shared
    if ((rc = run_solve(&ctx->slot, n, m, edge_list, L, 0, 0, nullptr))) return rc;
    return slot_sync(&ctx->slot, nullptr);
}

extern "C" int cc_solve_async(cc_ctx* ctx, uint64_t n, uint64_t m, const uint32_t* edge_list,
                              uint32_t* L, uint32_t flags, uint32_t zroot_hint, void* stream,
                              cc_status_t* st) {
    if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
    int rc = check_graph(n, m, edge_list, L);
    if (rc) return rc;
    if ((rc = check_flags(flags))) return rc;
    if ((flags & CC_F_ZROOT_HINT) && n && zroot_hint >= n)
        return fail(CC_EINVAL, "zroot_hint must be < n");
    if ((rc = set_dev(ctx))) return rc;
    if ((rc = run_solve(&ctx->slot, n, m, edge_list, L, flags, zroot_hint, (hipStream_t)stream)))
        return rc;
    return finish_status(ctx, (hipStream_t)stream, st);
}

extern "C" int cc_solve_csr(cc_ctx* ctx, uint64_t n, const uint64_t* offsets, const uint32_t* adj,
                            uint32_t* L, uint32_t flags, uint32_t zroot_hint, void* stream,
                            cc_status_t* st) {
    if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
    if (n >= (1ull << 32)) return fail(CC_EINVAL, "n must be < 2^32");
    if (check_flags(flags)) return CC_EINVAL;
    if (n == 0) return finish_status(ctx, (hipStream_t)stream, st);
    if (!offsets || !L) return fail(CC_EINVAL, "NULL offsets or L");
    if ((flags & CC_F_ZROOT_HINT) && zroot_hint >= n) return fail(CC_EINVAL, "zroot_hint must be < n");
    int rc = set_dev(ctx);
    if (rc) return rc;
    hipStream_t hs = (hipStream_t)stream;
    // the entry count sizes the launches: read off[n] (a coherent copy)
    if ((rc = cohere(hs))) return rc;
    uint64_t* hm = reinterpret_cast<uint64_t*>(ctx->slot.host_status);
    CCM_HIP(hipMemcpyAsync(hm, offsets + n, sizeof(uint64_t), hipMemcpyDeviceToHost, hs));
    CCM_HIP(hipStreamSynchronize(hs));
    const uint64_t m = *hm;
    *hm = 0;
    if (m && !adj) return fail(CC_EINVAL, "NULL adj with a nonzero entry count");
    if (m > (1ull << 40)) return fail(CC_EINVAL, "offsets[n] is implausibly large");
    if ((rc = run_solve_csr(&ctx->slot, n, m, offsets, adj, L, flags, zroot_hint, hs))) return rc;
    return finish_status(ctx, hs, st);
}

extern "C" int cc_solve_u64(cc_ctx* ctx, uint64_t n, uint64_t m, const uint64_t* edges, uint64_t* L,
                            uint32_t flags, void* stream, cc_status_t* st) {
    if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
    if (n >> 62) return fail(CC_EINVAL, "n must be < 2^62");
    if (check_flags(flags)) return CC_EINVAL;
    int rc = set_dev(ctx);
    if (rc) return rc;
    if (n == 0) return finish_status(ctx, (hipStream_t)stream, st);
    if (!L || (m && !edges)) return fail(CC_EINVAL, "NULL L, or NULL edges with m > 0");
    if ((rc = run_solve_w(&ctx->slot, n, m, edges, L, flags, (hipStream_t)stream))) return rc;
    return finish_status(ctx, (hipStream_t)stream, st);
}

extern "C" int cc_sync(cc_ctx* ctx, void* stream) {
    if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
    int rc = set_dev(ctx);
    if (rc) return rc;
    return slot_sync(&ctx->slot, (hipStream_t)stream);
}

// ---- steps -------------------------------------------------------------------------------------

extern "C" int cc_init(cc_ctx* ctx, uint64_t n, uint32_t* P, void* stream) {
    if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
    int rc = check_graph(n, 0, nullptr, P);
    if (rc || n == 0) return rc;
    if ((rc = set_dev(ctx))) return rc;
    if ((rc = cohere((hipStream_t)stream))) return rc;
    if ((rc = run_init(&ctx->slot, n, P, (hipStream_t)stream))) return rc;
    return cohere((hipStream_t)stream);
}

extern "C" int cc_zroot(cc_ctx* ctx, uint64_t n, uint64_t m, const uint32_t* edges,
                        uint32_t flags, uint32_t zroot_hint, void* stream) {
    if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
    if (check_flags(flags)) return CC_EINVAL;
    int rc = check_graph(n, m, edges, (const void*)1);
    if (rc) return rc;
    if (n == 0) return fail(CC_EINVAL, "zero root of an empty vertex set");
    if ((flags & CC_F_ZROOT_HINT) && zroot_hint >= n)
        return fail(CC_EINVAL, "zroot_hint must be < n");
    if ((rc = set_dev(ctx))) return rc;
    if ((rc = cohere((hipStream_t)stream))) return rc;
    if ((rc = run_zroot(&ctx->slot, n, m, edges, flags, zroot_hint, (hipStream_t)stream))) return rc;
    return cohere((hipStream_t)stream);
}

extern "C" int cc_push(cc_ctx* ctx, uint64_t n, uint64_t m, const uint32_t* edges, uint32_t* P,
                       void* stream) {
    if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
    int rc = check_graph(n, m, edges, P);
    if (rc || n == 0) return rc;
    if ((rc = set_dev(ctx))) return rc;
    if ((rc = cohere((hipStream_t)stream))) return rc;
    if ((rc = run_push(&ctx->slot, n, m, edges, P, (hipStream_t)stream))) return rc;
    return cohere((hipStream_t)stream);
}

extern "C" int cc_hook(cc_ctx* ctx, uint64_t n, uint64_t m, const uint32_t* edges, uint32_t* P,
                       uint32_t flags, void* stream) {
    if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
    if (check_flags(flags)) return CC_EINVAL;
    int rc = check_graph(n, m, edges, P);
    if (rc || n == 0) return rc;
    if ((rc = set_dev(ctx))) return rc;
    if ((rc = cohere((hipStream_t)stream))) return rc;
    if ((rc = run_hook(&ctx->slot, n, m, edges, P, flags, (hipStream_t)stream))) return rc;
    return cohere((hipStream_t)stream);
}

extern "C" int cc_hook_log(cc_ctx* ctx, uint64_t n, uint64_t m, const uint32_t* edges,
                           uint32_t* P, uint32_t flags, uint32_t* log, uint64_t log_cap,
                           uint64_t* log_count, void* stream) {
    if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
    if (check_flags(flags)) return CC_EINVAL;
    int rc = check_graph(n, m, edges, P);
    if (rc || n == 0) return rc;
    if (!log_count) return fail(CC_EINVAL, "log_count is NULL");
    if (log_cap && !log) return fail(CC_EINVAL, "log is NULL with a nonzero capacity");
    if ((rc = set_dev(ctx))) return rc;
    if ((rc = cohere((hipStream_t)stream))) return rc;
    if ((rc = run_hook_log(&ctx->slot, n, m, edges, P, flags, log, log_cap, log_count,
                           (hipStream_t)stream)))
        return rc;
    return cohere((hipStream_t)stream);
}

// The context's drain resources, created on first use (caller holds dr_mu).
static int drain_setup(cc_ctx* ctx, uint32_t chunks) {
    if (!ctx->dr_stream) {
        hipStream_t s = nullptr;
        CCM_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        ctx->dr_stream = s;
    }
    if (!ctx->dr_counts) {
        void* p = nullptr;
        if (hipHostMalloc(&p, sizeof(uint64_t) * CC_DRAIN_MAX_CHUNKS, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CC_ENOMEM, "pinned drain counters");
        }
        ctx->dr_counts = static_cast<uint64_t*>(p);
    }
    for (uint32_t k = 0; k < chunks; ++k)
        if (!ctx->dr_ev[k]) CCM_HIP(hipEventCreateWithFlags(&ctx->dr_ev[k], hipEventDisableTiming));
    return CC_OK;
}

extern "C" int cc_hook_log_drain(cc_ctx* ctx, uint64_t n, uint64_t m, const uint32_t* edges,
                                 uint32_t* P, uint32_t flags, uint32_t* log, uint64_t log_cap,
                                 uint32_t* host_log, uint64_t host_cap, uint32_t chunks,
                                 uint64_t* n_messages, void* stream) {
    if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
    if (!n_messages) return fail(CC_EINVAL, "n_messages is NULL");
    *n_messages = 0;
    if (check_flags(flags)) return CC_EINVAL;
    int rc = check_graph(n, m, edges, P);
    if (rc || n == 0) return rc;
    if (chunks == 0 || chunks > CC_DRAIN_MAX_CHUNKS) return fail(CC_EINVAL, "chunks must be in 1..1024");
    if (log_cap && !log) return fail(CC_EINVAL, "log is NULL with a nonzero capacity");
    if (host_cap && !host_log) return fail(CC_EINVAL, "host_log is NULL with a nonzero capacity");
    if (flags & CC_F_ZROOT)
        return fail(CC_EINVAL, "the update log is defined for the plain path (no CC_F_ZROOT)");
    if ((rc = set_dev(ctx))) return rc;
    std::lock_guard<std::mutex> lk(ctx->dr_mu);
    if ((rc = drain_setup(ctx, chunks))) return rc;
    hipStream_t hs = (hipStream_t)stream;
    Slot* s = &ctx->slot;
    uint64_t* hc = ctx->dr_counts;
    // every launch is enqueued first, so the device never waits for the host
    if ((rc = cohere(hs))) return rc;
    if ((rc = log_count_reset(s, hs))) return rc;
    const uint64_t per = (m + chunks - 1) / chunks;
    uint32_t used = 0;
    for (uint64_t k = 0; k < chunks; ++k) {
        const uint64_t a = std::min(m, k * per), b = std::min(m, a + per);
        if (k > 0 && a >= m) break;
        if (b > a)
            if ((rc = run_hook_log(s, n, b - a, edges + 2 * a, P, flags, log, log_cap,
                                   &s->st->log_count, hs)))
                return rc;
        // the messages appended so far, and the point after which the copy
        // engine may read them
        if ((rc = cohere(hs))) return rc;
        if ((rc = log_count_snap(s, &hc[k], hs))) return rc;
        CCM_HIP(hipEventRecord(ctx->dr_ev[k], hs));
        ++used;
    }
    // the copies: each finished range, while the later launches run
    const uint64_t cap = std::min(log_cap, host_cap);
    uint64_t done = 0, total = 0;
    for (uint32_t k = 0; k < used; ++k) {
        CCM_HIP(hipEventSynchronize(ctx->dr_ev[k]));
        total = __atomic_load_n(&hc[k], __ATOMIC_ACQUIRE);
        const uint64_t upto = std::min(total, cap);
        if (upto > done) {
            CCM_HIP(hipStreamWaitEvent(ctx->dr_stream, ctx->dr_ev[k], 0));
            CCM_HIP(hipMemcpyAsync(host_log + 2 * done, log + 2 * done, (upto - done) * 8,
                                   hipMemcpyDeviceToHost, ctx->dr_stream));
            done = upto;
        }
    }
    CCM_HIP(hipStreamSynchronize(ctx->dr_stream));
    *n_messages = total;
    if (total > cap)
        return fail(CC_ENOMEM, "update log capacity exceeded: " + std::to_string(total) +
                                   " messages, room for " + std::to_string(cap));
    return CC_OK;
}

extern "C" int cc_compress(cc_ctx* ctx, uint64_t n, uint32_t* P, uint32_t flags, void* stream) {
    if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
    if (check_flags(flags)) return CC_EINVAL;
    int rc = check_graph(n, 0, nullptr, P);
    if (rc || n == 0) return rc;
    if ((rc = set_dev(ctx))) return rc;
    if ((rc = cohere((hipStream_t)stream))) return rc;
    if ((rc = run_compress(&ctx->slot, n, P, flags, (hipStream_t)stream))) return rc;
    return cohere((hipStream_t)stream);
}

extern "C" int cc_canon(cc_ctx* ctx, uint64_t n, uint32_t* L, void* stream) {
    if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
    int rc = check_graph(n, 0, nullptr, L);
    if (rc || n == 0) return rc;
    if ((rc = set_dev(ctx))) return rc;
    if ((rc = cohere((hipStream_t)stream))) return rc;
    if ((rc = run_canon(&ctx->slot, n, L, (hipStream_t)stream))) return rc;
    return cohere((hipStream_t)stream);
}

extern "C" int cc_export(cc_ctx* ctx, uint64_t n, const uint32_t* P, uint32_t zroot,
                         uint32_t* pairs, uint64_t pairs_cap, uint32_t* zero_ids, uint64_t zero_cap,
                         uint64_t* n_pairs, uint64_t* n_zero, void* stream) {
    if (!ctx || !n_pairs || !n_zero) return fail(CC_EINVAL, "NULL argument");
    *n_pairs = 0;
    *n_zero = 0;
    int rc = check_graph(n, 0, nullptr, P);
    if (rc || n == 0) return rc;
    if ((rc = set_dev(ctx))) return rc;
    return run_export(&ctx->slot, n, P, zroot, pairs, pairs_cap, zero_ids, zero_cap, n_pairs, n_zero,
                      (hipStream_t)stream);
}

extern "C" int cc_hook_ids(cc_ctx* ctx, uint64_t n, uint64_t count, const uint32_t* ids,
                           uint32_t target, uint32_t* P, uint32_t flags, void* stream) {
    if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
    if (check_flags(flags)) return CC_EINVAL;
    int rc = check_graph(n, count, ids, P);
    if (rc || n == 0 || count == 0) return rc;
    if (target >= n) return fail(CC_EINVAL, "target must be < n");
    if ((rc = set_dev(ctx))) return rc;
    if ((rc = cohere((hipStream_t)stream))) return rc;
    if ((rc = run_hook_ids(&ctx->slot, n, count, ids, target, P, flags, (hipStream_t)stream)))
        return rc;
    return cohere((hipStream_t)stream);
}

extern "C" uint32_t cc_id_bytes(uint64_t n) {
    uint32_t k = 1;
    while (k < 8 && (n - 1) >> (8 * k)) ++k;
    return n <= 1 ? 1u : k;
}

static int check_codec(uint64_t count, const void* a, const void* b, uint32_t id_bytes) {
    if (id_bytes < 1 || id_bytes > 4) return fail(CC_EINVAL, "id_bytes must be 1..4");
    if (count && (!a || !b)) return fail(CC_EINVAL, "NULL buffer with a nonzero count");
    if (((uintptr_t)a | (uintptr_t)b) & 3u) return fail(CC_EINVAL, "buffers must be 4-byte aligned");
    if (count > (UINT64_MAX >> 3)) return fail(CC_EINVAL, "count too large");
    return CC_OK;
}

extern "C" int cc_pack_ids(cc_ctx* ctx, uint64_t count, const uint32_t* ids, uint32_t id_bytes,
                           uint8_t* out, void* stream) {
    if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
    int rc = check_codec(count, ids, out, id_bytes);
    if (rc || count == 0) return rc;
    if ((rc = set_dev(ctx))) return rc;
    if ((rc = cohere((hipStream_t)stream))) return rc;
    if ((rc = run_pack_ids(&ctx->slot, count, ids, id_bytes, out, (hipStream_t)stream))) return rc;
    return cohere((hipStream_t)stream);
}

extern "C" int cc_unpack_ids(cc_ctx* ctx, uint64_t count, const uint8_t* in, uint32_t id_bytes,
                             uint32_t* ids, void* stream) {
    if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
    int rc = check_codec(count, in, ids, id_bytes);
    if (rc || count == 0) return rc;
    if ((rc = set_dev(ctx))) return rc;
    if ((rc = cohere((hipStream_t)stream))) return rc;
    if ((rc = run_unpack_ids(&ctx->slot, count, in, id_bytes, ids, (hipStream_t)stream))) return rc;
    return cohere((hipStream_t)stream);
}

extern "C" int cc_get_zroot(cc_ctx* ctx, void* stream, uint32_t* zroot_out) {
    if (!ctx || !zroot_out) return fail(CC_EINVAL, "NULL argument");
    int rc = set_dev(ctx);
    if (rc) return rc;
    if ((rc = cohere((hipStream_t)stream))) return rc;
    CCM_HIP(hipMemcpyAsync(ctx->slot.host_status, &ctx->slot.st->zroot, sizeof(uint32_t),
                           hipMemcpyDeviceToHost, (hipStream_t)stream));
    CCM_HIP(hipStreamSynchronize((hipStream_t)stream));
    *zroot_out = *ctx->slot.host_status;
    *ctx->slot.host_status = 0;
    return CC_OK;
}

// ---- batch -------------------------------------------------------------------------------------

// Arguments of cc_batch and its variants checked, descriptors built.
static int batch_args(cc_ctx* ctx, uint32_t G, const int64_t* vtx_off, const int64_t* edge_off,
                      const int32_t* edges, int32_t* L, int32_t* status, void* stream,
                      std::vector<GraphDesc>* descs) {
    if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
    if (!vtx_off || !edge_off || !status) return fail(CC_EINVAL, "NULL offsets or status");
    int rc = set_dev(ctx);
    if (rc) return rc;
    return batch_descs(G, vtx_off, edge_off, edges, L, status, (hipStream_t)stream, descs);
}

static int check_sched(const cc_batch_sched* s) {
    if (s && s->wave_max_n > CC_BATCH_WAVE_MAX_N)
        return fail(CC_EINVAL, "wave_max_n above CC_BATCH_WAVE_MAX_N");
    return CC_OK;
}

extern "C" int cc_batch_graph_create(cc_ctx* ctx, uint32_t G, const int64_t* vtx_off,
                                     const int64_t* edge_off, const int32_t* edges, int32_t* L,
                                     int32_t* status, void* stream, cc_batch_graph** out) {
    if (!out) return fail(CC_EINVAL, "out is NULL");
    *out = nullptr;
    if (G == 0) return fail(CC_EINVAL, "G must be > 0");
    std::vector<GraphDesc> descs;
    int rc = batch_args(ctx, G, vtx_off, edge_off, edges, L, status, stream, &descs);
    if (rc) return rc;
    BatchSched sc;
    uint32_t source = 0;
    if ((rc = tuner_choose(&ctx->tuner, &ctx->slot, G, descs.data(), (hipStream_t)stream, &sc,
                           &source)))
        return rc;
    void* h = nullptr;
    if ((rc = batch_graph_create(&ctx->slot, G, descs.data(), sc, &h))) return rc;
    *out = reinterpret_cast<cc_batch_graph*>(h);
    return CC_OK;
}

extern "C" int cc_batch_graph_launch(cc_batch_graph* g, void* stream) {
    if (!g) return fail(CC_EINVAL, "graph is NULL");
    return batch_graph_launch(g, (hipStream_t)stream);
}

extern "C" void cc_batch_graph_destroy(cc_batch_graph* g) {
    if (g) batch_graph_destroy(g);
}

extern "C" int cc_batch_ex(cc_ctx* ctx, uint32_t G, const int64_t* vtx_off, const int64_t* edge_off,
                           const int32_t* edges, int32_t* L, int32_t* status,
                           const cc_batch_sched* sched, void* stream) {
    if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
    if (G == 0) return CC_OK;
    int rc = check_sched(sched);
    if (rc) return rc;
    std::vector<GraphDesc> descs;
    if ((rc = batch_args(ctx, G, vtx_off, edge_off, edges, L, status, stream, &descs))) return rc;
    hipStream_t hs = (hipStream_t)stream;
    BatchSched sc;
    if (sched) {
        sc = *sched;
    } else {
        uint32_t source = 0;
        if ((rc = tuner_choose(&ctx->tuner, &ctx->slot, G, descs.data(), hs, &sc, &source)))
            return rc;
    }
    if ((rc = launch_batch(&ctx->slot, G, descs.data(), sc, hs))) return rc;
    CCM_HIP(hipStreamSynchronize(hs));
    return CC_OK;
}

extern "C" int cc_batch(cc_ctx* ctx, uint32_t G, const int64_t* vtx_off, const int64_t* edge_off,
                        const int32_t* edges, int32_t* L, int32_t* status, void* stream) {
    return cc_batch_ex(ctx, G, vtx_off, edge_off, edges, L, status, nullptr, stream);
}

extern "C" int cc_batch_sched_force(cc_ctx* ctx, const cc_batch_sched* sched) {
    if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
    int rc = check_sched(sched);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(ctx->tuner.mu);
    ctx->tuner.forced = sched != nullptr;
    if (sched) ctx->tuner.force = *sched;
    return CC_OK;
}

extern "C" int cc_batch_tune(cc_ctx* ctx, uint32_t G, const int64_t* vtx_off, const int64_t* edge_off,
                             const int32_t* edges, int32_t* L, int32_t* status, uint32_t reps,
                             cc_batch_tune_result* out, void* stream) {
    if (!out) return fail(CC_EINVAL, "out is NULL");
    std::memset(out, 0, sizeof(*out));
    if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
    if (G == 0) return fail(CC_EINVAL, "G must be > 0");
    if (reps > 1000) return fail(CC_EINVAL, "reps above 1000");
    std::vector<GraphDesc> descs;
    int rc = batch_args(ctx, G, vtx_off, edge_off, edges, L, status, stream, &descs);
    if (rc) return rc;
    return tuner_tune(&ctx->tuner, &ctx->slot, G, descs.data(), reps, (hipStream_t)stream, out);
}
