// cc_batch.hip — many graphs in one persistent launch.
//
// Each workgroup takes whole graphs from a largest-first work list (one atomic
// ticket per graph) and runs Algorithm 1 for that graph on its own: init, one
// pass of hooking over the graph's entries, pointer jumping, separated by
// workgroup barriers, so the launch needs no grid-wide synchronisation. A graph
// of at most 2^16 vertices keeps its parent array in the workgroup's LDS as
// 16-bit entries (128 KB at n = 2^16; a link is a compare-and-swap on the
// 32-bit word holding the entry); labels go to HBM once, coalesced. A larger
// graph keeps its parent array in its label slice in HBM. Every thread keeps
// kBatchEPT edge loads in flight.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "cc_internal.h"

namespace ccm {

typedef int32_t i32x2 __attribute__((ext_vector_type(2)));
// Pointers read from the descriptors are generic; marking them global keeps the
// compiler from emitting flat accesses, which also count as LDS operations and
// would make every LDS wait also wait for the edge loads in flight.
#define CCM_GLOBAL __attribute__((address_space(1)))
typedef const CCM_GLOBAL i32x2 gedge_t;
typedef CCM_GLOBAL uint32_t glabel_t;

constexpr int kBatchBlock = 1024;
constexpr size_t kTicketBytes = 256;

constexpr int kBatchEPT = 8;

// Agent-scope store to a global word (see the store rule in cc_kernels.hip).
__device__ __forceinline__ void gstore(glabel_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}


// ---- 16-bit parent array in LDS (n <= 2^16) ------------------------------------------

__device__ __forceinline__ uint32_t bfind16(uint16_t* P, uint32_t x, uint32_t px) {
    while (px != x) {
        const uint32_t gp = P[px];
        if (gp == px) return px;
        stress_delay(x);
        P[x] = (uint16_t)gp;
        x = px;
        px = gp;
    }
    return x;
}

// CAS of the 16-bit entry hi from hi (a root) to lo, on the 32-bit word that
// holds it; a change of the other half only makes the word CAS retry. Returns
// hi on success, else the entry's current (non-root) value.
__device__ __forceinline__ uint32_t cas16(uint32_t* P32, uint32_t hi, uint32_t lo) {
    uint32_t* w = &P32[hi >> 1];
    const uint32_t sh = (hi & 1u) << 4;
    uint32_t cur = *w;
    while (true) {
        const uint32_t h = (cur >> sh) & 0xFFFFu;
        if (h != hi) return h;
        const uint32_t des = (cur & ~(0xFFFFu << sh)) | (lo << sh);
        const uint32_t prev = atomicCAS(w, cur, des);
        if (prev == cur) return hi;
        cur = prev;
    }
}

// Hooking of one entry whose endpoints u, v have parents pu, pv (read earlier).
__device__ __forceinline__ void blink16(uint16_t* P, uint32_t* P32, uint32_t u, uint32_t pu,
                                        uint32_t v, uint32_t pv) {
    if (pu == pv || pu == v || pv == u) return;
    while (true) {
        const uint32_t ru = bfind16(P, u, pu);
        const uint32_t rv = bfind16(P, v, pv);
        if (ru == rv) return;
        const uint32_t hi = ru < rv ? rv : ru;
        const uint32_t lo = ru < rv ? ru : rv;
        stress_delay(hi);
        const uint32_t old = cas16(P32, hi, lo);
        if (old == hi) return;
        u = hi; pu = old;
        v = lo; pv = lo;
    }
}

__device__ __forceinline__ void solve_graph16(uint32_t* P32, uint32_t n, gedge_t* E, int64_t m,
                                              glabel_t* out, int* bad_flag) {
    const int tid = threadIdx.x;
    uint16_t* P = reinterpret_cast<uint16_t*>(P32);
    for (uint32_t i = tid; 2 * i < n; i += kBatchBlock) P32[i] = (2 * i) | ((2 * i + 1) << 16);
    __syncthreads();
    bool bad = false;
    // Software pipeline over rounds of kBatchEPT entries per thread: register k
    // is reloaded with entry k of the next round right after entry k is linked,
    // so the next round's loads are in flight while this round is processed.
    constexpr int64_t kRound = (int64_t)kBatchBlock * kBatchEPT;
    // A graph without entries issues no edge load at all: its entry pointer may
    // be NULL (an edge-free batch) or point one past the batch's last entry.
    i32x2 x[kBatchEPT];
#pragma unroll
    for (int k = 0; k < kBatchEPT; ++k) {
        const int64_t e = tid + (int64_t)k * kBatchBlock;
        x[k] = i32x2{0, 0};
        if (m > 0) x[k] = __builtin_nontemporal_load(E + (e < m ? e : 0));
    }
    for (int64_t e0 = tid; e0 < m; e0 += kRound) {
        // every entry's two parent reads first (LDS latency overlaps), then the links
        uint32_t pu[kBatchEPT], pv[kBatchEPT];
        bool live[kBatchEPT];
#pragma unroll
        for (int k = 0; k < kBatchEPT; ++k) {
            const uint32_t u = (uint32_t)x[k].x, v = (uint32_t)x[k].y;
            const bool in = e0 + (int64_t)k * kBatchBlock < m;
            const bool ok = u < n && v < n;
            bad |= in && !ok;
            live[k] = in && ok && u != v;
            pu[k] = live[k] ? P[u] : 0u;
            pv[k] = live[k] ? P[v] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kBatchEPT; ++k) {
            if (live[k]) blink16(P, P32, (uint32_t)x[k].x, pu[k], (uint32_t)x[k].y, pv[k]);
            const int64_t e = e0 + kRound + (int64_t)k * kBatchBlock;
            x[k] = __builtin_nontemporal_load(E + (e < m ? e : 0));
        }
    }
    if (bad) *bad_flag = 1;
    __syncthreads();
    for (uint32_t v = tid; v < n; v += kBatchBlock) {
        uint32_t r = P[v];
        uint32_t q = P[r];
        while (q != r) { r = q; q = P[r]; }
        gstore(&out[v], r);
    }
}

// ---- 32-bit parent array in the label slice (HBM) --------------------------------------

// Root of x with path splitting (each visited vertex takes its grandparent).
__device__ __forceinline__ uint32_t bfind(glabel_t* P, uint32_t x, uint32_t px) {
    while (px != x) {
        const uint32_t gp = P[px];
        if (gp == px) return px;
        stress_delay(x);
        gstore(&P[x], gp);
        x = px;
        px = gp;
    }
    return x;
}

// Algorithm 1 hooking of one entry: the root of greater ID is linked under the
// smaller; a failed CAS resumes from the value it returns.
__device__ __forceinline__ void blink(glabel_t* P, uint32_t u, uint32_t v) {
    uint32_t pu = P[u], pv = P[v];
    if (pu == pv || pu == v || pv == u) return;
    while (true) {
        const uint32_t ru = bfind(P, u, pu);
        const uint32_t rv = bfind(P, v, pv);
        if (ru == rv) return;
        const uint32_t hi = ru < rv ? rv : ru;
        const uint32_t lo = ru < rv ? ru : rv;
        uint32_t old = hi;
        stress_delay(hi);
        if (__hip_atomic_compare_exchange_strong(&P[hi], &old, lo, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return;
        u = hi; pu = old;
        v = lo; pv = lo;
    }
}

__device__ __forceinline__ void solve_graph_hbm(glabel_t* P, uint32_t n, gedge_t* E, int64_t m,
                                                int* bad_flag) {
    const int tid = threadIdx.x;
    for (uint32_t v = tid; v < n; v += kBatchBlock) gstore(&P[v], v);
    __threadfence_block();
    __syncthreads();
    bool bad = false;
    for (int64_t e0 = tid; e0 < m; e0 += (int64_t)kBatchBlock * kBatchEPT) {
        i32x2 x[kBatchEPT];
#pragma unroll
        for (int k = 0; k < kBatchEPT; ++k) {
            const int64_t e = e0 + (int64_t)k * kBatchBlock;
            x[k] = __builtin_nontemporal_load(E + (e < m ? e : 0));
        }
#pragma unroll
        for (int k = 0; k < kBatchEPT; ++k) {
            if (e0 + (int64_t)k * kBatchBlock >= m) continue;
            const uint32_t u = (uint32_t)x[k].x, v = (uint32_t)x[k].y;
            if (u >= n || v >= n) { bad = true; continue; }
            if (u != v) blink(P, u, v);
        }
    }
    if (bad) *bad_flag = 1;
    __threadfence_block();
    __syncthreads();
    for (uint32_t v = tid; v < n; v += kBatchBlock) {
        uint32_t r = P[v];
        uint32_t q = P[r];
        while (q != r) { r = q; q = P[r]; }
        gstore(&P[v], r);
    }
}

__global__ __launch_bounds__(kBatchBlock) void k_batch(uint32_t G, const GraphDesc* __restrict__ descs,
                                                       const uint32_t* __restrict__ order,
                                                       uint32_t* ticket, uint32_t lds16_cap) {
    extern __shared__ uint32_t sP[];
    __shared__ uint32_t s_next;
    __shared__ int s_bad;
    while (true) {
        if (threadIdx.x == 0) {
            s_next = atomicAdd(ticket, 1u);
            s_bad = 0;
        }
        __syncthreads();
        const uint32_t t = s_next;
        if (t >= G) break;
        const GraphDesc d = descs[order[t]];
        gedge_t* E = (gedge_t*)d.edges;
        if (d.n <= lds16_cap) solve_graph16(sP, d.n, E, d.m, (glabel_t*)d.L, &s_bad);
        else solve_graph_hbm((glabel_t*)d.L, d.n, E, d.m, &s_bad);
        __syncthreads();
        if (threadIdx.x == 0) *(CCM_GLOBAL int32_t*)d.status = s_bad ? CC_ERANGE : CC_OK;
        __syncthreads();
    }
}

void batch_scratch_free(BatchScratch* b) {
    if (b->dev) (void)hipFree(b->dev);
    if (b->host) (void)hipHostFree(b->host);
    *b = BatchScratch{};
}

static size_t batch_bytes(uint64_t G) {
    return kTicketBytes + ((4 * G + 63) & ~63ull) + sizeof(GraphDesc) * G;
}

// Dynamic LDS for the 16-bit parent array: 2^16 entries (128 KB), or what the
// device allows beside the static words; graphs above that size use HBM.
static int lds_capacity(int device, size_t* bytes, uint32_t* entries16) {
    int max_lds = 0;
    CCM_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    size_t b = (size_t)max_lds > 1024 ? (size_t)max_lds - 1024 : 0;   // static words beside
    b = std::min<size_t>(b, (size_t)1 << 17);
    b &= ~(size_t)255;
    *bytes = b;
    *entries16 = (uint32_t)std::min<size_t>(b / sizeof(uint16_t), (size_t)1 << 16);
    return CC_OK;
}

static int batch_alloc(BatchScratch* bs, uint64_t G) {
    uint64_t cap = std::max<uint64_t>(G, 1024);
    if (hipMalloc(&bs->dev, batch_bytes(cap)) != hipSuccess ||
        hipHostMalloc(&bs->host, batch_bytes(cap), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        batch_scratch_free(bs);
        return fail(CC_ENOMEM, "batch scratch allocation failed");
    }
    bs->cap = cap;
    return CC_OK;
}

// Host staging of one launch: the zeroed ticket, the largest-first order (by
// entries + vertices) and the descriptors, in the device layout.
static void batch_prepare(BatchScratch* bs, uint32_t G, const GraphDesc* descs) {
    std::vector<uint32_t> order(G);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        return descs[a].m + (int64_t)descs[a].n > descs[b].m + (int64_t)descs[b].n;
    });
    char* h = bs->host;
    std::memset(h, 0, kTicketBytes);
    uint32_t* h_order = reinterpret_cast<uint32_t*>(h + kTicketBytes);
    GraphDesc* h_desc = reinterpret_cast<GraphDesc*>(h + kTicketBytes + ((4 * (uint64_t)G + 63) & ~63ull));
    std::copy(order.begin(), order.end(), h_order);
    std::copy(descs, descs + G, h_desc);
}

// The device part of one launch: upload of the staging (which also zeroes the
// ticket, so a captured copy of this sequence replays correctly), the
// persistent kernel, and the coherence points around it. Only stream work: it
// can be captured into a graph.
static int batch_enqueue(int device, BatchScratch* bs, uint32_t G, hipStream_t stream) {
    const size_t bytes = batch_bytes(G);
    CCM_HIP(hipMemcpyAsync(bs->dev, bs->host, bytes, hipMemcpyHostToDevice, stream));
    size_t lds_bytes = 0;
    uint32_t lds_cap = 0;
    int rc = lds_capacity(device, &lds_bytes, &lds_cap);
    if (rc) return rc;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    (void)hipGetLastError();
    const int cus = device_cu_count(device);
    const uint32_t grid = (uint32_t)std::min<int64_t>((int64_t)cus, (int64_t)G);
    char* d = bs->dev;
    const uint64_t desc_off = kTicketBytes + ((4 * (uint64_t)G + 63) & ~63ull);
    rc = cohere(stream);
    if (rc) return rc;
    k_batch<<<grid, kBatchBlock, lds_bytes, stream>>>(
        G, reinterpret_cast<const GraphDesc*>(d + desc_off),
        reinterpret_cast<const uint32_t*>(d + kTicketBytes), reinterpret_cast<uint32_t*>(d), lds_cap);
    CCM_HIP(hipGetLastError());
    return cohere(stream);
}

int batch_reserve(Slot* s, uint32_t G) {
    BatchScratch& bs = s->batch;
    if (bs.cap >= G) return CC_OK;
    batch_scratch_free(&bs);
    return batch_alloc(&bs, G);
}

// The host staging is reused per call: the caller waits for the previous launch
// on this slot (its upload) before the next one.
int launch_batch(Slot* s, uint32_t G, const GraphDesc* descs, hipStream_t stream) {
    if (G == 0) return CC_OK;
    BatchScratch& bs = s->batch;
    if (bs.cap < G) {
        // the previous launch on this slot must be done with the staging
        CCM_HIP(hipStreamSynchronize(stream));
        batch_scratch_free(&bs);
        int rc = batch_alloc(&bs, G);
        if (rc) return rc;
    }
    batch_prepare(&bs, G, descs);
    return batch_enqueue(s->device, &bs, G, stream);
}

// Offsets read back and checked, descriptors built (cc_batch's arguments).
static int batch_descs(uint32_t G, const int64_t* vtx_off, const int64_t* edge_off,
                       const int32_t* edges, int32_t* L, int32_t* status, hipStream_t stream,
                       std::vector<GraphDesc>* out) {
    std::vector<int64_t> vo(G + 1), eo(G + 1);
    CCM_HIP(hipMemcpyAsync(vo.data(), vtx_off, (G + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    CCM_HIP(hipMemcpyAsync(eo.data(), edge_off, (G + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    CCM_HIP(hipStreamSynchronize(stream));
    if (vo[0] != 0 || eo[0] != 0) return fail(CC_EINVAL, "offsets must start at 0");
    for (uint32_t g = 0; g < G; ++g) {
        if (vo[g + 1] < vo[g] || eo[g + 1] < eo[g]) return fail(CC_EINVAL, "offsets must be non-decreasing");
        if (vo[g + 1] - vo[g] >= (1ll << 31)) return fail(CC_EINVAL, "graph too large for int32 IDs");
    }
    if (eo[G] && !edges) return fail(CC_EINVAL, "edges is NULL");
    if (vo[G] && !L) return fail(CC_EINVAL, "L is NULL");
    out->resize(G);
    for (uint32_t g = 0; g < G; ++g) {
        GraphDesc& d = (*out)[g];
        d.edges = edges + 2 * eo[g];
        d.L = L + vo[g];
        d.status = status + g;
        d.n = (uint32_t)(vo[g + 1] - vo[g]);
        d.pad = 0;
        d.m = eo[g + 1] - eo[g];
    }
    return CC_OK;
}

// A captured batch: its own staging and device copy of the work list (so later
// cc_batch calls on the context cannot change what a replay uploads), and the
// instantiated graph of batch_enqueue.
struct BatchGraph {
    int device = 0;
    BatchScratch bs;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

int batch_graph_create(Slot* s, uint32_t G, const int64_t* vtx_off, const int64_t* edge_off,
                       const int32_t* edges, int32_t* L, int32_t* status, hipStream_t stream,
                       void** out) {
    *out = nullptr;
    std::vector<GraphDesc> descs;
    int rc = batch_descs(G, vtx_off, edge_off, edges, L, status, stream, &descs);
    if (rc) return rc;
    BatchGraph* bg = new BatchGraph;
    bg->device = s->device;
    if ((rc = batch_alloc(&bg->bs, G))) {
        delete bg;
        return rc;
    }
    batch_prepare(&bg->bs, G, descs.data());
    // capture on a private stream of default priority (the null stream cannot be
    // captured); nothing else runs on it
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        batch_scratch_free(&bg->bs);
        delete bg;
        return fail(CC_EDEVICE, "capture stream creation failed");
    }
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        rc = batch_enqueue(bg->device, &bg->bs, G, cs);
        hipGraph_t gr = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &gr);
        bg->graph = gr;
        if (!rc && e2 != hipSuccess) rc = hip_fail(e2, "hipStreamEndCapture");
        if (!rc && hipGraphInstantiate(&bg->exec, bg->graph, nullptr, nullptr, 0) != hipSuccess)
            rc = fail(CC_EDEVICE, "graph instantiation failed");
    } else {
        rc = hip_fail(e, "hipStreamBeginCapture");
    }
    (void)hipStreamDestroy(cs);
    if (rc) {
        (void)hipGetLastError();
        batch_graph_destroy(bg);
        return rc;
    }
    *out = bg;
    return CC_OK;
}

int batch_graph_launch(void* h, hipStream_t stream) {
    BatchGraph* bg = static_cast<BatchGraph*>(h);
    CCM_HIP(hipSetDevice(bg->device));
    CCM_HIP(hipGraphLaunch(bg->exec, stream));
    return CC_OK;
}

void batch_graph_destroy(void* h) {
    BatchGraph* bg = static_cast<BatchGraph*>(h);
    if (!bg) return;
    (void)hipSetDevice(bg->device);
    if (bg->exec) (void)hipGraphExecDestroy(bg->exec);
    if (bg->graph) (void)hipGraphDestroy(bg->graph);
    batch_scratch_free(&bg->bs);
    delete bg;
}

int run_batch(Slot* s, uint32_t G, const int64_t* vtx_off, const int64_t* edge_off,
              const int32_t* edges, int32_t* L, int32_t* status, hipStream_t stream) {
    std::vector<GraphDesc> descs;
    int rc = batch_descs(G, vtx_off, edge_off, edges, L, status, stream, &descs);
    if (rc) return rc;
    if ((rc = launch_batch(s, G, descs.data(), stream))) return rc;
    CCM_HIP(hipStreamSynchronize(stream));
    return CC_OK;
}

}  // namespace ccm
