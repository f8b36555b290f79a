// cc_batch.hip — many graphs in one persistent launch.
//
// Each workgroup takes whole graphs from a largest-first work list (one atomic
// ticket per graph) and runs Algorithm 1 for that graph on its own: init, one
// pass of hooking over the graph's entries, pointer jumping, separated by
// workgroup barriers, so the launch needs no grid-wide synchronisation. A graph
// whose parent array fits the workgroup's LDS is solved there (LDS
// compare-and-swap; labels go to HBM once, coalesced); a larger graph keeps its
// parent array in its label slice in HBM.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "cc_internal.h"

namespace ccm {

typedef int32_t i32x2 __attribute__((ext_vector_type(2)));

constexpr int kBatchBlock = 1024;
constexpr size_t kTicketBytes = 256;

// Root of x with path splitting (each visited vertex takes its grandparent).
__device__ __forceinline__ uint32_t bfind(uint32_t* P, uint32_t x, uint32_t px) {
    while (px != x) {
        const uint32_t gp = P[px];
        if (gp == px) return px;
        P[x] = gp;
        x = px;
        px = gp;
    }
    return x;
}

// Algorithm 1 hooking of one entry on parent array P (LDS or HBM): the root of
// greater ID is linked under the smaller; a failed CAS resumes from the value
// it returns.
__device__ __forceinline__ void blink(uint32_t* P, uint32_t u, uint32_t v) {
    uint32_t pu = P[u], pv = P[v];
    if (pu == pv || pu == v || pv == u) return;
    while (true) {
        const uint32_t ru = bfind(P, u, pu);
        const uint32_t rv = bfind(P, v, pv);
        if (ru == rv) return;
        const uint32_t hi = ru < rv ? rv : ru;
        const uint32_t lo = ru < rv ? ru : rv;
        const uint32_t old = atomicCAS(&P[hi], hi, lo);
        if (old == hi) return;
        u = hi; pu = old;
        v = lo; pv = lo;
    }
}

__device__ __forceinline__ void solve_graph(uint32_t* P, uint32_t n, const i32x2* E, int64_t m,
                                            uint32_t* out, int* bad_flag) {
    const int tid = threadIdx.x;
    for (uint32_t v = tid; v < n; v += kBatchBlock) P[v] = v;
    __syncthreads();
    bool bad = false;
    for (int64_t e = tid; e < m; e += kBatchBlock) {
        const i32x2 uv = __builtin_nontemporal_load(E + e);
        const uint32_t u = (uint32_t)uv.x, v = (uint32_t)uv.y;
        if (u >= n || v >= n) { bad = true; continue; }
        if (u != v) blink(P, u, v);
    }
    if (bad) *bad_flag = 1;
    __syncthreads();
    for (uint32_t v = tid; v < n; v += kBatchBlock) {
        uint32_t r = P[v];
        uint32_t q = P[r];
        while (q != r) { r = q; q = P[r]; }
        if (out) out[v] = r;
        else P[v] = r;
    }
}

__global__ __launch_bounds__(kBatchBlock) void k_batch(uint32_t G, const GraphDesc* __restrict__ descs,
                                                       const uint32_t* __restrict__ order,
                                                       uint32_t* ticket, uint32_t lds_cap) {
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
        const i32x2* E = reinterpret_cast<const i32x2*>(d.edges);
        uint32_t* Lg = reinterpret_cast<uint32_t*>(d.L);
        if (d.n <= lds_cap) solve_graph(sP, d.n, E, d.m, Lg, &s_bad);
        else solve_graph(Lg, d.n, E, d.m, nullptr, &s_bad);
        __syncthreads();
        if (threadIdx.x == 0) *d.status = s_bad ? CC_ERANGE : CC_OK;
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

static int lds_capacity(int device, size_t* bytes, uint32_t* entries) {
    int max_lds = 0;
    CCM_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    size_t b = (size_t)max_lds > 1024 ? (size_t)max_lds - 1024 : 0;   // static words beside
    b &= ~(size_t)255;
    *bytes = b;
    *entries = (uint32_t)(b / sizeof(uint32_t));
    return CC_OK;
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
        uint64_t cap = std::max<uint64_t>(G, 1024);
        if (hipMalloc(&bs.dev, batch_bytes(cap)) != hipSuccess ||
            hipHostMalloc(&bs.host, batch_bytes(cap), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            batch_scratch_free(&bs);
            return fail(CC_ENOMEM, "batch scratch allocation failed");
        }
        bs.cap = cap;
    }
    // largest-first by work (entries + vertices)
    std::vector<uint32_t> order(G);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        return descs[a].m + (int64_t)descs[a].n > descs[b].m + (int64_t)descs[b].n;
    });
    char* h = bs.host;
    std::memset(h, 0, kTicketBytes);
    uint32_t* h_order = reinterpret_cast<uint32_t*>(h + kTicketBytes);
    GraphDesc* h_desc = reinterpret_cast<GraphDesc*>(h + kTicketBytes + ((4 * (uint64_t)G + 63) & ~63ull));
    std::copy(order.begin(), order.end(), h_order);
    std::copy(descs, descs + G, h_desc);
    const size_t bytes = batch_bytes(G);
    CCM_HIP(hipMemcpyAsync(bs.dev, h, bytes, hipMemcpyHostToDevice, stream));
    size_t lds_bytes = 0;
    uint32_t lds_cap = 0;
    int rc = lds_capacity(s->device, &lds_bytes, &lds_cap);
    if (rc) return rc;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    (void)hipGetLastError();
    const int cus = device_cu_count(s->device);
    const uint32_t grid = (uint32_t)std::min<int64_t>((int64_t)cus, (int64_t)G);
    char* d = bs.dev;
    rc = cohere(stream);
    if (rc) return rc;
    k_batch<<<grid, kBatchBlock, lds_bytes, stream>>>(
        G, reinterpret_cast<const GraphDesc*>(d + ((char*)h_desc - h)),
        reinterpret_cast<const uint32_t*>(d + kTicketBytes), reinterpret_cast<uint32_t*>(d), lds_cap);
    CCM_HIP(hipGetLastError());
    return cohere(stream);
}

int run_batch(Slot* s, uint32_t G, const int64_t* vtx_off, const int64_t* edge_off,
              const int32_t* edges, int32_t* L, int32_t* status, hipStream_t stream) {
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
    std::vector<GraphDesc> descs(G);
    for (uint32_t g = 0; g < G; ++g) {
        descs[g].edges = edges + 2 * eo[g];
        descs[g].L = L + vo[g];
        descs[g].status = status + g;
        descs[g].n = (uint32_t)(vo[g + 1] - vo[g]);
        descs[g].pad = 0;
        descs[g].m = eo[g + 1] - eo[g];
    }
    int rc = launch_batch(s, G, descs.data(), stream);
    if (rc) return rc;
    CCM_HIP(hipStreamSynchronize(stream));
    return CC_OK;
}

}  // namespace ccm
