// cc_wide.hip — the plain path with 64-bit vertex IDs.
//
// Sec. V keeps 4-byte IDs below 2^32 vertices and 8-byte IDs beyond. This file
// is the 8-byte form of Algorithm 1: P holds uint64 parents, links are 64-bit
// CAS on a root's own entry, the finds split paths, and compress is the same
// pointer jumping. The rules of the 32-bit kernels carry over unchanged: every
// store to P is a device-coherent store (another XCD's L2 must not keep an old
// copy), and compress reads the two values the label rests on coherently.
#include "cc_internal.h"

namespace ccm {

typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

constexpr int kWBlock = 256;
constexpr int kWEPT = 4;            // entries per thread per tile

__device__ __forceinline__ uint64_t ld_agent_w(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent_w(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kWBlock) void k_init_w(uint64_t* __restrict__ P, uint64_t n) {
    for (uint64_t v = (uint64_t)blockIdx.x * kWBlock + threadIdx.x; v < n;
         v += (uint64_t)gridDim.x * kWBlock)
        st_agent_w(&P[v], v);
}

// Root of x; SPLIT: path splitting with device-coherent stores (the rule of
// cc_kernels.hip's find_root).
template <int SPLIT>
__device__ __forceinline__ uint64_t find_w(uint64_t* P, uint64_t x, uint64_t px) {
    if (px == x) return x;
    uint64_t gp = P[px];
    while (gp != px) {
        const uint64_t ggp = P[gp];
        if (SPLIT) {
            stress_delay((uint32_t)x);
            st_agent_w(&P[x], gp);
        }
        x = px;
        px = gp;
        gp = ggp;
    }
    return px;
}

// One tile of kWBlock * kWEPT entries per workgroup, non-temporal 16-byte
// loads; all parent reads of a thread are issued before any walk.
template <int SPLIT>
__global__ __launch_bounds__(kWBlock) void k_hook_w(const uint64_t* __restrict__ edges, uint64_t m,
                                                    uint64_t n, uint64_t* P, DevState* st,
                                                    uint32_t sym) {
    const uint64_t tile = (uint64_t)blockIdx.x * (kWBlock * kWEPT);
    const u64x2* E = reinterpret_cast<const u64x2*>(edges);
    uint64_t u[kWEPT], v[kWEPT];
#pragma unroll
    for (int k = 0; k < kWEPT; ++k) {
        const uint64_t e = tile + (uint64_t)k * kWBlock + threadIdx.x;
        u64x2 uv = {0ull, 0ull};
        if (e < m) uv = __builtin_nontemporal_load(E + e);
        u[k] = uv.x;
        v[k] = uv.y;
    }
    bool bad = false;
#pragma unroll
    for (int k = 0; k < kWEPT; ++k)
        if (u[k] >= n || v[k] >= n) { bad = true; u[k] = v[k] = 0; }
    if (bad) atomicOr(&st->status, kStatusRange);
    // a list with every pair in both orders: hook each edge once, as u < v
    if (sym) {
#pragma unroll
        for (int k = 0; k < kWEPT; ++k)
            if (v[k] < u[k]) v[k] = u[k];
    }
    uint64_t pu[kWEPT], pv[kWEPT];
#pragma unroll
    for (int k = 0; k < kWEPT; ++k) {
        pu[k] = u[k] != v[k] ? P[u[k]] : 0ull;
        pv[k] = u[k] != v[k] ? P[v[k]] : 0ull;
    }
#pragma unroll
    for (int k = 0; k < kWEPT; ++k) {
        if (u[k] == v[k]) continue;
        uint64_t a = u[k], pa = pu[k], b = v[k], pb = pv[k];
        if (pa == pb || pa == b || pb == a) continue;     // same tree already
        while (true) {
            const uint64_t ra = find_w<SPLIT>(P, a, pa);
            const uint64_t rb = find_w<SPLIT>(P, b, pb);
            if (ra == rb) break;
            const uint64_t hi = ra < rb ? rb : ra;
            const uint64_t lo = ra < rb ? ra : rb;
            stress_delay((uint32_t)hi);
            // a coherent read before the CAS, as in cc_kernels.hip's link
            const uint64_t cur = __hip_atomic_load(&P[hi], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (cur != hi) {
                a = hi; pa = cur;
                b = lo; pb = lo;
                continue;
            }
            const uint64_t old = atomicCAS((unsigned long long*)&P[hi], (unsigned long long)hi,
                                           (unsigned long long)lo);
            if (old == hi) break;
            a = hi; pa = old;             // hi was linked meanwhile: continue from its parent
            b = lo; pb = lo;
        }
    }
}

__global__ __launch_bounds__(kWBlock) void k_compress_w(uint64_t* P, uint64_t n) {
    for (uint64_t v = (uint64_t)blockIdx.x * kWBlock + threadIdx.x; v < n;
         v += (uint64_t)gridDim.x * kWBlock) {
        const uint64_t p = ld_agent_w(&P[v]);
        if (p == v) continue;
        uint64_t r = p;
        while (true) {
            uint64_t q = P[r];
            while (q != r) { r = q; q = P[r]; }
            q = ld_agent_w(&P[r]);          // a stale "root" would end the walk early
            if (q == r) break;
            r = q;
        }
        if (r != p) st_agent_w(&P[v], r);
    }
}

int run_solve_w(Slot* s, uint64_t n, uint64_t m, const uint64_t* edges, uint64_t* L,
                uint32_t flags, hipStream_t stream) {
    if (n == 0) return CC_OK;
    if (flags & ~(uint32_t)(CC_F_NO_SPLIT | CC_F_SYMMETRIC))
        return fail(CC_EINVAL,
                    "64-bit IDs take the plain path only (flags: CC_F_NO_SPLIT, CC_F_SYMMETRIC)");
    const uint32_t sym = (flags & CC_F_SYMMETRIC) ? 1u : 0u;
    const uint64_t per = (uint64_t)kWBlock * kWEPT;
    const uint64_t tiles = (m + per - 1) / per;
    if (tiles > 0x7FFFFFFFull) return fail(CC_EINVAL, "entry count too large for one launch");
    uint64_t g = (n + kWBlock - 1) / kWBlock;
    const uint32_t gn = (uint32_t)(g < kGridCap ? g : kGridCap);
    int rc;
    k_init_w<<<gn, kWBlock, 0, stream>>>(L, n);
    CCM_HIP(hipGetLastError());
    if ((rc = cohere(stream))) return rc;
    if (tiles) {
        if (!split_walks(flags, n, sizeof(uint64_t)))
            k_hook_w<0><<<(uint32_t)tiles, kWBlock, 0, stream>>>(edges, m, n, L, s->st, sym);
        else
            k_hook_w<1><<<(uint32_t)tiles, kWBlock, 0, stream>>>(edges, m, n, L, s->st, sym);
        CCM_HIP(hipGetLastError());
    }
    if ((rc = cohere(stream))) return rc;
    k_compress_w<<<gn, kWBlock, 0, stream>>>(L, n);
    CCM_HIP(hipGetLastError());
    return cohere(stream);
}

}  // namespace ccm
