// cc_batch.hip — many graphs in one batch: three roles, one enqueue.
//
// Every graph runs Algorithm 1 on its own (init, one pass of hooking over its
// entries with path splitting, pointer jumping); what differs is how much of
// the device one graph gets (the schedule, cc_batch_sched):
//  - tile: one workgroup takes whole graphs from a largest-first work list (one
//    atomic ticket per graph), its steps separated by workgroup barriers, so
//    the launch needs no grid-wide synchronisation. A graph of at most 2^16
//    vertices keeps its parent array in the workgroup's LDS (32-bit entries up
//    to 2^15 vertices, else 16-bit entries: 128 KB at n = 2^16, a link being a
//    compare-and-swap on the 32-bit word holding the entry); labels go to HBM
//    once, coalesced. A larger graph keeps its parent array in its label slice
//    in HBM.
//  - wave: one wavefront takes a small graph from a second work list and solves
//    it in an 8 KB partition of the workgroup's LDS, its steps separated by
//    wavefront-level ordering only; 16 graphs per workgroup run at once. The
//    persistent kernel runs the tile list first, then the wave list.
//  - multi: a large graph is solved by the whole device before the persistent
//    kernel: three launches (init, hook, compress) cover all such graphs of the
//    batch, each block taking a chunk of one graph's vertices or entries from a
//    host-built chunk table; the parent array is the label slice in HBM.
// Every thread keeps two rounds of edge loads in flight.
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
constexpr int kWaves = kBatchBlock / 64;
constexpr size_t kTicketBytes = 256;
constexpr int kTileTicket = 0;     // word of the tile list's ticket
constexpr int kWaveTicket = 16;    // the wave list's, on its own 64-byte line

constexpr int kBatchEPT = 8;     // entries per thread and round on the HBM paths
constexpr int kLdsEPT = 4;       // the same with the parent array in LDS
constexpr int kLinkQueue = 127;  // per-wave LDS slots of entries that need a walk

// Agent-scope store to a global word (see the store rule in cc_kernels.hip).
__device__ __forceinline__ void gstore(glabel_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t gload_agent(glabel_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The lanes of one wavefront execute together and its LDS operations complete
// in issue order; this keeps the compiler from moving LDS accesses across the
// point, so what one lane wrote before it is what another lane reads after it.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- parent array in LDS: 32-bit entries up to half the capacity, else 16-bit --------
// A graph of at most 2^15 vertices keeps 32-bit entries (a link is one CAS on
// the entry); up to 2^16 vertices the entries are 16-bit and a link is a CAS on
// the 32-bit word holding the entry (4,096-graph batch: 1.55 ms against 1.64 ms
// with 16-bit entries throughout).

template <typename PT>
__device__ __forceinline__ uint32_t lfind(PT* P, uint32_t x, uint32_t px) {
    while (px != x) {
        const uint32_t gp = P[px];
        if (gp == px) return px;
        stress_delay(x);
        P[x] = (PT)gp;
        x = px;
        px = gp;
    }
    return x;
}

// CAS of the entry hi from hi (a root) to lo. Returns hi on success, else the
// entry's current (non-root) value. 16-bit entries: the CAS is on the 32-bit
// word that holds the entry; a change of the other half only makes it retry.
template <typename PT>
__device__ __forceinline__ uint32_t lcas(PT* P, uint32_t hi, uint32_t lo) {
    if (sizeof(PT) == 4) return atomicCAS(reinterpret_cast<uint32_t*>(&P[hi]), hi, lo);
    uint32_t* w = reinterpret_cast<uint32_t*>(P) + (hi >> 1);
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
template <typename PT>
__device__ __forceinline__ void llink(PT* P, uint32_t u, uint32_t pu, uint32_t v, uint32_t pv) {
    if (pu == pv || pu == v || pv == u) return;
    while (true) {
        const uint32_t ru = lfind(P, u, pu);
        const uint32_t rv = lfind(P, v, pv);
        if (ru == rv) return;
        const uint32_t hi = ru < rv ? rv : ru;
        const uint32_t lo = ru < rv ? ru : rv;
        stress_delay(hi);
        const uint32_t old = lcas(P, hi, lo);
        if (old == hi) return;
        u = hi; pu = old;
        v = lo; pv = lo;
    }
}

// One graph with its parent array in LDS (entries of type PT), by a group of T
// threads (T = 64: one wavefront; T = kBatchBlock: the workgroup); idx is the
// thread's index in the group. Returns whether this thread saw an endpoint out
// of range.
template <int T, typename PT>
__device__ __forceinline__ bool solve_graph_lds(uint32_t* S, uint32_t n, gedge_t* E, int64_t m,
                                                glabel_t* out, int idx, uint2* q) {
    auto sync = [] {
        if (T == 64) wave_sync();
        else __syncthreads();
    };
    PT* P = reinterpret_cast<PT*>(S);
    if (sizeof(PT) == 4) {
        for (uint32_t i = idx; i < n; i += T) S[i] = i;
    } else {
        for (uint32_t i = idx; 2 * i < n; i += T) S[i] = (2 * i) | ((2 * i + 1) << 16);
    }
    sync();
    bool bad = false;
    // Two rounds of kLdsEPT entries per thread in flight: A holds round r and
    // B round r + 1; right after an entry of a round is tested, its register is
    // reloaded with that entry's place two rounds on. A graph without entries
    // issues no edge load at all: its entry pointer may be NULL (an edge-free
    // batch) or point one past the batch's last entry.
    //
    // An entry whose endpoints' parents already show them joined (a common
    // parent, or one endpoint the other's parent) is done. The others need
    // walks and a link, of very different lengths from lane to lane; linked in
    // place they would leave most of the wave idle while its longest walk
    // runs. They go to the wave's queue q (kLinkQueue slots: endpoints and the
    // parents read for them, 16 bits each, as n <= 2^16 here), and whenever 64
    // are queued the wave links them together, one per lane (4,096-graph
    // batch: 1.55 -> 1.28 ms). The parents read may have changed meanwhile;
    // they are still ancestors, which is all a walk needs.
    constexpr int64_t kRound = (int64_t)T * kLdsEPT;
    const int lane = idx & 63;
    uint32_t qn = 0;                 // queued entries: the same in every lane
    i32x2 A[kLdsEPT], B[kLdsEPT];
#pragma unroll
    for (int k = 0; k < kLdsEPT; ++k) {
        const int64_t e = idx + (int64_t)k * T, f = e + kRound;
        A[k] = i32x2{0, 0};
        B[k] = i32x2{0, 0};
        if (m > 0) {
            A[k] = __builtin_nontemporal_load(E + (e < m ? e : 0));
            B[k] = __builtin_nontemporal_load(E + (f < m ? f : 0));
        }
    }
    auto round = [&](i32x2 (&x)[kLdsEPT], int64_t e0) {
        // every entry's two parent reads first (LDS latency overlaps), then the tests
        uint32_t pu[kLdsEPT], pv[kLdsEPT];
        bool live[kLdsEPT];
        const int64_t rem = m - e0;
#pragma unroll
        for (int k = 0; k < kLdsEPT; ++k) {
            const uint32_t u = (uint32_t)x[k].x, v = (uint32_t)x[k].y;
            const bool in = (int64_t)k * T < rem;
            const bool ok = u < n && v < n;
            bad |= in && !ok;
            live[k] = in && ok && u != v;
            pu[k] = live[k] ? (uint32_t)P[u] : 0u;
            pv[k] = live[k] ? (uint32_t)P[v] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kLdsEPT; ++k) {
            const uint32_t u = (uint32_t)x[k].x, v = (uint32_t)x[k].y;
            const bool walk = live[k] && !(pu[k] == pv[k] || pu[k] == v || pv[k] == u);
            const uint64_t ball = __ballot(walk);
            if (walk)
                q[qn + (uint32_t)__popcll(ball & ((1ull << lane) - 1ull))] =
                    uint2{u | (v << 16), pu[k] | (pv[k] << 16)};
            qn += (uint32_t)__popcll(ball);
            if (qn >= 64) {
                wave_sync();
                const uint2 a = q[lane];
                llink(P, a.x & 0xFFFFu, a.y & 0xFFFFu, a.x >> 16, a.y >> 16);
                const uint2 rest = (uint32_t)lane < qn - 64 ? q[64 + lane] : uint2{0u, 0u};
                wave_sync();
                if ((uint32_t)lane < qn - 64) q[lane] = rest;
                qn -= 64;
                wave_sync();
            }
            const int64_t e = e0 + 2 * kRound + (int64_t)k * T;
            x[k] = __builtin_nontemporal_load(E + (e < m ? e : 0));
        }
    };
    // loop control from the wave's first index, so that every lane of the wave
    // runs every round (the queue's ballots and count need the whole wave)
    for (int64_t b0 = idx - lane; b0 < m; b0 += 2 * kRound) {
        round(A, b0 + lane);
        if (b0 + kRound >= m) break;
        round(B, b0 + lane + kRound);
    }
    if (qn) {
        wave_sync();
        if ((uint32_t)lane < qn) {
            const uint2 a = q[lane];
            llink(P, a.x & 0xFFFFu, a.y & 0xFFFFu, a.x >> 16, a.y >> 16);
        }
    }
    sync();
    for (uint32_t v = idx; v < n; v += T) {
        uint32_t r = P[v];
        uint32_t q = P[r];
        while (q != r) { r = q; q = P[r]; }
        gstore(&out[v], r);
    }
    return bad;
}

// ---- 32-bit parent array in the label slice (HBM) --------------------------------------

// Root of x; with split, path splitting (each visited vertex takes its
// grandparent) with device-coherent stores (the rule of cc_kernels.hip's
// find_root): the whole-device role splits where the graph's parent array
// outgrows one XCD's L2 (split_walks), the tile role always.
__device__ __forceinline__ uint32_t bfind(glabel_t* P, uint32_t x, uint32_t px, bool split) {
    while (px != x) {
        const uint32_t gp = P[px];
        if (gp == px) return px;
        stress_delay(x);
        if (split) gstore(&P[x], gp);
        x = px;
        px = gp;
    }
    return x;
}

// Algorithm 1 hooking of one entry (u, v) whose parents pu, pv were read
// earlier: the root of greater ID is linked under the smaller; a failed CAS
// resumes from the value it returns.
__device__ __forceinline__ void blink(glabel_t* P, uint32_t u, uint32_t pu, uint32_t v, uint32_t pv,
                                      bool split) {
    if (pu == pv || pu == v || pv == u) return;
    while (true) {
        const uint32_t ru = bfind(P, u, pu, split);
        const uint32_t rv = bfind(P, v, pv, split);
        if (ru == rv) return;
        const uint32_t hi = ru < rv ? rv : ru;
        const uint32_t lo = ru < rv ? ru : rv;
        stress_delay(hi);
        // a coherent read before the CAS, as in cc_kernels.hip's link
        uint32_t old = gload_agent(&P[hi]);
        if (old != hi) {
            u = hi; pu = old;
            v = lo; pv = lo;
            continue;
        }
        if (__hip_atomic_compare_exchange_strong(&P[hi], &old, lo, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return;
        u = hi; pu = old;
        v = lo; pv = lo;
    }
}

// Hooking of entries [first, end) of a graph with its parent array P in HBM, by
// T threads (idx: this thread's index) stepping T entries at a time. Each
// thread keeps kBatchEPT entries and their 2 * kBatchEPT parent reads in flight:
// the entries of the next round are loaded while this round links, and a
// round's parent reads are all issued before its first link. Returns whether
// this thread saw an endpoint out of range.
template <int T>
__device__ __forceinline__ bool hook_hbm(glabel_t* P, uint32_t n, gedge_t* E, int64_t first,
                                         int64_t end, int idx, bool split) {
    bool bad = false;
    if (first >= end) return bad;
    constexpr int64_t kRound = (int64_t)T * kBatchEPT;
    i32x2 x[kBatchEPT];
#pragma unroll
    for (int k = 0; k < kBatchEPT; ++k) {
        const int64_t e = first + idx + (int64_t)k * T;
        x[k] = __builtin_nontemporal_load(E + (e < end ? e : first));
    }
    for (int64_t e0 = first + idx; e0 < end; e0 += kRound) {
        uint32_t pu[kBatchEPT], pv[kBatchEPT];
        bool live[kBatchEPT];
#pragma unroll
        for (int k = 0; k < kBatchEPT; ++k) {
            const uint32_t u = (uint32_t)x[k].x, v = (uint32_t)x[k].y;
            const bool in = e0 + (int64_t)k * T < end;
            const bool ok = u < n && v < n;
            bad |= in && !ok;
            live[k] = in && ok && u != v;
            pu[k] = live[k] ? P[u] : 0u;
            pv[k] = live[k] ? P[v] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kBatchEPT; ++k) {
            if (live[k]) blink(P, (uint32_t)x[k].x, pu[k], (uint32_t)x[k].y, pv[k], split);
            const int64_t e = e0 + kRound + (int64_t)k * T;
            x[k] = __builtin_nontemporal_load(E + (e < end ? e : first));
        }
    }
    return bad;
}

__device__ __forceinline__ void solve_graph_hbm(glabel_t* P, uint32_t n, gedge_t* E, int64_t m,
                                                int* bad_flag) {
    const int tid = threadIdx.x;
    for (uint32_t v = tid; v < n; v += kBatchBlock) gstore(&P[v], v);
    __threadfence_block();
    __syncthreads();
    // one workgroup's walks: without splitting its trees grow deep (R-MAT
    // n = 2^20, 2^23 entries: 117 ms against 28 ms), so it always splits
    if (hook_hbm<kBatchBlock>(P, n, E, 0, m, tid, true)) *bad_flag = 1;
    __threadfence_block();
    __syncthreads();
    // Links are CASes performed at the memory side, which leave this XCD's L2
    // copy of a linked root as it was: the vertex's own entry and the root a
    // walk stops at are read coherently, and a coherent value that differs
    // continues the walk (as k_bm_compress).
    for (uint32_t v = tid; v < n; v += kBatchBlock) {
        const uint32_t p = gload_agent(&P[v]);
        if (p == v) continue;
        uint32_t r = p;
        while (true) {
            uint32_t q = P[r];
            while (q != r) { r = q; q = P[r]; }
            q = gload_agent(&P[r]);
            if (q == r) break;
            r = q;
        }
        if (r != p) gstore(&P[v], r);
    }
}

// The persistent kernel: tile graphs order[0, Gt) first, then wave graphs
// order[Gt, Gt + Gw). lds16_cap: largest n whose 16-bit parent array fits the
// dynamic LDS; wave_words: 32-bit words of LDS per wavefront in the wave role.
__global__ __launch_bounds__(kBatchBlock) void k_batch(const GraphDesc* __restrict__ descs,
                                                       const uint32_t* __restrict__ order,
                                                       uint32_t Gt, uint32_t Gw, uint32_t* tickets,
                                                       uint32_t lds16_cap, uint32_t wave_words) {
    extern __shared__ uint32_t sP[];
    __shared__ uint32_t s_next;
    __shared__ int s_bad;
    __shared__ uint2 s_q[kWaves * kLinkQueue];          // each wave's link queue
    uint2* const myq = s_q + (threadIdx.x >> 6) * kLinkQueue;
    while (Gt) {
        if (threadIdx.x == 0) {
            s_next = atomicAdd(&tickets[kTileTicket], 1u);
            s_bad = 0;
        }
        __syncthreads();
        const uint32_t t = s_next;
        if (t >= Gt) break;
        const GraphDesc d = descs[order[t]];
        gedge_t* E = (gedge_t*)d.edges;
        if (d.n <= lds16_cap / 2) {
            if (solve_graph_lds<kBatchBlock, uint32_t>(sP, d.n, E, d.m, (glabel_t*)d.L, threadIdx.x, myq))
                s_bad = 1;
        } else if (d.n <= lds16_cap) {
            if (solve_graph_lds<kBatchBlock, uint16_t>(sP, d.n, E, d.m, (glabel_t*)d.L, threadIdx.x, myq))
                s_bad = 1;
        } else {
            solve_graph_hbm((glabel_t*)d.L, d.n, E, d.m, &s_bad);
        }
        __syncthreads();
        if (threadIdx.x == 0) *(CCM_GLOBAL int32_t*)d.status = s_bad ? CC_ERANGE : CC_OK;
        __syncthreads();
    }
    // Wave role: from here on no workgroup barrier (waves leave independently).
    // The tile role's last barrier has passed, so the LDS is free.
    const int lane = threadIdx.x & 63;
    uint32_t* wP = sP + (threadIdx.x >> 6) * wave_words;
    while (Gw) {
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(&tickets[kWaveTicket], 1u);
        t = __shfl(t, 0);
        if (t >= Gw) break;
        const GraphDesc d = descs[order[Gt + t]];
        gedge_t* E = (gedge_t*)d.edges;
        const bool bad = d.n <= wave_words
                             ? solve_graph_lds<64, uint32_t>(wP, d.n, E, d.m, (glabel_t*)d.L, lane, myq)
                             : solve_graph_lds<64, uint16_t>(wP, d.n, E, d.m, (glabel_t*)d.L, lane, myq);
        const bool any_bad = __ballot(bad) != 0;
        if (lane == 0) *(CCM_GLOBAL int32_t*)d.status = any_bad ? CC_ERANGE : CC_OK;
        wave_sync();   // the next graph's init must not overtake this one's reads
    }
}

// ---- multi role: whole-device launches over chunk tables -------------------------------

constexpr int kMultiBlock = 256;
constexpr int kMultiVPT = 8;
constexpr uint64_t kMultiVChunk = (uint64_t)kMultiBlock * kMultiVPT;   // vertices per chunk
constexpr uint64_t kMultiEChunk = (uint64_t)kMultiBlock * kBatchEPT * 4;   // entries per chunk

// The multi graph owning chunk b: pre holds K+1 chunk-count prefixes
// (pre[0] = 0, pre[K] = total > b); returns k with pre[k] <= b < pre[k+1].
__device__ __forceinline__ uint32_t chunk_owner(const uint32_t* pre, uint32_t K, uint32_t b) {
    uint32_t lo = 0, hi = K;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

// P_v = v over every multi graph; the first chunk of a graph also sets its
// status to CC_OK (every multi graph has at least one vertex chunk).
__global__ __launch_bounds__(kMultiBlock) void k_bm_init(const GraphDesc* __restrict__ descs,
                                                         const uint32_t* __restrict__ mlist,
                                                         const uint32_t* __restrict__ vpre, uint32_t K) {
    const uint32_t total = vpre[K];
    for (uint32_t b = blockIdx.x; b < total; b += gridDim.x) {
        const uint32_t k = chunk_owner(vpre, K, b);
        const GraphDesc d = descs[mlist[k]];
        glabel_t* P = (glabel_t*)d.L;
        const uint64_t v0 = (uint64_t)(b - vpre[k]) * kMultiVChunk;
#pragma unroll
        for (int i = 0; i < kMultiVPT; ++i) {
            const uint64_t v = v0 + (uint64_t)i * kMultiBlock + threadIdx.x;
            if (v < d.n) gstore(&P[v], (uint32_t)v);
        }
        if (v0 == 0 && threadIdx.x == 0) gstore((glabel_t*)d.status, (uint32_t)CC_OK);
    }
}

// Hooking of every multi graph's entries, a chunk of kMultiEChunk entries per
// block step (Algorithm 1, as the HBM tile role, across the device). part 0
// takes each graph's entries below its split point (the first quarter of a
// graph hooked in two parts, hook_in_two_parts; all entries of any other
// graph), part 1 the rest, after a pointer-jumping pass.
__global__ __launch_bounds__(kMultiBlock) void k_bm_hook(const GraphDesc* __restrict__ descs,
                                                         const uint32_t* __restrict__ mlist,
                                                         const uint32_t* __restrict__ epre, uint32_t K,
                                                         int part) {
    const uint32_t total = epre[K];
    for (uint32_t b = blockIdx.x; b < total; b += gridDim.x) {
        const uint32_t k = chunk_owner(epre, K, b);
        const GraphDesc d = descs[mlist[k]];
        glabel_t* P = (glabel_t*)d.L;
        gedge_t* E = (gedge_t*)d.edges;
        const bool split = split_walks(0, d.n);
        const int64_t q = hook_in_two_parts(d.n, (uint64_t)d.m, split) ? d.m / 4 : d.m;
        int64_t e0 = (int64_t)(b - epre[k]) * (int64_t)kMultiEChunk;
        int64_t e1 = std::min<int64_t>(e0 + (int64_t)kMultiEChunk, d.m);
        if (part == 0) e1 = std::min<int64_t>(e1, q);
        else e0 = std::max<int64_t>(e0, q);
        if (e0 >= e1) continue;
        const bool bad = hook_hbm<kMultiBlock>(P, d.n, E, e0, e1, threadIdx.x, split);
        if (bad) gstore((glabel_t*)d.status, (uint32_t)CC_ERANGE);
    }
}

// P_v <- root(v) over every multi graph. Other XCDs linked these entries, so the
// vertex's own entry and the root the walk stops at are read coherently (a
// stale copy in this XCD's L2 is an ancestor, but a stale "root" would end the
// walk early); a coherent value that differs continues the walk.
__global__ __launch_bounds__(kMultiBlock) void k_bm_compress(const GraphDesc* __restrict__ descs,
                                                             const uint32_t* __restrict__ mlist,
                                                             const uint32_t* __restrict__ vpre, uint32_t K) {
    const uint32_t total = vpre[K];
    for (uint32_t b = blockIdx.x; b < total; b += gridDim.x) {
        const uint32_t k = chunk_owner(vpre, K, b);
        const GraphDesc d = descs[mlist[k]];
        glabel_t* P = (glabel_t*)d.L;
        const uint64_t v0 = (uint64_t)(b - vpre[k]) * kMultiVChunk;
        uint32_t pv[kMultiVPT];
#pragma unroll
        for (int i = 0; i < kMultiVPT; ++i) {
            const uint64_t v = v0 + (uint64_t)i * kMultiBlock + threadIdx.x;
            pv[i] = v < d.n ? gload_agent(&P[v]) : (uint32_t)v;
        }
#pragma unroll
        for (int i = 0; i < kMultiVPT; ++i) {
            const uint64_t v = v0 + (uint64_t)i * kMultiBlock + threadIdx.x;
            if (v >= d.n || pv[i] == (uint32_t)v) continue;
            uint32_t r = pv[i];
            while (true) {
                uint32_t q = P[r];
                while (q != r) { r = q; q = P[r]; }
                q = gload_agent(&P[r]);
                if (q == r) break;
                r = q;
            }
            if (r != pv[i]) gstore(&P[v], r);
        }
    }
}

// ---- host side ---------------------------------------------------------------------------

void batch_scratch_free(BatchScratch* b) {
    if (b->dev) (void)hipFree(b->dev);
    if (b->host) (void)hipHostFree(b->host);
    *b = BatchScratch{};
}

// Layout of the work list block (device and pinned host staging alike):
// [tickets: 256 B][order: 4G][mlist: 4G][vpre: 4(G+1)][epre: 4(G+1)][descs: 40G],
// every part on a 64-byte boundary. order = tile graphs, then wave graphs;
// mlist = multi graphs; vpre / epre = their vertex / entry chunk-count prefixes.
struct BatchLayout {
    uint64_t order, mlist, vpre, epre, descs, bytes;
};
static BatchLayout batch_layout(uint64_t G) {
    auto al = [](uint64_t x) { return (x + 63) & ~63ull; };
    BatchLayout l;
    l.order = kTicketBytes;
    l.mlist = l.order + al(4 * G);
    l.vpre = l.mlist + al(4 * G);
    l.epre = l.vpre + al(4 * (G + 1));
    l.descs = l.epre + al(4 * (G + 1));
    l.bytes = l.descs + sizeof(GraphDesc) * G;
    return l;
}

// Dynamic LDS of the persistent kernel: 2^16 16-bit entries (128 KB), or what
// the device allows beside the static words; tile graphs above that size use
// HBM. The wave role splits the same bytes into kWaves partitions.
struct LdsPlan {
    size_t bytes;
    uint32_t tile_cap;     // largest n of a tile graph in LDS
    uint32_t wave_words;   // 32-bit words per wavefront
    uint32_t wave_cap;     // largest n of a wave graph
};
static int lds_plan(int device, LdsPlan* out) {
    int max_lds = 0;
    CCM_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    // beside it: the link queues (16 KB) and a few static words
    size_t b = (size_t)max_lds > 20480 ? (size_t)max_lds - 20480 : 0;
    b = std::min<size_t>(b, (size_t)1 << 17);
    b &= ~(size_t)255;
    out->bytes = b;
    out->tile_cap = (uint32_t)std::min<size_t>(b / sizeof(uint16_t), (size_t)1 << 16);
    out->wave_words = (uint32_t)std::min<size_t>(b / 4 / kWaves, CC_BATCH_WAVE_MAX_N / 2);
    out->wave_cap = 2 * out->wave_words;
    return CC_OK;
}

static int batch_alloc(BatchScratch* bs, uint64_t G) {
    uint64_t cap = std::max<uint64_t>(G, 1024);
    const uint64_t bytes = batch_layout(cap).bytes;
    if (hipMalloc(&bs->dev, bytes) != hipSuccess ||
        hipHostMalloc(&bs->host, bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        batch_scratch_free(bs);
        return fail(CC_ENOMEM, "batch scratch allocation failed");
    }
    bs->cap = cap;
    return CC_OK;
}

int batch_wave_cap(int device, uint32_t* cap) {
    LdsPlan lds;
    int rc = lds_plan(device, &lds);
    if (rc) return rc;
    *cap = lds.wave_cap;
    return CC_OK;
}

int batch_role(const GraphDesc& d, const BatchSched& sc, uint32_t wave_cap) {
    const uint32_t wave_n = std::min(sc.wave_max_n, wave_cap);
    if (sc.multi_min_n && d.n >= sc.multi_min_n) return kRoleMulti;
    if (wave_n && d.n <= wave_n && d.m <= (int64_t)CC_BATCH_WAVE_MAX_M) return kRoleWave;
    return kRoleTile;
}

BatchSched batch_default_sched() {
    BatchSched s;
    s.wave_max_n = 0;
    s.multi_min_n = (1u << 16) + 1;   // beyond the LDS-resident tile graphs
    return s;
}

// What one launch runs: graph counts per role and the multi chunk totals.
struct BatchPlan {
    uint32_t G = 0, Gt = 0, Gw = 0, Gm = 0;
    uint32_t vchunks = 0, echunks = 0;
    bool two_part = false;   // some multi graph is hooked in two parts
};

// Host staging of one launch: the zeroed tickets, the role lists (tile and wave
// largest-first by entries + vertices), the chunk tables and the descriptors.
static int batch_prepare(BatchScratch* bs, uint32_t G, const GraphDesc* descs,
                         const BatchSched& sc, const LdsPlan& lds, BatchPlan* plan) {
    std::vector<uint32_t> tile, wave, multi;
    tile.reserve(G);
    for (uint32_t g = 0; g < G; ++g) {
        const int role = batch_role(descs[g], sc, lds.wave_cap);
        (role == kRoleMulti ? multi : role == kRoleWave ? wave : tile).push_back(g);
    }
    auto larger = [&](uint32_t a, uint32_t b) {
        return descs[a].m + (int64_t)descs[a].n > descs[b].m + (int64_t)descs[b].n;
    };
    std::stable_sort(tile.begin(), tile.end(), larger);
    std::stable_sort(wave.begin(), wave.end(), larger);
    const BatchLayout l = batch_layout(G);
    char* h = bs->host;
    std::memset(h, 0, kTicketBytes);
    uint32_t* order = reinterpret_cast<uint32_t*>(h + l.order);
    std::copy(tile.begin(), tile.end(), order);
    std::copy(wave.begin(), wave.end(), order + tile.size());
    uint32_t* mlist = reinterpret_cast<uint32_t*>(h + l.mlist);
    uint32_t* vpre = reinterpret_cast<uint32_t*>(h + l.vpre);
    uint32_t* epre = reinterpret_cast<uint32_t*>(h + l.epre);
    uint64_t vt = 0, et = 0;
    vpre[0] = epre[0] = 0;
    for (size_t k = 0; k < multi.size(); ++k) {
        const GraphDesc& d = descs[multi[k]];
        mlist[k] = multi[k];
        vt += std::max<uint64_t>(1, (d.n + kMultiVChunk - 1) / kMultiVChunk);
        et += ((uint64_t)d.m + kMultiEChunk - 1) / kMultiEChunk;
        if (vt > 0xFFFFFFFFull || et > 0xFFFFFFFFull)
            return fail(CC_EINVAL, "multi graphs too large for one batch");
        vpre[k + 1] = (uint32_t)vt;
        epre[k + 1] = (uint32_t)et;
        plan->two_part = plan->two_part ||
                         hook_in_two_parts(d.n, (uint64_t)d.m, split_walks(0, d.n));
    }
    std::copy(descs, descs + G, reinterpret_cast<GraphDesc*>(h + l.descs));
    plan->G = G;
    plan->Gt = (uint32_t)tile.size();
    plan->Gw = (uint32_t)wave.size();
    plan->Gm = (uint32_t)multi.size();
    plan->vchunks = (uint32_t)vt;
    plan->echunks = (uint32_t)et;
    return CC_OK;
}

// The device part of one launch: upload of the staging (which also zeroes the
// tickets, so a captured copy of this sequence replays correctly), the
// whole-device launches of the multi graphs, the persistent kernel, and the
// coherence points around them. Only stream work: it can be captured.
static int batch_enqueue(int device, BatchScratch* bs, const BatchPlan& p, const LdsPlan& lds,
                         hipStream_t stream) {
    const BatchLayout l = batch_layout(p.G);
    CCM_HIP(hipMemcpyAsync(bs->dev, bs->host, l.bytes, hipMemcpyHostToDevice, stream));
    char* d = bs->dev;
    const GraphDesc* descs = reinterpret_cast<const GraphDesc*>(d + l.descs);
    const int cus = device_cu_count(device);
    int rc = cohere(stream);
    if (rc) return rc;
    if (p.Gm) {
        const uint32_t* mlist = reinterpret_cast<const uint32_t*>(d + l.mlist);
        const uint32_t* vpre = reinterpret_cast<const uint32_t*>(d + l.vpre);
        const uint32_t* epre = reinterpret_cast<const uint32_t*>(d + l.epre);
        const uint32_t cap = (uint32_t)cus * 8;
        k_bm_init<<<std::min(p.vchunks, cap), kMultiBlock, 0, stream>>>(descs, mlist, vpre, p.Gm);
        CCM_HIP(hipGetLastError());
        if ((rc = cohere(stream))) return rc;
        if (p.echunks) {
            k_bm_hook<<<std::min(p.echunks, cap), kMultiBlock, 0, stream>>>(descs, mlist, epre, p.Gm,
                                                                          0);
            CCM_HIP(hipGetLastError());
            if ((rc = cohere(stream))) return rc;
        }
        if (p.two_part) {
            k_bm_compress<<<std::min(p.vchunks, cap), kMultiBlock, 0, stream>>>(descs, mlist, vpre,
                                                                              p.Gm);
            CCM_HIP(hipGetLastError());
            if ((rc = cohere(stream))) return rc;
            k_bm_hook<<<std::min(p.echunks, cap), kMultiBlock, 0, stream>>>(descs, mlist, epre, p.Gm,
                                                                          1);
            CCM_HIP(hipGetLastError());
            if ((rc = cohere(stream))) return rc;
        }
        k_bm_compress<<<std::min(p.vchunks, cap), kMultiBlock, 0, stream>>>(descs, mlist, vpre, p.Gm);
        CCM_HIP(hipGetLastError());
    }
    if (p.Gt + p.Gw) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds.bytes);
        (void)hipGetLastError();
        const uint64_t want = (uint64_t)p.Gt + (p.Gw + kWaves - 1) / kWaves;
        const uint32_t grid = (uint32_t)std::min<uint64_t>((uint64_t)cus, want);
        k_batch<<<grid, kBatchBlock, lds.bytes, stream>>>(
            descs, reinterpret_cast<const uint32_t*>(d + l.order), p.Gt, p.Gw,
            reinterpret_cast<uint32_t*>(d), lds.tile_cap, lds.wave_words);
        CCM_HIP(hipGetLastError());
    }
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
int launch_batch(Slot* s, uint32_t G, const GraphDesc* descs, const BatchSched& sc,
                 hipStream_t stream) {
    if (G == 0) return CC_OK;
    BatchScratch& bs = s->batch;
    if (bs.cap < G) {
        // the previous launch on this slot must be done with the staging
        CCM_HIP(hipStreamSynchronize(stream));
        batch_scratch_free(&bs);
        int rc = batch_alloc(&bs, G);
        if (rc) return rc;
    }
    LdsPlan lds;
    int rc = lds_plan(s->device, &lds);
    if (rc) return rc;
    BatchPlan plan;
    if ((rc = batch_prepare(&bs, G, descs, sc, lds, &plan))) return rc;
    return batch_enqueue(s->device, &bs, plan, lds, stream);
}

// Offsets read back and checked, descriptors built (cc_batch's arguments).
int batch_descs(uint32_t G, const int64_t* vtx_off, const int64_t* edge_off, const int32_t* edges,
                int32_t* L, int32_t* status, hipStream_t stream, std::vector<GraphDesc>* out) {
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

int batch_graph_create(Slot* s, uint32_t G, const GraphDesc* descs, const BatchSched& sc,
                       void** out) {
    *out = nullptr;
    LdsPlan lds;
    int rc = lds_plan(s->device, &lds);
    if (rc) return rc;
    BatchGraph* bg = new BatchGraph;
    bg->device = s->device;
    if ((rc = batch_alloc(&bg->bs, G))) {
        delete bg;
        return rc;
    }
    BatchPlan plan;
    if ((rc = batch_prepare(&bg->bs, G, descs, sc, lds, &plan))) {
        batch_scratch_free(&bg->bs);
        delete bg;
        return rc;
    }
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
        rc = batch_enqueue(bg->device, &bg->bs, plan, lds, cs);
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

}  // namespace ccm
