// cc_tiled.hip — the zero-root hook with both membership tests in LDS.
//
// The plain bitmap hook pays two random L2/MALL line reads per entry (the
// bitmap is n/8 bytes, 8.5 MB at RMAT-26, twice one XCD's L2). Here the
// entries are first regrouped so that each workgroup sees only entries whose
// endpoints fall in two fixed vertex ranges ("slices" of 2^kSliceBits
// vertices), and it holds the bitmap words of both slices in LDS:
//
//  1. k_t1_part   — every chunk of kC1 entries is sorted in LDS by the slice
//                   of its first endpoint (a) and written back in place order;
//                   per chunk, the start of each a-segment; per a, the counts.
//  2. k_t1_scan   — per a, exclusive prefix of the segment counts over chunks
//                   (each a-bucket becomes one virtual array).
//  3. k_t1_bases  — where each a-bucket starts in the second buffer and how
//                   many level-2 chunks it has.
//  4. k_t2_part   — every kC2-entry piece of an a-bucket is gathered from its
//                   segments, sorted in LDS by the slice of the second
//                   endpoint (b) and written contiguously, with its b-runs.
//  5. k_t3_filter — one workgroup per (a, b): both slices' bitmap words in
//                   LDS; an entry with both endpoints marked is dropped, one
//                   with a single marked endpoint marks the other (LDS and
//                   global) and is dropped, the rest go to a survivor list.
//  6. k_t4_hook   — the ordinary hook over the survivor list.
//
// After this step the components are given by P and the bitmap together
// (k_compress / k_resolve in cc_kernels.hip read both).
//
// The regrouping only reorders entries (and drops self-loops, which are
// no-ops), hooking is order-independent (Sec. II), and every dropped entry is
// either redundant or recorded as a mark, so the labels are those of the plain
// pass. Entries whose endpoints are out of range are dropped with
// the status bit set, as in the plain hook.
#include <algorithm>

#include "cc_internal.h"

namespace ccm {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

constexpr int kSliceBits = 19;                       // 2^19 vertices per slice
constexpr uint32_t kSliceWords = (1u << kSliceBits) / 32;   // 16384 words = 64 KB
constexpr uint32_t kLoMask = (1u << kSliceBits) - 1;

// Packed entries. With at most 256 slices every ID is below 2^27, and inside a
// bucket the slice bits of an endpoint are known, so the buffers between the
// passes hold fewer than 8 bytes per entry:
//  level 1 (bucket a known): w = u_lo | v << 19, h = v >> 13 (4 + 2 bytes)
// (u_lo: the low 19 bits of u; the top 13 bits of w carry the low 13 bits of v).
// The survivor regions reuse this format.
//  level 2 (both slices known from the run): w = u_lo | v_lo << 19,
//  h = v_lo >> 13 (4 + 1 bytes), two arrays.
__device__ __forceinline__ uint32_t pk_w(uint32_t ulo, uint32_t v) { return ulo | (v << kSliceBits); }
__device__ __forceinline__ uint32_t pk_v1(uint32_t w, uint16_t h) {
    return (w >> kSliceBits) | ((uint32_t)h << (32 - kSliceBits));
}

// The level-2 buffer: the two arrays of the 5-byte relative form.
struct L2Buf {
    uint32_t* w;
    uint8_t* h;
};

constexpr int kMaxSlices = 256;
constexpr int kC1 = 8192;                            // level-1 chunk (entries)
constexpr int kC2 = 8192;                            // level-2 chunk (entries)
constexpr int kPartBlock = 1024;
constexpr int kPartEPT = kC1 / kPartBlock;           // 8

// ---- shared device helpers (same rules as the plain hook) ---------------------

__device__ __forceinline__ bool t_key_less(uint32_t a, uint32_t b, uint32_t z) {
    return (a == z) | ((b != z) & (a < b));
}

// Root of x with path splitting: device-coherent splitting stores, each issued
// after the next step's load (the rule and its reasons are those of
// cc_kernels.hip's find_root).
__device__ __forceinline__ uint32_t t_find(uint32_t* P, uint32_t x, uint32_t px) {
    if (px == x) return x;
    uint32_t gp = P[px];
    while (gp != px) {
        const uint32_t ggp = P[gp];
        stress_delay(x);
        st_agent(&P[x], gp);
        x = px;
        px = gp;
        gp = ggp;
    }
    return px;
}

__device__ __forceinline__ uint32_t t_link(uint32_t* P, uint32_t u, uint32_t pu, uint32_t v,
                                           uint32_t pv, uint32_t z) {
    while (true) {
        const uint32_t ru = t_find(P, u, pu);
        const uint32_t rv = t_find(P, v, pv);
        if (ru == rv) return ru;
        const bool u_low = t_key_less(ru, rv, z);
        const uint32_t hi = u_low ? rv : ru;
        const uint32_t lo = u_low ? ru : rv;
        stress_delay(hi);
        // a coherent read before the CAS, as in cc_kernels.hip's link: a root
        // seen through a stale L2 copy is not CASed
        const uint32_t cur = ld_agent(&P[hi]);
        if (cur != hi) {
            u = hi; pu = cur;
            v = lo; pv = lo;
            continue;
        }
        const uint32_t old = atomicCAS(&P[hi], hi, lo);
        if (old == hi) return lo;
        u = hi; pu = old;
        v = lo; pv = lo;
    }
}

// Exclusive scan of cnt[0..R) into start[0..R] by the first wave (R <= 256);
// start[R] is the total.
__device__ __forceinline__ void wave_scan_256(const uint32_t* cnt, uint32_t* start, int R) {
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < 64) {
        uint32_t c[4], s = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int d = lane * 4 + j;
            c[j] = d < R ? cnt[d] : 0u;
            s += c[j];
        }
        uint32_t incl = s;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        uint32_t run = incl - s;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int d = lane * 4 + j;
            if (d < R) start[d] = run;
            run += c[j];
        }
        if (lane == 63) start[R] = incl;
    }
}

// ---- 1. level-1 partition by the first endpoint's slice -----------------------------
__global__ __launch_bounds__(kPartBlock) void k_t1_part(const uint32_t* __restrict__ edges,
                                                        uint64_t m, uint32_t n, int R,
                                                        uint64_t nch1, uint32_t* __restrict__ t1w,
                                                        uint16_t* __restrict__ t1h,
                                                        uint16_t* __restrict__ segT,
                                                        uint32_t* __restrict__ cnt1,
                                                        DevState* st, uint32_t sym) {
    __shared__ u32x2 stage[kC1];
    __shared__ uint32_t hist[kMaxSlices + 1];
    __shared__ uint32_t start[kMaxSlices + 1];
    const uint64_t c = blockIdx.x;
    for (int i = threadIdx.x; i <= kMaxSlices; i += kPartBlock) hist[i] = 0;
    __syncthreads();
    const u32x2* E = reinterpret_cast<const u32x2*>(edges);
    u32x2 e[kPartEPT];
    uint16_t rank[kPartEPT];
    bool bad = false;
#pragma unroll
    for (int k = 0; k < kPartEPT; ++k) {
        // unconditional load (clamped index): keeps all loads of the thread in flight
        const uint64_t i = c * kC1 + (uint64_t)k * kPartBlock + threadIdx.x;
        e[k] = __builtin_nontemporal_load(E + (i < m ? i : m - 1));
    }
#pragma unroll
    for (int k = 0; k < kPartEPT; ++k) {
        const uint64_t i = c * kC1 + (uint64_t)k * kPartBlock + threadIdx.x;
        if (i >= m) e[k].x = e[k].y = 0u;
        else if (e[k].x >= n || e[k].y >= n) { bad = true; e[k].x = e[k].y = 0u; }
    }
    if (bad) atomicOr(&st->status, kStatusRange);
#pragma unroll
    for (int k = 0; k < kPartEPT; ++k) {
        rank[k] = 0xFFFF;
        // self-loops are dropped; with sym (every pair listed in both orders) so
        // are the entries with u > v
        const bool live = sym ? e[k].x < e[k].y : e[k].x != e[k].y;
        if (live) rank[k] = (uint16_t)atomicAdd(&hist[e[k].x >> kSliceBits], 1u);
    }
    __syncthreads();
    wave_scan_256(hist, start, R);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPartEPT; ++k)
        if (rank[k] != 0xFFFF) stage[start[e[k].x >> kSliceBits] + rank[k]] = e[k];
    __syncthreads();
    const uint32_t kept = start[R];
    for (uint32_t i = threadIdx.x; i < kept; i += kPartBlock) {
        const u32x2 x = stage[i];
        t1w[c * kC1 + i] = pk_w(x.x & kLoMask, x.y);
        t1h[c * kC1 + i] = (uint16_t)(x.y >> (32 - kSliceBits));
    }
    for (int d = threadIdx.x; d < R; d += kPartBlock) {
        segT[(uint64_t)d * nch1 + c] = (uint16_t)start[d];
        cnt1[(uint64_t)d * nch1 + c] = hist[d];
    }
}

// ---- 2. per slice a: exclusive prefix of segment counts over chunks ------------------
// pre1 has nch1 + 1 entries per row (the last is the total). Two launches over
// (a, tile of kScanTile chunks): tile sums, then the scan of each tile offset by
// the sum of the tiles before it.
constexpr int kScanTile = 1024;
constexpr int kScanBlock = 256;

__global__ __launch_bounds__(kScanBlock) void k_t1_tsum(const uint32_t* __restrict__ cnt1,
                                                        uint64_t nch1, uint32_t ntile,
                                                        uint32_t* __restrict__ tsum) {
    __shared__ uint32_t ws[kScanBlock / 64];
    const uint64_t a = blockIdx.x / ntile, tile = blockIdx.x % ntile;
    const uint32_t* row = cnt1 + a * nch1;
    uint32_t s = 0;
    for (int k = 0; k < kScanTile / kScanBlock; ++k) {
        const uint64_t c = tile * kScanTile + (uint64_t)k * kScanBlock + threadIdx.x;
        if (c < nch1) s += row[c];
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kScanBlock / 64; ++w) t += ws[w];
        tsum[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kScanBlock) void k_t1_scan(const uint32_t* __restrict__ cnt1,
                                                        uint64_t nch1, uint32_t ntile,
                                                        const uint32_t* __restrict__ tsum,
                                                        uint32_t* __restrict__ pre1) {
    __shared__ uint32_t ws[kScanBlock / 64];
    __shared__ uint32_t s_off;
    const uint64_t a = blockIdx.x / ntile, tile = blockIdx.x % ntile;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (wave == 0) {
        // sum of the tiles before this one (ntile may exceed 64: strided lanes)
        uint32_t s = 0;
        for (uint64_t i = lane; i < tile; i += 64) s += tsum[a * ntile + i];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) s_off = s;
    }
    const uint32_t* row = cnt1 + a * nch1;
    uint32_t* out = pre1 + a * (nch1 + 1);
    // each thread scans 4 consecutive chunks of the tile
    constexpr int PER = kScanTile / kScanBlock;
    const uint64_t c0 = tile * kScanTile + (uint64_t)threadIdx.x * PER;
    uint32_t v[PER], s = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        v[k] = c0 + k < nch1 ? row[c0 + k] : 0u;
        s += v[k];
    }
    uint32_t incl = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) ws[wave] = incl;
    __syncthreads();
    uint32_t run = s_off + incl - s;
    for (int w = 0; w < wave; ++w) run += ws[w];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        if (c0 + k < nch1) out[c0 + k] = run;
        run += v[k];
    }
    // the thread holding the last chunk writes the row total
    if (c0 < nch1 && nch1 <= c0 + PER) out[nch1] = run;
}

// ---- 3. bucket bases and level-2 chunk counts ---------------------------------------------
// base2[a]: first entry of bucket a in the second buffer; cbase[a]: first level-2
// chunk of bucket a; cbase[R] is the total.
__global__ __launch_bounds__(256) void k_t1_bases(const uint32_t* __restrict__ pre1, uint64_t nch1,
                                                  int R, uint64_t* __restrict__ base2,
                                                  uint32_t* __restrict__ cbase) {
    // one thread per slice (R <= 256): sizes, then block-wide exclusive prefixes
    __shared__ uint64_t s_b[256];
    __shared__ uint32_t s_c[256];
    const int a = threadIdx.x;
    const uint32_t size = a < R ? pre1[(uint64_t)a * (nch1 + 1) + nch1] : 0u;
    s_b[a] = size;
    s_c[a] = (size + kC2 - 1) / kC2;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {          // inclusive Hillis-Steele scan
        const uint64_t xb = a >= off ? s_b[a - off] : 0ull;
        const uint32_t xc = a >= off ? s_c[a - off] : 0u;
        __syncthreads();
        s_b[a] += xb;
        s_c[a] += xc;
        __syncthreads();
    }
    if (a < R) {
        base2[a] = s_b[a] - size;
        cbase[a] = s_c[a] - (size + kC2 - 1) / kC2;
    }
    if (a == R - 1) {
        base2[R] = s_b[a];
        cbase[R] = s_c[a];
    }
}

// ---- 4a. level-2 chunk descriptors ----------------------------------------------------------
// Level-2 chunk t of bucket a covers virtual positions [t*kC2, min((t+1)*kC2, size_a)).
// Its descriptor (8 words at desc[8 g], g = cbase[a] + t) holds what k_t2_part
// needs in one read: the first (c0) and last (c1) level-1 chunk it gathers
// from, a | count << 8, t, and the 64-bit output offset base2[a] + t*kC2. One
// thread per (a, c): it writes the fields of the chunks that start or end in
// its segment [pre[c], pre[c+1]).
__global__ __launch_bounds__(256) void k_t2_bounds(const uint32_t* __restrict__ pre1, uint64_t nch1,
                                                   int R, const uint32_t* __restrict__ cbase,
                                                   const uint64_t* __restrict__ base2,
                                                   uint32_t* __restrict__ desc) {
    const uint64_t id = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (id >= (uint64_t)R * nch1) return;
    const uint64_t a = id / nch1, c = id % nch1;
    const uint32_t* pre = pre1 + a * (nch1 + 1);
    const uint32_t p0 = pre[c], p1 = pre[c + 1], size = pre[nch1];
    if (p1 <= p0) return;
    for (uint32_t t = p0 / kC2; t <= (p1 - 1) / kC2; ++t) {
        const uint32_t first = t * kC2;
        const uint32_t last = min(first + (uint32_t)kC2, size) - 1;
        uint32_t* d = desc + (uint64_t)(cbase[a] + t) * 8;
        if (first >= p0 && first < p1) {
            const uint64_t o = base2[a] + first;
            d[0] = (uint32_t)c;
            d[2] = (uint32_t)a | ((last + 1 - first) << 8);
            d[3] = t;
            d[4] = (uint32_t)o;
            d[5] = (uint32_t)(o >> 32);
        }
        if (last >= p0 && last < p1) d[1] = (uint32_t)c;
    }
}

// ---- 4b. level-2 partition by the second endpoint's slice ----------------------------------
constexpr int kWin2 = 256;   // level-1 chunks per gather window (owner index fits a byte)

// The chunk's cnt entries (entry i in e[i / kPartBlock] of thread i % kPartBlock,
// hist zeroed beforehand) sorted by the second endpoint's slice through LDS and
// written contiguously to out in the level-2 form, with the start of every
// slice's run in run2T.
__device__ __forceinline__ void t2_sort_write(const u32x2 (&e)[kPartEPT], uint32_t cnt, int R,
                                              uint32_t* hist, uint32_t* start, u32x2* stage,
                                              L2Buf out, uint16_t* __restrict__ run2T,
                                              uint64_t nch2, uint32_t g) {
    uint16_t rank[kPartEPT];
#pragma unroll
    for (int k = 0; k < kPartEPT; ++k) {
        const uint32_t i = (uint32_t)k * kPartBlock + threadIdx.x;
        rank[k] = 0xFFFF;
        if (i < cnt) rank[k] = (uint16_t)atomicAdd(&hist[e[k].y >> kSliceBits], 1u);
    }
    __syncthreads();
    wave_scan_256(hist, start, R);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPartEPT; ++k)
        if (rank[k] != 0xFFFF) stage[start[e[k].y >> kSliceBits] + rank[k]] = e[k];
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < cnt; i += kPartBlock) {
        const u32x2 x = stage[i];
        const uint32_t vlo = x.y & kLoMask;
        out.w[i] = (x.x & kLoMask) | (vlo << kSliceBits);
        out.h[i] = (uint8_t)(vlo >> (32 - kSliceBits));
    }
    for (int d = threadIdx.x; d <= R; d += kPartBlock) run2T[(uint64_t)d * nch2 + g] = (uint16_t)start[d];
}

// Gathers level-2 chunk g of slice a from the slice's level-1 segments: entry i
// of the chunk lands in e[i / kPartBlock] of thread i % kPartBlock as (u, v).
// Returns the entry count; a and the output offset come back through a_out and
// obase. Every thread of the block calls it (it uses barriers).
__device__ __forceinline__ uint32_t t2_gather(uint32_t g, const uint32_t* __restrict__ t1w,
                                              const uint16_t* __restrict__ t1h,
                                              const uint16_t* __restrict__ segT,
                                              const uint32_t* __restrict__ pre1, uint64_t nch1,
                                              const uint32_t* __restrict__ desc, uint8_t* owner,
                                              uint32_t* s_pre, uint32_t* s_seg,
                                              u32x2 (&e)[kPartEPT], int& a_out, uint64_t& obase) {
    const uint4 d0 = reinterpret_cast<const uint4*>(desc)[2 * (uint64_t)g];
    const uint4 d1 = reinterpret_cast<const uint4*>(desc)[2 * (uint64_t)g + 1];
    const uint64_t c0 = d0.x, c1 = d0.y;
    const int a = (int)(d0.z & 0xFFu);
    const uint32_t cnt = d0.z >> 8;
    const uint32_t t = d0.w;
    obase = (uint64_t)d1.x | ((uint64_t)d1.y << 32);
    a_out = a;
    const uint32_t* pre = pre1 + (uint64_t)a * (nch1 + 1);
    const uint32_t vlo = t * (uint32_t)kC2;
    const uint32_t vhi = vlo + cnt;
    for (uint64_t cw = c0; cw <= c1; cw += kWin2) {
        const uint32_t nw = (uint32_t)min<uint64_t>((uint64_t)kWin2, c1 - cw + 1);
        for (uint32_t i = threadIdx.x; i <= nw; i += kPartBlock) s_pre[i] = pre[cw + i];
        for (uint32_t i = threadIdx.x; i < nw; i += kPartBlock)
            s_seg[i] = segT[(uint64_t)a * nch1 + cw + i];
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < nw; i += kPartBlock) {
            const uint32_t lo = max(s_pre[i], vlo), hi = min(s_pre[i + 1], vhi);
            for (uint32_t p = lo; p < hi; ++p) owner[p - vlo] = (uint8_t)i;
        }
        __syncthreads();
        const uint32_t wlo = max(s_pre[0], vlo), whi = min(s_pre[nw], vhi);
        uint32_t xw[kPartEPT];
        uint16_t xh[kPartEPT];
        bool in[kPartEPT];
#pragma unroll
        for (int k = 0; k < kPartEPT; ++k) {
            // unconditional loads (a safe in-bounds address when the position is
            // not in this window) so that all loads of the thread are in flight
            const uint32_t p = vlo + (uint32_t)k * kPartBlock + threadIdx.x;
            in[k] = p >= wlo && p < whi;
            const uint32_t i = in[k] ? owner[p - vlo] : 0u;
            const uint64_t at = in[k] ? (cw + i) * kC1 + s_seg[i] + (p - s_pre[i]) : 0ull;
            xw[k] = t1w[at];
            xh[k] = t1h[at];
        }
#pragma unroll
        for (int k = 0; k < kPartEPT; ++k)
            if (in[k]) {
                e[k].x = ((uint32_t)a << kSliceBits) | (xw[k] & kLoMask);
                e[k].y = pk_v1(xw[k], xh[k]);
            }
        __syncthreads();
    }
    return cnt;
}

__global__ __launch_bounds__(kPartBlock) void k_t2_part(const uint32_t* __restrict__ t1w,
                                                        const uint16_t* __restrict__ t1h,
                                                        const uint16_t* __restrict__ segT,
                                                        const uint32_t* __restrict__ pre1,
                                                        uint64_t nch1, int R,
                                                        const uint32_t* __restrict__ cbase,
                                                        const uint32_t* __restrict__ desc,
                                                        L2Buf tmp2, uint16_t* __restrict__ run2T,
                                                        uint64_t nch2) {
    __shared__ u32x2 stage[kC2];
    __shared__ uint8_t owner[kC2];
    __shared__ uint32_t s_pre[kWin2 + 1];
    __shared__ uint32_t s_seg[kWin2];
    __shared__ uint32_t hist[kMaxSlices + 1];
    __shared__ uint32_t start[kMaxSlices + 1];
    const uint32_t g = blockIdx.x;
    if (g >= cbase[R]) return;                  // the grid is an upper bound
    for (int i = threadIdx.x; i <= kMaxSlices; i += kPartBlock) hist[i] = 0;
    u32x2 e[kPartEPT];
    int a;
    uint64_t obase;
    const uint32_t cnt = t2_gather(g, t1w, t1h, segT, pre1, nch1, desc, owner, s_pre, s_seg, e, a,
                                   obase);
    t2_sort_write(e, cnt, R, hist, start, stage, L2Buf{tmp2.w + obase, tmp2.h + obase}, run2T,
                  nch2, g);
}

// Plain path (key = ID) on the level-1 buckets: each workgroup gathers one
// level-2 chunk, whose first endpoints all lie in one slice of 2^19 vertices,
// and hooks it. The workgroups running at one time mostly take consecutive
// chunks of one slice, so their first endpoints' parent entries (2 MB) stay in
// L2; only the second endpoints' reads are random over the whole array.
__global__ __launch_bounds__(kPartBlock) void k_t2_hookplain(const uint32_t* __restrict__ t1w,
                                                             const uint16_t* __restrict__ t1h,
                                                             const uint16_t* __restrict__ segT,
                                                             const uint32_t* __restrict__ pre1,
                                                             uint64_t nch1, int R,
                                                             const uint32_t* __restrict__ cbase,
                                                             const uint32_t* __restrict__ desc,
                                                             uint32_t* P) {
    __shared__ uint8_t owner[kC2];
    __shared__ uint32_t s_pre[kWin2 + 1];
    __shared__ uint32_t s_seg[kWin2];
    const uint32_t g = blockIdx.x;
    if (g >= cbase[R]) return;                  // the grid is an upper bound
    u32x2 e[kPartEPT];
    int a;
    uint64_t obase;
    const uint32_t cnt = t2_gather(g, t1w, t1h, segT, pre1, nch1, desc, owner, s_pre, s_seg, e, a,
                                   obase);
    bool h[kPartEPT];
    uint32_t pu[kPartEPT], pv[kPartEPT];
#pragma unroll
    for (int k = 0; k < kPartEPT; ++k) {
        h[k] = (uint32_t)k * kPartBlock + threadIdx.x < cnt;
        if (!h[k]) e[k].x = e[k].y = 0u;
    }
#pragma unroll
    for (int k = 0; k < kPartEPT; ++k) {
        pu[k] = P[e[k].x];
        pv[k] = P[e[k].y];
    }
#pragma unroll
    for (int k = 0; k < kPartEPT; ++k) {
        const uint32_t u = e[k].x, v = e[k].y;
        if (!h[k] || u == v) continue;
        if (pu[k] == pv[k] || pu[k] == v || pv[k] == u) continue;   // same tree already
        (void)t_link(P, u, pu[k], v, pv[k], kEmpty);               // no zero root: key = ID
    }
}

// ---- CSR input: the rows are the level-1 buckets ---------------------------------
// On CSR input the entries are already grouped by first endpoint: bucket a is
// the contiguous range of adj that holds the rows of slice a, so steps 1-3 are
// replaced by reading the offsets, and the level-2 pass reads adj directly and
// recovers each position's row (as the CSR hook does). The level-2 buffer uses
// adj's positions (base2[a] = start of slice a's rows), so steps 5-6 run
// unchanged. Every bound below is clamped to a monotone sequence inside
// [0, m], so offsets that are not a valid row index (reported separately) can
// change the result but never make an access leave its array.

// base2[a] = running maximum of off[a * 2^19] clamped to m (base2[R] = m);
// cbase = prefix of the chunk counts. One block, R <= 256.
__global__ __launch_bounds__(256) void k_c_bases(const uint64_t* __restrict__ off, uint64_t n,
                                                 uint64_t m, int R, uint64_t* __restrict__ base2,
                                                 uint32_t* __restrict__ cbase) {
    __shared__ uint64_t s_b[257];
    __shared__ uint32_t s_c[256];
    const int a = threadIdx.x;
    uint64_t lo = 0;
    if (a < R) {
        lo = off[(uint64_t)a << kSliceBits];
        lo = lo < m ? lo : m;
    }
    s_b[a] = lo;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {                 // inclusive running maximum
        const uint64_t x = a >= o ? s_b[a - o] : 0ull;
        __syncthreads();
        s_b[a] = s_b[a] > x ? s_b[a] : x;
        __syncthreads();
    }
    if (a == 0) s_b[256] = m;
    __syncthreads();
    const uint64_t hi = a + 1 < R ? s_b[a + 1] : m;
    const uint32_t chunks = a < R ? (uint32_t)((hi - s_b[a] + kC2 - 1) / kC2) : 0u;
    s_c[a] = chunks;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint32_t x = a >= o ? s_c[a - o] : 0u;
        __syncthreads();
        s_c[a] += x;
        __syncthreads();
    }
    if (a < R) {
        base2[a] = s_b[a];
        cbase[a] = s_c[a] - chunks;
    }
    if (a == R - 1) {
        base2[R] = m;
        cbase[R] = s_c[a];
    }
}

// cfirst[g]: the row holding the first position of level-2 chunk g. One thread
// per row: it writes the chunks of its slice that start inside it.
__global__ __launch_bounds__(256) void k_c_first(const uint64_t* __restrict__ off, uint64_t n,
                                                 const uint64_t* __restrict__ base2,
                                                 const uint32_t* __restrict__ cbase,
                                                 uint32_t* __restrict__ cfirst) {
    for (uint64_t v = (uint64_t)blockIdx.x * 256 + threadIdx.x; v < n;
         v += (uint64_t)gridDim.x * 256) {
        const uint64_t a = v >> kSliceBits;
        const uint64_t B0 = base2[a], B1 = base2[a + 1];
        uint64_t lo = off[v], hi = off[v + 1];
        lo = lo > B0 ? lo : B0;
        hi = hi < B1 ? hi : B1;
        if (hi <= lo) continue;
        const uint32_t cb = cbase[a];
        for (uint64_t t = (lo - B0 + kC2 - 1) / kC2; B0 + t * kC2 < hi; ++t)
            cfirst[cb + t] = (uint32_t)v;
    }
}

constexpr uint32_t kSweepMax2 = 4 * kC2;   // rows a chunk sweeps before it searches instead

__global__ __launch_bounds__(kPartBlock) void k_t2_csr(const uint64_t* __restrict__ off,
                                                       const uint32_t* __restrict__ adj,
                                                       uint64_t n, int R,
                                                       const uint64_t* __restrict__ base2,
                                                       const uint32_t* __restrict__ cbase,
                                                       const uint32_t* __restrict__ cfirst,
                                                       L2Buf tmp2,
                                                       uint16_t* __restrict__ run2T,
                                                       uint64_t nch2, DevState* st, uint32_t sym) {
    __shared__ u32x2 stage[kC2];
    // the rows of the positions live in the first half of the sort's staging
    // area: they are read into registers before t2_sort_write first writes it
    // (after two barriers), so both fit with two workgroups per CU
    uint32_t* head = reinterpret_cast<uint32_t*>(stage);
    __shared__ uint32_t hist[kMaxSlices + 1];
    __shared__ uint32_t start[kMaxSlices + 1];
    __shared__ uint32_t s_w[kPartBlock / 64];
    __shared__ int s_a;
    const uint32_t g = blockIdx.x;
    if (g >= cbase[R]) return;                  // the grid is an upper bound
    if (threadIdx.x == 0) {                     // the slice whose chunks hold g
        int lo = 0, hi = R - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (cbase[mid] <= g) lo = mid;
            else hi = mid - 1;
        }
        s_a = lo;
    }
    for (int i = threadIdx.x; i <= kMaxSlices; i += kPartBlock) hist[i] = 0;
    for (int i = threadIdx.x; i < kC2; i += kPartBlock) head[i] = 0;
    __syncthreads();
    const int a = s_a;
    const uint64_t pos0 = base2[a] + (uint64_t)(g - cbase[a]) * kC2;
    const uint64_t pend = base2[a + 1];
    const uint32_t cnt = (uint32_t)min<uint64_t>((uint64_t)kC2, pend - pos0);
    const uint32_t vlo = (uint32_t)a << kSliceBits;
    const uint32_t vhi = (uint32_t)min<uint64_t>(((uint64_t)a + 1) << kSliceBits, n) - 1;
    auto clampv = [&](uint32_t x) { return x < vlo ? vlo : (x > vhi ? vhi : x); };
    const uint32_t ua = clampv(cfirst[g]);
    uint32_t ub = (g + 1 < cbase[a + 1]) ? clampv(cfirst[g + 1]) : vhi;
    if (ub < ua) ub = ua;
    uint32_t v[kPartEPT];
#pragma unroll
    for (int k = 0; k < kPartEPT; ++k) {
        const uint32_t i = (uint32_t)k * kPartBlock + threadIdx.x;
        v[k] = i < cnt ? __builtin_nontemporal_load(adj + pos0 + i) : 0u;
    }
    uint32_t u[kPartEPT];
    if (ub - ua <= kSweepMax2) {
        if (threadIdx.x == 0) head[0] = ua;
        for (uint64_t x0 = (uint64_t)ua + 1; x0 <= ub; x0 += 4 * kPartBlock) {
            uint64_t lo[4], hi[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint64_t x = x0 + r * kPartBlock + threadIdx.x;
                const uint64_t xs = x <= ub ? x : ub;
                lo[r] = off[xs];
                hi[r] = off[xs + 1];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint64_t x = x0 + r * kPartBlock + threadIdx.x;
                if (x <= ub && lo[r] < hi[r] && lo[r] >= pos0 && lo[r] < pos0 + cnt)
                    head[lo[r] - pos0] = (uint32_t)x;
            }
        }
        __syncthreads();
        // inclusive max-scan of head: thread i owns head[8i .. 8i + 7]
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        uint32_t h[kPartEPT];
#pragma unroll
        for (int r = 0; r < kPartEPT; ++r) h[r] = head[kPartEPT * threadIdx.x + r];
#pragma unroll
        for (int r = 1; r < kPartEPT; ++r) h[r] = max(h[r], h[r - 1]);
        uint32_t incl = h[kPartEPT - 1];
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o, 64);
            if (lane >= o) incl = max(incl, y);
        }
        if (lane == 63) s_w[wave] = incl;
        uint32_t before = __shfl_up(incl, 1, 64);
        if (lane == 0) before = 0;
        __syncthreads();
        for (int w = 0; w < wave; ++w) before = max(before, s_w[w]);
#pragma unroll
        for (int r = 0; r < kPartEPT; ++r) head[kPartEPT * threadIdx.x + r] = max(h[r], before);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPartEPT; ++k) u[k] = head[k * kPartBlock + threadIdx.x];
    } else {
        // the last row x in [ua, ub] with off[x] <= p owns position p
#pragma unroll
        for (int k = 0; k < kPartEPT; ++k) {
            const uint64_t p = pos0 + (uint64_t)k * kPartBlock + threadIdx.x;
            uint32_t lo = ua, hi = ub;
            while (lo < hi) {
                const uint32_t mid = lo + (hi - lo + 1) / 2;
                if (off[mid] <= p) lo = mid;
                else hi = mid - 1;
            }
            u[k] = lo;
        }
    }
    bool bad = false;
    u32x2 e[kPartEPT];
#pragma unroll
    for (int k = 0; k < kPartEPT; ++k) {
        const uint32_t uu = clampv(u[k]);
        uint32_t vv = v[k];
        if ((uint32_t)k * kPartBlock + threadIdx.x < cnt && vv >= n) {
            bad = true;
            vv = uu;                              // skipped as a self-loop
        }
        if (sym && vv < uu) vv = uu;              // the reverse entry covers it
        e[k].x = uu;
        e[k].y = vv;
    }
    if (bad) atomicOr(&st->status, kStatusRange);
    t2_sort_write(e, cnt, R, hist, start, stage, L2Buf{tmp2.w + pos0, tmp2.h + pos0}, run2T, nch2,
                  g);
}

// ---- 5. the filter over bucket (a, b) with both slices' bitmap words in LDS ---------------
//
// A set bit means "connected to the zero root" (the Initial Push's bits are
// stronger: in z's tree already), as in the direct hook. An entry with
// both endpoints marked is dropped: the two are connected anyway. An entry with
// exactly one marked endpoint is dropped too, after marking the other endpoint:
// that mark is the entry's link to z, and compress later puts every tree that
// holds a marked vertex into z's component. Each mark rests on an entry and an
// earlier mark, so the marks never claim a connection the graph lacks. Only
// entries with neither endpoint marked are kept, for the survivor hook, which
// does not consult the bitmap.
constexpr int kHook3Block = 1024;
constexpr int kWaves3 = kHook3Block / 64;
constexpr int kWin3 = 2000;      // level-2 chunks per window
constexpr int kRunsInFlight = 12; // entries a lane loads at once (a wave: 12 x 64 consecutive)
constexpr int kPendQueue = 127;  // per-wave LDS staging of entries that need a second look

// Exclusive scan in place of n <= 2 * kHook3Block values (x[n] receives the
// total); every thread of the workgroup calls it.
__device__ __forceinline__ void block_scan_2048(uint32_t* x, uint32_t n, uint32_t* wsum) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t i0 = 2 * tid, i1 = 2 * tid + 1;
    const uint32_t a0 = i0 < n ? x[i0] : 0u, a1 = i1 < n ? x[i1] : 0u;
    const uint32_t s = a0 + a1;
    uint32_t incl = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    if (tid == 0) {
        uint32_t run = 0;
        for (int w = 0; w < kHook3Block / 64; ++w) { const uint32_t t = wsum[w]; wsum[w] = run; run += t; }
        wsum[kHook3Block / 64] = run;
    }
    __syncthreads();
    const uint32_t excl = wsum[wave] + incl - s;
    if (i0 < n) x[i0] = excl;
    if (i1 < n) x[i1] = excl + a0;
    if (tid == 0) x[n] = wsum[kHook3Block / 64];
    __syncthreads();
}

constexpr int kBPerBlock = 2;    // second-endpoint slices handled by one workgroup

// Survivor regions: workgroup (a, bg) of the filter reads exactly the entries of
// tiles (a, b), b in [2 bg, 2 bg + 2); its kept entries go to a region of that
// size inside [base2[a], base2[a+1]) of the survivor buffer; regions are
// consecutive, so wgoff[w + 1] ends region w (wgoff has R * nbg + 1 entries).
// One block per a.
__global__ __launch_bounds__(256) void k_t3_regions(const uint16_t* __restrict__ run2T,
                                                    uint64_t nch2, int R,
                                                    const uint32_t* __restrict__ cbase,
                                                    uint32_t* __restrict__ wgsize) {
    // one block per (a, bg): the group's entries summed over bucket a's chunks
    __shared__ uint32_t ws[4];
    const int nbg = (R + kBPerBlock - 1) / kBPerBlock;
    const int a = blockIdx.x / nbg, bg = blockIdx.x % nbg;
    const int blo = bg * kBPerBlock, bhi = min(R, blo + kBPerBlock);
    const uint32_t g0 = cbase[a], g1 = cbase[a + 1];
    uint32_t t = 0;
    for (uint32_t g = g0 + threadIdx.x; g < g1; g += 256)
        t += (uint32_t)run2T[(uint64_t)bhi * nch2 + g] - (uint32_t)run2T[(uint64_t)blo * nch2 + g];
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) wgsize[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// Per slice a, the regions' offsets: base2[a] plus the sizes of the groups
// before bg. One thread per a.
__global__ __launch_bounds__(256) void k_t3_offsets(const uint32_t* __restrict__ wgsize, int R,
                                                    const uint64_t* __restrict__ base2,
                                                    uint64_t* __restrict__ wgoff) {
    const int a = blockIdx.x * 256 + threadIdx.x;
    if (a >= R) return;
    const int nbg = (R + kBPerBlock - 1) / kBPerBlock;
    uint64_t run = base2[a];
    for (int bg = 0; bg < nbg; ++bg) {
        wgoff[(uint64_t)a * nbg + bg] = run;
        run += wgsize[(uint64_t)a * nbg + bg];
    }
    if (a == R - 1) wgoff[(uint64_t)R * nbg] = run;   // end of the last region
}

// Run holding index j0 of the window (last t < nw with s_pre[t] <= j0), found
// by the whole wave in two 64-way ballot steps (nw <= 64 * 64).
__device__ __forceinline__ uint32_t t3_find_run(const uint32_t* s_pre, uint32_t nw, uint32_t j0,
                                                int lane) {
    const uint32_t stride = (nw + 63) / 64;
    const uint32_t i1 = (uint32_t)lane * stride;
    const bool c1 = i1 < nw && s_pre[i1] <= j0;
    const uint64_t b1 = __ballot(c1);
    const uint32_t base = (63u - (uint32_t)__clzll((long long)b1)) * stride;
    const uint32_t i2 = base + (uint32_t)lane;
    const bool c2 = (uint32_t)lane < stride && i2 < nw && s_pre[i2] <= j0;
    const uint64_t b2 = __ballot(c2);
    return base + (63u - (uint32_t)__clzll((long long)b2));
}

// Offset of index j of the window (j in [jb, jb + 64), the indices one wave
// handles together): t is the run holding index jb, kept wave-uniform and
// advanced here to the run holding jb + 63. Runs are about as long as a wave,
// so this is usually one step; lanes past a run's end take the next run's
// offset. Every branch depends on wave-uniform values only.
__device__ __forceinline__ uint32_t t3_offset(const uint32_t* s_pre, const uint32_t* s_off,
                                              uint32_t nw, uint32_t& t, uint32_t jb, uint32_t j) {
    // the table reads have one address for the whole wave: keep them scalar
    uint32_t off = __builtin_amdgcn_readfirstlane(s_off[t]);
    uint32_t nxt = __builtin_amdgcn_readfirstlane(s_pre[t + 1]);
    while (t + 1 < nw && nxt < jb + 64) {
        ++t;
        const uint32_t o = __builtin_amdgcn_readfirstlane(s_off[t]);
        off = j >= nxt ? o : off;
        nxt = __builtin_amdgcn_readfirstlane(s_pre[t + 1]);
    }
    return off;
}

// Second look at up to 64 pending entries of this wave (lane l takes pq[l],
// endpoints relative to the slices' first IDs), with the bits as they are now:
// both marked, dropped; one marked, the other is marked (LDS, and the global
// word when this set the bit); neither, kept: written to the workgroup's
// survivor region (level-1 packing, its place from an LDS counter).
__device__ __forceinline__ void t3_settle(const u32x2* pq, uint32_t cnt, int lane, uint32_t* sa,
                                          uint32_t* lb, uint32_t abase, uint32_t bbase,
                                          uint32_t* zbits, uint32_t* ow, uint16_t* oh,
                                          uint32_t cap, uint32_t* s_used, DevState* st) {
    const bool act = (uint32_t)lane < cnt;
    const u32x2 x = act ? pq[lane] : u32x2{0u, 0u};
    const uint32_t iu = x.x >> 5, iv = x.y >> 5;
    const uint32_t bu = 1u << (x.x & 31), bv = 1u << (x.y & 31);
    const bool mu = (sa[iu] & bu) != 0u, mv = (lb[iv] & bv) != 0u;
    if (act && mu != mv) {
        // the entry's whole effect: mark the unmarked endpoint
        uint32_t* w = mu ? &lb[iv] : &sa[iu];
        const uint32_t bit = mu ? bv : bu;
        const uint32_t y = mu ? bbase + x.y : abase + x.x;
        if (!(atomicOr(w, bit) & bit)) atomicOr(&zbits[y >> 5], 1u << (y & 31));
    }
    const bool keep = act && !mu && !mv;
    const uint64_t ball = __ballot(keep);
    if (ball) {
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(s_used, (uint32_t)__popcll(ball));
        base = __shfl(base, 0, 64);
        if (keep) {
            const uint32_t i = base + (uint32_t)__popcll(ball & ((1ull << lane) - 1ull));
            if (i < cap) {
                const uint32_t v = bbase + x.y;
                ow[i] = pk_w(x.x, v);
                oh[i] = (uint16_t)(v >> (32 - kSliceBits));
            } else {
                // cannot happen (the region holds all of the workgroup's entries)
                atomicOr(&st->status, kStatusInternal);
            }
        }
    }
}

__global__ __launch_bounds__(kHook3Block) void k_t3_filter(L2Buf tmp2,
                                                           const uint16_t* __restrict__ run2T,
                                                           uint64_t nch2, int R,
                                                           const uint64_t* __restrict__ base2,
                                                           const uint32_t* __restrict__ cbase,
                                                           uint32_t* zbits, uint64_t words,
                                                           uint32_t* __restrict__ sw,
                                                           uint16_t* __restrict__ sh,
                                                           const uint64_t* __restrict__ wgoff,
                                                           uint32_t* __restrict__ wgcnt,
                                                           DevState* st) {
    __shared__ uint32_t sa[kSliceWords];
    __shared__ uint32_t sb[kSliceWords];
    __shared__ uint32_t s_off[kWin3];
    __shared__ uint32_t s_pre[kWin3 + 1];
    __shared__ u32x2 pqueue[kWaves3 * kPendQueue];
    __shared__ uint32_t wsum[kWaves3 + 1];
    __shared__ uint32_t s_used;
    // Launch order: consecutive workgroups take different a (and spread over
    // the b groups), so the workgroups running at the same time hold few
    // copies of any one slice and see each other's marks through the global
    // bitmap sooner. (a, bg) = (i mod R, (i div R + a) mod nbg) is a bijection.
    const int nbg = (R + kBPerBlock - 1) / kBPerBlock;
    const int a = (int)(blockIdx.x % (uint32_t)R);
    const int bg = (int)((blockIdx.x / (uint32_t)R + (uint32_t)a) % (uint32_t)nbg);
    const uint32_t wi = (uint32_t)a * (uint32_t)nbg + (uint32_t)bg;   // region index
    const uint32_t cb = cbase[a];
    const uint32_t nch = cbase[a + 1] - cb;
    if (nch == 0) {
        if (threadIdx.x == 0) wgcnt[wi] = 0;
        return;
    }
    if (threadIdx.x == 0) s_used = 0;
    uint32_t* ow = sw + wgoff[wi];
    uint16_t* oh = sh + wgoff[wi];
    const uint32_t cap = (uint32_t)(wgoff[wi + 1] - wgoff[wi]);
    constexpr int PER = kSliceWords / kHook3Block;       // 16 words per thread per slice
    {
        const uint64_t wa = (uint64_t)a * kSliceWords;
        uint32_t xa[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const uint64_t i = (uint64_t)k * kHook3Block + threadIdx.x;
            xa[k] = wa + i < words ? zbits[wa + i] : 0u;
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) sa[(uint32_t)k * kHook3Block + threadIdx.x] = xa[k];
    }
    const uint32_t abase = (uint32_t)a << kSliceBits;
    const uint32_t* srcw = tmp2.w + base2[a];
    const uint8_t* srch = tmp2.h + base2[a];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    u32x2* pq = pqueue + wave * kPendQueue;
    constexpr uint32_t kRange = 64 * kRunsInFlight;      // entries per wave per range
    constexpr uint32_t kStep = kWaves3 * kRange;
    for (int bi = 0; bi < kBPerBlock; ++bi) {
        const int b = bg * kBPerBlock + bi;
        if (b >= R) break;
        __syncthreads();                                  // previous slice b fully used
        if (b != a) {
            const uint64_t wb = (uint64_t)b * kSliceWords;
            uint32_t xb[PER];
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const uint64_t i = (uint64_t)k * kHook3Block + threadIdx.x;
                xb[k] = wb + i < words ? zbits[wb + i] : 0u;
            }
#pragma unroll
            for (int k = 0; k < PER; ++k) sb[(uint32_t)k * kHook3Block + threadIdx.x] = xb[k];
        }
        uint32_t* lb = (a == b) ? sa : sb;
        const uint32_t bbase = (uint32_t)b << kSliceBits;
        uint32_t pn = 0;                                  // wave-uniform pending count
        for (uint32_t w0 = 0; w0 < nch; w0 += kWin3) {
            const uint32_t nw = min((uint32_t)kWin3, nch - w0);
            __syncthreads();
            for (uint32_t t = threadIdx.x; t < nw; t += kHook3Block) {
                const uint64_t g = (uint64_t)cb + w0 + t;
                const uint32_t r0 = run2T[(uint64_t)b * nch2 + g];
                const uint32_t r1 = run2T[(uint64_t)(b + 1) * nch2 + g];
                s_off[t] = r0;
                s_pre[t] = r1 - r0;
            }
            __syncthreads();
            block_scan_2048(s_pre, nw, wsum);        // run lengths -> starts; s_pre[nw] = total
            // index of the window's j-th entry in run t: j + s_off[t] (mod 2^32;
            // every index of a bucket is below 2^32)
            for (uint32_t t = threadIdx.x; t < nw; t += kHook3Block)
                s_off[t] = (w0 + t) * (uint32_t)kC2 + s_off[t] - s_pre[t];
            __syncthreads();
            const uint32_t total = s_pre[nw];
            // The window's entries form one index space [0, total); each wave
            // takes ranges of kRange consecutive indices. Register k holds index
            // j0 + 64k + lane; right after it is tested it is reloaded with index
            // jn + 64k + lane of the next range (index 0 past the end), so the
            // next range's loads are in flight meanwhile.
            uint32_t j0 = (uint32_t)wave * kRange;
            if (j0 >= total) continue;
            uint32_t ew[kRunsInFlight], eh[kRunsInFlight];
            uint32_t t = __builtin_amdgcn_readfirstlane(t3_find_run(s_pre, nw, j0, lane));
#pragma unroll
            for (int k = 0; k < kRunsInFlight; ++k) {
                const uint32_t jb = j0 + (uint32_t)k * 64, j = jb + (uint32_t)lane;
                const uint32_t off = t3_offset(s_pre, s_off, nw, t, jb, j);
                const uint32_t at = j < total ? j + off : 0u;
                ew[k] = __builtin_nontemporal_load(srcw + at);
                eh[k] = __builtin_nontemporal_load(srch + at);
            }
            while (true) {
                const uint32_t jn = j0 + kStep;
                const bool more = jn < total;
                uint32_t tn = more ? __builtin_amdgcn_readfirstlane(t3_find_run(s_pre, nw, jn, lane)) : 0u;
#pragma unroll
                for (int k = 0; k < kRunsInFlight; ++k) {
                    const u32x2 x = {ew[k] & kLoMask, (ew[k] >> kSliceBits) | (eh[k] << (32 - kSliceBits))};
                    {
                        const uint32_t jb = jn + (uint32_t)k * 64, j = jb + (uint32_t)lane;
                        const uint32_t off = more ? t3_offset(s_pre, s_off, nw, tn, jb, j) : 0u;
                        const uint32_t at = more && j < total ? j + off : 0u;
                        ew[k] = __builtin_nontemporal_load(srcw + at);
                        eh[k] = __builtin_nontemporal_load(srch + at);
                    }
                    const bool h = j0 + (uint32_t)k * 64 + (uint32_t)lane < total;
                    const uint32_t both =
                        (sa[x.x >> 5] >> (x.x & 31)) & (lb[x.y >> 5] >> (x.y & 31)) & 1u;
                    const bool pend = h && !both;
                    const uint64_t ball = __ballot(pend);
                    if (pend) pq[pn + (uint32_t)__popcll(ball & ((1ull << lane) - 1ull))] = x;
                    pn += (uint32_t)__popcll(ball);
                    if (pn >= 64) {
                        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        t3_settle(pq, 64, lane, sa, lb, abase, bbase, zbits, ow, oh, cap, &s_used,
                                  st);
                        const u32x2 rest = (uint32_t)lane < pn - 64 ? pq[64 + lane] : u32x2{0u, 0u};
                        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        if ((uint32_t)lane < pn - 64) pq[lane] = rest;
                        pn -= 64;
                        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                    }
                }
                if (!more) break;
                j0 = jn;
            }
        }
        // this slice's pending entries are settled before the next slice's
        // bitmap replaces it
        if (pn) {
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            t3_settle(pq, pn, lane, sa, lb, abase, bbase, zbits, ow, oh, cap, &s_used, st);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) wgcnt[wi] = min(s_used, cap);
}

// ---- 6. the survivor hook -------------------------------------------------------------------
// Work items of kItem consecutive entries of one region: an exclusive prefix of
// the regions' item counts, then a grid-stride loop over items, each mapped to
// its region by a binary search of that prefix.
constexpr int kPackBlock = 1024;
constexpr uint32_t kItem = 1024;     // entries per work item (4 per thread)

// ipref[w] = sum over v < w of ceil(cnt[v] / kItem); ipref[nw] = total; one block.
__global__ __launch_bounds__(kPackBlock) void k_t4_scan(const uint32_t* __restrict__ cnt,
                                                        uint32_t nw, uint32_t* __restrict__ ipref) {
    __shared__ uint32_t ws[kPackBlock / 64 + 1];
    __shared__ uint32_t s_carry;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_carry = 0;
    for (uint32_t base = 0; base < nw; base += kPackBlock) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t x = i < nw ? (cnt[i] + kItem - 1) / kItem : 0u;
        uint32_t incl = x;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) ws[wave] = incl;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t run = s_carry;
            for (int w = 0; w < kPackBlock / 64; ++w) { const uint32_t t = ws[w]; ws[w] = run; run += t; }
            ws[kPackBlock / 64] = run;
        }
        __syncthreads();
        if (i < nw) ipref[i] = ws[wave] + incl - x;
        __syncthreads();
        if (threadIdx.x == 0) s_carry = ws[kPackBlock / 64];
        __syncthreads();
    }
    if (threadIdx.x == 0) ipref[nw] = s_carry;
}

// Algorithm 3's hooking loop (keys of Formula 1 as an order, path splitting)
// over the kept entries, with no bitmap: a mark is a link to z that is not in
// P, so a marked vertex cannot stand in for z here.
constexpr int kHook4Block = 256;
constexpr int kHook4EPT = (int)kItem / kHook4Block;
constexpr int kHook4Grid = 2048;     // 8 workgroups per CU

__global__ __launch_bounds__(kHook4Block) void k_t4_hook(const uint32_t* __restrict__ sw,
                                                         const uint16_t* __restrict__ sh,
                                                         const uint64_t* __restrict__ wgoff,
                                                         const uint32_t* __restrict__ cnt,
                                                         const uint32_t* __restrict__ ipref,
                                                         uint32_t nw, int nbg, uint32_t* P,
                                                         DevState* st) {
    __shared__ uint32_t s_w;
    const uint32_t z = ld_agent(&st->zroot);
    const uint32_t items = ld_agent(&ipref[nw]);
    for (uint32_t it = blockIdx.x; it < items; it += gridDim.x) {
        __syncthreads();                       // s_w of the previous item consumed
        if (threadIdx.x == 0) {
            uint32_t lo = 0, hi = nw - 1;      // last w with ipref[w] <= it
            while (lo < hi) {
                const uint32_t mid = (lo + hi + 1) / 2;
                if (ipref[mid] <= it) lo = mid; else hi = mid - 1;
            }
            s_w = lo;
        }
        __syncthreads();
        const uint32_t w = s_w;
        const uint32_t abase = (uint32_t)(w / (uint32_t)nbg) << kSliceBits;
        const uint32_t k0 = (it - ipref[w]) * kItem;
        const uint32_t c = min(cnt[w] - k0, kItem);
        const uint64_t base = wgoff[w] + k0;
        uint32_t u[kHook4EPT], v[kHook4EPT];
        bool h[kHook4EPT];
#pragma unroll
        for (int k = 0; k < kHook4EPT; ++k) {
            const uint32_t i = (uint32_t)k * kHook4Block + threadIdx.x;
            h[k] = i < c;
            const uint64_t at = base + (h[k] ? i : 0u);
            const uint32_t x = sw[at];
            u[k] = abase | (x & kLoMask);
            v[k] = pk_v1(x, sh[at]);
        }
        uint32_t pu[kHook4EPT], pv[kHook4EPT];
#pragma unroll
        for (int k = 0; k < kHook4EPT; ++k) {
            pu[k] = P[u[k]];
            pv[k] = P[v[k]];
        }
#pragma unroll
        for (int k = 0; k < kHook4EPT; ++k) {
            if (!h[k]) continue;
            if (pu[k] == pv[k] || pu[k] == v[k] || pv[k] == u[k]) continue;
            (void)t_link(P, u[k], pu[k], v[k], pv[k], z);
        }
    }
}

// ---- host side --------------------------------------------------------------------

struct TiledPlan {
    int R;
    uint64_t nch1, nch2_max;
};

static TiledPlan tiled_plan(uint64_t n, uint64_t m) {
    TiledPlan p;
    p.R = (int)((n + (1ull << kSliceBits) - 1) >> kSliceBits);
    p.nch1 = (m + kC1 - 1) / kC1;
    p.nch2_max = m / kC2 + (uint64_t)p.R + 1;
    return p;
}

// The regrouping pays from 4 slices on the plain path (ER n = 2^21, 16 entries
// per vertex: 1.04 ms regrouped against 1.79 ms direct) and from 8 with a zero
// root, whose filter drops little until the root's component is large (R-MAT
// n = 2^21: 2.3 ms regrouped against 1.5 ms direct; n = 2^22: 1.8 against 2.2).
bool tiled_eligible(uint64_t n, uint64_t m, bool zr) {
    const uint64_t R = (n + (1ull << kSliceBits) - 1) >> kSliceBits;
    return R >= (zr ? 8u : 4u) && R <= (uint64_t)kMaxSlices && m >= (1ull << 24) &&
           m < (1ull << 32);
}

static int grow(Slot* s, void** p, uint64_t* cap, uint64_t bytes, hipStream_t stream) {
    if (*cap >= bytes) return CC_OK;
    if (s->no_grow) return fail(CC_ENOMEM, "regrouped-hook scratch exceeds the fixed scratch");
    CCM_HIP(hipStreamSynchronize(stream));
    if (*p) CCM_HIP(hipFree(*p));
    *p = nullptr;
    *cap = 0;
    if (hipMalloc(p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(CC_ENOMEM, "tiled hook scratch allocation failed");
    }
    *cap = bytes;
    return CC_OK;
}

// Bytes of the regrouped hook's buffers for a COO list of m entries (with the
// zero root's warm-up taken off the front, as run_hook_tiled does); the same
// arithmetic as the layout below.
uint64_t tiled_scratch_bytes(uint64_t n, uint64_t m, bool plain) {
    const uint64_t m0 = plain ? 0 : m >> 10;
    const TiledPlan pl = tiled_plan(n, m - m0);
    const uint64_t R = (uint64_t)pl.R;
    auto al = [](uint64_t x) { return (x + 255) & ~255ull; };
    const uint64_t cap = pl.nch1 * kC1;
    const uint64_t ntile = (pl.nch1 + kScanTile - 1) / kScanTile;
    const uint64_t nbg = (R + kBPerBlock - 1) / kBPerBlock;
    const uint64_t nwg = R * nbg;
    return al(4 * cap) + al(2 * cap) + al(4 * cap) + al(cap) + al(2 * pl.nch1 * R) +
           al(4 * pl.nch1 * R) +
           al(4 * (pl.nch1 + 1) * R) + al(8 * (R + 1)) + al(4 * (R + 1)) +
           al(2 * pl.nch2_max * (R + 1)) + al(32 * pl.nch2_max) + al(4 * ntile * R) +
           al(8 * (nwg + 1)) + al(4 * nwg) + al(4 * (nwg + 1));
}

void tiled_free(TiledScratch* t) {
    if (t->buf) (void)hipFree(t->buf);
    *t = TiledScratch{};
}

int run_hook_tiled(Slot* s, uint64_t n, uint64_t m, const uint32_t* edges, uint32_t* P,
                   hipStream_t stream, bool plain, bool sym) {
    // Warm-up (zero root): the first 1/1024 of the entries go through the direct
    // hook, so the membership bitmap already holds the core of the zero root's
    // tree when the first tiles load their slices. (Measured on R-MAT-26: from
    // 1/64 to 1/4096 the step time barely moves; a longer warm-up trades its own
    // random accesses for marks the filter would otherwise set.)
    const uint64_t m0 = plain ? 0 : m >> 10;
    if (m0) {
        int rc0 = run_hook(s, n, m0, edges, P,
                           CC_F_ZROOT | CC_F_NO_TILE | kHookLinkZ | (sym ? CC_F_SYMMETRIC : 0u),
                           stream);
        if (rc0) return rc0;
        edges += 2 * m0;
        m -= m0;
    }
    const TiledPlan pl = tiled_plan(n, m);
    const int R = pl.R;
    auto al = [](uint64_t x) { return (x + 255) & ~255ull; };
    const uint64_t cap = pl.nch1 * kC1;                  // entries of each buffer
    const uint64_t b_t1w = al(4 * cap), b_t1h = al(2 * cap), b_tmp2 = al(4 * cap) + al(cap);
    const uint64_t b_seg1 = al(2 * pl.nch1 * R);
    const uint32_t ntile = (uint32_t)((pl.nch1 + kScanTile - 1) / kScanTile);
    const uint64_t b_tsum = al(4 * (uint64_t)ntile * R);
    const uint64_t b_cnt1 = al(4 * pl.nch1 * R);
    const uint64_t b_pre1 = al(4 * (pl.nch1 + 1) * R);
    const uint64_t b_base2 = al(8 * (R + 1));
    const uint64_t b_cbase = al(4 * (R + 1));
    const uint64_t b_run2 = al(2 * pl.nch2_max * (R + 1));
    const uint64_t b_desc = al(32 * pl.nch2_max);
    const uint32_t nbg = (uint32_t)((R + kBPerBlock - 1) / kBPerBlock);
    const uint32_t nwg = (uint32_t)R * nbg;
    const uint64_t b_wgoff = al(8 * ((uint64_t)nwg + 1)), b_wgcnt = al(4 * (uint64_t)nwg);
    const uint64_t b_ipref = al(4 * ((uint64_t)nwg + 1));
    const uint64_t total = b_t1w + b_t1h + b_tmp2 + b_seg1 + b_cnt1 + b_pre1 + b_base2 +
                           b_cbase + b_run2 + b_desc + b_tsum + b_wgoff + b_wgcnt + b_ipref;
    if (total != tiled_scratch_bytes(n, m0 + m, plain))
        return fail(CC_EDEVICE, "regrouped-hook scratch size mismatch (a bug)");
    int rc = grow(s, reinterpret_cast<void**>(&s->tiled.buf), &s->tiled.cap, total, stream);
    if (rc) return rc;
    char* q = s->tiled.buf;
    uint32_t* t1w = reinterpret_cast<uint32_t*>(q); q += b_t1w;
    uint16_t* t1h = reinterpret_cast<uint16_t*>(q); q += b_t1h;
    const L2Buf tmp2{reinterpret_cast<uint32_t*>(q), reinterpret_cast<uint8_t*>(q + al(4 * cap))};
    q += b_tmp2;
    uint16_t* segT = reinterpret_cast<uint16_t*>(q); q += b_seg1;
    uint32_t* cnt1 = reinterpret_cast<uint32_t*>(q); q += b_cnt1;
    uint32_t* pre1 = reinterpret_cast<uint32_t*>(q); q += b_pre1;
    uint64_t* base2 = reinterpret_cast<uint64_t*>(q); q += b_base2;
    uint32_t* cbase = reinterpret_cast<uint32_t*>(q); q += b_cbase;
    uint16_t* run2 = reinterpret_cast<uint16_t*>(q); q += b_run2;
    uint32_t* desc = reinterpret_cast<uint32_t*>(q); q += b_desc;
    uint32_t* tsum = reinterpret_cast<uint32_t*>(q); q += b_tsum;
    uint64_t* wgoff = reinterpret_cast<uint64_t*>(q); q += b_wgoff;
    uint32_t* wgcnt = reinterpret_cast<uint32_t*>(q); q += b_wgcnt;
    uint32_t* ipref = reinterpret_cast<uint32_t*>(q);
    // the survivor regions live in the level-1 buffers, free once the level-2
    // partition has read them (positions [base2[a], base2[a+1]) for slice a)
    // every kernel below reads tables the previous one wrote: coherence points between
    int rc1;
    if ((rc1 = cohere(stream))) return rc1;
    k_t1_part<<<(uint32_t)pl.nch1, kPartBlock, 0, stream>>>(edges, m, (uint32_t)n, R, pl.nch1, t1w,
                                                           t1h, segT, cnt1, s->st, sym ? 1u : 0u);
    if ((rc1 = cohere(stream))) return rc1;
    k_t1_tsum<<<(uint32_t)R * ntile, kScanBlock, 0, stream>>>(cnt1, pl.nch1, ntile, tsum);
    if ((rc1 = cohere(stream))) return rc1;
    k_t1_scan<<<(uint32_t)R * ntile, kScanBlock, 0, stream>>>(cnt1, pl.nch1, ntile, tsum, pre1);
    if ((rc1 = cohere(stream))) return rc1;
    k_t1_bases<<<1, 256, 0, stream>>>(pre1, pl.nch1, R, base2, cbase);
    if ((rc1 = cohere(stream))) return rc1;
    const uint64_t pairs = (uint64_t)R * pl.nch1;
    k_t2_bounds<<<(uint32_t)((pairs + 255) / 256), 256, 0, stream>>>(pre1, pl.nch1, R, cbase, base2,
                                                                    desc);
    if ((rc1 = cohere(stream))) return rc1;
    if (plain) {
        // the plain path hooks the level-2 chunks as they are gathered
        k_t2_hookplain<<<(uint32_t)pl.nch2_max, kPartBlock, 0, stream>>>(t1w, t1h, segT, pre1,
                                                                        pl.nch1, R, cbase, desc, P);
        CCM_HIP(hipGetLastError());
        return CC_OK;
    }
    k_t2_part<<<(uint32_t)pl.nch2_max, kPartBlock, 0, stream>>>(t1w, t1h, segT, pre1, pl.nch1, R,
                                                               cbase, desc, tmp2, run2, pl.nch2_max);
    if ((rc1 = cohere(stream))) return rc1;
    k_t3_regions<<<nwg, 256, 0, stream>>>(run2, pl.nch2_max, R, cbase, wgcnt);
    if ((rc1 = cohere(stream))) return rc1;
    k_t3_offsets<<<(uint32_t)((R + 255) / 256), 256, 0, stream>>>(wgcnt, R, base2, wgoff);
    if ((rc1 = cohere(stream))) return rc1;
    k_t3_filter<<<nwg, kHook3Block, 0, stream>>>(tmp2, run2, pl.nch2_max, R, base2, cbase,
                                                s->zbits, (n + 31) / 32, t1w, t1h, wgoff, wgcnt,
                                                s->st);
    if ((rc1 = cohere(stream))) return rc1;
    k_t4_scan<<<1, kPackBlock, 0, stream>>>(wgcnt, nwg, ipref);
    if ((rc1 = cohere(stream))) return rc1;
    k_t4_hook<<<kHook4Grid, kHook4Block, 0, stream>>>(t1w, t1h, wgoff, wgcnt, ipref, nwg, (int)nbg,
                                                      P, s->st);
    CCM_HIP(hipGetLastError());
    return CC_OK;
}

// The regrouped zero-root hook on CSR input (steps 4-6 on adj's own buckets).
int run_hook_tiled_csr(Slot* s, uint64_t n, uint64_t m, const uint64_t* off, const uint32_t* adj,
                       uint32_t* P, hipStream_t stream, bool sym) {
    const int R = (int)((n + (1ull << kSliceBits) - 1) >> kSliceBits);
    const uint64_t nch2 = m / kC2 + (uint64_t)R + 1;
    auto al = [](uint64_t x) { return (x + 255) & ~255ull; };
    const uint64_t b_sw = al(4 * m), b_sh = al(2 * m), b_tmp2 = al(4 * m) + al(m);
    const uint64_t b_base2 = al(8 * (R + 1)), b_cbase = al(4 * (R + 1));
    const uint64_t b_cfirst = al(4 * nch2), b_run2 = al(2 * nch2 * (R + 1));
    const uint32_t nbg = (uint32_t)((R + kBPerBlock - 1) / kBPerBlock);
    const uint32_t nwg = (uint32_t)R * nbg;
    const uint64_t b_wgoff = al(8 * ((uint64_t)nwg + 1)), b_wgcnt = al(4 * (uint64_t)nwg);
    const uint64_t b_ipref = al(4 * ((uint64_t)nwg + 1));
    const uint64_t total = b_sw + b_sh + b_tmp2 + b_base2 + b_cbase + b_cfirst + b_run2 + b_wgoff +
                           b_wgcnt + b_ipref;
    int rc = grow(s, reinterpret_cast<void**>(&s->tiled.buf), &s->tiled.cap, total, stream);
    if (rc) return rc;
    char* q = s->tiled.buf;
    uint32_t* sw = reinterpret_cast<uint32_t*>(q); q += b_sw;
    uint16_t* sh = reinterpret_cast<uint16_t*>(q); q += b_sh;
    const L2Buf tmp2{reinterpret_cast<uint32_t*>(q), reinterpret_cast<uint8_t*>(q + al(4 * m))};
    q += b_tmp2;
    uint64_t* base2 = reinterpret_cast<uint64_t*>(q); q += b_base2;
    uint32_t* cbase = reinterpret_cast<uint32_t*>(q); q += b_cbase;
    uint32_t* cfirst = reinterpret_cast<uint32_t*>(q); q += b_cfirst;
    uint16_t* run2 = reinterpret_cast<uint16_t*>(q); q += b_run2;
    uint64_t* wgoff = reinterpret_cast<uint64_t*>(q); q += b_wgoff;
    uint32_t* wgcnt = reinterpret_cast<uint32_t*>(q); q += b_wgcnt;
    uint32_t* ipref = reinterpret_cast<uint32_t*>(q);
    int rc1;
    if ((rc1 = cohere(stream))) return rc1;
    k_c_bases<<<1, 256, 0, stream>>>(off, n, m, R, base2, cbase);
    if ((rc1 = cohere(stream))) return rc1;
    const uint64_t gv = std::min<uint64_t>((n + 255) / 256, 8192);
    k_c_first<<<(uint32_t)gv, 256, 0, stream>>>(off, n, base2, cbase, cfirst);
    if ((rc1 = cohere(stream))) return rc1;
    k_t2_csr<<<(uint32_t)nch2, kPartBlock, 0, stream>>>(off, adj, n, R, base2, cbase, cfirst, tmp2,
                                                       run2, nch2, s->st, sym ? 1u : 0u);
    if ((rc1 = cohere(stream))) return rc1;
    k_t3_regions<<<nwg, 256, 0, stream>>>(run2, nch2, R, cbase, wgcnt);
    if ((rc1 = cohere(stream))) return rc1;
    k_t3_offsets<<<(uint32_t)((R + 255) / 256), 256, 0, stream>>>(wgcnt, R, base2, wgoff);
    if ((rc1 = cohere(stream))) return rc1;
    k_t3_filter<<<nwg, kHook3Block, 0, stream>>>(tmp2, run2, nch2, R, base2, cbase, s->zbits,
                                                (n + 31) / 32, sw, sh, wgoff, wgcnt, s->st);
    if ((rc1 = cohere(stream))) return rc1;
    k_t4_scan<<<1, kPackBlock, 0, stream>>>(wgcnt, nwg, ipref);
    if ((rc1 = cohere(stream))) return rc1;
    k_t4_hook<<<kHook4Grid, kHook4Block, 0, stream>>>(sw, sh, wgoff, wgcnt, ipref, nwg, (int)nbg,
                                                      P, s->st);
    CCM_HIP(hipGetLastError());
    return CC_OK;
}

}  // namespace ccm
