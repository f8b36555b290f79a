// cc_kernels.hip — the single-graph path on gfx950: init, zero root, Initial
// Push, hook, compress (pointer jumping) and the zero-component relabelling.
//
// Memory model. P is one uint32 array shared by every wave of the device
// (Sec. I: one shared array per machine instead of per-core copies). Links
// are made only by device-scope compare-and-swap on a root's own entry, so
// two workers can never both hook the same root. Parent reads are ordinary
// L2-cached loads: on a multi-XCD device another XCD's L2 may hold an older
// value, but every value an entry ever holds is an ancestor of that vertex
// (an entry changes from itself to a root of smaller key when hooked, and
// afterwards only to further ancestors by path splitting), so a stale read
// walks a shorter prefix of the true path. A stale "root" is caught by the
// CAS, which fails and returns the current parent; the walk resumes there
// (Sec. II: a failed CAS repeats the root search). Splitting stores go only
// to non-roots, which no CAS can succeed on, so they never race with links.
// Every store to P is an agent-scope atomic store: plain stores have been
// observed to leave copies in the writing XCD's L2 that outlive later kernels'
// writes from other XCDs, so that a later reader on that XCD sees an old value.
#include <algorithm>

#include "cc_internal.h"

namespace ccm {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

constexpr int kBlock = 256;

// ---- keys: Formula 1's R used as an order while P stores vertex IDs ----------
// key(x) = x on the plain path; with a zero root z, key(z) = 0 and key(x) = x+1.
template <bool ZR>
__device__ __forceinline__ bool key_less(uint32_t a, uint32_t b, uint32_t z) {
    if (ZR) return (a == z) | ((b != z) & (a < b));
    return a < b;
}

// ---- init --------------------------------------------------------------------
// P_v = v (Algorithm 1 / 3 initialisation; with R the stored values stay vertex
// IDs and only the order changes). Like every store to P, a device-coherent one
// (see find_root); lanes write consecutive words, so each wave writes whole lines.
__global__ __launch_bounds__(kBlock) void k_init(uint32_t* __restrict__ P, uint64_t n,
                                                 DevState* st) {
    const uint64_t tid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    if (tid == 0) st_agent(&st->minz, kEmpty);
    for (uint64_t v = tid; v < n; v += stride) st_agent(&P[v], (uint32_t)v);
}

// ---- zero root: sampled endpoint counts in an open-addressing table ----------

__device__ __forceinline__ uint64_t sample_index(uint64_t j, uint64_t m, uint64_t K) {
    // floor(j*m/K) without 128-bit arithmetic: m = q*K + r
    const uint64_t q = m / K, r = m % K;
    return j * q + (j * r) / K;
}

__global__ __launch_bounds__(kBlock) void k_zfill(uint32_t* keys, uint32_t* counts, uint32_t T,
                                                  DevState* st) {
    uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i == 0) st_agent64(&st->zsel, 0);
    for (; i < T; i += gridDim.x * kBlock) { keys[i] = kEmpty; counts[i] = 0; }
}

__device__ __forceinline__ void table_add(uint32_t* keys, uint32_t* counts, uint32_t mask,
                                          uint32_t x) {
    uint32_t h = (x * 0x9E3779B1u) & mask;
    while (true) {
        uint32_t k = ld_agent(&keys[h]);
        if (k == kEmpty) {
            k = atomicCAS(&keys[h], kEmpty, x);
            if (k == kEmpty) k = x;
        }
        if (k == x) { atomicAdd(&counts[h], 1u); return; }
        h = (h + 1) & mask;
    }
}

__global__ __launch_bounds__(kBlock) void k_zcount(const uint32_t* __restrict__ edges, uint64_t m,
                                                   uint64_t K, uint64_t cnt, uint64_t n,
                                                   uint32_t* keys, uint32_t* counts, uint32_t mask,
                                                   DevState* st) {
    for (uint64_t j = (uint64_t)blockIdx.x * kBlock + threadIdx.x; j < cnt;
         j += (uint64_t)gridDim.x * kBlock) {
        const uint64_t i = (cnt == m) ? j : sample_index(j, m, K);
        const uint32_t u = edges[2 * i], v = edges[2 * i + 1];
        if (u >= n || v >= n) { atomicOr(&st->status, kStatusRange); continue; }
        if (u == v) continue;
        table_add(keys, counts, mask, u);
        table_add(keys, counts, mask, v);
    }
}

// Exact degree: dense counts over all entries.
__global__ __launch_bounds__(kBlock) void k_degfill(uint32_t* deg, uint64_t n, DevState* st) {
    uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i == 0) st_agent64(&st->zsel, 0);
    for (; i < n; i += (uint64_t)gridDim.x * kBlock) deg[i] = 0;
}

__global__ __launch_bounds__(kBlock) void k_degcount(const uint32_t* __restrict__ edges, uint64_t m,
                                                     uint64_t n, uint32_t* deg, DevState* st) {
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
         i += (uint64_t)gridDim.x * kBlock) {
        const uint32_t u = edges[2 * i], v = edges[2 * i + 1];
        if (u >= n || v >= n) { atomicOr(&st->status, kStatusRange); continue; }
        if (u == v) continue;
        atomicAdd(&deg[u], 1u);
        atomicAdd(&deg[v], 1u);
    }
}

__device__ __forceinline__ uint64_t pack_sel(uint32_t count, uint32_t id) {
    return count ? ((uint64_t)count << 32) | (uint64_t)(0xFFFFFFFFu - id) : 0;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t x) {
    for (int off = 32; off > 0; off >>= 1) {
        uint64_t y = __shfl_xor(x, off, 64);
        x = y > x ? y : x;
    }
    return x;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
    for (int off = 32; off > 0; off >>= 1) {
        uint32_t y = __shfl_xor(x, off, 64);
        x = y < x ? y : x;
    }
    return x;
}

// argmax over (count desc, id asc); ids come from a table (keys != nullptr) or
// are the indices of a dense count array.
// One atomic per workgroup on the packed key (atomics on one word serialise).
__global__ __launch_bounds__(kBlock) void k_zargmax(const uint32_t* keys, const uint32_t* counts,
                                                    uint64_t T, DevState* st) {
    __shared__ uint64_t s_best[kBlock / 64];
    uint64_t best = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < T;
         i += (uint64_t)gridDim.x * kBlock) {
        uint32_t id = keys ? ld_agent(&keys[i]) : (uint32_t)i;
        uint32_t c = ld_agent(&counts[i]);
        if (id != kEmpty || !keys) {
            uint64_t s = pack_sel(c, id);
            best = s > best ? s : best;
        }
    }
    best = wave_max_u64(best);
    if ((threadIdx.x & 63) == 0) s_best[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) best = s_best[w] > best ? s_best[w] : best;
        if (best) atomicMax((unsigned long long*)&st->zsel, (unsigned long long)best);
    }
}

__global__ void k_zfinish(DevState* st, int use_hint, uint32_t hint) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        uint32_t z;
        if (use_hint) z = hint;
        else {
            uint64_t s = ld_agent64(&st->zsel);
            z = s ? 0xFFFFFFFFu - (uint32_t)(s & 0xFFFFFFFFu) : 0u;
        }
        st_agent(&st->zroot, z);
    }
}

// ---- Initial Push -------------------------------------------------------------
// For sampled entries (x, z) / (z, x) with x != z: P_x = z. Every x is still a
// root (run right after init), z has the smallest key, and all writers store
// the same value, so plain stores suffice.
__global__ __launch_bounds__(kBlock) void k_push(const uint32_t* __restrict__ edges, uint64_t m,
                                                 uint64_t K, uint64_t cnt, uint64_t n,
                                                 uint32_t* P, uint32_t* zbits, DevState* st) {
    const uint32_t z = ld_agent(&st->zroot);
    for (uint64_t j = (uint64_t)blockIdx.x * kBlock + threadIdx.x; j < cnt;
         j += (uint64_t)gridDim.x * kBlock) {
        const uint64_t i = (cnt == m) ? j : sample_index(j, m, K);
        const uint32_t u = edges[2 * i], v = edges[2 * i + 1];
        if (u >= n || v >= n || u == v) continue;
        uint32_t x = kEmpty;
        if (u == z) x = v;
        else if (v == z) x = u;
        if (x != kEmpty) {
            st_agent(&P[x], z);
            atomicOr(&zbits[x >> 5], 1u << (x & 31));
        }
    }
}

// Membership bitmap of the vertices connected to the zero root: cleared, with
// only z itself set.
__global__ __launch_bounds__(kBlock) void k_zbits_clear(uint32_t* zbits, uint64_t words,
                                                        const DevState* st) {
    const uint32_t z = ld_agent(&st->zroot);
    const uint64_t zw = z >> 5;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < words;
         i += (uint64_t)gridDim.x * kBlock)
        zbits[i] = (i == zw) ? (1u << (z & 31)) : 0u;
}

// ---- hook ---------------------------------------------------------------------

// Root of x, given px = a value read from P[x]. SPLIT = 1: path splitting (each
// visited vertex takes its grandparent); SPLIT = 0: plain walk.
// The splitting writes are device-coherent stores. A plain store would leave a
// dirty line in the writing XCD's L2 whose other words are that XCD's copies;
// links are CASes performed at the memory side, which that copy does not see,
// so the line's write-back can undo a link made meanwhile in the same line (a
// whole-device batch lost links this way). Each store is issued after the next
// step's load, so that its latency overlaps the walk instead of adding to it.
template <int SPLIT>
__device__ __forceinline__ uint32_t find_root(uint32_t* P, uint32_t x, uint32_t px) {
    if (px == x) return x;
    uint32_t gp = P[px];
    while (gp != px) {
        const uint32_t ggp = P[gp];
        if (SPLIT) {
            stress_delay(x);
            st_agent(&P[x], gp);
        }
        x = px;
        px = gp;
        gp = ggp;
    }
    return px;
}

// The check before each link's CAS. Global atomics are performed at the memory
// side, past the XCD's L2, and leave the L2's copy of the word as it was; a
// walk that reads P through the L2 can therefore end at a root that has since
// been linked. A CAS on such an entry fails, but only after its round trip, and
// every CAS on one word waits for the ones before it: a giant component's
// former root collects thousands (ER n = 2^16, 2^20 entries: 16,000 CAS on one
// word, a 1.6 ms hook). The entry is read coherently first (a load, which does
// not wait behind the CASes) and a changed entry continues the walk from its
// new value; the CAS is issued only on an entry that still reads as a root.
// ER n = 2^16, 2^20 entries: 1.7 M CAS -> 0.11 M, 1.6-3.4 ms -> 0.16 ms.
// Algorithm 1 / 3 hooking of one entry whose endpoints u, v have parents pu, pv.
// Returns the root under which both endpoints ended up (the surviving root of
// the link, or the common root found). When it is the zero root z, both
// endpoints are certainly in z's tree: z has the smallest key and is never
// linked under anything. If this call's CAS is the one that links, *linked
// (when given) receives the root that was linked; the return value is then its
// new parent.
template <bool ZR, int SPLIT>
__device__ __forceinline__ uint32_t link(uint32_t* P, uint32_t u, uint32_t pu, uint32_t v,
                                         uint32_t pv, uint32_t z, uint32_t* linked = nullptr) {
    while (true) {
        const uint32_t ru = find_root<SPLIT>(P, u, pu);
        const uint32_t rv = find_root<SPLIT>(P, v, pv);
        if (ru == rv) return ru;
        const bool u_low = key_less<ZR>(ru, rv, z);
        const uint32_t hi = u_low ? rv : ru;
        const uint32_t lo = u_low ? ru : rv;
        stress_delay(hi);
        // hi's entry read coherently first (the check described above)
        const uint32_t cur = ld_agent(&P[hi]);
        if (cur != hi) {
            u = hi; pu = cur;
            v = lo; pv = lo;
            continue;
        }
        const uint32_t old = atomicCAS(&P[hi], hi, lo);
        if (old == hi) {
            if (linked) *linked = hi;
            return lo;
        }
        // hi was linked by someone else: its current parent is `old`
        u = hi; pu = old;
        v = lo; pv = lo;
    }
}

__device__ __forceinline__ bool zbit(const uint32_t* zbits, uint32_t x) {
    return (zbits[x >> 5] >> (x & 31)) & 1u;
}

// Sets x's bit. The word is read coherently first and the atomic (performed at
// the memory side, where the atomics on one word wait for each other) is issued
// only if the bit is still clear: most of a giant component's members are
// reached by many entries, and their word would otherwise take an atomic for
// each (bits only go from 0 to 1, so a set bit read anywhere stays set).
__device__ __forceinline__ void zbit_set(uint32_t* zbits, uint32_t x) {
    const uint32_t b = 1u << (x & 31);
    if (!(ld_agent(&zbits[x >> 5]) & b)) atomicOr(&zbits[x >> 5], b);
}

constexpr int kEPT = 4;  // entries per thread per tile

// SiskinCC's messages (Sec. III, Algorithm 2): every successful link appends
// (linked root, new parent) to the log. One counter update per workgroup: the
// waves' counts are summed in LDS, thread 0 reserves the block's range, and
// each lane writes its records at its rank among the block's. Records past
// cap are counted but not written (the status word reports it). Must be
// reached by every thread of the block.
__device__ __forceinline__ void log_append(const uint32_t (&child)[kEPT],
                                           const uint32_t (&parent)[kEPT], uint32_t* log,
                                           uint64_t cap, unsigned long long* count,
                                           DevState* st) {
    __shared__ uint32_t s_w[kBlock / 64];
    __shared__ unsigned long long s_base;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t mk[kEPT];
    uint32_t tot = 0;
#pragma unroll
    for (int k = 0; k < kEPT; ++k) {
        mk[k] = __ballot(child[k] != kEmpty);
        tot += (uint32_t)__popcll(mk[k]);
    }
    if (lane == 0) s_w[wave] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            const uint32_t x = s_w[w];
            s_w[w] = t;
            t += x;
        }
        s_base = t ? atomicAdd(count, (unsigned long long)t) : 0ull;
    }
    __syncthreads();
    uint64_t at = s_base + s_w[wave];
    const uint64_t below = (1ull << lane) - 1ull;
    bool full = false;
#pragma unroll
    for (int k = 0; k < kEPT; ++k) {
        if (child[k] != kEmpty) {
            const uint64_t i = at + (uint32_t)__popcll(mk[k] & below);
            if (i < cap) {
                u32x2 rec = {child[k], parent[k]};
                *reinterpret_cast<u32x2*>(log + 2 * i) = rec;
            } else {
                full = true;
            }
        }
        at += (uint32_t)__popcll(mk[k]);
    }
    if (full) atomicOr(&st->status, kStatusLogFull);
}

// Hooking of the kEPT entries (u[k], v[k]) a thread holds (entries beyond the
// input are passed as (0, 0): a self-loop, skipped); z is the zero root (ZR). Shared by the COO and the
// CSR launches. LOG (plain path only): the links made are appended to `log`
// (see log_append); every thread of the block must then call it. sym: the
// list holds every pair in both orders, so only the entries with u < v are
// hooked (each edge once; Sec. II: processing (u,v) makes (v,u) a no-op).
template <bool ZR, int SPLIT, bool LOG, bool LINKZ = false>
__device__ __forceinline__ void hook_entries(uint32_t (&u)[kEPT], uint32_t (&v)[kEPT], uint32_t n,
                                             uint32_t z, uint32_t* P, uint32_t* zbits,
                                             DevState* st, uint32_t* log, uint64_t log_cap,
                                             unsigned long long* log_count, bool sym) {
    static_assert(!(ZR && LOG), "the update log belongs to the plain path");
    bool bad = false;
#pragma unroll
    for (int k = 0; k < kEPT; ++k) {
        if (u[k] >= n || v[k] >= n) { bad = true; u[k] = v[k] = 0; }
    }
    if (bad) atomicOr(&st->status, kStatusRange);
    bool live[kEPT];
#pragma unroll
    for (int k = 0; k < kEPT; ++k) live[k] = sym ? u[k] < v[k] : u[k] != v[k];
    // A set bit means "connected to z". Both endpoints set: the entry is
    // redundant. Exactly one set: by default the entry's whole effect is to
    // connect the other endpoint to z, which its bit records (compress passes a
    // mark on to the root of its tree), so it is set and P is not touched; only
    // entries with neither endpoint marked go on to the walks. LINKZ instead
    // walks the unmarked endpoint's tree and links it under z, marking both:
    // dearer per entry, but every vertex of that tree then walks to z and is
    // marked when an entry reaches it, so the bitmap grows faster (the
    // regrouped hook's short warm-up, which seeds its filter, wants that).
    bool inu[kEPT] = {}, inv[kEPT] = {};
    if (ZR) {
        // Marking: the second endpoint's word is read coherently, so that the
        // commonest mark (first endpoint marked, second not) needs only the atomic.
        uint32_t bu[kEPT], bv[kEPT];
#pragma unroll
        for (int k = 0; k < kEPT; ++k) {
            bu[k] = live[k] ? zbits[u[k] >> 5] : 0u;
            bv[k] = !live[k] ? 0u : (LINKZ ? zbits[v[k] >> 5] : ld_agent(&zbits[v[k] >> 5]));
        }
#pragma unroll
        for (int k = 0; k < kEPT; ++k) {
            inu[k] = (bu[k] >> (u[k] & 31)) & 1u;
            inv[k] = (bv[k] >> (v[k] & 31)) & 1u;
            if (!LINKZ && live[k] && inu[k] != inv[k]) {
                if (inu[k]) atomicOr(&zbits[v[k] >> 5], 1u << (v[k] & 31));
                else zbit_set(zbits, u[k]);
            }
            live[k] = live[k] && !(inu[k] && inv[k]) && (LINKZ || (!inu[k] && !inv[k]));
        }
    }
    // LINKZ: a marked endpoint has root z (walk from z, no read of P)
    uint32_t wu[kEPT], wv[kEPT];
#pragma unroll
    for (int k = 0; k < kEPT; ++k) {
        wu[k] = (LINKZ && inu[k]) ? z : u[k];
        wv[k] = (LINKZ && inv[k]) ? z : v[k];
    }
    uint32_t pu[kEPT], pv[kEPT];
#pragma unroll
    for (int k = 0; k < kEPT; ++k) {
        pu[k] = !live[k] ? 0u : ((LINKZ && inu[k]) ? z : P[wu[k]]);
        pv[k] = !live[k] ? 0u : ((LINKZ && inv[k]) ? z : P[wv[k]]);
    }
    uint32_t child[kEPT], parent[kEPT];
#pragma unroll
    for (int k = 0; k < kEPT; ++k) {
        child[k] = kEmpty;
        parent[k] = kEmpty;
        if (!live[k]) continue;
        // a common parent, or one endpoint the parent of the other: same tree
        uint32_t r;
        if (pu[k] == pv[k]) r = pu[k];
        else if (pu[k] == wv[k]) r = wv[k];
        else if (pv[k] == wu[k]) r = wu[k];
        else r = link<ZR, SPLIT>(P, wu[k], pu[k], wv[k], pv[k], z, LOG ? &child[k] : nullptr);
        if (LOG) parent[k] = r;
        if (ZR && r == z) {
            if (!inu[k]) zbit_set(zbits, u[k]);
            if (!inv[k]) zbit_set(zbits, v[k]);
        }
    }
    if (LOG) log_append(child, parent, log, log_cap, log_count, st);
}

// One tile of kBlock*kEPT entries per workgroup; each thread loads its kEPT
// entries (coalesced, non-temporal: the edge stream must not evict P) and
// issues all their parent reads before walking any of them.
// With a zero root (ZR) the membership bitmap is consulted first: an entry
// with an endpoint known to be connected to z is settled by its bits without
// reading P (the single-GPU form of treating zero-converged vertices
// specially, Sec. IV). Bits only go from 0 to 1 and only for vertices
// connected to z, so a stale or missing bit just sends the entry down the
// ordinary path.
template <bool ZR, int SPLIT, bool LOG = false, bool LINKZ = false>
__global__ __launch_bounds__(kBlock) void k_hook(const uint32_t* __restrict__ edges, uint64_t m,
                                                 uint32_t n, uint32_t* P, uint32_t* zbits,
                                                 DevState* st, uint32_t sym,
                                                 uint32_t* log = nullptr, uint64_t log_cap = 0,
                                                 unsigned long long* log_count = nullptr) {
    const uint32_t z = ZR ? ld_agent(&st->zroot) : 0u;
    const uint64_t tile = (uint64_t)blockIdx.x * (kBlock * kEPT);
    const u32x2* E = reinterpret_cast<const u32x2*>(edges);
    uint32_t u[kEPT], v[kEPT];
#pragma unroll
    for (int k = 0; k < kEPT; ++k) {
        const uint64_t e = tile + (uint64_t)k * kBlock + threadIdx.x;
        u32x2 uv = {0u, 0u};
        if (e < m) uv = __builtin_nontemporal_load(E + e);
        u[k] = uv.x;
        v[k] = uv.y;
    }
    hook_entries<ZR, SPLIT, LOG, LINKZ>(u, v, n, z, P, zbits, st, log, log_cap, log_count,
                                        sym != 0);
}

// ---- CSR input -------------------------------------------------------------------
// Row u of a CSR graph holds the entries (u, adj[j]) for j in [off[u], off[u+1]);
// these are the same unordered pairs as a COO list, sorted by first endpoint,
// so every consecutive run of a tile shares u (and its parent reads).
// A workgroup takes kCsrTile consecutive positions and needs the row of each:
// tstart[t] is the row that holds position t*kCsrTile (written by k_csr_tiles,
// one thread per row), and the rows that start inside the tile are found by a
// sweep of the rows between the tile's first and next tile's first row plus a
// max-scan in LDS. A tile that spans more than kSweepMax rows (long runs of
// empty rows) searches each position's row instead, so no workgroup's work
// grows with the length of such runs beyond a logarithm.
constexpr int kCsrTile = kBlock * kEPT;
constexpr uint32_t kSweepMax = 4 * kCsrTile;

// Checks the offsets (non-decreasing, off[0] = 0, off[n] = m) and writes the
// first row of every tile. Indices are clamped so that invalid offsets never
// make an access leave its array; the result is then only reported.
__global__ __launch_bounds__(kBlock) void k_csr_tiles(const uint64_t* __restrict__ off, uint64_t n,
                                                      uint64_t m, uint32_t* __restrict__ tstart,
                                                      uint64_t ntiles, DevState* st) {
    bool bad = false;
    for (uint64_t v = (uint64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (uint64_t)gridDim.x * kBlock) {
        const uint64_t lo = off[v], hi = off[v + 1];
        if (hi < lo || hi > m || (v == 0 && lo != 0)) { bad = true; continue; }
        if (hi == lo) continue;
        for (uint64_t t = (lo + kCsrTile - 1) / kCsrTile; t * kCsrTile < hi && t < ntiles; ++t)
            tstart[t] = (uint32_t)v;
    }
    if (bad) atomicOr(&st->status, kStatusBadOffsets);
}

// Exact maximum degree from the row lengths (Algorithm 4 reads it from CSR),
// ties to the lowest ID: the packed (count, ~ID) key is reduced over the
// workgroup first and takes one atomic per workgroup (atomics on one word
// serialise), four rows in flight per thread.
__global__ __launch_bounds__(kBlock) void k_csr_zmax(const uint64_t* __restrict__ off, uint64_t n,
                                                     DevState* st) {
    __shared__ uint64_t s_best[kBlock / 64];
    uint64_t best = 0;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t v0 = (uint64_t)blockIdx.x * kBlock + threadIdx.x; v0 < n; v0 += 4 * stride) {
        uint64_t lo[4], hi[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint64_t v = v0 + r * stride;
            const uint64_t vs = v < n ? v : n - 1;
            lo[r] = off[vs];
            hi[r] = off[vs + 1];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint64_t v = v0 + r * stride;
            const uint64_t d = (v < n && hi[r] > lo[r]) ? hi[r] - lo[r] : 0;
            const uint64_t sel = pack_sel(d > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)d, (uint32_t)v);
            best = sel > best ? sel : best;
        }
    }
    best = wave_max_u64(best);
    if ((threadIdx.x & 63) == 0) s_best[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) best = s_best[w] > best ? s_best[w] : best;
        if (best) atomicMax((unsigned long long*)&st->zsel, (unsigned long long)best);
    }
}

__global__ void k_zsel_reset(DevState* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) st_agent64(&st->zsel, 0);
}

// Initial Push over the zero root's whole row (Algorithm 4 initial-push loop).
__global__ __launch_bounds__(kBlock) void k_csr_push(const uint64_t* __restrict__ off,
                                                     const uint32_t* __restrict__ adj, uint64_t n,
                                                     uint64_t m, uint32_t* P, uint32_t* zbits,
                                                     DevState* st) {
    const uint32_t z = ld_agent(&st->zroot);
    uint64_t lo = off[z], hi = off[z + 1];
    if (hi > m) hi = m;
    bool bad = false;
    for (uint64_t j = lo + (uint64_t)blockIdx.x * kBlock + threadIdx.x; j < hi;
         j += (uint64_t)gridDim.x * kBlock) {
        const uint32_t x = adj[j];
        if (x >= n) { bad = true; continue; }
        if (x == z) continue;
        st_agent(&P[x], z);
        zbit_set(zbits, x);
    }
    if (bad) atomicOr(&st->status, kStatusRange);
}

// Workgroup t takes tile t (a launch may cover a prefix of the tiles, as the
// warm-up does).
template <bool ZR, int SPLIT, bool LINKZ = false>
__global__ __launch_bounds__(kBlock) void k_csr_hook(const uint64_t* __restrict__ off,
                                                     const uint32_t* __restrict__ adj, uint32_t n,
                                                     uint64_t m, const uint32_t* __restrict__ tstart,
                                                     uint64_t ntiles, uint32_t* P, uint32_t* zbits,
                                                     DevState* st, uint32_t sym) {
    __shared__ uint32_t head[kCsrTile];
    __shared__ uint32_t s_wmax[kBlock / 64];
    const uint32_t z = ZR ? ld_agent(&st->zroot) : 0u;
    if (blockIdx.x >= ntiles) return;
    {
    const uint64_t t = blockIdx.x;
    const uint64_t p0 = t * kCsrTile;
    uint32_t ua = tstart[t];
    uint32_t ub = (t + 1 < ntiles) ? tstart[t + 1] : n - 1;
    if (ua >= n) ua = n - 1;                            // only with invalid offsets
    if (ub >= n || ub < ua) ub = ua;
    uint32_t v[kEPT];
#pragma unroll
    for (int k = 0; k < kEPT; ++k) {
        const uint64_t p = p0 + (uint64_t)k * kBlock + threadIdx.x;
        v[k] = p < m ? __builtin_nontemporal_load(adj + p) : 0u;
    }
    uint32_t u[kEPT];
    if (ub - ua <= kSweepMax) {
        for (int i = threadIdx.x; i < kCsrTile; i += kBlock) head[i] = 0;
        __syncthreads();
        if (threadIdx.x == 0) head[0] = ua;
        for (uint64_t x0 = (uint64_t)ua + 1; x0 <= ub; x0 += 4 * kBlock) {
            uint64_t lo[4], hi[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint64_t x = x0 + r * kBlock + threadIdx.x;
                const uint64_t xs = x <= ub ? x : ub;
                lo[r] = off[xs];
                hi[r] = off[xs + 1];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint64_t x = x0 + r * kBlock + threadIdx.x;
                if (x <= ub && lo[r] < hi[r] && lo[r] >= p0 && lo[r] < p0 + kCsrTile)
                    head[lo[r] - p0] = (uint32_t)x;
            }
        }
        __syncthreads();
        // inclusive max-scan of head: thread i owns head[4i .. 4i + 3]
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        uint32_t h[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) h[r] = head[4 * threadIdx.x + r];
#pragma unroll
        for (int r = 1; r < 4; ++r) h[r] = max(h[r], h[r - 1]);
        uint32_t incl = h[3];
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o, 64);
            if (lane >= o) incl = max(incl, y);
        }
        if (lane == 63) s_wmax[wave] = incl;
        uint32_t before = __shfl_up(incl, 1, 64);
        if (lane == 0) before = 0;
        __syncthreads();
        for (int w = 0; w < wave; ++w) before = max(before, s_wmax[w]);
#pragma unroll
        for (int r = 0; r < 4; ++r) head[4 * threadIdx.x + r] = max(h[r], before);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kEPT; ++k) u[k] = head[k * kBlock + threadIdx.x];
    } else {
        // the last row x in [ua, ub] with off[x] <= p owns p
#pragma unroll
        for (int k = 0; k < kEPT; ++k) {
            const uint64_t p = p0 + (uint64_t)k * kBlock + threadIdx.x;
            uint32_t lo = ua, hi = ub;
            while (lo < hi) {
                const uint32_t mid = lo + (hi - lo + 1) / 2;
                if (off[mid] <= p) lo = mid;
                else hi = mid - 1;
            }
            u[k] = lo;
        }
    }
#pragma unroll
    for (int k = 0; k < kEPT; ++k) {
        const uint64_t p = p0 + (uint64_t)k * kBlock + threadIdx.x;
        if (p >= m) u[k] = v[k] = 0;
    }
    hook_entries<ZR, SPLIT, false, LINKZ>(u, v, n, z, P, zbits, st, nullptr, 0, nullptr,
                                          sym != 0);
    __syncthreads();                                    // head of this tile fully used
    }
}

// ---- compress (pointer jumping) ----------------------------------------------------
// P_v <- root(v). No entry is linked any more, but another XCD's L2 can still
// hold a copy of an entry read while its vertex was a root, and that copy has
// been observed to survive into this kernel. A walk may follow such stale
// (still ancestor) values freely, but the two facts the label rests on are read
// coherently: the vertex's own entry, and the root the walk stops at (a stale
// "root" would end the walk early); if the coherent value differs, the walk
// continues from it.
// With a zero root the membership bitmap is part of the result: a set bit means
// "connected to z" (the tiled hook records such links only as bits, see
// cc_tiled.hip), so a tree that holds a marked vertex belongs to z's component.
// Here every marked vertex passes its mark on to its root; k_resolve then
// relabels the members of marked trees.
// The same pass finds the smallest member of z's component (minz, reduced over
// the blocks by k_minz). Outside z's tree every tree is rooted at its smallest
// ID (its keys are the IDs), so the candidates are: each member of z's tree
// (z included), each root whose own bit is set, and the root of each marked
// vertex. A root whose bit is set during this pass is the root of a marked
// vertex, so it is counted through that vertex.
// Each thread takes kVPT vertices per step of its grid-stride loop and issues
// their first reads together (one read in flight per thread would leave these
// whole-array passes latency-bound).
constexpr int kVPT = 4;

template <bool ZR>
__global__ __launch_bounds__(kBlock) void k_compress(uint32_t* P, uint64_t n, DevState* st,
                                                     uint32_t* zbits, uint32_t* bmin) {
    const uint32_t z = ZR ? ld_agent(&st->zroot) : 0u;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    uint32_t local_min = kEmpty;
    for (uint64_t v0 = (uint64_t)blockIdx.x * kBlock + threadIdx.x; v0 < n; v0 += kVPT * stride) {
        uint32_t pv[kVPT], bw[kVPT];
#pragma unroll
        for (int i = 0; i < kVPT; ++i) {
            const uint64_t v = v0 + i * stride;
            pv[i] = v < n ? ld_agent(&P[v]) : (uint32_t)v;
            if (ZR) bw[i] = v < n ? ld_agent(&zbits[v >> 5]) : 0u;
        }
#pragma unroll
        for (int i = 0; i < kVPT; ++i) {
        const uint64_t v = v0 + i * stride;
        const uint32_t p = pv[i];
        uint32_t r = (uint32_t)v;
        const bool marked = ZR && ((bw[i] >> (v & 31)) & 1u);
        if (ZR && v < n && p == (uint32_t)v && ((uint32_t)v == z || marked))
            local_min = min(local_min, (uint32_t)v);
        if (v < n && p != (uint32_t)v) {
            r = p;
            while (true) {
                uint32_t q = P[r];
                while (q != r) { r = q; q = P[r]; }
                if (ZR && r == z) break;          // the zero root is never linked
                q = ld_agent(&P[r]);
                if (q == r) break;
                r = q;
            }
            if (r != p) st_agent(&P[v], r);
            if (ZR && r == z) {
                local_min = min(local_min, (uint32_t)v);
            } else if (marked) {
                zbit_set(zbits, r);
                local_min = min(local_min, r);
            }
        }
        }
    }
    if (ZR) {
        // one value per block; k_minz reduces them (one atomic per block on a
        // single word would serialise)
        __shared__ uint32_t s_min[kBlock / 64];
        local_min = wave_min_u32(local_min);
        if ((threadIdx.x & 63) == 0) s_min[threadIdx.x >> 6] = local_min;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t b = s_min[0];
            for (int w = 1; w < kBlock / 64; ++w) b = min(b, s_min[w]);
            bmin[blockIdx.x] = b;
        }
    }
}

// Zero root only, after k_compress and k_minz: every member of z's component
// (its root is z, or v or its root is marked) gets the label z, or with FINAL
// the component's smallest ID minz at once (no k_canon pass needed). Marks are
// read coherently: they were set by atomics.
template <bool FINAL>
__global__ __launch_bounds__(kBlock) void k_resolve(uint32_t* P, uint64_t n, DevState* st,
                                                    const uint32_t* zbits) {
    const uint32_t z = ld_agent(&st->zroot);
    const uint32_t lab = FINAL ? ld_agent(&st->minz) : z;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t v0 = (uint64_t)blockIdx.x * kBlock + threadIdx.x; v0 < n; v0 += kVPT * stride) {
        uint32_t rr[kVPT], bv[kVPT];
#pragma unroll
        for (int i = 0; i < kVPT; ++i) {
            const uint64_t v = v0 + i * stride;
            const uint64_t vs = v < n ? v : v0;          // v0 < n
            rr[i] = ld_agent(&P[vs]);
            bv[i] = ld_agent(&zbits[vs >> 5]);
        }
#pragma unroll
        for (int i = 0; i < kVPT; ++i) {
            const uint64_t v = v0 + i * stride;
            if (v >= n) continue;
            const uint32_t r = rr[i];
            const bool inz = r == z || ((bv[i] >> (v & 31)) & 1u) ||
                             (r != (uint32_t)v && ((ld_agent(&zbits[r >> 5]) >> (r & 31)) & 1u));
            if (inz && r != lab) st_agent(&P[v], lab);
        }
    }
}

// minz = the smallest of the per-block minima (one block).
__global__ __launch_bounds__(1024) void k_minz(const uint32_t* __restrict__ bmin, uint32_t nb,
                                               DevState* st) {
    __shared__ uint32_t s_min[1024 / 64];
    uint32_t x = kEmpty;
    for (uint32_t i = threadIdx.x; i < nb; i += 1024) x = min(x, bmin[i]);
    x = wave_min_u32(x);
    if ((threadIdx.x & 63) == 0) s_min[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 1024 / 64; ++w) x = min(x, s_min[w]);
        st_agent(&st->minz, x);
    }
}

// ---- relabel the zero root's component to its smallest ID ---------------------------
__global__ __launch_bounds__(kBlock) void k_canon(uint32_t* L, uint64_t n, const DevState* st) {
    const uint32_t z = ld_agent(&st->zroot), mz = ld_agent(&st->minz);
    if (mz == z || mz == kEmpty) return;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t v0 = (uint64_t)blockIdx.x * kBlock + threadIdx.x; v0 < n; v0 += kVPT * stride) {
        uint32_t l[kVPT];
#pragma unroll
        for (int i = 0; i < kVPT; ++i) {
            const uint64_t v = v0 + i * stride;
            l[i] = v < n ? ld_agent(&L[v]) : kEmpty;
        }
#pragma unroll
        for (int i = 0; i < kVPT; ++i)
            if (l[i] == z) st_agent(&L[v0 + i * stride], mz);
    }
}

// ---- coherence point ----------------------------------------------------------------------
__global__ void k_cohere() {
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        __builtin_amdgcn_s_waitcnt(0);           // the write-back and invalidate complete here
    }
}

int cohere(hipStream_t stream) {
    // 64 single-wave workgroups: consecutive workgroups are dealt to the XCDs in
    // turn, so every XCD runs several of them.
    k_cohere<<<64, 64, 0, stream>>>();
    CCM_HIP(hipGetLastError());
    return CC_OK;
}

// ---- host-side launchers ---------------------------------------------------------------


static uint32_t grid_for(uint64_t work, uint64_t per_block, uint32_t cap) {
    uint64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return (uint32_t)(g < cap ? g : cap);
}


int run_init(Slot* s, uint64_t n, uint32_t* P, hipStream_t stream) {
    s->cur_n = n;
    s->zr_ready = false;
    k_init<<<grid_for(n, kBlock * 4, kGridCap), kBlock, 0, stream>>>(P, n, s->st);
    CCM_HIP(hipGetLastError());
    return CC_OK;
}

static uint64_t sample_count(uint64_t m, uint64_t K) { return m <= K ? m : K; }

// Size the membership bitmap for n vertices and clear it (only z set). Marks the
// slot ready for a zero-root hook when n is the current solve's.
int zbits_reset(Slot* s, uint64_t n, hipStream_t stream) {
    const uint64_t words = (n + 31) / 32;
    if (s->zbits_cap < words) {
        if (s->no_grow) return fail(CC_ENOMEM, "zero-root bitmap exceeds the fixed scratch");
        CCM_HIP(hipStreamSynchronize(stream));
        if (s->zbits) CCM_HIP(hipFree(s->zbits));
        s->zbits = nullptr;
        s->zbits_cap = 0;
        if (hipMalloc(&s->zbits, words * sizeof(uint32_t)) != hipSuccess) {
            (void)hipGetLastError();
            s->zbits = nullptr;
            return fail(CC_ENOMEM, "zero-root bitmap allocation failed");
        }
        s->zbits_cap = words;
    }
    k_zbits_clear<<<grid_for(words, kBlock, kGridCap), kBlock, 0, stream>>>(s->zbits, words, s->st);
    CCM_HIP(hipGetLastError());
    int rcc = cohere(stream);       // cleared words written back before push's atomics
    if (rcc) return rcc;
    s->zr_ready = (n == s->cur_n);
    return CC_OK;
}

int run_zroot(Slot* s, uint64_t n, uint64_t m, const uint32_t* edges, uint32_t flags,
              uint32_t hint, hipStream_t stream) {
    if (flags & CC_F_ZROOT_HINT) {
        k_zfinish<<<1, 64, 0, stream>>>(s->st, 1, hint);
        CCM_HIP(hipGetLastError());
        return zbits_reset(s, n, stream);
    }
    if (flags & CC_F_ZROOT_EXACT) {
        if (s->deg_cap < n && s->no_grow)
            return fail(CC_ENOMEM, "exact-degree counts need memory beyond the fixed scratch");
        if (s->deg_cap < n) {
            if (s->deg) CCM_HIP(hipFree(s->deg));
            s->deg = nullptr;
            s->deg_cap = 0;
            if (hipMalloc(&s->deg, n * sizeof(uint32_t)) != hipSuccess) {
                (void)hipGetLastError();
                s->deg = nullptr;
                return fail(CC_ENOMEM, "exact-degree scratch allocation failed");
            }
            s->deg_cap = n;
        }
        k_degfill<<<grid_for(n, kBlock, kGridCap), kBlock, 0, stream>>>(s->deg, n, s->st);
        int rcc = cohere(stream);   // zero-filled lines written back before the atomics
        if (rcc) return rcc;
        if (m) k_degcount<<<grid_for(m, kBlock, kGridCap), kBlock, 0, stream>>>(edges, m, n, s->deg, s->st);
        k_zargmax<<<grid_for(n, kBlock, kGridCap), kBlock, 0, stream>>>(nullptr, s->deg, n, s->st);
    } else {
        const uint64_t K = s->samples;
        const uint64_t cnt = sample_count(m, K);
        k_zfill<<<grid_for(s->table, kBlock, 1024), kBlock, 0, stream>>>(s->hkeys, s->hcounts,
                                                                          s->table, s->st);
        int rcc = cohere(stream);   // filled lines written back before the atomics
        if (rcc) return rcc;
        if (cnt)
            k_zcount<<<grid_for(cnt, kBlock, 1024), kBlock, 0, stream>>>(
                edges, m, K, cnt, n, s->hkeys, s->hcounts, s->table - 1, s->st);
        k_zargmax<<<grid_for(s->table, kBlock, 1024), kBlock, 0, stream>>>(s->hkeys, s->hcounts,
                                                                            s->table, s->st);
    }
    k_zfinish<<<1, 64, 0, stream>>>(s->st, 0, 0);
    CCM_HIP(hipGetLastError());
    return zbits_reset(s, n, stream);
}

int run_push(Slot* s, uint64_t n, uint64_t m, const uint32_t* edges, uint32_t* P,
             hipStream_t stream) {
    if (!s->zr_ready || s->cur_n != n)
        return fail(CC_EINVAL, "cc_push needs cc_init then cc_zroot on the same n");
    const uint64_t K = s->samples;
    const uint64_t cnt = sample_count(m, K);
    if (!cnt) return CC_OK;
    k_push<<<grid_for(cnt, kBlock, 1024), kBlock, 0, stream>>>(edges, m, K, cnt, n, P, s->zbits,
                                                               s->st);
    CCM_HIP(hipGetLastError());
    return CC_OK;
}

int run_hook(Slot* s, uint64_t n, uint64_t m, const uint32_t* edges, uint32_t* P,
             uint32_t flags, hipStream_t stream) {
    if (!m) return CC_OK;
    const uint64_t per = (uint64_t)kBlock * kEPT;
    const uint64_t blocks = (m + per - 1) / per;
    if (blocks > 0x7FFFFFFFull) return fail(CC_EINVAL, "edge count too large for one launch");
    const bool zr = flags & CC_F_ZROOT;
    const uint32_t sym = (flags & CC_F_SYMMETRIC) ? 1u : 0u;
    if (zr && (!s->zr_ready || s->cur_n != n))
        return fail(CC_EINVAL, "a CC_F_ZROOT hook needs cc_init then cc_zroot on the same n");
    if (!(flags & (CC_F_NO_SPLIT | CC_F_NO_TILE)) && !s->no_tiled && tiled_eligible(n, m, zr))
        return run_hook_tiled(s, n, m, edges, P, stream, /*plain=*/!zr, sym != 0);
    const bool split = split_walks(flags, n);
    const uint32_t n32 = (uint32_t)n;
    uint32_t* zb = s->zbits;
    const uint32_t g = (uint32_t)blocks;
    const bool linkz = hook_links_z(flags, n);
    if (!(flags & CC_F_NO_SPLIT) && hook_in_two_parts(n, m, split)) {
        // in two parts (whole solves, ER n = 2^16 with 2^20 entries: plain 0.150
        // -> 0.115 ms; the zero-root hook alone 0.266 -> 0.198 ms). With a zero
        // root the pass between is compress's: trees pointer-jumped and the
        // roots of marked vertices marked, which the rest of the hook reads as
        // connections to z like any other mark.
        const uint64_t m1 = m / 4;
        const uint32_t g1 = (uint32_t)((m1 + per - 1) / per);
        const uint32_t g2 = (uint32_t)((m - m1 + per - 1) / per);
        const uint32_t gn = grid_for(n, kBlock, kGridCap);
        for (int part = 0; part < 2; ++part) {
            const uint32_t* e = part ? edges + 2 * m1 : edges;
            const uint64_t mp = part ? m - m1 : m1;
            const uint32_t gp = part ? g2 : g1;
            if (!zr) k_hook<false, 0><<<gp, kBlock, 0, stream>>>(e, mp, n32, P, zb, s->st, sym);
            else if (linkz)
                k_hook<true, 0, false, true><<<gp, kBlock, 0, stream>>>(e, mp, n32, P, zb, s->st, sym);
            else k_hook<true, 0><<<gp, kBlock, 0, stream>>>(e, mp, n32, P, zb, s->st, sym);
            CCM_HIP(hipGetLastError());
            if (part) break;
            int rc = cohere(stream);
            if (rc) return rc;
            if (zr) k_compress<true><<<gn, kBlock, 0, stream>>>(P, n, s->st, zb, s->bmin);
            else k_compress<false><<<gn, kBlock, 0, stream>>>(P, n, s->st, nullptr, nullptr);
            CCM_HIP(hipGetLastError());
            if ((rc = cohere(stream))) return rc;
        }
        return CC_OK;
    }
    if (zr && linkz && split)
        k_hook<true, 1, false, true><<<g, kBlock, 0, stream>>>(edges, m, n32, P, zb, s->st, sym);
    else if (zr && linkz)
        k_hook<true, 0, false, true><<<g, kBlock, 0, stream>>>(edges, m, n32, P, zb, s->st, sym);
    else if (zr && split) k_hook<true, 1><<<g, kBlock, 0, stream>>>(edges, m, n32, P, zb, s->st, sym);
    else if (zr) k_hook<true, 0><<<g, kBlock, 0, stream>>>(edges, m, n32, P, zb, s->st, sym);
    else if (split) k_hook<false, 1><<<g, kBlock, 0, stream>>>(edges, m, n32, P, zb, s->st, sym);
    else k_hook<false, 0><<<g, kBlock, 0, stream>>>(edges, m, n32, P, zb, s->st, sym);
    CCM_HIP(hipGetLastError());
    return CC_OK;
}

int run_hook_log(Slot* s, uint64_t n, uint64_t m, const uint32_t* edges, uint32_t* P,
                 uint32_t flags, uint32_t* log, uint64_t log_cap, uint64_t* log_count,
                 hipStream_t stream) {
    if (flags & CC_F_ZROOT)
        return fail(CC_EINVAL, "the update log is defined for the plain path (no CC_F_ZROOT)");
    if (!m) return CC_OK;
    const uint64_t per = (uint64_t)kBlock * kEPT;
    const uint64_t blocks = (m + per - 1) / per;
    if (blocks > 0x7FFFFFFFull) return fail(CC_EINVAL, "edge count too large for one launch");
    const uint32_t g = (uint32_t)blocks;
    auto* cnt = reinterpret_cast<unsigned long long*>(log_count);
    const uint32_t sym = (flags & CC_F_SYMMETRIC) ? 1u : 0u;
    if (!split_walks(flags, n))
        k_hook<false, 0, true><<<g, kBlock, 0, stream>>>(edges, m, (uint32_t)n, P, nullptr, s->st,
                                                         sym, log, log_cap, cnt);
    else
        k_hook<false, 1, true><<<g, kBlock, 0, stream>>>(edges, m, (uint32_t)n, P, nullptr, s->st,
                                                         sym, log, log_cap, cnt);
    CCM_HIP(hipGetLastError());
    return CC_OK;
}

__global__ void k_log_count_reset(DevState* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) st_agent64(&st->log_count, 0ull);
}

__global__ void k_log_count_snap(DevState* st, uint64_t* host_word) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        __hip_atomic_store(host_word, ld_agent64(&st->log_count), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
}

int log_count_reset(Slot* s, hipStream_t stream) {
    k_log_count_reset<<<1, 64, 0, stream>>>(s->st);
    CCM_HIP(hipGetLastError());
    return CC_OK;
}

int log_count_snap(Slot* s, uint64_t* host_word, hipStream_t stream) {
    k_log_count_snap<<<1, 64, 0, stream>>>(s->st, host_word);
    CCM_HIP(hipGetLastError());
    return CC_OK;
}

int run_compress(Slot* s, uint64_t n, uint32_t* P, uint32_t flags, hipStream_t stream,
                 bool final_labels) {
    const uint32_t g = grid_for(n, kBlock, kGridCap);
    final_labels = final_labels || (flags & CC_F_CANON);
    if (flags & CC_F_ZROOT) {
        if (!s->zr_ready || s->cur_n != n)
            return fail(CC_EINVAL, "a CC_F_ZROOT compress needs cc_init then cc_zroot on the same n");
        k_compress<true><<<g, kBlock, 0, stream>>>(P, n, s->st, s->zbits, s->bmin);
        CCM_HIP(hipGetLastError());
        int rc = cohere(stream);
        if (rc) return rc;
        k_minz<<<1, 1024, 0, stream>>>(s->bmin, g, s->st);
        CCM_HIP(hipGetLastError());
        if ((rc = cohere(stream))) return rc;
        if (final_labels) k_resolve<true><<<g, kBlock, 0, stream>>>(P, n, s->st, s->zbits);
        else k_resolve<false><<<g, kBlock, 0, stream>>>(P, n, s->st, s->zbits);
    } else {
        k_compress<false><<<g, kBlock, 0, stream>>>(P, n, s->st, nullptr, nullptr);
    }
    CCM_HIP(hipGetLastError());
    return CC_OK;
}

// Every ids[i] is connected to target (the Reducer's zero-converged messages).
// With a zero root equal to target the link is the bitmap mark itself.
template <bool ZR, int SPLIT>
__global__ __launch_bounds__(kBlock) void k_hook_ids(const uint32_t* __restrict__ ids,
                                                     uint64_t count, uint32_t target, uint32_t n,
                                                     uint32_t* P, uint32_t* zbits, DevState* st) {
    const uint32_t z = ZR ? ld_agent(&st->zroot) : 0u;
    const bool mark = ZR && target == z;
    bool bad = false;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * kBlock) {
        const uint32_t x = ids[i];
        if (x >= n) { bad = true; continue; }
        if (x == target) continue;
        if (mark) {
            zbit_set(zbits, x);
            continue;
        }
        const uint32_t px = P[x], pt = P[target];
        if (px == pt || px == target || pt == x) continue;
        (void)link<ZR, SPLIT>(P, x, px, target, pt, z);
    }
    if (bad) atomicOr(&st->status, kStatusRange);
}

int run_hook_ids(Slot* s, uint64_t n, uint64_t count, const uint32_t* ids, uint32_t target,
                 uint32_t* P, uint32_t flags, hipStream_t stream) {
    const bool zr = flags & CC_F_ZROOT;
    const bool split = split_walks(flags, n);
    if (zr && (!s->zr_ready || s->cur_n != n))
        return fail(CC_EINVAL, "a CC_F_ZROOT id hook needs cc_init then cc_zroot on the same n");
    const uint32_t g = grid_for(count, kBlock, kGridCap);
    const uint32_t n32 = (uint32_t)n;
    if (zr && split) k_hook_ids<true, 1><<<g, kBlock, 0, stream>>>(ids, count, target, n32, P, s->zbits, s->st);
    else if (zr) k_hook_ids<true, 0><<<g, kBlock, 0, stream>>>(ids, count, target, n32, P, s->zbits, s->st);
    else if (split) k_hook_ids<false, 1><<<g, kBlock, 0, stream>>>(ids, count, target, n32, P, s->zbits, s->st);
    else k_hook_ids<false, 0><<<g, kBlock, 0, stream>>>(ids, count, target, n32, P, s->zbits, s->st);
    CCM_HIP(hipGetLastError());
    return CC_OK;
}

int run_canon(Slot* s, uint64_t n, uint32_t* L, hipStream_t stream) {
    k_canon<<<grid_for(n, kBlock, kGridCap), kBlock, 0, stream>>>(L, n, s->st);
    CCM_HIP(hipGetLastError());
    return CC_OK;
}

int run_solve_csr(Slot* s, uint64_t n, uint64_t m, const uint64_t* off, const uint32_t* adj,
                  uint32_t* L, uint32_t flags, uint32_t hint, hipStream_t stream) {
    if (n == 0) return CC_OK;
    int rc;
    const bool zr = flags & CC_F_ZROOT;
    const bool split = split_walks(flags, n);
    const uint32_t sym = (flags & CC_F_SYMMETRIC) ? 1u : 0u;
    const uint64_t ntiles = (m + kCsrTile - 1) / kCsrTile;
    if (ntiles > 0x7FFFFFFFull) return fail(CC_EINVAL, "entry count too large for one launch");
    if (s->csr_tiles_cap < ntiles + 1) {
        CCM_HIP(hipStreamSynchronize(stream));
        if (s->csr_tiles) CCM_HIP(hipFree(s->csr_tiles));
        s->csr_tiles = nullptr;
        s->csr_tiles_cap = 0;
        if (hipMalloc(&s->csr_tiles, (ntiles + 1) * sizeof(uint32_t)) != hipSuccess) {
            (void)hipGetLastError();
            s->csr_tiles = nullptr;
            return fail(CC_ENOMEM, "CSR tile table allocation failed");
        }
        s->csr_tiles_cap = ntiles + 1;
    }
    if ((rc = run_init(s, n, L, stream))) return rc;
    const uint32_t gn = grid_for(n, kBlock, kGridCap);
    k_csr_tiles<<<gn, kBlock, 0, stream>>>(off, n, m, s->csr_tiles, ntiles, s->st);
    CCM_HIP(hipGetLastError());
    if (zr) {
        if (flags & CC_F_ZROOT_HINT) {
            k_zfinish<<<1, 64, 0, stream>>>(s->st, 1, hint);
        } else {
            k_zsel_reset<<<1, 64, 0, stream>>>(s->st);
            if ((rc = cohere(stream))) return rc;
            k_csr_zmax<<<grid_for(n, 4 * kBlock, 2048), kBlock, 0, stream>>>(off, n, s->st);
            if ((rc = cohere(stream))) return rc;
            k_zfinish<<<1, 64, 0, stream>>>(s->st, 0, 0);
        }
        CCM_HIP(hipGetLastError());
        if ((rc = zbits_reset(s, n, stream))) return rc;
        k_csr_push<<<64, kBlock, 0, stream>>>(off, adj, n, m, L, s->zbits, s->st);
        CCM_HIP(hipGetLastError());
    }
    if ((rc = cohere(stream))) return rc;
    if (zr && !(flags & (CC_F_NO_SPLIT | CC_F_NO_TILE)) && tiled_eligible(n, m, true)) {
        // as on COO input: a warm-up over the first 1/1024 of the tiles seeds the
        // bitmap, then the regrouped hook covers every position (the warm-up's
        // entries again too, which finds them joined)
        const uint64_t w = ntiles >> 10;
        if (w) {
            k_csr_hook<true, 1, true><<<(uint32_t)w, kBlock, 0, stream>>>(
                off, adj, (uint32_t)n, m, s->csr_tiles, ntiles, L, s->zbits, s->st, sym);
            CCM_HIP(hipGetLastError());
        }
        if ((rc = run_hook_tiled_csr(s, n, m, off, adj, L, stream, sym != 0))) return rc;
    } else if (ntiles) {
        const uint32_t g = (uint32_t)ntiles;
        const uint32_t n32 = (uint32_t)n;
        uint32_t* zb = s->zbits;
        const uint32_t* ts = s->csr_tiles;
        const bool linkz = hook_links_z(flags, n);
        if (zr && linkz && split)
            k_csr_hook<true, 1, true><<<g, kBlock, 0, stream>>>(off, adj, n32, m, ts, ntiles, L, zb, s->st, sym);
        else if (zr && linkz)
            k_csr_hook<true, 0, true><<<g, kBlock, 0, stream>>>(off, adj, n32, m, ts, ntiles, L, zb, s->st, sym);
        else if (zr && split) k_csr_hook<true, 1><<<g, kBlock, 0, stream>>>(off, adj, n32, m, s->csr_tiles, ntiles, L, zb, s->st, sym);
        else if (zr) k_csr_hook<true, 0><<<g, kBlock, 0, stream>>>(off, adj, n32, m, s->csr_tiles, ntiles, L, zb, s->st, sym);
        else if (split) k_csr_hook<false, 1><<<g, kBlock, 0, stream>>>(off, adj, n32, m, s->csr_tiles, ntiles, L, zb, s->st, sym);
        else k_csr_hook<false, 0><<<g, kBlock, 0, stream>>>(off, adj, n32, m, s->csr_tiles, ntiles, L, zb, s->st, sym);
        CCM_HIP(hipGetLastError());
    }
    if ((rc = cohere(stream))) return rc;
    if ((rc = run_compress(s, n, L, flags, stream, true))) return rc;
    return cohere(stream);
}

static uint64_t al256(uint64_t x) { return (x + 255) & ~255ull; }

uint64_t solve_scratch_bytes(uint64_t n, uint64_t m, uint32_t flags) {
    const bool zr = flags & CC_F_ZROOT;
    uint64_t b = 0;
    if (zr) b += al256(4 * ((n + 31) / 32));
    if (zr && (flags & CC_F_ZROOT_EXACT)) b += al256(4 * n);
    if (m && !(flags & (CC_F_NO_SPLIT | CC_F_NO_TILE)) && tiled_eligible(n, m, zr))
        b += al256(tiled_scratch_bytes(n, m, !zr));
    return b;
}

void slot_lend_scratch(Slot* s, char* block, uint64_t n, uint64_t m, uint32_t flags,
                       LentScratch* saved) {
    saved->zbits = s->zbits;
    saved->zbits_cap = s->zbits_cap;
    saved->deg = s->deg;
    saved->deg_cap = s->deg_cap;
    saved->tiled = s->tiled;
    const bool zr = flags & CC_F_ZROOT;
    char* q = block;
    s->zbits = nullptr;
    s->zbits_cap = 0;
    s->deg = nullptr;
    s->deg_cap = 0;
    s->tiled = TiledScratch{};
    if (zr) {
        const uint64_t words = (n + 31) / 32;
        s->zbits = reinterpret_cast<uint32_t*>(q);
        s->zbits_cap = words;
        q += al256(4 * words);
    }
    if (zr && (flags & CC_F_ZROOT_EXACT)) {
        s->deg = reinterpret_cast<uint32_t*>(q);
        s->deg_cap = n;
        q += al256(4 * n);
    }
    if (m && !(flags & (CC_F_NO_SPLIT | CC_F_NO_TILE)) && tiled_eligible(n, m, zr)) {
        s->tiled.buf = q;
        s->tiled.cap = tiled_scratch_bytes(n, m, !zr);
    }
    s->no_grow = true;
}

void slot_return_scratch(Slot* s, const LentScratch* saved) {
    s->zbits = saved->zbits;
    s->zbits_cap = saved->zbits_cap;
    s->deg = saved->deg;
    s->deg_cap = saved->deg_cap;
    s->tiled = saved->tiled;
    s->no_grow = false;
    s->zr_ready = false;
}

int run_solve(Slot* s, uint64_t n, uint64_t m, const uint32_t* edges, uint32_t* L,
              uint32_t flags, uint32_t hint, hipStream_t stream) {
    if (n == 0) return CC_OK;
    int rc;
    if ((rc = run_init(s, n, L, stream))) return rc;
    if (flags & CC_F_ZROOT) {
        if ((rc = run_zroot(s, n, m, edges, flags, hint, stream))) return rc;
        if ((rc = run_push(s, n, m, edges, L, stream))) return rc;
    }
    if ((rc = cohere(stream))) return rc;
    if ((rc = run_hook(s, n, m, edges, L, flags, stream))) return rc;
    if ((rc = cohere(stream))) return rc;
    if ((rc = run_compress(s, n, L, flags, stream, true))) return rc;
    return cohere(stream);
}

}  // namespace ccm
