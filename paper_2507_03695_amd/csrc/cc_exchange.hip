// cc_exchange.hip — export of a share's parent array for the Reducer.
//
// Sec. III: after processing its share of the edges, a machine sends the pairs
// (v, P_v) with P_v != v; Sec. IV: members of the zero root's component are
// sent as the ID alone. Here P is the share's array after compress, and the
// two lists are written in increasing v: block b owns a contiguous range of v,
// counts its pairs and IDs (pass 1), an exclusive prefix over blocks gives each
// block its output offsets, and pass 2 writes with an order-preserving
// compaction inside the block.
#include <algorithm>

#include "cc_internal.h"

namespace ccm {

constexpr int kXBlock = 256;
constexpr int kXWaves = kXBlock / 64;
constexpr int kXRounds = 4;

__global__ __launch_bounds__(kXBlock) void k_export_count(const uint32_t* P, uint64_t n,
                                                          uint64_t span, uint32_t zroot,
                                                          uint32_t* __restrict__ cnt,
                                                          uint32_t nb) {
    __shared__ uint32_t s_p[kXWaves], s_z[kXWaves];
    const uint64_t lo = (uint64_t)blockIdx.x * span;
    const uint64_t hi = lo + span < n ? lo + span : n;
    uint32_t cp = 0, cz = 0;
    // kXRounds reads in flight per thread (one at a time would leave the pass
    // latency-bound)
    for (uint64_t v0 = lo + threadIdx.x; v0 < hi; v0 += kXRounds * kXBlock) {
        uint32_t p[kXRounds];
#pragma unroll
        for (int r = 0; r < kXRounds; ++r) {
            const uint64_t v = v0 + (uint64_t)r * kXBlock;
            p[r] = v < hi ? ld_agent(&P[v]) : (uint32_t)v;
        }
#pragma unroll
        for (int r = 0; r < kXRounds; ++r) {
            const uint64_t v = v0 + (uint64_t)r * kXBlock;
            if (v < hi && p[r] != (uint32_t)v) {
                if (p[r] == zroot) ++cz;
                else ++cp;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        cp += __shfl_xor(cp, off, 64);
        cz += __shfl_xor(cz, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        s_p[threadIdx.x >> 6] = cp;
        s_z[threadIdx.x >> 6] = cz;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tp = 0, tz = 0;
        for (int w = 0; w < kXWaves; ++w) { tp += s_p[w]; tz += s_z[w]; }
        cnt[blockIdx.x] = tp;
        cnt[nb + blockIdx.x] = tz;
    }
}

// Exclusive prefix of the two count rows (nb each) into off (nb + 1 each; the
// last entry of a row is its total). One block of 1024 threads per row.
__global__ __launch_bounds__(1024) void k_export_scan(const uint32_t* __restrict__ cnt, uint32_t nb,
                                                      uint32_t* __restrict__ off) {
    __shared__ uint32_t ws[1024 / 64 + 1];
    __shared__ uint32_t s_carry;
    const uint32_t* in = cnt + (uint64_t)blockIdx.x * nb;
    uint32_t* out = off + (uint64_t)blockIdx.x * (nb + 1);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_carry = 0;
    for (uint32_t base = 0; base < nb; base += 1024) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t x = i < nb ? in[i] : 0u;
        uint32_t incl = x;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        if (lane == 63) ws[wave] = incl;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t run = s_carry;
            for (int w = 0; w < 1024 / 64; ++w) { const uint32_t t = ws[w]; ws[w] = run; run += t; }
            ws[1024 / 64] = run;
        }
        __syncthreads();
        if (i < nb) out[i] = ws[wave] + incl - x;
        __syncthreads();
        if (threadIdx.x == 0) s_carry = ws[1024 / 64];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[nb] = s_carry;
}

__global__ __launch_bounds__(kXBlock) void k_export_write(const uint32_t* P, uint64_t n,
                                                          uint64_t span, uint32_t zroot,
                                                          const uint32_t* __restrict__ off,
                                                          uint32_t nb, uint32_t* __restrict__ pairs,
                                                          uint64_t pairs_cap,
                                                          uint32_t* __restrict__ zero_ids,
                                                          uint64_t zero_cap) {
    __shared__ uint32_t s_p[kXWaves], s_z[kXWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t lo = (uint64_t)blockIdx.x * span;
    const uint64_t hi = lo + span < n ? lo + span : n;
    uint32_t bp = off[blockIdx.x], bz = off[nb + 1 + blockIdx.x];   // running block offsets
    for (uint64_t g0 = lo; g0 < hi; g0 += kXRounds * kXBlock) {
    // the reads of kXRounds consecutive 256-vertex rounds first, then the
    // order-preserving compaction of each round in turn
    uint32_t pr[kXRounds];
#pragma unroll
    for (int r = 0; r < kXRounds; ++r) {
        const uint64_t v = g0 + (uint64_t)r * kXBlock + threadIdx.x;
        pr[r] = v < hi ? ld_agent(&P[v]) : (uint32_t)v;
    }
#pragma unroll
    for (int r = 0; r < kXRounds; ++r) {
        const uint64_t v0 = g0 + (uint64_t)r * kXBlock;
        const uint64_t v = v0 + threadIdx.x;
        const uint32_t p = pr[r];
        const bool nonroot = v < hi && p != (uint32_t)v;
        const bool fz = nonroot && p == zroot;
        const bool fp = nonroot && p != zroot;
        const uint64_t bpm = __ballot(fp), bzm = __ballot(fz);
        const uint64_t below = (1ull << lane) - 1ull;
        if (lane == 0) {
            s_p[wave] = (uint32_t)__popcll(bpm);
            s_z[wave] = (uint32_t)__popcll(bzm);
        }
        __syncthreads();
        uint32_t wp = 0, wz = 0, tp = 0, tz = 0;
        for (int w = 0; w < kXWaves; ++w) {
            if (w < wave) { wp += s_p[w]; wz += s_z[w]; }
            tp += s_p[w];
            tz += s_z[w];
        }
        // (the bounds hold whenever P did not change since the counting pass)
        if (fp) {
            const uint64_t at = (uint64_t)bp + wp + (uint32_t)__popcll(bpm & below);
            if (at < pairs_cap) {
                pairs[2 * at] = (uint32_t)v;
                pairs[2 * at + 1] = p;
            }
        }
        if (fz) {
            const uint64_t at = (uint64_t)bz + wz + (uint32_t)__popcll(bzm & below);
            if (at < zero_cap) zero_ids[at] = (uint32_t)v;
        }
        bp += tp;
        bz += tz;
        __syncthreads();                          // s_p / s_z of this chunk consumed
    }
    }
}

int run_export(Slot* s, uint64_t n, const uint32_t* P, uint32_t zroot, uint32_t* pairs,
               uint64_t pairs_cap, uint32_t* zero_ids, uint64_t zero_cap, uint64_t* n_pairs,
               uint64_t* n_zero, hipStream_t stream) {
    *n_pairs = 0;
    *n_zero = 0;
    if (n == 0) return CC_OK;
    uint64_t nb = (n + kXBlock - 1) / kXBlock;
    if (nb > kGridCap) nb = kGridCap;
    const uint64_t span = (n + nb - 1) / nb;
    nb = (n + span - 1) / span;                         // no empty trailing block
    uint32_t* cnt = s->xs;                               // 2 * kGridCap
    uint32_t* off = s->xs + 2 * kGridCap;                // 2 * (kGridCap + 1)
    int rc;
    if ((rc = cohere(stream))) return rc;
    k_export_count<<<(uint32_t)nb, kXBlock, 0, stream>>>(P, n, span, zroot, cnt, (uint32_t)nb);
    CCM_HIP(hipGetLastError());
    if ((rc = cohere(stream))) return rc;
    k_export_scan<<<2, 1024, 0, stream>>>(cnt, (uint32_t)nb, off);
    CCM_HIP(hipGetLastError());
    if ((rc = cohere(stream))) return rc;
    uint32_t tot[2] = {0, 0};
    CCM_HIP(hipMemcpyAsync(&tot[0], off + nb, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    CCM_HIP(hipMemcpyAsync(&tot[1], off + (nb + 1) + nb, sizeof(uint32_t), hipMemcpyDeviceToHost,
                           stream));
    CCM_HIP(hipStreamSynchronize(stream));
    *n_pairs = tot[0];
    *n_zero = tot[1];
    if (tot[0] > pairs_cap || tot[1] > zero_cap)
        return fail(CC_ENOMEM, "export buffers too small for the counts returned");
    if ((tot[0] && !pairs) || (tot[1] && !zero_ids)) return fail(CC_EINVAL, "NULL export buffer");
    k_export_write<<<(uint32_t)nb, kXBlock, 0, stream>>>(P, n, span, zroot, off, (uint32_t)nb, pairs,
                                                        pairs_cap, zero_ids, zero_cap);
    CCM_HIP(hipGetLastError());
    if ((rc = cohere(stream))) return rc;
    CCM_HIP(hipStreamSynchronize(stream));
    return CC_OK;
}

// ---- compact IDs (Sec. V) --------------------------------------------------------
// ID i of a list occupies bytes [i*K, i*K + K) of the stream, least significant
// byte first. Packing: one thread per 4-byte output word, which draws on at
// most four consecutive IDs; full words are one aligned store, the tail word
// byte stores. Unpacking: one thread per ID, aligned word loads, byte loads
// where a word would reach past the end of the stream.

template <int K>
__global__ __launch_bounds__(kXBlock) void k_pack_ids(const uint32_t* __restrict__ ids,
                                                      uint64_t count, uint8_t* __restrict__ out,
                                                      DevState* st) {
    const uint64_t total = count * K;
    const uint64_t words = (total + 3) / 4;
    bool bad = false;
    for (uint64_t w = (uint64_t)blockIdx.x * kXBlock + threadIdx.x; w < words;
         w += (uint64_t)gridDim.x * kXBlock) {
        const uint64_t b0 = 4 * w;
        const uint64_t i0 = b0 / K;
        // the word's bytes lie in IDs i0 .. i0 + (K + 2) / K
        constexpr int kIds = (K + 2) / K + 1;
        uint32_t x[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const uint64_t i = i0 + t;
            x[t] = (t < kIds && i < count) ? ids[i] : 0u;
        }
        if (K < 4) {
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if ((x[t] >> (8 * K)) != 0u && (i0 + t) * K >= b0 && (i0 + t) * K < b0 + 4) bad = true;
        }
        uint32_t word = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t b = b0 + j;
            const uint32_t t = (uint32_t)(b / K - i0);     // 0..3
            const uint32_t sh = 8u * (uint32_t)(b % K);
            const uint32_t v = t == 0 ? x[0] : t == 1 ? x[1] : t == 2 ? x[2] : x[3];
            word |= ((v >> sh) & 0xFFu) << (8 * j);
        }
        if (b0 + 4 <= total) {
            *reinterpret_cast<uint32_t*>(out + b0) = word;
        } else {
            for (int j = 0; b0 + j < total; ++j) out[b0 + j] = (uint8_t)(word >> (8 * j));
        }
    }
    if (bad) atomicOr(&st->status, kStatusRange);
}

template <int K>
__global__ __launch_bounds__(kXBlock) void k_unpack_ids(const uint8_t* __restrict__ in,
                                                        uint64_t count, uint32_t* __restrict__ ids) {
    const uint64_t total = count * K;
    const uint32_t mask = K == 4 ? 0xFFFFFFFFu : ((1u << (8 * K)) - 1u);
    for (uint64_t i = (uint64_t)blockIdx.x * kXBlock + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * kXBlock) {
        const uint64_t b = i * K;
        const uint64_t w0 = b / 4;
        const uint32_t off = (uint32_t)(b % 4);
        const uint64_t w1 = (b + K - 1) / 4;                 // last word touched
        uint32_t x;
        if (4 * w1 + 4 <= total) {
            const uint32_t* W = reinterpret_cast<const uint32_t*>(in);
            const uint64_t lo = W[w0];
            const uint64_t hi = (w1 != w0) ? W[w1] : 0u;
            x = (uint32_t)(((hi << 32) | lo) >> (8 * off)) & mask;
        } else {
            x = 0;
            for (int j = 0; j < K; ++j) x |= (uint32_t)in[b + j] << (8 * j);
        }
        ids[i] = x;
    }
}

int run_pack_ids(Slot* s, uint64_t count, const uint32_t* ids, uint32_t k, uint8_t* out,
                 hipStream_t stream) {
    if (!count) return CC_OK;
    const uint32_t g = (uint32_t)std::min<uint64_t>((count * k / 4 + kXBlock) / kXBlock + 1, kGridCap);
    switch (k) {
        case 1: k_pack_ids<1><<<g, kXBlock, 0, stream>>>(ids, count, out, s->st); break;
        case 2: k_pack_ids<2><<<g, kXBlock, 0, stream>>>(ids, count, out, s->st); break;
        case 3: k_pack_ids<3><<<g, kXBlock, 0, stream>>>(ids, count, out, s->st); break;
        default: k_pack_ids<4><<<g, kXBlock, 0, stream>>>(ids, count, out, s->st); break;
    }
    CCM_HIP(hipGetLastError());
    return CC_OK;
}

int run_unpack_ids(Slot* s, uint64_t count, const uint8_t* in, uint32_t k, uint32_t* ids,
                   hipStream_t stream) {
    (void)s;
    if (!count) return CC_OK;
    const uint32_t g = (uint32_t)std::min<uint64_t>((count + kXBlock - 1) / kXBlock, kGridCap);
    switch (k) {
        case 1: k_unpack_ids<1><<<g, kXBlock, 0, stream>>>(in, count, ids); break;
        case 2: k_unpack_ids<2><<<g, kXBlock, 0, stream>>>(in, count, ids); break;
        case 3: k_unpack_ids<3><<<g, kXBlock, 0, stream>>>(in, count, ids); break;
        default: k_unpack_ids<4><<<g, kXBlock, 0, stream>>>(in, count, ids); break;
    }
    CCM_HIP(hipGetLastError());
    return CC_OK;
}

}  // namespace ccm
