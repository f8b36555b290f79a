// cc_exchange.hip — export of a share's parent array for the Reducer.
//
// Sec. III: after processing its share of the edges, a machine sends the pairs
// (v, P_v) with P_v != v; Sec. IV: members of the zero root's component are
// sent as the ID alone. Here P is the share's array after compress, and the
// two lists are written in increasing v: block b owns a contiguous range of v,
// counts its pairs and IDs (pass 1), an exclusive prefix over blocks gives each
// block its output offsets, and pass 2 writes with an order-preserving
// compaction inside the block.
#include "cc_internal.h"

namespace ccm {

constexpr int kXBlock = 256;
constexpr int kXWaves = kXBlock / 64;

__global__ __launch_bounds__(kXBlock) void k_export_count(const uint32_t* P, uint64_t n,
                                                          uint64_t span, uint32_t zroot,
                                                          uint32_t* __restrict__ cnt,
                                                          uint32_t nb) {
    __shared__ uint32_t s_p[kXWaves], s_z[kXWaves];
    const uint64_t lo = (uint64_t)blockIdx.x * span;
    const uint64_t hi = lo + span < n ? lo + span : n;
    uint32_t cp = 0, cz = 0;
    for (uint64_t v = lo + threadIdx.x; v < hi; v += kXBlock) {
        const uint32_t p = ld_agent(&P[v]);
        if (p != (uint32_t)v) {
            if (p == zroot) ++cz;
            else ++cp;
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
    for (uint64_t v0 = lo; v0 < hi; v0 += kXBlock) {
        const uint64_t v = v0 + threadIdx.x;
        uint32_t p = (uint32_t)v;
        if (v < hi) p = ld_agent(&P[v]);
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

}  // namespace ccm
