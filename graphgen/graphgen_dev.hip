// graphgen_dev.hip — device twin of graphgen.c for the large R-MAT inputs.
//
// Same counter-based arithmetic as the CPU generator (SplitMix64 draws keyed
// by (seed, index), integer-threshold R-MAT quadrants, the keyed permutation),
// so every entry is bit-identical to the CPU output; only the execution moves
// to the GPU. Holds no connected-components arithmetic.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t draw(uint64_t seed, uint64_t i) {
    return mix64(seed + (i + 1) * kGamma);
}

struct Perm {
    uint64_t mask;
    uint32_t shift;
    uint64_t mul[4], add[4];
};

Perm perm_make(uint32_t bits, uint64_t seed) {
    // host side: the same round keys as the CPU generator
    auto hmix = [](uint64_t z) {
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    auto hdraw = [&](uint64_t s, uint64_t i) { return hmix(s + (i + 1) * kGamma); };
    Perm p;
    p.shift = (bits + 1) / 2;
    if (p.shift == 0) p.shift = 1;
    p.mask = bits >= 64 ? ~0ull : ((1ull << bits) - 1);
    for (int r = 0; r < 4; ++r) {
        p.mul[r] = hdraw(seed, 2 * (uint64_t)r) | 1ull;
        p.add[r] = hdraw(seed, 2 * (uint64_t)r + 1);
    }
    return p;
}

__device__ __forceinline__ uint64_t perm_apply(const Perm& p, uint64_t x) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        x = (x * p.mul[r] + p.add[r]) & p.mask;
        x ^= x >> p.shift;
    }
    return x;
}

__device__ __forceinline__ void rmat_entry(uint64_t seed, uint64_t i, uint32_t scale, uint32_t t1,
                                           uint32_t t2, uint32_t t3, uint64_t* uo, uint64_t* vo) {
    uint64_t u = 0, v = 0;
    for (uint32_t l = 0; l < scale; l += 2) {
        const uint64_t r = draw(seed, i * 16 + (l >> 1));
        const uint32_t lo = (uint32_t)r, hi = (uint32_t)(r >> 32);
        u = (u << 1) | (uint64_t)(lo >= t2);
        v = (v << 1) | (uint64_t)(((lo >= t1) & (lo < t2)) | (lo >= t3));
        if (l + 1 < scale) {
            u = (u << 1) | (uint64_t)(hi >= t2);
            v = (v << 1) | (uint64_t)(((hi >= t1) & (hi < t2)) | (hi >= t3));
        }
    }
    *uo = u;
    *vo = v;
}

constexpr int kB = 256;

__global__ __launch_bounds__(kB) void k_rmat(uint32_t scale, uint64_t m, uint32_t t1, uint32_t t2,
                                             uint32_t t3, uint64_t seed, int permute, Perm p,
                                             uint32_t* out) {
    for (uint64_t i = (uint64_t)blockIdx.x * kB + threadIdx.x; i < m; i += (uint64_t)gridDim.x * kB) {
        uint64_t u, v;
        rmat_entry(seed, i, scale, t1, t2, t3, &u, &v);
        if (permute) { u = perm_apply(p, u); v = perm_apply(p, v); }
        out[2 * i] = (uint32_t)u;
        out[2 * i + 1] = (uint32_t)v;
    }
}

// Share filter, pass 1: kept-entry count of each span of `span` entries.
__global__ __launch_bounds__(kB) void k_share_count(uint32_t scale, uint64_t m, uint32_t t1,
                                                    uint32_t t2, uint32_t t3, uint64_t seed, Perm p,
                                                    uint64_t lo, uint64_t hi, uint64_t span,
                                                    uint32_t* counts) {
    __shared__ uint32_t s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const uint64_t b = (uint64_t)blockIdx.x * span;
    const uint64_t e = b + span < m ? b + span : m;
    uint32_t k = 0;
    for (uint64_t i = b + threadIdx.x; i < e; i += kB) {
        uint64_t u, v;
        rmat_entry(seed, i, scale, t1, t2, t3, &u, &v);
        u = perm_apply(p, u);
        k += (u >= lo && u < hi);
    }
    atomicAdd(&s_cnt, k);
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = s_cnt;
}

// Share filter, pass 2: order-preserving write of the kept entries of each span
// starting at offs[span] (exclusive prefix of the counts).
__global__ __launch_bounds__(kB) void k_share_write(uint32_t scale, uint64_t m, uint32_t t1,
                                                    uint32_t t2, uint32_t t3, uint64_t seed, Perm p,
                                                    uint64_t lo, uint64_t hi, uint64_t span,
                                                    const uint64_t* offs, uint32_t* out) {
    __shared__ uint32_t s_wave[kB / 64];
    uint64_t base = offs[blockIdx.x];
    const uint64_t b = (uint64_t)blockIdx.x * span;
    const uint64_t e = b + span < m ? b + span : m;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (uint64_t r0 = b; r0 < e; r0 += kB) {
        const uint64_t i = r0 + threadIdx.x;
        uint64_t u = 0, v = 0;
        bool keep = false;
        if (i < e) {
            rmat_entry(seed, i, scale, t1, t2, t3, &u, &v);
            u = perm_apply(p, u);
            keep = (u >= lo && u < hi);
        }
        const uint64_t ball = __ballot(keep);
        const uint32_t below = (uint32_t)__popcll(ball & ((1ull << lane) - 1ull));
        if (lane == 0) s_wave[wave] = (uint32_t)__popcll(ball);
        __syncthreads();
        uint32_t before = 0, total = 0;
        for (int w = 0; w < kB / 64; ++w) {
            if (w < wave) before += s_wave[w];
            total += s_wave[w];
        }
        if (keep) {
            const uint64_t at = base + before + below;
            out[2 * at] = (uint32_t)u;
            out[2 * at + 1] = (uint32_t)perm_apply(p, v);
        }
        base += total;
        __syncthreads();
    }
}

}  // namespace

extern "C" {

// R-MAT into device memory out (2*m uint32); permute != 0 relabels IDs.
int gg_dev_rmat(uint32_t scale, uint64_t m, uint32_t t1, uint32_t t2, uint32_t t3, uint64_t seed,
                uint64_t perm_seed, uint32_t* out) {
    Perm p = perm_make(scale, perm_seed);
    if (m) {
        k_rmat<<<4096, kB>>>(scale, m, t1, t2, t3, seed, perm_seed != 0, p, out);
    }
    if (hipGetLastError() != hipSuccess) return -1;
    return hipDeviceSynchronize() == hipSuccess ? 0 : -1;
}

// Share filter into device memory. counts: device scratch of ceil(m/span)
// uint32; offs: device scratch of the same number of uint64 (filled by the
// caller from counts, see graphgen.dev). Pass offs == NULL to only count.
int gg_dev_share_count(uint32_t scale, uint64_t m, uint32_t t1, uint32_t t2, uint32_t t3,
                       uint64_t seed, uint64_t perm_seed, uint64_t lo, uint64_t hi, uint64_t span,
                       uint32_t* counts) {
    Perm p = perm_make(scale, perm_seed);
    const uint64_t blocks = (m + span - 1) / span;
    if (blocks) k_share_count<<<(uint32_t)blocks, kB>>>(scale, m, t1, t2, t3, seed, p, lo, hi, span, counts);
    if (hipGetLastError() != hipSuccess) return -1;
    return hipDeviceSynchronize() == hipSuccess ? 0 : -1;
}

int gg_dev_share_write(uint32_t scale, uint64_t m, uint32_t t1, uint32_t t2, uint32_t t3,
                       uint64_t seed, uint64_t perm_seed, uint64_t lo, uint64_t hi, uint64_t span,
                       const uint64_t* offs, uint32_t* out) {
    Perm p = perm_make(scale, perm_seed);
    const uint64_t blocks = (m + span - 1) / span;
    if (blocks) k_share_write<<<(uint32_t)blocks, kB>>>(scale, m, t1, t2, t3, seed, p, lo, hi, span, offs, out);
    if (hipGetLastError() != hipSuccess) return -1;
    return hipDeviceSynchronize() == hipSuccess ? 0 : -1;
}

}  // extern "C"
