/*
 * graphgen.c — seeded synthetic graph generators (ER, R-MAT, permuted IDs,
 * isolated vertices, appended paths, batches).
 *
 * This module only produces inputs. It holds none of the connected-components
 * arithmetic: both the oracle and the GPU library consume its output, and
 * neither is linked into it.
 *
 * Randomness is counter based, so every entry is a pure function of
 * (seed, index) and generation parallelises without changing results:
 *   draw(seed, i) = the i-th output of SplitMix64 seeded with `seed`
 *                 = mix64(seed + (i + 1) * 0x9E3779B97F4A7C15)
 * where mix64 is the SplitMix64 finaliser (Steele, Lea & Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014).
 *
 * R-MAT follows Chakrabarti, Zhan & Faloutsos (SDM 2004): per edge and per
 * level one quadrant is chosen with probabilities (a, b, c, d); here the
 * cumulative probabilities arrive as 32-bit integer thresholds so that the
 * choice is an exact integer comparison.
 *
 * Vertex relabelling uses a keyed bijection on [0, 2^bits): four rounds of
 * (odd multiply + add mod 2^bits, then x ^= x >> ceil(bits/2)). Each step is
 * invertible, so the composition is a permutation; non-power-of-two ranges
 * use cycle walking.
 */
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#define GG_GAMMA 0x9E3779B97F4A7C15ull

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static inline uint64_t draw(uint64_t seed, uint64_t i) {
    return mix64(seed + (i + 1) * GG_GAMMA);
}

uint64_t gg_draw(uint64_t seed, uint64_t i) { return draw(seed, i); }

/* ---- keyed permutation on [0, 2^bits) ---- */

typedef struct {
    uint32_t bits;
    uint32_t shift;
    uint64_t mask;
    uint64_t mul[4];
    uint64_t add[4];
} perm_t;

static void perm_init(perm_t* p, uint32_t bits, uint64_t seed) {
    p->bits = bits;
    p->shift = (bits + 1) / 2;
    if (p->shift == 0) p->shift = 1;
    p->mask = bits >= 64 ? ~0ull : ((1ull << bits) - 1);
    for (int r = 0; r < 4; ++r) {
        p->mul[r] = draw(seed, 2 * (uint64_t)r) | 1ull;
        p->add[r] = draw(seed, 2 * (uint64_t)r + 1);
    }
}

static inline uint64_t perm_apply(const perm_t* p, uint64_t x) {
    for (int r = 0; r < 4; ++r) {
        x = (x * p->mul[r] + p->add[r]) & p->mask;
        x ^= x >> p->shift;
    }
    return x;
}

/* permutation of [0, n) by cycle walking on the enclosing power of two */
static inline uint64_t perm_apply_n(const perm_t* p, uint64_t x, uint64_t n) {
    do { x = perm_apply(p, x); } while (x >= n);
    return x;
}

static uint32_t ceil_log2(uint64_t n) {
    uint32_t b = 0;
    while ((1ull << b) < n) ++b;
    return b;
}

uint64_t gg_perm(uint32_t bits, uint64_t seed, uint64_t x) {
    perm_t p; perm_init(&p, bits, seed);
    return perm_apply(&p, x);
}

/* ---- Erdos-Renyi G(n, m): endpoints uniform on [0, n) ---- */

static inline void er_entry(uint64_t seed, uint64_t i, uint64_t n, uint32_t* u, uint32_t* v) {
    uint64_t r = draw(seed, i);
    *u = (uint32_t)(((r & 0xFFFFFFFFull) * n) >> 32);
    *v = (uint32_t)(((r >> 32) * n) >> 32);
}

/* out: 2*m uint32, (u_i, v_i) interleaved. n <= 2^32. */
void gg_er(uint64_t n, uint64_t m, uint64_t seed, uint32_t* out) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)m; ++i) {
        uint32_t u, v;
        er_entry(seed, (uint64_t)i, n, &u, &v);
        out[2 * i] = u;
        out[2 * i + 1] = v;
    }
}

/* ---- R-MAT ---- */

/* one R-MAT draw at `scale` levels: counter block i*16 (16 draws = 32 levels) */
static inline void rmat_entry(uint64_t seed, uint64_t i, uint32_t scale,
                              uint32_t t1, uint32_t t2, uint32_t t3,
                              uint64_t* uo, uint64_t* vo) {
    uint64_t u = 0, v = 0;
    for (uint32_t l = 0; l < scale; l += 2) {
        const uint64_t r = draw(seed, i * 16 + (l >> 1));
        const uint32_t lo = (uint32_t)r, hi = (uint32_t)(r >> 32);
        /* quadrant 0: r < t1; 1: t1 <= r < t2; 2: t2 <= r < t3; 3: r >= t3.
           u's bit is set in quadrants 2 and 3, v's in quadrants 1 and 3. */
        u = (u << 1) | (uint64_t)(lo >= t2);
        v = (v << 1) | (uint64_t)(((lo >= t1) & (lo < t2)) | (lo >= t3));
        if (l + 1 < scale) {
            u = (u << 1) | (uint64_t)(hi >= t2);
            v = (v << 1) | (uint64_t)(((hi >= t1) & (hi < t2)) | (hi >= t3));
        }
    }
    *uo = u; *vo = v;
}

/*
 * R-MAT on 2^scale vertices, m entries written to out (2*m uint32).
 * perm_seed != 0 relabels every ID through the keyed permutation.
 */
void gg_rmat(uint32_t scale, uint64_t m, uint32_t t1, uint32_t t2, uint32_t t3,
             uint64_t seed, uint64_t perm_seed, uint32_t* out) {
    perm_t p; perm_init(&p, scale, perm_seed);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)m; ++i) {
        uint64_t u, v;
        rmat_entry(seed, (uint64_t)i, scale, t1, t2, t3, &u, &v);
        if (perm_seed) { u = perm_apply(&p, u); v = perm_apply(&p, v); }
        out[2 * i] = (uint32_t)u;
        out[2 * i + 1] = (uint32_t)v;
    }
}

/*
 * One share of a vertex-range partition of a permuted R-MAT graph: of the
 * m_total generated entries keep those whose first endpoint lies in
 * [lo, hi), in generation order. Entries are generated once: each round of
 * chunks is filtered into per-chunk staging, then copied out at prefix
 * offsets. Writes at most out_cap entries; returns the number of kept
 * entries (when that exceeds out_cap, only the count is meaningful).
 */
uint64_t gg_rmat_share(uint32_t scale, uint64_t m_total, uint32_t t1, uint32_t t2, uint32_t t3,
                       uint64_t seed, uint64_t perm_seed, uint64_t lo, uint64_t hi,
                       uint32_t* out, uint64_t out_cap) {
    perm_t p; perm_init(&p, scale, perm_seed);
    const int64_t CHUNK = 1 << 18, ROUND = 256;
    const int64_t nchunks = (int64_t)((m_total + CHUNK - 1) / CHUNK);
    uint32_t* stage = (uint32_t*)malloc((size_t)ROUND * CHUNK * 2 * sizeof(uint32_t));
    if (!stage) return ~0ull;
    uint64_t total = 0;
    for (int64_t c0 = 0; c0 < nchunks; c0 += ROUND) {
        const int64_t c1 = c0 + ROUND < nchunks ? c0 + ROUND : nchunks;
        uint64_t counts[256];
        #pragma omp parallel for schedule(dynamic, 1)
        for (int64_t c = c0; c < c1; ++c) {
            const uint64_t b = (uint64_t)c * CHUNK;
            const uint64_t e = b + CHUNK < m_total ? b + CHUNK : m_total;
            uint32_t* st = stage + (size_t)(c - c0) * CHUNK * 2;
            uint64_t k = 0;
            for (uint64_t i = b; i < e; ++i) {
                uint64_t u, v;
                rmat_entry(seed, i, scale, t1, t2, t3, &u, &v);
                u = perm_apply(&p, u);
                if (u >= lo && u < hi) {
                    st[2 * k] = (uint32_t)u;
                    st[2 * k + 1] = (uint32_t)perm_apply(&p, v);
                    ++k;
                }
            }
            counts[c - c0] = k;
        }
        for (int64_t c = c0; c < c1; ++c) {
            const uint64_t k = counts[c - c0];
            if (out && total + k <= out_cap)
                memcpy(out + 2 * total, stage + (size_t)(c - c0) * CHUNK * 2, k * 2 * sizeof(uint32_t));
            total += k;
        }
    }
    free(stage);
    return total;
}

/* Append the reversed copy of every entry: out[2m..4m) = (v_i, u_i). */
void gg_symmetrise(uint64_t m, uint32_t* out) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)m; ++i) {
        out[2 * (m + i)] = out[2 * i + 1];
        out[2 * (m + i) + 1] = out[2 * i];
    }
}

/*
 * Path components: `count` paths, path p has len_p = lmin + draw(seed,p) %
 * (lmax-lmin+1) vertices with consecutive IDs starting at `base` (packed one
 * after the other). Each path's edges are written highest ID first:
 * (s+L-1, s+L-2), ..., (s+1, s). Writes starts[count] (first ID of each path)
 * and returns the number of edges written. out == NULL: count only
 * (returns edges; *n_vertices receives the vertex total).
 */
uint64_t gg_paths(uint64_t base, uint64_t count, uint32_t lmin, uint32_t lmax, uint64_t seed,
                  uint32_t* out, uint64_t* starts, uint64_t* n_vertices) {
    uint64_t s = base, k = 0, span = (uint64_t)(lmax - lmin + 1);
    for (uint64_t p = 0; p < count; ++p) {
        uint64_t len = lmin + draw(seed, p) % span;
        if (starts) starts[p] = s;
        if (out) {
            for (uint64_t j = len - 1; j >= 1; --j) {
                out[2 * k] = (uint32_t)(s + j);
                out[2 * k + 1] = (uint32_t)(s + j - 1);
                ++k;
            }
        } else {
            k += len - 1;
        }
        s += len;
    }
    if (n_vertices) *n_vertices = s - base;
    return k;
}

/*
 * Batch of graphs with local int32 IDs. For graph g: n[g] vertices, m[g]
 * entries, kind[g] (0 = ER, 1 = R-MAT), seed[g]; entries land at
 * out[2*edge_off[g] .. 2*edge_off[g+1]).
 * R-MAT graphs run at scale ceil(log2 n) and redraw an entry (next attempt
 * counter) until both endpoints are < n; IDs are then relabelled by the
 * keyed permutation of [0, n) (cycle walking).
 */
void gg_batch(uint64_t G, const int64_t* n, const int64_t* edge_off, const int32_t* kind,
              const uint64_t* seed, uint32_t t1, uint32_t t2, uint32_t t3, int32_t* out) {
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t g = 0; g < (int64_t)G; ++g) {
        uint64_t ng = (uint64_t)n[g];
        uint64_t mg = (uint64_t)(edge_off[g + 1] - edge_off[g]);
        int32_t* o = out + 2 * edge_off[g];
        if (kind[g] == 0) {
            for (uint64_t i = 0; i < mg; ++i) {
                uint32_t u, v;
                er_entry(seed[g], i, ng, &u, &v);
                o[2 * i] = (int32_t)u;
                o[2 * i + 1] = (int32_t)v;
            }
        } else {
            uint32_t sc = ceil_log2(ng);
            perm_t p; perm_init(&p, sc, mix64(seed[g] ^ 0x5045524D5045524Dull));
            for (uint64_t i = 0; i < mg; ++i) {
                uint64_t u, v;
                for (uint64_t t = 0;; ++t) {
                    /* attempt t of entry i uses its own counter block */
                    rmat_entry(seed[g], i + t * mg, sc, t1, t2, t3, &u, &v);
                    if (u < ng && v < ng) break;
                }
                u = perm_apply_n(&p, u, ng);
                v = perm_apply_n(&p, v, ng);
                o[2 * i] = (int32_t)u;
                o[2 * i + 1] = (int32_t)v;
            }
        }
    }
}
