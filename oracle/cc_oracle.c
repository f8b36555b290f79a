/*
 * cc_oracle.c — sequential CPU oracle for connected-components labelling.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * bench's CPU-baseline leg load this file; the GPU library never links it,
 * and this file includes nothing from the GPU library.
 *
 * What the labelling path computes has a plain definition (Sec. II,
 * "Terminology"): L maps each vertex to its component, L_u == L_v iff u and v
 * are connected, edges being unordered pairs. Jayanti-Tarjan with link by
 * index identifies each component by its lowest vertex ID (Sec. II, text
 * after Algorithm 1), so the unique target is
 *      L_v = min { u : u is connected to v }.
 * oracle_cc_labels computes exactly that with a deliberately different
 * method from the GPU path: union by size with full path compression (so it
 * never relies on the min-ID linking rule under test), then a separate pass
 * that takes the minimum ID per set.
 *
 * The remaining functions write out the other deterministic steps:
 *   - oracle_zroot:   the zero root (Sec. IV, Zero Planting; Algorithm 4,
 *                     max_degree): the vertex with the most endpoint
 *                     occurrences among sampled non-self-loop entries,
 *                     ties to the lowest ID.
 *   - oracle_push:    the parent array after initialisation and the Initial
 *                     Push (Sec. II Thrifty paragraph; Algorithm 4
 *                     initial-push loop): sampled neighbours of the zero root
 *                     point at it.
 *   - oracle_jt_seq:  Algorithm 1 run sequentially over a prefix of the
 *                     entries, for the worked example of Fig. 1.
 *   - oracle_siskin_log: the messages one SiskinCC machine sends (Sec. III,
 *                     Algorithm 2): Algorithm 1 on one thread, recording
 *                     (child, new parent) at every link.
 *   - oracle_rf_jt:   Algorithm 3 with the root function R (Formulas 1-2),
 *                     run sequentially, returning the final P (root values).
 *   - oracle_check_forest: structural checks on a parent array taken after
 *                     hooking (a forest whose parents have smaller keys).
 *
 * Status codes: 0 ok, -1 invalid argument, -2 some endpoint >= n,
 * -3 out of memory.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ERANGE (-2)
#define OR_ENOMEM (-3)

/* ---- union-find (union by size, full path compression) ---- */

static uint32_t uf_find(uint32_t* parent, uint32_t x) {
    uint32_t r = x;
    while (parent[r] != r) r = parent[r];
    while (parent[x] != r) {          /* second pass: point the path at r */
        uint32_t next = parent[x];
        parent[x] = r;
        x = next;
    }
    return r;
}

static void uf_union(uint32_t* parent, uint32_t* size, uint32_t a, uint32_t b) {
    uint32_t ra = uf_find(parent, a), rb = uf_find(parent, b);
    if (ra == rb) return;
    /* larger set becomes the parent; equal sizes: smaller index wins */
    if (size[ra] < size[rb] || (size[ra] == size[rb] && rb < ra)) {
        uint32_t t = ra; ra = rb; rb = t;
    }
    parent[rb] = ra;
    size[ra] += size[rb];
}

/*
 * Labels for an undirected graph given as m unordered pairs (u_i, v_i),
 * edges[2i], edges[2i+1], IDs < n. Self-loops and repeated pairs are allowed.
 * L receives n labels: L_v = the smallest ID in v's component.
 */
int oracle_cc_labels(uint64_t n, uint64_t m, const uint32_t* edges, uint32_t* L) {
    if (n > 0xFFFFFFFFull) return OR_EINVAL;
    if (n == 0) return m == 0 ? OR_OK : OR_ERANGE;
    for (uint64_t i = 0; i < 2 * m; ++i)
        if (edges[i] >= n) return OR_ERANGE;
    uint32_t* parent = (uint32_t*)malloc(n * sizeof(uint32_t));
    uint32_t* size = (uint32_t*)malloc(n * sizeof(uint32_t));
    if (!parent || !size) { free(parent); free(size); return OR_ENOMEM; }
    for (uint64_t v = 0; v < n; ++v) { parent[v] = (uint32_t)v; size[v] = 1; }
    for (uint64_t i = 0; i < m; ++i)
        uf_union(parent, size, edges[2 * i], edges[2 * i + 1]);
    /* minimum ID per set: visit vertices in increasing order, the first
       member seen of each set is its minimum */
    uint32_t* minid = size;                    /* reuse: sizes are no longer needed */
    for (uint64_t v = 0; v < n; ++v) minid[v] = 0xFFFFFFFFu;
    for (uint64_t v = 0; v < n; ++v) {
        uint32_t r = uf_find(parent, (uint32_t)v);
        if (minid[r] == 0xFFFFFFFFu) minid[r] = (uint32_t)v;
    }
    for (uint64_t v = 0; v < n; ++v) L[v] = minid[uf_find(parent, (uint32_t)v)];
    free(parent); free(size);
    return OR_OK;
}

/* number of distinct labels in a labelling where each label is a vertex ID */
uint64_t oracle_count_labels(uint64_t n, const uint32_t* L) {
    uint64_t c = 0;
    for (uint64_t v = 0; v < n; ++v) c += (L[v] == v);
    return c;
}

/*
 * Batch: G graphs with local int32 IDs. Graph g has vertices
 * [vtx_off[g], vtx_off[g+1]) and entries edges[2*edge_off[g] .. 2*edge_off[g+1]).
 * L (int32) receives local min-ID labels; status[g] the per-graph code.
 */
int oracle_cc_labels_batch(uint64_t G, const int64_t* vtx_off, const int64_t* edge_off,
                           const int32_t* edges, int32_t* L, int32_t* status) {
    for (uint64_t g = 0; g < G; ++g) {
        int64_t n = vtx_off[g + 1] - vtx_off[g];
        int64_t m = edge_off[g + 1] - edge_off[g];
        if (n < 0 || m < 0) return OR_EINVAL;
        status[g] = oracle_cc_labels((uint64_t)n, (uint64_t)m,
                                     (const uint32_t*)(edges + 2 * edge_off[g]),
                                     (uint32_t*)(L + vtx_off[g]));
    }
    return OR_OK;
}

/*
 * Zero root: the sample is entries i_j = floor(j*m/K), j = 0..K-1 when m > K,
 * else every entry. Count, for every vertex, its endpoint occurrences in the
 * sampled entries that are not self-loops; the zero root is the vertex with
 * the largest count, ties to the lowest ID; with no counted occurrence it is
 * vertex 0. K == 0 means every entry (the exact degree).
 */
int oracle_zroot(uint64_t n, uint64_t m, const uint32_t* edges, uint64_t K, uint32_t* zmax) {
    if (n == 0 || n > 0xFFFFFFFFull) return OR_EINVAL;
    uint64_t cnt = (K == 0 || m <= K) ? m : K;
    uint32_t* deg = (uint32_t*)calloc(n, sizeof(uint32_t));
    if (!deg) return OR_ENOMEM;
    for (uint64_t j = 0; j < cnt; ++j) {
        uint64_t i = (cnt == m) ? j : (uint64_t)(((unsigned __int128)j * m) / K);
        uint32_t u = edges[2 * i], v = edges[2 * i + 1];
        if (u >= n || v >= n) { free(deg); return OR_ERANGE; }
        if (u == v) continue;
        deg[u]++; deg[v]++;
    }
    uint32_t best = 0;
    for (uint64_t v = 1; v < n; ++v)
        if (deg[v] > deg[best]) best = (uint32_t)v;
    free(deg);
    *zmax = best;
    return OR_OK;
}

/*
 * Parent array after initialisation (P_v = v) and the Initial Push from zmax:
 * for every sampled entry (same sample as oracle_zroot) with exactly one
 * endpoint equal to zmax, the other endpoint x gets P_x = zmax.
 */
int oracle_push(uint64_t n, uint64_t m, const uint32_t* edges, uint64_t K, uint32_t zmax,
                uint32_t* P) {
    if (n == 0 || n > 0xFFFFFFFFull || zmax >= n) return OR_EINVAL;
    for (uint64_t v = 0; v < n; ++v) P[v] = (uint32_t)v;
    uint64_t cnt = (K == 0 || m <= K) ? m : K;
    for (uint64_t j = 0; j < cnt; ++j) {
        uint64_t i = (cnt == m) ? j : (uint64_t)(((unsigned __int128)j * m) / K);
        uint32_t u = edges[2 * i], v = edges[2 * i + 1];
        if (u >= n || v >= n) return OR_ERANGE;
        if (u == v) continue;
        if (u == zmax) P[v] = zmax;
        else if (v == zmax) P[u] = zmax;
    }
    return OR_OK;
}

/*
 * Algorithm 1 (Jayanti-Tarjan CC) executed by one thread: initialise P_v = v,
 * then hook the first `steps` entries in order (each: walk both endpoints to
 * their roots, stop if equal, otherwise the root with the greater ID takes
 * the smaller as parent). If `jump` is nonzero, finish with pointer jumping
 * (each P_v replaced by its root). With one thread every CAS succeeds, so the
 * retry loop never repeats.
 */
int oracle_jt_seq(uint64_t n, uint64_t m, const uint32_t* edges, uint64_t steps, int jump,
                  uint32_t* P) {
    if (n > 0xFFFFFFFFull) return OR_EINVAL;
    if (steps > m) steps = m;
    for (uint64_t v = 0; v < n; ++v) P[v] = (uint32_t)v;
    for (uint64_t i = 0; i < steps; ++i) {
        uint32_t u = edges[2 * i], v = edges[2 * i + 1];
        if (u >= n || v >= n) return OR_ERANGE;
        while (P[u] != u) u = P[u];
        while (P[v] != v) v = P[v];
        if (u == v) continue;
        if (u < v) P[v] = u; else P[u] = v;
    }
    if (jump) {
        for (uint64_t v = 0; v < n; ++v) {
            uint32_t r = (uint32_t)v;
            while (P[r] != r) r = P[r];
            P[v] = r;
        }
    }
    return OR_OK;
}

/*
 * SiskinCC's update messages (Sec. III, Algorithm 2), one machine, one thread.
 * Each entry is processed as in Algorithm 1; whenever the root with the greater
 * ID is given the smaller root as its parent, the pair (that root, its new
 * parent) is a message to the Reducer, recorded in processing order. Non-roots
 * are never changed, so every vertex appears as a child at most once and the
 * messages number n minus the number of components of the processed entries.
 * Writes min(count, cap) pairs to log (2 uint32 each) and the full count to
 * *count; returns -3 when count > cap.
 */
int oracle_siskin_log(uint64_t n, uint64_t m, const uint32_t* edges, uint32_t* log, uint64_t cap,
                      uint64_t* count) {
    if (n > 0xFFFFFFFFull) return OR_EINVAL;
    uint32_t* P = (uint32_t*)malloc((n ? n : 1) * sizeof(uint32_t));
    if (!P) return OR_ENOMEM;
    for (uint64_t v = 0; v < n; ++v) P[v] = (uint32_t)v;
    uint64_t k = 0;
    for (uint64_t i = 0; i < m; ++i) {
        uint32_t u = edges[2 * i], v = edges[2 * i + 1];
        if (u >= n || v >= n) { free(P); *count = k; return OR_ERANGE; }
        while (P[u] != u) u = P[u];
        while (P[v] != v) v = P[v];
        if (u == v) continue;
        const uint32_t child = u < v ? v : u, parent = u < v ? u : v;
        P[child] = parent;
        if (k < cap) { log[2 * k] = child; log[2 * k + 1] = parent; }
        ++k;
    }
    free(P);
    *count = k;
    return k > cap ? OR_ENOMEM : OR_OK;
}

/*
 * Algorithm 3 (Root-Function JT CC) with RobinCC's R (Formula 1):
 * R_v = 0 for v == zmax, else v + 1; R^{-1} (Formula 2): 0 -> zmax, c -> c-1.
 * P holds root values; v is a root iff P_v == R_v. Executed by one thread
 * over all entries, then pointer jumping through R^{-1}. Output P (n entries,
 * as uint64 because R reaches n) holds, for every v, the root value of v's
 * component: 0 for zmax's component, (root ID + 1) for the others.
 */
static inline uint64_t R_of(uint64_t v, uint64_t z) { return v == z ? 0 : v + 1; }
static inline uint64_t Rinv(uint64_t c, uint64_t z) { return c == 0 ? z : c - 1; }

int oracle_rf_jt(uint64_t n, uint64_t m, const uint32_t* edges, uint32_t zmax, uint64_t* P) {
    if (n == 0 || n > 0xFFFFFFFFull || zmax >= n) return OR_EINVAL;
    for (uint64_t v = 0; v < n; ++v) P[v] = R_of(v, zmax);
    for (uint64_t i = 0; i < m; ++i) {
        uint64_t u = edges[2 * i], v = edges[2 * i + 1];
        if (u >= n || v >= n) return OR_ERANGE;
        while (P[u] != R_of(u, zmax)) u = Rinv(P[u], zmax);
        while (P[v] != R_of(v, zmax)) v = Rinv(P[v], zmax);
        if (u == v) continue;
        if (R_of(u, zmax) < R_of(v, zmax)) P[v] = R_of(u, zmax);
        else P[u] = R_of(v, zmax);
    }
    for (uint64_t v = 0; v < n; ++v) {
        uint64_t u = v;
        while (P[u] != R_of(u, zmax)) u = Rinv(P[u], zmax);
        P[v] = P[u];
    }
    return OR_OK;
}

/*
 * Structural checks on a parent array P (vertex IDs) taken after hooking.
 * key(x) = x on the plain path; with zroot_on, key(zmax) = 0 and
 * key(x) = x + 1 otherwise. Checks that every P_x < n and that every
 * non-root has a parent of strictly smaller key (so P is a forest).
 * Returns the number of roots (P_x == x), or -1 if a check fails
 * (*bad receives the first failing vertex).
 */
int64_t oracle_check_forest(uint64_t n, const uint32_t* P, int zroot_on, uint32_t zmax,
                            uint64_t* bad) {
    int64_t roots = 0;
    for (uint64_t x = 0; x < n; ++x) {
        uint64_t p = P[x];
        if (p >= n) { *bad = x; return -1; }
        if (p == x) { ++roots; continue; }
        uint64_t kx = zroot_on ? R_of(x, zmax) : x;
        uint64_t kp = zroot_on ? R_of(p, zmax) : p;
        if (!(kp < kx)) { *bad = x; return -1; }
    }
    return roots;
}
