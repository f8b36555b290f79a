"""Pins for the CPU oracle: brute force, BFS, a library routine, closed forms,
the worked example of Fig. 1 and the properties of Algorithm 3 with R.

None of these re-derives the oracle's own code: each check computes the
expected value by an independent route (transitive closure, breadth-first
search, scipy's connected_components, hand-built graphs with known answers).
"""
import itertools
import os
from collections import deque

import numpy as np
import pytest

import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---- independent references -------------------------------------------------

def closure_labels(n, edges):
    """L_v = min{u : reach(u, v)} from the boolean reachability closure."""
    R = np.eye(n, dtype=bool)
    for u, v in edges:
        R[u, v] = R[v, u] = True
    for k in range(n):                       # Warshall
        R |= R[:, k:k + 1] & R[k:k + 1, :]
    return np.array([int(np.flatnonzero(R[:, v])[0]) for v in range(n)], dtype=np.uint32)


def bfs_labels(n, edges):
    """Scan start vertices in increasing ID order; BFS labels each new component
    with its start, which is then its smallest ID."""
    adj = [[] for _ in range(n)]
    for u, v in edges:
        adj[int(u)].append(int(v))
        adj[int(v)].append(int(u))
    L = np.full(n, -1, dtype=np.int64)
    for s in range(n):
        if L[s] >= 0:
            continue
        L[s] = s
        q = deque([s])
        while q:
            x = q.popleft()
            for y in adj[x]:
                if L[y] < 0:
                    L[y] = s
                    q.append(y)
    return L.astype(np.uint32)


def scipy_min_labels(n, edges):
    """Partition from scipy.sparse.csgraph, relabelled by each class's minimum."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    A = coo_matrix((np.ones(len(e), np.int8), (e[:, 0], e[:, 1])), shape=(n, n))
    _, comp = connected_components(A, directed=True, connection="weak")
    first = np.full(comp.max() + 1 if n else 0, np.iinfo(np.int64).max, dtype=np.int64)
    np.minimum.at(first, comp, np.arange(n))
    return first[comp].astype(np.uint32)


def check_label_invariants(n, edges, L):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    L = np.asarray(L, dtype=np.int64)
    assert np.all(L[e[:, 0]] == L[e[:, 1]]), "an edge's endpoints have different labels"
    assert np.all(L <= np.arange(n)), "a label exceeds its vertex ID"
    assert np.all(L[L] == L), "a label is not a fixed point"


# ---- brute force ------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_exhaustive_simple_graphs(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        edges = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        e = np.array(edges, dtype=np.uint32).reshape(-1, 2)
        got = oracle.cc_labels(n, e)
        np.testing.assert_array_equal(got, closure_labels(n, edges), err_msg=f"n={n} {edges}")


def test_random_multigraphs_small():
    rng = np.random.default_rng(12345)
    for trial in range(400):
        n = int(rng.integers(1, 13))
        m = int(rng.integers(0, 3 * n + 1))
        e = rng.integers(0, n, size=(m, 2)).astype(np.uint32)   # self-loops, repeats allowed
        if m and trial % 3 == 0:
            e = np.concatenate([e, e[: m // 2], e[:, ::-1]])      # explicit repeats / reversals
        got = oracle.cc_labels(n, e)
        np.testing.assert_array_equal(got, closure_labels(n, e.tolist()))


# ---- BFS and library routine -----------------------------------------------

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_bfs_er_sparse(seed):
    n = 3000
    e = graphgen.er(n, 1400 + 300 * seed, seed)          # sparse: many components
    got = oracle.cc_labels(n, e)
    np.testing.assert_array_equal(got, bfs_labels(n, e))
    check_label_invariants(n, e, got)


def test_bfs_rmat():
    e = graphgen.rmat(12, 3 * 4096, 77)
    n = 4096
    got = oracle.cc_labels(n, e)
    np.testing.assert_array_equal(got, bfs_labels(n, e))


@pytest.mark.parametrize("kind", ["er", "rmat", "rmat_sym"])
def test_scipy_partition_large(kind):
    if kind == "er":
        n, e = 1 << 18, graphgen.er(1 << 18, 1 << 17, 5)
    elif kind == "rmat":
        n, e = 1 << 18, graphgen.rmat(18, 1 << 20, 6)
    else:
        n, e = 1 << 16, graphgen.rmat_sym(16, 1 << 19, 7)
    got = oracle.cc_labels(n, e)
    np.testing.assert_array_equal(got, scipy_min_labels(n, e))
    check_label_invariants(n, e, got)


# ---- closed forms -------------------------------------------------------------

def test_empty_graph():
    for n in [1, 7, 1000]:
        np.testing.assert_array_equal(oracle.cc_labels(n, np.empty((0, 2), np.uint32)),
                                      np.arange(n, dtype=np.uint32))


def test_path_star_clique():
    n = 50
    path = [(i + 1, i) for i in range(n - 1)][::-1]
    star = [(17, i) for i in range(n) if i != 17]
    clique = list(itertools.combinations(range(n), 2))
    for edges in (path, star, clique):
        np.testing.assert_array_equal(oracle.cc_labels(n, edges), np.zeros(n, np.uint32))
    # a star that does not include vertex 0 ... 4
    star2 = [(40, i) for i in range(5, n) if i != 40]
    want = np.arange(n, dtype=np.uint32)
    want[5:] = 5
    np.testing.assert_array_equal(oracle.cc_labels(n, star2), want)


def test_disjoint_cliques_with_known_minima():
    rng = np.random.default_rng(3)
    n = 600
    perm = rng.permutation(n)
    groups = np.array_split(perm, 37)
    edges = []
    want = np.empty(n, np.uint32)
    for grp in groups:
        want[grp] = grp.min()
        edges += [(int(a), int(b)) for a, b in itertools.combinations(grp, 2)]
    rng.shuffle(edges)
    got = oracle.cc_labels(n, edges)
    np.testing.assert_array_equal(got, want)
    assert oracle.count_components(got) == 37


def test_extras_closed_form():
    g = graphgen.rmat_extras(10, 4, 99, n_paths=50)
    L = oracle.cc_labels(g.n, g.edges)
    lo, hi = g.isolated
    np.testing.assert_array_equal(L[lo:hi], np.arange(lo, hi, dtype=np.uint32))
    for s, ln in zip(g.path_starts, g.path_lens):
        np.testing.assert_array_equal(L[int(s):int(s) + int(ln)], np.full(int(ln), s, np.uint32))
    assert np.all(L[: g.n_rmat] < g.n_rmat)


def test_out_of_range_endpoint():
    with pytest.raises(oracle.OracleError) as ei:
        oracle.cc_labels(4, [(0, 1), (2, 4)])
    assert ei.value.code == oracle.ERANGE


# ---- the worked example (Fig. 1) ---------------------------------------------

def _read_fig1():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "fig1_jt_steps.txt"))
            if ln.strip() and not ln.startswith("#")]
    n = int(rows[0][0])
    edges = [tuple(map(int, r)) for r in rows[1:] if len(r) == 2]
    states = [list(map(int, r)) for r in rows[1:] if len(r) == n + 1]
    return n, edges, states


def test_fig1_worked_example():
    n, edges, states = _read_fig1()
    e = np.array(edges, np.uint32)
    for row in states:
        steps, want = row[0], row[1:]
        np.testing.assert_array_equal(oracle.jt_seq(n, e, steps=steps), np.array(want, np.uint32))


def test_jt_seq_reaches_min_labels():
    """Algorithm 1 with pointer jumping gives each component its lowest ID."""
    rng = np.random.default_rng(8)
    for _ in range(200):
        n = int(rng.integers(1, 40))
        e = rng.integers(0, n, size=(int(rng.integers(0, 2 * n)), 2)).astype(np.uint32)
        np.testing.assert_array_equal(oracle.jt_seq(n, e, jump=True), closure_labels(n, e.tolist()))


# ---- SiskinCC's update messages (Sec. III, Algorithm 2) -----------------------

def test_siskin_log_fig1():
    """The two Fig. 1 steps change P_3 to 2, then P_2 to 1: each change is one
    message (vertex, new parent), read off the printed parent arrays."""
    n, edges, states = _read_fig1()
    want = []
    for a, b in zip(states, states[1:]):
        changed = [v for v in range(n) if a[1 + v] != b[1 + v]]
        assert len(changed) == 1
        want.append([changed[0], b[1 + changed[0]]])
    got = oracle.siskin_log(n, np.array(edges, np.uint32))
    np.testing.assert_array_equal(got, np.array(want, np.uint32))


def test_siskin_log_against_closure():
    """Every vertex but its component's lowest ID is a child exactly once (non-roots
    are never updated again), parents have smaller IDs and share the child's
    component, and the messages taken as edges connect exactly what the graph does."""
    rng = np.random.default_rng(31)
    for _ in range(300):
        n = int(rng.integers(1, 40))
        e = rng.integers(0, n, size=(int(rng.integers(0, 2 * n)), 2)).astype(np.uint32)
        L = closure_labels(n, e.tolist())
        log = oracle.siskin_log(n, e)
        kids = sorted(log[:, 0].tolist())
        assert kids == [v for v in range(n) if L[v] != v]
        assert np.all(log[:, 1] < log[:, 0])
        assert np.array_equal(L[log[:, 0]], L[log[:, 1]])
        np.testing.assert_array_equal(closure_labels(n, log.tolist()), L)


def test_siskin_log_capacity_and_range():
    e = np.array([[0, 1], [1, 2], [3, 4]], np.uint32)
    assert oracle.siskin_log(5, e).tolist() == [[1, 0], [2, 0], [4, 3]]
    with pytest.raises(oracle.OracleError) as ei:
        oracle.siskin_log(4, e)
    assert ei.value.code == oracle.ERANGE


# ---- compact IDs of the exchange (Sec. V) --------------------------------------

def test_id_bytes_closed_forms():
    """ceil(log2(n) / 8) bytes hold every ID below n (one byte at least)."""
    cases = {1: 1, 2: 1, 256: 1, 257: 2, 65536: 2, 65537: 3, 1 << 24: 3, (1 << 24) + 1: 4,
             68109812: 4, 1 << 30: 4, 1 << 32: 4}
    for n, k in cases.items():
        assert oracle.id_bytes(n) == k, n


def test_pack_ids_worked_bytes():
    assert oracle.pack_ids([0x010203, 0xA0B0C0], 3).tolist() == [3, 2, 1, 0xC0, 0xB0, 0xA0]
    assert oracle.pack_ids([0x1234, 0xFF, 0], 2).tolist() == [0x34, 0x12, 0xFF, 0, 0, 0]
    assert oracle.pack_ids([7, 200], 1).tolist() == [7, 200]
    assert oracle.pack_ids([0xDEADBEEF], 4).tolist() == [0xEF, 0xBE, 0xAD, 0xDE]
    assert oracle.pack_ids([], 3).size == 0
    assert oracle.unpack_ids([3, 2, 1, 0xC0, 0xB0, 0xA0], 3).tolist() == [0x010203, 0xA0B0C0]
    with pytest.raises(oracle.OracleError):
        oracle.pack_ids([1 << 24], 3)
    with pytest.raises(oracle.OracleError):
        oracle.unpack_ids([1, 2, 3, 4], 3)


def test_pack_ids_round_trip_and_width():
    rng = np.random.default_rng(41)
    for n in [1, 2, 255, 256, 257, 70000, 1 << 24, (1 << 24) + 3, 1 << 31]:
        k = oracle.id_bytes(n)
        ids = rng.integers(0, n, size=int(rng.integers(0, 500)), dtype=np.uint64).astype(np.uint32)
        ids[:1] = n - 1 if ids.size else ids[:1]
        buf = oracle.pack_ids(ids, k)
        assert buf.size == ids.size * k
        np.testing.assert_array_equal(oracle.unpack_ids(buf, k), ids)
        # the same bytes as the low k bytes of each little-endian 32-bit word
        np.testing.assert_array_equal(
            buf.reshape(-1, k), ids.astype("<u4").view(np.uint8).reshape(-1, 4)[:, :k])


# ---- CSR input ---------------------------------------------------------------------

def test_csr_pairs_by_hand():
    # rows: 0 -> {1, 2}, 1 -> {}, 2 -> {0}, 3 -> {3, 1}
    off = [0, 2, 2, 3, 5]
    adj = [1, 2, 0, 3, 1]
    assert oracle.csr_pairs(off, adj).tolist() == [[0, 1], [0, 2], [2, 0], [3, 3], [3, 1]]
    assert oracle.cc_labels_csr(off, adj).tolist() == [0, 0, 0, 0]
    assert oracle.zroot_csr(off) == 0                  # rows 0 and 3 tie at 2: lowest ID
    with pytest.raises(oracle.OracleError):
        oracle.csr_pairs([0, 3, 2], [0, 1, 1])
    assert oracle.zroot_csr([0, 0, 0]) == 0
    assert oracle.cc_labels_csr([0, 0, 0], []).tolist() == [0, 1]


def test_csr_star_and_isolated_run():
    """A star centred at 7 with both directions listed, plus empty rows: the centre
    has the longest row and every leaf's label is the star's lowest ID."""
    n = 20
    leaves = [3, 9, 15, 19]
    rows = [[] for _ in range(n)]
    for x in leaves:
        rows[7].append(x)
        rows[x].append(7)
    off = np.cumsum([0] + [len(r) for r in rows])
    adj = [x for r in rows for x in r]
    assert oracle.zroot_csr(off) == 7
    L = oracle.cc_labels_csr(off, adj)
    want = np.arange(n)
    want[[3, 7, 9, 15, 19]] = 3
    np.testing.assert_array_equal(L, want)


# ---- 64-bit IDs ---------------------------------------------------------------------

def test_sparse64_by_hand():
    big = 1 << 40
    e = [[big + 5, 7], [7, big], [3 << 33, 3 << 33], [(3 << 33) + 1, 1 << 32]]
    ids, lab = oracle.cc_labels_sparse64(e)
    got = dict(zip(ids.tolist(), lab.tolist()))
    assert got == {7: 7, big: 7, big + 5: 7, 1 << 32: 1 << 32, 3 << 33: 3 << 33,
                   (3 << 33) + 1: 1 << 32}


def test_sparse64_against_closure():
    """Random small graphs on IDs spread over 2^48: labels equal the closure's on the
    same graph with the IDs written in increasing order as 0..k-1, mapped back."""
    rng = np.random.default_rng(51)
    for _ in range(200):
        k = int(rng.integers(1, 25))
        pool = np.sort(rng.choice(1 << 48, size=k, replace=False).astype(np.uint64))
        idx = rng.integers(0, k, size=(int(rng.integers(1, 2 * k)), 2))
        ids, lab = oracle.cc_labels_sparse64(pool[idx])
        used = np.unique(idx)
        np.testing.assert_array_equal(ids, pool[used])
        L = closure_labels(k, idx.tolist())
        np.testing.assert_array_equal(lab, pool[L[used]])


# ---- Algorithm 3 with the root function R (Formulas 1-2) ----------------------

def test_root_function_jt_closed_form():
    """With R, the root of a component is zmax if it belongs to it (R = 0), else its
    lowest ID (R = ID + 1); Algorithm 3's P holds that root's R value."""
    rng = np.random.default_rng(21)
    for _ in range(200):
        n = int(rng.integers(1, 30))
        e = rng.integers(0, n, size=(int(rng.integers(0, 2 * n)), 2)).astype(np.uint32)
        z = int(rng.integers(0, n))
        L = closure_labels(n, e.tolist())
        want = np.where(L == L[z], 0, L.astype(np.uint64) + 1)
        np.testing.assert_array_equal(oracle.rf_jt(n, e, z), want)


def test_root_function_zero_at_vertex0_matches_alg1():
    """zmax = 0 makes R order-isomorphic to the identity, so Algorithm 3 reduces to
    Algorithm 1 (Sec. IV: f = identity gives JT)."""
    e = graphgen.er(500, 300, 4)
    P1 = oracle.jt_seq(500, e, jump=True).astype(np.uint64)
    P3 = oracle.rf_jt(500, e, 0)
    np.testing.assert_array_equal(P3, np.where(P1 == 0, 0, P1 + 1))


# ---- zero root and initial push -------------------------------------------------

def test_zroot_star_and_ties():
    star = [(i, 9) for i in range(20) if i != 9]
    assert oracle.zroot(20, star, 0) == 9
    # a perfect matching on 2..9: every counted vertex has count 1 -> lowest is 2
    assert oracle.zroot(10, [(3, 2), (5, 4), (7, 6), (9, 8)], 0) == 2
    # self-loops do not count
    loops = [(5, 5)] * 10 + [(3, 1), (3, 2)]
    assert oracle.zroot(6, loops, 0) == 3
    # nothing counted -> vertex 0
    assert oracle.zroot(6, [(4, 4)], 0) == 0
    assert oracle.zroot(6, np.empty((0, 2), np.uint32), 0) == 0


def test_zroot_stride_sample():
    """K-sampling reads entries floor(j*m/K): sampled positions hold a star at 7,
    the others a larger star at 11."""
    m, K = 1000, 100
    sampled = {(j * m) // K for j in range(K)}
    e = np.empty((m, 2), np.uint32)
    a = b = 0
    for i in range(m):
        if i in sampled:
            e[i] = (7, 20 + a % 50); a += 1
        else:
            e[i] = (11, 20 + b % 50); b += 1
    assert oracle.zroot(100, e, K) == 7
    assert oracle.zroot(100, e, 0) == 11


def test_push_star():
    n, z = 30, 12
    e = np.array([(z, i) for i in range(0, n, 3) if i != z] + [(1, 2), (z, z)], np.uint32)
    P = oracle.push(n, e, 0, z)
    want = np.arange(n, dtype=np.uint32)
    for i in range(0, n, 3):
        want[i] = z
    want[z] = z
    np.testing.assert_array_equal(P, want)


def test_push_stride_sample():
    """The Initial Push over a K-entry stride sample (K < m, m not a multiple of K):
    only the entries at the sampled positions floor(j*m/K) push. Each sampled
    position holds the zero root with its own partner vertex (as first endpoint at
    even j, as second at odd j; j = 5 is a self-loop of z); every other position
    holds z with a vertex of a separate range. A truncated stride (j*(m//K)), a
    rounded-up one or a swapped endpoint test moves at least one push."""
    m, K, z = 1003, 97, 3
    base_s, base_u = 10, 200                           # partners: sampled / unsampled
    n = base_u + m
    sampled = {}
    for j in range(K):
        i = (j * m) // K
        assert i not in sampled
        sampled[i] = j
    e = np.empty((m, 2), np.uint32)
    for i in range(m):
        if i in sampled:
            j = sampled[i]
            x = base_s + j
            e[i] = (z, z) if j == 5 else ((z, x) if j % 2 == 0 else (x, z))
        else:
            e[i] = (base_u + i, z) if i % 2 else (z, base_u + i)
    P = oracle.push(n, e, K, z)
    want = np.arange(n, dtype=np.uint32)
    for j in range(K):
        if j != 5:
            want[base_s + j] = z
    np.testing.assert_array_equal(P, want)
    # every position sampled when K >= m: the unsampled partners are pushed too
    P_all = oracle.push(n, e, m, z)
    assert all(P_all[base_u + i] == z for i in range(m) if i not in sampled)
    assert P_all[base_s + 5] == base_s + 5             # the self-loop pushes nothing


# ---- forest checker -------------------------------------------------------------

def test_check_forest():
    assert oracle.check_forest(np.array([0, 0, 1, 3], np.uint32)) == 2
    with pytest.raises(AssertionError):
        oracle.check_forest(np.array([1, 0], np.uint32))          # cycle
    with pytest.raises(AssertionError):
        oracle.check_forest(np.array([0, 2, 2], np.uint32))       # parent with greater key
    # with the zero root 2, 0 -> 2 is key-decreasing
    assert oracle.check_forest(np.array([2, 0, 2], np.uint32), True, 2) == 1


# ---- batch ----------------------------------------------------------------------

def test_batch_matches_single():
    b = graphgen.batch(40, 11, lg_n_lo=3, lg_n_hi=9)
    L, st = oracle.cc_labels_batch(b.vtx_off, b.edge_off, b.edges)
    assert np.all(st == 0)
    for g in range(b.G):
        e, n = b.graph(g)
        np.testing.assert_array_equal(L[b.vtx_off[g]:b.vtx_off[g + 1]].astype(np.uint32),
                                      closure_labels(n, e.tolist()) if n <= 64 else bfs_labels(n, e))


# ---- stored oracle results ----------------------------------------------------------

def test_share30_golden_file():
    """tests/golden/share30_oracle.txt holds the oracle's labels of the R-MAT-30
    share as digests; its script uses only the generators and the oracle, and the
    recorded facts are consistent (hex digests, components within n, each probe's
    label at most the vertex and a fixed point of the labelling where known)."""
    import re
    here = os.path.join(os.path.dirname(__file__), "golden")
    src = open(os.path.join(here, "make_share30_digest.py")).read()
    imports = set(re.findall(r"^\s*(?:import|from)\s+(\w+)", src, flags=re.M))
    assert imports <= {"hashlib", "os", "sys", "time", "numpy", "graphgen", "oracle"}, imports
    g = {"label": {}}
    for line in open(os.path.join(here, "share30_oracle.txt")):
        if line.startswith("#") or not line.strip():
            continue
        k, *v = line.split()
        if k == "label":
            g["label"][int(v[0])] = int(v[1])
        else:
            g[k] = v[0]
    n, m = int(g["n"]), int(g["m"])
    assert n == 1 << 30 and 0.9 * (1 << 30) < m < 1.1 * (1 << 30)
    assert re.fullmatch(r"[0-9a-f]{64}", g["entries_sha256"])
    assert re.fullmatch(r"[0-9a-f]{64}", g["labels_sha256"])
    assert 0 < int(g["components"]) <= n
    for v, lab in g["label"].items():
        assert 0 <= lab <= v < n
        if lab in g["label"]:
            assert g["label"][lab] == lab
