"""The seeded input generators: determinism, ranges and the structure each recipe
promises (permutation bijectivity, symmetrised halves, appended components)."""
import numpy as np
import pytest

import graphgen


def test_splitmix64_reference_values():
    # SplitMix64 seeded with 0: first outputs as published with the algorithm
    # (Steele, Lea & Flood 2014; also java.util.SplittableRandom(0).nextLong()).
    assert graphgen.draw(0, 0) == 0xE220A8397B1DCDAF
    assert graphgen.draw(0, 1) == 0x6E789E6AA1B965F4
    assert graphgen.draw(0, 2) == 0x06C45D188009454F


@pytest.mark.parametrize("bits", [1, 2, 3, 5, 8, 13, 16])
def test_permutation_is_bijective(bits):
    img = {graphgen._load().gg_perm(bits, 1234, x) for x in range(1 << bits)}
    assert img == set(range(1 << bits))


def test_er_deterministic_and_in_range():
    a = graphgen.er(1000, 5000, 1)
    b = graphgen.er(1000, 5000, 1)
    c = graphgen.er(1000, 5000, 2)
    np.testing.assert_array_equal(a, b)
    assert not np.array_equal(a, c)
    assert a.max() < 1000
    # roughly uniform: every decile gets ~10 % of the endpoints
    h = np.bincount(a.ravel() // 100, minlength=10)
    assert h.min() > 0.08 * a.size and h.max() < 0.12 * a.size


def test_rmat_skew_and_permutation():
    e0 = graphgen.rmat(14, 16 << 14, 3, permute=False)
    e1 = graphgen.rmat(14, 16 << 14, 3, permute=True)
    assert e0.max() < (1 << 14) and e1.max() < (1 << 14)
    d0 = np.bincount(e0.ravel(), minlength=1 << 14)
    d1 = np.bincount(e1.ravel(), minlength=1 << 14)
    # same degree multiset (relabelling only), heavy skew, vertex 0 is the hub before permuting
    np.testing.assert_array_equal(np.sort(d0), np.sort(d1))
    assert d0.argmax() == 0 and d0.max() > 50 * d0.mean()
    assert d1.argmax() != 0


def test_rmat_sym_halves():
    e = graphgen.rmat_sym(10, 5000, 9)
    np.testing.assert_array_equal(e[5000:], e[:5000, ::-1])


def test_extras_layout():
    g = graphgen.rmat_extras(12, 4, 5, n_paths=100)
    lo, hi = g.isolated
    assert lo == 1 << 12 and hi - lo == (1 << 12) // 100
    assert len(g.path_starts) == 100 and g.path_starts[0] == hi
    assert g.path_lens.min() >= 2 and g.path_lens.max() <= 64
    assert g.n == hi + g.path_lens.sum()
    tail = g.edges[4 << 12:]
    assert len(tail) == (g.path_lens - 1).sum()
    # first path's edges, highest ID first
    s, ln = int(g.path_starts[0]), int(g.path_lens[0])
    want = [(s + j, s + j - 1) for j in range(ln - 1, 0, -1)]
    np.testing.assert_array_equal(tail[: ln - 1], np.array(want, np.uint32))


def test_batch_ranges():
    b = graphgen.batch(64, 7)
    assert b.G == 64
    ns = np.diff(b.vtx_off)
    ms = np.diff(b.edge_off)
    assert ns.min() >= 256 and ns.max() <= 65536
    for g in range(b.G):
        e, n = b.graph(g)
        assert len(e) == ms[g]
        if len(e):
            assert e.min() >= 0 and e.max() < n
        assert ms[g] >= n  # average degree >= 2


def test_share_is_a_filter():
    full = graphgen.rmat(12, 16 << 12, graphgen.config_seed(9))
    sh, n = graphgen.rmat_share(12, 16, graphgen.config_seed(9), 16, 3)
    span = (1 << 12) // 16
    keep = full[(full[:, 0] >= 3 * span) & (full[:, 0] < 4 * span)]
    np.testing.assert_array_equal(sh, keep)
    assert n == 1 << 12


def test_pareto_truncation():
    assert graphgen.pareto_n(0.0) == 1024
    assert graphgen.pareto_n(1.0) in (2**24, 2**24 - 1)
    reqs = graphgen.serve_stream(2000, 5, rate_per_s=1000.0)
    ns = np.array([r.n for r in reqs])
    assert ns.min() >= 1024 and ns.max() <= 2**24
    assert 1200 < np.median(ns) < 2100
    arr = np.array([r.arrival_s for r in reqs])
    assert np.all(np.diff(arr) > 0)
    assert 1.6 < arr[-1] < 2.4
