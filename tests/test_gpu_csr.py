"""CSR input on the GPU (cc_solve_csr): labels bit-exact against the oracle on
the row-by-row pairs, the exact longest-row zero root, both ways of finding a
position's row (the LDS sweep and, across long runs of empty rows, the search),
ragged tails, empty graphs and the error paths."""
import numpy as np
import pytest
import torch

import graphgen
import oracle
from gpu_helpers import assert_same_labels, log, rmat26_extras_with_labels, to_dev, to_host_u32

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_2507_03695_amd")

FLAGS = {"plain": 0, "zroot": 0x1, "plain-nosplit": 0x8, "zroot-nosplit": 0x9}


def to_csr(n, e):
    """Rows of the entries (u, v) by u, in entry order within a row."""
    e = np.asarray(e, np.uint32).reshape(-1, 2)
    order = np.argsort(e[:, 0], kind="stable")
    adj = np.ascontiguousarray(e[order, 1])
    off = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(e[:, 0], minlength=n), out=off[1:])
    return off, adj


def dev(off, adj):
    return (torch.from_numpy(off).cuda(),
            torch.from_numpy(np.ascontiguousarray(adj, np.uint32).view(np.int32)).cuda())


def solve(c, off, adj, n, flags):
    o, a = dev(off, adj)
    return to_host_u32(c.solve_csr(o, a, n, flags=flags))


def graphs():
    yield "er", 1 << 16, graphgen.er(1 << 16, 1 << 18, 101)
    yield "rmat", 1 << 16, graphgen.rmat(16, 1 << 20, 102)
    yield "rmat_sym", 1 << 14, graphgen.rmat_sym(14, 1 << 17, 103)
    g = graphgen.rmat_extras(14, 16, 104, n_paths=300)
    yield "rmat_extras", g.n, g.edges


@pytest.mark.parametrize("flags", list(FLAGS))
def test_csr_labels_match_the_oracle(flags):
    with cc.Context() as c:
        for name, n, e in graphs():
            off, adj = to_csr(n, e)
            want = oracle.cc_labels_csr(off, adj)
            assert_same_labels(solve(c, off, adj, n, FLAGS[flags]), want, f"{name} {flags}")
            if FLAGS[flags] & 1:
                assert c.get_zroot() == oracle.zroot_csr(off), name


def test_rows_found_by_sweep_and_by_search():
    """Edges among 0..299 and 60000..60299 only: one tile spans the 59,700 empty
    rows between them (more than the sweep bound), the others sweep."""
    n = 70000
    rng = np.random.default_rng(105)
    a = rng.integers(0, 300, size=(3000, 2))
    b = rng.integers(60000, 60300, size=(3000, 2))
    cross = np.array([[5, 60007], [299, 60299]])
    e = np.concatenate([a, b, cross]).astype(np.uint32)
    off, adj = to_csr(n, e)
    want = oracle.cc_labels_csr(off, adj)
    with cc.Context() as c:
        for f in (0, 1):
            assert_same_labels(solve(c, off, adj, n, f), want, f"flags {f}")


def test_rows_longer_than_tiles_and_ragged_tail():
    """One row of 10,000 entries (many tiles share one row), a few short rows and
    an entry count that is not a multiple of the tile."""
    n = 5000
    rng = np.random.default_rng(106)
    hub = np.stack([np.full(10000, 17), rng.integers(0, n, 10000)], axis=1)
    rest = rng.integers(0, n, size=(1237, 2))
    e = np.concatenate([hub, rest]).astype(np.uint32)
    off, adj = to_csr(n, e)
    want = oracle.cc_labels_csr(off, adj)
    with cc.Context() as c:
        for f in FLAGS.values():
            assert_same_labels(solve(c, off, adj, n, f), want, f"flags {f}")
        solve(c, off, adj, n, 1)
        assert c.get_zroot() == 17


def test_csr_empty_and_errors():
    with cc.Context() as c:
        off = np.zeros(11, np.int64)
        assert np.array_equal(solve(c, off, np.zeros(0, np.uint32), 10, 1), np.arange(10))
        assert np.array_equal(solve(c, np.zeros(2, np.int64), np.zeros(0, np.uint32), 1, 0), [0])
        # an endpoint out of range
        o, a = dev(np.array([0, 1, 2], np.int64), np.array([1, 7], np.uint32))
        L = torch.empty(2, dtype=torch.int32, device="cuda")
        c.solve_csr_async(o, a, 2, L)
        assert c.sync() == cc.CC_ERANGE
        # offsets that decrease, or pass the entry count
        for bad in ([0, 3, 2, 3], [0, 5, 5, 3]):
            o, a = dev(np.array(bad, np.int64), np.array([0, 1, 2], np.uint32))
            L = torch.empty(3, dtype=torch.int32, device="cuda")
            c.solve_csr_async(o, a, 3, L, flags=1)
            assert c.sync() == cc.CC_EINVAL, bad
        assert c.sync() == cc.CC_OK
        with pytest.raises(cc.CCError) as ei:
            c.solve_csr_async(o, a, 3, L, flags=0x5, zroot_hint=3)
        assert ei.value.code == cc.CC_EINVAL


def test_csr_matches_coo_on_a_large_graph():
    """RMAT-20 (2^24 entries): CSR and COO solves give the same labels, equal to
    the oracle's."""
    n = 1 << 20
    e = graphgen.rmat(20, 1 << 24, 107)
    want = oracle.cc_labels(n, e)
    log("oracle done")
    off, adj = to_csr(n, e)
    with cc.Context() as c:
        for f in (0, 1):
            assert_same_labels(solve(c, off, adj, n, f), want, f"csr flags {f}")


def test_csr_regrouped_zero_root_path():
    """R-MAT-22 + extras (about 2^25 entries, nine vertex slices): the regrouped
    zero-root hook on CSR rows, the direct one (CC_F_NO_TILE) and the oracle
    agree; the rows include the empty block and the appended paths."""
    g = graphgen.rmat_extras(22, 8, 108, n_paths=2000)
    n, e = g.n, g.edges
    want = oracle.cc_labels(n, e)
    log(f"n={n} m={len(e)}: oracle done")
    off, adj = to_csr(n, e)
    with cc.Context() as c:
        for f in (0x1, 0x1 | 0x10):
            assert_same_labels(solve(c, off, adj, n, f), want, f"csr flags {f:#x}")
            assert c.get_zroot() == oracle.zroot_csr(off)


def test_csr_regrouped_at_256_slices():
    """n = 256 * 2^19 (the most slices the regrouped hook takes), 2^24 entries of an
    R-MAT-27 graph as CSR rows: the regrouped and direct zero-root paths equal the
    oracle."""
    n = 256 << 19
    e = graphgen.rmat(27, 1 << 24, 109)
    want = oracle.cc_labels(n, e)
    log("oracle done")
    off, adj = to_csr(n, e)
    with cc.Context() as c:
        for f in (0x1, 0x1 | 0x10):
            assert_same_labels(solve(c, off, adj, n, f), want, f"csr R=256 flags {f:#x}")


def test_csr_rmat26_extras_full():
    """The bench's R-MAT-26 + extras workload as CSR rows (built on the device by a
    stable sort on the first endpoint): both zero-root paths and the plain path
    equal the oracle's labels."""
    g, want = rmat26_extras_with_labels()
    n = g.n
    ed = to_dev(g.edges)
    u = ed[:, 0]
    order = torch.argsort(u, stable=True)
    adj = ed[:, 1][order].contiguous()
    del order
    off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    off[1:] = torch.cumsum(torch.bincount(u, minlength=n), 0)
    del ed, u
    with cc.Context() as c:
        for f in (0x1, 0x1 | 0x10, 0):
            L = c.solve_csr(off, adj, n, flags=f)
            assert_same_labels(to_host_u32(L), want, f"csr rmat26 flags {f:#x}")
            if f & 1:
                assert c.get_zroot() == oracle.zroot_csr(off.cpu().numpy())

