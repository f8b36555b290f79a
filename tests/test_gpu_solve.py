"""GPU parity of the single-graph path (cc_solve / cc_solve_async and the step
entry points) against the CPU oracle: bit-exact labels, on seeded inputs that
span several tiles and ragged tails, edge cases, and both variants."""
import numpy as np
import pytest
import torch

import graphgen
import oracle
from gpu_helpers import (assert_same_labels, check_properties_on_device, log,
                         rmat26_extras_with_labels, to_dev, to_host_u32)

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_2507_03695_amd")

FLAG_SETS = {
    "plain": 0,
    "nosplit": cc.F_NO_SPLIT,
    "zroot": cc.F_ZROOT,
    "zroot_exact": cc.F_ZROOT | cc.F_ZROOT_EXACT,
    "zroot_nosplit": cc.F_ZROOT | cc.F_NO_SPLIT,
}


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = cc.Context(zroot_samples=4096)
    yield c
    c.close()


def run_all_variants(ctx, e_np, n, want, what):
    ed = to_dev(e_np)
    for name, fl in FLAG_SETS.items():
        L = ctx.solve(ed, n, flags=fl)
        assert_same_labels(to_host_u32(L), want, f"{what} [{name}]")


def test_cc_solve_default_context_small_random():
    rng = np.random.default_rng(2024)
    for i in range(150):
        n = int(rng.integers(1, 3000))
        m = int(rng.integers(0, 4 * n))
        e = graphgen.er(n, m, 1000 + i)
        L = cc.solve(to_dev(e), n)
        assert_same_labels(to_host_u32(L), oracle.cc_labels(n, e), f"er n={n} m={m}")


@pytest.mark.parametrize("m", [1, 255, 256, 1023, 1024, 1025, 4095, 4097, 100_003, 1_000_001])
def test_tiles_and_ragged_tails(ctx, m):
    n = 20_000
    e = graphgen.er(n, m, 77 + m)
    log(f"ragged m={m}")
    run_all_variants(ctx, e, n, oracle.cc_labels(n, e), f"m={m}")


def test_adversarial_orders(ctx):
    n = 50_000
    ids = np.arange(n, dtype=np.uint32)
    chain_up = np.stack([ids[:-1], ids[1:]], 1)                     # (i, i+1)
    chain_down = chain_up[::-1, ::-1].copy()                        # (i+1, i), high IDs first
    rng = np.random.default_rng(5)
    chain_rand = chain_up[rng.permutation(n - 1)]
    star_hi = np.stack([np.full(n - 1, n - 1, np.uint32), ids[:-1]], 1)
    perm = rng.permutation(n).astype(np.uint32)
    perm_chain = np.stack([perm[:-1], perm[1:]], 1)
    for name, e in [("chain_up", chain_up), ("chain_down", chain_down), ("chain_rand", chain_rand),
                    ("star_hi", star_hi), ("perm_chain", perm_chain)]:
        run_all_variants(ctx, e, n, oracle.cc_labels(n, e), name)


def test_edge_cases(ctx):
    # n = 1, self-loops only, m = 0, duplicates
    for n, e in [(1, np.zeros((0, 2), np.uint32)), (1, np.zeros((5, 2), np.uint32)),
                 (7, np.zeros((0, 2), np.uint32)), (3, np.array([[2, 2], [1, 1]], np.uint32)),
                 (4, np.array([[3, 1]] * 1000, np.uint32))]:
        run_all_variants(ctx, e, n, oracle.cc_labels(n, e), f"edge case n={n} m={len(e)}")
    # n = 0 is a no-op
    L = torch.empty(0, dtype=torch.int32, device="cuda")
    ctx.solve_async(to_dev(np.zeros((0, 2), np.uint32)), 0, L)
    assert ctx.sync() == cc.CC_OK


def test_errors(ctx):
    e = to_dev(np.array([[0, 1], [2, 9]], np.uint32))
    L = torch.empty(4, dtype=torch.int32, device="cuda")
    ctx.solve_async(e, 4, L)
    assert ctx.sync() == cc.CC_ERANGE
    assert ctx.sync() == cc.CC_OK            # cleared by the previous sync
    with pytest.raises(cc.CCError) as ei:
        cc.solve(e, 4)
    assert ei.value.code == cc.CC_ERANGE
    lib = cc.load()
    assert lib.cc_solve(1 << 32, 0, None, None) == cc.CC_EINVAL
    assert lib.cc_solve(5, 3, None, L.data_ptr()) == cc.CC_EINVAL
    assert lib.cc_solve(5, 0, None, None) == cc.CC_EINVAL
    assert lib.cc_solve_async(ctx.handle, 4, 0, None, L.data_ptr(), cc.F_ZROOT | cc.F_ZROOT_HINT,
                              9, None, None) == cc.CC_EINVAL
    assert lib.cc_solve_async(ctx.handle, 4, 0, None, L.data_ptr(), 0x100, 0, None,
                              None) == cc.CC_EINVAL                    # unknown flag bit
    assert lib.cc_solve_async(ctx.handle, 4, 0, None, L.data_ptr(), 1 << 31, 0, None,
                              None) == cc.CC_EINVAL                    # the library's own bit
    with pytest.raises(cc.CCError) as ei:
        ctx.hook(e, 4, L, flags=cc.F_ZROOT | (1 << 31))
    assert ei.value.code == cc.CC_EINVAL
    # a zero-root hook needs cc_zroot after the latest cc_init
    ctx.init(4, L)
    with pytest.raises(cc.CCError) as ei:
        ctx.hook(e, 4, L, flags=cc.F_ZROOT)
    assert ei.value.code == cc.CC_EINVAL
    ctx.zroot(e[:1], 4)
    ctx.init(4, L)
    with pytest.raises(cc.CCError):
        ctx.push(e[:1], 4, L)
    assert ctx.sync() == cc.CC_OK


def test_symmetric_flag(ctx):
    """CC_F_SYMMETRIC hooks only the u < v entries of a list that holds every pair
    in both orders: the labels equal the oracle's on the whole list, through the
    direct and regrouped hooks (sizes on both sides of their limits) and
    the CSR and 64-bit paths. On a list that is not symmetric the labels are
    those of its u < v entries alone (the flag's definition)."""
    cases = [(graphgen.rmat_sym(12, 20_000, 3), 1 << 12),          # direct hook
             (graphgen.rmat_sym(17, 1 << 18, 4), 1 << 17),         # small array, dense
             (graphgen.rmat_sym(20, 1 << 23, 5), 1 << 20)]         # regrouped hooks
    for e, n in cases:
        want = oracle.cc_labels(n, e)
        ed = to_dev(e)
        for fl in (0, cc.F_ZROOT, cc.F_NO_SPLIT, cc.F_ZROOT | cc.F_NO_TILE):
            log(f"symmetric n={n} m={len(e)} flags={fl}")
            L = ctx.solve(ed, n, flags=fl | cc.F_SYMMETRIC)
            assert_same_labels(to_host_u32(L), want, f"symmetric n={n} flags={fl}")
        # CSR rows of the same list (a symmetric CSR graph)
        order = np.lexsort((e[:, 1], e[:, 0]))
        adj = np.ascontiguousarray(e[order, 1])
        off = np.zeros(n + 1, np.int64)
        np.cumsum(np.bincount(e[:, 0], minlength=n), out=off[1:])
        o_d = torch.from_numpy(off).cuda()
        a_d = torch.from_numpy(adj.view(np.int32)).cuda()
        for fl in (0, cc.F_ZROOT):
            L = ctx.solve_csr(o_d, a_d, n, flags=fl | cc.F_SYMMETRIC)
            assert_same_labels(to_host_u32(L), want, f"symmetric CSR n={n} flags={fl}")
    e, n = cases[0]
    L = ctx.solve_u64(torch.from_numpy(e.astype(np.int64)).cuda(), n, flags=cc.F_SYMMETRIC)
    assert np.array_equal(L.cpu().numpy(), oracle.cc_labels(n, e).astype(np.int64))
    # a list that is not symmetric: only its u < v entries count
    n = 5000
    e = graphgen.er(n, 12_000, 17)
    half = e[e[:, 0] < e[:, 1]]
    want_half = oracle.cc_labels(n, half)
    assert not np.array_equal(want_half, oracle.cc_labels(n, e))
    ed = to_dev(e)
    for fl in (0, cc.F_ZROOT):
        L = ctx.solve(ed, n, flags=fl | cc.F_SYMMETRIC)
        assert_same_labels(to_host_u32(L), want_half, f"asymmetric list flags={fl}")


def test_per_call_status(ctx):
    """Each whole-path call given a cc_status_t gets its own outcome, even with
    several calls queued on one stream before any wait: an out-of-range solve
    between two good ones reports CC_ERANGE and only there."""
    n = 3000
    good = to_dev(graphgen.er(n, 9000, 5))
    bad_np = graphgen.er(n, 9000, 6)
    bad_np[4567] = (n + 11, 3)
    bad = to_dev(bad_np)
    Ls = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in range(4)]
    sts = [cc.Status() for _ in range(4)]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx.solve_async(good, n, Ls[0], stream=s, status=sts[0])
        ctx.solve_async(bad, n, Ls[1], flags=cc.F_ZROOT, stream=s, status=sts[1])
        ctx.solve_async(good, n, Ls[2], flags=cc.F_ZROOT, stream=s, status=sts[2])
        ctx.solve_async(bad, n, Ls[3], stream=s)                   # no status: cc_sync gets it
    got = [ctx.status_wait(st) for st in sts[:3]]
    assert got == [cc.CC_OK, cc.CC_ERANGE, cc.CC_OK]
    assert ctx.status_wait(sts[1], 0) == cc.CC_ERANGE             # may be waited for again
    assert ctx.sync(s) == cc.CC_ERANGE
    want = oracle.cc_labels(n, graphgen.er(n, 9000, 5))
    for i in (0, 2):
        assert_same_labels(to_host_u32(Ls[i]), want, f"status solve {i}")
    assert sts[1].seq == sts[0].seq + 1 and sts[2].seq == sts[0].seq + 2
    # CSR: offsets that are not a row index give CC_EINVAL through the status
    o = torch.tensor([0, 2, 1, 2], dtype=torch.int64, device="cuda")
    a = torch.tensor([1, 2], dtype=torch.int32, device="cuda")
    L = torch.empty(3, dtype=torch.int32, device="cuda")
    st = cc.Status()
    ctx.solve_csr_async(o, a, 3, L, status=st)
    assert ctx.status_wait(st) == cc.CC_EINVAL
    # a record reused CC_STATUS_RING calls later is refused
    first = cc.Status()
    ctx.solve_async(good, n, Ls[0], status=first)
    for _ in range(cc.STATUS_RING):
        ctx.solve_async(good, n, Ls[0], status=cc.Status())
    assert ctx.status_wait(first) == cc.CC_EINVAL
    lib = cc.load()
    assert lib.cc_status_wait(None, 0) == cc.CC_EINVAL
    assert ctx.sync() == cc.CC_OK


def test_metamorphic(ctx):
    n = 30_000
    e = graphgen.rmat(15, 3 * n, 31)[: 3 * n]
    e = e % n
    want = oracle.cc_labels(n, e)
    rng = np.random.default_rng(0)
    variants = {
        "shuffled": e[rng.permutation(len(e))],
        "swapped": e[:, ::-1].copy(),
        "dups": np.concatenate([e, e[rng.integers(0, len(e), 5000)]]),
        "loops": np.concatenate([e, np.stack([np.arange(0, n, 7)] * 2, 1).astype(np.uint32)]),
    }
    for name, ev in variants.items():
        run_all_variants(ctx, ev, n, want, name)


def test_vertex_permutation(ctx):
    """Relabelling the vertices by a permutation pi maps the partition: on the
    permuted graph each vertex pi(v) is labelled with the smallest pi(w) over
    the component of v in the original graph (labels derived from the original
    graph's oracle labels, not from a second oracle call)."""
    n = 40_000
    e = graphgen.rmat(16, 200_000, 63) % n
    want = oracle.cc_labels(n, e)
    pi = np.random.default_rng(64).permutation(n).astype(np.uint32)
    low = np.full(n, n, np.int64)
    np.minimum.at(low, want, pi)
    expect = np.empty(n, np.uint32)
    expect[pi] = low[want]
    run_all_variants(ctx, pi[e], n, expect, "permuted")


@pytest.mark.parametrize("size", ["direct", "regrouped"])
def test_zero_root_choice_does_not_change_labels(ctx, size):
    """Variant Z: any vertex may be the zero root (the max-degree choice only
    saves work, Sec. IV), so forcing it through the hint leaves the labels
    equal to the oracle's: z = 0, n - 1, the true max-degree vertex, a random
    vertex and an isolated one. "regrouped": 2^24 entries over eight vertex
    slices, the size from which the zero-root hook regroups its entries; with
    CC_F_NO_SPLIT it takes the direct hook instead."""
    if size == "direct":
        n = 50_000
        e = graphgen.rmat(16, 400_000, 61) % n
    else:
        n = 1 << 22
        e = graphgen.rmat(22, 1 << 24, 62)
    want = oracle.cc_labels(n, e)
    deg = np.bincount(e.ravel(), minlength=n)
    iso = np.flatnonzero(deg == 0)
    assert len(iso), "the case needs an isolated vertex"
    rng = np.random.default_rng(65)
    hints = [0, n - 1, int(np.argmax(deg)), int(rng.integers(n)), int(iso[len(iso) // 2])]
    ed = to_dev(e)
    for z in hints:
        for extra in (0, cc.F_NO_SPLIT):
            fl = cc.F_ZROOT | cc.F_ZROOT_HINT | extra
            L = ctx.solve(ed, n, flags=fl, zroot_hint=z)
            assert ctx.get_zroot() == z
            assert_same_labels(to_host_u32(L), want, f"{size} z={z} flags={fl:#x}")


def test_repeat_stress(ctx):
    """Same graph, many runs: the schedule differs, the labels may not. Every run
    takes the entries in a new seeded order, with a new random half of them
    reversed, and the runs cycle through the plain and zero-root variants with
    and without splitting and with a forced zero root."""
    n = 1 << 16
    e = graphgen.rmat(16, 16 << 16, 12)
    want = oracle.cc_labels(n, e)
    ed = to_dev(e)
    L = torch.empty(n, dtype=torch.int32, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(12)
    flag_cycle = [0, cc.F_ZROOT, cc.F_NO_SPLIT, cc.F_ZROOT | cc.F_NO_SPLIT,
                  cc.F_ZROOT | cc.F_ZROOT_HINT]
    for rep in range(120):
        order = torch.randperm(len(e), device="cuda", generator=gen)
        er = ed[order]
        flip = torch.rand(len(e), device="cuda", generator=gen) < 0.5
        er[flip] = er[flip].flip(1)
        er = er.contiguous()
        fl = flag_cycle[rep % len(flag_cycle)]
        ctx.solve_async(er, n, L, flags=fl, zroot_hint=(rep * 7919) % n)
        assert ctx.sync() == cc.CC_OK
        assert_same_labels(to_host_u32(L), want, f"rep {rep} flags {fl:#x}")


# ---- the step entry points ----------------------------------------------------------

def test_zroot_step(ctx):
    for seed, n, m in [(1, 1000, 3000), (2, 1 << 16, 1 << 20), (3, 5, 2)]:
        e = graphgen.rmat(max(1, (n - 1).bit_length()), m, seed) % n
        ed = to_dev(e)
        ctx.zroot(ed, n)
        assert ctx.get_zroot() == oracle.zroot(n, e, 4096), f"sampled zroot n={n}"
        ctx.zroot(ed, n, flags=cc.F_ZROOT_EXACT)
        assert ctx.get_zroot() == oracle.zroot(n, e, 0), f"exact zroot n={n}"
        ctx.zroot(ed, n, flags=cc.F_ZROOT_HINT, zroot_hint=n - 1)
        assert ctx.get_zroot() == n - 1


def test_push_step(ctx):
    n, m = 1 << 14, 1 << 18
    e = graphgen.rmat(14, m, 8)
    ed = to_dev(e)
    P = torch.empty(n, dtype=torch.int32, device="cuda")
    ctx.init(n, P)
    ctx.zroot(ed, n)
    z = ctx.get_zroot()
    ctx.push(ed, n, P)
    torch.cuda.synchronize()
    assert_same_labels(to_host_u32(P), oracle.push(n, e, 4096, z), "push")


@pytest.mark.parametrize("flags", [0, 1, 8, 9])
def test_hook_leaves_a_key_monotone_forest(ctx, flags):
    n, m = 1 << 17, 1 << 20
    e = graphgen.rmat(17, m, 44)
    ed = to_dev(e)
    want = oracle.cc_labels(n, e)
    P = torch.empty(n, dtype=torch.int32, device="cuda")
    ctx.init(n, P)
    z = 0
    if flags & cc.F_ZROOT:
        ctx.zroot(ed, n)
        z = ctx.get_zroot()
        ctx.push(ed, n, P)
    ctx.hook(ed, n, P, flags=flags)
    torch.cuda.synchronize()
    Ph = to_host_u32(P)
    roots = oracle.check_forest(Ph, bool(flags & cc.F_ZROOT), z)
    ncomp = oracle.count_components(want)
    if flags & cc.F_ZROOT:
        # an entry with one endpoint in the membership bitmap links the other to
        # z by its bit alone, which compress resolves: P then holds more trees
        # than there are components, but no tree spans two components
        assert roots >= ncomp
        r = Ph.astype(np.int64)
        while True:
            r2 = r[r]
            if np.array_equal(r2, r):
                break
            r = r2
        assert np.array_equal(want[r], want), "a tree spans two components"
    else:
        assert roots == ncomp
    ctx.compress(n, P, flags=flags)
    if flags & cc.F_ZROOT:
        ctx.canon(n, P)
    assert ctx.sync() == cc.CC_OK
    assert_same_labels(to_host_u32(P), want, "steps")


@pytest.mark.parametrize("size", ["direct", "regrouped"])
def test_compress_relabels_with_or_without_canon(ctx, size):
    """cc_compress with a zero root leaves z's component labelled z (the form the
    share export reads) and cc_canon then gives each component its smallest ID;
    with CC_F_CANON cc_compress gives those labels itself. Both equal the
    oracle's, on the direct hook and on the regrouped one (whose links to z are
    partly bitmap marks that compress resolves)."""
    if size == "direct":
        n, e = 1 << 17, graphgen.rmat(17, 1 << 20, 45)
    else:
        n, e = 1 << 20, graphgen.rmat(20, 1 << 24, 46)
    want = oracle.cc_labels(n, e)
    ed = to_dev(e)
    P = torch.empty(n, dtype=torch.int32, device="cuda")
    for canon_flag in (False, True):
        ctx.init(n, P)
        ctx.zroot(ed, n)
        z = ctx.get_zroot()
        ctx.push(ed, n, P)
        ctx.hook(ed, n, P, flags=cc.F_ZROOT)
        if canon_flag:
            ctx.compress(n, P, flags=cc.F_ZROOT | cc.F_CANON)
        else:
            ctx.compress(n, P, flags=cc.F_ZROOT)
            assert ctx.sync() == cc.CC_OK
            Ph = to_host_u32(P)
            inz = want == want[z]
            assert np.all(Ph[inz] == z), "members of z's component not labelled z"
            assert_same_labels(Ph[~inz], want[~inz], "labels outside z's component")
            ctx.canon(n, P)
        assert ctx.sync() == cc.CC_OK
        assert_same_labels(to_host_u32(P), want, f"{size} CC_F_CANON={canon_flag}")


# ---- the named workloads at full size ---------------------------------------------------

def test_er_65k_full():
    e, n = graphgen.er_65k()
    want = oracle.cc_labels(n, e)
    with cc.Context() as c:
        run_all_variants(c, e, n, want, "ER n=65536 m=2^20")


def test_rmat22_sym_full():
    e, n = graphgen.rmat22_sym()
    log("rmat22 generated")
    want = oracle.cc_labels(n, e)
    log("rmat22 oracle done")
    with cc.Context() as c:
        ed = to_dev(e)
        for name, fl in [("plain", 0), ("zroot", cc.F_ZROOT)]:
            L = c.solve(ed, n, flags=fl)
            assert_same_labels(to_host_u32(L), want, f"rmat22 [{name}]")
            check_properties_on_device(ed, L, n)


def test_rmat26_extras_full():
    """The RMAT-26 + isolated + paths workload in the bench's launch configuration."""
    g, want = rmat26_extras_with_labels()
    ed = to_dev(g.edges)
    with cc.Context() as c:
        Lz = c.solve(ed, g.n, flags=cc.F_ZROOT)
        Lp = c.solve(ed, g.n, flags=0)                    # first-endpoint buckets
        Ld = c.solve(ed, g.n, flags=cc.F_NO_TILE)         # direct entry-order hook
        # the direct zero-root hook; its parent array (272 MB) is past the size
        # from which an entry with one marked endpoint only marks the other
        Lzd = c.solve(ed, g.n, flags=cc.F_ZROOT | cc.F_NO_TILE)
        torch.cuda.synchronize()
        log("rmat26 GPU done")
        assert torch.equal(Ld, Lp), "direct and bucketed plain hooks disagree"
        assert torch.equal(Lzd, Lp), "direct zero-root and plain hooks disagree"
        del Ld, Lzd
        check_properties_on_device(ed, Lz, g.n)
        assert torch.equal(Lz, Lp), "plain and zero-root paths disagree"
        Lh = to_host_u32(Lz)
    del ed
    lo, hi = g.isolated
    assert np.array_equal(Lh[lo:hi], np.arange(lo, hi, dtype=np.uint32))
    for s, ln in zip(g.path_starts[:2000], g.path_lens[:2000]):
        assert np.all(Lh[int(s):int(s) + int(ln)] == s)
    assert_same_labels(Lh, want, "rmat26 extras")


# ---- the tiled zero-root hook (entries regrouped by both endpoints' vertex ranges) -------

@pytest.mark.parametrize("case", ["er_R6", "rmat_unpermuted", "four_slices", "eight_slices",
                                  "loops_dups", "R256"])
def test_tiled_hook_parity(case):
    rng = np.random.default_rng(hash(case) % 2**32)
    if case == "er_R6":
        n = 3_000_000
        e = graphgen.er(n, (1 << 24) + 12_345, 61)
    elif case == "rmat_unpermuted":          # skewed: low slices hold most entries
        n = 1 << 22
        e = graphgen.rmat(22, (1 << 24) + 777, 62, permute=False)
    elif case == "four_slices":                # the fewest the plain path regroups
        n = 3 * (1 << 19) + 1
        e = graphgen.er(n, 1 << 24, 63)
    elif case == "eight_slices":               # the fewest the zero-root path regroups
        n = 7 * (1 << 19) + 1
        e = graphgen.rmat(22, 1 << 24, 67) % n
    elif case == "loops_dups":
        n = 4_000_000
        e = graphgen.er(n, 1 << 24, 64)
        e[::7, 1] = e[::7, 0]                  # self-loops
        e[1::11] = e[0:-1:11][: len(e[1::11])]  # repeats
    else:                                      # exactly 256 slices
        n = 256 << 19
        e = graphgen.rmat(27, 1 << 24, 65)
    want = oracle.cc_labels(n, e)
    ed = to_dev(e)
    with cc.Context() as c:
        for name, fl in [("tiled", cc.F_ZROOT), ("direct", cc.F_ZROOT | cc.F_NO_TILE),
                         ("plain bucketed", 0), ("plain direct", cc.F_NO_TILE)]:
            L = c.solve(ed, n, flags=fl)
            assert_same_labels(to_host_u32(L), want, f"{case} [{name}]")


def test_tiled_hook_out_of_range():
    n = 1 << 22
    e = graphgen.er(n, 1 << 24, 66)
    e[12345] = (n + 5, 3)
    with cc.Context() as c:
        L = torch.empty(n, dtype=torch.int32, device="cuda")
        for fl in (cc.F_ZROOT, 0):                 # the zero-root and the plain bucketed hook
            c.solve_async(to_dev(e), n, L, flags=fl)
            assert c.sync() == cc.CC_ERANGE, fl


def test_compress_never_trusts_a_stale_root():
    """Regression: a compress thread once stopped at a vertex whose entry it read as
    a root from a copy cached on another XCD while the vertex was still a root,
    although the hook had linked it. Repeated step-wise solves of a skewed graph
    (hook, host check of P, compress) must all give the oracle's labels."""
    n = 1 << 22
    e = graphgen.rmat(22, (1 << 24) + 777, 62, permute=False)
    want = oracle.cc_labels(n, e)
    ed = to_dev(e)
    with cc.Context() as c:
        P = torch.empty(n, dtype=torch.int32, device="cuda")
        for rep in range(24):
            fl = 0 if rep % 2 == 0 else cc.F_ZROOT | cc.F_NO_TILE
            c.init(n, P)
            if fl:
                c.zroot(ed, n)
                c.push(ed, n, P)
            c.hook(ed, n, P, flags=fl)
            torch.cuda.synchronize()
            _ = P.cpu()                      # the host read between the kernels, as before
            c.compress(n, P, flags=fl)
            if fl:
                c.canon(n, P)
            assert c.sync() == cc.CC_OK
            assert_same_labels(to_host_u32(P), want, f"rep {rep} flags {fl}")


def test_labels_read_back_by_the_next_kernel():
    """Regression: after a plain solve that followed a zero-root solve, the first
    torch kernel reading L saw an intermediate parent in one word (a splitting
    store's line, left in the writing XCD's L2 and rewritten by another XCD's
    compress), although the host copy was right. Alternate the two paths and
    compare a device-side read of L (a conversion kernel) with the host copy."""
    e, n = graphgen.rmat22_sym()
    ed = to_dev(e)
    want = None
    with cc.Context() as c:
        for rep in range(20):
            fl = cc.F_ZROOT if rep % 2 == 0 else 0
            L = c.solve(ed, n, flags=fl)
            torch.cuda.synchronize()
            host = L.cpu().numpy().view(np.uint32).astype(np.int64)
            dev = (L.to(torch.int64) & 0xFFFFFFFF).cpu().numpy()
            bad = np.flatnonzero(dev != host)
            assert len(bad) == 0, f"rep {rep} flags {fl}: {len(bad)} words differ, first v={bad[0]}"
            if want is None:
                want = host
            assert np.array_equal(host, want), f"rep {rep}: labels changed between solves"


def test_two_part_small_array_hook():
    """The plain direct hook on a small array takes its entries in two parts with
    a pointer-jumping pass between: an out-of-range entry is reported from
    either part, a symmetric list (every pair in both orders, u < v hooked)
    gives the oracle's labels of its pairs, and CC_F_NO_SPLIT (one part, no
    pass) gives the same labels."""
    n = 1 << 16
    e = graphgen.er(n, 1 << 20, 131)
    want = oracle.cc_labels(n, e)
    with cc.Context() as c:
        L = torch.empty(n, dtype=torch.int32, device="cuda")
        for at in (5, (1 << 18) - 1, 1 << 18, len(e) - 3):   # both sides of the split point
            bad = e.copy()
            bad[at] = (n + 7, 1)
            c.solve_async(to_dev(bad), n, L)
            assert c.sync() == cc.CC_ERANGE, at
        sym = np.ascontiguousarray(np.concatenate([e, e[:, ::-1]]))
        for fl in (cc.F_SYMMETRIC, cc.F_SYMMETRIC | cc.F_NO_SPLIT, 0, cc.F_NO_SPLIT):
            Ls = c.solve(to_dev(sym if fl & cc.F_SYMMETRIC else e), n, flags=fl)
            assert_same_labels(to_host_u32(Ls), want, f"flags {fl:#x}")


@pytest.mark.parametrize("case", ["er_16", "er_18", "rmat_17"])
def test_small_array_hook(case):
    """Small parent arrays with many entries per vertex (the case where walks end
    at roots read through stale L2 copies and the check before each CAS matters),
    ragged entry counts: with and without splitting, plain and zero-root, every
    solve equals the oracle."""
    if case == "er_16":
        n, e = 1 << 16, graphgen.er(1 << 16, (1 << 18) + 123, 121)
    elif case == "er_18":
        n, e = 1 << 18, graphgen.er(1 << 18, (1 << 20) + 7, 122)
    else:
        n, e = 1 << 17, graphgen.rmat(17, (1 << 19) + 999, 123)
    want = oracle.cc_labels(n, e)
    ed = to_dev(e)
    with cc.Context() as c:
        for fl in (0, cc.F_NO_SPLIT, cc.F_NO_TILE, cc.F_ZROOT, cc.F_ZROOT | cc.F_NO_SPLIT):
            L = c.solve(ed, n, flags=fl)
            assert_same_labels(to_host_u32(L), want, f"{case} flags {fl:#x}")
