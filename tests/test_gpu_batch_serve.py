"""GPU parity of the batched launch (cc_batch) and the continuous-batching server
(cc_serve_*): every graph's labels equal the oracle's and equal cc_solve on the
graph alone, whatever the mix it ran in."""
import time

import numpy as np
import pytest
import torch

import graphgen
import oracle
from gpu_helpers import (assert_same_labels, golden_share30, log, sha256_of, to_dev,
                         to_host_u32)

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_2507_03695_amd")


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = cc.Context()
    yield c
    c.close()


def batch_to_dev(b):
    return (torch.from_numpy(b.vtx_off).cuda(), torch.from_numpy(b.edge_off).cuda(),
            torch.from_numpy(np.ascontiguousarray(b.edges)).cuda())


def test_batch_small_mix(ctx):
    b = graphgen.batch(300, 17, lg_n_lo=0, lg_n_hi=13, deg_lo=0, deg_hi=20)
    vo, eo, ed = batch_to_dev(b)
    L, st = ctx.batch(vo, eo, ed)
    want, wst = oracle.cc_labels_batch(b.vtx_off, b.edge_off, b.edges)
    assert np.array_equal(st.cpu().numpy(), wst)
    assert_same_labels(L.cpu().numpy().view(np.uint32), want.view(np.uint32), "batch small mix")


def test_batch_graph_replays(ctx):
    """A captured batch replayed three times, with eager work between replays
    (labels and status clobbered, another batch run eagerly, the edges changed
    in place): every replay equals the oracle on the edges it saw."""
    graphs = [(graphgen.rmat(17, 1 << 19, 31), 90_000),           # above 2^16: HBM path
              (np.zeros((0, 2), np.uint32), 7)]
    graphs[0] = (graphs[0][0] % 90_000, 90_000)
    small = graphgen.batch(200, 18, lg_n_lo=0, lg_n_hi=14, deg_lo=0, deg_hi=24)
    for g in range(small.G):
        e = small.edges[small.edge_off[g]:small.edge_off[g + 1]]
        graphs.append((e, int(small.vtx_off[g + 1] - small.vtx_off[g])))
    b = graphgen.batch_from_graphs(graphs)
    vo, eo, ed = batch_to_dev(b)
    L = torch.empty(int(b.vtx_off[-1]), dtype=torch.int32, device="cuda")
    st = torch.empty(b.G, dtype=torch.int32, device="cuda")
    host_edges = b.edges.copy()
    with ctx.batch_graph(vo, eo, ed, L, st) as gr:
        other = graphgen.batch(50, 19, lg_n_lo=4, lg_n_hi=12)
        for rep in range(3):
            if rep == 1:                               # graph 5 loses its entries (self-loops)
                lo, hi = int(b.edge_off[5]), int(b.edge_off[6])
                host_edges[lo:hi] = 0
                ed[lo:hi] = 0
            if rep == 2:                               # graph 9 gets an out-of-range entry
                lo, hi = int(b.edge_off[9]), int(b.edge_off[10])
                n9 = int(b.vtx_off[10] - b.vtx_off[9])
                if hi > lo:
                    host_edges[lo] = (n9 + 3, 0)
                    ed[lo, 0] = n9 + 3
            L.fill_(-1)
            st.fill_(7)
            ovo, oeo, oed = batch_to_dev(other)
            ctx.batch(ovo, oeo, oed)                   # eager work in between
            torch.cuda.synchronize()
            gr.launch()
            torch.cuda.synchronize()
            want, wst = oracle.cc_labels_batch(b.vtx_off, b.edge_off, host_edges)
            got_st = st.cpu().numpy()
            assert np.array_equal(got_st, wst), f"replay {rep}: status"
            ok = np.repeat(wst == 0, np.diff(b.vtx_off))
            assert_same_labels(L.cpu().numpy().view(np.uint32)[ok], want.view(np.uint32)[ok],
                               f"replay {rep}")
        if int(b.edge_off[10]) > int(b.edge_off[9]):
            assert got_st[9] == cc.CC_ERANGE


def test_batch_handles_hbm_resident_graphs(ctx):
    """Graphs above the LDS capacity keep their parent array in HBM."""
    graphs = [(graphgen.rmat(17, 1 << 19, 3 + i) % (90_000 + i), 90_000 + i) for i in range(3)]
    graphs += [(graphgen.er(200, 150, 9), 200), (np.zeros((0, 2), np.uint32), 5),
               (graphgen.er(1 << 16, 1 << 18, 10), 1 << 16)]
    b = graphgen.batch_from_graphs(graphs)
    vo, eo, ed = batch_to_dev(b)
    L, st = ctx.batch(vo, eo, ed)
    want, _ = oracle.cc_labels_batch(b.vtx_off, b.edge_off, b.edges)
    assert np.all(st.cpu().numpy() == 0)
    assert_same_labels(L.cpu().numpy().view(np.uint32), want.view(np.uint32), "batch big graphs")


def test_batch_per_graph_status(ctx):
    graphs = [(np.array([[0, 1], [1, 2]], np.uint32), 3), (np.array([[0, 7]], np.uint32), 4),
              (np.array([[3, 2]], np.uint32), 4)]
    b = graphgen.batch_from_graphs(graphs)
    vo, eo, ed = batch_to_dev(b)
    L, st = ctx.batch(vo, eo, ed)
    assert st.cpu().tolist() == [cc.CC_OK, cc.CC_ERANGE, cc.CC_OK]
    Lh = L.cpu().numpy()
    assert Lh[0:3].tolist() == [0, 0, 0]
    assert Lh[7:11].tolist() == [0, 1, 2, 2]


def test_batch_edge_free(ctx):
    """Regression: graphs without entries issue no edge load. A batch with no
    entries at all passes a NULL edge pointer; a batch whose last graphs have no
    entries gives them a pointer one past the last entry. Both against the oracle."""
    sizes = [5, 1, 300, 70_000, 17]                    # 70,000 > 2^16: the HBM form
    b = graphgen.batch_from_graphs([(np.zeros((0, 2), np.uint32), n) for n in sizes])
    vo, eo, _ = batch_to_dev(b)
    ed = torch.empty((0, 2), dtype=torch.int32, device="cuda")   # passed as NULL
    log("edge-free batch: G=%d, NULL edges" % b.G)
    L, st = ctx.batch(vo, eo, ed)
    want, wst = oracle.cc_labels_batch(b.vtx_off, b.edge_off, b.edges)
    assert np.array_equal(st.cpu().numpy(), wst)
    assert_same_labels(L.cpu().numpy().view(np.uint32), want.view(np.uint32), "edge-free batch")

    graphs = [(graphgen.er(400, 900, 41), 400), (graphgen.er(3000, 5000, 42), 3000),
              (np.zeros((0, 2), np.uint32), 9), (np.zeros((0, 2), np.uint32), 70_001)]
    b = graphgen.batch_from_graphs(graphs)
    vo, eo, ed = batch_to_dev(b)
    log("batch ending in edge-free graphs: G=%d m=%d" % (b.G, int(b.edge_off[-1])))
    L, st = ctx.batch(vo, eo, ed)
    want, wst = oracle.cc_labels_batch(b.vtx_off, b.edge_off, b.edges)
    assert np.array_equal(st.cpu().numpy(), wst)
    assert_same_labels(L.cpu().numpy().view(np.uint32), want.view(np.uint32), "trailing empty")


def test_batch_4096_full(ctx):
    b = graphgen.batch_4096()
    log(f"batch generated: G={b.G} sum n={b.vtx_off[-1]} sum m={b.edge_off[-1]}")
    vo, eo, ed = batch_to_dev(b)
    L, st = ctx.batch(vo, eo, ed)
    want, wst = oracle.cc_labels_batch(b.vtx_off, b.edge_off, b.edges)
    log("batch oracle done")
    assert np.array_equal(st.cpu().numpy(), wst)
    Lh = L.cpu().numpy().view(np.uint32)
    assert_same_labels(Lh, want.view(np.uint32), "batch 4096")
    # the same graphs alone through cc_solve
    for g in list(range(0, b.G, 97)):
        e, n = b.graph(g)
        alone = to_host_u32(ctx.solve(to_dev(e.view(np.uint32)), n))
        assert_same_labels(Lh[b.vtx_off[g]:b.vtx_off[g + 1]], alone, f"graph {g} alone")


def _mixed_batch(seed, large=True):
    """Every role's case in one batch: tiny graphs on both sides of the wave
    limits (n 4,096, m 65,536), medium ones, graphs above 2^16 vertices on both
    sides of the whole-device thresholds, a tiny graph denser than the wave role
    takes, edge-free graphs (n = 0 included) and one out-of-range entry per size
    class. Returns the Batch and the indices of the bad graphs."""
    graphs = []
    tiny = graphgen.batch(500, seed, lg_n_lo=0, lg_n_hi=12.6, deg_lo=0, deg_hi=24)
    graphs += [tiny.graph(g) for g in range(tiny.G)]
    mid = graphgen.batch(30, seed + 1, lg_n_lo=12, lg_n_hi=16, deg_lo=1, deg_hi=16)
    graphs += [mid.graph(g) for g in range(mid.G)]
    graphs += [(graphgen.er(4096, 65536, seed + 2), 4096),      # at both wave limits
               (graphgen.er(4096, 65537, seed + 3), 4096),      # one entry too many
               (graphgen.er(64, 70_000, seed + 4), 64),         # dense tiny: tile role
               # either side of the 32-bit / 16-bit LDS entry limits (wave: 2,048
               # vertices; workgroup: 2^15) and of the LDS limit (2^16)
               (graphgen.er(2048, 9000, seed + 9), 2048), (graphgen.er(2049, 9000, seed + 10), 2049),
               (graphgen.er(1 << 15, 150_000, seed + 11), 1 << 15),
               (graphgen.er((1 << 15) + 1, 150_000, seed + 12), (1 << 15) + 1),
               (graphgen.er(1 << 16, 300_000, seed + 13), 1 << 16),
               (np.zeros((0, 2), np.uint32), 0), (np.zeros((0, 2), np.uint32), 5),
               (np.zeros((0, 2), np.uint32), 70_000)]
    if large:
        graphs += [(graphgen.rmat(17, 1 << 19, seed + 5) % 90_000, 90_000),
                   (graphgen.er(1 << 18, 1 << 20, seed + 6), 1 << 18),
                   (graphgen.rmat(19, 1 << 21, seed + 7), 1 << 19),
                   (graphgen.er(16_384, 40_000, seed + 8), 16_384)]
    with_entries = [g for g, (e, _) in enumerate(graphs) if len(e)]
    tiny_bad = next(g for g in with_entries if g < tiny.G)
    mid_bad = next(g for g in with_entries if g >= tiny.G)
    bad = [tiny_bad, mid_bad] + ([len(graphs) - 4] if large else [])
    for g in bad:
        e, n = graphs[g]
        e = np.array(e, np.int64)
        e[len(e) // 2, 1] = n + 1                                 # out of range
        graphs[g] = (e, n)
    return graphgen.batch_from_graphs(graphs), bad


SCHEDULES = [(0, 0), (4096, 0), (256, 0), (0, 1), (4096, 1), (4096, 65537), (1024, 16384),
             (0, 1 << 18)]


def _check_batch(b, L, st, what):
    want, wst = oracle.cc_labels_batch(b.vtx_off, b.edge_off, b.edges)
    assert np.array_equal(st.cpu().numpy(), wst), f"{what}: status"
    ok = np.repeat(wst == 0, np.diff(b.vtx_off))
    assert_same_labels(L.cpu().numpy().view(np.uint32)[ok], want.view(np.uint32)[ok], what)
    return wst


def test_batch_every_schedule(ctx):
    """Each schedule forced (cc_batch_ex), on a batch holding every role's
    cases: statuses and labels equal the oracle's."""
    b, bad = _mixed_batch(61)
    vo, eo, ed = batch_to_dev(b)
    log(f"mixed batch: G={b.G} sum n={int(b.vtx_off[-1])} sum m={int(b.edge_off[-1])} bad={bad}")
    for sc in SCHEDULES:
        log(f"schedule {sc}")
        L, st = ctx.batch(vo, eo, ed, sched=sc)
        wst = _check_batch(b, L, st, f"schedule {sc}")
        assert all(wst[g] == cc.CC_ERANGE for g in bad)


def _walk_heavy_batch(seed):
    """Graphs whose entries need long walks and many links at once: paths in
    shuffled, increasing and decreasing order (chains under link by index),
    stars with the hub last, a complete graph, on both sides of the wave role's
    2,048-vertex and the workgroup role's 2^15-vertex entry-width limits."""
    rng = np.random.default_rng(seed)
    graphs = []
    for n in (300, 2048, 2049, 4096, 20_000, 1 << 15, (1 << 15) + 1, 60_000):
        v = np.arange(n - 1, dtype=np.uint32)
        path = np.stack([v, v + 1], 1)
        graphs.append((path[rng.permutation(n - 1)], n))        # shuffled
        graphs.append((path, n))                                # increasing
        graphs.append((path[::-1].copy(), n))                   # decreasing
        star = np.stack([np.full(n - 1, n - 1, np.uint32), v], 1)
        graphs.append((star, n))
    k = 200
    iu = np.triu_indices(k, 1)
    graphs.append((np.stack(iu, 1).astype(np.uint32), k))       # complete graph
    return graphgen.batch_from_graphs(graphs)


def test_batch_long_walks(ctx):
    """Walk-heavy graphs under every schedule: labels equal the oracle's."""
    b = _walk_heavy_batch(63)
    vo, eo, ed = batch_to_dev(b)
    for sc in SCHEDULES:
        L, st = ctx.batch(vo, eo, ed, sched=sc)
        wst = _check_batch(b, L, st, f"walk-heavy schedule {sc}")
        assert np.all(wst == 0)


def test_batch_schedule_captured(ctx):
    """A captured batch takes the context's forced schedule (every role at once
    here) and its replays equal the oracle, with eager batches between them."""
    b, _ = _mixed_batch(62)
    vo, eo, ed = batch_to_dev(b)
    L = torch.empty(int(b.vtx_off[-1]), dtype=torch.int32, device="cuda")
    st = torch.empty(b.G, dtype=torch.int32, device="cuda")
    ctx.batch_sched_force((1024, 16384))
    try:
        with ctx.batch_graph(vo, eo, ed, L, st) as gr:
            for rep in range(3):
                L.fill_(-1)
                st.fill_(7)
                ctx.batch(vo, eo, ed, sched=(0, 0))            # eager work in between
                torch.cuda.synchronize()
                gr.launch()
                torch.cuda.synchronize()
                _check_batch(b, L, st, f"captured replay {rep}")
    finally:
        ctx.batch_sched_force(None)


def test_batch_tuner_and_cache(tmp_path):
    """cc_batch_tune times the candidates, stores the fastest for the batch's
    shape in the context and the cache file; a new context reads it back;
    forcing overrides it; batch_autotune tunes on first sight. Every run's labels
    equal the oracle's."""
    path = str(tmp_path / "tune.txt")
    b, _ = _mixed_batch(63)
    vo, eo, ed = batch_to_dev(b)
    c1 = cc.Context(tune_cache=path)
    try:
        r0, _, _ = c1.batch_tune(vo, eo, ed, reps=0)
        assert r0.source == cc.SCHED_DEFAULT and r0.n_cand == 0
        r, L, st = c1.batch_tune(vo, eo, ed, reps=2)
        _check_batch(b, L, st, "tuning runs")
        cands = r.candidates()
        log("candidates: " + ", ".join(f"{c}: {ms:.3f} ms" for c, ms in cands))
        assert r.source == cc.SCHED_TUNED and r.n_cand >= 4
        best = min(cands, key=lambda t: t[1])
        assert r.pick.as_tuple() == best[0]
        assert len({c for c, _ in cands}) == len(cands)
        r1, _, _ = c1.batch_tune(vo, eo, ed, reps=0)
        assert r1.source == cc.SCHED_STORED and r1.pick.as_tuple() == best[0]
        lines = open(path).read().splitlines()
        assert len(lines) == 1 and lines[0].startswith("ccmi-batch-tune-v1 ")
        f = lines[0].split()
        assert (int(f[3]), int(f[4])) == best[0]
        assert r.signature.decode() == f[1] + "|" + f[2]
    finally:
        c1.close()
    c2 = cc.Context(tune_cache=path)
    try:
        r2, _, _ = c2.batch_tune(vo, eo, ed, reps=0)
        assert r2.source == cc.SCHED_STORED and r2.pick.as_tuple() == best[0]
        L, st = c2.batch(vo, eo, ed)
        _check_batch(b, L, st, "stored pick")
        c2.batch_sched_force((4096, 0))
        r3, _, _ = c2.batch_tune(vo, eo, ed, reps=0)
        assert r3.source == cc.SCHED_FORCED and r3.pick.as_tuple() == (4096, 0)
        L, st = c2.batch(vo, eo, ed)
        _check_batch(b, L, st, "forced")
        c2.batch_sched_force(None)
        r4, _, _ = c2.batch_tune(vo, eo, ed, reps=0)
        assert r4.source == cc.SCHED_STORED
    finally:
        c2.close()
    c3 = cc.Context(tune_cache="", batch_autotune=True)
    try:
        L, st = c3.batch(vo, eo, ed)
        _check_batch(b, L, st, "autotuned")
        r5, _, _ = c3.batch_tune(vo, eo, ed, reps=0)
        assert r5.source == cc.SCHED_STORED
    finally:
        c3.close()
    with pytest.raises(cc.CCError):
        cc.Context(tune_cache="").batch(vo, eo, ed, sched=(8192, 0))   # above the wave cap


def _requests(count, seed, hi=2.0**24):
    reqs = graphgen.serve_stream(count, seed, rate_per_s=1e9, hi=hi)
    out = []
    for r in reqs:
        e = np.ascontiguousarray(r.edges().view(np.uint32).reshape(-1, 2))
        out.append((e, r.n))
    return out


def test_serve_full_pareto_range(ctx):
    """Served labels equal the oracle's and the graph solved alone, across the
    serving workload's whole size range: 160 requests drawn from it (n Pareto(1.5)
    on [2^10, 2^24], edgefactor 8..32, ER / R-MAT), plus its top end, which so few
    draws rarely reach: n = 2^24 (R-MAT, 2^27 entries), 2^22 (ER, 2^27 entries,
    zero root) and 2^20 (R-MAT, zero root), submitted mid-stream. Small requests
    go to batched launches, large ones to the single-graph path with scratch
    from the arena; every third request asks for the zero root."""
    reqs = [(e, n, cc.F_ZROOT if i % 3 == 0 else 0) for i, (e, n) in enumerate(_requests(160, 5))]
    top = [(graphgen.rmat(24, 8 << 24, 51), 1 << 24, 0),
           (graphgen.er(1 << 22, 32 << 22, 52), 1 << 22, cc.F_ZROOT),
           (graphgen.rmat(20, 16 << 20, 53), 1 << 20, cc.F_ZROOT)]
    reqs = reqs[:80] + top + reqs[80:]
    log(f"serving {len(reqs)} requests, largest n={max(n for _, n, _ in reqs)}")
    srv = cc.Server(ctx, streams=4, small_n=65536, coalesce_us=50)
    outs, tickets = [], []
    for e, n, fl in reqs:
        L = np.zeros(n, np.uint32)
        outs.append(L)
        tickets.append(srv.submit(e, n, L, flags=fl))
    stats = []
    for t in tickets:
        rc, st = srv.wait(t)
        assert rc == cc.CC_OK
        stats.append(st)
    srv.close()
    assert any(s.batched for s in stats) and any(not s.batched for s in stats)
    for s in stats:
        assert s.t_submit_ns <= s.t_admit_ns <= s.t_start_ns <= s.t_done_ns
    for i, ((e, n, fl), L) in enumerate(zip(reqs, outs)):
        assert_same_labels(L, oracle.cc_labels(n, e), f"served n={n} flags={fl}")
        if i % 10 == 0 or n >= 1 << 20:
            alone = to_host_u32(ctx.solve(to_dev(e), n, flags=fl))
            assert_same_labels(L, alone, f"served vs alone n={n}")
    log("served labels equal the oracle's")


def test_serve_share_mid_stream(ctx):
    """The serving workload's share-shaped request (one machine's 1/16 vertex-range
    share of R-MAT-30 ef16 with the global 2^30-entry parent array) submitted in
    the middle of a stream of small requests: its labels equal the oracle's (the
    recorded SHA-256 of all 2^30 labels), and so do the small requests' labels."""
    g = golden_share30()
    ed, n = graphgen.rmat30_share_dev()
    e_share = ed.cpu().numpy().view(np.uint32)
    del ed
    torch.cuda.empty_cache()
    assert sha256_of(e_share) == g["entries_sha256"]
    small = _requests(100, 77, hi=2.0**16)
    srv = cc.Server(ctx, streams=4, small_n=65536, hbm_budget=24 << 30)
    L_share = np.zeros(n, np.uint32)
    outs, tickets = [], []
    for i, (e, nn) in enumerate(small):
        if i == 50:
            t_share = srv.submit(e_share, n, L_share, flags=cc.F_ZROOT)
        L = np.zeros(nn, np.uint32)
        outs.append(L)
        tickets.append(srv.submit(e, nn, L))
    rc, st = srv.wait(t_share)
    assert rc == cc.CC_OK and not st.batched
    for t in tickets:
        assert srv.wait(t)[0] == cc.CC_OK
    srv.close()
    log(f"share served in {(st.t_done_ns - st.t_submit_ns) / 1e6:.1f} ms")
    assert sha256_of(L_share) == g["labels_sha256"], "served share labels differ from the oracle's"
    for (e, nn), L in zip(small, outs):
        assert_same_labels(L, oracle.cc_labels(nn, e), f"served n={nn}")


def test_serve_budget_errors_and_cancel(ctx):
    srv = cc.Server(ctx, streams=2, small_n=1024, hbm_budget=64 << 20)
    e = graphgen.er(4_000_000, 8_000_000, 3)          # 64 MB edges + 16 MB labels > arena
    L = np.zeros(4_000_000, np.uint32)
    with pytest.raises(cc.CCError) as ei:
        srv.submit(e, 4_000_000, L)
    assert ei.value.code == cc.CC_ENOMEM
    bad = np.array([[0, 5]], np.uint32)
    Lb = np.zeros(3, np.uint32)
    t = srv.submit(bad, 3, Lb)
    rc, _ = srv.wait(t)
    assert rc == cc.CC_ERANGE
    # requests submitted after close are refused; queued ones are cancelled or done
    ts = []
    for i in range(50):
        ee = graphgen.er(3000, 6000, 100 + i)
        ts.append((srv.submit(ee, 3000, np.zeros(3000, np.uint32)), ee))
    srv.close()


def test_serve_overlap_and_timestamps(ctx):
    reqs = _requests(300, 9, hi=2.0**15)
    srv = cc.Server(ctx, streams=4)
    outs, tickets = [], []
    t0 = time.monotonic()
    for e, n in reqs:
        L = np.zeros(n, np.uint32)
        outs.append(L)
        tickets.append(srv.submit(e, n, L))
    sts = [srv.wait(t)[1] for t in tickets]
    srv.close()
    log(f"300 requests in {time.monotonic() - t0:.3f} s")
    for s in sts:
        assert s.status == 0 and s.t_submit_ns <= s.t_admit_ns <= s.t_done_ns
    # requests in flight together: the most admit-to-done intervals that cover
    # one instant (a sweep over the interval ends)
    ev = sorted([(s.t_admit_ns, 1) for s in sts] + [(s.t_done_ns, -1) for s in sts],
                key=lambda x: (x[0], x[1]))
    depth = peak = 0
    for _, d in ev:
        depth += d
        peak = max(peak, depth)
    log(f"at most {peak} requests in flight together")
    assert peak >= 2, "no two requests were in flight together"
    for (e, n), L in zip(reqs[:40], outs[:40]):
        assert_same_labels(L, oracle.cc_labels(n, e), f"served n={n}")
