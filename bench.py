#!/usr/bin/env python3
"""Benchmark of the connected-components path on one MI355X.

A step is one pass of the whole single-graph path over the workload, with the
edge list already resident in HBM: init, zero root (sampled), Initial Push,
hook, compress and the zero-component relabelling (flags CC_F_ZROOT), i.e.
cc_init / cc_zroot / cc_push / cc_hook / cc_compress enqueued on one stream
(cc_compress with CC_F_CANON relabels the zero root's component in the same
pass, as cc_solve does). The hook step (one cc_hook call: on the zero-root path a short direct
hook over 1/1024 of the entries, two partition passes, the membership filter and
the hook of the surviving entries)
is bracketed by its own HIP events on that stream inside the timed region; the
roofline figure is its algorithmic bytes (8 per entry) over that duration,
against the 8 TB/s peak and against a 4 GiB device copy timed in the same run.

Prints one JSON line. Default workload: R-MAT scale 26, edgefactor 16, permuted
IDs, plus 1 % isolated vertices and 10,000 paths of 2..64 vertices.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the cc_hook step, from two rocprofv3 --pmc runs
# (FETCH_SIZE, WRITE_SIZE) of this script with --steps 1 --warmup 0 --calibrate,
# each counter scaled by what it reads for a 4 GiB device copy. Keyed by
# (workload, variant); valid only for the kernel sources they were taken on.
TRAFFIC = {
    ("rmat26", "zroot"): {"bytes": 47675427858,
                          "src_sha256": "79fdac7860482c903d4075846773a3fa101d6720866dc40dfa7e87b00ae6162c"},
}

HOOK_KERNELS = {
    "zroot": "cc_hook step: k_hook<ZR> on 1/1024 of the entries, k_t1_part, k_t1_tsum, k_t1_scan, "
             "k_t1_bases, k_t2_bounds, k_t2_part, k_t3_regions, k_t3_offsets, k_t3_filter, k_t4_scan, "
             "k_t4_hook",
    "plain": "cc_hook step: k_t1_part, k_t1_tsum, k_t1_scan, k_t1_bases, k_t2_bounds, "
             "k_t2_hookplain",
}


# The sources of the kernels of the timed hook step (every kernel of it, and
# the header they share); the HBM traffic figure is reported only while these
# hash to the value it was measured on.
HOOK_SOURCES = ("cc_internal.h", "cc_kernels.hip", "cc_tiled.hip")


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for name in HOOK_SOURCES:
        h.update(name.encode())
        with open(os.path.join(HERE, "paper_2507_03695_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload, variant):
    t = TRAFFIC.get((workload, variant))
    if t is None or t["src_sha256"] != kernel_sources_sha256():
        return None
    return t["bytes"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name):
    import graphgen
    if name == "rmat26":
        g = graphgen.rmat26_extras()
        return g.edges, g.n, {"workload": "rmat26_ef16_permuted+1pct_isolated+10k_paths",
                              "scale": 26, "edgefactor": 16, "n": g.n, "m": int(len(g.edges))}
    if name == "rmat22":
        e, n = graphgen.rmat22_sym()
        return e, n, {"workload": "rmat22_ef16_permuted_symmetrised", "scale": 22,
                      "edgefactor": 16, "n": n, "m": int(len(e))}
    if name == "er65k":
        e, n = graphgen.er_65k()
        return e, n, {"workload": "er_n65536_m1048576", "n": n, "m": int(len(e))}
    raise SystemExit(f"unknown workload {name}")


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(edges, n, target_s=15.0):
    """The oracle on a bounded prefix of the same entries, on one host thread
    pinned to one core (the first core this process may run on)."""
    import oracle
    allowed = sorted(os.sched_getaffinity(0))
    os.sched_setaffinity(0, {allowed[0]})
    m = len(edges)
    k = min(m, 1 << 22)
    while True:
        t0 = time.perf_counter()
        oracle.cc_labels(n, edges[:k])
        t1 = time.perf_counter() - t0
        if t1 >= 0.6 * target_s or k == m:
            break
        # the time per entry grows with the prefix (the touched part of the
        # parent array outgrows the caches), so grow the sample in steps
        k = int(min(m, k * min(4.0, max(1.5, target_s / max(t1, 1e-3)))))
    os.sched_setaffinity(0, set(allowed))
    return {"value": round(k / t1 / 1e9, 6), "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "host_cpu": host_cpu_model(), "pinned_core": allowed[0],
            "sample": f"first {k} of {m} entries with all {n} vertices; union-find + min-ID pass, "
                      f"{t1:.2f} s on one host thread pinned to core {allowed[0]}"}


def bench_single(cc, torch, ed, n, m, steps, warmup, flags):
    ctx = cc.Context()
    stream = torch.cuda.current_stream()
    L = torch.empty(n, dtype=torch.int32, device="cuda")

    def one_step(ev=None):
        ctx.init(n, L, stream)
        if flags & cc.F_ZROOT:
            ctx.zroot(ed, n, flags=flags, stream=stream)
            ctx.push(ed, n, L, stream=stream)
        if ev is not None:
            ev[0].record(stream)
        ctx.hook(ed, n, L, flags=flags, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        # with a zero root, the relabelling of its component is done in the
        # same pass (CC_F_CANON), as in cc_solve
        ctx.compress(n, L, flags=flags | cc.F_CANON, stream=stream)

    for _ in range(warmup):
        one_step()
    rc = ctx.sync(stream)
    assert rc == cc.CC_OK, rc
    hook_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for i in range(steps):
        one_step(hook_ev[i])
    end.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(end)
    hook_ms = [a.elapsed_time(b) for a, b in hook_ev]
    rc = ctx.sync(stream)
    assert rc == cc.CC_OK, rc
    ctx.close()
    return total_ms / steps, float(np.mean(hook_ms)), L


def bench_small(cc, torch, name, steps=40, warmup=5):
    """A configuration below the headline's size, plain path as the workload names
    it: the whole path (one cc_solve_async per step, steps back to back on one
    stream, HIP events around them) and the hook launch alone (events around
    cc_hook in a step-wise solve), each against the HBM roofline of its
    algorithmic bytes (whole path: 8 B per entry read, 12 B per vertex for init,
    compress and the label write; hook: 8 B per entry)."""
    edges, n, cfg = make_workload(name)
    m = len(edges)
    ed = torch.from_numpy(edges.view(np.int32)).cuda()
    flags = cc.F_SYMMETRIC if name == "rmat22" else 0
    ctx = cc.Context()
    stream = torch.cuda.current_stream()
    L = torch.empty(n, dtype=torch.int32, device="cuda")
    for _ in range(warmup):
        ctx.solve_async(ed, n, L, flags=flags, stream=stream)
    assert ctx.sync(stream) == cc.CC_OK
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(steps):
        ctx.solve_async(ed, n, L, flags=flags, stream=stream)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    assert ctx.sync(stream) == cc.CC_OK
    ctx.close()
    _, hook_ms, L2 = bench_single(cc, torch, ed, n, m, max(5, steps // 4), 2, flags)
    same = bool(torch.equal(L, L2))
    whole = (8 * m + 12 * n) / (ms * 1e-3) / 1e9
    hook = 8 * m / (hook_ms * 1e-3) / 1e9
    return {"workload": cfg["workload"], "n": n, "m": m,
            "flags": "CC_F_SYMMETRIC" if flags else "plain",
            "ms_per_solve": round(ms, 4), "GTEPS": round(m / (ms * 1e-3) / 1e9, 3),
            "whole_path_GBps": round(whole, 1),
            "whole_path_roofline_frac": round(whole / PEAK_HBM_GBS, 4),
            "hook_ms": round(hook_ms, 4), "hook_GBps": round(hook, 1),
            "hook_roofline_frac": round(hook / PEAK_HBM_GBS, 4),
            "identical_labels_step_vs_whole": same}


def _time_batch(ctx, torch, vo, eo, ed, L, st, reps, sched=None):
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        ctx.batch(vo, eo, ed, L, st, sched=sched)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def _tune_report(r):
    """The tuner's candidates (best-of-reps device time, upload to end of launch)
    and its pick."""
    return {"signature": r.signature.decode(),
            "candidates_ms": {f"wave{c[0]}_multi{c[1]}": round(ms, 4) for c, ms in r.candidates()},
            "pick": {"wave_max_n": int(r.pick.wave_max_n), "multi_min_n": int(r.pick.multi_min_n)}}


def bench_batch(cc, torch, reps=5):
    """4,096 graphs: the tuner's candidates, then one persistent cc_batch launch
    with its pick (and its captured graph replayed) vs the fixed
    workgroup-per-graph schedule and vs one cc_solve_async per graph."""
    import graphgen
    b = graphgen.batch_4096()
    vo = torch.from_numpy(b.vtx_off).cuda()
    eo = torch.from_numpy(b.edge_off).cuda()
    ed = torch.from_numpy(np.ascontiguousarray(b.edges)).cuda()
    ctx = cc.Context(tune_cache="")
    L = torch.empty(int(b.vtx_off[-1]), dtype=torch.int32, device="cuda")
    st = torch.empty(b.G, dtype=torch.int32, device="cuda")
    tune, _, _ = ctx.batch_tune(vo, eo, ed, L, st, reps=3)
    ctx.batch(vo, eo, ed, L, st)
    torch.cuda.synchronize()
    t_batch = _time_batch(ctx, torch, vo, eo, ed, L, st, reps)
    Lf = torch.empty_like(L)
    stf = torch.empty_like(st)
    t_fixed = _time_batch(ctx, torch, vo, eo, ed, Lf, stf, reps, sched=(0, 0))
    same_fixed = bool(torch.equal(Lf, L)) and bool(torch.equal(stf, st))
    del Lf, stf
    # the same batch captured once (host work done at capture) and replayed
    Lg = torch.empty_like(L)
    stg = torch.empty_like(st)
    gr = ctx.batch_graph(vo, eo, ed, Lg, stg)
    gr.launch()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        gr.launch()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    t_graph = float(np.median(ts))
    same_graph = bool(torch.equal(Lg, L)) and bool(torch.equal(stg, st))
    gr.close()
    # per-graph launches on one stream
    L2 = torch.empty_like(L)
    views = [(ed[b.edge_off[g]:b.edge_off[g + 1]], int(b.vtx_off[g + 1] - b.vtx_off[g]),
              L2[b.vtx_off[g]:b.vtx_off[g + 1]]) for g in range(b.G)]
    stream = torch.cuda.current_stream()
    for e, n, l in views:
        ctx.solve_async(e, n, l, stream=stream)
    ctx.sync(stream)
    ts = []
    for _ in range(max(1, reps // 2)):
        t0 = time.perf_counter()
        for e, n, l in views:
            ctx.solve_async(e, n, l, stream=stream)
        ctx.sync(stream)
        ts.append(time.perf_counter() - t0)
    t_loop = float(np.median(ts))
    same = bool(torch.equal(L, L2))
    ctx.close()
    m = int(b.edge_off[-1])
    sum_n = int(b.vtx_off[-1])
    # compulsory HBM bytes with parent arrays in LDS: the entries once (8 B) and
    # the labels written once (4 B per vertex)
    alg = 8 * m + 4 * sum_n
    return {"graphs": b.G, "sum_n": sum_n, "sum_m": m,
            "tuner": _tune_report(tune),
            "batched_graphs_per_s": round(b.G / t_batch, 1),
            "batched_ms": round(t_batch * 1e3, 3),
            "fixed_wg_per_graph_ms": round(t_fixed * 1e3, 3),
            "fixed_identical": same_fixed,
            "algorithmic_bytes": alg,
            "achieved_GBps": round(alg / t_batch / 1e9, 1),
            "hbm_roofline_frac": round(alg / t_batch / 1e9 / PEAK_HBM_GBS, 4),
            "graph_replay_ms": round(t_graph * 1e3, 3), "graph_replay_identical": same_graph,
            "per_graph_launch_graphs_per_s": round(b.G / t_loop, 1),
            "per_graph_launch_ms": round(t_loop * 1e3, 3),
            "speedup": round(t_loop / t_batch, 2), "identical_labels": same}


def _bench_batch_mix(cc, torch, b, reps=5):
    """The tuner's candidates and pick on batch b, then b under the pick against
    the fixed workgroup-per-graph schedule (labels equal; the oracle parity of
    every schedule is a GPU test)."""
    vo = torch.from_numpy(b.vtx_off).cuda()
    eo = torch.from_numpy(b.edge_off).cuda()
    ed = torch.from_numpy(np.ascontiguousarray(b.edges)).cuda()
    ctx = cc.Context(tune_cache="")
    L = torch.empty(int(b.vtx_off[-1]), dtype=torch.int32, device="cuda")
    st = torch.empty(b.G, dtype=torch.int32, device="cuda")
    tune, _, _ = ctx.batch_tune(vo, eo, ed, L, st, reps=3)
    t_pick = _time_batch(ctx, torch, vo, eo, ed, L, st, reps)
    Lf = torch.empty_like(L)
    stf = torch.empty_like(st)
    t_fixed = _time_batch(ctx, torch, vo, eo, ed, Lf, stf, max(1, reps // 2), sched=(0, 0))
    same = bool(torch.equal(Lf, L)) and bool(torch.equal(stf, st))
    ctx.close()
    m = int(b.edge_off[-1])
    return {"graphs": b.G, "sum_n": int(b.vtx_off[-1]), "sum_m": m,
            "tuner": _tune_report(tune),
            "pick_ms": round(t_pick * 1e3, 3), "fixed_wg_per_graph_ms": round(t_fixed * 1e3, 3),
            "pick_speedup_over_fixed": round(t_fixed / t_pick, 2),
            "pick_graphs_per_s": round(b.G / t_pick, 1),
            "identical_labels": same}


def bench_batch_tail(cc, torch, reps=5):
    """The 4,096-graph mix with its last 8 graphs replaced by R-MAT scale-20,
    edgefactor-8 graphs (the whole-device role's case)."""
    import graphgen
    return _bench_batch_mix(cc, torch, graphgen.batch_with_tail(graphgen.config_seed(4)), reps)


def bench_batch_tiny(cc, torch, reps=5):
    """16,384 small graphs: n log-uniform in [2^5, 2^10], average degree uniform in
    [2, 8] (the wavefront role's case)."""
    import graphgen
    b = graphgen.batch(16384, graphgen.config_seed(4) ^ 0x7157, lg_n_lo=5.0, lg_n_hi=10.0,
                       deg_lo=2.0, deg_hi=8.0)
    return _bench_batch_mix(cc, torch, b, reps)


def bench_reducer(cc, torch, ed, n, L_ref, g=16, reps=3):
    """Reducer emulation (Sec. III / IV / V): the workload's entries split into g
    shares by the first endpoint's vertex range, each solved into its own
    global-size parent array with the global zero root, exported as (v, P_v)
    pairs and zero-converged IDs, sent through the compact-ID codec (Sec. V) and
    merged by a Reducer. Reports the message counts against Sec. V's
    min(|E|, (g-1)|V|), the bytes on the wire and the time of each phase."""
    m = ed.shape[0]
    u = ed[:, 0].to(torch.int64) & 0xFFFFFFFF
    k = (u * g) // n
    parts = [ed[k == s].contiguous() for s in range(g)]
    del u, k
    ctx = cc.Context()
    stream = torch.cuda.current_stream()
    Ps = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in range(g)]
    L = torch.empty(n, dtype=torch.int32, device="cuda")
    ctx.init(n, L)
    ctx.zroot(ed, n)
    z = ctx.get_zroot()
    hint = cc.F_ZROOT | cc.F_ZROOT_HINT
    ev = lambda: torch.cuda.Event(enable_timing=True)
    kb = ctx.id_bytes(n)                                    # compact IDs of Sec. V
    res = []
    for rep in range(reps):
        e0, e1, e2, e3, e4, e5 = ev(), ev(), ev(), ev(), ev(), ev()
        e0.record(stream)
        for P, es in zip(Ps, parts):
            ctx.init(n, P, stream)
            ctx.zroot(es, n, flags=hint, zroot_hint=z, stream=stream)
            ctx.push(es, n, P, stream=stream)
            ctx.hook(es, n, P, flags=cc.F_ZROOT, stream=stream)
            ctx.compress(n, P, flags=cc.F_ZROOT, stream=stream)
        e1.record(stream)
        exported = [ctx.export_lists(P, n, z, stream=stream) for P in Ps]
        pairs = torch.cat([p for p, _ in exported])
        zero = torch.cat([q for _, q in exported])
        del exported
        e2.record(stream)
        # on the wire: every ID in kb bytes; the Reducer works on what it decodes
        wire_p = ctx.pack_ids(pairs, kb, stream=stream)
        wire_z = ctx.pack_ids(zero, kb, stream=stream)
        e3.record(stream)
        pairs2 = ctx.unpack_ids(wire_p, pairs.numel(), kb, stream=stream).view(-1, 2)
        zero2 = ctx.unpack_ids(wire_z, zero.numel(), kb, stream=stream)
        e4.record(stream)
        wire_bytes = wire_p.numel() + wire_z.numel()
        del wire_p, wire_z
        assert torch.equal(pairs2, pairs) and torch.equal(zero2, zero)
        pairs, zero = pairs2, zero2
        e4b = ev()
        e4b.record(stream)
        ctx.init(n, L, stream)
        ctx.zroot(pairs, n, flags=hint, zroot_hint=z, stream=stream)
        ctx.hook(pairs, n, L, flags=cc.F_ZROOT, stream=stream)
        ctx.hook_ids(zero, z, n, L, flags=cc.F_ZROOT, stream=stream)
        ctx.compress(n, L, flags=cc.F_ZROOT, stream=stream)
        ctx.canon(n, L, stream=stream)
        e5.record(stream)
        assert ctx.sync(stream) == cc.CC_OK
        res.append((e0.elapsed_time(e1), e1.elapsed_time(e2), e4b.elapsed_time(e5),
                    int(pairs.shape[0]), int(zero.shape[0]), e2.elapsed_time(e3),
                    e3.elapsed_time(e4), wire_bytes))
        del pairs, zero
    same = bool(torch.equal(L, L_ref))
    ctx.close()
    med = lambda i: float(np.median([r[i] for r in res]))
    npairs, nzero = res[-1][3], res[-1][4]
    return {"shares": g, "zero_root": z,
            "pairs": npairs, "zero_ids": nzero,
            "bound_min_E_gm1V": min(m, (g - 1) * n),
            "id_bytes": kb, "message_bytes": res[-1][7],
            "message_bytes_without_zero_ids": (npairs + nzero) * 2 * kb,
            "share_solves_ms": round(med(0), 3), "export_ms": round(med(1), 3),
            "pack_ms": round(med(5), 3), "unpack_ms": round(med(6), 3),
            "reducer_ms": round(med(2), 3), "identical_labels": same}


def bench_serve(cc, torch, count=3000, seed=0x2507036950000005):
    """Poisson streams of requests (truncated Pareto n in [2^10, 2^24], edgefactor
    8-32, R-MAT/ER) through cc_serve and through a FIFO plain-path server (one
    stream, no batching, one request in flight) at the same offered rates:
    rho = 0.5, 0.9 and 1.2 of the FIFO server's capacity, and 1.25 of the
    server's own. Capacities are whole streams submitted at once (the better of
    two runs). At rho = 0.9
    the R-MAT-30 share (one machine's 1/16 vertex range with the global 2^30
    parent array) is submitted in the middle of the stream. p50/p99 latency from
    submission to labels in host memory."""
    import graphgen
    reqs = graphgen.serve_stream(count, seed, rate_per_s=1.0)
    data = []
    for r in reqs:
        e = np.ascontiguousarray(r.edges().view(np.uint32).reshape(-1, 2))
        data.append((e, r.n))

    def run(srv_kwargs, rate, share=None):
        ctx = cc.Context()
        srv = cc.Server(ctx, **srv_kwargs)
        outs = [np.empty(n, np.uint32) for _, n in data]
        tickets = []
        t_share = None
        t0 = time.perf_counter()
        for i, ((e, n), r) in enumerate(zip(data, reqs)):
            due = t0 + r.arrival_s / rate
            while time.perf_counter() < due:
                pass
            if share is not None and i == count // 2:
                t_share = srv.submit(share[0], share[1], share[2], flags=cc.F_ZROOT)
            tickets.append(srv.submit(e, n, outs[i]))
        lat, first, last = [], None, 0
        for t in tickets:
            rc, s = srv.wait(t)
            assert rc == cc.CC_OK, rc
            lat.append((s.t_done_ns - s.t_submit_ns) / 1e6)
            first = s.t_submit_ns if first is None else min(first, s.t_submit_ns)
            last = max(last, s.t_done_ns)
        share_ms = None
        if t_share is not None:
            rc, s = srv.wait(t_share)
            assert rc == cc.CC_OK, rc
            share_ms = (s.t_done_ns - s.t_submit_ns) / 1e6
        srv.close()
        ctx.close()
        lat = np.array(lat)
        # the stream's own requests over their own span (first submission to last
        # labels in host memory), the share excluded
        return outs, {"served_graphs_per_s": round(count / ((last - first) * 1e-9), 1),
                      "p50_ms": round(float(np.percentile(lat, 50)), 3),
                      "p99_ms": round(float(np.percentile(lat, 99)), 3)}, share_ms

    fifo = {"streams": 1, "small_n": 1, "max_inflight": 1}
    served = {"streams": 4}

    def capacity(kw):
        # the better of two all-at-once runs (a single one varied by a third)
        a, b = run(kw, 1e12), run(kw, 1e12)
        return a if a[1]["served_graphs_per_s"] >= b[1]["served_graphs_per_s"] else b

    outs_fifo, st_fifo, _ = capacity(fifo)
    cap_fifo = st_fifo["served_graphs_per_s"]
    outs_cap, st_cap, _ = capacity(served)
    cap_srv = st_cap["served_graphs_per_s"]
    same = all(np.array_equal(a, b) for a, b in zip(outs_cap, outs_fifo))
    # the share, generated on the device and held in host memory like any request
    ed, n_share = graphgen.rmat30_share_dev()
    e_share = ed.cpu().numpy().view(np.uint32)
    del ed
    torch.cuda.empty_cache()
    L_share = np.empty(n_share, np.uint32)
    loads = []
    for rho, base in ((0.5, cap_fifo), (0.9, cap_fifo), (1.2, cap_fifo), (1.25, cap_srv)):
        rate = rho * base
        with_share = rho == 0.9 and base == cap_fifo
        outs, st, share_ms = run(served, rate, (e_share, n_share, L_share) if with_share else None)
        same = same and all(np.array_equal(a, b) for a, b in zip(outs, outs_fifo))
        _, st_f, _ = run(fifo, rate)
        entry = {"offered_per_s": round(rate, 1),
                 "rho_of": "fifo_capacity" if base == cap_fifo else "server_capacity",
                 "rho": rho, "server": st, "fifo": st_f}
        if share_ms is not None:
            entry["share_rmat30_in_stream_ms"] = round(share_ms, 1)
        loads.append(entry)
    return {"requests": count, "fifo_capacity_graphs_per_s": cap_fifo,
            "server_capacity_graphs_per_s": cap_srv,
            "server_p50_ms_at_capacity": st_cap["p50_ms"], "server_p99_ms_at_capacity": st_cap["p99_ms"],
            "fifo_p50_ms_at_capacity": st_fifo["p50_ms"], "fifo_p99_ms_at_capacity": st_fifo["p99_ms"],
            "loads": loads, "identical_to_fifo": same,
            "share_rmat30": {"n": n_share, "m": int(len(e_share)), "flags": "CC_F_ZROOT",
                             "submitted_at_request": count // 2}}


def bench_update_log(cc, torch, ed, n, L_ref, g=16, reps=3):
    """SiskinCC's update log (Sec. III, Algorithm 2). (1) The direct plain hook over
    the whole workload with every link appended to a log, against the same hook
    without it; the message count must be n minus the number of components.
    (2) SiskinCC over g shares: each share hooks into its own parent array and
    appends its links to one receive buffer (no compress, no export); the
    Reducer hooks the buffer as edges and compresses."""
    m = ed.shape[0]
    ctx = cc.Context()
    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    want = int((L_ref != torch.arange(n, device=L_ref.device, dtype=L_ref.dtype)).sum())
    P = torch.empty(n, dtype=torch.int32, device="cuda")
    buf = torch.empty((n, 2), dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    t_log, t_direct = [], []
    for rep in range(reps + 1):
        # the logged hook is the direct (entry-order) hook; its cost is compared
        # with the same hook without the log
        ctx.init(n, P, stream)
        a, b = ev(), ev()
        a.record(stream)
        ctx.hook(ed, n, P, flags=cc.F_NO_TILE, stream=stream)
        b.record(stream)
        ctx.init(n, P, stream)
        cnt.zero_()
        c_, d_ = ev(), ev()
        c_.record(stream)
        ctx.hook_log(ed, n, P, buf, cnt, stream=stream)
        d_.record(stream)
        assert ctx.sync(stream) == cc.CC_OK
        assert int(cnt.item()) == want, (int(cnt.item()), want)
        if rep:
            t_direct.append(a.elapsed_time(b))
            t_log.append(c_.elapsed_time(d_))
    hook_plain_ms = float(np.median(t_direct))
    ctx.compress(n, P, stream=stream)
    assert ctx.sync(stream) == cc.CC_OK
    same_single = bool(torch.equal(P, L_ref))
    # the messages delivered to host memory: drained launch by launch while the
    # pass runs (cc_hook_log_drain, 8 launches), against the logged hook followed
    # by one copy of the whole log (the same pinned buffer); wall time of each
    host = torch.empty((n, 2), dtype=torch.int32, pin_memory=True)
    t_drain, t_after = [], []
    for rep in range(reps + 1):
        ctx.init(n, P, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k_drain = ctx.hook_log_drain(ed, n, P, buf, host, chunks=8, stream=stream)
        t1 = time.perf_counter()
        ctx.init(n, P, stream)
        cnt.zero_()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ctx.hook_log(ed, n, P, buf, cnt, stream=stream)
        k_after = int(cnt.item())                       # waits for the hook
        host[:k_after].copy_(buf[:k_after])
        t3 = time.perf_counter()
        assert k_drain == k_after == want, (k_drain, k_after, want)
        if rep:
            t_drain.append((t1 - t0) * 1e3)
            t_after.append((t3 - t2) * 1e3)
    assert ctx.sync(stream) == cc.CC_OK
    drained = {"launches": 8, "messages": k_drain,
               "drained_ms": round(float(np.median(t_drain)), 3),
               "hook_then_copy_ms": round(float(np.median(t_after)), 3),
               "message_bytes_to_host": 8 * k_drain}
    del buf, host
    torch.cuda.empty_cache()

    u = ed[:, 0].to(torch.int64) & 0xFFFFFFFF
    k = (u * g) // n
    parts = [ed[k == s].contiguous() for s in range(g)]
    del u, k
    Ps = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in range(g)]
    recv = torch.empty((m, 2), dtype=torch.int32, device="cuda")   # <= min(|E|, g|V|) messages
    res = []
    for rep in range(reps):
        e0, e1, e2 = ev(), ev(), ev()
        cnt.zero_()
        e0.record(stream)
        for Ps_, es in zip(Ps, parts):
            ctx.init(n, Ps_, stream)
            ctx.hook_log(es, n, Ps_, recv, cnt, stream=stream)
        e1.record(stream)
        assert ctx.sync(stream) == cc.CC_OK
        sent = int(cnt.item())
        ctx.init(n, P, stream)
        # a message list: every vertex recurs once per share, so it is hooked in
        # the given order (grouping it by first endpoint makes the links contend)
        ctx.hook(recv[:sent], n, P, flags=cc.F_NO_TILE, stream=stream)
        ctx.compress(n, P, stream=stream)
        e2.record(stream)
        assert ctx.sync(stream) == cc.CC_OK
        res.append((e0.elapsed_time(e1), e1.elapsed_time(e2), sent))
    same = bool(torch.equal(P, L_ref))
    ctx.close()
    del Ps, recv, parts, P
    torch.cuda.empty_cache()
    med = lambda i: float(np.median([r[i] for r in res]))
    id_bytes = max(1, ((n - 1).bit_length() + 7) // 8)
    hl = float(np.median(t_log))
    return {"messages": want, "n_minus_components": want,
            "hook_log_ms": round(hl, 3), "hook_ms": round(hook_plain_ms, 3),
            "overhead": round(hl / hook_plain_ms - 1.0, 4), "identical_labels": same_single,
            "drained_to_host": drained,
            "siskin_shares": g, "siskin_messages": res[-1][2],
            "siskin_bound_min_E_gV": min(m, g * n),
            "siskin_message_bytes": res[-1][2] * 2 * id_bytes,
            "siskin_share_hooks_ms": round(med(0), 3), "siskin_reducer_ms": round(med(1), 3),
            "siskin_identical_labels": same}


def bench_csr(cc, torch, ed, n, L_ref, steps=3):
    """CSR input (cc_solve_csr): the workload's entries grouped by first endpoint
    (stable, so rows keep entry order), solved with the exact longest-row zero
    root and on the plain path. The conversion is not timed; each step is one
    cc_solve_csr (init, zero root, push, hook, compress, canon)."""
    m = ed.shape[0]
    u = ed[:, 0]
    order = torch.argsort(u, stable=True)
    adj = ed[:, 1][order].contiguous()
    del order
    off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    off[1:] = torch.cumsum(torch.bincount(u, minlength=n), 0)
    torch.cuda.synchronize()
    ctx = cc.Context()
    stream = torch.cuda.current_stream()
    L = torch.empty(n, dtype=torch.int32, device="cuda")
    out = {}
    for name, flags in (("zroot", cc.F_ZROOT), ("plain", 0)):
        ctx.solve_csr_async(off, adj, n, L, flags=flags, stream=stream)
        assert ctx.sync(stream) == cc.CC_OK
        ts = []
        for _ in range(steps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            ctx.solve_csr_async(off, adj, n, L, flags=flags, stream=stream)
            b.record(stream)
            assert ctx.sync(stream) == cc.CC_OK
            ts.append(a.elapsed_time(b))
        ms = float(np.median(ts))
        # compulsory bytes: adj once (4 B per entry), the offsets once (8 B per
        # row), and 12 B per vertex (init, compress, labels)
        alg = 4 * m + 8 * (n + 1) + 12 * n
        out[name] = {"ms_per_step": round(ms, 3), "GTEPS": round(m / (ms * 1e-3) / 1e9, 3),
                     "hbm_roofline_frac_whole_path": round(alg / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                     "identical_labels": bool(torch.equal(L, L_ref))}
        if flags:
            out[name]["zero_root_exact"] = ctx.get_zroot()
    ctx.close()
    del adj, off, L
    torch.cuda.empty_cache()
    return out


def bench_u64(cc, torch, ed, n, L_ref, steps=3):
    """8-byte IDs (cc_solve_u64, plain path): the same workload with every ID
    widened to uint64 (16 B per entry, 8 B per vertex)."""
    m = ed.shape[0]
    e64 = ed.to(torch.int64) & 0xFFFFFFFF
    ctx = cc.Context()
    stream = torch.cuda.current_stream()
    L = torch.empty(n, dtype=torch.int64, device="cuda")
    ctx.solve_u64_async(e64, n, L, stream=stream)
    assert ctx.sync(stream) == cc.CC_OK
    ts = []
    for _ in range(steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        ctx.solve_u64_async(e64, n, L, stream=stream)
        b.record(stream)
        assert ctx.sync(stream) == cc.CC_OK
        ts.append(a.elapsed_time(b))
    same = bool(torch.equal(L, L_ref.to(torch.int64) & 0xFFFFFFFF))
    ctx.close()
    del e64, L
    torch.cuda.empty_cache()
    ms = float(np.median(ts))
    return {"variant": "plain", "ms_per_step": round(ms, 3),
            "GTEPS": round(m / (ms * 1e-3) / 1e9, 3), "identical_labels": same}


def bench_share30(cc, torch, steps=2):
    """One machine's share of R-MAT-30 ef16 (entries whose first endpoint lies in the
    first of 16 equal vertex ranges; n = 2^30 stays global, about 2^30 entries),
    generated on the device; whole solves on both paths."""
    import graphgen
    ed, n = graphgen.rmat30_share_dev()
    m = ed.shape[0]
    ctx = cc.Context()
    stream = torch.cuda.current_stream()
    out = {"n": n, "m": m}
    Ls = {}
    for name, flags in (("zroot", cc.F_ZROOT), ("plain", 0)):
        L = torch.empty(n, dtype=torch.int32, device="cuda")
        ctx.solve_async(ed, n, L, flags=flags, stream=stream)
        assert ctx.sync(stream) == cc.CC_OK
        ts = []
        for _ in range(steps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            ctx.solve_async(ed, n, L, flags=flags, stream=stream)
            b.record(stream)
            assert ctx.sync(stream) == cc.CC_OK
            ts.append(a.elapsed_time(b))
        ms = float(np.median(ts))
        out[name] = {"ms_per_step": round(ms, 3), "GTEPS": round(m / (ms * 1e-3) / 1e9, 3),
                     "hbm_roofline_frac_whole_path":
                         round((8 * m + 12 * n) / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
        Ls[name] = L
    out["identical_labels"] = bool(torch.equal(Ls["zroot"], Ls["plain"]))
    ctx.close()
    del ed, Ls
    torch.cuda.empty_cache()
    return out


def copy_ceiling_gbs(torch, reps=5):
    """Measured HBM ceiling: a plain device copy of 4 GiB (4 GiB read and 4 GiB
    written per launch), timed with HIP events on the current stream."""
    src = torch.ones(1 << 30, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * (4 << 30) / (ms * 1e-3) / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat26", choices=["rmat26", "rmat22", "er65k"])
    ap.add_argument("--variant", default="zroot", choices=["zroot", "plain"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip every section after the headline and the other variant")
    ap.add_argument("--only", default=None,
                    choices=["small_configs", "reducer", "update_log", "csr", "u64_ids",
                             "share_rmat30", "batch", "batch_tail", "batch_tiny", "serve"],
                    help="run just this one further section (for profiling it)")
    ap.add_argument("--calibrate", action="store_true",
                    help="also run a plain 4 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the multi-GPU sharding is a design, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2507_03695_amd as cc
    cc.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    t0 = time.time()
    edges, n, cfg = make_workload(args.workload)
    m = len(edges)
    log(f"workload {cfg['workload']}: n={n} m={m} generated in {time.time() - t0:.1f} s")
    ed = torch.from_numpy(edges.view(np.int32)).cuda()
    torch.cuda.synchronize()

    if args.calibrate:
        # a plain copy of known size: 4 GiB read + 4 GiB written, for scaling the
        # FETCH_SIZE / WRITE_SIZE counters of the profiled kernels
        src = torch.ones(1 << 30, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()

    flags = cc.F_ZROOT if args.variant == "zroot" else 0
    ms, hook_ms, L = bench_single(cc, torch, ed, n, m, args.steps, args.warmup, flags)
    log(f"step {ms:.3f} ms, hook {hook_ms:.3f} ms")
    other = "plain" if args.variant == "zroot" else "zroot"
    ms_o, hook_o, L_o = bench_single(cc, torch, ed, n, m, max(3, args.steps // 2), 1,
                                     0 if flags else cc.F_ZROOT)
    assert torch.equal(L, L_o), "variants disagree"
    del L_o
    copy_gbs = copy_ceiling_gbs(torch)
    log(f"copy ceiling {copy_gbs:.0f} GB/s")
    def want(section):
        return not args.no_extras and args.only in (None, section)

    reducer = upd = csr = u64 = None
    if want("reducer"):
        t1 = time.time()
        reducer = bench_reducer(cc, torch, ed, n, L)
        log(f"reducer emulation done in {time.time() - t1:.1f} s")
    if want("update_log"):
        t1 = time.time()
        upd = bench_update_log(cc, torch, ed, n, L)
        log(f"update log done in {time.time() - t1:.1f} s")
    if want("csr"):
        t1 = time.time()
        csr = bench_csr(cc, torch, ed, n, L)
        log(f"csr done in {time.time() - t1:.1f} s")
    if want("u64_ids"):
        t1 = time.time()
        u64 = bench_u64(cc, torch, ed, n, L)
        log(f"u64 done in {time.time() - t1:.1f} s")

    alg_bytes = 8 * m + 12 * n
    gteps = m / (ms * 1e-3) / 1e9
    hook_gbs = 8 * m / (hook_ms * 1e-3) / 1e9
    line = {
        "metric": "GTEPS (COO entries per second, whole path: init+zroot+push+hook+compress+canon)",
        "value": round(gteps, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": dict(cfg, variant=args.variant, parallelism="single_gpu"),
        "hbm_roofline_frac_whole_path": round(alg_bytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
        "roofline": {"bound": "hbm", "achieved": round(hook_gbs, 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(hook_gbs / PEAK_HBM_GBS, 4),
                     "traffic": measured_traffic(args.workload, args.variant),
                     "kernel": HOOK_KERNELS[args.variant],
                     "algorithmic_bytes_per_launch": 8 * m, "avg_launch_ms": round(hook_ms, 4),
                     "measured_copy_GBps": round(copy_gbs, 1),
                     "frac_of_measured_copy": round(hook_gbs / copy_gbs, 4)},
        other: {"ms_per_step": round(ms_o, 4), "hook_ms": round(hook_o, 4),
                "GTEPS": round(m / (ms_o * 1e-3) / 1e9, 3)},
    }
    t = line["roofline"]["traffic"]
    if t is not None:
        # the rate at which the step moves its measured HBM bytes
        line["roofline"]["traffic_GBps"] = round(t / (hook_ms * 1e-3) / 1e9, 1)
    if reducer is not None:
        line["reducer"] = reducer
    if upd is not None:
        line["update_log"] = upd
    if csr is not None:
        line["csr"] = csr
    if u64 is not None:
        line["u64_ids"] = u64
    del ed, L
    torch.cuda.empty_cache()
    if want("small_configs"):
        t1 = time.time()
        line["small_configs"] = {w: bench_small(cc, torch, w) for w in ("er65k", "rmat22")}
        log(f"small configurations done in {time.time() - t1:.1f} s")
    if want("share_rmat30"):
        t1 = time.time()
        line["share_rmat30"] = bench_share30(cc, torch)
        log(f"share done in {time.time() - t1:.1f} s")
    if want("batch"):
        t1 = time.time()
        line["batch"] = bench_batch(cc, torch)
        log(f"batch done in {time.time() - t1:.1f} s")
    if want("batch_tail"):
        t1 = time.time()
        line["batch_tail"] = bench_batch_tail(cc, torch)
        log(f"batch with tail done in {time.time() - t1:.1f} s")
    if want("batch_tiny"):
        t1 = time.time()
        line["batch_tiny"] = bench_batch_tiny(cc, torch)
        log(f"batch of small graphs done in {time.time() - t1:.1f} s")
    if want("serve"):
        t1 = time.time()
        line["serve"] = bench_serve(cc, torch)
        log(f"serve done in {time.time() - t1:.1f} s")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(edges, n)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
