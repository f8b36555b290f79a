"""Parity under injected delays, run in a child process whose CCMI_LIBRARY is the
race-testing build (libccmi_stress.so: every link CAS and path-splitting store
is preceded by a varying pause of its wave). Every solve, each on the entries
in a new seeded order, must give the oracle's labels; the direct hooks (with
path splitting above 4 MB of parent array, without it below; the zero-root
one linking under z below 256 MB, marking above), the regrouped
hooks, the 64-bit path and the batched launch (parent arrays in LDS and in HBM)
are all exercised. Exit status 0 when every
solve agrees. Started by tests/test_gpu_stress_delays.py; with --full it also
solves the bench's R-MAT-26 + extras workload (about a minute more)."""
import os
import sys

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import graphgen  # noqa: E402
import oracle  # noqa: E402
import paper_2507_03695_amd as cc  # noqa: E402


def main(full: bool = False) -> int:
    assert os.path.basename(cc.LIB_PATH) == "libccmi_stress.so", cc.LIB_PATH
    cc.load()
    cases = []
    if full:
        g = graphgen.rmat26_extras()
        cases.append(("rmat26_extras", g.n, g.edges, 1))
    cases += [
        ("er_2^14", 1 << 14, graphgen.er(1 << 14, 1 << 16, 301), 4),
        ("rmat_2^16", 1 << 16, graphgen.rmat(16, 1 << 20, 302), 3),   # small array: no splitting
        ("rmat_2^21", 1 << 21, graphgen.rmat(21, 1 << 22, 304), 2),   # direct hooks split
        ("rmat_2^22_2^24", 1 << 22, graphgen.rmat(22, 1 << 24, 303), 2),  # regrouped hooks
        # a 512 MB parent array: the direct zero-root hook only marks the other
        # endpoint of an entry with one marked endpoint
        ("rmat_2^27_2^22", 1 << 27, graphgen.rmat(27, 1 << 22, 309), 1),
    ]
    flagsets = {"plain": 0, "plain_nosplit": cc.F_NO_SPLIT, "plain_direct": cc.F_NO_TILE,
                "zroot": cc.F_ZROOT, "zroot_direct": cc.F_ZROOT | cc.F_NO_TILE}
    gen = torch.Generator(device="cuda")
    gen.manual_seed(304)
    with cc.Context() as c:
        for name, n, e, reps in cases:
            want = oracle.cc_labels(n, e)
            ed = torch.from_numpy(e.view(np.int32)).cuda()
            for fname, fl in flagsets.items():
                for rep in range(reps):
                    er = ed[torch.randperm(len(e), device="cuda", generator=gen)].contiguous()
                    got = c.solve(er, n, flags=fl).cpu().numpy().view(np.uint32)
                    if not np.array_equal(got, want):
                        bad = np.flatnonzero(got != want)
                        print(f"FAIL {name} {fname} rep {rep}: {len(bad)} labels differ, "
                              f"first v={bad[0]}", flush=True)
                        return 1
                print(f"ok {name} {fname} x{reps}", flush=True)
            if name == "er_2^14":
                e64 = torch.from_numpy(np.ascontiguousarray(e.astype(np.uint64)).view(np.int64)).cuda()
                for fl in (0, cc.F_NO_SPLIT):
                    got = c.solve_u64(e64, n, flags=fl).cpu().numpy().view(np.uint64)
                    if not np.array_equal(got, want.astype(np.uint64)):
                        print(f"FAIL {name} 64-bit flags {fl}", flush=True)
                        return 1
                print(f"ok {name} 64-bit", flush=True)
        # many graphs in one launch: parent arrays in LDS (16-bit entries) and,
        # above the LDS capacity, in HBM
        graphs = [(graphgen.rmat(17, 1 << 19, 305 + i) % (90_000 + i), 90_000 + i) for i in range(2)]
        graphs += [(graphgen.er(1 << 16, 1 << 18, 307), 1 << 16)]
        graphs += [(graphgen.rmat(12, 1 << 15, 308 + i), 1 << 12) for i in range(200)]
        b = graphgen.batch_from_graphs(graphs)
        want, _ = oracle.cc_labels_batch(b.vtx_off, b.edge_off, b.edges)
        vo = torch.from_numpy(b.vtx_off).cuda()
        eo = torch.from_numpy(b.edge_off).cuda()
        eb = torch.from_numpy(np.ascontiguousarray(b.edges)).cuda()
        for rep in range(3):
            L, st = c.batch(vo, eo, eb)
            if not (np.all(st.cpu().numpy() == 0) and
                    np.array_equal(L.cpu().numpy().view(np.uint32), want.view(np.uint32))):
                print(f"FAIL batch rep {rep}", flush=True)
                return 1
        print("ok batch x3", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main(full="--full" in sys.argv[1:]))
