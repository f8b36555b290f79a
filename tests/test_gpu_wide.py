"""64-bit vertex IDs on the GPU (cc_solve_u64): labels against the oracle below
2^32, and a graph whose IDs straddle 2^32 with n = 2^32 + 2^20 (a 34 GB parent
array) checked on every vertex: the touched ones against the oracle's sparse
labels, the rest equal to themselves."""
import numpy as np
import pytest
import torch

import graphgen
import oracle
from gpu_helpers import assert_same_labels, log, rmat26_extras_with_labels

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_2507_03695_amd")


def dev64(e):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(e, np.uint64).reshape(-1, 2))
                            .view(np.int64)).cuda()


@pytest.mark.parametrize("flags", [0, 0x8])
def test_wide_matches_the_oracle_below_2_32(flags):
    with cc.Context() as c:
        for name, n, e in [("er", 1 << 16, graphgen.er(1 << 16, 1 << 18, 111)),
                           ("rmat", 1 << 16, graphgen.rmat(16, 1 << 20, 112)),
                           ("ragged", 3001, graphgen.er(3001, 7777, 113))]:
            L = c.solve_u64(dev64(e), n, flags=flags)
            got = L.cpu().numpy().view(np.uint64)
            want = oracle.cc_labels(n, e).astype(np.uint64)
            assert_same_labels(got, want, f"{name} flags {flags}")


def test_wide_ids_across_2_32():
    n = (1 << 32) + (1 << 20)
    rng = np.random.default_rng(114)
    e = graphgen.rmat(16, 1 << 19, 115).astype(np.uint64)
    ids = np.sort(rng.choice(np.arange((1 << 32) - (1 << 19), n, dtype=np.uint64), 1 << 16,
                             replace=False))
    e = ids[e]                                      # R-MAT's structure on IDs across 2^32
    e = np.concatenate([e, np.array([[5, ids[7]], [ids[-1], 1 << 31]], np.uint64)])
    uid, lab = oracle.cc_labels_sparse64(e)
    log(f"{len(uid)} touched IDs, {int((lab != uid).sum())} non-minimal")
    with cc.Context() as c:
        L = torch.empty(n, dtype=torch.int64, device="cuda")
        c.solve_u64_async(dev64(e), n, L)
        assert c.sync() == cc.CC_OK
        got = L[torch.from_numpy(uid.view(np.int64)).cuda()].cpu().numpy().view(np.uint64)
        assert_same_labels(got, lab, "touched IDs")
        differ = 0
        step = 1 << 28
        for a in range(0, n, step):
            b = min(n, a + step)
            differ += int((L[a:b] != torch.arange(a, b, device="cuda", dtype=torch.int64)).sum())
        assert differ == int((lab != uid).sum()), "an untouched vertex is not its own label"
        del L
        torch.cuda.empty_cache()


def test_wide_edges_and_errors():
    with cc.Context() as c:
        L = c.solve_u64(dev64(np.zeros((0, 2))), 10)
        assert L.cpu().tolist() == list(range(10))
        e = dev64([[1, 2], [3, 12]])
        L = torch.empty(10, dtype=torch.int64, device="cuda")
        c.solve_u64_async(e, 10, L)
        assert c.sync() == cc.CC_ERANGE
        with pytest.raises(cc.CCError) as ei:
            c.solve_u64_async(e, 10, L, flags=cc.F_ZROOT)
        assert ei.value.code == cc.CC_EINVAL


def test_wide_rmat26_extras_full():
    """The bench's R-MAT-26 + extras workload with every ID widened to 64 bits."""
    g, want = rmat26_extras_with_labels()
    e64 = torch.from_numpy(g.edges.view(np.int32)).cuda().to(torch.int64) & 0xFFFFFFFF
    with cc.Context() as c:
        L = c.solve_u64(e64, g.n)
        got = L.cpu().numpy().view(np.uint64)
    assert_same_labels(got, want.astype(np.uint64), "u64 rmat26")

