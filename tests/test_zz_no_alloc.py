"""The allocation-free entry point (cc_solve_noalloc) through the C ABI: its labels
and status equal those of cc_solve_async (the existing entry point whose kernels
it shares) and the oracle's, on two calls in a row, the second with a smaller
input (the fixed scratch keeps the first call's contents), for the plain and the
zero-root variants; sizes beyond its fixed scratch are refused at once."""
import numpy as np
import pytest
import torch

import graphgen
import oracle
from gpu_helpers import assert_same_labels, log, to_dev, to_host_u32

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_2507_03695_amd")


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = cc.Context()
    yield c
    c.close()


def _pair(ctx, e_np, n, flags):
    ed = to_dev(e_np)
    ref = ctx.solve(ed, n, flags=flags)
    L = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    cc.solve_noalloc(ed, n, L, flags=flags, status=st)
    torch.cuda.synchronize()
    return to_host_u32(L), to_host_u32(ref), int(st.item())


@pytest.mark.parametrize("flags", [0, 0x1, 0x1 | 0x8, 0x40])
def test_noalloc_equals_solve_async_twice(ctx, flags):
    big = (graphgen.rmat(22, 1 << 25, 11), 1 << 22)          # 2^25 entries, many tiles
    small = (graphgen.er(70_001, 150_003, 12), 70_001)        # ragged, smaller, second
    if flags & 0x40:
        big = (graphgen.rmat_sym(20, 1 << 22, 13), 1 << 20)
        small = (graphgen.rmat_sym(14, 40_000, 14), 1 << 14)
    for e, n in (big, small):
        log(f"noalloc flags={flags:#x} n={n} m={len(e)}")
        got, ref, st = _pair(ctx, e, n, flags)
        assert st == cc.CC_OK
        assert_same_labels(got, ref, f"noalloc vs cc_solve_async n={n}")
        assert_same_labels(got, oracle.cc_labels(n, e), f"noalloc vs oracle n={n}")


@pytest.mark.parametrize("flags", [0, 0x1])
def test_noalloc_two_part_hook(ctx, flags):
    """Small arrays with many entries per vertex, where the direct hook runs in
    two parts with a pointer-jumping (or, with a zero root, compress) pass between
    them on the fixed scratch: two calls in a row, the second smaller."""
    for e, n in ((graphgen.er(1 << 16, 1 << 20, 15), 1 << 16),
                 (graphgen.rmat(15, (1 << 18) + 33, 16), 1 << 15)):
        log(f"noalloc two-part flags={flags:#x} n={n} m={len(e)}")
        got, ref, st = _pair(ctx, e, n, flags)
        assert st == cc.CC_OK
        assert_same_labels(got, ref, f"noalloc two-part vs cc_solve_async n={n}")
        assert_same_labels(got, oracle.cc_labels(n, e), f"noalloc two-part vs oracle n={n}")


def test_noalloc_status_and_limits(ctx):
    n = 5000
    e = graphgen.er(n, 20_000, 21)
    e[777] = (n + 5, 1)
    ed = to_dev(e)
    L = torch.empty(n, dtype=torch.int32, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    cc.solve_noalloc(ed, n, L, flags=cc.F_ZROOT, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == cc.CC_ERANGE
    # the next call starts from a clear status word
    good = to_dev(graphgen.er(n, 20_000, 22))
    cc.solve_noalloc(good, n, L, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == cc.CC_OK
    lib = cc.load()
    # beyond the zero-root bitmap of the fixed scratch: refused, nothing enqueued
    too_big = 8 * (cc.NOALLOC_SCRATCH_BYTES - 557_312) + 64
    assert lib.cc_solve_noalloc(too_big, 0, None, L.data_ptr(), cc.F_ZROOT, 0, None,
                                None) == cc.CC_ENOMEM
    assert lib.cc_solve_noalloc(n, 0, None, L.data_ptr(), cc.F_ZROOT | cc.F_ZROOT_EXACT, 0, None,
                                None) == cc.CC_EINVAL
    assert lib.cc_solve_noalloc(1 << 32, 0, None, L.data_ptr(), 0, 0, None, None) == cc.CC_EINVAL
