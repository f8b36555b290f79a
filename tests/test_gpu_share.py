"""One machine's share at real shape (Sec. IV: a machine owns a contiguous block
of vertices; Sec. V: each machine keeps a global-size parent array): the
entries of a permuted R-MAT graph whose first endpoint lies in the first of 16
equal vertex ranges, solved with the global n.

Also checks that the generators' GPU twin produces exactly the CPU generator's
entries, since the full-size share is generated on the GPU."""
import os

import numpy as np
import pytest
import torch

import graphgen
import oracle
from gpu_helpers import (assert_same_labels, check_properties_on_device, golden_share30, log,
                         sha256_of, to_dev, to_host_u32)

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_2507_03695_amd")


def test_device_generator_matches_cpu():
    for scale, m, perm in [(12, 5000, True), (20, 1 << 22, True), (20, 1 << 20, False)]:
        cpu = graphgen.rmat(scale, m, 99, permute=perm)
        dev = graphgen.rmat_dev(scale, m, 99, permute=perm)
        assert np.array_equal(dev.cpu().numpy().view(np.uint32), cpu), f"rmat {scale}"
    for scale, k in [(16, 0), (22, 5)]:
        cpu, n = graphgen.rmat_share(scale, 16, 7, 16, k)
        dev, n2 = graphgen.rmat_share_dev(scale, 16, 7, 16, k, span=1 << 16)
        assert n == n2
        assert np.array_equal(dev.cpu().numpy().view(np.uint32), cpu), f"share {scale}/{k}"


def test_share_rmat26_parity():
    """The same share recipe at scale 26 (n = 2^26 global), bit-exact vs the oracle."""
    e, n = graphgen.rmat_share(26, 16, graphgen.config_seed(5), 16, 0)
    log(f"share26 generated: m={len(e)}")
    want = oracle.cc_labels(n, e)
    ed = to_dev(e)
    with cc.Context() as c:
        for fl in (0, cc.F_ZROOT):
            L = c.solve(ed, n, flags=fl)
            assert_same_labels(to_host_u32(L), want, f"share26 flags={fl}")


def test_share_rmat30_full_oracle_digest():
    """Full size: n = 2^30 (a 4 GiB parent array), about 2^30 entries. The device
    generator's entries are the CPU generator's (digest), and the labels of both
    paths equal the oracle's bit for bit (SHA-256 of all 2^30 labels, the
    component count and probe vertices recorded by the oracle-only script)."""
    free, _ = torch.cuda.mem_get_info()
    assert free > 20 << 30, "needs ~16 GiB of free device memory"
    g = golden_share30()
    ed, n = graphgen.rmat30_share_dev()
    log(f"share30 generated on device: m={ed.shape[0]}")
    assert n == int(g["n"]) and ed.shape[0] == int(g["m"])
    assert sha256_of(ed) == g["entries_sha256"], "device entries differ from the CPU generator's"
    with cc.Context() as c:
        for fl in (cc.F_ZROOT, 0):
            L = c.solve(ed, n, flags=fl)
            torch.cuda.synchronize()
            log(f"share30 solved, flags={fl}")
            assert sha256_of(L) == g["labels_sha256"], f"share30 labels differ (flags={fl})"
            ar = torch.arange(n, device="cuda", dtype=torch.int64)
            L64 = L.to(torch.int64) & 0xFFFFFFFF
            assert int((L64 == ar).sum().item()) == int(g["components"])
            for v, want in g["label"].items():
                assert int(L64[v].item()) == want, f"label of {v}"
            del L, L64, ar
        check_properties_on_device(ed, c.solve(ed, n, flags=cc.F_ZROOT), n)
