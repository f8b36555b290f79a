"""SiskinCC's update log on the GPU (Sec. III, Algorithm 2): cc_hook_log appends
(linked root, new parent) at every successful link.

The order of the messages depends on the schedule, so what is compared exactly
is what is unique: the set of linked vertices (every vertex but its component's
lowest ID, once each, since non-roots are never linked) and the labels that the
messages give when taken as edges. Both are checked against the oracle, and the
count against the oracle's sequential Algorithm 2."""
import numpy as np
import pytest
import torch

import graphgen
import oracle
from gpu_helpers import assert_same_labels, log, rmat26_extras_with_labels, to_dev, to_host_u32

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_2507_03695_amd")


def check_log(n, msgs, want, what):
    """msgs: (k, 2) uint32 host array of messages; want: oracle labels."""
    v = np.arange(n)
    kids = np.sort(msgs[:, 0])
    assert np.array_equal(kids, v[want != v]), f"{what}: linked vertices differ"
    assert np.all(msgs[:, 1] < msgs[:, 0]), f"{what}: a parent has the greater ID"
    assert np.array_equal(want[msgs[:, 0]], want[msgs[:, 1]]), f"{what}: a message crosses components"
    assert_same_labels(oracle.cc_labels(n, msgs), want, f"{what}: messages as edges")


def run_log(c, ed, n, chunks=1, flags=0, cap=None):
    P = torch.empty(n, dtype=torch.int32, device="cuda")
    cap = n if cap is None else cap
    L = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    c.init(n, P)
    for part in torch.tensor_split(ed, chunks):
        c.hook_log(part, n, P, L, cnt, flags=flags)
    return P, L, cnt


@pytest.mark.parametrize("split", [True, False])
@pytest.mark.parametrize("kind", ["rmat", "er"])
def test_log_is_the_set_of_links(kind, split):
    n = 1 << 16
    e = graphgen.rmat(16, 1 << 20, 81) if kind == "rmat" else graphgen.er(n, 1 << 17, 82)
    want = oracle.cc_labels(n, e)
    seq = oracle.siskin_log(n, e)
    flags = 0 if split else cc.F_NO_SPLIT
    with cc.Context() as c:
        P, L, cnt = run_log(c, to_dev(e), n, flags=flags)
        c.compress(n, P)
        assert c.sync() == cc.CC_OK
        k = int(cnt.item())
        log(f"{kind}: {k} messages, sequential Algorithm 2: {len(seq)}")
        assert k == len(seq) == n - oracle.count_components(want)
        msgs = L[:k].cpu().numpy().view(np.uint32)
        check_log(n, msgs, want, kind)
        assert np.array_equal(np.sort(msgs[:, 0]), np.sort(seq[:, 0]))
        assert_same_labels(to_host_u32(P), want, f"{kind}: labels after the logged hook")


def test_log_appends_across_calls_and_tails():
    n = 3001                                       # ragged against every block size
    e = graphgen.er(n, 2 * n + 77, 83)
    want = oracle.cc_labels(n, e)
    with cc.Context() as c:
        P, L, cnt = run_log(c, to_dev(e), n, chunks=7)
        assert c.sync() == cc.CC_OK
        k = int(cnt.item())
        assert k == n - oracle.count_components(want)
        check_log(n, L[:k].cpu().numpy().view(np.uint32), want, "7 calls")


def test_log_capacity_and_arguments():
    n = 1 << 12
    e = graphgen.er(n, 4 * n, 84)
    want = oracle.cc_labels(n, e)
    total = n - oracle.count_components(want)
    with cc.Context() as c:
        ed = to_dev(e)
        P, L, cnt = run_log(c, ed, n, cap=100)
        assert c.sync() == cc.CC_ENOMEM
        assert int(cnt.item()) == total            # counted past the capacity
        kept = L[:100].cpu().numpy().view(np.uint32)
        assert len(np.unique(kept[:, 0])) == 100 and np.all(kept[:, 1] < kept[:, 0])
        assert np.array_equal(want[kept[:, 0]], want[kept[:, 1]])
        assert c.sync() == cc.CC_OK                # the status word was cleared
        with pytest.raises(cc.CCError) as ei:
            c.hook_log(ed, n, P, L, cnt, flags=cc.F_ZROOT)
        assert ei.value.code == cc.CC_EINVAL
        cnt.zero_()
        c.init(n, P)
        c.hook_log(ed[:0], n, P, L, cnt)
        assert c.sync() == cc.CC_OK and int(cnt.item()) == 0
        bad = torch.tensor([[1, 2], [3, n + 5]], dtype=torch.int32, device="cuda")
        c.hook_log(bad, n, P, L, cnt)
        assert c.sync() == cc.CC_ERANGE
        assert int(cnt.item()) == 1                # (2, 1); the bad entry is skipped


@pytest.mark.parametrize("chunks", [1, 7, 64])
def test_log_drained_while_hooking(chunks):
    """cc_hook_log_drain: the log copied to pinned host memory launch by launch.
    The host copy holds exactly the links (each vertex but its component's lowest
    ID once; the messages as edges give the oracle's labels), as many as the
    sequential Algorithm 2 sends, and P is left hooked as by cc_hook_log."""
    n = 1 << 20
    e = graphgen.rmat(20, (1 << 22) + 333, 86)               # ragged against the chunks
    want = oracle.cc_labels(n, e)
    ed = to_dev(e)
    with cc.Context() as c:
        P = torch.empty(n, dtype=torch.int32, device="cuda")
        dev_log = torch.empty((n, 2), dtype=torch.int32, device="cuda")
        host = torch.empty((n, 2), dtype=torch.int32, pin_memory=True)
        c.init(n, P)
        k = c.hook_log_drain(ed, n, P, dev_log, host, chunks=chunks)
        assert k == n - oracle.count_components(want)
        check_log(n, host[:k].numpy().view(np.uint32), want, f"drained, {chunks} launches")
        c.compress(n, P)
        assert c.sync() == cc.CC_OK
        assert_same_labels(to_host_u32(P), want, "labels after the drained hook")
        # a pageable host buffer works too; a second call counts from 0 again
        host2 = torch.empty((n, 2), dtype=torch.int32)
        c.init(n, P)
        k2 = c.hook_log_drain(ed, n, P, dev_log, host2, chunks=chunks)
        assert k2 == k
        check_log(n, host2[:k2].numpy().view(np.uint32), want, "pageable host buffer")


def test_log_drain_capacity_and_arguments():
    n = 1 << 12
    e = graphgen.er(n, 4 * n, 87)
    want = oracle.cc_labels(n, e)
    total = n - oracle.count_components(want)
    ed = to_dev(e)
    with cc.Context() as c:
        P = torch.empty(n, dtype=torch.int32, device="cuda")
        dev_log = torch.empty((n, 2), dtype=torch.int32, device="cuda")
        small = torch.empty((100, 2), dtype=torch.int32, pin_memory=True)
        c.init(n, P)
        with pytest.raises(cc.CCError) as ei:                 # host room for 100 only
            c.hook_log_drain(ed, n, P, dev_log, small, chunks=5)
        assert ei.value.code == cc.CC_ENOMEM
        kept = small.numpy().view(np.uint32)
        assert len(np.unique(kept[:, 0])) == 100 and np.array_equal(want[kept[:, 0]], want[kept[:, 1]])
        assert total > 100
        host = torch.empty((n, 2), dtype=torch.int32, pin_memory=True)
        for bad_chunks in (0, cc.DRAIN_MAX_CHUNKS + 1):
            with pytest.raises(cc.CCError) as ei:
                c.hook_log_drain(ed, n, P, dev_log, host, chunks=bad_chunks)
            assert ei.value.code == cc.CC_EINVAL
        with pytest.raises(cc.CCError) as ei:
            c.hook_log_drain(ed, n, P, dev_log, host, flags=cc.F_ZROOT)
        assert ei.value.code == cc.CC_EINVAL
        c.init(n, P)
        assert c.hook_log_drain(ed[:0], n, P, dev_log, host, chunks=3) == 0
        assert c.sync() == cc.CC_OK


def test_siskin_reducer_16_shares():
    """Each of 16 edge shares hooks into its own P with a log and sends nothing
    else; the Reducer hooks all messages as edges and compresses (Sec. III)."""
    n, g = 1 << 20, 16
    e = graphgen.rmat(20, 1 << 24, 85)
    want = oracle.cc_labels(n, e)
    log("oracle done")
    k = (e[:, 0].astype(np.uint64) * g) // n
    with cc.Context() as c:
        logs, sent = [], 0
        for s in range(g):
            es = np.ascontiguousarray(e[k == s])
            P, L, cnt = run_log(c, to_dev(es), n)
            assert c.sync() == cc.CC_OK
            ks = int(cnt.item())
            assert ks == n - oracle.count_components(oracle.cc_labels(n, es))
            logs.append(L[:ks])
            sent += ks
        assert sent <= min(len(e), g * n)          # Sec. V volume bound
        log(f"messages {sent}, bound {min(len(e), g * n)}")
        R = torch.empty(n, dtype=torch.int32, device="cuda")
        c.init(n, R)
        c.hook(torch.cat(logs), n, R)
        c.compress(n, R)
        assert c.sync() == cc.CC_OK
        assert_same_labels(to_host_u32(R), want, "Reducer over the update logs")


def test_log_rmat26_extras_full():
    """The bench's workload: the linked vertices are exactly the oracle's
    non-minimal vertices (compared as sorted lists on the device), and a Reducer
    over 16 shares' logs, hooked in their given order, gives the oracle's labels."""
    g, want = rmat26_extras_with_labels()
    n = g.n
    ed = to_dev(g.edges)
    wd = torch.from_numpy(want.view(np.int32)).cuda()
    nonmin = torch.nonzero(wd != torch.arange(n, device="cuda", dtype=torch.int32)).flatten()
    with cc.Context() as c:
        P, L, cnt = run_log(c, ed, n)
        assert c.sync() == cc.CC_OK
        k = int(cnt.item())
        assert k == nonmin.numel()
        kids = torch.sort(L[:k, 0].to(torch.int64) & 0xFFFFFFFF).values
        assert torch.equal(kids, nonmin.to(torch.int64))
        del P, L
        g16 = 16
        u = ed[:, 0].to(torch.int64) & 0xFFFFFFFF
        share = (u * g16) // n
        recv = torch.empty((ed.shape[0], 2), dtype=torch.int32, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        P = torch.empty(n, dtype=torch.int32, device="cuda")
        for s in range(g16):
            c.init(n, P)
            c.hook_log(ed[share == s].contiguous(), n, P, recv, cnt)
        assert c.sync() == cc.CC_OK
        sent = int(cnt.item())
        log(f"siskin messages at full size: {sent}")
        c.init(n, P)
        c.hook(recv[:sent], n, P, flags=cc.F_NO_TILE)
        c.compress(n, P)
        assert c.sync() == cc.CC_OK
        assert_same_labels(to_host_u32(P), want, "SiskinCC Reducer, rmat26")

