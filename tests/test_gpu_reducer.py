"""Reducer emulation on one GPU (Sec. III high-level algorithm; Sec. IV
zero-converged vertices sent as IDs; Sec. V volume bound).

g edge shares (entries whose first endpoint lies in one of g equal vertex
ranges) are each solved into their own global-size parent array; cc_export
turns each array into (v, P_v) pairs and zero-converged IDs; a Reducer hooks
all of them (cc_hook over the pairs, cc_hook_ids for the IDs) and compresses.
The export of a share is unique once the share is compressed, so it is
compared exactly with the oracle's labels of that share; the Reducer's labels
are compared with the oracle's labels of the whole graph."""
import numpy as np
import pytest
import torch

import graphgen
import oracle
from gpu_helpers import assert_same_labels, log, rmat26_extras_with_labels, to_dev, to_host_u32

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_2507_03695_amd")

NONE = 0xFFFFFFFF


def shares(e: np.ndarray, n: int, g: int):
    k = (e[:, 0].astype(np.uint64) * g) // n
    return [np.ascontiguousarray(e[k == s]) for s in range(g)]


def expected_export(labels: np.ndarray, z: int):
    """Pairs (v, L_v) for L_v not in {v, z}, and the v != z with L_v == z, in
    increasing v. With z = NONE every non-root is a pair."""
    v = np.arange(len(labels), dtype=np.int64)
    lab = labels.astype(np.int64)
    nonroot = lab != v
    zero = nonroot & (lab == z)
    pair = nonroot & (lab != z)
    pairs = np.stack([v[pair], lab[pair]], axis=1).astype(np.uint32)
    return pairs, v[zero].astype(np.uint32)


def solve_share(c, ed, n, P, z=None):
    """Steps up to compress (no canon): P_v is v's root, z for z's component."""
    c.init(n, P)
    if z is None:
        c.hook(ed, n, P)
        c.compress(n, P)
    else:
        c.zroot(ed, n, flags=cc.F_ZROOT | cc.F_ZROOT_HINT, zroot_hint=z)
        c.push(ed, n, P)
        c.hook(ed, n, P, flags=cc.F_ZROOT)
        c.compress(n, P, flags=cc.F_ZROOT)
    assert c.sync() == cc.CC_OK


@pytest.mark.parametrize("use_z", [False, True])
def test_export_matches_the_share_labels(use_z):
    n, g = 1 << 16, 4
    e = graphgen.rmat(16, 1 << 20, 71)
    z = oracle.zroot(n, e, 1 << 16) if use_z else None
    with cc.Context() as c:
        P = torch.empty(n, dtype=torch.int32, device="cuda")
        for s, es in enumerate(shares(e, n, g)):
            solve_share(c, to_dev(es), n, P, z)
            want = oracle.cc_labels(n, es).astype(np.int64)
            if z is not None:
                want[want == want[z]] = z          # z's component carries z before canon
            wp, wz = expected_export(want, NONE if z is None else z)
            pairs, zero = c.export_lists(P, n, NONE if z is None else z)
            gp = pairs.cpu().numpy().view(np.uint32)
            gz = zero.cpu().numpy().view(np.uint32)
            assert np.array_equal(gp, wp), f"share {s}: pairs differ"
            assert np.array_equal(gz, wz), f"share {s}: zero IDs differ"


def test_export_capacity_and_empty_cases():
    n = 1000
    with cc.Context() as c:
        P = torch.arange(n, dtype=torch.int32, device="cuda")       # all roots
        assert c.export(P, n) == (0, 0)
        P[5] = 3
        P[7] = 3
        P[9] = 0
        assert c.export(P, n, zroot=0) == (2, 1)
        small = torch.empty((1, 2), dtype=torch.int32, device="cuda")
        with pytest.raises(cc.CCError) as ei:
            c.export(P, n, 0, small, torch.empty(1, dtype=torch.int32, device="cuda"))
        assert ei.value.code == cc.CC_ENOMEM
        pairs, zero = c.export_lists(P, n, zroot=0)
        assert pairs.cpu().tolist() == [[5, 3], [7, 3]]
        assert zero.cpu().tolist() == [9]


@pytest.mark.parametrize("use_z", [False, True])
def test_reducer_emulation_16_shares(use_z):
    n, g = 1 << 20, 16
    e = graphgen.rmat(20, 1 << 24, 72)
    want = oracle.cc_labels(n, e)
    log("oracle done")
    with cc.Context() as c:
        z = None
        if use_z:
            Pz = torch.empty(n, dtype=torch.int32, device="cuda")
            c.init(n, Pz)
            c.zroot(to_dev(e), n)                 # the global max-degree choice
            z = c.get_zroot()
        zr = NONE if z is None else z
        all_pairs, all_zero = [], []
        for es in shares(e, n, g):
            P = torch.empty(n, dtype=torch.int32, device="cuda")
            solve_share(c, to_dev(es), n, P, z)
            p, q = c.export_lists(P, n, zr)
            all_pairs.append(p)
            all_zero.append(q)
        pairs = torch.cat(all_pairs)
        zero = torch.cat(all_zero)
        sent = pairs.shape[0] + zero.shape[0]
        log(f"pairs {pairs.shape[0]}, zero IDs {zero.shape[0]}, bound {min(len(e), g * n)}")
        assert sent <= min(len(e), g * n)         # Sec. V: at most min(|E|, g|V|) messages
        L = torch.empty(n, dtype=torch.int32, device="cuda")
        c.init(n, L)
        if z is None:
            c.hook(pairs, n, L)
            c.compress(n, L)
        else:
            c.zroot(pairs, n, flags=cc.F_ZROOT | cc.F_ZROOT_HINT, zroot_hint=z)
            c.hook(pairs, n, L, flags=cc.F_ZROOT)
            c.hook_ids(zero, z, n, L, flags=cc.F_ZROOT)
            c.compress(n, L, flags=cc.F_ZROOT)
            c.canon(n, L)
        assert c.sync() == cc.CC_OK
        assert_same_labels(to_host_u32(L), want, f"reducer (z={z})")


def test_hook_ids_plain_and_out_of_range():
    n = 5000
    ids = torch.tensor([10, 20, 30, 4999, 20], dtype=torch.int32, device="cuda")
    with cc.Context() as c:
        L = torch.empty(n, dtype=torch.int32, device="cuda")
        c.init(n, L)
        c.hook_ids(ids, 7, n, L)
        c.compress(n, L)
        assert c.sync() == cc.CC_OK
        want = np.arange(n)
        want[[7, 10, 20, 30, 4999]] = 7
        assert np.array_equal(L.cpu().numpy(), want)
        bad = torch.tensor([1, n + 3], dtype=torch.int32, device="cuda")
        c.init(n, L)
        c.hook_ids(bad, 0, n, L)
        assert c.sync() == cc.CC_ERANGE


def test_reducer_rmat26_extras_full():
    """RobinCC's exchange at the bench's size: 16 shares solved with the global zero
    root, exported, sent through 4-byte compact IDs, merged by a Reducer; the
    labels equal the oracle's."""
    g, want = rmat26_extras_with_labels()
    n = g.n
    ed = to_dev(g.edges)
    u = ed[:, 0].to(torch.int64) & 0xFFFFFFFF
    share = (u * 16) // n
    with cc.Context() as c:
        Pz = torch.empty(n, dtype=torch.int32, device="cuda")
        c.init(n, Pz)
        c.zroot(ed, n)
        z = c.get_zroot()
        k = c.id_bytes(n)
        pairs_all, zero_all = [], []
        for s in range(16):
            es = ed[share == s].contiguous()
            solve_share(c, es, n, Pz, z)
            p, q = c.export_lists(Pz, n, z)
            pairs_all.append(c.unpack_ids(c.pack_ids(p, k), p.numel(), k).view(-1, 2))
            zero_all.append(c.unpack_ids(c.pack_ids(q, k), q.numel(), k))
        pairs = torch.cat(pairs_all)
        zero = torch.cat(zero_all)
        log(f"pairs {pairs.shape[0]}, zero IDs {zero.shape[0]}")
        L = torch.empty(n, dtype=torch.int32, device="cuda")
        c.init(n, L)
        c.zroot(pairs, n, flags=cc.F_ZROOT | cc.F_ZROOT_HINT, zroot_hint=z)
        c.hook(pairs, n, L, flags=cc.F_ZROOT)
        c.hook_ids(zero, z, n, L, flags=cc.F_ZROOT)
        c.compress(n, L, flags=cc.F_ZROOT)
        c.canon(n, L)
        assert c.sync() == cc.CC_OK
        assert_same_labels(to_host_u32(L), want, "RobinCC Reducer, rmat26")

