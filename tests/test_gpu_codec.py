"""Compact vertex IDs of the exchange on the GPU (Sec. V): cc_pack_ids /
cc_unpack_ids against the oracle's byte-exact encoding, and a Reducer fed
through the codec."""
import numpy as np
import pytest
import torch

import graphgen
import oracle
from gpu_helpers import assert_same_labels, log, to_dev, to_host_u32

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_2507_03695_amd")

COUNTS = [1, 2, 3, 5, 7, 8, 1000, 4097, 100003]


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_pack_is_byte_exact_and_round_trips(k):
    rng = np.random.default_rng(90 + k)
    with cc.Context() as c:
        for count in COUNTS:
            ids = rng.integers(0, 256 ** k, size=count, dtype=np.uint64).astype(np.uint32)
            ids[0] = 256 ** k - 1                      # the widest ID of this width
            dev = torch.from_numpy(ids.view(np.int32)).cuda()
            buf = c.pack_ids(dev, k)
            back = c.unpack_ids(buf, count, k)
            assert c.sync() == cc.CC_OK
            want = oracle.pack_ids(ids, k)
            got = buf.cpu().numpy()
            assert np.array_equal(got, want), f"k={k} count={count}: bytes differ"
            assert np.array_equal(to_host_u32(back), ids), f"k={k} count={count}: round trip"


def test_codec_edges_and_errors():
    with cc.Context() as c:
        assert [c.id_bytes(n) for n in (0, 1, 256, 257, 1 << 24, (1 << 24) + 1, 1 << 32)] == \
            [1, 1, 1, 2, 3, 4, 4]
        ids = torch.tensor([1, 70000, 3], dtype=torch.int32, device="cuda")
        buf = c.pack_ids(ids, 2)
        assert c.sync() == cc.CC_ERANGE                # 70000 needs 3 bytes
        assert buf.cpu().tolist() == [1, 0, 70000 & 0xFF, (70000 >> 8) & 0xFF, 3, 0]
        big = torch.empty(64, dtype=torch.uint8, device="cuda")
        with pytest.raises(cc.CCError) as ei:
            c.pack_ids(ids, 2, out=big[1:])            # not 4-byte aligned
        assert ei.value.code == cc.CC_EINVAL
        with pytest.raises(cc.CCError) as ei:
            c.pack_ids(ids, 5, out=big)
        assert ei.value.code == cc.CC_EINVAL
        empty = c.pack_ids(ids[:0], 3)
        assert empty.numel() == 0 and c.unpack_ids(empty, 0, 3).numel() == 0
        assert c.sync() == cc.CC_OK


def test_reducer_through_the_codec():
    """16 shares exported, every message packed in cc_id_bytes(n) = 3 bytes per
    ID, unpacked on the Reducer side, hooked and compressed."""
    n, g = 1 << 20, 16
    e = graphgen.rmat(20, 1 << 24, 91)
    want = oracle.cc_labels(n, e)
    shares = (e[:, 0].astype(np.uint64) * g) // n
    with cc.Context() as c:
        k = c.id_bytes(n)
        assert k == 3
        wire = []
        for s in range(g):
            es = np.ascontiguousarray(e[shares == s])
            P = torch.empty(n, dtype=torch.int32, device="cuda")
            c.init(n, P)
            c.hook(to_dev(es), n, P)
            c.compress(n, P)
            pairs, _ = c.export_lists(P, n)
            wire.append((pairs.shape[0], c.pack_ids(pairs, k)))
        assert c.sync() == cc.CC_OK
        nbytes = sum(b.numel() for _, b in wire)
        npairs = sum(p for p, _ in wire)
        assert nbytes == npairs * 2 * k
        log(f"{npairs} pairs in {nbytes} bytes")
        got = torch.cat([c.unpack_ids(b, 2 * p, k).view(-1, 2) for p, b in wire])
        R = torch.empty(n, dtype=torch.int32, device="cuda")
        c.init(n, R)
        c.hook(got, n, R)
        c.compress(n, R)
        assert c.sync() == cc.CC_OK
        assert_same_labels(to_host_u32(R), want, "Reducer through the codec")
