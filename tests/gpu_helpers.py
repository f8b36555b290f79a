"""Helpers shared by the GPU tests: moving seeded inputs to the device and
checking labels against the oracle and against properties that hold at any size."""
import functools
import hashlib
import os
import sys

import numpy as np
import torch


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(edges: np.ndarray) -> torch.Tensor:
    """(m, 2) uint32 numpy -> (m, 2) int32 device tensor with the same bits."""
    e = np.ascontiguousarray(edges.reshape(-1, 2))
    if e.dtype == np.uint32:
        e = e.view(np.int32)
    return torch.from_numpy(e).cuda()


def to_host_u32(L: torch.Tensor) -> np.ndarray:
    return L.cpu().numpy().view(np.uint32)


def assert_same_labels(got: np.ndarray, want: np.ndarray, what: str):
    if not np.array_equal(got, want):
        bad = np.flatnonzero(got != want)
        raise AssertionError(f"{what}: {len(bad)} labels differ; first at v={bad[0]}: "
                             f"got {got[bad[0]]}, want {want[bad[0]]}")


def check_properties_on_device(edges_dev: torch.Tensor, L_dev: torch.Tensor, n: int):
    """Every entry's endpoints share a label, L_v <= v, L_{L_v} = L_v (device-side)."""
    L = L_dev.to(torch.int64) & 0xFFFFFFFF
    E = edges_dev.to(torch.int64) & 0xFFFFFFFF
    step = 1 << 26
    for a in range(0, E.shape[0], step):
        blk = E[a:a + step]
        assert torch.equal(L[blk[:, 0]], L[blk[:, 1]]), "an entry's endpoints differ in label"
    ar = torch.arange(n, device=L.device, dtype=torch.int64)
    assert bool((L <= ar).all()), "a label exceeds its vertex"
    assert torch.equal(L[L], L), "a label is not a fixed point"


def golden_share30():
    """tests/golden/share30_oracle.txt (written by make_share30_digest.py from the
    generators and the oracle only): entry count, digests, components, probes."""
    out = {"label": {}}
    with open(os.path.join(os.path.dirname(__file__), "golden", "share30_oracle.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *v = line.split()
            if k == "label":
                out["label"][int(v[0])] = int(v[1])
            else:
                out[k] = v[0]
    return out


def sha256_of(a) -> str:
    """SHA-256 of an array's bytes (a device tensor is copied to the host first)."""
    if isinstance(a, torch.Tensor):
        a = a.cpu().numpy()
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@functools.lru_cache(maxsize=1)
def rmat26_extras_with_labels():
    """The R-MAT-26 + extras workload (the bench's) and the oracle's labels of it,
    computed once per test process and shared by the full-size tests."""
    import graphgen
    import oracle
    g = graphgen.rmat26_extras()
    log(f"rmat26 generated: n={g.n} m={len(g.edges)}")
    want = oracle.cc_labels(g.n, g.edges)
    log("rmat26 oracle done")
    return g, want

