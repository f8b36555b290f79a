"""Write share30_oracle.txt: the oracle's labels of one machine's share of
R-MAT-30, recorded as digests so that a GPU test can compare full-size labels
bit for bit without running the oracle (minutes of CPU time at n = 2^30).

The share (Sec. IV: a machine owns a contiguous block of vertices; Sec. V: its
parent array stays global-size) is share 0 of 16 of a permuted R-MAT graph of
scale 30, edgefactor 16: the generated entries whose first endpoint lies in
[0, 2^26), n = 2^30. This script calls only the seeded generators (graphgen)
and the oracle; nothing here touches the GPU library.

Recorded: the entry count and the SHA-256 of the entries (so that the GPU
test can check that the device generator produced the same input), the
SHA-256 of the oracle's labels (uint32, little-endian, vertex order), the
component count, and the labels of a few fixed vertices.

Run: python tests/golden/make_share30_digest.py   (about 25 GB of host memory)
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import graphgen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "share30_oracle.txt")
PROBES = [0, 1, 2, 3, (1 << 26) - 1, 1 << 26, (1 << 26) + 1, 123_456_789, (1 << 30) - 1]


def main():
    t0 = time.time()
    e, n = graphgen.rmat30_share()
    print(f"generated m={len(e)} in {time.time() - t0:.0f} s", flush=True)
    e_sha = hashlib.sha256(np.ascontiguousarray(e).tobytes()).hexdigest()
    t1 = time.time()
    L = oracle.cc_labels(n, e)
    print(f"oracle labels in {time.time() - t1:.0f} s", flush=True)
    l_sha = hashlib.sha256(L.tobytes()).hexdigest()
    comps = oracle.count_components(L)
    lines = [
        "# oracle labels of share 0 of 16 of R-MAT scale 30, edgefactor 16, permuted",
        f"# (seed {graphgen.config_seed(5):#x}); written by make_share30_digest.py,",
        "# which calls only graphgen and oracle",
        f"n {n}",
        f"m {len(e)}",
        f"entries_sha256 {e_sha}",
        f"labels_sha256 {l_sha}",
        f"components {comps}",
    ] + [f"label {v} {int(L[v])}" for v in PROBES]
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
