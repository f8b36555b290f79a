"""Build libccmi.so (the HIP library behind include/cc.h) for gfx950 with hipcc.

build(stress=True) builds libccmi_stress.so instead: the same sources with
CCM_STRESS_DELAYS, which pauses each wave for a varying time before every link
CAS and path-splitting store (race testing only; load it with CCMI_LIBRARY)."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libccmi.so")
STRESS_LIB = os.path.join(PKG, "libccmi_stress.so")
SOURCES = ["cc_api.hip", "cc_kernels.hip", "cc_tiled.hip", "cc_batch.hip", "cc_serve.hip",
           "cc_exchange.hip", "cc_wide.hip", "cc_noalloc.hip", "cc_tune.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep the compiler from forming packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def build(verbose: bool = False, stress: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    out = STRESS_LIB if stress else LIB
    tmp = out + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, *(["-DCCM_STRESS_DELAYS=1"] if stress else []),
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
