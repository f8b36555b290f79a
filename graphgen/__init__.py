"""Seeded synthetic graph inputs (uint32 COO edge lists) for tests and benches.

The generators are written in C (``graphgen.c``) and hold no connected-components
arithmetic: the oracle and the GPU library both take their output as plain
arrays. Every entry is a pure function of (seed, index), so a workload is
reproducible from its recipe alone.

Workloads (sizes as used by the parity tests and the bench):

* ``er``            Erdos-Renyi G(n, m), endpoints uniform on [0, n), self-loops
                    and duplicates kept.
* ``rmat``          R-MAT (a, b, c) = (0.57, 0.19, 0.19), 2^scale vertices,
                    IDs relabelled by a keyed permutation.
* ``rmat_sym``      the same, each entry followed (in a second half) by its
                    reversed copy.
* ``rmat_extras``   R-MAT plus 1 % isolated vertices and paths of 2..64
                    vertices appended with consecutive new IDs.
* ``batch``         many small graphs with local int32 IDs and offsets.
* ``rmat_share``    one vertex-range share of a permuted R-MAT graph.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")

SEED_BASE = 0x2507036950000000
RMAT_ABC = (Fraction(57, 100), Fraction(19, 100), Fraction(19, 100))


def build(force: bool = True) -> str:
    """Compile libgraphgen.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        u64, u32, p = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
        lib.gg_draw.argtypes = [u64, u64]; lib.gg_draw.restype = u64
        lib.gg_perm.argtypes = [u32, u64, u64]; lib.gg_perm.restype = u64
        lib.gg_er.argtypes = [u64, u64, u64, p]; lib.gg_er.restype = None
        lib.gg_rmat.argtypes = [u32, u64, u32, u32, u32, u64, u64, p]; lib.gg_rmat.restype = None
        lib.gg_rmat_share.argtypes = [u32, u64, u32, u32, u32, u64, u64, u64, u64, p, u64]
        lib.gg_rmat_share.restype = u64
        lib.gg_symmetrise.argtypes = [u64, p]; lib.gg_symmetrise.restype = None
        lib.gg_paths.argtypes = [u64, u64, u32, u32, u64, p, p, p]; lib.gg_paths.restype = u64
        lib.gg_batch.argtypes = [u64, p, p, p, p, u32, u32, u32, p]; lib.gg_batch.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def draw(seed: int, i: int) -> int:
    """The i-th SplitMix64 output for `seed` (the generators' counter-based draw)."""
    return int(_load().gg_draw(seed & (2**64 - 1), i))


def subseed(seed: int, tag: int) -> int:
    return draw(seed, tag)


def rmat_thresholds(a=RMAT_ABC[0], b=RMAT_ABC[1], c=RMAT_ABC[2]):
    """Cumulative quadrant probabilities as 32-bit integer thresholds."""
    a, b, c = Fraction(a), Fraction(b), Fraction(c)
    to32 = lambda f: min(int(f * 2**32), 2**32 - 1)
    return to32(a), to32(a + b), to32(a + b + c)


def er(n: int, m: int, seed: int) -> np.ndarray:
    out = np.empty((m, 2), dtype=np.uint32)
    if m:
        _load().gg_er(n, m, seed, _ptr(out))
    return out


def rmat(scale: int, m: int, seed: int, permute: bool = True) -> np.ndarray:
    t1, t2, t3 = rmat_thresholds()
    out = np.empty((m, 2), dtype=np.uint32)
    if m:
        perm_seed = subseed(seed, 0x5045524D) | 1 if permute else 0
        _load().gg_rmat(scale, m, t1, t2, t3, seed, perm_seed, _ptr(out))
    return out


def rmat_sym(scale: int, m_undirected: int, seed: int) -> np.ndarray:
    """R-MAT entries followed by their reversed copies (2*m_undirected entries)."""
    t1, t2, t3 = rmat_thresholds()
    out = np.empty((2 * m_undirected, 2), dtype=np.uint32)
    if m_undirected:
        _load().gg_rmat(scale, m_undirected, t1, t2, t3, seed,
                        subseed(seed, 0x5045524D) | 1, _ptr(out))
        _load().gg_symmetrise(m_undirected, _ptr(out))
    return out


@dataclass
class ExtrasGraph:
    edges: np.ndarray          # (m, 2) uint32
    n: int                     # total vertices
    n_rmat: int                # R-MAT vertex range [0, n_rmat)
    isolated: tuple            # [lo, hi) of isolated IDs
    path_starts: np.ndarray    # first ID of each path (uint64)
    path_lens: np.ndarray      # vertices per path


def rmat_extras(scale: int, edgefactor: int, seed: int, isolated_frac=Fraction(1, 100),
                n_paths: int = 10000, lmin: int = 2, lmax: int = 64) -> ExtrasGraph:
    """R-MAT(scale, edgefactor) + floor(isolated_frac*2^scale) isolated IDs + paths.

    Path p has lmin + draw % (lmax-lmin+1) vertices with consecutive IDs after the
    isolated block; its edges are emitted highest ID first.
    """
    lib = _load()
    n_rmat = 1 << scale
    m_rmat = edgefactor * n_rmat
    n_iso = int(Fraction(isolated_frac) * n_rmat)
    base = n_rmat + n_iso
    pseed = subseed(seed, 0x50415448)
    nv = ctypes.c_uint64(0)
    m_paths = lib.gg_paths(base, n_paths, lmin, lmax, pseed, None, None, ctypes.byref(nv))
    n_total = base + nv.value
    if n_total >= 2**32:
        raise ValueError("vertex count exceeds uint32")
    out = np.empty((m_rmat + m_paths, 2), dtype=np.uint32)
    t1, t2, t3 = rmat_thresholds()
    if m_rmat:
        lib.gg_rmat(scale, m_rmat, t1, t2, t3, seed, subseed(seed, 0x5045524D) | 1, _ptr(out))
    starts = np.empty(n_paths, dtype=np.uint64)
    tail = out[m_rmat:]
    lib.gg_paths(base, n_paths, lmin, lmax, pseed, _ptr(tail) if m_paths else None,
                 _ptr(starts), ctypes.byref(nv))
    lens = np.diff(np.append(starts, np.uint64(n_total))).astype(np.int64) if n_paths else \
        np.empty(0, np.int64)
    return ExtrasGraph(out, n_total, n_rmat, (n_rmat, base), starts, lens)


def rmat_share(scale: int, edgefactor: int, seed: int, shares: int, k: int) -> tuple:
    """Share k of `shares` equal vertex ranges of a permuted R-MAT graph.

    Returns (edges, n) where n = 2^scale (the parent array stays global-size):
    the generated entries whose first endpoint lies in the share's range, in
    generation order.
    """
    lib = _load()
    t1, t2, t3 = rmat_thresholds()
    n = 1 << scale
    m_total = edgefactor * n
    span = n // shares
    lo, hi = k * span, (k + 1) * span
    perm_seed = subseed(seed, 0x5045524D) | 1
    cap = int(m_total / shares * 1.03) + (1 << 20)
    out = np.empty((cap, 2), dtype=np.uint32)
    cnt = lib.gg_rmat_share(scale, m_total, t1, t2, t3, seed, perm_seed, lo, hi, _ptr(out), cap)
    if cnt == 2**64 - 1:
        raise MemoryError("share staging allocation failed")
    if cnt > cap:
        out = np.empty((cnt, 2), dtype=np.uint32)
        got = lib.gg_rmat_share(scale, m_total, t1, t2, t3, seed, perm_seed, lo, hi, _ptr(out), cnt)
        if got != cnt:
            raise RuntimeError("share generation count mismatch")
        return out, n
    return out[:cnt], n


def rmat30_share() -> tuple:
    """Share 0 of 16 of R-MAT scale 30, edgefactor 16 (n = 2^30, about 2^30 entries)."""
    return rmat_share(30, 16, config_seed(5), 16, 0)


@dataclass
class Batch:
    edges: np.ndarray      # (sum m, 2) int32 local IDs
    vtx_off: np.ndarray    # int64[G+1]
    edge_off: np.ndarray   # int64[G+1]
    kinds: np.ndarray      # int32[G]: 0 ER, 1 R-MAT

    @property
    def G(self) -> int:
        return len(self.kinds)

    def graph(self, g: int):
        a, b = int(self.edge_off[g]), int(self.edge_off[g + 1])
        return self.edges[a:b], int(self.vtx_off[g + 1] - self.vtx_off[g])


def batch(G: int, seed: int, lg_n_lo: float = 8.0, lg_n_hi: float = 16.0,
          deg_lo: float = 2.0, deg_hi: float = 32.0) -> Batch:
    """G graphs: n log-uniform in [2^lg_n_lo, 2^lg_n_hi], average degree d uniform in
    [deg_lo, deg_hi] (m = round(n*d/2) entries stored once), even g ER, odd g R-MAT."""
    ns = np.empty(G, np.int64)
    ms = np.empty(G, np.int64)
    seeds = np.empty(G, np.uint64)
    for g in range(G):
        r0 = draw(seed, 3 * g) >> 11
        r1 = draw(seed, 3 * g + 1) >> 11
        u0 = r0 / float(1 << 53)
        u1 = r1 / float(1 << 53)
        ng = int(math.floor(2.0 ** (lg_n_lo + (lg_n_hi - lg_n_lo) * u0)))
        ng = max(1, min(ng, int(2 ** lg_n_hi)))
        d = deg_lo + (deg_hi - deg_lo) * u1
        ns[g] = ng
        ms[g] = int(round(ng * d / 2.0))
        seeds[g] = draw(seed, 3 * g + 2)
    kinds = (np.arange(G) % 2).astype(np.int32)
    vtx_off = np.zeros(G + 1, np.int64)
    edge_off = np.zeros(G + 1, np.int64)
    np.cumsum(ns, out=vtx_off[1:])
    np.cumsum(ms, out=edge_off[1:])
    out = np.empty((int(edge_off[-1]), 2), dtype=np.int32)
    t1, t2, t3 = rmat_thresholds()
    if G:
        _load().gg_batch(G, _ptr(ns), _ptr(edge_off), _ptr(kinds), _ptr(seeds), t1, t2, t3,
                         _ptr(out))
    return Batch(out, vtx_off, edge_off, kinds)


def batch_from_graphs(graphs) -> Batch:
    """Pack a list of (edges (k,2) int-like, n) into a Batch with local int32 IDs."""
    G = len(graphs)
    vtx_off = np.zeros(G + 1, np.int64)
    edge_off = np.zeros(G + 1, np.int64)
    for g, (e, n) in enumerate(graphs):
        vtx_off[g + 1] = vtx_off[g] + n
        edge_off[g + 1] = edge_off[g] + len(e)
    out = np.empty((int(edge_off[-1]), 2), np.int32)
    for g, (e, n) in enumerate(graphs):
        out[edge_off[g]:edge_off[g + 1]] = np.asarray(e, dtype=np.int64).astype(np.int32)
    return Batch(out, vtx_off, edge_off, np.zeros(G, np.int32))


# ---- the named workloads -------------------------------------------------

def config_seed(idx: int) -> int:
    return SEED_BASE + idx


def er_65k():
    """ER G(n=65,536, m=1,048,576), seeded; returns (edges, n)."""
    return er(65536, 1 << 20, config_seed(1)), 65536


def rmat22_sym():
    """R-MAT scale 22, edgefactor 16, permuted, symmetrised; returns (edges, n)."""
    return rmat_sym(22, 16 << 22, config_seed(2)), 1 << 22


def rmat26_extras() -> ExtrasGraph:
    """R-MAT scale 26, edgefactor 16, permuted, + 1 % isolated + 10,000 paths of 2..64."""
    return rmat_extras(26, 16, config_seed(3))


def batch_4096() -> Batch:
    return batch(4096, config_seed(4))


def batch_with_tail(seed: int, G: int = 4096, tail: int = 8, tail_scale: int = 20,
                    tail_ef: int = 8) -> Batch:
    """G - tail graphs drawn as in batch() (n log-uniform in [2^8, 2^16], degree
    uniform in [2, 32]) followed by `tail` R-MAT graphs of 2^tail_scale vertices
    and tail_ef * 2^tail_scale entries: the same mix with a few graphs too large
    for one workgroup."""
    head = batch(G - tail, seed)
    graphs = [head.graph(g) for g in range(head.G)]
    for t in range(tail):
        graphs.append((rmat(tail_scale, tail_ef << tail_scale, subseed(seed, 0x7A11 + t)),
                       1 << tail_scale))
    return batch_from_graphs(graphs)


def pareto_n(u: float, alpha: float = 1.5, lo: float = 2.0**10, hi: float = 2.0**24) -> int:
    """Inverse CDF of a Pareto(alpha) truncated to [lo, hi] at quantile u."""
    la, ha = lo ** -alpha, hi ** -alpha
    x = (la - u * (la - ha)) ** (-1.0 / alpha)
    return int(min(max(math.floor(x * (1.0 + 1e-12)), lo), hi))


@dataclass
class Request:
    n: int
    ef: int
    kind: int          # 0 ER, 1 R-MAT
    seed: int
    arrival_s: float   # offset from stream start

    @property
    def m(self) -> int:
        return self.n * self.ef

    def edges(self) -> np.ndarray:
        if self.kind == 0:
            return er(self.n, self.m, self.seed)
        sc = max(1, (self.n - 1).bit_length())
        if (1 << sc) == self.n:
            return rmat(sc, self.m, self.seed)
        b = batch_single(self.n, self.m, self.seed)
        return b.view(np.uint32)


def batch_single(n: int, m: int, seed: int) -> np.ndarray:
    """One R-MAT graph on [0, n) with rejection (the batch recipe), int32 (m, 2)."""
    ns = np.array([n], np.int64)
    eo = np.array([0, m], np.int64)
    kinds = np.array([1], np.int32)
    seeds = np.array([seed], np.uint64)
    out = np.empty((m, 2), np.int32)
    t1, t2, t3 = rmat_thresholds()
    if m:
        _load().gg_batch(1, _ptr(ns), _ptr(eo), _ptr(kinds), _ptr(seeds), t1, t2, t3, _ptr(out))
    return out


def serve_stream(count: int, seed: int, rate_per_s: float, lo=2.0**10, hi=2.0**24,
                 alpha: float = 1.5) -> list:
    """Poisson arrivals at `rate_per_s`; n ~ truncated Pareto(alpha) on [lo, hi];
    edgefactor uniform in 8..32; ER / R-MAT alternate by a fair draw."""
    reqs = []
    t = 0.0
    for i in range(count):
        r = [draw(seed, 4 * i + j) for j in range(4)]
        u_gap = ((r[0] >> 11) + 1) / float((1 << 53) + 1)
        t += -math.log(u_gap) / rate_per_s
        n = pareto_n((r[1] >> 11) / float(1 << 53), alpha, lo, hi)
        ef = 8 + int(r[2] % 25)
        kind = int((r[2] >> 32) & 1)
        reqs.append(Request(n, ef, kind, r[3], t))
    return reqs


# ---- device twin (graphgen_dev.hip): the same entries, generated on the GPU ----

_DEV_SRC = os.path.join(_HERE, "graphgen_dev.hip")
_DEV_LIB_PATH = os.path.join(_HERE, "libgraphgen_dev.so")
_dev_lib = None


def build_dev() -> str:
    """Compile libgraphgen_dev.so for gfx950 with hipcc."""
    tmp = _DEV_LIB_PATH + ".tmp"
    subprocess.check_call(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-fPIC", "-shared",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-Wno-unused-command-line-argument", "-o", tmp, _DEV_SRC],
                          stderr=subprocess.DEVNULL)
    os.replace(tmp, _DEV_LIB_PATH)
    return _DEV_LIB_PATH


def _load_dev():
    global _dev_lib
    if _dev_lib is None:
        if not os.path.exists(_DEV_LIB_PATH):
            raise ImportError(f"{_DEV_LIB_PATH} is missing: run graphgen.build_dev()")
        lib = ctypes.CDLL(_DEV_LIB_PATH)
        u64, u32, p = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
        lib.gg_dev_rmat.argtypes = [u32, u64, u32, u32, u32, u64, u64, p]
        lib.gg_dev_rmat.restype = ctypes.c_int
        lib.gg_dev_share_count.argtypes = [u32, u64, u32, u32, u32, u64, u64, u64, u64, u64, p]
        lib.gg_dev_share_count.restype = ctypes.c_int
        lib.gg_dev_share_write.argtypes = [u32, u64, u32, u32, u32, u64, u64, u64, u64, u64, p, p]
        lib.gg_dev_share_write.restype = ctypes.c_int
        _dev_lib = lib
    return _dev_lib


def rmat_dev(scale: int, m: int, seed: int, permute: bool = True):
    """rmat() generated on the current GPU: an (m, 2) int32 torch tensor, same bits."""
    import torch
    lib = _load_dev()
    t1, t2, t3 = rmat_thresholds()
    out = torch.empty((m, 2), dtype=torch.int32, device="cuda")
    perm_seed = subseed(seed, 0x5045524D) | 1 if permute else 0
    if m and lib.gg_dev_rmat(scale, m, t1, t2, t3, seed, perm_seed, out.data_ptr()) != 0:
        raise RuntimeError("gg_dev_rmat failed")
    return out


def rmat_share_dev(scale: int, edgefactor: int, seed: int, shares: int, k: int,
                   span: int = 1 << 20):
    """rmat_share() generated on the current GPU: ((cnt, 2) int32 tensor, n)."""
    import torch
    lib = _load_dev()
    t1, t2, t3 = rmat_thresholds()
    n = 1 << scale
    m_total = edgefactor * n
    width = n // shares
    lo, hi = k * width, (k + 1) * width
    perm_seed = subseed(seed, 0x5045524D) | 1
    blocks = (m_total + span - 1) // span
    counts = torch.empty(blocks, dtype=torch.int32, device="cuda")
    if lib.gg_dev_share_count(scale, m_total, t1, t2, t3, seed, perm_seed, lo, hi, span,
                              counts.data_ptr()) != 0:
        raise RuntimeError("gg_dev_share_count failed")
    c64 = counts.to(torch.int64)
    offs = torch.zeros(blocks, dtype=torch.int64, device="cuda")
    if blocks > 1:
        offs[1:] = torch.cumsum(c64, 0)[:-1]
    total = int(c64.sum().item())
    out = torch.empty((total, 2), dtype=torch.int32, device="cuda")
    if total and lib.gg_dev_share_write(scale, m_total, t1, t2, t3, seed, perm_seed, lo, hi, span,
                                        offs.data_ptr(), out.data_ptr()) != 0:
        raise RuntimeError("gg_dev_share_write failed")
    return out, n


def rmat30_share_dev():
    """rmat30_share() generated on the GPU."""
    return rmat_share_dev(30, 16, config_seed(5), 16, 0)
