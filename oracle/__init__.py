"""Sequential CPU oracle for connected-components labelling (test infrastructure).

Only the tests, the smoke check and the bench's CPU-baseline leg may import this
package. The GPU library never imports or links it, and it imports nothing from
the GPU library. See ``cc_oracle.c`` for the definitions each function follows
and the paper passages they cite.

All functions take numpy arrays: ``edges`` is an (m, 2) uint32 array of
unordered pairs, ``n`` the vertex count.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libccoracle.so")

OK, EINVAL, ERANGE, ENOMEM = 0, -1, -2, -3


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle returned status {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile libccoracle.so with gcc (single-threaded, -O2)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        u64, u32, i32, p = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p
        lib.oracle_cc_labels.argtypes = [u64, u64, p, p]; lib.oracle_cc_labels.restype = i32
        lib.oracle_count_labels.argtypes = [u64, p]; lib.oracle_count_labels.restype = u64
        lib.oracle_cc_labels_batch.argtypes = [u64, p, p, p, p, p]
        lib.oracle_cc_labels_batch.restype = i32
        lib.oracle_zroot.argtypes = [u64, u64, p, u64, p]; lib.oracle_zroot.restype = i32
        lib.oracle_push.argtypes = [u64, u64, p, u64, u32, p]; lib.oracle_push.restype = i32
        lib.oracle_jt_seq.argtypes = [u64, u64, p, u64, i32, p]; lib.oracle_jt_seq.restype = i32
        lib.oracle_siskin_log.argtypes = [u64, u64, p, p, u64, ctypes.POINTER(u64)]
        lib.oracle_siskin_log.restype = i32
        lib.oracle_rf_jt.argtypes = [u64, u64, p, u32, p]; lib.oracle_rf_jt.restype = i32
        lib.oracle_check_forest.argtypes = [u64, p, i32, u32, p]
        lib.oracle_check_forest.restype = ctypes.c_int64
        _lib = lib
    return _lib


def _edges(edges) -> np.ndarray:
    e = np.ascontiguousarray(np.asarray(edges).reshape(-1, 2))
    if e.dtype != np.uint32:
        e = e.astype(np.uint32)
    return e


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


def cc_labels(n: int, edges) -> np.ndarray:
    """L_v = min{u : u connected to v} (union-find, then min-ID pass)."""
    e = _edges(edges)
    L = np.empty(n, np.uint32)
    rc = _load().oracle_cc_labels(n, len(e), _p(e), _p(L))
    if rc != OK:
        raise OracleError(rc)
    return L


def count_components(L: np.ndarray) -> int:
    L = np.ascontiguousarray(L, dtype=np.uint32)
    return int(_load().oracle_count_labels(len(L), _p(L)))


def cc_labels_batch(vtx_off, edge_off, edges):
    """Per-graph local min-ID labels (int32) and per-graph status codes."""
    vo = np.ascontiguousarray(vtx_off, np.int64)
    eo = np.ascontiguousarray(edge_off, np.int64)
    e = np.ascontiguousarray(np.asarray(edges).reshape(-1, 2), np.int32)
    G = len(vo) - 1
    L = np.empty(int(vo[-1]), np.int32)
    st = np.empty(G, np.int32)
    rc = _load().oracle_cc_labels_batch(G, _p(vo), _p(eo), _p(e), _p(L), _p(st))
    if rc != OK:
        raise OracleError(rc)
    return L, st


def zroot(n: int, edges, K: int) -> int:
    """Most frequent endpoint among the K stride-sampled non-self-loop entries
    (K == 0: all entries), ties to the lowest ID; 0 if nothing is counted."""
    e = _edges(edges)
    z = ctypes.c_uint32(0)
    rc = _load().oracle_zroot(n, len(e), _p(e), K, ctypes.byref(z))
    if rc != OK:
        raise OracleError(rc)
    return int(z.value)


def push(n: int, edges, K: int, zmax: int) -> np.ndarray:
    """P after initialisation and the Initial Push from zmax over the sample."""
    e = _edges(edges)
    P = np.empty(n, np.uint32)
    rc = _load().oracle_push(n, len(e), _p(e), K, zmax, _p(P))
    if rc != OK:
        raise OracleError(rc)
    return P


def jt_seq(n: int, edges, steps: int | None = None, jump: bool = False) -> np.ndarray:
    """Algorithm 1 on one thread over the first `steps` entries (optional jumping)."""
    e = _edges(edges)
    P = np.empty(n, np.uint32)
    rc = _load().oracle_jt_seq(n, len(e), _p(e), len(e) if steps is None else steps,
                               1 if jump else 0, _p(P))
    if rc != OK:
        raise OracleError(rc)
    return P


def siskin_log(n: int, edges) -> np.ndarray:
    """Algorithm 2's messages on one thread: (child, new parent) per link, in order."""
    e = _edges(edges)
    cap = max(n, 1)
    log = np.empty((cap, 2), np.uint32)
    k = ctypes.c_uint64(0)
    rc = _load().oracle_siskin_log(n, len(e), _p(e), _p(log), cap, ctypes.byref(k))
    if rc != OK:
        raise OracleError(rc)
    return log[: k.value].copy()


def rf_jt(n: int, edges, zmax: int) -> np.ndarray:
    """Algorithm 3 with R (Formulas 1-2) on one thread; final root values (uint64)."""
    e = _edges(edges)
    P = np.empty(n, np.uint64)
    rc = _load().oracle_rf_jt(n, len(e), _p(e), zmax, _p(P))
    if rc != OK:
        raise OracleError(rc)
    return P


def check_forest(P: np.ndarray, zroot_on: bool = False, zmax: int = 0) -> int:
    """Number of roots of the parent forest P, or raise if P is not a key-monotone
    forest (see cc_oracle.c)."""
    P = np.ascontiguousarray(P, np.uint32)
    bad = ctypes.c_uint64(0)
    r = _load().oracle_check_forest(len(P), _p(P), 1 if zroot_on else 0, zmax, ctypes.byref(bad))
    if r < 0:
        raise AssertionError(f"parent array is not a key-monotone forest at vertex {bad.value}")
    return int(r)


# ---- compact vertex IDs of the exchange (Sec. V) ---------------------------------
# Each ID travels in ceil(log2(|V|) / 8) bytes (at least one), least significant
# byte first; a list of IDs is the concatenation of their byte groups.

def id_bytes(n: int) -> int:
    """Bytes per compact ID for IDs in [0, n): the smallest k >= 1 with 256^k >= n."""
    k = 1
    while 256 ** k < n:
        k += 1
    return k


def pack_ids(ids, k: int) -> np.ndarray:
    """uint8 array of len(ids) * k bytes; raises OracleError(ERANGE) if an ID
    does not fit in k bytes."""
    a = np.asarray(ids, dtype=np.uint64).ravel()
    if k < 1 or k > 4:
        raise OracleError(EINVAL)
    if a.size and int(a.max()) >= 256 ** k:
        raise OracleError(ERANGE)
    out = np.empty(a.size * k, np.uint8)
    for j in range(k):                                 # byte j of every ID
        out[j::k] = (a >> np.uint64(8 * j)) & np.uint64(0xFF)
    return out


def unpack_ids(buf, k: int) -> np.ndarray:
    """Inverse of pack_ids: uint32 IDs from len(buf) / k byte groups."""
    b = np.asarray(buf, dtype=np.uint8).ravel()
    if k < 1 or k > 4 or b.size % k:
        raise OracleError(EINVAL)
    out = np.zeros(b.size // k, np.uint64)
    for j in range(k):
        out |= b[j::k].astype(np.uint64) << np.uint64(8 * j)
    return out.astype(np.uint32)


# ---- CSR input ---------------------------------------------------------------------
# Row u of a CSR graph holds the entries (u, adj[j]), offsets[u] <= j < offsets[u+1];
# as unordered pairs they are a COO list, which is what the labels are defined on.

def csr_pairs(offsets, adj) -> np.ndarray:
    """The (m, 2) uint32 entries of a CSR graph, row by row."""
    off = np.asarray(offsets, dtype=np.int64)
    if off.size == 0 or off[0] != 0 or np.any(np.diff(off) < 0):
        raise OracleError(EINVAL)
    n = off.size - 1
    a = np.asarray(adj, dtype=np.uint32)[: off[-1]]
    u = np.repeat(np.arange(n, dtype=np.uint32), np.diff(off))
    return np.stack([u, a], axis=1)


def cc_labels_csr(offsets, adj) -> np.ndarray:
    off = np.asarray(offsets, dtype=np.int64)
    return cc_labels(off.size - 1, csr_pairs(off, adj))


def zroot_csr(offsets) -> int:
    """The vertex with the longest row (Algorithm 4's max degree on CSR), ties to the
    lowest ID; 0 when every row is empty."""
    d = np.diff(np.asarray(offsets, dtype=np.int64))
    return int(np.argmax(d)) if d.size and d.max() > 0 else 0


# ---- 64-bit vertex IDs (Sec. V: 8-byte IDs at 2^32 vertices and beyond) ----------------

def cc_labels_sparse64(edges) -> tuple[np.ndarray, np.ndarray]:
    """Labels of a graph whose IDs may exceed 32 bits, on the vertices that occur in
    an entry: returns (ids, labels), ids sorted ascending, labels[i] = the smallest
    ID connected to ids[i]. Every other vertex is alone (its label is itself).
    The occurring IDs are renumbered 0..k-1 in increasing order, labelled by
    cc_labels, and mapped back; renumbering in order keeps each component's
    smallest member the smallest."""
    e = np.asarray(edges, dtype=np.uint64).reshape(-1, 2)
    ids = np.unique(e)
    if ids.size >= 2 ** 32:
        raise OracleError(EINVAL)
    dense = np.searchsorted(ids, e).astype(np.uint32)
    lab = cc_labels(ids.size, dense)
    return ids, ids[lab.astype(np.int64)]

