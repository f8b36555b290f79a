"""Python binding of libccmi (include/cc.h): connected components on MI355X.

Argument marshalling only: every step runs in the HIP library. PyTorch provides
device memory and streams; tensors are passed as raw device pointers. The
binding refuses to run when the library is missing (no CPU fallback).

Entry points mirror the C ABI:

    solve(edges, n)                      -> int32/uint32 labels (synchronous)
    Context().solve_async(edges, n, L, flags=..., stream=...)
    Context().sync(stream)
    Context().init / zroot / push / hook / compress / canon   (one step each)
    Context().batch(vtx_off, edge_off, edges, L, status)
    Server(ctx).submit / wait / close
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
# CCMI_LIBRARY selects another build of the same library, such as the
# race-testing build libccmi_stress.so next to this file.
LIB_PATH = os.environ.get("CCMI_LIBRARY") or os.path.join(_PKG, "libccmi.so")

CC_OK, CC_EINVAL, CC_ERANGE, CC_ENOMEM, CC_EDEVICE, CC_EAGAIN, CC_ECANCELED, CC_ETIMEDOUT = \
    0, -1, -2, -3, -4, -5, -6, -7
F_ZROOT, F_ZROOT_EXACT, F_ZROOT_HINT, F_NO_SPLIT, F_NO_TILE = 0x1, 0x2, 0x4, 0x8, 0x10
F_CANON, F_SYMMETRIC = 0x20, 0x40
STATUS_RING = 256
DRAIN_MAX_CHUNKS = 1024
NOALLOC_SCRATCH_BYTES = 16 << 20


class CCError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = _lib_or_none()
        detail = lib.cc_last_error_detail().decode() if lib else ""
        name = lib.cc_strerror(code).decode() if lib else str(code)
        super().__init__(f"{where}: {name} ({detail})")
        self.code = code


class _CtxOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("zroot_samples", ctypes.c_uint32),
                ("hbm_budget", ctypes.c_uint64), ("tune_cache", ctypes.c_char_p),
                ("batch_autotune", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


BATCH_WAVE_MAX_N = 4096
BATCH_WAVE_MAX_M = 65536
TUNE_MAX_CAND = 16
SCHED_DEFAULT, SCHED_TUNED, SCHED_STORED, SCHED_FORCED = 0, 1, 2, 3


class BatchSched(ctypes.Structure):
    """cc_batch_sched: graphs with n >= multi_min_n (if > 0) run on the whole
    device, graphs with n <= wave_max_n (and m <= BATCH_WAVE_MAX_M) on one
    wavefront, the rest on one workgroup each."""
    _fields_ = [("wave_max_n", ctypes.c_uint32), ("multi_min_n", ctypes.c_uint32)]

    def as_tuple(self):
        return (int(self.wave_max_n), int(self.multi_min_n))

    def __repr__(self):
        return f"BatchSched(wave_max_n={self.wave_max_n}, multi_min_n={self.multi_min_n})"


class TuneResult(ctypes.Structure):
    """cc_batch_tune_result."""
    _fields_ = [("pick", BatchSched), ("source", ctypes.c_uint32), ("n_cand", ctypes.c_uint32),
                ("cand", BatchSched * TUNE_MAX_CAND), ("cand_ms", ctypes.c_float * TUNE_MAX_CAND),
                ("signature", ctypes.c_char * 320)]

    def candidates(self):
        """[((wave_max_n, multi_min_n), ms), ...] of the timed candidates."""
        return [(self.cand[i].as_tuple(), float(self.cand_ms[i])) for i in range(self.n_cand)]


class _ServeOpts(ctypes.Structure):
    _fields_ = [("max_inflight", ctypes.c_uint32), ("queue_capacity", ctypes.c_uint32),
                ("streams", ctypes.c_uint32), ("small_n", ctypes.c_uint32),
                ("hbm_budget", ctypes.c_uint64), ("coalesce_us", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class Status(ctypes.Structure):
    """cc_status_t: the outcome of one asynchronous whole-path call; pass it as
    `status=` and resolve it with Context.status_wait."""
    _fields_ = [("ctx", ctypes.c_void_p), ("seq", ctypes.c_uint64), ("slot", ctypes.c_uint32),
                ("pad", ctypes.c_uint32)]


class ReqStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("batched", ctypes.c_uint32),
                ("t_submit_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64),
                ("t_start_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64)]


_lib = None

# name -> (restype, argtypes)
_P, _U64, _U32, _I32, _I64 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, \
    ctypes.c_int64
SIGNATURES = {
    "cc_strerror": (ctypes.c_char_p, [_I32]),
    "cc_last_error_detail": (ctypes.c_char_p, []),
    "cc_version": (_I32, []),
    "cc_create": (_I32, [ctypes.POINTER(_P), ctypes.POINTER(_CtxOpts)]),
    "cc_destroy": (None, [_P]),
    "cc_solve": (_I32, [_U64, _U64, _P, _P]),
    "cc_solve_async": (_I32, [_P, _U64, _U64, _P, _P, _U32, _U32, _P, ctypes.POINTER(Status)]),
    "cc_status_wait": (_I32, [ctypes.POINTER(Status), _I64]),
    "cc_solve_noalloc": (_I32, [_U64, _U64, _P, _P, _U32, _U32, _P, _P]),
    "cc_sync": (_I32, [_P, _P]),
    "cc_solve_csr": (_I32, [_P, _U64, _P, _P, _P, _U32, _U32, _P, ctypes.POINTER(Status)]),
    "cc_solve_u64": (_I32, [_P, _U64, _U64, _P, _P, _U32, _P, ctypes.POINTER(Status)]),
    "cc_init": (_I32, [_P, _U64, _P, _P]),
    "cc_zroot": (_I32, [_P, _U64, _U64, _P, _U32, _U32, _P]),
    "cc_push": (_I32, [_P, _U64, _U64, _P, _P, _P]),
    "cc_hook": (_I32, [_P, _U64, _U64, _P, _P, _U32, _P]),
    "cc_hook_log": (_I32, [_P, _U64, _U64, _P, _P, _U32, _P, _U64, _P, _P]),
    "cc_hook_log_drain": (_I32, [_P, _U64, _U64, _P, _P, _U32, _P, _U64, _P, _U64, _U32,
                                 ctypes.POINTER(_U64), _P]),
    "cc_compress": (_I32, [_P, _U64, _P, _U32, _P]),
    "cc_canon": (_I32, [_P, _U64, _P, _P]),
    "cc_get_zroot": (_I32, [_P, _P, ctypes.POINTER(_U32)]),
    "cc_export": (_I32, [_P, _U64, _P, _U32, _P, _U64, _P, _U64, ctypes.POINTER(_U64),
                         ctypes.POINTER(_U64), _P]),
    "cc_hook_ids": (_I32, [_P, _U64, _U64, _P, _U32, _P, _U32, _P]),
    "cc_id_bytes": (_U32, [_U64]),
    "cc_pack_ids": (_I32, [_P, _U64, _P, _U32, _P, _P]),
    "cc_unpack_ids": (_I32, [_P, _U64, _P, _U32, _P, _P]),
    "cc_batch": (_I32, [_P, _U32, _P, _P, _P, _P, _P, _P]),
    "cc_batch_ex": (_I32, [_P, _U32, _P, _P, _P, _P, _P, ctypes.POINTER(BatchSched), _P]),
    "cc_batch_sched_force": (_I32, [_P, ctypes.POINTER(BatchSched)]),
    "cc_batch_tune": (_I32, [_P, _U32, _P, _P, _P, _P, _P, _U32, ctypes.POINTER(TuneResult), _P]),
    "cc_batch_graph_create": (_I32, [_P, _U32, _P, _P, _P, _P, _P, _P, ctypes.POINTER(_P)]),
    "cc_batch_graph_launch": (_I32, [_P, _P]),
    "cc_batch_graph_destroy": (None, [_P]),
    "cc_serve_open": (_I32, [_P, ctypes.POINTER(_ServeOpts), ctypes.POINTER(_P)]),
    "cc_serve_submit": (_I32, [_P, _U64, _U64, _P, _P, _U32, ctypes.POINTER(_U64)]),
    "cc_serve_wait": (_I32, [_P, _U64, _I64, ctypes.POINTER(ReqStats)]),
    "cc_serve_close": (_I32, [_P]),
}


def _lib_or_none():
    return _lib


def load():
    """Load libccmi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              f"`python -c 'import __graft_entry__ as g; g.build()'`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int, where: str):
    if rc != CC_OK:
        raise CCError(rc, where)


def _dptr(t: torch.Tensor | None, dtypes) -> int | None:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if t.dtype not in dtypes:
        raise TypeError(f"dtype {t.dtype} not in {dtypes}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr() if t.numel() else None


_ID = (torch.int32, torch.uint32)


def _stream(stream) -> int | None:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream or None
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream or None
    return int(stream) or None


def _st(status):
    return None if status is None else ctypes.byref(status)


def solve_noalloc(edges: torch.Tensor, n: int, L: torch.Tensor, flags: int = 0,
                  zroot_hint: int = 0, status: torch.Tensor | None = None, stream=None):
    """cc_solve_noalloc: the whole path with the library's fixed scratch, no
    allocation; `status` an int32 device tensor of one element (or None)."""
    lib = load()
    m = edges.shape[0] if edges.dim() == 2 else edges.numel() // 2
    _check(lib.cc_solve_noalloc(n, m, _dptr(edges, _ID), _dptr(L, _ID), flags, zroot_hint,
                                _dptr(status, (torch.int32,)), _stream(stream)),
           "cc_solve_noalloc")


def solve(edges: torch.Tensor, n: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """cc_solve: labels L (n entries, dtype of `edges`) with L_v = min ID of v's component.

    `edges` is an (m, 2) int32/uint32 device tensor of unordered pairs. Runs on the
    null stream and waits for it; the current torch stream is synchronised first.
    """
    lib = load()
    m = edges.shape[0] if edges.dim() == 2 else edges.numel() // 2
    if out is None:
        out = torch.empty(n, dtype=edges.dtype, device=edges.device)
    torch.cuda.current_stream().synchronize()
    _check(lib.cc_solve(n, m, _dptr(edges, _ID), _dptr(out, _ID)), "cc_solve")
    return out


class Context:
    """A cc_ctx: scratch for one solve at a time per stream (see cc.h)."""

    def __init__(self, device: int | None = None, zroot_samples: int = 0, hbm_budget: int = 0,
                 tune_cache: str | None = None, batch_autotune: bool = False):
        lib = load()
        o = _CtxOpts(-1 if device is None else device, zroot_samples, hbm_budget,
                     None if tune_cache is None else tune_cache.encode(), int(batch_autotune), 0)
        h = ctypes.c_void_p()
        _check(lib.cc_create(ctypes.byref(h), ctypes.byref(o)), "cc_create")
        self._h = h
        self.lib = lib

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            self.lib.cc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # whole path
    def solve_async(self, edges, n, L, flags=0, zroot_hint=0, stream=None, status=None):
        """cc_solve_async; with status (a Status), the call's own outcome goes there
        (Context.status_wait) instead of to the context's status word."""
        m = edges.shape[0] if edges.dim() == 2 else edges.numel() // 2
        _check(self.lib.cc_solve_async(self._h, n, m, _dptr(edges, _ID), _dptr(L, _ID), flags,
                                       zroot_hint, _stream(stream), _st(status)), "cc_solve_async")

    def status_wait(self, status, timeout_us: int = -1) -> int:
        """cc_status_wait: the outcome of the call that filled `status` (CC_OK,
        CC_ERANGE, CC_EINVAL or CC_ETIMEDOUT), without raising for those."""
        rc = self.lib.cc_status_wait(ctypes.byref(status), timeout_us)
        if rc not in (CC_OK, CC_ERANGE, CC_EINVAL, CC_ETIMEDOUT):
            _check(rc, "cc_status_wait")
        return rc

    def solve_csr_async(self, offsets, adj, n, L, flags=0, zroot_hint=0, stream=None, status=None):
        """cc_solve_csr: offsets (n+1,) int64 and adj (m,) ID tensors on the device."""
        _check(self.lib.cc_solve_csr(self._h, n, _dptr(offsets, (torch.int64, torch.uint64)),
                                     _dptr(adj, _ID), _dptr(L, _ID), flags, zroot_hint,
                                     _stream(stream), _st(status)), "cc_solve_csr")

    def solve_csr(self, offsets, adj, n, flags=0, zroot_hint=0, out=None, stream=None):
        if out is None:
            out = torch.empty(n, dtype=adj.dtype, device=adj.device)
        self.solve_csr_async(offsets, adj, n, out, flags, zroot_hint, stream)
        _check(self.sync(stream), "solve_csr")
        return out

    def solve_u64_async(self, edges, n, L, flags=0, stream=None, status=None):
        """cc_solve_u64: edges (m, 2) and L (n,) int64 device tensors (IDs as uint64 bits)."""
        _W = (torch.int64, torch.uint64)
        _check(self.lib.cc_solve_u64(self._h, n, edges.shape[0], _dptr(edges, _W), _dptr(L, _W),
                                     flags, _stream(stream), _st(status)), "cc_solve_u64")

    def solve_u64(self, edges, n, flags=0, out=None, stream=None):
        if out is None:
            out = torch.empty(n, dtype=torch.int64, device=edges.device)
        self.solve_u64_async(edges, n, out, flags, stream)
        _check(self.sync(stream), "solve_u64")
        return out

    def sync(self, stream=None) -> int:
        """Wait for the stream; returns the status word's outcome, CC_OK, CC_ERANGE,
        CC_ENOMEM (a full update log) or CC_EINVAL (bad CSR offsets), without raising
        for those."""
        rc = self.lib.cc_sync(self._h, _stream(stream))
        if rc not in (CC_OK, CC_ERANGE, CC_ENOMEM, CC_EINVAL):
            _check(rc, "cc_sync")
        return rc

    def solve(self, edges, n, flags=0, zroot_hint=0, out=None, stream=None):
        if out is None:
            out = torch.empty(n, dtype=edges.dtype, device=edges.device)
        self.solve_async(edges, n, out, flags, zroot_hint, stream)
        rc = self.sync(stream)
        _check(rc, "solve")
        return out

    # steps
    def init(self, n, P, stream=None):
        _check(self.lib.cc_init(self._h, n, _dptr(P, _ID), _stream(stream)), "cc_init")

    def zroot(self, edges, n, flags=0, zroot_hint=0, stream=None):
        m = edges.shape[0]
        _check(self.lib.cc_zroot(self._h, n, m, _dptr(edges, _ID), flags, zroot_hint,
                                 _stream(stream)), "cc_zroot")

    def get_zroot(self, stream=None) -> int:
        z = ctypes.c_uint32(0)
        _check(self.lib.cc_get_zroot(self._h, _stream(stream), ctypes.byref(z)), "cc_get_zroot")
        return int(z.value)

    def push(self, edges, n, P, stream=None):
        _check(self.lib.cc_push(self._h, n, edges.shape[0], _dptr(edges, _ID), _dptr(P, _ID),
                                _stream(stream)), "cc_push")

    def hook(self, edges, n, P, flags=0, stream=None):
        _check(self.lib.cc_hook(self._h, n, edges.shape[0], _dptr(edges, _ID), _dptr(P, _ID), flags,
                                _stream(stream)), "cc_hook")

    def hook_log(self, edges, n, P, log, count, flags=0, stream=None):
        """cc_hook_log: log (cap, 2) device tensor of P's dtype, count a device int64
        tensor of one element (the messages so far; appended to)."""
        if count.dtype != torch.int64 or count.numel() != 1:
            raise TypeError("count must be a one-element int64 tensor")
        _check(self.lib.cc_hook_log(self._h, n, edges.shape[0], _dptr(edges, _ID), _dptr(P, _ID),
                                    flags, _dptr(log, _ID), 0 if log is None else log.shape[0],
                                    _dptr(count, (torch.int64,)), _stream(stream)), "cc_hook_log")

    def hook_log_drain(self, edges, n, P, log, host_log, chunks=8, flags=0, stream=None):
        """cc_hook_log_drain: log (cap, 2) device tensor of P's dtype; host_log a
        (cap, 2) CPU tensor (pinned for overlap) of the same dtype, filled; returns
        the number of messages."""
        if host_log.device.type != "cpu" or host_log.dtype != log.dtype:
            raise TypeError("host_log must be a CPU tensor of the log's dtype")
        if not host_log.is_contiguous():
            raise ValueError("host_log must be contiguous")
        out = ctypes.c_uint64(0)
        rc = self.lib.cc_hook_log_drain(self._h, n, edges.shape[0], _dptr(edges, _ID), _dptr(P, _ID),
                                        flags, _dptr(log, _ID), log.shape[0], host_log.data_ptr(),
                                        host_log.shape[0], chunks, ctypes.byref(out), _stream(stream))
        _check(rc, "cc_hook_log_drain")
        return int(out.value)

    def compress(self, n, P, flags=0, stream=None):
        _check(self.lib.cc_compress(self._h, n, _dptr(P, _ID), flags, _stream(stream)), "cc_compress")

    def canon(self, n, L, stream=None):
        _check(self.lib.cc_canon(self._h, n, _dptr(L, _ID), _stream(stream)), "cc_canon")

    # exchange between edge shares
    def export(self, P, n, zroot=0xFFFFFFFF, pairs=None, zero_ids=None, stream=None):
        """cc_export: (n_pairs, n_zero). pairs: (cap, 2) and zero_ids: (cap,) device
        tensors of P's dtype, or None to only count (raises CCError(CC_ENOMEM) when
        a capacity is too small)."""
        npairs, nzero = ctypes.c_uint64(0), ctypes.c_uint64(0)
        pcap = 0 if pairs is None else pairs.shape[0]
        zcap = 0 if zero_ids is None else zero_ids.shape[0]
        rc = self.lib.cc_export(self._h, n, _dptr(P, _ID), zroot, _dptr(pairs, _ID), pcap,
                                _dptr(zero_ids, _ID), zcap, ctypes.byref(npairs),
                                ctypes.byref(nzero), _stream(stream))
        if rc != CC_OK and not (rc == CC_ENOMEM and pairs is None and zero_ids is None):
            _check(rc, "cc_export")
        return int(npairs.value), int(nzero.value)

    def export_lists(self, P, n, zroot=0xFFFFFFFF, stream=None):
        """Count, allocate and export: returns (pairs (k, 2), zero_ids (j,))."""
        npairs, nzero = self.export(P, n, zroot, stream=stream)
        pairs = torch.empty((npairs, 2), dtype=P.dtype, device=P.device)
        zero = torch.empty(nzero, dtype=P.dtype, device=P.device)
        self.export(P, n, zroot, pairs, zero, stream=stream)
        return pairs, zero

    def hook_ids(self, ids, target, n, P, flags=0, stream=None):
        """cc_hook_ids: every ids[i] is connected to target."""
        _check(self.lib.cc_hook_ids(self._h, n, ids.numel(), _dptr(ids, _ID), target, _dptr(P, _ID),
                                    flags, _stream(stream)), "cc_hook_ids")

    # compact IDs (Sec. V)
    def id_bytes(self, n) -> int:
        return int(self.lib.cc_id_bytes(n))

    def pack_ids(self, ids, id_bytes, out=None, stream=None):
        """cc_pack_ids: ids (any shape, P's dtype) -> uint8 tensor of ids.numel() * id_bytes."""
        if out is None:
            out = torch.empty(ids.numel() * id_bytes, dtype=torch.uint8, device=ids.device)
        if out.numel() < ids.numel() * id_bytes:
            raise ValueError("out is too small")
        _check(self.lib.cc_pack_ids(self._h, ids.numel(), _dptr(ids, _ID), id_bytes,
                                    _dptr(out, (torch.uint8,)), _stream(stream)), "cc_pack_ids")
        return out

    def unpack_ids(self, buf, count, id_bytes, out=None, stream=None):
        """cc_unpack_ids: the first count IDs of a packed uint8 tensor -> int32 tensor."""
        if buf.numel() < count * id_bytes:
            raise ValueError("buf is too small")
        if out is None:
            out = torch.empty(count, dtype=torch.int32, device=buf.device)
        _check(self.lib.cc_unpack_ids(self._h, count, _dptr(buf, (torch.uint8,)), id_bytes,
                                      _dptr(out, _ID), _stream(stream)), "cc_unpack_ids")
        return out

    # batch
    def batch_graph(self, vtx_off, edge_off, edges, L, status, stream=None):
        """cc_batch_graph_create: capture the batch once; BatchGraph.launch replays it."""
        h = ctypes.c_void_p()
        _check(self.lib.cc_batch_graph_create(self._h, vtx_off.numel() - 1,
                                              _dptr(vtx_off, (torch.int64,)),
                                              _dptr(edge_off, (torch.int64,)),
                                              _dptr(edges, (torch.int32,)), _dptr(L, (torch.int32,)),
                                              _dptr(status, (torch.int32,)), _stream(stream),
                                              ctypes.byref(h)), "cc_batch_graph_create")
        return BatchGraph(self, h, (vtx_off, edge_off, edges, L, status))

    def _batch_out(self, vtx_off, edges, L, status):
        G = vtx_off.numel() - 1
        if L is None:
            L = torch.empty(int(vtx_off[-1].item()), dtype=torch.int32, device=edges.device)
        if status is None:
            status = torch.empty(G, dtype=torch.int32, device=edges.device)
        return G, L, status

    def batch(self, vtx_off, edge_off, edges, L=None, status=None, stream=None, sched=None):
        """cc_batch (sched None: the context's choice) or cc_batch_ex with
        sched = (wave_max_n, multi_min_n) or a BatchSched."""
        G, L, status = self._batch_out(vtx_off, edges, L, status)
        args = (self._h, G, _dptr(vtx_off, (torch.int64,)), _dptr(edge_off, (torch.int64,)),
                _dptr(edges, (torch.int32,)), _dptr(L, (torch.int32,)),
                _dptr(status, (torch.int32,)))
        if sched is None:
            _check(self.lib.cc_batch(*args, _stream(stream)), "cc_batch")
        else:
            sc = sched if isinstance(sched, BatchSched) else BatchSched(*sched)
            _check(self.lib.cc_batch_ex(*args, ctypes.byref(sc), _stream(stream)), "cc_batch_ex")
        return L, status

    def batch_sched_force(self, sched=None):
        """cc_batch_sched_force: (wave_max_n, multi_min_n), a BatchSched, or None."""
        if sched is None:
            _check(self.lib.cc_batch_sched_force(self._h, None), "cc_batch_sched_force")
            return
        sc = sched if isinstance(sched, BatchSched) else BatchSched(*sched)
        _check(self.lib.cc_batch_sched_force(self._h, ctypes.byref(sc)), "cc_batch_sched_force")

    def batch_tune(self, vtx_off, edge_off, edges, L=None, status=None, reps=3, stream=None):
        """cc_batch_tune -> (TuneResult, L, status)."""
        G, L, status = self._batch_out(vtx_off, edges, L, status)
        r = TuneResult()
        _check(self.lib.cc_batch_tune(self._h, G, _dptr(vtx_off, (torch.int64,)),
                                      _dptr(edge_off, (torch.int64,)), _dptr(edges, (torch.int32,)),
                                      _dptr(L, (torch.int32,)), _dptr(status, (torch.int32,)),
                                      reps, ctypes.byref(r), _stream(stream)), "cc_batch_tune")
        return r, L, status


class BatchGraph:
    """A captured cc_batch (cc_batch_graph_*). Keeps the tensors it was captured
    with alive; launch() replays the batch on a stream."""

    def __init__(self, ctx, handle, keep):
        self.ctx = ctx
        self.lib = ctx.lib
        self._h = handle
        self._keep = keep

    def launch(self, stream=None):
        _check(self.lib.cc_batch_graph_launch(self._h, _stream(stream)), "cc_batch_graph_launch")

    def close(self):
        if self._h:
            self.lib.cc_batch_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Server:
    """cc_serve_*: continuous batching of CC requests held in host memory."""

    def __init__(self, ctx: Context, max_inflight=0, queue_capacity=0, streams=0, small_n=0,
                 hbm_budget=0, coalesce_us=0):
        self.ctx = ctx
        self.lib = ctx.lib
        o = _ServeOpts(max_inflight, queue_capacity, streams, small_n, hbm_budget, coalesce_us, 0)
        h = ctypes.c_void_p()
        _check(self.lib.cc_serve_open(ctx.handle, ctypes.byref(o), ctypes.byref(h)), "cc_serve_open")
        self._h = h
        self._keep = {}

    def submit(self, edges_host, n: int, L_host, flags: int = 0) -> int:
        """edges_host: numpy (m, 2) uint32 C-contiguous; L_host: numpy uint32[n] (written)."""
        import numpy as np
        assert edges_host.dtype == np.uint32 and edges_host.flags.c_contiguous
        assert L_host.dtype == np.uint32 and L_host.flags.c_contiguous and len(L_host) >= n
        t = ctypes.c_uint64(0)
        m = edges_host.shape[0]
        rc = self.lib.cc_serve_submit(self._h, n, m, edges_host.ctypes.data if m else None,
                                      L_host.ctypes.data if n else None, flags, ctypes.byref(t))
        if rc != CC_OK:
            raise CCError(rc, "cc_serve_submit")
        self._keep[t.value] = (edges_host, L_host)
        return t.value

    def wait(self, ticket: int, timeout_us: int = -1):
        st = ReqStats()
        rc = self.lib.cc_serve_wait(self._h, ticket, timeout_us, ctypes.byref(st))
        if rc != CC_ETIMEDOUT:
            self._keep.pop(ticket, None)
        return rc, st

    def close(self):
        if self._h:
            _check(self.lib.cc_serve_close(self._h), "cc_serve_close")
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
