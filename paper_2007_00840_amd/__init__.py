"""Python binding of the gfx950 symbolic LU factorisation library.

Thin ctypes marshalling over ``libgsofa.so`` (C ABI in ``include/gsofa.h``):
the same entry points (``symbolic``, ``batch``, ``Server`` for
``gsofa_serve_*``), numpy arrays or device tensors in, numpy arrays (or
device-resident results) out. Every step of the computation runs in the HIP
library; there is no CPU fallback -- importing fails loudly when the library
has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsofa.so")

OK, EINVAL, ENOMEM, EDEVICE, EAGAIN, ECAPACITY, ENOTFOUND = range(7)
NO_SUPERNODES = 0x1
L_CSR = 0x2
RESULT_ON_DEVICE = 0x4
INPUT_ON_DEVICE = 0x8
NO_LINE95 = 0x10
LEVEL_ORDER = 0x20
MAP_WAVE32 = 0x40
MAP_WG8 = 0x80
MAP_WG16 = 0x100
EAGER = 0x200
MAP_BYTE = 0x800
MAP_WAVE32_7 = 0x1000
TUNE_NOW = 0x400
NO_TUNE = 0x2000
BUDGET_MODE = 0x4000
MAP_THREAD = 0x8000
RESET_LABELS = 0x10000
SERVE_YIELD = 0x20000

EXPORTED = ["gsofa_symbolic", "gsofa_batch", "gsofa_serve_open", "gsofa_serve_submit",
            "gsofa_serve_poll", "gsofa_serve_close", "gsofa_result_free", "gsofa_strerror",
            "gsofa_release_cache", "gsofa_graph_counters", "gsofa_memory_counters",
            "gsofa_symbolic_noalloc"]
NOALLOC_SCRATCH_BYTES = 128 << 20
MAX_N = (1 << 30) - 1  # largest supported matrix order


class GsofaError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})" if what else f"{strerror(code)} ({code})")


class Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("concurrent_sources", ctypes.c_int32),
                ("iterations", ctypes.c_uint64), ("windows", ctypes.c_uint64),
                ("edges_alg", ctypes.c_uint64), ("edges_gpu", ctypes.c_uint64),
                ("peak_device_bytes", ctypes.c_uint64), ("t_traverse_ms", ctypes.c_double),
                ("t_emit_ms", ctypes.c_double), ("t_supernode_ms", ctypes.c_double),
                ("t_total_ms", ctypes.c_double), ("window", ctypes.c_int32),
                ("mapping", ctypes.c_int32), ("t_tune_ms", ctypes.c_double),
                ("spilled_entries", ctypes.c_uint64), ("launches", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Opts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("max_supernode", ctypes.c_int32),
                ("mem_budget_bytes", ctypes.c_int64), ("flags", ctypes.c_uint32),
                ("window", ctypes.c_int32), ("concurrent_sources", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("dev_alloc", ALLOC_FN),
                ("dev_free", FREE_FN), ("alloc_ctx", ctypes.c_void_p),
                ("queue_cap", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class Counts(ctypes.Structure):
    _fields_ = [("nnz_a", ctypes.c_int64), ("nnz_l", ctypes.c_int64), ("nnz_u", ctypes.c_int64),
                ("fills", ctypes.c_int64), ("nsuper", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("scratch_bytes", ctypes.c_int64), ("stats", Stats)]


class Result(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz_a", ctypes.c_int64), ("nnz_l", ctypes.c_int64),
                ("nnz_u", ctypes.c_int64), ("fills", ctypes.c_int64),
                ("l_ptr", ctypes.c_void_p), ("l_idx", ctypes.c_void_p),
                ("u_ptr", ctypes.c_void_p), ("u_idx", ctypes.c_void_p),
                ("nsuper", ctypes.c_int32), ("xsup", ctypes.c_void_p), ("supno", ctypes.c_void_p),
                ("flags", ctypes.c_uint32), ("stats", Stats), ("internal_", ctypes.c_void_p)]


_lib = None


def load():
    """Load the built library; raises if it is missing (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "or python -m paper_2007_00840_amd._build")
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        lib.gsofa_symbolic.restype = ctypes.c_int
        lib.gsofa_symbolic.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                       P(Opts), P(P(Result))]
        lib.gsofa_batch.restype = ctypes.c_int
        lib.gsofa_batch.argtypes = [ctypes.c_int32, P(Csr), P(Opts), P(P(Result))]
        lib.gsofa_serve_open.restype = ctypes.c_int
        lib.gsofa_serve_open.argtypes = [P(Opts), ctypes.c_int32, P(ctypes.c_void_p)]
        lib.gsofa_serve_submit.restype = ctypes.c_int
        lib.gsofa_serve_submit.argtypes = [ctypes.c_void_p, P(Csr), P(ctypes.c_uint64)]
        lib.gsofa_serve_poll.restype = ctypes.c_int
        lib.gsofa_serve_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32,
                                         P(P(Result))]
        lib.gsofa_serve_close.restype = ctypes.c_int
        lib.gsofa_serve_close.argtypes = [ctypes.c_void_p]
        lib.gsofa_result_free.restype = None
        lib.gsofa_result_free.argtypes = [P(Result)]
        lib.gsofa_strerror.restype = ctypes.c_char_p
        lib.gsofa_strerror.argtypes = [ctypes.c_int]
        lib.gsofa_release_cache.restype = ctypes.c_int
        lib.gsofa_release_cache.argtypes = []
        lib.gsofa_graph_counters.restype = ctypes.c_int
        lib.gsofa_graph_counters.argtypes = [ctypes.POINTER(ctypes.c_uint64)]
        lib.gsofa_symbolic_noalloc.restype = ctypes.c_int
        lib.gsofa_symbolic_noalloc.argtypes = [
            ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, P(Opts),
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_void_p, P(Counts)]
        lib.gsofa_memory_counters.restype = ctypes.c_int
        lib.gsofa_memory_counters.argtypes = [ctypes.POINTER(ctypes.c_uint64)]
        _lib = lib
    return _lib


def strerror(code: int) -> str:
    try:
        return load().gsofa_strerror(int(code)).decode()
    except ImportError:
        return f"status {code}"


class TorchAllocator:
    """Device memory for the library from torch's caching allocator (the
    gsofa_opts dev_alloc / dev_free hooks). Each block is a uint8 tensor kept
    alive until the library frees it; counts what went through it."""

    def __init__(self, device=None):
        import torch
        self._torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        self.live = {}
        self.bytes = 0
        self.allocs = 0
        self.frees = 0
        self.peak_live_bytes = 0
        self._live_bytes = 0

        def _alloc(nbytes, ctx):
            try:
                t = self._torch.empty(int(nbytes), dtype=self._torch.uint8, device=self.device)
            except RuntimeError:
                return None
            p = t.data_ptr()
            self.live[p] = t
            self.bytes += int(nbytes)
            self.allocs += 1
            self._live_bytes += int(nbytes)
            self.peak_live_bytes = max(self.peak_live_bytes, self._live_bytes)
            return p

        def _free(ptr, ctx):
            t = self.live.pop(ptr, None)
            if t is not None:
                self._live_bytes -= t.numel()
            self.frees += 1

        # the ctypes callbacks must outlive every call and result that uses them
        self.alloc_fn = ALLOC_FN(_alloc)
        self.free_fn = FREE_FN(_free)

    def install(self, o: Opts):
        o.dev_alloc = self.alloc_fn
        o.dev_free = self.free_fn
        o.alloc_ctx = None


def make_opts(flags=0, max_supernode=0, mem_budget_bytes=0, window=0,
              concurrent_sources=0, stream=None, allocator=None, queue_cap=0) -> Opts:
    o = Opts()
    o.struct_size = ctypes.sizeof(Opts)
    o.max_supernode = int(max_supernode)
    o.mem_budget_bytes = int(mem_budget_bytes)
    o.flags = int(flags)
    o.window = int(window)
    o.concurrent_sources = int(concurrent_sources)
    o.stream = stream
    o.queue_cap = int(queue_cap)
    if allocator is not None:
        allocator.install(o)
    return o


@dataclass
class SymbolicResult:
    """A host gsofa_result: its arrays are numpy views of the library's result
    memory (page-locked where available), released when the last view is gone.
    The results of one batch call share one block, released with the last of
    them."""
    n: int
    nnz_a: int
    nnz_l: int
    nnz_u: int
    fills: int
    l_ptr: np.ndarray
    l_idx: np.ndarray
    u_ptr: np.ndarray
    u_idx: np.ndarray
    nsuper: int
    xsup: np.ndarray | None
    supno: np.ndarray | None
    flags: int
    stats: dict


class _Hold:
    """Owns a library host result while numpy arrays view its memory (a copy of
    a 64^3 stencil's 1.6 GB of indices would hold the interpreter for 0.1 s)."""

    __slots__ = ("_rp", "_free")

    def __init__(self, rp, free):
        self._rp = rp
        self._free = free

    def __del__(self):
        try:
            self._free(self._rp)
        except Exception:
            pass


def _np_view(ptr, count, dtype, hold):
    if count <= 0 or not ptr:
        return np.zeros(max(count, 0), dtype=dtype)
    ct = np.ctypeslib.as_ctypes_type(np.dtype(dtype))
    buf = (ct * count).from_address(ptr)
    buf._hold = hold  # the array's base keeps the result alive
    return np.frombuffer(buf, dtype=dtype)


def _stats(r: Result) -> dict:
    s = r.stats
    return {f: getattr(s, f) for f, _ in Stats._fields_}


def _to_host(rp, lib) -> SymbolicResult:
    """Takes ownership of the library result rp (freed with the last array)."""
    hold = _Hold(rp, lib.gsofa_result_free)
    r = rp.contents
    n = r.n
    has_sn = bool(r.xsup)
    return SymbolicResult(
        n=n, nnz_a=r.nnz_a, nnz_l=r.nnz_l, nnz_u=r.nnz_u, fills=r.fills,
        l_ptr=_np_view(r.l_ptr, n + 1, np.int64, hold), l_idx=_np_view(r.l_idx, r.nnz_l, np.int32, hold),
        u_ptr=_np_view(r.u_ptr, n + 1, np.int64, hold), u_idx=_np_view(r.u_idx, r.nnz_u, np.int32, hold),
        nsuper=r.nsuper,
        xsup=_np_view(r.xsup, r.nsuper + 1, np.int32, hold) if has_sn else None,
        supno=_np_view(r.supno, n, np.int32, hold) if has_sn else None,
        flags=r.flags, stats=_stats(r))


class DeviceResult:
    """A result whose arrays stay in device memory (RESULT_ON_DEVICE).
    Holds the library result until ``free()``."""

    def __init__(self, rp):
        self._rp = rp
        r = rp.contents
        self.n, self.nnz_l, self.nnz_u, self.nsuper = r.n, r.nnz_l, r.nnz_u, r.nsuper
        self.fills = r.fills
        # the statistics are copied as they are and turned into a dict on first
        # use (a batch returns thousands of results); they outlive free()
        self._st = Stats.from_buffer_copy(r.stats)
        self._stats = None

    @property
    def stats(self) -> dict:
        if self._stats is None:
            self._stats = {f: getattr(self._st, f) for f, _ in Stats._fields_}
        return self._stats

    @property
    def ptrs(self) -> dict:
        """Device addresses of the result arrays (valid until free())."""
        if self._rp is None:
            raise ValueError("result already freed")
        r = self._rp.contents
        return {k: getattr(r, k) for k in ("l_ptr", "l_idx", "u_ptr", "u_idx", "xsup", "supno")}

    def to_torch(self, device="cuda"):
        """Copy the device arrays into torch tensors (device to device)."""
        import torch
        out = {}
        ptrs = self.ptrs
        sizes = {"l_ptr": (self.n + 1, torch.int64), "u_ptr": (self.n + 1, torch.int64),
                 "l_idx": (self.nnz_l, torch.int32), "u_idx": (self.nnz_u, torch.int32),
                 "xsup": (self.nsuper + 1, torch.int32), "supno": (self.n, torch.int32)}
        for k, (cnt, dt) in sizes.items():
            t = torch.empty(max(cnt, 0), dtype=dt, device=device)
            p = ptrs[k]
            if cnt > 0 and p:
                _d2d(t.data_ptr(), p, t.numel() * t.element_size())
            out[k] = t
        return out

    def free(self):
        if self._rp is not None:
            load().gsofa_result_free(self._rp)
            self._rp = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _d2d(dst, src, nbytes):
    import torch
    torch.cuda.synchronize()
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.restype = ctypes.c_int
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    rc = hip.hipMemcpy(ctypes.c_void_p(dst), ctypes.c_void_p(src), ctypes.c_size_t(nbytes), 3)
    if rc != 0:
        raise GsofaError(EDEVICE, "hipMemcpy")


_torch = None


def _torch_mod():
    global _torch
    if _torch is None:
        try:
            import torch
            _torch = torch
        except ImportError:  # pragma: no cover
            _torch = False
    return _torch


def _arr_ptr(a):
    """(pointer, keepalive, on_device) of a numpy array or a torch tensor."""
    if isinstance(a, np.ndarray) and a.dtype == np.int32 and a.flags.c_contiguous:
        return a.ctypes.data, a, False
    torch = _torch_mod()
    if torch and isinstance(a, torch.Tensor):
        if a.dtype != torch.int32 or not a.is_contiguous():
            raise TypeError("CSR tensors must be contiguous int32")
        return a.data_ptr(), a, a.is_cuda
    arr = np.ascontiguousarray(a, dtype=np.int32)
    return arr.ctypes.data, arr, False


def symbolic(n, row_ptr, col_idx, flags=0, max_supernode=0, mem_budget_bytes=0, window=0,
             concurrent_sources=0, stream=None, allocator=None, queue_cap=0):
    """gsofa_symbolic. Host numpy arrays or device int32 tensors (then the
    INPUT_ON_DEVICE flag is set). Returns SymbolicResult, or DeviceResult with
    RESULT_ON_DEVICE."""
    lib = load()
    rp_p, rp_keep, rp_dev = _arr_ptr(row_ptr)
    ci_p, ci_keep, ci_dev = _arr_ptr(col_idx)
    if rp_dev != ci_dev:
        raise ValueError("row_ptr and col_idx must both be host or both be device arrays")
    if rp_dev:
        flags |= INPUT_ON_DEVICE
    o = make_opts(flags, max_supernode, mem_budget_bytes, window, concurrent_sources, stream,
                  allocator, queue_cap)
    out = ctypes.POINTER(Result)()
    rc = lib.gsofa_symbolic(int(n), rp_p, ci_p, ctypes.byref(o), ctypes.byref(out))
    del rp_keep, ci_keep
    if rc != OK:
        raise GsofaError(rc, "gsofa_symbolic")
    if flags & RESULT_ON_DEVICE:
        return DeviceResult(out)
    return _to_host(out, lib)


def batch(mats, flags=0, max_supernode=0, mem_budget_bytes=0, window=0,
          concurrent_sources=0, stream=None, raise_on_error=True, allocator=None, queue_cap=0):
    """gsofa_batch over a list of (n, row_ptr, col_idx). Returns a list of
    SymbolicResult (or DeviceResult), with None where a matrix failed when
    raise_on_error is False."""
    lib = load()
    count = len(mats)
    arr = (Csr * max(count, 1))()
    keep = []
    on_dev = None
    for i, (n, rp, ci) in enumerate(mats):
        rp_p, k1, d1 = _arr_ptr(rp)
        ci_p, k2, d2 = _arr_ptr(ci)
        if d1 != d2 or (on_dev is not None and on_dev != d1):
            raise ValueError("mixed host and device inputs")
        on_dev = d1
        keep += [k1, k2]
        arr[i].n = int(n)
        arr[i].row_ptr = rp_p
        arr[i].col_idx = ci_p
    if on_dev:
        flags |= INPUT_ON_DEVICE
    o = make_opts(flags, max_supernode, mem_budget_bytes, window, concurrent_sources, stream,
                  allocator, queue_cap)
    outs = (ctypes.POINTER(Result) * max(count, 1))()
    rc = lib.gsofa_batch(count, arr, ctypes.byref(o), outs)
    del keep
    if count == 0:
        return []
    results = []
    first_err = None
    for i in range(count):
        p = outs[i]
        if not p:
            results.append(None)
            continue
        st = p.contents.stats.status
        if st != OK:
            first_err = first_err or st
            results.append(None)
            lib.gsofa_result_free(p)
        elif flags & RESULT_ON_DEVICE:
            results.append(DeviceResult(p))
        else:
            results.append(_to_host(p, lib))
    if rc != OK and raise_on_error:
        for r in results:
            if isinstance(r, DeviceResult):
                r.free()
        raise GsofaError(rc, "gsofa_batch")
    return results


def _dptr(t):
    """Device pointer of a contiguous torch tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("no-allocation arrays must be contiguous device tensors")
    return t.data_ptr()


def symbolic_noalloc(n, row_ptr, col_idx, u_ptr, u_idx, l_ptr, l_idx, xsup=None, supno=None,
                     flags=0, max_supernode=0, window=0, concurrent_sources=0, stream=None):
    """gsofa_symbolic_noalloc: device int32 CSR in, results written into the
    caller's device tensors (u_ptr/l_ptr int64 [n+1], u_idx/l_idx int32 with
    their lengths as capacities, xsup int32 [n+1], supno int32 [n]); no device
    allocation. Returns the counts as a dict; raises GsofaError (with
    ``.counts`` set on ECAPACITY)."""
    import torch
    for name, t, dt in (("row_ptr", row_ptr, torch.int32), ("col_idx", col_idx, torch.int32),
                        ("u_ptr", u_ptr, torch.int64), ("l_ptr", l_ptr, torch.int64),
                        ("u_idx", u_idx, torch.int32), ("l_idx", l_idx, torch.int32),
                        ("xsup", xsup, torch.int32), ("supno", supno, torch.int32)):
        if t is not None and t.dtype != dt:
            raise TypeError(f"{name} must be {dt}")
    o = make_opts(flags | INPUT_ON_DEVICE, max_supernode, 0, window, concurrent_sources, stream)
    c = Counts()
    rc = load().gsofa_symbolic_noalloc(
        int(n), _dptr(row_ptr), _dptr(col_idx), ctypes.byref(o),
        _dptr(u_ptr), _dptr(u_idx), int(u_idx.numel()),
        _dptr(l_ptr), _dptr(l_idx), int(l_idx.numel()),
        _dptr(xsup), _dptr(supno), ctypes.byref(c))
    out = {f: getattr(c, f) for f, _ in Counts._fields_ if f not in ("stats", "pad_")}
    out["stats"] = {f: getattr(c.stats, f) for f, _ in Stats._fields_}
    if rc != OK:
        err = GsofaError(rc, "gsofa_symbolic_noalloc")
        err.counts = out if rc == ECAPACITY else None
        raise err
    return out


class Server:
    """gsofa_serve_open / submit / poll / close."""

    def __init__(self, max_inflight=4, flags=0, max_supernode=0, mem_budget_bytes=0,
                 window=0, concurrent_sources=0, allocator=None, queue_cap=0):
        self._lib = load()
        self._allocator = allocator  # its callbacks must outlive the server
        o = make_opts(flags, max_supernode, mem_budget_bytes, window, concurrent_sources, None,
                      allocator, queue_cap)
        self._h = ctypes.c_void_p()
        rc = self._lib.gsofa_serve_open(ctypes.byref(o), int(max_inflight), ctypes.byref(self._h))
        if rc != OK:
            raise GsofaError(rc, "gsofa_serve_open")
        self.flags = flags

    def submit(self, n, row_ptr, col_idx) -> int:
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        m = Csr(int(n), rp.ctypes.data, ci.ctypes.data)
        t = ctypes.c_uint64()
        rc = self._lib.gsofa_serve_submit(self._h, ctypes.byref(m), ctypes.byref(t))
        if rc != OK:
            raise GsofaError(rc, "gsofa_serve_submit")
        return int(t.value)

    def poll(self, ticket, timeout_us=0):
        """Returns a SymbolicResult, or None while the request is not done
        (EAGAIN). Other statuses raise."""
        out = ctypes.POINTER(Result)()
        rc = self._lib.gsofa_serve_poll(self._h, ctypes.c_uint64(ticket), int(timeout_us),
                                        ctypes.byref(out))
        if rc == EAGAIN:
            return None
        if rc != OK:
            raise GsofaError(rc, "gsofa_serve_poll")
        return _to_host(out, self._lib)

    def close(self):
        if self._h:
            self._lib.gsofa_serve_close(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def release_cache():
    return load().gsofa_release_cache()


def memory_counters():
    """(bytes held from the library's own hipMalloc, its hipMalloc calls, bytes
    from caller allocators, dev_alloc calls, dev_free calls) since load."""
    out = (ctypes.c_uint64 * 5)()
    rc = load().gsofa_memory_counters(out)
    if rc != OK:
        raise GsofaError(rc, "gsofa_memory_counters")
    return tuple(int(x) for x in out)


def graph_counters():
    """(instantiated, updated in place, launched) executable HIP graphs since load."""
    out = (ctypes.c_uint64 * 3)()
    rc = load().gsofa_graph_counters(out)
    if rc != OK:
        raise GsofaError(rc, "gsofa_graph_counters")
    return tuple(int(x) for x in out)
