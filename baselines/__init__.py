"""CPU comparison baseline (not the oracle, not the product): the
Gilbert-Peierls column-by-column symbolic factorisation, timed beside the GPU
path. ``bench.py`` times it; ``tests/test_baselines.py`` checks it against the
oracle. It shares no code with the GPU library or the oracle."""
from __future__ import annotations

import ctypes
import os
import subprocess
import time
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gilbert_peierls.c")
_LIB = os.path.join(_HERE, "libbaselines.so")


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_CLOCK = ctypes.CFUNCTYPE(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        lib.gp_symbolic.restype = ctypes.c_int
        lib.gp_symbolic.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                    P(ctypes.c_void_p), P(ctypes.c_void_p), P(ctypes.c_void_p),
                                    P(ctypes.c_void_p), P(ctypes.c_int64), _CLOCK, ctypes.c_double,
                                    P(ctypes.c_int32)]
        lib.gp_free.restype = None
        lib.gp_free.argtypes = [ctypes.c_void_p]
        _lib = lib
    return _lib


@dataclass
class GPResult:
    n: int
    l_ptr: np.ndarray   # CSC of strict L
    l_idx: np.ndarray
    u_ptr: np.ndarray   # CSC of U (diagonal included)
    u_idx: np.ndarray
    edges: int          # L entries the searches scanned
    cols_done: int
    seconds: float      # the factorisation itself (not the input transpose)


def _csc_of(n, row_ptr, col_idx):
    rp = np.asarray(row_ptr, dtype=np.int64)
    ci = np.asarray(col_idx, dtype=np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int32), np.diff(rp))
    order = np.argsort(ci, kind="stable")
    cp = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(np.bincount(ci, minlength=n), out=cp[1:])
    return cp, np.ascontiguousarray(rows[order], dtype=np.int32)


def _arr(ptr, count, dtype):
    if count <= 0:
        return np.zeros(0, dtype=dtype)
    ct = np.ctypeslib.as_ctypes_type(np.dtype(dtype))
    return np.frombuffer((ct * count).from_address(ptr), dtype=dtype).copy()


_clock_cb = _CLOCK(time.perf_counter)


def gilbert_peierls(n, row_ptr, col_idx, time_limit_s: float = 0.0) -> GPResult:
    """Symbolic factorisation of the CSR pattern by Gilbert-Peierls (one
    thread). With time_limit_s > 0 it stops after the column where the limit
    passed (cols_done < n)."""
    lib = _load()
    cp, ri = _csc_of(n, row_ptr, col_idx)
    lp, li, up, ui = (ctypes.c_void_p() for _ in range(4))
    edges = ctypes.c_int64()
    done = ctypes.c_int32()
    t0 = time.perf_counter()
    rc = lib.gp_symbolic(int(n), cp.ctypes.data, ri.ctypes.data if len(ri) else None,
                         ctypes.byref(lp), ctypes.byref(li), ctypes.byref(up), ctypes.byref(ui),
                         ctypes.byref(edges), _clock_cb, float(time_limit_s), ctypes.byref(done))
    secs = time.perf_counter() - t0
    if rc != 0:
        raise MemoryError("gp_symbolic failed")
    l_ptr = _arr(lp.value, n + 1, np.int64)
    u_ptr = _arr(up.value, n + 1, np.int64)
    res = GPResult(n, l_ptr, _arr(li.value, int(l_ptr[-1]) if n else 0, np.int32), u_ptr,
                   _arr(ui.value, int(u_ptr[-1]) if n else 0, np.int32), int(edges.value),
                   int(done.value), secs)
    for p in (lp, li, up, ui):
        lib.gp_free(p)
    return res
