"""Seeded synthetic stencil matrices: the inputs every test and benchmark uses.

The paper evaluates on SuiteSparse matrices preprocessed with a fill-reducing
ordering and stored as CSR (evaluation section, dataset table). None of those
matrices ship here; these generated grid stencils stand in for them:

* ``config(1)`` .. ``config(3)``: the plain single-matrix workloads
  (40x40 5-point natural order; 1000x1000 9-point ND; 64^3 27-point ND),
* ``batch_member(k)``: member k of the 4,096-matrix batch,
* ``serve_request(r)``: request r of the Poisson request stream.

This module holds no part of the symbolic factorisation. It only builds
inputs (``row_ptr``, ``col_idx`` as int32 numpy arrays, columns sorted
within each row, diagonal always present).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stencil.c")
_LIB = os.path.join(_HERE, "libsynth.so")

DROP_02 = 858993459  # floor(0.2 * 2**32)
STENCIL_POINTS = {5: 4, 9: 8, 7: 6, 27: 26}


def build(force: bool = True) -> str:
    """Compile the generator with gcc into ``synth/libsynth.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-Wall",
                        "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.synth_sm64.restype = ctypes.c_uint64
        lib.synth_sm64.argtypes = [ctypes.c_uint64]
        lib.synth_stencil.restype = ctypes.c_int64
        lib.synth_stencil.argtypes = [ctypes.c_int, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_int, ctypes.c_uint64,
                                      ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
        lib.synth_order.restype = ctypes.c_int
        lib.synth_order.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int, ctypes.c_void_p]
        lib.synth_band_extras.restype = ctypes.c_int64
        lib.synth_band_extras.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32,
                                          ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def sm64(x: int) -> int:
    """SplitMix64 output function of x (counter-based hash)."""
    return int(_load().synth_sm64(ctypes.c_uint64(x & 0xFFFFFFFFFFFFFFFF)))


@dataclass
class Matrix:
    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col_idx: np.ndarray  # int32[nnz]
    desc: str

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


def order(nx: int, ny: int, nz: int, nd: bool) -> np.ndarray:
    """rank[natural id] -> position in the chosen ordering."""
    rank = np.empty(nx * ny * nz, dtype=np.int32)
    rc = _load().synth_order(nx, ny, nz, 1 if nd else 0, rank.ctypes.data)
    if rc != 0:
        raise ValueError(f"synth_order failed ({rc})")
    return rank


def stencil(kind: int, dims, nd: bool, seed: int, drop_thresh: int = DROP_02) -> Matrix:
    """Stencil matrix of ``kind`` in {5, 9, 7, 27} on a grid of ``dims``."""
    dims = tuple(int(d) for d in dims)
    if len(dims) == 2:
        dims = dims + (1,)
    nx, ny, nz = dims
    n = nx * ny * nz
    cap = n * (STENCIL_POINTS[kind] + 1)
    row_ptr = np.empty(n + 1, dtype=np.int32)
    col = np.empty(cap, dtype=np.int32)
    nnz = _load().synth_stencil(kind, nx, ny, nz, 1 if nd else 0,
                                ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF),
                                ctypes.c_uint32(drop_thresh),
                                row_ptr.ctypes.data, col.ctypes.data)
    if nnz < 0:
        raise ValueError(f"synth_stencil failed ({nnz})")
    desc = f"{kind}pt {'x'.join(map(str, dims if nz > 1 else dims[:2]))} " \
           f"{'nd' if nd else 'natural'} seed={seed} drop={drop_thresh}"
    return Matrix(n, row_ptr, col[:nnz].copy(), desc)


def band_extras(m: Matrix, draws: int, seed: int, bw: int = 32) -> Matrix:
    """Add up to ``draws`` random entries (i, i +- d), 1 <= d <= bw."""
    out_rp = np.empty(m.n + 1, dtype=np.int32)
    out_col = np.empty(m.nnz + max(draws, 0), dtype=np.int32)
    nnz = _load().synth_band_extras(m.n, m.row_ptr.ctypes.data, m.col_idx.ctypes.data,
                                    int(draws), ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF),
                                    int(bw), out_rp.ctypes.data, out_col.ctypes.data)
    if nnz < 0:
        raise ValueError("synth_band_extras failed")
    return Matrix(m.n, out_rp, out_col[:nnz].copy(), m.desc + f" +extras({draws},bw={bw})")


def _isqrt(v: int) -> int:
    return math.isqrt(v)


def _icbrt(v: int) -> int:
    a = int(round(v ** (1.0 / 3.0)))
    while a * a * a > v:
        a -= 1
    while (a + 1) ** 3 <= v:
        a += 1
    return a


def grid_2d(n: int):
    a = _isqrt(n)
    return a, n // a


def grid_3d(n: int):
    a = _icbrt(n)
    b = _isqrt(n // a)
    c = n // (a * b)
    return a, b, c


# ---- the five workloads -------------------------------------------------

def config(i: int) -> Matrix:
    """The plain single-matrix workloads 1..3 (seeds 1..3)."""
    if i == 1:
        return stencil(5, (40, 40), nd=False, seed=1)
    if i == 2:
        return stencil(9, (1000, 1000), nd=True, seed=2)
    if i == 3:
        return stencil(27, (64, 64, 64), nd=True, seed=3)
    raise ValueError(i)


BATCH_COUNT = 4096
BATCH_SEED = 4


def batch_member(k: int, seed: int = BATCH_SEED) -> Matrix:
    """Member k of the batch: n ~ U[200, 5000]; even k 2D 5-point, odd k 3D
    7-point; ND order; drop 0.2; then floor(0.10 * nnz_offdiag) band draws
    (bandwidth 32) in the final ordering."""
    sk = sm64((seed << 32) + k)
    n_req = 200 + (sk >> 32) % 4801
    if k % 2 == 0:
        m = stencil(5, grid_2d(n_req), nd=True, seed=sk)
    else:
        m = stencil(7, grid_3d(n_req), nd=True, seed=sk)
    offdiag = m.nnz - m.n
    return band_extras(m, offdiag // 10, seed=sk, bw=32)


SERVE_SEED = 5
SERVE_RATE = 200.0
SERVE_SECONDS = 60.0


@dataclass
class Request:
    rid: int
    arrival_s: float
    n_req: int
    kind: int
    seed: int

    def matrix(self) -> Matrix:
        if self.kind == 9:
            return stencil(9, grid_2d(self.n_req), nd=True, seed=self.seed)
        return stencil(27, grid_3d(self.n_req), nd=True, seed=self.seed)


def _unit(h: int) -> float:
    return (h >> 11) * (1.0 / 9007199254740992.0)


def serve_trace(count: int | None = None, seed: int = SERVE_SEED,
                rate: float = SERVE_RATE, seconds: float = SERVE_SECONDS):
    """Poisson arrivals (exponential gaps, mean 1/rate) up to ``seconds``
    (or the first ``count`` requests). Request r: n = round(10**(3 + 3u)),
    2D 9-point or 3D 27-point by a coin flip, ND order, drop 0.2."""
    out = []
    t = 0.0
    r = 0
    base = sm64(seed << 32)
    while True:
        h = sm64(base ^ sm64(r))
        gap = -math.log(1.0 - _unit(sm64(h + 1))) / rate
        t += gap
        if count is None and t > seconds:
            break
        if count is not None and r >= count:
            break
        u = _unit(h)
        n_req = int(round(10.0 ** (3.0 + 3.0 * u)))
        kind = 27 if (sm64(h + 2) & 1) else 9
        out.append(Request(r, t, n_req, kind, sm64(h + 3)))
        r += 1
    return out


def fingerprint(m: Matrix) -> str:
    import hashlib
    h = hashlib.sha256()
    h.update(np.int64(m.n).tobytes())
    h.update(np.ascontiguousarray(m.row_ptr, dtype=np.int32).tobytes())
    h.update(np.ascontiguousarray(m.col_idx, dtype=np.int32).tobytes())
    return h.hexdigest()
