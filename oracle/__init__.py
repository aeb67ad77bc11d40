"""CPU ORACLE for sparse symbolic LU factorisation -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import this package. The GPU library never imports, links or calls
it, and it shares no code with the GPU path.

Contents (all exact, integer-only):

* ``symbolic``      -- O1, the fill2 threshold search in plain C, one thread
                        per row (fill-path theorem; fill2 description in the
                        Background section). Returns U in CSR, L in CSR and
                        in CSC, supernodes and per-row algorithmic edges.
* ``ge_filled``     -- O2, structural Gaussian elimination on a 0/1 matrix
                        (no pivoting, no cancellation): the plain definition
                        of the filled pattern (Background, symbolic
                        factorisation paragraph).
* ``path_filled``   -- O3, the fill-path theorem written out: for each pair
                        (i, j) a search that only passes through vertices
                        smaller than min(i, j).
* ``supernodes``    -- S1, Definition T3 per block of max_supernode rows (C).
* ``supernodes_structural`` -- S2, an equivalent form used as a pin:
                        s joins r's supernode iff L(s, r) != 0 and
                        U(s,:) == U(s-1,:) minus {s-1}.
* ``trace``         -- plain simulation of the paper's level-by-level
                        fine-grained traversal (Section 4) for worked examples.

Parity status: every function here is pinned by tests in
``tests/test_oracle_*.py`` (worked examples, closed forms, brute force,
transpose duality); none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from collections import deque
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gsofa_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-Wall",
                        "-pthread", "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_rows.restype = ctypes.c_int
        lib.oracle_rows.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_int32, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.POINTER(ctypes.c_void_p)]
        lib.oracle_free.restype = None
        lib.oracle_free.argtypes = [ctypes.c_void_p]
        lib.oracle_transpose.restype = ctypes.c_int
        lib.oracle_transpose.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_supernodes.restype = ctypes.c_int32
        lib.oracle_supernodes.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def rows_struct(n, row_ptr, col_idx, rows=None, threads=None):
    """O1 on the given rows (all rows if None).

    Returns (cnt, lcnt, edges, ptr, entries): per requested row the structure
    size, |L| part, algorithmic edge count, and the concatenated sorted
    structures with int64 offsets ``ptr``.
    """
    lib = _load()
    row_ptr = _i32(row_ptr)
    col_idx = _i32(col_idx)
    if rows is None:
        nrows = n
        rows_p = None
    else:
        rows = _i32(rows)
        nrows = len(rows)
        rows_p = rows.ctypes.data
    cnt = np.zeros(nrows, dtype=np.int64)
    lcnt = np.zeros(nrows, dtype=np.int64)
    edges = np.zeros(nrows, dtype=np.int64)
    out = ctypes.c_void_p()
    rc = lib.oracle_rows(int(n), row_ptr.ctypes.data, col_idx.ctypes.data, rows_p,
                         int(nrows), int(threads or default_threads()),
                         cnt.ctypes.data, lcnt.ctypes.data, edges.ctypes.data,
                         ctypes.byref(out))
    if rc != 0:
        raise MemoryError("oracle_rows failed")
    total = int(cnt.sum())
    ptr = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(cnt, out=ptr[1:])
    if total:
        buf = (ctypes.c_int32 * total).from_address(out.value)
        entries = np.frombuffer(buf, dtype=np.int32).copy()
    else:
        entries = np.zeros(0, dtype=np.int32)
    lib.oracle_free(out)
    return cnt, lcnt, edges, ptr, entries


@dataclass
class Symbolic:
    n: int
    u_ptr: np.ndarray    # int64[n+1]  CSR of U (diagonal included)
    u_idx: np.ndarray    # int32       columns ascending
    l_rptr: np.ndarray   # int64[n+1]  CSR of strict L
    l_ridx: np.ndarray   # int32       columns ascending
    l_ptr: np.ndarray    # int64[n+1]  CSC of strict L
    l_idx: np.ndarray    # int32       rows ascending
    edges: np.ndarray    # int64[n]    algorithmic edges per row
    nnz_a: int
    xsup: np.ndarray | None = None
    supno: np.ndarray | None = None

    @property
    def nnz_l(self):
        return int(self.l_ptr[-1])

    @property
    def nnz_u(self):
        return int(self.u_ptr[-1])

    @property
    def edges_alg(self):
        return int(self.edges.sum())

    @property
    def nsuper(self):
        return None if self.xsup is None else len(self.xsup) - 1


def csr_to_csc(n, ptr, idx):
    """Transpose a CSR pattern (rows ascending within each column): a counting
    sort in C that visits the rows in order (``oracle_transpose``)."""
    lib = _load()
    ptr = np.ascontiguousarray(ptr, dtype=np.int64)
    idx = _i32(idx)
    t_ptr = np.zeros(n + 1, dtype=np.int64)
    t_idx = np.zeros(max(int(ptr[n]) if n > 0 else 0, 0), dtype=np.int32)
    if n > 0:
        rc = lib.oracle_transpose(int(n), ptr.ctypes.data, idx.ctypes.data if len(idx) else None,
                                  t_ptr.ctypes.data, t_idx.ctypes.data if len(t_idx) else None)
        if rc != 0:
            raise MemoryError("oracle_transpose failed")
    return t_ptr, t_idx


def pattern_with_diag_nnz(n, row_ptr, col_idx) -> int:
    """nnz(pattern(A) union diag): the stored entries plus one for every row
    without a stored diagonal entry (the denominator of the dataset table's
    fill-in count)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    diag_present = np.zeros(n, dtype=bool)
    diag_present[rows[col_idx == rows]] = True
    return int(len(col_idx) + (~diag_present).sum())


def fills(res, row_ptr, col_idx) -> int:
    """fills = nnz(L) + nnz(U) - nnz(pattern(A) union diag) (dataset table,
    "#Fill-in")."""
    return res.nnz_l + res.nnz_u - pattern_with_diag_nnz(res.n, row_ptr, col_idx)


def symbolic(n, row_ptr, col_idx, max_supernode=128, threads=None,
             with_supernodes=True) -> Symbolic:
    """O1 on every row, then S1. L in both CSR and CSC."""
    cnt, lcnt, edges, ptr, entries = rows_struct(n, row_ptr, col_idx, None, threads)
    rows = np.repeat(np.arange(n, dtype=np.int32), cnt)
    is_l = entries < rows
    u_idx = entries[~is_l]
    l_ridx = entries[is_l]
    u_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt - lcnt, out=u_ptr[1:])
    l_rptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lcnt, out=l_rptr[1:])
    l_ptr, l_idx = csr_to_csc(n, l_rptr, l_ridx)
    res = Symbolic(n, u_ptr, u_idx, l_rptr, l_ridx, l_ptr, l_idx, edges,
                   int(np.asarray(row_ptr)[-1]))
    if with_supernodes:
        res.xsup, res.supno = supernodes(n, np.diff(u_ptr), l_rptr, l_ridx, max_supernode)
    return res


def supernodes(n, u_cnt, l_rptr, l_ridx, max_supernode=128):
    """S1 (Definition T3 within blocks of max_supernode rows)."""
    lib = _load()
    u_cnt = np.ascontiguousarray(u_cnt, dtype=np.int64)
    l_rptr = np.ascontiguousarray(l_rptr, dtype=np.int64)
    l_ridx = _i32(l_ridx)
    xsup = np.zeros(n + 1, dtype=np.int32)
    supno = np.zeros(max(n, 1), dtype=np.int32)
    ns = lib.oracle_supernodes(int(n), u_cnt.ctypes.data, l_rptr.ctypes.data,
                               l_ridx.ctypes.data if len(l_ridx) else None,
                               int(max_supernode), xsup.ctypes.data, supno.ctypes.data)
    return xsup[:ns + 1].copy(), supno[:n].copy()


def supernodes_structural(n, u_ptr, u_idx, l_rptr, l_ridx, max_supernode=128):
    """S2, a structural restatement of Definition T3 used to pin S1: row s
    joins the supernode starting at r iff L(s, r) != 0 and U(s,:) equals
    U(s-1,:) with column s-1 removed. Pure Python; small inputs only."""
    M = max_supernode if max_supernode > 0 else max(n, 1)
    urow = [set(u_idx[u_ptr[i]:u_ptr[i + 1]].tolist()) for i in range(n)]
    lrow = [set(l_ridx[l_rptr[i]:l_rptr[i + 1]].tolist()) for i in range(n)]
    starts = []
    for b in range(0, n, M):
        r = b
        starts.append(b)
        for s in range(b + 1, min(b + M, n)):
            if r in lrow[s] and urow[s] == (urow[s - 1] - {s - 1}):
                continue
            r = s
            starts.append(s)
    xsup = np.array(starts + [n], dtype=np.int32)
    supno = np.zeros(n, dtype=np.int32)
    for k in range(len(starts)):
        supno[xsup[k]:xsup[k + 1]] = k
    return xsup, supno


# ---- O2: structural Gaussian elimination --------------------------------

def ge_filled(n, row_ptr, col_idx) -> np.ndarray:
    """Filled pattern of L+U by elimination on a 0/1 matrix: start from
    pattern(A) plus the diagonal; for k = 0..n-1, every row i > k with a
    nonzero in column k receives row k's nonzeros right of column k.
    Rows are held as packed 64-bit words; returns a dense bool matrix."""
    W = (n + 63) // 64
    M = np.zeros((n, W), dtype=np.uint64)
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    cols = np.asarray(col_idx, dtype=np.int64)
    one = np.uint64(1)
    np.bitwise_or.at(M, (rows, cols // 64), one << (cols % 64).astype(np.uint64))
    d = np.arange(n)
    np.bitwise_or.at(M, (d, d // 64), one << (d % 64).astype(np.uint64))
    for k in range(n):
        w, b = divmod(k, 64)
        col_k = (M[k + 1:, w] >> np.uint64(b)) & one
        below = np.nonzero(col_k)[0] + k + 1
        if below.size == 0:
            continue
        right = M[k].copy()                      # row k restricted to columns > k
        right[:w] = 0
        right[w] &= ~((one << np.uint64(b + 1)) - one) if b < 63 else np.uint64(0)
        M[below] |= right
    bits = np.unpackbits(M.view(np.uint8), axis=1, bitorder="little")
    return bits[:, :n].astype(bool)


# ---- O3: per-pair fill-path search ---------------------------------------

def path_filled(n, row_ptr, col_idx) -> np.ndarray:
    """(i, j) filled iff i == j or a directed path i -> j exists whose
    intermediates are all < min(i, j). One breadth-first search per pair."""
    adj = [col_idx[row_ptr[i]:row_ptr[i + 1]].tolist() for i in range(n)]
    F = np.zeros((n, n), dtype=bool)
    for i in range(n):
        for j in range(n):
            if i == j:
                F[i, j] = True
                continue
            bound = min(i, j)
            seen = {i}
            dq = deque([i])
            found = False
            while dq and not found:
                x = dq.popleft()
                for w in adj[x]:
                    if w == j:
                        found = True
                        break
                    if w < bound and w not in seen:
                        seen.add(w)
                        dq.append(w)
            F[i, j] = found
    return F


def dense_from_symbolic(res: Symbolic) -> np.ndarray:
    n = res.n
    F = np.zeros((n, n), dtype=bool)
    rows = np.repeat(np.arange(n), np.diff(res.u_ptr))
    F[rows, res.u_idx] = True
    rows = np.repeat(np.arange(n), np.diff(res.l_rptr))
    F[rows, res.l_ridx] = True
    return F


from . import trace  # noqa: E402  (plain simulation of the parallel traversal)
