import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running case")


def read_golden(name):
    """Parse a ``key value`` fixture file (comments start with #)."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, val = line.partition(" ")
            out[key] = val.strip()
    return out


def parse_adj(spec, n):
    adj = [[] for _ in range(n)]
    for tok in spec.split():
        v, _, lst = tok.partition(":")
        adj[int(v)] = [int(x) for x in lst.split(",") if x != ""]
    return adj


def adj_to_csr(adj):
    import numpy as np
    n = len(adj)
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    cols = []
    for i, a in enumerate(adj):
        cols.extend(a)
        row_ptr[i + 1] = len(cols)
    return row_ptr, np.array(cols, dtype=np.int32)


@pytest.fixture(scope="session")
def golden():
    return read_golden


def oracle_members(mats):
    """O1 for many matrices in one call: their block-diagonal concatenation
    (no path crosses a block, so every row's structure is its matrix's row
    structure shifted by the block's first row), then per matrix the L
    transpose and the supernodes."""
    import numpy as np
    import oracle
    ns = [m.n for m in mats]
    base = np.zeros(len(mats) + 1, dtype=np.int64)
    np.cumsum(ns, out=base[1:])
    nnz = np.zeros(len(mats) + 1, dtype=np.int64)
    np.cumsum([m.nnz for m in mats], out=nnz[1:])
    rp = np.concatenate([mats[0].row_ptr[:1].astype(np.int64)] +
                        [m.row_ptr[1:].astype(np.int64) + nnz[k] for k, m in enumerate(mats)])
    ci = np.concatenate([m.col_idx.astype(np.int64) + base[k] for k, m in enumerate(mats)])
    cnt, lcnt, edges, ptr, ent = oracle.rows_struct(int(base[-1]), rp.astype(np.int32),
                                                    ci.astype(np.int32))
    out = []
    for k, m in enumerate(mats):
        r0, r1 = int(base[k]), int(base[k + 1])
        e = ent[ptr[r0]:ptr[r1]] - np.int32(r0)
        c, lc = cnt[r0:r1], lcnt[r0:r1]
        rows = np.repeat(np.arange(m.n, dtype=np.int32), c)
        is_u = e >= rows
        u_ptr = np.zeros(m.n + 1, dtype=np.int64)
        np.cumsum(c - lc, out=u_ptr[1:])
        l_rptr = np.zeros(m.n + 1, dtype=np.int64)
        np.cumsum(lc, out=l_rptr[1:])
        l_ridx = e[~is_u]
        l_ptr, l_idx = oracle.csr_to_csc(m.n, l_rptr, l_ridx)
        xsup, supno = oracle.supernodes(m.n, c - lc, l_rptr, l_ridx, 128)
        out.append(oracle.Symbolic(m.n, u_ptr, e[is_u], l_rptr, l_ridx, l_ptr, l_idx,
                                   edges[r0:r1], m.nnz, xsup, supno))
    return out
