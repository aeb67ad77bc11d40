"""Full-size parity on the 2D (1000x1000 9-point) and 3D (64^3 27-point)
workloads, in the launch configuration bench.py times (automatic mapping and
slots, device-resident input): U rows, supernodes and every total are compared
in full against the oracle; L columns are compared on a sample through the
transpose duality filled(A^T) = filled(A)^T (column k of L(A) is the strict
upper part of row k of U(A^T))."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("cfg", [3, 2])
def test_fullsize(cfg):
    import torch
    import paper_2007_00840_amd as g
    m = synth.config(cfg)
    _say(f"config {cfg}: {m.desc} n={m.n} nnz={m.nnz}")
    rp = torch.from_numpy(m.row_ptr).cuda()
    ci = torch.from_numpy(m.col_idx).cuda()
    res = g.symbolic(m.n, rp, ci)
    _say(f"gpu done: nnz_l={res.nnz_l} nnz_u={res.nnz_u} nsuper={res.nsuper} "
         f"traverse={res.stats['t_traverse_ms']:.1f} ms")
    cnt, lcnt, edges, ptr, ent = oracle.rows_struct(m.n, m.row_ptr, m.col_idx)
    _say("oracle rows done")
    assert res.stats["edges_alg"] == int(edges.sum())
    assert res.nnz_l == int(lcnt.sum()) and res.nnz_u == int((cnt - lcnt).sum())
    rows = np.repeat(np.arange(m.n, dtype=np.int32), cnt)
    is_u = ent >= rows
    del rows
    u_ptr = np.zeros(m.n + 1, dtype=np.int64)
    np.cumsum(cnt - lcnt, out=u_ptr[1:])
    assert np.array_equal(res.u_ptr, u_ptr)
    assert np.array_equal(res.u_idx, ent[is_u])
    l_rptr = np.zeros(m.n + 1, dtype=np.int64)
    np.cumsum(lcnt, out=l_rptr[1:])
    l_ridx = ent[~is_u]
    del ent, is_u
    xsup, supno = oracle.supernodes(m.n, cnt - lcnt, l_rptr, l_ridx, 128)
    assert res.nsuper == len(xsup) - 1
    assert np.array_equal(res.xsup, xsup) and np.array_equal(res.supno, supno)
    # column counts of L: bincount of the row-wise column ids
    col_cnt = np.bincount(l_ridx, minlength=m.n)
    assert np.array_equal(np.diff(res.l_ptr), col_cnt)
    # sampled L columns through the transpose
    tp, ti = oracle.csr_to_csc(m.n, m.row_ptr, m.col_idx)
    rng = np.random.default_rng(cfg)
    cols = np.unique(np.concatenate([np.arange(m.n - 256, m.n), np.arange(0, 64),
                                     rng.choice(m.n, 512, replace=False)])).astype(np.int32)
    c2, l2, e2, p2, ent2 = oracle.rows_struct(m.n, tp.astype(np.int32), ti, cols)
    for k, c in enumerate(cols):
        seg = ent2[p2[k]:p2[k + 1]]
        want = seg[seg > c]
        got = res.l_idx[res.l_ptr[c]:res.l_ptr[c + 1]]
        assert np.array_equal(got, want), f"L column {c}"
    _say("full-size parity ok")
