"""Full-size parity on the 2D (1000x1000 9-point) and 3D (64^3 27-point)
workloads, in the launch configuration bench.py times (automatic mapping and
slots, device-resident input): every output array -- U in CSR, L in CSC,
supernodes -- and every total is compared in full against the oracle. L's
column layout comes from the oracle's rows through its counting-sort
transpose."""
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
    # L column-wise, every array in full
    l_ptr, l_idx = oracle.csr_to_csc(m.n, l_rptr, l_ridx)
    del l_rptr, l_ridx
    assert np.array_equal(res.l_ptr, l_ptr), "L column pointers differ"
    assert np.array_equal(res.l_idx, l_idx), "L row indices differ"
    assert res.fills == res.nnz_l + res.nnz_u - oracle.pattern_with_diag_nnz(m.n, m.row_ptr, m.col_idx)
    _say(f"full-size parity ok: {res.nnz_l + res.nnz_u} entries compared")
