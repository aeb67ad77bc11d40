"""The CPU comparison baseline (Gilbert-Peierls, column by column) against the
oracle: L by columns equal, U by columns equal to the transpose of the
oracle's U rows. CPU only."""
import numpy as np
import pytest

import baselines
import oracle
import synth


def _check(n, rp, ci):
    r = baselines.gilbert_peierls(n, rp, ci)
    ref = oracle.symbolic(n, rp, ci, with_supernodes=False)
    assert r.cols_done == n
    assert np.array_equal(r.l_ptr, ref.l_ptr) and np.array_equal(r.l_idx, ref.l_idx)
    up, ui = oracle.csr_to_csc(n, ref.u_ptr, ref.u_idx)
    assert np.array_equal(r.u_ptr, up) and np.array_equal(r.u_idx, ui)
    return r


def test_gp_config1():
    m = synth.config(1)
    _check(m.n, m.row_ptr, m.col_idx)


@pytest.mark.parametrize("seed", range(10))
def test_gp_random(seed):
    rng = np.random.default_rng(700 + seed)
    n = int(rng.integers(1, 120))
    D = rng.random((n, n)) < 0.05
    D[np.diag_indices(n)] = rng.random(n) < 0.7
    rp = np.zeros(n + 1, dtype=np.int32)
    cols = []
    for i in range(n):
        c = np.nonzero(D[i])[0]
        rng.shuffle(c)
        cols.extend(c.tolist())
        rp[i + 1] = len(cols)
    _check(n, rp, np.array(cols, dtype=np.int32))


@pytest.mark.parametrize("m", [synth.stencil(27, (9, 8, 7), nd=True, seed=71),
                               synth.stencil(9, (30, 25), nd=True, seed=72),
                               synth.batch_member(73)], ids=lambda m: m.desc[:24])
def test_gp_families(m):
    _check(m.n, m.row_ptr, m.col_idx)


def test_gp_empty_and_time_limit():
    r = baselines.gilbert_peierls(0, np.zeros(1, np.int32), np.zeros(0, np.int32))
    assert r.cols_done == 0 and r.l_ptr.tolist() == [0]
    m = synth.stencil(9, (60, 60), nd=True, seed=74)
    part = baselines.gilbert_peierls(m.n, m.row_ptr, m.col_idx, time_limit_s=1e-9)
    assert 0 < part.cols_done < m.n
    full = _check(m.n, m.row_ptr, m.col_idx)
    k = part.cols_done
    assert np.array_equal(part.l_ptr[:k + 1], full.l_ptr[:k + 1])
    assert np.array_equal(part.l_idx, full.l_idx[:full.l_ptr[k]])
