"""Memory-budget mode (Space Optimization section): sources run in bands of
decreasing ids with label arrays sized to the band (bubble removal), more
sources in flight for lower bands (dynamic space allocation), and worklist /
row-buffer overflow written to pinned host memory and read back (external
frontier management). Results must equal the oracle's bit for bit whatever
the budget and queue capacity."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import torch
    assert torch.cuda.is_available()
    import paper_2007_00840_amd as g
    g.load()
    return g


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _same(res, ref):
    assert np.array_equal(res.u_ptr, ref.u_ptr) and np.array_equal(res.u_idx, ref.u_idx)
    assert np.array_equal(res.l_ptr, ref.l_ptr) and np.array_equal(res.l_idx, ref.l_idx)
    assert np.array_equal(res.xsup, ref.xsup) and np.array_equal(res.supno, ref.supno)
    assert res.stats["edges_alg"] == ref.edges_alg


CASES = [synth.stencil(27, (16, 15, 14), nd=True, seed=401),
         synth.stencil(9, (70, 60), nd=True, seed=402),
         synth.stencil(5, (50, 50), nd=False, seed=403),
         synth.batch_member(404)]


@pytest.mark.parametrize("m", CASES, ids=lambda m: m.desc[:28])
@pytest.mark.parametrize("queue_cap,budget", [(64, 1 << 20), (64, 16 << 20), (2048, 4 << 20), (0, 0)])
def test_budget_mode_matches_oracle(g, m, queue_cap, budget):
    ref = oracle.symbolic(m.n, m.row_ptr, m.col_idx)
    _say(f"budget mode {m.desc} queue_cap={queue_cap} budget={budget}")
    res = g.symbolic(m.n, m.row_ptr, m.col_idx, flags=g.BUDGET_MODE, queue_cap=queue_cap,
                     mem_budget_bytes=budget)
    _same(res, ref)
    st = res.stats
    assert st["mapping"] == 5 and st["launches"] >= 1 and st["concurrent_sources"] >= 1
    if queue_cap == 64:
        # a 64-entry row buffer cannot hold the larger rows: they spill
        assert st["spilled_entries"] > 0
    if budget == 1 << 20 and m.n > 4096:
        # a 1 MiB budget holds few top-band slots: several bands
        assert st["launches"] > 1


def test_budget_mode_spill_volume_accounts_row_overflow(g):
    """With a 64-entry device part, every row with more than 64 structure
    entries spills at least its excess."""
    m = CASES[0]
    ref = oracle.symbolic(m.n, m.row_ptr, m.col_idx)
    res = g.symbolic(m.n, m.row_ptr, m.col_idx, flags=g.BUDGET_MODE, queue_cap=64)
    _same(res, ref)
    cnt = np.diff(ref.u_ptr) + np.diff(ref.l_rptr)
    assert res.stats["spilled_entries"] >= int(np.maximum(cnt - 64, 0).sum())


def test_budget_mode_batch_and_device_io(g):
    import torch
    mats = [synth.batch_member(k) for k in range(410, 426)]
    res = g.batch([(m.n, m.row_ptr, m.col_idx) for m in mats], flags=g.BUDGET_MODE, queue_cap=64,
                  mem_budget_bytes=2 << 20)
    for m, r in zip(mats, res):
        _same(r, oracle.symbolic(m.n, m.row_ptr, m.col_idx))
    m = CASES[1]
    ref = oracle.symbolic(m.n, m.row_ptr, m.col_idx)
    d = g.symbolic(m.n, torch.from_numpy(m.row_ptr).cuda(), torch.from_numpy(m.col_idx).cuda(),
                   flags=g.BUDGET_MODE | g.RESULT_ON_DEVICE, queue_cap=64)
    t = d.to_torch()
    assert np.array_equal(t["u_idx"].cpu().numpy(), ref.u_idx)
    assert np.array_equal(t["l_idx"].cpu().numpy(), ref.l_idx)
    d.free()


def test_budget_mode_output_pool_regrowth(g):
    """A low fill ratio recorded for a size class (a banded matrix of the same
    size and row length, which does not fill) under-sizes the output pool of a
    high-fill call of that class: overflowing rows are redone in budget mode
    after the pool grows."""
    import time
    n, bw = 10000, 10
    i = np.repeat(np.arange(n), 2 * bw + 1)
    j = i + np.tile(np.arange(-bw, bw + 1), n)
    keep = (j >= 0) & (j < n)
    ci = j[keep].astype(np.int32)
    rp = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(np.bincount(i[keep], minlength=n), out=rp[1:])
    t0 = time.time()
    band = g.symbolic(n, rp, ci, flags=g.NO_TUNE)
    assert band.fills == 0
    _say(f"banded call done in {time.time() - t0:.1f} s")
    m = synth.stencil(27, (22, 22, 22), nd=True, seed=405)
    ref = oracle.symbolic(m.n, m.row_ptr, m.col_idx)
    t0 = time.time()
    res = g.symbolic(m.n, m.row_ptr, m.col_idx, flags=g.BUDGET_MODE, queue_cap=256)
    _say(f"budget call done in {time.time() - t0:.1f} s, launches={res.stats['launches']}")
    _same(res, ref)
    assert res.stats["launches"] >= 2  # the bands, then the redone rows


def test_budget_below_one_slot_is_enomem(g):
    m = CASES[0]
    with pytest.raises(g.GsofaError) as e:
        g.symbolic(m.n, m.row_ptr, m.col_idx, flags=g.BUDGET_MODE, mem_budget_bytes=4096)
    assert e.value.code == g.ENOMEM
    # the library is still usable
    _same(g.symbolic(m.n, m.row_ptr, m.col_idx), oracle.symbolic(m.n, m.row_ptr, m.col_idx))
