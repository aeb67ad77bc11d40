"""GPU parity: the HIP path (called through the C ABI) against the CPU oracle,
element by element on the same seeded inputs. Integer results: bit-exact."""
import ctypes
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


def assert_same(res, ref, check_sn=True, l_csr=False):
    assert res.n == ref.n
    assert np.array_equal(res.u_ptr, ref.u_ptr), "U pointers differ"
    assert np.array_equal(res.u_idx, ref.u_idx), "U indices differ"
    if l_csr:
        assert np.array_equal(res.l_ptr, ref.l_rptr) and np.array_equal(res.l_idx, ref.l_ridx)
    else:
        assert np.array_equal(res.l_ptr, ref.l_ptr), "L pointers differ"
        assert np.array_equal(res.l_idx, ref.l_idx), "L indices differ"
    if check_sn:
        assert res.nsuper == ref.nsuper
        assert np.array_equal(res.xsup, ref.xsup) and np.array_equal(res.supno, ref.supno)
    assert res.stats["edges_alg"] == ref.edges_alg
    assert res.nnz_l == ref.nnz_l and res.nnz_u == ref.nnz_u
    assert res.fills == oracle.fills(ref, *_csr_of(ref))


_CSR = {}


def _csr_of(ref):
    return _CSR[id(ref)]


def run_ref(n, rp, ci, **kw):
    ref = oracle.symbolic(n, rp, ci, **kw)
    _CSR[id(ref)] = (rp, ci)
    return ref


def _csr_from_dense(D):
    n = D.shape[0]
    rp = np.zeros(n + 1, dtype=np.int32)
    cols = []
    for i in range(n):
        c = np.nonzero(D[i])[0]
        cols.extend(c.tolist())
        rp[i + 1] = len(cols)
    return rp, np.array(cols, dtype=np.int32)


def test_config1_full(g):
    m = synth.config(1)
    _say(f"config1 {m.desc}")
    ref = run_ref(m.n, m.row_ptr, m.col_idx)
    res = g.symbolic(m.n, m.row_ptr, m.col_idx)
    assert_same(res, ref)


@pytest.mark.parametrize("seed", range(24))
def test_random_small(g, seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 300))
    D = rng.random((n, n)) < float(rng.uniform(0.3, 6.0)) / n
    if seed % 3:
        np.fill_diagonal(D, True)
    rp, ci = _csr_from_dense(D)
    if seed % 4 == 1:  # unsorted columns are accepted
        for i in range(n):
            seg = ci[rp[i]:rp[i + 1]]
            rng.shuffle(seg)
    _say(f"random_small seed={seed} n={n} nnz={len(ci)}")
    ref = run_ref(n, rp, ci)
    res = g.symbolic(n, rp, ci)
    assert_same(res, ref)


def test_edge_sizes(g):
    # n = 0
    r = g.symbolic(0, np.zeros(1, dtype=np.int32), np.zeros(0, dtype=np.int32))
    assert r.n == 0 and r.nnz_l == 0 and r.nnz_u == 0 and r.nsuper == 0
    assert list(r.xsup) == [0]
    # n = 1, with and without diagonal
    for ci in (np.zeros(0, dtype=np.int32), np.zeros(1, dtype=np.int32)):
        rp = np.array([0, len(ci)], dtype=np.int32)
        r = g.symbolic(1, rp, ci)
        assert list(r.u_ptr) == [0, 1] and list(r.u_idx) == [0] and r.nnz_l == 0
        assert r.nsuper == 1 and list(r.xsup) == [0, 1] and list(r.supno) == [0]
    # empty pattern, n = 70: only the diagonal
    n = 70
    r = g.symbolic(n, np.zeros(n + 1, dtype=np.int32), np.zeros(0, dtype=np.int32))
    assert r.nnz_u == n and r.nnz_l == 0 and r.nsuper == n and r.fills == 0


@pytest.mark.parametrize("mapping", [0x40, 0x80, 0x100, 0x800, 0x1000])
@pytest.mark.parametrize("name", ["dense", "arrow_first", "arrow_last", "tril", "triu"])
def test_closed_forms_on_gpu(g, name, mapping):
    n = 300
    if name == "dense":
        D = np.ones((n, n), dtype=bool)
    elif name == "arrow_first":
        D = np.eye(n, dtype=bool); D[0, :] = True; D[:, 0] = True
    elif name == "arrow_last":
        D = np.eye(n, dtype=bool); D[-1, :] = True; D[:, -1] = True
    elif name == "tril":
        D = np.tril(np.ones((n, n), dtype=bool))
    else:
        D = np.triu(np.ones((n, n), dtype=bool))
    rp, ci = _csr_from_dense(D)
    _say(f"closed form {name} mapping={mapping:#x}")
    ref = run_ref(n, rp, ci)
    assert_same(g.symbolic(n, rp, ci, flags=mapping), ref)


def _families():
    return [synth.stencil(9, (32, 32), nd=True, seed=11),
            synth.stencil(9, (61, 47), nd=True, seed=12),
            synth.stencil(27, (8, 8, 8), nd=True, seed=13),
            synth.stencil(27, (13, 11, 9), nd=True, seed=14),
            synth.stencil(7, (20, 19, 18), nd=True, seed=15),
            synth.stencil(5, (70, 70), nd=False, seed=16),
            synth.batch_member(0), synth.batch_member(1), synth.batch_member(7),
            synth.stencil(27, (27, 26, 25), nd=True, seed=17),
            synth.stencil(9, (150, 140), nd=True, seed=18)]


@pytest.mark.parametrize("idx", range(11))
def test_generator_families(g, idx):
    m = _families()[idx]
    _say(f"family {m.desc} n={m.n}")
    ref = run_ref(m.n, m.row_ptr, m.col_idx)
    assert_same(g.symbolic(m.n, m.row_ptr, m.col_idx), ref)


def _shared_targets(k, width, n, seed):
    """Rows 0..k-1 all have entries in the same `width` columns k..k+width-1, and
    later rows (sources above and inside that column range) reach rows 0..k-1: one
    traversal round then holds several edges to each not yet reached target, on
    the L side and on the U side of the source (the in-round atomic filter keeps
    one per target)."""
    rng = np.random.default_rng(seed)
    D = np.eye(n, dtype=bool)
    D[:k, k:k + width] = True
    D[k + width:k + width + 12, :k] = True      # sources above the shared columns
    D[k:k + 6, :k] = True                       # sources inside them (U-side targets)
    D |= rng.random((n, n)) < 1.5 / n
    return _csr_from_dense(D)


@pytest.mark.parametrize("case", [(16, 64, 300, 1, 0), (16, 200, 300, 2, 0), (40, 32, 300, 3, 0),
                                  (8, 250, 300, 4, 0), (60, 150, 300, 5, 64), (16, 64, 300, 6, 1),
                                  (64, 200, 400, 7, 253)], ids=str)
def test_shared_targets_in_one_round(g, case):
    k, width, n, seed, window = case
    rp, ci = _shared_targets(k, width, n, seed)
    _say(f"shared targets k={k} width={width} n={n} window={window}")
    ref = run_ref(n, rp, ci)
    assert_same(g.symbolic(n, rp, ci, window=window), ref)
    assert_same(g.symbolic(n, rp, ci, window=window, flags=0x800), ref)
    assert_same(g.symbolic(n, rp, ci, window=window, flags=0x1000), ref)


def test_full_rows_span_several_sort_chunks(g):
    """Row 0 and the last three rows hold every column and each other row a band
    entry: the U row of 0 and the L rows of the last three span more ids than one
    LDS bitmap chunk of the row sort, so they are ranked over several chunks."""
    n = 300_000
    rows = []
    full = np.arange(n, dtype=np.int32)
    for i in range(n):
        if i == 0 or i >= n - 3:
            rows.append(full)
        elif i + 7 < n:
            rows.append(np.array([i, i + 7], dtype=np.int32))
        else:
            rows.append(np.array([i], dtype=np.int32))
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.concatenate(rows).astype(np.int32)
    _say(f"full rows n={n} nnz={len(ci)}")
    ref = run_ref(n, rp, ci)
    assert_same(g.symbolic(n, rp, ci), ref)


@pytest.mark.parametrize("kw", [
    {"window": 1}, {"window": 3}, {"window": 64}, {"window": 5000},
    {"flags": 0x20}, {"flags": 0x10}, {"concurrent_sources": 1}, {"concurrent_sources": 7},
    {"concurrent_sources": 64, "window": 2}, {"max_supernode": 16}, {"max_supernode": -1},
    {"max_supernode": 1}, {"flags": 0x2}, {"flags": 0x1},
    {"flags": 0x40}, {"flags": 0x80}, {"flags": 0x100}, {"flags": 0x100 | 0x20},
    {"flags": 0x80, "concurrent_sources": 3}, {"flags": 0x100, "window": 1},
    {"flags": 0x80 | 0x10, "window": 64},
    {"window": 253}, {"window": 200, "concurrent_sources": 5}, {"window": 254},
    {"flags": 0x200}, {"flags": 0x200 | 0x1 | 0x2},
    {"flags": 0x800}, {"flags": 0x800, "window": 1}, {"flags": 0x800, "window": 3},
    {"flags": 0x800, "window": 253}, {"flags": 0x800, "window": 200, "concurrent_sources": 5},
    {"flags": 0x800 | 0x20}, {"flags": 0x800 | 0x10},
    {"flags": 0x1000}, {"flags": 0x1000, "window": 3}, {"flags": 0x1000, "concurrent_sources": 7},
    # label reset before every source (ablation of the value-range scheme)
    {"flags": 0x10000}, {"flags": 0x10000 | 0x1000}, {"flags": 0x10000 | 0x80},
    # one thread per source (fill2 comparison baseline)
    {"flags": 0x8000}, {"flags": 0x8000, "concurrent_sources": 5}, {"flags": 0x8000 | 0x2},
    # memory-budget mode: bands, U bitmap, host spill of worklists and row buffers
    {"flags": 0x4000}, {"flags": 0x4000, "queue_cap": 64},
    {"flags": 0x4000 | 0x10, "queue_cap": 64, "window": 3},
    {"flags": 0x4000 | 0x20, "queue_cap": 100},
    {"flags": 0x4000 | 0x10000, "queue_cap": 64, "concurrent_sources": 6},
], ids=str)
def test_knobs_do_not_change_results(g, kw):
    m = synth.stencil(27, (11, 10, 9), nd=True, seed=21)
    ms = kw.get("max_supernode", 0)
    M = 128 if ms == 0 else (0 if ms < 0 else ms)
    _say(f"knobs {kw}")
    ref = run_ref(m.n, m.row_ptr, m.col_idx, max_supernode=M)
    res = g.symbolic(m.n, m.row_ptr, m.col_idx, **kw)
    flags = kw.get("flags", 0)
    assert_same(res, ref, check_sn=not (flags & 0x1), l_csr=bool(flags & 0x2))
    if flags & 0x1:
        assert res.nsuper == 0 and res.xsup is None


def test_small_budget_forces_pool_regrowth(g):
    """A tight memory budget leaves a tiny output pool, so most rows overflow
    it on the first pass and are recomputed after the pool grows."""
    m = synth.stencil(9, (40, 40), nd=True, seed=31)
    ref = run_ref(m.n, m.row_ptr, m.col_idx)
    _say("small budget")
    res = g.symbolic(m.n, m.row_ptr, m.col_idx, mem_budget_bytes=96 << 20, concurrent_sources=4)
    assert_same(res, ref)


def test_budget_below_one_source_is_enomem(g):
    m = synth.stencil(9, (40, 40), nd=True, seed=31)
    with pytest.raises(g.GsofaError) as e:
        g.symbolic(m.n, m.row_ptr, m.col_idx, mem_budget_bytes=1 << 16)
    assert e.value.code == g.ENOMEM


def test_device_input_and_output(g):
    import torch
    m = synth.stencil(27, (9, 9, 9), nd=True, seed=41)
    ref = run_ref(m.n, m.row_ptr, m.col_idx)
    rp = torch.from_numpy(m.row_ptr).cuda()
    ci = torch.from_numpy(m.col_idx).cuda()
    _say("device in, host out")
    assert_same(g.symbolic(m.n, rp, ci), ref)
    _say("device in, device out")
    d = g.symbolic(m.n, rp, ci, flags=g.RESULT_ON_DEVICE)
    t = d.to_torch()
    assert np.array_equal(t["u_ptr"].cpu().numpy(), ref.u_ptr)
    assert np.array_equal(t["u_idx"].cpu().numpy(), ref.u_idx)
    assert np.array_equal(t["l_ptr"].cpu().numpy(), ref.l_ptr)
    assert np.array_equal(t["l_idx"].cpu().numpy(), ref.l_idx)
    assert np.array_equal(t["xsup"].cpu().numpy(), ref.xsup)
    assert np.array_equal(t["supno"].cpu().numpy(), ref.supno)
    d.free()


def test_device_input_errors(g):
    import torch
    m = synth.stencil(9, (10, 10), nd=True, seed=51)
    ci = m.col_idx.copy()
    ci[5] = m.n + 3  # out of range
    with pytest.raises(g.GsofaError) as e:
        g.symbolic(m.n, torch.from_numpy(m.row_ptr).cuda(), torch.from_numpy(ci).cuda())
    assert e.value.code == g.EINVAL
    ci = m.col_idx.copy()
    r = 7
    ci[m.row_ptr[r] + 1] = ci[m.row_ptr[r]]  # repeated column in row 7
    with pytest.raises(g.GsofaError) as e:
        g.symbolic(m.n, torch.from_numpy(m.row_ptr).cuda(), torch.from_numpy(ci).cuda())
    assert e.value.code == g.EINVAL
    # entries but no column array: rejected before any kernel reads it
    lib = g.load()
    out = ctypes.POINTER(g.Result)()
    o = g.Opts()
    o.flags = g.INPUT_ON_DEVICE
    rp_d = torch.from_numpy(m.row_ptr).cuda()
    assert lib.gsofa_symbolic(m.n, ctypes.c_void_p(rp_d.data_ptr()), None, ctypes.byref(o),
                              ctypes.byref(out)) == g.EINVAL
    # the library stays usable afterwards
    ref = run_ref(m.n, m.row_ptr, m.col_idx)
    assert_same(g.symbolic(m.n, m.row_ptr, m.col_idx), ref)


def test_repeat_calls_are_deterministic(g):
    m = synth.stencil(9, (50, 50), nd=True, seed=61)
    a = g.symbolic(m.n, m.row_ptr, m.col_idx)
    for _ in range(3):
        b = g.symbolic(m.n, m.row_ptr, m.col_idx)
        assert np.array_equal(a.u_idx, b.u_idx) and np.array_equal(a.l_idx, b.l_idx)
        assert np.array_equal(a.supno, b.supno)


def test_autotuner_trials_keep_results(g):
    """Forcing the tuner's trial launches on a mid-size matrix: every candidate
    runs on a sample of its sources, the fastest is kept, and the result still
    equals the oracle; a later call of the same class reuses the choice."""
    m = synth.stencil(27, (22, 21, 20), nd=True, seed=71)
    ref = run_ref(m.n, m.row_ptr, m.col_idx)
    _say(f"tuner on n={m.n}")
    res = g.symbolic(m.n, m.row_ptr, m.col_idx, flags=g.TUNE_NOW)
    assert res.stats["t_tune_ms"] > 0
    # the tuner's candidates: 32-bit labels at eight (0) or seven (4) wavefronts
    # per SIMD, byte states (3)
    assert res.stats["mapping"] in (0, 3, 4) and 1 <= res.stats["window"] <= 64
    assert_same(res, ref)
    again = g.symbolic(m.n, m.row_ptr, m.col_idx)
    assert again.stats["t_tune_ms"] == 0
    assert (again.stats["mapping"], again.stats["window"]) == (res.stats["mapping"], res.stats["window"])
    assert_same(again, ref)


def test_host_results_outlive_their_result_object(g):
    """Host result arrays view the library's result memory: they stay valid after
    the result object is gone and later calls have taken and returned result
    memory, and a result in a page-locked block (above 1 MiB) equals the
    device-resident result of the same call."""
    import gc
    m = synth.stencil(27, (30, 30, 30), nd=True, seed=81)
    other = synth.stencil(27, (30, 30, 29), nd=True, seed=82)
    _say(f"host result views n={m.n}")
    a = g.symbolic(m.n, m.row_ptr, m.col_idx, flags=g.NO_TUNE)
    assert 4 * (a.nnz_l + a.nnz_u) > (8 << 20)
    d = g.symbolic(m.n, m.row_ptr, m.col_idx, flags=g.NO_TUNE | g.RESULT_ON_DEVICE)
    t = d.to_torch()
    d.free()
    for k in ("l_ptr", "l_idx", "u_ptr", "u_idx", "xsup", "supno"):
        assert np.array_equal(getattr(a, k), t[k].cpu().numpy()), k
    keep = {k: getattr(a, k) for k in ("l_idx", "u_idx", "supno")}
    want = {k: v.copy() for k, v in keep.items()}
    del a
    gc.collect()
    for _ in range(2):
        b = g.symbolic(other.n, other.row_ptr, other.col_idx, flags=g.NO_TUNE)
        del b
        gc.collect()
    for k in keep:
        assert np.array_equal(keep[k], want[k]), k
    del keep
    gc.collect()
    c = g.symbolic(m.n, m.row_ptr, m.col_idx, flags=g.NO_TUNE)
    for k in want:
        assert np.array_equal(getattr(c, k), want[k]), k
