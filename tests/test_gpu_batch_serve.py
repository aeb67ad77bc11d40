"""GPU parity of the batch and serve entry points against the CPU oracle and
against the one-matrix path."""
import sys
import time

import numpy as np
import pytest

import oracle
import synth
from conftest import oracle_members

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


def same(res, ref):
    return (np.array_equal(res.u_ptr, ref.u_ptr) and np.array_equal(res.u_idx, ref.u_idx)
            and np.array_equal(res.l_ptr, ref.l_ptr) and np.array_equal(res.l_idx, ref.l_idx)
            and res.nsuper == ref.nsuper and np.array_equal(res.xsup, ref.xsup)
            and np.array_equal(res.supno, ref.supno) and res.stats["edges_alg"] == ref.edges_alg)


def same_result(a, b):
    return (np.array_equal(a.u_ptr, b.u_ptr) and np.array_equal(a.u_idx, b.u_idx)
            and np.array_equal(a.l_ptr, b.l_ptr) and np.array_equal(a.l_idx, b.l_idx)
            and np.array_equal(a.xsup, b.xsup) and np.array_equal(a.supno, b.supno))


def test_batch_members_match_oracle(g):
    """The whole 4,096-matrix batch in one gsofa_batch call, every member
    compared in full against the oracle."""
    mats = [synth.batch_member(k) for k in range(4096)]
    _say(f"batch of {len(mats)} members, sum n = {sum(m.n for m in mats)}")
    res = g.batch([(m.n, m.row_ptr, m.col_idx) for m in mats])
    assert len(res) == len(mats)
    _say("gpu batch done")
    for lo in range(0, len(mats), 512):
        refs = oracle_members(mats[lo:lo + 512])
        for k, (m, r, ref) in enumerate(zip(mats[lo:lo + 512], res[lo:lo + 512], refs)):
            assert same(r, ref), f"member {lo + k}"
        _say(f"members {lo}..{lo + 511} ok")


def test_batch_equals_single_calls_and_mixed_sizes(g):
    mats = [synth.stencil(27, (12, 11, 10), nd=True, seed=5), synth.batch_member(3),
            synth.stencil(9, (1, 1), nd=True, seed=1), synth.stencil(5, (60, 2), nd=False, seed=9),
            synth.batch_member(8)]
    empty = (0, np.zeros(1, dtype=np.int32), np.zeros(0, dtype=np.int32))
    args = [(m.n, m.row_ptr, m.col_idx) for m in mats] + [empty]
    for flags in (0, 0x40, 0x100, 0x800, 0x1000):
        res = g.batch(args, flags=flags)
        for m, r in zip(mats, res):
            assert same_result(r, g.symbolic(m.n, m.row_ptr, m.col_idx))
        assert res[-1].n == 0 and res[-1].nsuper == 0


def test_batch_reports_per_matrix_errors(g):
    good = synth.batch_member(2)
    bad_ci = good.col_idx.copy()
    bad_ci[3] = good.n + 5
    res = g.batch([(good.n, good.row_ptr, good.col_idx), (good.n, good.row_ptr, bad_ci),
                   (good.n, good.row_ptr, good.col_idx)], raise_on_error=False)
    assert res[1] is None
    ref = oracle.symbolic(good.n, good.row_ptr, good.col_idx)
    assert same(res[0], ref) and same(res[2], ref)
    with pytest.raises(g.GsofaError) as e:
        g.batch([(good.n, good.row_ptr, bad_ci)])
    assert e.value.code == g.EINVAL


def test_batch_device_inputs_and_results(g):
    import torch
    mats = [synth.batch_member(k) for k in (10, 11, 12)]
    args = [(m.n, torch.from_numpy(m.row_ptr).cuda(), torch.from_numpy(m.col_idx).cuda())
            for m in mats]
    res = g.batch(args, flags=g.RESULT_ON_DEVICE)
    for m, d in zip(mats, res):
        ref = oracle.symbolic(m.n, m.row_ptr, m.col_idx)
        t = d.to_torch()
        assert np.array_equal(t["u_ptr"].cpu().numpy(), ref.u_ptr)
        assert np.array_equal(t["u_idx"].cpu().numpy(), ref.u_idx)
        assert np.array_equal(t["l_ptr"].cpu().numpy(), ref.l_ptr)
        assert np.array_equal(t["l_idx"].cpu().numpy(), ref.l_idx)
        assert np.array_equal(t["xsup"].cpu().numpy(), ref.xsup)
        assert np.array_equal(t["supno"].cpu().numpy(), ref.supno)
        d.free()


def test_serve_results_alone_and_in_mix(g):
    reqs = synth.serve_trace(count=12)
    mats = [r.matrix() for r in reqs if r.n_req <= 40000][:8]
    assert len(mats) >= 4
    _say(f"serve: {len(mats)} requests, n = {[m.n for m in mats]}")
    # alone: one request at a time
    with g.Server(max_inflight=1) as srv:
        alone = []
        for m in mats:
            t = srv.submit(m.n, m.row_ptr, m.col_idx)
            alone.append(srv.poll(t, timeout_us=-1))
    # mixed: all submitted at once, several in flight
    with g.Server(max_inflight=4) as srv:
        tickets = [srv.submit(m.n, m.row_ptr, m.col_idx) for m in mats]
        mixed = {}
        deadline = time.time() + 60
        while len(mixed) < len(tickets) and time.time() < deadline:
            for t in tickets:
                if t not in mixed:
                    r = srv.poll(t, timeout_us=1000)
                    if r is not None:
                        mixed[t] = r
        assert len(mixed) == len(tickets)
    for m, a, t in zip(mats, alone, tickets):
        ref = oracle.symbolic(m.n, m.row_ptr, m.col_idx)
        assert same(a, ref)
        assert same_result(a, mixed[t])


def test_serve_trace_sample_with_large_requests(g):
    """Requests of the served stream above 10^5 rows, one 2D 9-point and one
    3D 27-point, mixed with small ones of the same trace: all in flight
    together, every array of every result compared in full with the oracle."""
    reqs = synth.serve_trace(count=60)
    big2 = next(r for r in reqs if r.n_req > 100000 and r.kind == 9)
    big3 = next(r for r in reqs if r.n_req > 100000 and r.kind == 27)
    small = [r for r in reqs if r.n_req <= 20000][:6]
    chosen = [big2, big3] + small
    mats = [r.matrix() for r in chosen]
    _say(f"serve trace sample: requests {[r.rid for r in chosen]}, n = {[m.n for m in mats]}")
    with g.Server(max_inflight=4) as srv:
        tickets = [srv.submit(m.n, m.row_ptr, m.col_idx) for m in mats]
        got = [srv.poll(t, timeout_us=-1) for t in tickets]
    _say("served; checking against the oracle")
    for r, m, res in zip(chosen, mats, got):
        assert same(res, oracle.symbolic(m.n, m.row_ptr, m.col_idx)), f"request {r.rid}"


def test_serve_status_codes(g):
    m = synth.stencil(27, (30, 30, 30), nd=True, seed=77)
    with g.Server(max_inflight=2) as srv:
        t = srv.submit(m.n, m.row_ptr, m.col_idx)
        # immediately after submission the request cannot be done yet
        assert srv.poll(t, timeout_us=0) is None
        r = srv.poll(t, timeout_us=-1)
        assert r.n == m.n
        with pytest.raises(g.GsofaError) as e:
            srv.poll(t, timeout_us=0)  # already collected
        assert e.value.code == g.ENOTFOUND
        with pytest.raises(g.GsofaError) as e:
            srv.poll(987654, timeout_us=0)
        assert e.value.code == g.ENOTFOUND
        bad = m.col_idx.copy()
        bad[0] = -3
        with pytest.raises(g.GsofaError) as e:
            srv.submit(m.n, m.row_ptr, bad)
        assert e.value.code == g.EINVAL
        # an order above GSOFA_MAX_N is refused before its arrays are read
        with pytest.raises(g.GsofaError) as e:
            srv.submit(g.MAX_N + 1, m.row_ptr[:2], m.col_idx[:1])
        assert e.value.code == g.EINVAL
    with g.Server(max_inflight=1, mem_budget_bytes=1 << 20) as srv:
        with pytest.raises(g.GsofaError) as e:
            srv.submit(m.n, m.row_ptr, m.col_idx)
        assert e.value.code == g.ECAPACITY


def test_serve_many_concurrent_requests(g):
    """Regression: requests running on different streams must never reuse a
    device buffer that another stream's kernels still read. Many mixed-size
    requests in flight at once, every result checked against the oracle."""
    mats = []
    for k in range(24):
        if k % 3 == 0:
            mats.append(synth.stencil(27, (14 + k % 5, 13, 12), nd=True, seed=900 + k))
        elif k % 3 == 1:
            mats.append(synth.stencil(9, (90 + 7 * k, 80), nd=True, seed=900 + k))
        else:
            mats.append(synth.batch_member(100 + k))
    _say(f"serve stress: {len(mats)} requests, n = {[m.n for m in mats]}")
    with g.Server(max_inflight=4) as srv:
        tickets = [srv.submit(m.n, m.row_ptr, m.col_idx) for m in mats]
        got = [srv.poll(t, timeout_us=-1) for t in tickets]
    for m, r in zip(mats, got):
        assert same(r, oracle.symbolic(m.n, m.row_ptr, m.col_idx))


def test_graph_replays_match_eager(g):
    """Each phase of a call is captured once, and its executable graph is
    updated in place for later calls. Every replay, with eager calls and calls
    of another graph shape in between, gives the eager results."""
    mats = [synth.batch_member(k) for k in (20, 21, 22, 23)]
    args = [(m.n, m.row_ptr, m.col_idx) for m in mats]
    eager = g.batch(args, flags=g.EAGER)
    for m, r in zip(mats, eager):
        assert same(r, oracle.symbolic(m.n, m.row_ptr, m.col_idx))
    c0 = g.graph_counters()
    for rep in range(4):
        _say(f"graph replay {rep}")
        res = g.batch(args)
        for a, b in zip(res, eager):
            assert same_result(a, b)
        again = g.batch(args, flags=g.EAGER)
        for a, b in zip(again, eager):
            assert same_result(a, b)
        one = g.symbolic(*args[rep])
        assert same_result(one, eager[rep])
    c1 = g.graph_counters()
    assert c1[2] > c0[2]
    assert c1[1] > c0[1]


_LARGE = []


def _two_large():
    """Two 48^3 27-point stencils (110,592 rows: large requests) and their oracle
    results, computed once for the tests that use them."""
    if not _LARGE:
        big = [synth.stencil(27, (48, 48, 48), nd=True, seed=311 + k) for k in range(2)]
        _LARGE.append((big, [oracle.symbolic(m.n, m.row_ptr, m.col_idx) for m in big]))
    return _LARGE[0]


def test_serve_lone_request_takes_the_device(g):
    """A request admitted onto an idle server runs with every resident
    wavefront but the reserve; a large request admitted while it traverses gets
    the ordinary share and starts its traversal when the first one's ends.
    Both results, and those of small requests admitted meanwhile, equal the
    oracle's."""
    big, refs_big = _two_large()
    small = [synth.batch_member(700 + k) for k in range(10)]
    refs_small = oracle_members(small)
    _say(f"lone request then another: 2 x n={big[0].n} + {len(small)} small")
    with g.Server(max_inflight=4) as srv:
        ta = srv.submit(big[0].n, big[0].row_ptr, big[0].col_idx)
        time.sleep(0.02)
        tb = srv.submit(big[1].n, big[1].row_ptr, big[1].col_idx)
        ts = []
        for m in small:
            ts.append(srv.submit(m.n, m.row_ptr, m.col_idx))
            time.sleep(0.005)
        ra = srv.poll(ta, timeout_us=-1)
        rb = srv.poll(tb, timeout_us=-1)
        rs = [srv.poll(t, timeout_us=-1) for t in ts]
    ca, cb = ra.stats["concurrent_sources"], rb.stats["concurrent_sources"]
    _say(f"sources in flight: lone {ca}, admitted meanwhile {cb}")
    assert ca > cb and ca <= big[0].n
    assert same(ra, refs_big[0]) and same(rb, refs_big[1])
    for r, ref in zip(rs, refs_small):
        assert same(r, ref)


def test_serve_work_item_admission(g):
    """Two large requests with 4,096 sources in flight each fill the device;
    with GSOFA_SERVE_YIELD small requests admitted while they traverse make
    them yield (stop taking sources, let the small ones in, resume from the
    work counter). Every result equals the oracle's with and without yielding;
    with yielding at least one large traversal is relaunched, without it none
    is (a pool-regrowth re-run at most)."""
    big, refs_big = _two_large()
    small = [synth.batch_member(500 + k) for k in range(40)]
    refs_small = oracle_members(small)
    launches = {}
    for flags in (g.SERVE_YIELD, 0):
        _say(f"work-item admission, flags {flags:#x}: 2 x n={big[0].n} + {len(small)} small")
        with g.Server(max_inflight=4, concurrent_sources=4096, flags=flags) as srv:
            tb = [srv.submit(m.n, m.row_ptr, m.col_idx) for m in big]
            time.sleep(0.02)
            ts = []
            for m in small:
                ts.append(srv.submit(m.n, m.row_ptr, m.col_idx))
                time.sleep(0.01)
            rb = [srv.poll(t, timeout_us=-1) for t in tb]
            rs = [srv.poll(t, timeout_us=-1) for t in ts]
        launches[flags] = [r.stats["launches"] for r in rb]
        _say(f"large requests' traversal launches: {launches[flags]}")
        for r, ref in zip(rb, refs_big):
            assert same(r, ref)
        for r, ref in zip(rs, refs_small):
            assert same(r, ref)
    assert sum(launches[g.SERVE_YIELD]) >= 3
    assert max(launches[0]) <= 2


def test_serve_groups_many_small_requests(g):
    """Many small requests queued at once share launches (a worker takes the
    queued small requests that fit its budget together); every result must
    still equal the oracle's, also with a large request among them."""
    mats = [synth.batch_member(200 + k) for k in range(60)]
    mats.insert(30, synth.stencil(27, (30, 29, 28), nd=True, seed=301))
    _say(f"serve grouping: {len(mats)} requests")
    with g.Server(max_inflight=3) as srv:
        tickets = [srv.submit(m.n, m.row_ptr, m.col_idx) for m in mats]
        got = [srv.poll(t, timeout_us=-1) for t in tickets]
    for m, r in zip(mats, got):
        assert same(r, oracle.symbolic(m.n, m.row_ptr, m.col_idx))
