"""The caller-allocator boundary (gsofa_opts dev_alloc / dev_free): with a
torch-backed allocator every device byte of a call comes from torch's caching
allocator -- the library makes no hipMalloc of its own and its cache does not
grow -- every block goes back, and the results still equal the oracle's."""
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


@pytest.mark.parametrize("flags_name", ["default", "eager", "tune_now"])
def test_symbolic_through_torch_allocator(g, flags_name):
    import torch
    flags = {"default": 0, "eager": g.EAGER, "tune_now": g.TUNE_NOW}[flags_name]
    m = synth.stencil(27, (14, 13, 12), nd=True, seed=81)
    ref = oracle.symbolic(m.n, m.row_ptr, m.col_idx)
    g.release_cache()
    before = g.memory_counters()
    al = g.TorchAllocator()
    stream = torch.cuda.current_stream().cuda_stream
    _say(f"allocator call {flags_name}: n={m.n}")
    res = g.symbolic(m.n, m.row_ptr, m.col_idx, flags=flags, allocator=al, stream=stream)
    _same(res, ref)
    after = g.memory_counters()
    assert after[1] == before[1], "the library called hipMalloc"
    assert after[0] == before[0], "the library's cache grew"
    assert al.allocs > 0 and after[3] - before[3] == al.allocs
    assert al.frees == al.allocs and not al.live, "blocks not returned"
    assert after[2] - before[2] == al.bytes


def test_device_results_through_torch_allocator(g):
    import torch
    m = synth.stencil(9, (40, 37), nd=True, seed=82)
    ref = oracle.symbolic(m.n, m.row_ptr, m.col_idx)
    g.release_cache()
    before = g.memory_counters()
    al = g.TorchAllocator()
    rp = torch.from_numpy(m.row_ptr).cuda()
    ci = torch.from_numpy(m.col_idx).cuda()
    d = g.symbolic(m.n, rp, ci, flags=g.RESULT_ON_DEVICE, allocator=al,
                   stream=torch.cuda.current_stream().cuda_stream)
    # the result arrays live in blocks the allocator handed out
    live = {p: t.numel() for p, t in al.live.items()}
    for k in ("u_ptr", "u_idx", "l_ptr", "l_idx", "xsup", "supno"):
        p = d.ptrs[k]
        assert any(b <= p < b + sz for b, sz in live.items()), k
    t = d.to_torch()
    assert np.array_equal(t["u_ptr"].cpu().numpy(), ref.u_ptr)
    assert np.array_equal(t["u_idx"].cpu().numpy(), ref.u_idx)
    assert np.array_equal(t["l_ptr"].cpu().numpy(), ref.l_ptr)
    assert np.array_equal(t["l_idx"].cpu().numpy(), ref.l_idx)
    assert np.array_equal(t["xsup"].cpu().numpy(), ref.xsup)
    assert np.array_equal(t["supno"].cpu().numpy(), ref.supno)
    assert al.live, "result blocks released before the result"
    d.free()
    assert not al.live and al.frees == al.allocs
    after = g.memory_counters()
    assert after[1] == before[1] and after[0] == before[0]


def test_batch_through_torch_allocator(g):
    mats = [synth.batch_member(k) for k in range(12)]
    g.release_cache()
    before = g.memory_counters()
    al = g.TorchAllocator()
    res = g.batch([(m.n, m.row_ptr, m.col_idx) for m in mats], allocator=al)
    for m, r in zip(mats, res):
        _same(r, oracle.symbolic(m.n, m.row_ptr, m.col_idx))
    after = g.memory_counters()
    assert after[1] == before[1] and after[0] == before[0]
    assert al.allocs > 0 and al.frees == al.allocs


def test_failing_allocator_reports_enomem(g):
    import torch
    m = synth.stencil(5, (30, 30), nd=False, seed=83)
    state = {"n": 0}

    def alloc(nbytes, ctx):
        state["n"] += 1
        return None

    o_alloc = g.ALLOC_FN(alloc)
    o_free = g.FREE_FN(lambda p, c: None)

    class Failing:
        def install(self, o):
            o.dev_alloc = o_alloc
            o.dev_free = o_free

    with pytest.raises(g.GsofaError) as e:
        g.symbolic(m.n, m.row_ptr, m.col_idx, allocator=Failing())
    assert e.value.code == g.ENOMEM and state["n"] >= 1
    # the library still works afterwards, with its own memory
    ref = oracle.symbolic(m.n, m.row_ptr, m.col_idx)
    _same(g.symbolic(m.n, m.row_ptr, m.col_idx), ref)
