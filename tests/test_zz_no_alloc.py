"""The no-allocation entry point (gsofa_symbolic_noalloc) through the C ABI:
its arrays equal gsofa_symbolic's on the same input, bit for bit, on two calls
in a row (the second with a smaller matrix, over the scratch the first left
behind), it allocates no device memory, and it rejects what does not fit its
fixed scratch with GSOFA_ECAPACITY."""
import sys

import numpy as np
import pytest

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


def _outputs(n, u_cap, l_cap):
    import torch
    d = "cuda"
    return dict(u_ptr=torch.full((n + 1,), -7, dtype=torch.int64, device=d),
                u_idx=torch.full((max(u_cap, 1),), -7, dtype=torch.int32, device=d),
                l_ptr=torch.full((n + 1,), -7, dtype=torch.int64, device=d),
                l_idx=torch.full((max(l_cap, 1),), -7, dtype=torch.int32, device=d),
                xsup=torch.full((n + 1,), -7, dtype=torch.int32, device=d),
                supno=torch.full((max(n, 1),), -7, dtype=torch.int32, device=d))


def _check_against_symbolic(g, m, flags=0, **kw):
    import torch
    ref = g.symbolic(m.n, m.row_ptr, m.col_idx, flags=flags, **kw)
    rp = torch.from_numpy(m.row_ptr).cuda()
    ci = torch.from_numpy(m.col_idx).cuda()
    out = _outputs(m.n, ref.nnz_u + 3, ref.nnz_l + 3)
    torch.cuda.synchronize()
    before = g.memory_counters()
    _say(f"noalloc: {m.desc} n={m.n} flags={flags:#x}")
    c = g.symbolic_noalloc(m.n, rp, ci, **out, flags=flags, **kw)
    after = g.memory_counters()
    assert after[1] == before[1], "hipMalloc was called"
    assert after[3] == before[3], "an allocator was called"
    assert c["nnz_u"] == ref.nnz_u and c["nnz_l"] == ref.nnz_l and c["fills"] == ref.fills
    assert c["nnz_a"] == m.nnz
    assert c["stats"]["edges_alg"] == ref.stats["edges_alg"]
    assert np.array_equal(out["u_ptr"].cpu().numpy(), ref.u_ptr)
    assert np.array_equal(out["u_idx"][:ref.nnz_u].cpu().numpy(), ref.u_idx)
    assert np.array_equal(out["l_ptr"].cpu().numpy(), ref.l_ptr)
    assert np.array_equal(out["l_idx"][:ref.nnz_l].cpu().numpy(), ref.l_idx)
    if flags & g.NO_SUPERNODES:
        assert c["nsuper"] == 0
    else:
        assert c["nsuper"] == ref.nsuper
        assert np.array_equal(out["xsup"][:ref.nsuper + 1].cpu().numpy(), ref.xsup)
        assert np.array_equal(out["supno"][:m.n].cpu().numpy(), ref.supno)
    assert c["scratch_bytes"] <= g.NOALLOC_SCRATCH_BYTES
    return c


def test_noalloc_two_calls_second_smaller(g):
    big = synth.stencil(27, (16, 15, 14), nd=True, seed=91)
    small = synth.stencil(9, (30, 25), nd=True, seed=92)
    assert small.n < big.n
    _check_against_symbolic(g, big)
    _check_against_symbolic(g, small)


@pytest.mark.parametrize("flags_name", ["l_csr", "no_supernodes", "wave7", "line95_off"])
def test_noalloc_options(g, flags_name):
    flags = {"l_csr": g.L_CSR, "no_supernodes": g.NO_SUPERNODES, "wave7": g.MAP_WAVE32_7,
             "line95_off": g.NO_LINE95}[flags_name]
    m = synth.batch_member(33)
    _check_against_symbolic(g, m, flags=flags)
    _check_against_symbolic(g, synth.config(1), flags=flags, max_supernode=16, window=8)


def test_noalloc_empty_and_tiny(g):
    import torch
    out = _outputs(0, 0, 0)
    rp = torch.zeros(1, dtype=torch.int32, device="cuda")
    ci = torch.zeros(1, dtype=torch.int32, device="cuda")
    c = g.symbolic_noalloc(0, rp, ci, **out)
    assert c["nnz_u"] == 0 and c["nnz_l"] == 0 and c["nsuper"] == 0
    assert out["u_ptr"].cpu().tolist() == [0] and out["l_ptr"].cpu().tolist() == [0]
    assert out["xsup"].cpu().tolist() == [0]
    m = synth.stencil(5, (1, 1), nd=False, seed=3)
    _check_against_symbolic(g, m)


def test_noalloc_rejects_what_does_not_fit(g):
    import torch
    m = synth.stencil(9, (40, 40), nd=True, seed=93)
    ref = g.symbolic(m.n, m.row_ptr, m.col_idx)
    rp = torch.from_numpy(m.row_ptr).cuda()
    ci = torch.from_numpy(m.col_idx).cuda()
    # output capacity below nnz(U): the totals come back for a retry
    out = _outputs(m.n, ref.nnz_u - 1, ref.nnz_l)
    with pytest.raises(g.GsofaError) as e:
        g.symbolic_noalloc(m.n, rp, ci, **out)
    assert e.value.code == g.ECAPACITY
    assert e.value.counts["nnz_u"] == ref.nnz_u and e.value.counts["nnz_l"] == ref.nnz_l
    # per-row arrays alone beyond the scratch: rejected before any input is read
    huge = 3_000_000
    out = _outputs(4, 1, 1)
    with pytest.raises(g.GsofaError) as e:
        g.symbolic_noalloc(huge, rp, ci, u_ptr=out["u_ptr"], u_idx=out["u_idx"],
                           l_ptr=out["l_ptr"], l_idx=out["l_idx"], xsup=out["xsup"],
                           supno=out["supno"])
    assert e.value.code == g.ECAPACITY
    assert e.value.counts["scratch_bytes"] > g.NOALLOC_SCRATCH_BYTES
    # an output structure larger than the scratch: found after fill detection
    big = synth.stencil(27, (40, 40, 40), nd=True, seed=94)
    _say(f"noalloc overflow case: n={big.n}")
    rp = torch.from_numpy(big.row_ptr).cuda()
    ci = torch.from_numpy(big.col_idx).cuda()
    out = _outputs(big.n, 1, 1)
    with pytest.raises(g.GsofaError) as e:
        g.symbolic_noalloc(big.n, rp, ci, **out)
    assert e.value.code == g.ECAPACITY
    assert e.value.counts["scratch_bytes"] > g.NOALLOC_SCRATCH_BYTES
    # and the entry point still works afterwards
    _check_against_symbolic(g, m)


def test_noalloc_rejects_bad_input_and_options(g):
    import torch
    m = synth.batch_member(34)
    rp = torch.from_numpy(m.row_ptr).cuda()
    bad = m.col_idx.copy()
    bad[5] = m.n + 3
    ci = torch.from_numpy(bad).cuda()
    out = _outputs(m.n, 1 << 20, 1 << 20)
    with pytest.raises(g.GsofaError) as e:
        g.symbolic_noalloc(m.n, rp, ci, **out)
    assert e.value.code == g.EINVAL
    ci = torch.from_numpy(m.col_idx).cuda()
    for flags in (g.BUDGET_MODE, g.MAP_BYTE, g.TUNE_NOW):
        with pytest.raises(g.GsofaError) as e:
            g.symbolic_noalloc(m.n, rp, ci, **out, flags=flags)
        assert e.value.code == g.EINVAL
    _check_against_symbolic(g, m)
