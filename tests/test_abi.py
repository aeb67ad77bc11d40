"""The C-ABI library: it loads, exports every declared entry point, the
binding's struct layouts match the header, and argument errors are reported
without touching a GPU. CPU only."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "gsofa.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"GSOFA_API\s+[\w\s\*]*?\b(gsofa_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def g():
    import paper_2007_00840_amd as g
    if not os.path.exists(g.LIB_PATH):
        from paper_2007_00840_amd import _build
        _build.build(force=False)
    g.load()
    return g


def test_exports_every_declared_symbol(g):
    decl = _declared()
    assert len(decl) == len(g.EXPORTED) and set(decl) == set(g.EXPORTED)
    out = subprocess.run(["nm", "-D", "--defined-only", g.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (gsofa_\w+)", out))
    assert set(decl) <= exported
    lib = ctypes.CDLL(g.LIB_PATH)
    for name in decl:
        assert getattr(lib, name)


def test_struct_layout_matches_header(g, tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include "gsofa.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(gsofa_opts),'
                   ' sizeof(gsofa_result), sizeof(gsofa_stats), sizeof(gsofa_csr),'
                   ' offsetof(gsofa_result, stats), offsetof(gsofa_result, xsup),'
                   ' offsetof(gsofa_opts, stream), offsetof(gsofa_opts, queue_cap),'
                   ' offsetof(gsofa_stats, spilled_entries), offsetof(gsofa_stats, iterations));'
                   'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    want = [ctypes.sizeof(g.Opts), ctypes.sizeof(g.Result), ctypes.sizeof(g.Stats),
            ctypes.sizeof(g.Csr), g.Result.stats.offset, g.Result.xsup.offset, g.Opts.stream.offset,
            g.Opts.queue_cap.offset, g.Stats.spilled_entries.offset, g.Stats.iterations.offset]
    assert got == want


def test_strerror(g):
    for code in range(7):
        assert len(g.strerror(code)) > 0
    assert g.strerror(99) == "unknown status"


@pytest.mark.parametrize("case", ["neg_n", "bad_first", "non_monotone", "col_range", "duplicate",
                                  "neg_col"])
def test_invalid_csr_rejected_on_host(g, case):
    n = 4
    rp = np.array([0, 2, 3, 5, 6], dtype=np.int32)
    ci = np.array([0, 1, 1, 2, 3, 3], dtype=np.int32)
    if case == "neg_n":
        n = -1
    elif case == "bad_first":
        rp = rp + 1
    elif case == "non_monotone":
        rp = np.array([0, 3, 2, 5, 6], dtype=np.int32)
    elif case == "col_range":
        ci = ci.copy(); ci[3] = 4
    elif case == "duplicate":
        ci = np.array([0, 0, 1, 2, 3, 3], dtype=np.int32)
    elif case == "neg_col":
        ci = ci.copy(); ci[0] = -1
    with pytest.raises(g.GsofaError) as e:
        g.symbolic(n, rp, ci)
    assert e.value.code == g.EINVAL


def test_bad_opts_rejected(g):
    rp = np.array([0, 1], dtype=np.int32)
    ci = np.array([0], dtype=np.int32)
    for kw in ({"window": -1}, {"mem_budget_bytes": -5}, {"concurrent_sources": -2}):
        with pytest.raises(g.GsofaError) as e:
            g.symbolic(1, rp, ci, **kw)
        assert e.value.code == g.EINVAL
    lib = g.load()
    o = g.make_opts()
    o.struct_size = 4  # too small for this ABI
    out = ctypes.POINTER(g.Result)()
    assert lib.gsofa_symbolic(1, rp.ctypes.data, ci.ctypes.data, ctypes.byref(o),
                              ctypes.byref(out)) == g.EINVAL
    assert not out
    # an allocator needs both hooks: one alone is rejected before anything runs
    calls = []
    o = g.make_opts()
    o.dev_alloc = g.ALLOC_FN(lambda nbytes, ctx: calls.append(nbytes) or None)
    assert lib.gsofa_symbolic(1, rp.ctypes.data, ci.ctypes.data, ctypes.byref(o),
                              ctypes.byref(out)) == g.EINVAL
    o = g.make_opts()
    o.dev_free = g.FREE_FN(lambda ptr, ctx: calls.append(ptr))
    assert lib.gsofa_symbolic(1, rp.ctypes.data, ci.ctypes.data, ctypes.byref(o),
                              ctypes.byref(out)) == g.EINVAL
    assert not out and calls == []
    o = g.make_opts(queue_cap=-1)
    assert lib.gsofa_symbolic(1, rp.ctypes.data, ci.ctypes.data, ctypes.byref(o),
                              ctypes.byref(out)) == g.EINVAL


def test_order_above_limit_rejected(g):
    """n above GSOFA_MAX_N is refused before any array is read or any GPU call."""
    txt = open(HEADER).read()
    assert int(re.search(r"#define GSOFA_MAX_N (\d+)", txt).group(1)) == g.MAX_N == (1 << 30) - 1
    lib = g.load()
    rp = np.zeros(2, dtype=np.int32)
    ci = np.zeros(1, dtype=np.int32)
    out = ctypes.POINTER(g.Result)()
    for flags in (0, g.INPUT_ON_DEVICE):
        o = g.make_opts(flags=flags)
        assert lib.gsofa_symbolic(g.MAX_N + 1, rp.ctypes.data, ci.ctypes.data, ctypes.byref(o),
                                  ctypes.byref(out)) == g.EINVAL
        assert not out
    u_ptr = np.zeros(2, dtype=np.int64)
    l_ptr = np.zeros(2, dtype=np.int64)
    xs = np.zeros(2, dtype=np.int32)
    c = g.Counts()
    assert lib.gsofa_symbolic_noalloc(g.MAX_N + 1, rp.ctypes.data, ci.ctypes.data, None,
                                      u_ptr.ctypes.data, None, 0, l_ptr.ctypes.data, None, 0,
                                      xs.ctypes.data, xs.ctypes.data, ctypes.byref(c)) == g.EINVAL
    # a batch whose every member is refused runs nothing and reports each one
    for flags in (0, g.INPUT_ON_DEVICE):
        mats = (g.Csr * 2)(g.Csr(g.MAX_N + 1, rp.ctypes.data, ci.ctypes.data),
                           g.Csr(-1, rp.ctypes.data, ci.ctypes.data))
        outs = (ctypes.POINTER(g.Result) * 2)()
        o = g.make_opts(flags=flags)
        assert lib.gsofa_batch(2, mats, ctypes.byref(o), outs) == g.EINVAL
        for r in outs:
            assert r and r.contents.stats.status == g.EINVAL
            lib.gsofa_result_free(r)


def test_batch_argument_errors(g):
    lib = g.load()
    assert lib.gsofa_batch(-1, None, None, None) == g.EINVAL
    assert lib.gsofa_batch(2, None, None, None) == g.EINVAL
    assert lib.gsofa_batch(0, None, None, None) == g.OK


def test_serve_argument_errors(g):
    lib = g.load()
    assert lib.gsofa_serve_open(None, 1, None) == g.EINVAL
    out = ctypes.POINTER(g.Result)()
    assert lib.gsofa_serve_poll(None, 1, 0, ctypes.byref(out)) == g.EINVAL
    assert lib.gsofa_serve_close(None) == g.EINVAL


def test_graph_counters_argument_error(g):
    lib = g.load()
    assert lib.gsofa_graph_counters(None) == g.EINVAL
    a = g.graph_counters()
    assert len(a) == 3 and all(x >= 0 for x in a)


def test_memory_counters_argument_error(g):
    lib = g.load()
    assert lib.gsofa_memory_counters(None) == g.EINVAL
    a = g.memory_counters()
    assert len(a) == 5 and all(x >= 0 for x in a)


def test_bench_reads_its_traffic_record():
    """bench.py takes roofline.traffic from the committed PMC record only for
    the configuration the record names."""
    import os
    import sys
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, here)
    import bench
    import re
    text = open(os.path.join(here, "profiles", "k_traverse_64cube_27pt.md")).read()
    recs = list(re.finditer(r"traffic-record: kernel=(\S+) source_sha256_16=(\S+) mapping=(\d+) window=(\d+) "
                            r"sources=(\d+) fetch_bytes=(\d+) write_bytes=(\d+)", text))
    assert recs, "profile summary lacks its traffic record"
    windows = {int(m.group(4)) for m in recs}
    for m in recs:
        kernel, mapping, window, sources = m.group(1), int(m.group(3)), int(m.group(4)), int(m.group(5))
        want = int(m.group(6)) + int(m.group(7))
        got = bench.recorded_traffic(kernel, mapping, window, sources)
        if m.group(2) == bench.traversal_source_hash():
            assert got == want
        else:
            assert got is None  # the kernel changed since the counters were taken
        if window + 1 not in windows:
            assert bench.recorded_traffic(kernel, mapping, window + 1, sources) is None
        assert bench.recorded_traffic(kernel, mapping, window, sources + 4) is None


def test_host_result_views_keep_the_result_alive(g):
    """Host result arrays are numpy views of the library's memory; the library
    result is freed once, when the last of them is gone (binding logic only:
    a result assembled in host memory and a counting stand-in for
    gsofa_result_free)."""
    import gc

    n, nnz_l, nnz_u, nsuper = 5, 7, 6, 3
    arrs = {"l_ptr": np.arange(n + 1, dtype=np.int64), "u_ptr": np.arange(n + 1, dtype=np.int64) * 2,
            "l_idx": np.arange(nnz_l, dtype=np.int32) + 10, "u_idx": np.arange(nnz_u, dtype=np.int32) + 20,
            "xsup": np.array([0, 2, 4, 5], dtype=np.int32), "supno": np.array([0, 0, 1, 1, 2], dtype=np.int32)}
    res = g.Result()
    res.n, res.nnz_l, res.nnz_u, res.nsuper = n, nnz_l, nnz_u, nsuper
    for k, a in arrs.items():
        setattr(res, k, a.ctypes.data)
    rp = ctypes.pointer(res)
    freed = []

    class Lib:
        @staticmethod
        def gsofa_result_free(p):
            freed.append(ctypes.addressof(p.contents))

    r = g._to_host(rp, Lib)
    for k, a in arrs.items():
        v = getattr(r, k)
        assert np.array_equal(v, a) and v.ctypes.data == a.ctypes.data, k
    del v
    keep = r.u_idx
    del r
    gc.collect()
    assert freed == []
    assert np.array_equal(keep, arrs["u_idx"])
    del keep
    gc.collect()
    assert freed == [ctypes.addressof(res)]

    # an empty result: zero-length arrays, freed with the result object
    empty = g.Result()
    r = g._to_host(ctypes.pointer(empty), Lib)
    assert r.l_idx.size == 0 and r.u_ptr.size == 1 and r.xsup is None
    del r
    gc.collect()
    assert len(freed) == 2


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU per process: --gpus above 1 exits with a
    message (before touching a GPU)."""
    import json
    import sys
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]
