"""Benchmark of the symbolic LU factorisation hot path on one MI355X.

Default workload: the 3D 27-point stencil on a 64^3 grid (n = 262,144),
nested-dissection order, off-diagonals dropped with p = 0.2 (seed 3), int32
CSR resident in HBM. One step = one gsofa_symbolic call: input checks,
planning, fill detection, row sorting and CSR assembly, L transpose,
supernodes, with the result left in device memory.

Prints one JSON line: GTEPS (algorithmic edges / wall time per step), the
traversal kernel's algorithmic HBM rate against the 8 TB/s peak, and the CPU
oracle timed on a bounded sample of the same rows.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "symbolic GTEPS + achieved HBM GB/s; served matrices/s and p99 latency"
HBM_PEAK_GBS = 8000.0
BYTES_PER_EDGE = 8  # 4 B column index + 4 B label per algorithmic edge


def log(msg):
    print(msg, file=sys.stderr, flush=True)


TRAVERSAL_SOURCE_END = b"// ------------------------------------------------- byte-state variant"


def traversal_source_hash():
    """SHA-256 (16 hex digits) of the kernel source up to the byte-state
    section: the helpers and k_traverse, which the PMC record describes."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    src = open(os.path.join(here, "paper_2007_00840_amd", "csrc", "gsofa_kernels.hip"), "rb").read()
    end = src.find(TRAVERSAL_SOURCE_END)
    return hashlib.sha256(src[:end] if end >= 0 else src).hexdigest()[:16]


PROFILE_OF_WORKLOAD = {"3d": "k_traverse_64cube_27pt.md", "2d": "k_traverse_1000sq_9pt.md",
                       "batch": "k_traverse_batch4096.md"}


def recorded_traffic(kernel, mapping, window, sources, workload="3d"):
    """HBM bytes per launch of the traversal kernel from the rocprofv3 PMC record
    in profiles/ (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings),
    or None when no record matches this kernel source and configuration."""
    import re
    here = os.path.dirname(os.path.abspath(__file__))
    rec = os.path.join(here, "profiles", PROFILE_OF_WORKLOAD[workload])
    try:
        sha = traversal_source_hash()
        text = open(rec).read()
    except OSError:
        return None
    # one record per configuration the tuner may pick (its near-tie windows)
    for m in re.finditer(r"traffic-record: kernel=(\S+) source_sha256_16=(\S+) mapping=(\d+) window=(\d+) "
                         r"sources=(\d+) fetch_bytes=(\d+) write_bytes=(\d+)", text):
        if m.group(1) != kernel or m.group(2) != sha:
            continue
        if int(m.group(3)) != mapping or int(m.group(4)) != window or int(m.group(5)) != sources:
            continue
        return int(m.group(6)) + int(m.group(7))
    return None


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(m, stride, threads=None):
    """The oracle (fill2 search; all host threads unless given) on every
    stride-th row."""
    import numpy as np
    import oracle
    rows = np.arange(m.n - 1, -1, -stride, dtype=np.int32)
    threads = threads or oracle.default_threads()
    t0 = time.perf_counter()
    cnt, lcnt, edges, ptr, ent = oracle.rows_struct(m.n, m.row_ptr, m.col_idx, rows, threads)
    dt = time.perf_counter() - t0
    e = int(edges.sum())
    return {"value": e / dt / 1e9, "unit": "GTEPS", "cores": threads, "kind": "oracle",
            "cpu_model": host_cpu_model(),
            "sample": f"{len(rows)} of {m.n} rows (every {stride}th, from the last), "
                      f"{e:.3e} algorithmic edges in {dt:.2f} s"}


def cpu_baseline_batch(mats, every, threads=None):
    """The oracle on every `every`-th matrix of the batch, one call per matrix,
    all host threads unless given; reported as GTEPS and matrices/s."""
    import oracle
    threads = threads or oracle.default_threads()
    sub = mats[::every]
    t0 = time.perf_counter()
    e = 0
    for m in sub:
        e += int(oracle.rows_struct(m.n, m.row_ptr, m.col_idx, None, threads)[2].sum())
    dt = time.perf_counter() - t0
    return {"value": e / dt / 1e9, "unit": "GTEPS", "cores": threads, "kind": "oracle",
            "matrices_per_s": round(len(sub) / dt, 2), "cpu_model": host_cpu_model(),
            "sample": f"{len(sub)} of {len(mats)} matrices (every {every}th), "
                      f"{e:.3e} algorithmic edges in {dt:.2f} s"}


def roofline(e_alg, t_trav_ms, mapping, window, sources, workload):
    """Algorithmic HBM rate of the traversal kernel against the 8 TB/s peak
    (8 B per algorithmic edge), with the PMC traffic record if one matches."""
    kern = KERNEL_OF_MAPPING.get(mapping, "k_traverse<8>")
    achieved = BYTES_PER_EDGE * e_alg / (t_trav_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": recorded_traffic(kern, mapping, window, sources, workload),
            "kernel": kern, "bytes_per_unit": BYTES_PER_EDGE, "unit_count": e_alg,
            "kernel_ms": round(t_trav_ms, 3)}


def bench_batch(g, torch, synth, reps, cpu=True, single=True, window=0, extra_flags=0):
    """The 4,096-matrix batch (config 4): one gsofa_batch call against one
    gsofa_symbolic call per matrix, inputs and results in device memory."""
    import numpy as np
    t0 = time.perf_counter()
    mats = [synth.batch_member(k) for k in range(synth.BATCH_COUNT)]
    log(f"batch: generated {len(mats)} matrices in {time.perf_counter() - t0:.1f} s, "
        f"sum n = {sum(m.n for m in mats)}")
    dev = [(m.n, torch.from_numpy(m.row_ptr).cuda(), torch.from_numpy(m.col_idx).cuda()) for m in mats]
    stream = torch.cuda.current_stream().cuda_stream
    flags = g.RESULT_ON_DEVICE | extra_flags
    def phases_of(st):
        ph = {k: round(st[k], 3) for k in ("t_traverse_ms", "t_emit_ms", "t_supernode_ms", "t_total_ms")}
        ph["concurrent_sources"] = st["concurrent_sources"]
        ph["window"] = st["window"]
        ph["mapping"] = st["mapping"]
        return ph

    res = g.batch(dev, flags=flags, stream=stream, window=window)  # warm-up (tuning, output-pool sizing)
    e_alg = sum(r.stats["edges_alg"] for r in res)
    warm = phases_of(res[0].stats)
    warm["t_tune_ms"] = round(res[0].stats["t_tune_ms"], 3)
    phases = None
    for r in res:
        r.free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        res = g.batch(dev, flags=flags, stream=stream, window=window)
        phases = phases_of(res[0].stats)  # HIP-event phase times of the timed call
        for r in res:
            r.free()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    # the same batch launched kernel by kernel instead of one graph per phase
    t_eager = t_single = float("nan")
    if single:
        t0 = time.perf_counter()
        for _ in range(reps):
            res = g.batch(dev, flags=flags | g.EAGER, stream=stream, window=window)
            for r in res:
                r.free()
        torch.cuda.synchronize()
        t_eager = (time.perf_counter() - t0) / reps
        t0 = time.perf_counter()
        for n, rp, ci in dev:
            r = g.symbolic(n, rp, ci, flags=flags, stream=stream)
            r.free()
        torch.cuda.synchronize()
        t_single = time.perf_counter() - t0
    log(f"batch: {t_batch * 1e3:.1f} ms per batch, one call per matrix {t_single * 1e3:.1f} ms, "
        f"edges_alg {e_alg:.3e}, phases {phases}")
    roof = roofline(e_alg, phases["t_traverse_ms"], phases["mapping"], phases["window"],
                    phases["concurrent_sources"], "batch")
    base = base1 = None
    if cpu:
        log("batch: cpu baseline (oracle on every 16th matrix, all threads; every 64th, one thread)")
        base = cpu_baseline_batch(mats, 16)
        base1 = cpu_baseline_batch(mats, 64, threads=1)
        log(f"batch cpu: {base} / one thread {base1}")
    return {"matrices": len(mats), "sum_n": int(sum(m.n for m in mats)), "edges_alg": e_alg,
            "roofline": roof, "cpu_baseline": base, "cpu_baseline_1thread": base1,
            "ms_per_batch": round(t_batch * 1e3, 3),
            "eager_ms_per_batch": round(t_eager * 1e3, 3),
            "graph_counters": list(g.graph_counters()),
            "matrices_per_s": round(len(mats) / t_batch, 1),
            "gteps": round(e_alg / t_batch / 1e9, 3),
            "one_call_per_matrix_ms": round(t_single * 1e3, 3),
            "one_call_per_matrix_matrices_per_s": round(len(mats) / t_single, 1),
            "speedup_vs_one_call_per_matrix": round(t_single / t_batch, 3),
            "phases_ms": phases, "warmup_phases_ms": warm}


def bench_ablations(g, torch, synth, m, rp, ci):
    """The paper's ablations on the headline workload, one call each after a
    warm-up: the access-order check off (line 9.5), the paper's breadth-first
    frontier order instead of windows, 32-bit labels vs byte states, the window
    span, the label array reset before every source instead of the value-range
    scheme (maxId re-initialisation, Section 4), and the memory-budget mode at
    16, 5 and 1 GB of source-slot state (the budgets of the paper's space
    study). Results are identical; time, revisits and sources in flight differ."""
    stream = torch.cuda.current_stream().cuda_stream
    cases = [("windowed, window 16 (default)", dict(window=16, flags=g.MAP_WAVE32)),
             ("windowed, window 64", dict(window=64, flags=g.MAP_WAVE32)),
             ("access-order check off (line 9.5)", dict(window=16, flags=g.MAP_WAVE32 | g.NO_LINE95)),
             ("breadth-first order (paper)", dict(flags=g.MAP_WAVE32 | g.LEVEL_ORDER)),
             ("byte states, window 16", dict(window=16, flags=g.MAP_BYTE)),
             ("labels reset before every source (no maxId re-init scheme)",
              dict(window=16, flags=g.MAP_WAVE32 | g.RESET_LABELS))]
    for gb in (16, 5, 1):
        cases.append((f"memory budget {gb} GB (bands, host spill)",
                      dict(window=16, flags=g.BUDGET_MODE, mem_budget_bytes=gb << 30)))
    out = []
    ref = None
    base_ms = None
    for name, kw in cases:
        kw = dict(kw)
        kw["flags"] |= g.RESULT_ON_DEVICE | g.NO_TUNE
        r = g.symbolic(m.n, rp, ci, stream=stream, **kw)  # warm-up (slot sets, pool size)
        r.free()
        r = g.symbolic(m.n, rp, ci, stream=stream, **kw)
        st = r.stats
        fills = r.fills
        r.free()
        torch.cuda.synchronize()
        if ref is None:
            ref = fills
            base_ms = st["t_traverse_ms"]
        row = {"case": name, "t_traverse_ms": round(st["t_traverse_ms"], 3),
               "slowdown_vs_default": round(st["t_traverse_ms"] / base_ms, 3), "edges_alg": st["edges_alg"],
               "edges_gpu": st["edges_gpu"], "revisit_ratio": round(st["edges_gpu"] / max(st["edges_alg"], 1), 4),
               "levels": st["iterations"], "windows": st["windows"],
               "concurrent_sources": st["concurrent_sources"], "launches": st["launches"],
               "spilled_entries": st["spilled_entries"], "same_fills": fills == ref}
        log(f"ablation: {row}")
        out.append(row)
    return out


def bench_baselines(g, torch, synth, gp_cap_s):
    """Comparison baselines on the three single-matrix workloads: the fill2
    search with one GPU thread per source (the paper's GPU fill2 comparison)
    against the default kernel, and the CPU Gilbert-Peierls column-by-column
    symbolic factorisation (one thread, stopped after gp_cap_s seconds on the
    larger workloads; then the columns done are reported)."""
    import baselines
    out = []
    stream = torch.cuda.current_stream().cuda_stream
    for cfg in (1, 2, 3):
        m = synth.config(cfg)
        rp = torch.from_numpy(m.row_ptr).cuda()
        ci = torch.from_numpy(m.col_idx).cuda()
        row = {"config": cfg, "workload": m.desc, "n": m.n}
        for name, flags in (("default", 0), ("thread_per_source_fill2", g.MAP_THREAD)):
            kw = dict(flags=flags | g.RESULT_ON_DEVICE | g.NO_TUNE, stream=stream)
            if flags == 0 or cfg == 1:
                # warm-up (the one-thread baseline runs for tens of seconds on the
                # larger workloads, where a warm-up would change nothing)
                r = g.symbolic(m.n, rp, ci, **kw)
                r.free()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = g.symbolic(m.n, rp, ci, **kw)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0)
            row[name] = {"ms": round(ms, 3), "t_traverse_ms": round(r.stats["t_traverse_ms"], 3),
                         "gteps": round(r.stats["edges_alg"] / ms / 1e6, 3),
                         "concurrent_sources": r.stats["concurrent_sources"]}
            row["edges_alg"] = r.stats["edges_alg"]
            r.free()
        row["default_speedup_vs_thread_per_source"] = round(
            row["thread_per_source_fill2"]["ms"] / row["default"]["ms"], 2)
        gp = baselines.gilbert_peierls(m.n, m.row_ptr, m.col_idx, time_limit_s=gp_cap_s)
        row["cpu_gilbert_peierls"] = {"seconds": round(gp.seconds, 3), "columns_done": gp.cols_done,
                                      "complete": gp.cols_done == m.n, "threads": 1,
                                      "l_entries_scanned": gp.edges, "cpu_model": host_cpu_model()}
        if gp.cols_done == m.n:
            row["default_speedup_vs_cpu_gilbert_peierls"] = round(1e3 * gp.seconds / row["default"]["ms"], 1)
        log(f"baselines: {row}")
        out.append(row)
    return out


def bench_config1(g, torch, synth, steps, cpu=True):
    """The tiny workload (40 x 40 5-point stencil, natural order): GPU time per
    call and the oracle on all host threads and on one thread."""
    m = synth.config(1)
    rp = torch.from_numpy(m.row_ptr).cuda()
    ci = torch.from_numpy(m.col_idx).cuda()
    stream = torch.cuda.current_stream().cuda_stream
    r = g.symbolic(m.n, rp, ci, flags=g.RESULT_ON_DEVICE, stream=stream)
    r.free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = g.symbolic(m.n, rp, ci, flags=g.RESULT_ON_DEVICE, stream=stream)
        st = r.stats
        r.free()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    out = {"workload": "2D 5-point stencil 40x40, natural order, drop 0.2, seed 1", "n": m.n,
           "ms_per_call": round(ms, 3), "gteps": round(st["edges_alg"] / ms / 1e6, 3),
           "edges_alg": st["edges_alg"], "t_traverse_ms": round(st["t_traverse_ms"], 3)}
    if cpu:
        out["cpu_baseline"] = cpu_baseline(m, 1)
        out["cpu_baseline_1thread"] = cpu_baseline(m, 1, threads=1)
    log(f"config 1: {out}")
    return out


def bench_2d(g, torch, synth, steps, cpu=True, window=0, extra_flags=0):
    """The 2D workload (9-point stencil on a 1000 x 1000 grid, nested
    dissection, drop 0.2): one warm-up call (tunes its size class), then
    `steps` timed calls, inputs and results in device memory."""
    m = synth.config(2)
    log(f"2d: {m.desc} n={m.n} nnz={m.nnz}")
    rp = torch.from_numpy(m.row_ptr).cuda()
    ci = torch.from_numpy(m.col_idx).cuda()
    stream = torch.cuda.current_stream().cuda_stream
    kw = dict(flags=g.RESULT_ON_DEVICE | extra_flags, window=window, stream=stream)
    r = g.symbolic(m.n, rp, ci, **kw)
    tune_ms = r.stats["t_tune_ms"]
    r.free()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        r = g.symbolic(m.n, rp, ci, **kw)
        stats.append(r.stats)
        fills = r.fills
        r.free()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    e_alg = stats[-1]["edges_alg"]
    t_trav = sum(x["t_traverse_ms"] for x in stats) / steps
    out = {"workload": "2D 9-point stencil 1000x1000, nested dissection, drop 0.2, seed 2",
           "n": m.n, "nnz": m.nnz, "ms_per_call": round(ms, 3), "gteps": round(e_alg / ms / 1e6, 3),
           "edges_alg": e_alg, "fills": fills, "t_traverse_ms": round(t_trav, 3),
           "traverse_algorithmic_gbs": round(BYTES_PER_EDGE * e_alg / t_trav / 1e6, 1),
           "traverse_frac_of_hbm_peak": round(BYTES_PER_EDGE * e_alg / t_trav / 1e6 / HBM_PEAK_GBS, 4),
           "t_emit_ms": round(sum(x["t_emit_ms"] for x in stats) / steps, 3),
           "window": stats[-1]["window"], "mapping": stats[-1]["mapping"],
           "concurrent_sources": stats[-1]["concurrent_sources"], "t_tune_ms_warmup": round(tune_ms, 3)}
    out["roofline"] = roofline(e_alg, t_trav, stats[-1]["mapping"], stats[-1]["window"],
                               stats[-1]["concurrent_sources"], "2d")
    if cpu:
        log("2d: cpu baseline (oracle on every row, all threads)")
        out["cpu_baseline"] = cpu_baseline(m, 1)
    log(f"2d: {out}")
    return out


def _serve_run(g, synth, trace, cap_s, mode, drain_s=0.0, max_inflight=4, max_outstanding=64):
    """Offers the requests of the trace that arrive within cap_s seconds, on
    their arrival schedule, and waits up to drain_s more for them to finish.
    mode 'serve' uses the continuous-batching server, 'plain' one
    gsofa_symbolic call at a time in arrival order; neither runs tuner trials.
    Latency = completion - scheduled arrival; requests not finished by
    cap_s + drain_s count as censored."""
    import threading
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    done_at = {}
    pool = ThreadPoolExecutor(max_workers=8)
    futs = {}
    arrived = [r for r in trace if r.arrival_s <= cap_s]
    for r in arrived[:2 * max_outstanding]:
        futs[r.rid] = pool.submit(r.matrix)
    t0 = time.perf_counter()
    nxt = 0
    end_s = cap_s + drain_s
    if mode == "serve":
        srv = g.Server(max_inflight=max_inflight, mem_budget_bytes=200 << 30)
        outstanding = {}
        while True:
            now = time.perf_counter() - t0
            if now > end_s or len(done_at) == len(arrived):
                break
            # submit everything that has arrived, within the outstanding bound
            while (nxt < len(arrived) and arrived[nxt].arrival_s <= now
                   and len(outstanding) < max_outstanding):
                r = arrived[nxt]
                m = futs.pop(r.rid).result()
                k = nxt + 2 * max_outstanding
                if k < len(arrived):
                    futs[arrived[k].rid] = pool.submit(arrived[k].matrix)
                outstanding[srv.submit(m.n, m.row_ptr, m.col_idx)] = r
                nxt += 1
            for t in list(outstanding):
                res = srv.poll(t, timeout_us=0)
                if res is not None:
                    done_at[outstanding.pop(t).rid] = time.perf_counter() - t0
            time.sleep(0.0005)
        srv.close()
    else:
        while nxt < len(arrived):
            now = time.perf_counter() - t0
            if now > end_s:
                break
            r = arrived[nxt]
            if r.arrival_s > now:
                time.sleep(min(r.arrival_s - now, 0.01))
                continue
            m = futs.pop(r.rid).result()
            k = nxt + 2 * max_outstanding
            if k < len(arrived):
                futs[arrived[k].rid] = pool.submit(arrived[k].matrix)
            g.symbolic(m.n, m.row_ptr, m.col_idx, flags=g.NO_TUNE)
            done_at[r.rid] = time.perf_counter() - t0
            nxt += 1
    pool.shutdown(wait=False, cancel_futures=True)
    lat = np.array([done_at[r.rid] - r.arrival_s if r.rid in done_at else np.inf for r in arrived])
    lat.sort()
    def pct(q):
        v = lat[min(len(lat) - 1, int(np.ceil(q * len(lat))) - 1)]
        return round(float(v) * 1e3, 1) if np.isfinite(v) else f"> {end_s * 1e3:.0f} (censored)"
    span = max(done_at.values()) if done_at else end_s
    return {"offered": len(arrived), "completed": len(done_at),
            "completed_per_s": round(len(done_at) / max(span, 1e-9), 2),
            "p50_ms": pct(0.5), "p99_ms": pct(0.99),
            "censored_frac": round(float(np.mean(~np.isfinite(lat))), 4)}


def bench_serve(g, synth, cap_s, low_rate):
    """The request stream: Poisson arrivals at 200 requests/s, n log-uniform
    in [1e3, 1e6], 2D 9-point or 3D 27-point, ND order, drop 0.2, memory
    budget 200 GB; offered for cap_s seconds. That rate is far above what one
    GPU completes, so most latencies are censored; the same request mix at
    low_rate requests/s, drained to the end, gives the latency distribution."""
    trace = synth.serve_trace()
    log(f"serve: {len(trace)} requests in the 60 s trace; offering the first {cap_s:.0f} s")
    out = {"cap_s": cap_s, "rate_per_s": synth.SERVE_RATE}
    out["continuous_batching"] = _serve_run(g, synth, trace, cap_s, "serve")
    log(f"serve: {out['continuous_batching']}")
    out["plain_sequential"] = _serve_run(g, synth, trace, cap_s, "plain")
    log(f"serve plain: {out['plain_sequential']}")
    a = out["continuous_batching"]["completed"]
    b = out["plain_sequential"]["completed"]
    out["throughput_vs_plain"] = round(a / b, 3) if b else None
    if low_rate > 0:
        low = synth.serve_trace(rate=low_rate)
        low_cap = min(cap_s / 2, 10.0)
        res = {"rate_per_s": low_rate, "cap_s": low_cap, "drain_s": 3 * low_cap}
        res["continuous_batching"] = _serve_run(g, synth, low, low_cap, "serve", drain_s=3 * low_cap)
        log(f"serve at {low_rate}/s: {res['continuous_batching']}")
        res["plain_sequential"] = _serve_run(g, synth, low, low_cap, "plain", drain_s=3 * low_cap)
        log(f"serve plain at {low_rate}/s: {res['plain_sequential']}")
        out["low_rate"] = res
    return out


def _admission_run(g, big, small, flags, gap_s=0.01):
    """Two copies of a large request (none if big is None), then the small
    requests one every gap_s seconds, on a server whose large requests fill
    the device (4 workers, each lone large request with half the resident
    wavefronts less a small reserve). Returns the small
    requests' latencies (completion - submission) and the large ones'
    completion times and traversal launches."""
    import numpy as np
    srv = g.Server(max_inflight=4, flags=flags, mem_budget_bytes=200 << 30)
    t0 = time.perf_counter()
    tb = [srv.submit(big.n, big.row_ptr, big.col_idx) for _ in range(2)] if big is not None else []
    time.sleep(0.02)
    sub, done, big_done, big_launches, st_of = {}, {}, {}, {}, {}
    pending = set()
    k = 0
    nxt = time.perf_counter()
    while len(done) < len(small) or len(big_done) < len(tb):
        now = time.perf_counter()
        if k < len(small) and now >= nxt:
            m = small[k]
            t = srv.submit(m.n, m.row_ptr, m.col_idx)
            sub[t] = time.perf_counter()
            pending.add(t)
            k += 1
            nxt += gap_s
        for t in list(pending):
            r = srv.poll(t, timeout_us=0)
            if r is not None:
                done[t] = time.perf_counter() - sub[t]
                st_of[t] = (round(r.stats["t_total_ms"], 1), round(r.stats["t_traverse_ms"], 1))
                pending.discard(t)
        for t in tb:
            if t not in big_done:
                r = srv.poll(t, timeout_us=0)
                if r is not None:
                    big_done[t] = time.perf_counter() - t0
                    big_launches[t] = r.stats["launches"]
        if now - t0 > 60:
            break
        time.sleep(0.0002)
    srv.close()
    out = {"large_done_ms": sorted(round(1e3 * v, 1) for v in big_done.values()),
           "large_launches": [big_launches[t] for t in tb if t in big_launches]}
    if done:
        lat = np.sort(np.array(list(done.values())))
        pct = lambda q: round(1e3 * float(lat[min(len(lat) - 1, int(np.ceil(q * len(lat))) - 1)]), 2)
        out.update({"small_completed": len(done), "small_p50_ms": pct(0.5), "small_p99_ms": pct(0.99),
                    "small_max_ms": round(1e3 * float(lat[-1]), 2)})
        # the slowest small requests: (submission after the start, latency, the
        # engine call's wall time, its traversal time), ms
        slow = sorted(done, key=lambda t: -done[t])[:5]
        out["small_slowest"] = [(round(1e3 * (sub[t] - t0), 1), round(1e3 * done[t], 1)) + st_of[t]
                                for t in slow]
    return out


def bench_admission(g, synth, big):
    """Latency of small requests (4,096-matrix batch members, one every
    10 ms) submitted while two large requests (the 64^3 27-point stencil) fill
    the device: on an idle device, with the default server (a reserve of wave
    slots, copies as the library's own small-workgroup kernels), and with the
    large traversals also yielding their wave slots (GSOFA_SERVE_YIELD); the
    large requests alone for their cost."""
    small = [synth.batch_member(9000 + k) for k in range(60)]
    out = {"large": f"2 x {big.desc}", "small": f"{len(small)} batch members, one every 10 ms"}
    _admission_run(g, big, small[:8], 0)  # warm-up: size classes, slot sets
    out["idle"] = _admission_run(g, None, small, 0)  # the small requests on an idle device
    log(f"admission idle: {out['idle']}")
    out["large_only"] = _admission_run(g, big, [], 0)  # the large requests without small ones
    log(f"admission large only: {out['large_only']}")
    for name, flags in (("default", 0), ("yield", g.SERVE_YIELD)):
        out[name] = _admission_run(g, big, small, flags)
        log(f"admission {name}: {out[name]}")
    return out


# traversal kernel launched for each mapping code reported in the stats
KERNEL_OF_MAPPING = {3: "k_traverse8", 0: "k_traverse<8>", 4: "k_traverse<7>", 2: "k_traverse_wg<8>",
                     1: "k_traverse_wg<16>", 5: "k_traverse<6, true>", 6: "k_fill2_thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-stride", type=int, default=1,
                    help="oracle baseline on every k-th row (0 = skip)")
    ap.add_argument("--window", type=int, default=0)
    ap.add_argument("--slots", type=int, default=0)
    ap.add_argument("--flags", type=int, default=0)
    ap.add_argument("--twod-steps", type=int, default=2, help="timed calls on the 2D workload (0 = skip)")
    ap.add_argument("--skip-ablations", action="store_true",
                    help="do not time the paper's ablations on the headline workload")
    ap.add_argument("--batch-reps", type=int, default=3, help="0 = skip the batch measurement")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="arrivals offered and wall cap of the request-stream measurement, in seconds; "
                         "60 offers the whole trace (0 = skip)")
    ap.add_argument("--baselines-cap", type=float, default=15.0,
                    help="seconds the CPU Gilbert-Peierls baseline may run per workload (0 = skip the "
                         "comparison baselines)")
    ap.add_argument("--serve-low-rate", type=float, default=1.0,
                    help="requests/s of the drained low-rate request stream (0 = skip)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (calibrates "
                         "the FETCH_SIZE / WRITE_SIZE counters) and exit")
    ap.add_argument("--admission", type=int, default=1,
                    help="1 = measure small-request latency behind large requests with and "
                         "without work-item admission (0 = skip)")
    ap.add_argument("--only", choices=["2d", "batch", "admission"], default=None,
                    help="time only this workload (with --window / --flags pinned; for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the symbolic engine runs on one GPU per process; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import synth
    import paper_2007_00840_amd as g

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes}))
        return
    if args.only == "2d":
        print(json.dumps(bench_2d(g, torch, synth, max(args.twod_steps, 1), False, args.window, args.flags)))
        return
    if args.only == "batch":
        print(json.dumps(bench_batch(g, torch, synth, max(args.batch_reps, 1), False, False, args.window,
                                     args.flags), default=str))
        return
    m = synth.config(3)
    if args.only == "admission":
        print(json.dumps(bench_admission(g, synth, m)))
        return
    log(f"workload: {m.desc} n={m.n} nnz={m.nnz}")
    rp = torch.from_numpy(m.row_ptr).cuda()
    ci = torch.from_numpy(m.col_idx).cuda()
    stream = torch.cuda.current_stream().cuda_stream
    flags = g.RESULT_ON_DEVICE | args.flags
    kw = dict(flags=flags, window=args.window, concurrent_sources=args.slots, stream=stream)

    warm_stats = []
    for i in range(args.warmup):
        t0 = time.perf_counter()
        r = g.symbolic(m.n, rp, ci, **kw)
        warm_stats.append(r.stats)
        log(f"warmup {i}: {1e3 * (time.perf_counter() - t0):.1f} ms, "
            f"traverse {r.stats['t_traverse_ms']:.1f} ms, tuner {r.stats['t_tune_ms']:.1f} ms -> "
            f"mapping {r.stats['mapping']} window {r.stats['window']} "
            f"sources {r.stats['concurrent_sources']}")
        r.free()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = g.symbolic(m.n, rp, ci, **kw)
        stats.append(r.stats)
        nnz_l, nnz_u, nsuper, fills = r.nnz_l, r.nnz_u, r.nsuper, r.fills
        r.free()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = 1e3 * dt / args.steps
    e_alg = stats[-1]["edges_alg"]
    e_gpu = stats[-1]["edges_gpu"]
    t_trav = sum(s["t_traverse_ms"] for s in stats) / len(stats)
    t_emit = sum(s["t_emit_ms"] for s in stats) / len(stats)
    t_sn = sum(s["t_supernode_ms"] for s in stats) / len(stats)
    gteps = e_alg / (ms * 1e-3) / 1e9
    log(f"steps: {ms:.1f} ms/step, traverse {t_trav:.1f} ms, emit {t_emit:.1f} ms, "
        f"supernode {t_sn:.1f} ms, {gteps:.1f} GTEPS")

    ablations = None if args.skip_ablations else bench_ablations(g, torch, synth, m, rp, ci)
    cpu_legs = args.cpu_stride > 0
    cfg1 = bench_config1(g, torch, synth, max(args.steps, 3), cpu_legs)
    twod = bench_2d(g, torch, synth, args.twod_steps, cpu_legs) if args.twod_steps > 0 else None
    g.release_cache()  # the 2D workload's slot sets are not reused below
    batch = bench_batch(g, torch, synth, args.batch_reps, cpu_legs) if args.batch_reps > 0 else None
    base_cmp = bench_baselines(g, torch, synth, args.baselines_cap) if args.baselines_cap > 0 else None
    g.release_cache()
    serve = bench_serve(g, synth, args.serve_seconds, args.serve_low_rate) if args.serve_seconds > 0 else None
    if serve is not None and args.admission:
        serve["admission"] = bench_admission(g, synth, m)

    base = None
    if args.cpu_stride > 0:
        log(f"cpu baseline: oracle on every {args.cpu_stride}th row ...")
        base = cpu_baseline(m, args.cpu_stride)
        log(f"cpu baseline: {base['value']:.3f} GTEPS on {base['cores']} threads")

    out = {
        "metric": METRIC,
        "value": round(gteps, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "3D 27-point stencil 64x64x64, nested dissection, drop 0.2, seed 3",
                   "n": m.n, "nnz": m.nnz, "result": "device-resident L (CSC), U (CSR), supernodes",
                   "max_supernode": 128, "parallelism": "single GPU"},
        "roofline": roofline(e_alg, t_trav, stats[-1]["mapping"], stats[-1]["window"],
                             stats[-1]["concurrent_sources"], "3d"),
        "cpu_baseline": base,
        "edges_alg": e_alg,
        "edges_gpu": e_gpu,
        "revisit_ratio": round(e_gpu / max(e_alg, 1), 4),
        "nnz_l": nnz_l, "nnz_u": nnz_u, "fills": fills, "nsuper": nsuper,
        "fills_per_s": round(fills / (ms * 1e-3), 1),
        "t_traverse_ms": round(t_trav, 3), "t_emit_ms": round(t_emit, 3),
        "t_supernode_ms": round(t_sn, 3),
        "concurrent_sources": stats[-1]["concurrent_sources"],
        "window": stats[-1]["window"], "mapping": stats[-1]["mapping"],
        "t_tune_ms_warmup": round(max(s["t_tune_ms"] for s in warm_stats), 3) if warm_stats else 0.0,
        "ablations": ablations,
        "workload_1": cfg1,
        "workload_2d": twod,
        "baselines": base_cmp,
        "batch": batch,
        "serve": serve,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
