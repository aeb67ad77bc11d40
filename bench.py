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


def cpu_baseline(m, stride):
    """The oracle (fill2 search, all host threads) on every stride-th row."""
    import numpy as np
    import oracle
    rows = np.arange(m.n - 1, -1, -stride, dtype=np.int32)
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    cnt, lcnt, edges, ptr, ent = oracle.rows_struct(m.n, m.row_ptr, m.col_idx, rows, threads)
    dt = time.perf_counter() - t0
    e = int(edges.sum())
    return {"value": e / dt / 1e9, "unit": "GTEPS", "cores": threads, "kind": "oracle",
            "sample": f"{len(rows)} of {m.n} rows (every {stride}th, from the last), "
                      f"{e:.3e} algorithmic edges in {dt:.1f} s"}


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
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (calibrates "
                         "the FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
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
    m = synth.config(3)
    log(f"workload: {m.desc} n={m.n} nnz={m.nnz}")
    rp = torch.from_numpy(m.row_ptr).cuda()
    ci = torch.from_numpy(m.col_idx).cuda()
    stream = torch.cuda.current_stream().cuda_stream
    flags = g.RESULT_ON_DEVICE | args.flags
    kw = dict(flags=flags, window=args.window, concurrent_sources=args.slots, stream=stream)

    for i in range(args.warmup):
        t0 = time.perf_counter()
        r = g.symbolic(m.n, rp, ci, **kw)
        log(f"warmup {i}: {1e3 * (time.perf_counter() - t0):.1f} ms, "
            f"traverse {r.stats['t_traverse_ms']:.1f} ms")
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
    achieved = BYTES_PER_EDGE * e_alg / (t_trav * 1e-3) / 1e9
    log(f"steps: {ms:.1f} ms/step, traverse {t_trav:.1f} ms, emit {t_emit:.1f} ms, "
        f"supernode {t_sn:.1f} ms, {gteps:.1f} GTEPS")

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
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_traverse", "bytes_per_unit": BYTES_PER_EDGE,
                     "unit_count": e_alg, "kernel_ms": round(t_trav, 3)},
        "cpu_baseline": base,
        "edges_alg": e_alg,
        "edges_gpu": e_gpu,
        "revisit_ratio": round(e_gpu / max(e_alg, 1), 4),
        "nnz_l": nnz_l, "nnz_u": nnz_u, "fills": fills, "nsuper": nsuper,
        "fills_per_s": round(fills / (ms * 1e-3), 1),
        "t_traverse_ms": round(t_trav, 3), "t_emit_ms": round(t_emit, 3),
        "t_supernode_ms": round(t_sn, 3),
        "concurrent_sources": stats[-1]["concurrent_sources"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
