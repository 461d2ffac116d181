#!/usr/bin/env python3
"""Benchmark of the aggregate risk analysis hot path on one MI355X.

A step is one whole analysis of one layer over the resident YET, every stage of
the path in libara's kernels:
  1. ELT direct access tables rebuilt from the resident (event, loss) records,
     combined table and occurrence filter (ara_layer_build with ARA_BUILD_TABLES);
  2. the trial kernel: YLT of every trial, with the event-ID range checks of the
     YET fused into the same pass (ara_analyze);
  3. descending radix sort of the YLT and PML/TVaR at the return periods, results
     copied to the host (ara_risk_measures, blocking).

Default workload: the paper's headline shape -- 1,000,000 trials x 1,000 events,
IDs uniform over a 1,000,000-event catalog, one layer of 16 ELTs x 20,000
lognormal(11, 2.5) losses, occurrence R/L 1e5/5e6, aggregate R/L 1e6/5e7,
binary64 (synthetic data; the paper's industrial inputs are not public).

Prints one JSON line.  `value` = trial-events x layers per second of the whole
step; `roofline` rates the trial kernel against HBM bandwidth with algorithmic
bytes (event IDs + offsets + YLT + the layer's filter tables, each once) over its
average duration measured with events on the kernel's stream; `cpu_baseline`
times the CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["paper", "small"], default="paper")
    ap.add_argument("--trials", type=int, default=1_000_000)
    ap.add_argument("--precision", choices=["f64", "f32"], default="f64")
    ap.add_argument("--placement", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--grid-per-cu", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU-oracle sample time (0 = skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one plain device copy of this size (for counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(multi-GPU sharding is a design note, not implemented)"}))
        sys.exit(2)

    import torch
    import synth
    from paper_1308_2066_amd import ara, session

    t = time.time()
    if args.workload == "paper":
        w = synth.workload_paper_scale(n_trials=args.trials)
        wname = (f"paper-scale plain ARA: {w.n_trials} trials x 1000 events, catalog {w.catalog_size}, "
                 f"1 layer of {len(w.elts)} ELTs x 20000 lognormal(11,2.5), occ 1e5/5e6, agg 1e6/5e7")
    else:
        w = synth.workload_plain_small()
        wname = ("plain ARA: 10000 trials, Poisson(100) events, catalog 10000, 1 layer of 4 ELTs x 2000 "
                 "lognormal(10,2), occ 5e4/1e6, agg 2e5/5e6")
    log(f"generated {w.name}: {w.n_events} events in {time.time() - t:.1f}s")

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ctx = ara.ara_ctx_create(0, stream)
    ara.ara_set_option(ctx, ara.ARA_OPT_PLACEMENT, args.placement)
    ara.ara_set_option(ctx, ara.ARA_OPT_BLOCK_THREADS, args.block)
    ara.ara_set_option(ctx, ara.ARA_OPT_GRID_PER_CU, args.grid_per_cu)
    prec = ara.ARA_F32 if args.precision == "f32" else ara.ARA_F64
    t = time.time()
    an = session.open_analysis(ctx, w.event_ids, w.trial_offsets, w.catalog_size, w.elts, w.layer_terms,
                               None, prec)
    torch.cuda.synchronize()
    log(f"uploaded + validated in {time.time() - t:.1f}s")
    n_flagged, placement, lds_bytes = ara.ara_layer_stats(ctx, an.layer)
    log(f"placement={ara.PLACEMENT_NAMES.get(placement, placement)} lds={lds_bytes} flagged={n_flagged}")

    ylt = torch.empty(w.n_trials, dtype=torch.float64, device="cuda")
    ws = torch.empty(ara.ara_sort_workspace_size(w.n_trials), dtype=torch.uint8, device="cuda")
    rps = list(w.return_periods)

    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]

    def step(i=None):
        ara.ara_layer_build(ctx, an.layer, ara.ARA_BUILD_TABLES)
        if i is not None:
            ev0[i].record(stream)
        ara.ara_analyze(ctx, an.yet, an.layer, 0, w.n_trials, ylt)
        if i is not None:
            ev1[i].record(stream)
        return ara.ara_risk_measures(ctx, ylt, rps, ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")
    t0 = time.perf_counter()
    for i in range(args.steps):
        pml, tvar = step(i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    kern_ms = [ev0[i].elapsed_time(ev1[i]) for i in range(args.steps)]
    k_avg = float(np.mean(kern_ms))
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step; trial kernel avg {k_avg:.4f} ms "
        f"(min {min(kern_ms):.4f}, max {max(kern_ms):.4f}); PML {pml.tolist()} TVaR {tvar.tolist()}")

    nblk = (w.catalog_size + 127) // 128
    alg_bytes = 4 * w.n_events + 8 * (w.n_trials + 1) + 8 * w.n_trials + 20 * nblk + 8 * n_flagged
    achieved = alg_bytes / (k_avg * 1e-3) / 1e9
    te = float(w.n_events)   # trial-events x layers (1 layer)
    value = te / (ms_step * 1e-3)

    if args.copy_probe_mib:
        src = torch.empty(args.copy_probe_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe {args.copy_probe_mib} MiB done")

    an.release()
    ara.ara_ctx_destroy(ctx)

    cpu = None
    if args.cpu_seconds > 0:
        import oracle
        threads = oracle.max_threads()
        ids, offs = w.event_ids, w.trial_offsets
        n = 200 if args.workload == "paper" else 1000
        t = time.perf_counter()
        oracle.analyze(ids, offs, w.catalog_size, w.elts, w.layer_terms, t_begin=0, t_end=n, threads=threads)
        dt = time.perf_counter() - t
        n2 = int(min(w.n_trials, max(n, n * args.cpu_seconds / max(dt, 1e-3))))
        t = time.perf_counter()
        oracle.analyze(ids, offs, w.catalog_size, w.elts, w.layer_terms, t_begin=0, t_end=n2, threads=threads)
        dt = time.perf_counter() - t
        ev = float(offs[n2] - offs[0])
        cpu = {"value": ev / dt, "unit": "trial-events·layers/s", "cores": threads, "kind": "oracle",
               "sample": f"first {n2} trials ({int(ev)} events) of the same workload, {dt:.1f}s wall, "
                         f"OpenMP over trials"}
        log(f"cpu oracle: {cpu['value']:.3g} trial-events/s on {threads} threads ({dt:.1f}s)")

    out = {
        "metric": "trial-events·layers/s (1M trials x 1000 events, 16-ELT layer, whole path incl. sort + PML/TVaR)",
        "value": value,
        "unit": "trial-events·layers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == ara.ARA_F64 else "f64 arithmetic, f32 tables",
        "data": "synthetic",
        "config": {"workload": wname, "trials": w.n_trials, "events": w.n_events, "layers": 1,
                   "elts": len(w.elts), "catalog": w.catalog_size,
                   "placement": ara.PLACEMENT_NAMES.get(placement, str(placement)), "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_trial_ylt", "kernel_ms": k_avg, "algorithmic_bytes": alg_bytes},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
