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
import hashlib
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

# The headline trial kernel of each placement that the paper-scale workload can take,
# and the sources that define it (recorded counter readings stand only while these
# are unchanged).  The paper-scale YET has a catalog-binned copy, so the default
# placement is the tiled kernel; ARA_PLACE_LDS_BITMAP (--placement 1) measures the
# LDS-filter kernel that reads the packed copy.
KERNELS = {
    "k_trial_tiled": ("paper_1308_2066_amd/csrc/k_trial_tiled.hip", "paper_1308_2066_amd/csrc/trial_common.h",
                      "paper_1308_2066_amd/csrc/ara_internal.h"),
    "k_trial_ylt_bitmap": ("paper_1308_2066_amd/csrc/k_trial_bitmap.hip", "paper_1308_2066_amd/csrc/trial_bitmap.h",
                           "paper_1308_2066_amd/csrc/trial_common.h", "paper_1308_2066_amd/csrc/ara_internal.h"),
}


# the instantiation the headline figures time: the YLT kernel on 4-byte run starts
KERNEL_INSTANCE = {"k_trial_tiled": "k_trial_tiled<false, false>"}


def is_instance(kernel: str, name: str) -> bool:
    return KERNEL_INSTANCE.get(kernel, kernel) in name


def traffic_file(kernel: str) -> str:
    return os.path.join(ROOT, "profiles", f"{kernel}.paper_1Mx1000_f64.traffic.txt")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_digest(kernel: str) -> str:
    h = hashlib.sha256()
    for rel in KERNELS[kernel]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read() + b"\0")
    return h.hexdigest()


def read_kv(path: str) -> dict:
    out = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#") and ":" in line:
                k, v = line.split(":", 1)
                out[k.strip()] = v.strip()
    return out


def recorded_traffic(args, kernel: str):
    """HBM bytes per launch of the headline trial kernel from the committed counter
    summary, if it was taken on this workload with the current kernel sources."""
    if not (args.workload == "paper" and args.trials == 1_000_000 and args.precision == "f64"
            and not args.block and not args.grid_per_cu and not args.no_packing and not args.no_binning):
        return None, "no counter summary for this configuration"
    path = traffic_file(kernel)
    if kernel not in KERNELS or not os.path.exists(path):
        return None, "no counter summary recorded"
    kv = read_kv(path)
    if kv.get("source_sha256") != kernel_source_digest(kernel):
        return None, "kernel changed since the counters were taken"
    return float(kv["traffic_bytes"]), os.path.relpath(path, ROOT)


def headline_kernel_in(rows) -> str:
    """The headline trial kernel a rocprofv3 run recorded (the tiled kernel when present)."""
    names = {r["Kernel_Name"] for r in rows}
    for k in KERNELS:
        if any(k in n for n in names):
            return k
    raise SystemExit(f"none of {list(KERNELS)} in the recorded dispatches")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, target_s: float):
    """The CPU oracle (all host threads, OpenMP over trials) on the first trials of
    the same workload, the sample sized to take about target_s seconds: a fixed
    per-call cost (dense tables of every ELT) plus a per-trial cost, fitted from two
    short calibration runs.  Includes PML/TVaR of the sample's YLT."""
    import oracle
    threads = oracle.max_threads()

    def run(n):
        t = time.perf_counter()
        r = oracle.analyze(w.event_ids, w.trial_offsets, w.catalog_size, w.elts, w.layer_terms,
                           elt_terms=w.elt_terms, t_begin=0, t_end=n, threads=threads)
        oracle.risk(r["ylt"], w.return_periods)
        return time.perf_counter() - t

    run(min(w.n_trials, 100))            # first touch of the oracle's code and inputs
    na = min(w.n_trials, 4000)
    nb = min(w.n_trials, 4 * na)
    ta, tb = run(na), run(nb)
    per = max((tb - ta) / max(nb - na, 1), 1e-9)
    fixed = max(ta - na * per, 0.0)
    n = int(min(w.n_trials, max(nb, (target_s - fixed) / per)))
    dt = run(n)
    ev = float(w.trial_offsets[n] - w.trial_offsets[0])
    log(f"cpu oracle: calibration {na} trials {ta:.2f}s, {nb} trials {tb:.2f}s; sample {n} trials {dt:.1f}s")
    # the sequential role: one thread on a smaller first slice (about a quarter of the time)
    n1 = int(min(w.n_trials, max(100, (target_s / 4) / (per * threads))))
    t = time.perf_counter()
    r1 = oracle.analyze(w.event_ids, w.trial_offsets, w.catalog_size, w.elts, w.layer_terms,
                        elt_terms=w.elt_terms, t_begin=0, t_end=n1, threads=1)
    oracle.risk(r1["ylt"], w.return_periods)
    dt1 = time.perf_counter() - t
    ev1 = float(w.trial_offsets[n1] - w.trial_offsets[0])
    log(f"cpu oracle 1 thread: {n1} trials {dt1:.1f}s")
    return {"value": ev / dt, "unit": "trial-events·layers/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": len(os.sched_getaffinity(0)),
            "sample": f"first {n} of {w.n_trials} trials ({int(ev)} trial-events, 1 layer) of the same workload, "
                      f"dense tables built per call, YLT then PML/TVaR; {dt:.1f}s wall",
            "value_1_thread": ev1 / dt1,
            "sample_1_thread": f"first {n1} trials ({int(ev1)} trial-events), {dt1:.1f}s wall"}


def _counter_rows(path: str):
    import csv
    if os.path.isdir(path):
        found = [os.path.join(d, f) for d, _, fs in os.walk(path) for f in fs if f.endswith("counter_collection.csv")]
        if len(found) != 1:
            raise SystemExit(f"expected one counter_collection.csv under {path}, found {found}")
        path = found[0]
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def derive_traffic(fetch_path: str, write_path: str, copy_mib: int, cmd: str):
    """Write the counter summary of the headline kernel: FETCH_SIZE and WRITE_SIZE
    per dispatch, each scaled by the same counter's reading for the plain device
    copy of copy_mib MiB that the profiled run ends with."""
    copy_bytes = copy_mib << 20
    kernel = headline_kernel_in(_counter_rows(fetch_path))

    def per_dispatch(path, counter):
        rows = [r for r in _counter_rows(path) if r["Counter_Name"] == counter]
        kern = [float(r["Counter_Value"]) for r in rows if is_instance(kernel, r["Kernel_Name"])]
        copies = [r for r in rows if "copyBuffer" in r["Kernel_Name"]]
        if not kern or not copies:
            raise SystemExit(f"{path}: no {kernel} or copy dispatches with {counter}")
        big = max(copies, key=lambda r: int(r["Grid_Size"]))
        return float(np.mean(kern)), len(kern), float(big["Counter_Value"])

    fk, fn, fc = per_dispatch(fetch_path, "FETCH_SIZE")
    wk, wn, wc = per_dispatch(write_path, "WRITE_SIZE")
    f_scale = copy_bytes / 1024.0 / fc
    w_scale = copy_bytes / 1024.0 / wc
    traffic = (fk * f_scale + wk * w_scale) * 1024.0
    lines = [
        f"# HBM traffic of {kernel}, 1,000,000 trials x 1000 events, catalog 1,000,000, 16-ELT layer, binary64",
        f"# FETCH_SIZE pass: {cmd.format(counter='FETCH_SIZE')}",
        f"# WRITE_SIZE pass: {cmd.format(counter='WRITE_SIZE')}",
        "# Each counter is scaled by its own reading for a plain device copy of copy_bytes (the profiled run",
        "# ends with one): fetch_scale = copy KiB / FETCH_SIZE of the copy, likewise write_scale.",
        f"kernel: {kernel}",
        f"source_sha256: {kernel_source_digest(kernel)}",
        f"fetch_kib_per_dispatch: {fk:.1f}  (mean of {fn} dispatches)",
        f"write_kib_per_dispatch: {wk:.1f}  (mean of {wn} dispatches)",
        f"copy_bytes: {copy_bytes}",
        f"copy_fetch_kib: {fc:.1f}",
        f"copy_write_kib: {wc:.1f}",
        f"fetch_scale: {f_scale:.4f}",
        f"write_scale: {w_scale:.4f}",
        f"traffic_bytes: {traffic:.6g}",
    ]
    with open(traffic_file(kernel), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_counters(path: str, out_path: str, cmd: str):
    """Per-dispatch means of every counter of a rocprofv3 --pmc run for the headline
    kernel, with the L2 hit rate and busy fractions derived from them."""
    all_rows = _counter_rows(path)
    kernel = headline_kernel_in(all_rows)
    rows = [r for r in all_rows if is_instance(kernel, r["Kernel_Name"])]
    per = {}
    for r in rows:
        per.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    m = {k: float(np.mean(v)) for k, v in per.items()}
    n = len(next(iter(per.values()))) if per else 0
    lines = [f"# rocprofv3 counters of {kernel}, 1,000,000 trials x 1000 events, catalog 1,000,000, "
             f"16-ELT layer, binary64 (mean of {n} dispatches)", f"# command: {cmd}",
             f"source_sha256: {kernel_source_digest(kernel)}", ""]
    lines += [f"{k}: {v:.6g}" for k, v in sorted(m.items())]
    if "TCC_HIT_sum" in m and "TCC_MISS_sum" in m:
        lines.append(f"derived L2 hit rate: {m['TCC_HIT_sum'] / (m['TCC_HIT_sum'] + m['TCC_MISS_sum']):.3f}")
    if "GRBM_GUI_ACTIVE" in m:
        cyc = m["GRBM_GUI_ACTIVE"] / 8          # summed over the 8 XCDs
        lines.append(f"derived cycles per XCD: {cyc:.4g}")
        if "TA_BUSY_avr" in m:
            lines.append(f"derived TA busy fraction: {m['TA_BUSY_avr'] / cyc:.3f}")
        if "TD_TD_BUSY_sum" in m:
            lines.append(f"derived TD busy fraction (256 CUs): {m['TD_TD_BUSY_sum'] / 256 / cyc:.3f}")
    if "SQ_WAIT_INST_ANY" in m and "SQ_WAVE_CYCLES" in m:
        lines.append(f"derived wave time waiting on dependencies: {m['SQ_WAIT_INST_ANY'] / m['SQ_WAVE_CYCLES']:.3f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_stats(stats_csv: str, out_path: str, cmd: str, top: int = 16):
    """Short text summary of a rocprofv3 --stats kernel table."""
    import csv
    with open(stats_csv, newline="") as f:
        rows = list(csv.DictReader(f))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# rocprofv3 kernel statistics", f"# command: {cmd}", "",
             f"{'kernel':<60} {'calls':>6} {'avg us':>10} {'min us':>10} {'max us':>10} {'total %':>8}"]
    for r in rows[:top]:
        name = r["Name"]
        name = name if len(name) <= 60 else name[:57] + "..."
        lines.append(f"{name:<60} {int(r['Calls']):>6} {float(r['AverageNs']) / 1e3:>10.1f} "
                     f"{float(r['MinNs']) / 1e3:>10.1f} {float(r['MaxNs']) / 1e3:>10.1f} {float(r['Percentage']):>8.2f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def bench_portfolio(args):
    """Batched portfolio: the plain small YET (10,000 trials, Poisson(100) events,
    10,000-event catalog) against 64 layers of 1-32 binary32 ELTs from a 256-ELT pool.
    A step computes every layer's YLT and PML/TVaR at the return periods (results on
    the host).  Batched: ara_batch_run (graph replay) + ara_batch_risk; plain: per
    layer ara_analyze + ara_risk_measures.  Both give identical results."""
    import torch
    import synth
    from paper_1308_2066_amd import ara, session

    pf = synth.portfolio_batched()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ctx = ara.ara_ctx_create(0, stream)
    h = session.open_portfolio(ctx, pf.event_ids, pf.trial_offsets, pf.catalog_size, pf.pool, pf.layers)
    n, L = pf.n_trials, len(pf.layers)
    rps = list(pf.return_periods)
    outs = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(L)]
    plain = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(L)]
    ws = torch.empty(ara.ara_sort_workspace_size(n), dtype=torch.uint8, device="cuda")
    b = ara.ara_batch_create(ctx, [(h.yet, layer, 0, n, o) for layer, o in zip(h.layers, outs)])

    def step_batched():
        ara.ara_batch_run(b)
        return ara.ara_batch_risk(b, rps)

    def step_plain():
        res = []
        for layer, o in zip(h.layers, plain):
            ara.ara_analyze(ctx, h.yet, layer, 0, n, o)
            res.append(ara.ara_risk_measures(ctx, o, rps, ws))
        return res

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps, r

    pout = torch.empty(n, dtype=torch.float64, device="cuda")

    def step_portfolio():
        # every layer's YLT, the portfolio YLT (their per-trial sum, in job order) and
        # its PML/TVaR
        ara.ara_batch_run(b)
        ara.ara_batch_portfolio(b, pout)
        return ara.ara_risk_measures(ctx, pout, rps, ws)

    ms_b, (pml_b, tvar_b) = timed(step_batched)
    ms_pf, (pml_pf, tvar_pf) = timed(step_portfolio)
    ms_p, res_p = timed(step_plain)
    # the portfolio YLT is the job-order sum of the layers' YLTs
    acc = np.zeros(n)
    for o in outs:
        acc = acc + o.cpu().numpy()
    pf_same = pout.cpu().numpy().tobytes() == acc.tobytes()
    same = all(outs[j].cpu().numpy().tobytes() == plain[j].cpu().numpy().tobytes() for j in range(L))
    same = same and all(pml_b[j].tobytes() == np.asarray(res_p[j][0]).tobytes() and
                        tvar_b[j].tobytes() == np.asarray(res_p[j][1]).tobytes() for j in range(L))
    n_items, grid, epi, graph = ara.ara_batch_info(b)
    ara.ara_batch_release(b)
    h.release()
    ara.ara_ctx_destroy(ctx)
    te = float(pf.n_events) * L
    log(f"portfolio: batched {ms_b:.3f} ms/step ({n_items} items, {grid} workgroups, {epi} events/item, "
        f"graph={graph}); plain {ms_p:.3f} ms/step; identical={same}")
    out = {
        "metric": "trial-events·layers/s (batched portfolio: 10,000 trials x Poisson(100) events, 64 layers, "
                  "YLT + PML/TVaR per layer)",
        "value": te / (ms_b * 1e-3), "unit": "trial-events·layers/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_b, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 arithmetic, f32 tables", "data": "synthetic",
        "config": {"workload": f"{pf.name}: {pf.n_trials} trials, {pf.n_events} events, catalog {pf.catalog_size}, "
                               f"{L} layers of 1-32 ELTs from a 256-ELT pool (lognormal(11,2.5), dense), "
                               f"log-uniform terms", "layers": L, "parallelism": "1 GPU"},
        "plain_per_layer": {"ms_per_step": ms_p, "value": te / (ms_p * 1e-3)},
        "speedup_vs_plain": ms_p / ms_b, "identical_results": bool(same),
        "portfolio_ylt": {"ms_per_step": ms_pf, "value": te / (ms_pf * 1e-3),
                          "pml": [float(x) for x in pml_pf], "tvar": [float(x) for x in tvar_pf],
                          "equals_job_order_sum": bool(pf_same)},
        "schedule": {"items": n_items, "workgroups": grid, "events_per_item": epi, "graph": bool(graph & 1),
                     "interleaved": bool(graph & 2)},
    }
    print(json.dumps(out), flush=True)


def bench_events(args):
    """Per-occurrence outputs and occurrence maxima (the per-event outputs, OEP input
    and non-identity financial terms): the paper-scale shape at 10^5 trials (10^8
    occurrences, 1M-event catalog, 16 ELTs with fx/retention/limit terms).  A step of
    ara_analyze_events writes the gross, occurrence-net, cumulative and ceded loss of
    every occurrence and the YLT; ara_analyze_occ_max writes each trial's largest
    occurrence-net loss.  Each is timed with HIP events on the context's stream."""
    import torch
    import synth
    from paper_1308_2066_amd import ara, session

    w = synth.workload_paper_scale(n_trials=args.trials if args.trials != 1_000_000 else 100_000)
    elt_terms = [(1.0 + 0.01 * j, 1e3 * j, 2e7 + 1e6 * j) for j in range(len(w.elts))]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ctx = ara.ara_ctx_create(0, stream)
    an = session.open_analysis(ctx, w.event_ids, w.trial_offsets, w.catalog_size, w.elts, w.layer_terms, elt_terms,
                               ara.ARA_F64)
    n, e = w.n_trials, w.n_events
    ylt = torch.empty(n, dtype=torch.float64, device="cuda")
    ev = [torch.empty(e, dtype=torch.float64, device="cuda") for _ in range(4)]
    occ_max = torch.empty(n, dtype=torch.float64, device="cuda")

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
        e1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
        t0 = time.perf_counter()
        for i in range(args.steps):
            e0[i].record(stream)
            fn()
            e1[i].record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / args.steps
        return wall, float(np.mean([e0[i].elapsed_time(e1[i]) for i in range(args.steps)]))

    ms_ev, k_ev = timed(lambda: ara.ara_analyze_events(ctx, an.yet, an.layer, 0, n, ylt, *ev))
    ms_om, k_om = timed(lambda: ara.ara_analyze_occ_max(ctx, an.yet, an.layer, 0, n, occ_max))
    # the per-occurrence ceded losses of a trial add up to its year loss (telescoping;
    # reported as the largest relative difference, a sanity check beside the tests)
    offs = np.asarray(w.trial_offsets)
    has = offs[1:] > offs[:-1]
    ceded = ev[3].cpu().numpy()
    y = ylt.cpu().numpy()
    sums = np.add.reduceat(ceded, offs[:-1][has])
    ceded_rel = float(np.max(np.abs(sums - y[has]) / np.maximum(np.abs(y[has]), 1.0))) if has.any() else 0.0
    an.release()
    ara.ara_ctx_destroy(ctx)
    ev_bytes = 4 * e + 8 * (n + 1) + 32 * e + 8 * n          # IDs, offsets, 4 outputs, YLT
    log(f"events: step {ms_ev:.3f} ms (kernel {k_ev:.3f} ms); occ_max {ms_om:.3f} ms (kernel {k_om:.3f} ms)")
    out = {
        "metric": "trial-events/s (per-occurrence outputs: gross, occurrence-net, cumulative, ceded; 10^5 trials "
                  "x 1000 events, 16-ELT layer with financial terms)",
        "value": e / (ms_ev * 1e-3), "unit": "trial-events/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_ev, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{w.name} with ELT terms (fx 1.00-1.15, retention 0-15e3, limit 2e7-3.5e7)",
                   "trials": n, "events": e, "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": ev_bytes / (k_ev * 1e-3) / 1e9, "peak": 8000.0, "unit": "GB/s",
                     "frac": ev_bytes / (k_ev * 1e-3) / 1e9 / 8000.0, "traffic": None, "kernel": "k_trial_events",
                     "kernel_ms": k_ev, "algorithmic_bytes": ev_bytes},
        "ceded_sum_vs_ylt_max_rel_diff": ceded_rel,
        "occ_max": {"ms_per_step": ms_om, "kernel_ms": k_om, "value": e / (ms_om * 1e-3), "unit": "trial-events/s"},
    }
    print(json.dumps(out), flush=True)


def serving_rates(ctx, yet, pool, n_trials, n_events, catalog, rps, rates, n_requests, log_prefix="serving"):
    """Open-loop pricing requests (Poisson arrivals; U{1..32} ELTs of the pool,
    log-uniform terms, 10^5-10^6 contiguous trials) answered with PML/TVaR, once
    through the server and once through plain per-request launches on the same
    arrival trace.  Server latency = submission to completion as the server measures
    it; plain: one thread takes requests in arrival order (layer create + ara_analyze
    + ara_risk_measures + layer release), latency = completion - arrival.  Returns one
    record per arrival rate."""
    import threading
    import torch
    import synth
    from paper_1308_2066_amd import ara

    ws = torch.empty(ara.ara_sort_workspace_size(n_trials), dtype=torch.uint8, device="cuda")
    ylt = torch.empty(n_trials, dtype=torch.float64, device="cuda")
    lines = []
    for rate in rates:
        reqs = synth.serving_requests(n_requests, n_trials, rate=rate)
        srv = ara.ara_server_create(ctx, yet, pool, rps, max_batch=32)
        warm = [ara.ara_server_submit(srv, r[1], r[2], r[3], r[4]) for r in reqs[:8]]
        for t in warm:
            ara.ara_server_wait(srv, t)
        tickets = [None] * len(reqs)
        t_start = time.perf_counter()

        def submitter():
            for i, (at, idx, terms, t0, t1) in enumerate(reqs):
                d = t_start + at - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                tickets[i] = ara.ara_server_submit(srv, idx, terms, t0, t1)

        th = threading.Thread(target=submitter)
        th.start()
        lat_s, res_s = [], []
        for i in range(len(reqs)):
            while tickets[i] is None:
                time.sleep(0.0002)
            pml, tvar, sec = ara.ara_server_wait(srv, tickets[i])
            lat_s.append(sec)
            res_s.append((pml, tvar))
        th.join()
        wall_s = time.perf_counter() - t_start
        st = ara.ara_server_stats(srv)
        iters, most, slots = st["iterations"], st["max_in_iteration"], st["slots"]
        ara.ara_server_release(srv)
        lat_p, res_p = [], []
        t_start = time.perf_counter()
        for at, idx, terms, t0, t1 in reqs:
            d = t_start + at - time.perf_counter()
            if d > 0:
                time.sleep(d)
            layer = ara.ara_layer_create(ctx, [pool[i] for i in idx], catalog, terms)
            ara.ara_analyze(ctx, yet, layer, t0, t1, ylt[: t1 - t0])
            pml, tvar = ara.ara_risk_measures(ctx, ylt[: t1 - t0], rps, ws)
            ara.ara_layer_release(layer)
            lat_p.append(time.perf_counter() - (t_start + at))
            res_p.append((np.asarray(pml), np.asarray(tvar)))
        wall_p = time.perf_counter() - t_start
        same = all(a[0].tobytes() == b[0].tobytes() and a[1].tobytes() == b[1].tobytes()
                   for a, b in zip(res_s, res_p))
        q = lambda v, p: float(np.percentile(np.asarray(v) * 1e3, p))
        te = float(sum((r[4] - r[3]) for r in reqs)) * float(n_events) / n_trials
        log(f"{log_prefix} rate {rate}/s: server p50 {q(lat_s, 50):.3f} ms p99 {q(lat_s, 99):.3f} ms "
            f"({iters} iterations, max {most} per iteration, {slots} slots); plain p50 {q(lat_p, 50):.3f} ms "
            f"p99 {q(lat_p, 99):.3f} ms; identical={same}")
        lines.append({"rate_per_s": rate, "requests": len(reqs),
                      "server": {"p50_ms": q(lat_s, 50), "p99_ms": q(lat_s, 99), "queries_per_s": len(reqs) / wall_s,
                                 "iterations": iters, "max_per_iteration": most, "slots": slots,
                                 "max_in_flight": st["max_in_flight"], "held_for_memory": st["held"]},
                      "plain": {"p50_ms": q(lat_p, 50), "p99_ms": q(lat_p, 99), "queries_per_s": len(reqs) / wall_p},
                      "identical_results": bool(same), "trial_events_per_request": te / len(reqs)})
    return lines


SERVING_WORKLOAD = ("serving: resident YET of 10^6 trials (Poisson(100) events, catalog 10,000), 256 dense "
                    "lognormal(11,2.5) binary32 ELTs; Poisson arrivals of requests of 1-32 ELTs, log-uniform terms, "
                    "10^5-10^6 contiguous trials")


def open_serving(ctx):
    import synth
    from paper_1308_2066_amd import session
    pf = synth.portfolio_batched(n_layers=1)
    ids, offs, C = synth.serving_yet()
    h = session.open_portfolio(ctx, ids, offs, C, pf.pool, [])
    return h, pf, int(offs.shape[0] - 1), int(ids.shape[0]), C


def bench_serving(args):
    """Serving: p50/p99 quote latency and queries/s of the server against plain
    per-request launches, at each arrival rate of --rates (serving_rates)."""
    import torch
    from paper_1308_2066_amd import ara

    torch.cuda.set_device(0)
    ctx = ara.ara_ctx_create(0, torch.cuda.current_stream())
    h, pf, n_trials, n_events, C = open_serving(ctx)
    lines = serving_rates(ctx, h.yet, h.pool, n_trials, n_events, C, list(pf.return_periods),
                          [float(x) for x in args.rates.split(",")], args.requests)
    h.release()
    ara.ara_ctx_destroy(ctx)
    first = lines[0]
    out = {
        "metric": "p50/p99 quote latency (serving: 10^6-trial Poisson(100) YET, 256-ELT pool, 1-32 ELTs and "
                  "10^5-10^6 trials per request)",
        "value": first["server"]["p50_ms"], "unit": "ms", "n_gpus": 1, "steps": first["requests"], "warmup": 8,
        "ms_per_step": first["server"]["p50_ms"], "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 arithmetic, f32 tables", "data": "synthetic",
        "config": {"workload": SERVING_WORKLOAD, "parallelism": "1 GPU"},
        "rates": lines,
    }
    print(json.dumps(out), flush=True)


UNEVEN_WORKLOAD = ("{n} analyses: trials log-uniform 1e4-5e5, Poisson(200-2000) events, catalogs 1e5-1e6, "
                   "1-16 ELTs x 20000 lognormal(10,2); {ev} events")


def uneven_batch(ctx, n_analyses, steps):
    """Uneven-instance batching: independent analyses (trials log-uniform 10^4-5x10^5,
    Poisson events per trial with means uniform in 200-2000, catalogs 10^5-10^6, 1-16
    ELTs of 20,000 lognormal(10,2) losses) run as one batch (graph replay) against one
    ara_analyze per analysis.  Both give identical YLTs.  Returns the figures."""
    import torch
    import synth
    from paper_1308_2066_amd import ara, session

    # generated one analysis at a time and kept on the device only (the full set is
    # about 3.5e10 occurrences)
    t = time.time()
    shapes, opened = [], []
    stopped = None
    for w in synth.iter_uneven_analyses(n=n_analyses):
        try:
            opened.append(session.open_analysis(ctx, w.event_ids, w.trial_offsets, w.catalog_size, w.elts,
                                                w.layer_terms))
        except (ara.AraError, torch.cuda.OutOfMemoryError) as exc:   # the largest set that fits
            stopped = f"analysis {len(opened)} did not fit: {exc}"
            log(stopped)
            break
        shapes.append((w.n_trials, w.n_events, w.catalog_size, len(w.elts)))
        if len(opened) % 8 == 0:
            log(f"{len(opened)} analyses resident ({time.time() - t:.1f}s)")
    ev = sum(sh[1] for sh in shapes)
    torch.cuda.synchronize()
    log(f"generated and ingested {len(opened)} analyses, {ev} events in {time.time() - t:.1f}s")

    class _W:   # the sizes the rest of this function reads
        def __init__(self, sh):
            self.n_trials, self.n_events, self.catalog_size, self.n_elts = sh

    ws = [_W(sh) for sh in shapes]
    outs = [torch.empty(w.n_trials, dtype=torch.float64, device="cuda") for w in ws]
    plain = [torch.empty(w.n_trials, dtype=torch.float64, device="cuda") for w in ws]
    b = ara.ara_batch_create(ctx, [(an.yet, an.layer, 0, w.n_trials, o) for an, w, o in zip(opened, ws, outs)])
    ara.ara_batch_run(b)       # tuning + graph capture
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_b = timed(lambda: ara.ara_batch_run(b), steps)

    def run_plain():
        for an, w, o in zip(opened, ws, plain):
            ara.ara_analyze(ctx, an.yet, an.layer, 0, w.n_trials, o)

    ms_p = timed(run_plain, max(1, steps // 4))
    same = all(o.cpu().numpy().tobytes() == p.cpu().numpy().tobytes() for o, p in zip(outs, plain))
    n_items, grid, epi, graph = ara.ara_batch_info(b)
    id_bytes = [ara.ara_yet_info(an.yet)[2] for an in opened]
    ara.ara_batch_release(b)
    for an in opened:
        an.release()
    del outs, plain
    torch.cuda.empty_cache()
    trials = sum(w.n_trials for w in ws)
    alg = 4 * ev + 16 * trials
    moved = sum(bts * w.n_events for bts, w in zip(id_bytes, ws)) + 16 * trials
    log(f"uneven: batched {ms_b:.3f} ms ({n_items} items, {grid} workgroups, {epi} events/item, graph={graph}); "
        f"plain {ms_p:.3f} ms; identical={same}")
    return {"analyses": len(ws), "analyses_requested": n_analyses, "stopped": stopped, "events": ev,
            "trials": trials, "ms": ms_b, "steps": steps, "value": ev / (ms_b * 1e-3), "alg_bytes": alg,
            "moved_bytes": moved, "plain_ms": ms_p, "speedup_vs_plain": ms_p / ms_b, "identical_results": bool(same),
            "schedule": {"items": n_items, "workgroups": grid, "events_per_item": epi, "graph": bool(graph & 1),
                         "interleaved": bool(graph & 2)}}


def bench_uneven(args):
    """The uneven-instance batch as the bench line (see uneven_batch)."""
    import torch
    from paper_1308_2066_amd import ara

    torch.cuda.set_device(0)
    ctx = ara.ara_ctx_create(0, torch.cuda.current_stream())
    u = uneven_batch(ctx, args.analyses, args.steps)
    ara.ara_ctx_destroy(ctx)
    ms_b, alg = u["ms"], u["alg_bytes"]
    out = {
        "metric": f"trial-events·layers/s (uneven-instance batch: {u['analyses']} independent analyses)",
        "value": u["value"], "unit": "trial-events·layers/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": ms_b, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": UNEVEN_WORKLOAD.format(n=u["analyses"], ev=u["events"]), "analyses": u["analyses"],
                   "analyses_requested": args.analyses, "stopped": u["stopped"],
                   "events": u["events"], "trials": u["trials"], "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": alg / (ms_b * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg / (ms_b * 1e-3) / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes": alg,
                     "moved_bytes": u["moved_bytes"]},
        "plain_per_analysis": {"ms_per_step": u["plain_ms"], "value": u["events"] / (u["plain_ms"] * 1e-3)},
        "speedup_vs_plain": u["speedup_vs_plain"], "identical_results": u["identical_results"],
        "schedule": u["schedule"],
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # the GPU's clocks take some tens of steps after the setup's idle spells to settle:
    # 30 untimed steps, then 100 timed (about 60 ms at paper scale)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--workload", choices=["paper", "small", "portfolio", "serving", "uneven", "events"], default="paper",
                    help="portfolio: one YET x 64 layers, batched launch against per-layer launches; "
                         "serving: pricing requests with Poisson arrivals, server against per-request launches")
    ap.add_argument("--requests", type=int, default=600, help="serving: requests per rate")
    ap.add_argument("--analyses", type=int, default=16, help="uneven: number of analyses (256 = the full set)")
    ap.add_argument("--rates", default="50", help="serving: arrival rates per second, comma separated")
    ap.add_argument("--trials", type=int, default=1_000_000)
    ap.add_argument("--precision", choices=["f64", "f32"], default="f64")
    ap.add_argument("--placement", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--grid-per-cu", type=int, default=0)
    ap.add_argument("--no-packing", action="store_true", help="stream int32 IDs instead of the packed YET copy")
    ap.add_argument("--no-binning", action="store_true", help="no catalog-binned YET copy (no tiled kernel)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU-oracle sample time (0 = skip)")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="paper workload: requests of the serving leg per rate (0 = skip the leg)")
    ap.add_argument("--serve-rates", default="50", help="paper workload: arrival rates of the serving leg")
    ap.add_argument("--uneven-analyses", type=int, default=16,
                    help="paper workload: analyses of the uneven-instance batch leg (0 = skip the leg)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one plain device copy of this size (for counter calibration)")
    ap.add_argument("--derive-traffic", nargs=2, metavar=("FETCH", "WRITE"),
                    help="write the trial kernel's counter summary from two rocprofv3 --pmc outputs and exit")
    ap.add_argument("--profile-cmd", default="", help="command recorded in a written summary")
    ap.add_argument("--summarize-stats", nargs=2, metavar=("STATS_CSV", "OUT"),
                    help="write a text summary of a rocprofv3 kernel_stats.csv and exit")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("PMC_DIR", "OUT"),
                    help="write the trial kernel's counter means from a rocprofv3 --pmc output and exit")
    args = ap.parse_args()
    if args.derive_traffic:
        derive_traffic(args.derive_traffic[0], args.derive_traffic[1], args.copy_probe_mib or 1024, args.profile_cmd)
        return
    if args.summarize_stats:
        summarize_stats(args.summarize_stats[0], args.summarize_stats[1], args.profile_cmd)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters[0], args.summarize_counters[1], args.profile_cmd)
        return

    if args.gpus != 1:
        print(json.dumps({"error": "the analysis runs on one GPU only; --gpus must be 1 "
                                   "(sharding across GPUs is described, not implemented)"}))
        sys.exit(2)

    import torch
    import synth
    from paper_1308_2066_amd import ara, session

    if args.workload == "portfolio":
        return bench_portfolio(args)
    if args.workload == "events":
        return bench_events(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "uneven":
        return bench_uneven(args)

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
    ara.ara_set_option(ctx, ara.ARA_OPT_YET_PACKING, 0 if args.no_packing else 1)
    ara.ara_set_option(ctx, ara.ARA_OPT_YET_BINNING, 0 if args.no_binning else 1)
    prec = ara.ARA_F32 if args.precision == "f32" else ara.ARA_F64
    # ingest, once per resident YET: the int32 IDs and int64 offsets already in HBM,
    # ara_yet_create checks every ID and offset and builds the binned (or packed)
    # copy; it is blocking, so its wall time is the ingest time.  The first call in
    # the process also loads the library's kernels and makes its first device
    # allocations: it is reported beside the median of the next nine calls (each
    # YET released before the next, the last one kept for the analysis).
    ids_dev = session.to_device(np.asarray(w.event_ids, np.int32))
    offs_dev = session.to_device(np.asarray(w.trial_offsets, np.int64))
    # PML/TVaR input with as many distinct year losses (all eight radix passes run;
    # the workload's own year losses all equal the aggregate limit, so the step's
    # sort skips its passes).  Made here, before the GPU work that leads into the
    # timed steps, so that no long host-only spell precedes them
    y_distinct = torch.from_numpy(np.random.default_rng(7).lognormal(15.0, 2.0, size=w.n_trials)).cuda()
    # the layer's ELTs and the layer itself need no YET: created here for the same reason
    handles = [ara.ara_elt_create(ctx, session.to_device(np.asarray(i, np.int32)),
                                  session.to_device(np.asarray(l, np.float64)), w.catalog_size, precision=prec)
               for i, l in w.elts]
    layer = ara.ara_layer_create(ctx, handles, w.catalog_size, w.layer_terms)
    ingest_runs = []
    yet = None
    for r in range(10):
        if yet is not None:
            ara.ara_yet_release(yet)
        torch.cuda.synchronize()
        ig0, ig1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ig0.record(stream)
        t = time.perf_counter()
        yet = ara.ara_yet_create(ctx, ids_dev, offs_dev, w.catalog_size)
        wall = (time.perf_counter() - t) * 1e3
        ig1.record(stream)
        torch.cuda.synchronize()
        ingest_runs.append((wall, ig0.elapsed_time(ig1)))
    ingest_first_ms = ingest_runs[0][0]
    ingest_ms = float(np.median([x[0] for x in ingest_runs[1:]]))
    ingest_gpu_ms = float(np.median([x[1] for x in ingest_runs[1:]]))
    log("ingest calls (ms wall): " + " ".join(f"{x[0]:.2f}" for x in ingest_runs))
    id_bytes = ara.ara_yet_info(yet)[2]
    n_bins = ara.ara_yet_binned_count(yet) if id_bytes == 2 else 0
    # device memory the handle adds to the caller's int32 IDs and offsets, as the
    # library counts it: the binned copy (2 B per occurrence, its run starts, 3 or
    # 4 B per (bin, trial), and region starts) or the packed one
    yet_extra, run_bytes = ara.ara_yet_memory(yet)
    log(f"ingest (validate + {'binned' if id_bytes == 2 else 'packed' if id_bytes == 3 else 'no'} copy): "
        f"{ingest_ms:.2f} ms wall, {ingest_gpu_ms:.2f} ms on the stream (first call in the process "
        f"{ingest_first_ms:.2f} ms); {yet_extra / 1e9:.3f} GB added")
    an = session.Analysis(ctx, yet, handles, layer, w.n_trials, w.n_events)
    torch.cuda.synchronize()
    n_flagged, placement, lds_bytes = ara.ara_layer_stats(ctx, an.layer)
    # the layer alone would take the LDS filter; with the YET's binned copy the
    # analysis takes the tiled kernel unless a placement is forced
    if id_bytes == 2 and placement == ara.ARA_PLACE_LDS_BITMAP and args.placement in (0, ara.ARA_PLACE_LDS_TILES):
        placement = ara.ARA_PLACE_LDS_TILES
    kernel = {ara.ARA_PLACE_LDS_TILES: "k_trial_tiled", ara.ARA_PLACE_LDS_BITMAP: "k_trial_ylt_bitmap"}.get(
        placement, "k_trial_ylt")
    log(f"placement={ara.PLACEMENT_NAMES.get(placement, placement)} lds={lds_bytes} flagged={n_flagged}")

    ylt = torch.empty(w.n_trials, dtype=torch.float64, device="cuda")
    ws = torch.empty(ara.ara_sort_workspace_size(w.n_trials), dtype=torch.uint8, device="cuda")
    rps = list(w.return_periods)

    def run_steps(layer, steps, warmup, sort_input=None, on_yet=None):
        """steps x (table build, trial kernel, sort + PML/TVaR to the host): wall ms per
        step, and the trial kernel's mean duration over the timed steps from the HIP
        events the library attaches to the kernel's launch on its stream
        (ARA_OPT_KERNEL_TIMING, a ring of one pair per timed step, read once after the
        loop, so nothing runs on the host between the steps' calls)."""
        y_handle = an.yet if on_yet is None else on_yet

        def step():
            ara.ara_layer_build(ctx, layer, ara.ARA_BUILD_TABLES)
            ara.ara_analyze(ctx, y_handle, layer, 0, w.n_trials, ylt)
            return ara.ara_risk_measures(ctx, ylt if sort_input is None else sort_input, rps, ws)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        ara.ara_set_option(ctx, ara.ARA_OPT_KERNEL_TIMING, steps)
        t0 = time.perf_counter()
        for _ in range(steps):
            res = step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        k_mean = ara.ara_kernel_ms(ctx)
        ara.ara_set_option(ctx, ara.ARA_OPT_KERNEL_TIMING, 0)
        return ms, k_mean, res

    ms_step, k_avg, (pml, tvar) = run_steps(an.layer, args.steps, args.warmup)
    saturated = bool(torch.all(ylt == float(w.layer_terms[3])).item())
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step; trial kernel avg {k_avg:.4f} ms; "
        f"PML {pml.tolist()} TVaR {tvar.tolist()}")

    nblk = (w.catalog_size + 127) // 128
    # algorithmic bytes are defined on int32 event IDs and int64 trial offsets; the
    # kernels stream other forms, reported beside them as moved_bytes: the packed
    # 3-byte copy with the same offsets, or the binned 2-byte copy with a 3- or 4-byte
    # run start per (catalog bin, trial) instead of the trial offsets (the tiled kernel
    # then reads the layer's binary64 occurrence-net table, once per workgroup pass
    # from L2: counted once here)
    alg_bytes = 4 * w.n_events + 8 * (w.n_trials + 1) + 8 * w.n_trials + 20 * nblk + 8 * n_flagged
    if kernel == "k_trial_tiled":
        moved_bytes = 2 * w.n_events + run_bytes * n_bins * (w.n_trials + 1) + 8 * w.n_trials + 8 * w.catalog_size
    else:
        ib = 3 if not args.no_packing and w.catalog_size <= 1 << 24 else 4   # the packed copy, else int32
        moved_bytes = alg_bytes - (4 - ib) * w.n_events
    achieved = alg_bytes / (k_avg * 1e-3) / 1e9
    moved_gbs = moved_bytes / (k_avg * 1e-3) / 1e9
    te = float(w.n_events)   # trial-events x layers (1 layer)
    value = te / (ms_step * 1e-3)

    # the same step with the sort of distinct year losses in place of the saturated YLT
    ms_step_distinct, _, _ = run_steps(an.layer, args.steps, args.warmup, sort_input=y_distinct)
    for _ in range(2):
        ara.ara_risk_measures(ctx, y_distinct, rps, ws)
    torch.cuda.synchronize()
    t_r = time.perf_counter()
    for _ in range(10):
        ara.ara_risk_measures(ctx, y_distinct, rps, ws)
    torch.cuda.synchronize()
    risk_distinct_ms = (time.perf_counter() - t_r) * 1e3 / 10
    log(f"PML/TVaR of {w.n_trials} distinct year losses: {risk_distinct_ms:.3f} ms; step with that sort "
        f"{ms_step_distinct:.3f} ms")

    # the other table precision on the same resident YET
    other = ara.ARA_F32 if prec == ara.ARA_F64 else ara.ARA_F64
    an2 = session.open_analysis(ctx, w.event_ids, w.trial_offsets, w.catalog_size, w.elts, w.layer_terms,
                                None, other, yet=yet)
    ms2, k2, _ = run_steps(an2.layer, args.steps, args.warmup)
    nf2 = ara.ara_layer_stats(ctx, an2.layer)[0]
    alg2 = 4 * w.n_events + 8 * (w.n_trials + 1) + 8 * w.n_trials + 20 * nblk + 8 * nf2
    ara.ara_layer_release(an2.layer)
    for e in an2.elts:
        ara.ara_elt_release(e)
    log(f"{'binary32' if other == ara.ARA_F32 else 'binary64'} tables: {ms2:.3f} ms/step; trial kernel {k2:.4f} ms")

    # a copy of the YET built with 3-byte run starts (less memory, a slower tiled
    # kernel): its ingest after a first build, its memory, and the trial kernel on the
    # two copies in alternating rounds of 5 launches (legs run one after the other in
    # a process differ by more than the two forms do)
    lean = None
    if id_bytes == 2:
        ara.ara_set_option(ctx, ara.ARA_OPT_YET_RUN_BYTES, 3)
        try:
            yet3 = None
            lean_ingest = []
            for _ in range(2):
                if yet3 is not None:
                    ara.ara_yet_release(yet3)
                torch.cuda.synchronize()
                t = time.perf_counter()
                yet3 = ara.ara_yet_create(ctx, ids_dev, offs_dev, w.catalog_size)
                lean_ingest.append((time.perf_counter() - t) * 1e3)
        finally:
            ara.ara_set_option(ctx, ara.ARA_OPT_YET_RUN_BYTES, 4)
        extra3, rb3 = ara.ara_yet_memory(yet3)
        ara.ara_layer_build(ctx, an.layer, ara.ARA_BUILD_TABLES)
        pair = [("own", an.yet), ("lean", yet3)]
        kt = {k: [] for k, _ in pair}
        for r in range(8):
            for k, yh in (pair if r % 2 == 0 else pair[::-1]):
                ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
                for e0, e1 in ev:
                    e0.record(stream)
                    ara.ara_analyze(ctx, yh, an.layer, 0, w.n_trials, ylt)
                    e1.record(stream)
                torch.cuda.synchronize()
                kt[k] += [e0.elapsed_time(e1) for e0, e1 in ev]
        ara.ara_yet_release(yet3)
        k_own, k3 = float(np.median(kt["own"])), float(np.median(kt["lean"]))
        lean = {"run_bytes": rb3, "yet_extra_bytes": extra3, "ingest_ms": lean_ingest[-1],
                "kernel_ms_median": k3, "kernel_ms_median_4byte": k_own,
                "frac": alg_bytes / (k3 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "what": "the trial kernel on a copy of the YET with 3-byte run starts "
                        "(ARA_OPT_YET_RUN_BYTES = 3) and on the 4-byte one, alternating rounds"}
        log(f"{rb3}-byte run starts: {extra3 / 1e9:.3f} GB added, ingest {lean_ingest[-1]:.2f} ms; trial kernel "
            f"median {k3:.4f} ms vs {k_own:.4f} ms with 4-byte run starts (alternating)")

    if args.copy_probe_mib:
        src = torch.empty(args.copy_probe_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe {args.copy_probe_mib} MiB done")

    an.release()
    del ids_dev, offs_dev, ylt, ws, y_distinct
    torch.cuda.empty_cache()

    serving = None
    if args.serve_requests > 0:
        h, pf, s_trials, s_events, s_cat = open_serving(ctx)
        lines = serving_rates(ctx, h.yet, h.pool, s_trials, s_events, s_cat, list(pf.return_periods),
                              [float(x) for x in args.serve_rates.split(",")], args.serve_requests)
        h.release()
        serving = {"workload": SERVING_WORKLOAD, "rates": lines}
    uneven = None
    if args.uneven_analyses > 0:
        u = uneven_batch(ctx, args.uneven_analyses, 10)
        uneven = {"workload": UNEVEN_WORKLOAD.format(n=u["analyses"], ev=u["events"]),
                  "ms_batched": u["ms"], "ms_plain": u["plain_ms"], "speedup_vs_plain": u["speedup_vs_plain"],
                  "value": u["value"], "identical_results": u["identical_results"], "analyses": u["analyses"],
                  "events": u["events"], "schedule": u["schedule"],
                  "what": "independent analyses of different YETs, catalogs and trial counts: one ara_batch_run "
                          "(graph replay) against one ara_analyze per analysis, YLTs compared bit for bit"}
    ara.ara_ctx_destroy(ctx)

    cpu = cpu_baseline(w, args.cpu_seconds) if args.cpu_seconds > 0 else None
    traffic, traffic_note = recorded_traffic(args, kernel)

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
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel,
                     "kernel_ms": k_avg,
                     "kernel_timing": "HIP events attached to the trial kernel's launch on its stream "
                                      "(ARA_OPT_KERNEL_TIMING), mean over the timed steps",
                     "algorithmic_bytes": alg_bytes, "yet_id_bytes": id_bytes,
                     "moved_bytes": moved_bytes, "moved_gbs": moved_gbs, "moved_frac": moved_gbs / HBM_PEAK_GBS,
                     "traffic_source": traffic_note},
        "cpu_baseline": cpu,
        "ingest": {"ms": ingest_ms, "gpu_ms": ingest_gpu_ms, "first_call_ms": ingest_first_ms,
                   "yet_extra_bytes": yet_extra,
                   "what": "ara_yet_create on IDs and offsets resident in HBM: every ID and offset checked, "
                           "catalog-binned copy built; once per resident YET, not part of a step; median of "
                           "9 calls after the first, which also loads the kernels (first_call_ms)"},
        "ylt_saturated": {"all_equal_agg_limit": saturated,
                          "ms_per_step_with_distinct_ylt_sort": ms_step_distinct,
                          "value_with_distinct_ylt_sort": te / (ms_step_distinct * 1e-3)},
        "risk_measures_distinct_ylt": {"ms": risk_distinct_ms, "trials": w.n_trials,
                                       "data": "lognormal(15, 2) year losses, seed 7: all 8 radix passes run"},
        "lean_yet": lean,
        ("f32_tables" if other == ara.ARA_F32 else "f64_tables"): {
            "ms_per_step": ms2, "value": te / (ms2 * 1e-3), "kernel_ms": k2, "algorithmic_bytes": alg2,
            "achieved_gbs": alg2 / (k2 * 1e-3) / 1e9, "frac": alg2 / (k2 * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "dtype": "f64 arithmetic, f32 tables" if other == ara.ARA_F32 else "f64"},
        "serving": serving,
        "uneven_batch": uneven,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
