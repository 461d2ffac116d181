"""Batched analyses on the GPU: every job of a batch gives exactly the YLT of the
plain single-analysis launch (same device code, same order of additions), graph
replays repeat it, batched PML/TVaR equal ara_risk_measures, and the batched
portfolio matches the oracle within the binary32-table bound."""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def A(ara_lib):
    return ara_lib


@pytest.fixture(scope="module")
def S():
    from paper_1308_2066_amd import session
    return session


def _plain(A, ctx, yet, layer, t0, t1):
    import torch
    y = torch.empty(max(t1 - t0, 1), dtype=torch.float64, device="cuda")
    if t1 > t0:
        A.ara_analyze(ctx, yet, layer, t0, t1, y)
    A.ara_sync(ctx)
    return y[: t1 - t0].cpu().numpy()


def _edge(rng, lengths, catalog=5000, n_elts=3):
    counts = np.asarray(lengths, np.int64)
    offs = np.zeros(len(counts) + 1, np.int64)
    np.cumsum(counts, out=offs[1:])
    ids = rng.integers(0, catalog, size=int(offs[-1])).astype(np.int32)
    elts = [synth.elt_sparse(rng, catalog // 3, catalog, 10.0, 2.0) for _ in range(n_elts)]
    return synth.Workload("edge", ids, offs, catalog, elts, (5e4, 1e6, 2e5, math.inf), None, (2.0, 10.0), 0)


def test_batch_equals_plain_launches(A, S, gpu_ctx):
    """Jobs of three shapes in one batch: short trials over a 10k catalog (lane per
    trial, LDS table), long trials over a 1M catalog (LDS filter, packed IDs), and
    ragged trial lengths over a 5k catalog; whole and partial trial ranges."""
    import torch
    rng = np.random.default_rng(5)
    small = synth.workload_plain_small()
    paper = synth.workload_paper_scale(n_trials=20_000)
    edge = _edge(rng, list(rng.integers(0, 3000, size=300)) + [0, 1, 4099, 1023, 1025])
    layers, elts, yets = [], [], []

    def track(an, own_yet=True):
        layers.append(an.layer)
        elts.extend(an.elts)
        if own_yet:
            yets.append(an.yet)
        return an

    try:
        an_s = track(S.open_analysis(gpu_ctx, small.event_ids, small.trial_offsets, small.catalog_size, small.elts,
                                     small.layer_terms))
        # a second layer on the same YET: uncapped aggregate terms
        an_s2 = track(S.open_analysis(gpu_ctx, None, None, small.catalog_size, small.elts,
                                      (5e4, 1e6, 1e5, math.inf), yet=an_s.yet), own_yet=False)
        an_p = track(S.open_analysis(gpu_ctx, paper.event_ids, paper.trial_offsets, paper.catalog_size, paper.elts,
                                     (1e5, 5e6, 1.5e8, math.inf)))
        an_e = track(S.open_analysis(gpu_ctx, edge.event_ids, edge.trial_offsets, edge.catalog_size, edge.elts,
                                     edge.layer_terms))
        specs = [(an_s.yet, an_s.layer, 0, small.n_trials), (an_s.yet, an_s2.layer, 0, small.n_trials),
                 (an_s.yet, an_s.layer, 123, 4567), (an_p.yet, an_p.layer, 0, paper.n_trials),
                 (an_p.yet, an_p.layer, 17, 9001), (an_e.yet, an_e.layer, 0, edge.n_trials),
                 (an_e.yet, an_e.layer, 290, 305)]
        want = [_plain(A, gpu_ctx, y, layer, t0, t1) for y, layer, t0, t1 in specs]
        outs = [torch.full((max(t1 - t0, 1),), math.nan, dtype=torch.float64, device="cuda")
                for _, _, t0, t1 in specs]
        b = A.ara_batch_create(gpu_ctx, [(y, layer, t0, t1, o) for (y, layer, t0, t1), o in zip(specs, outs)])
        try:
            for rep in range(3):
                _say(f"batch run {rep}")
                for o in outs:
                    o.fill_(math.nan)
                A.ara_batch_run(b)
                A.ara_sync(gpu_ctx)
                for k, ((_, _, t0, t1), o) in enumerate(zip(specs, outs)):
                    got = o[: t1 - t0].cpu().numpy()
                    assert got.tobytes() == want[k].tobytes(), (rep, k)
            n_items, grid, epi, graph = A.ara_batch_info(b)
            assert graph & 1 and n_items >= len(specs) and grid >= 1 and epi > 0
            rps = [1.0, 2.0, 10.0, 100.0, 250.0]
            pml, tvar = A.ara_batch_risk(b, rps)
            for k, (_, _, t0, t1) in enumerate(specs):
                p1, v1 = A.ara_risk_measures(gpu_ctx, torch.from_numpy(want[k]).cuda(), rps)
                assert pml[k].tobytes() == np.asarray(p1).tobytes(), k
                assert tvar[k].tobytes() == np.asarray(v1).tobytes(), k
        finally:
            A.ara_batch_release(b)
    finally:
        for layer in layers:
            A.ara_layer_release(layer)
        for e in elts:
            A.ara_elt_release(e)
        for y in yets:
            A.ara_yet_release(y)


def test_batch_rejects_bad_jobs(A, S, gpu_ctx):
    import torch
    small = synth.workload_plain_small()
    an = S.open_analysis(gpu_ctx, small.event_ids, small.trial_offsets, small.catalog_size, small.elts,
                         small.layer_terms)
    other = S.open_analysis(gpu_ctx, small.event_ids[:10], np.array([0, 10], np.int64), 20_000,
                            [(np.array([1, 2], np.int32), np.array([3.0, 4.0]))], small.layer_terms)
    try:
        y = torch.empty(small.n_trials, dtype=torch.float64, device="cuda")
        with pytest.raises(A.AraError) as e:
            A.ara_batch_create(gpu_ctx, [(an.yet, other.layer, 0, 10, y)])      # catalogs differ
        assert e.value.status == A.ARA_E_INVALID_ARG
        with pytest.raises(A.AraError) as e:
            A.ara_batch_create(gpu_ctx, [(an.yet, an.layer, 5, small.n_trials + 1, y)])
        assert e.value.status == A.ARA_E_INVALID_ARG
        b = A.ara_batch_create(gpu_ctx, [(an.yet, an.layer, 7, 7, y)])
        try:
            A.ara_batch_run(b)
            with pytest.raises(A.AraError) as e:
                A.ara_batch_risk(b, [10.0])
            assert e.value.status == A.ARA_E_EMPTY
        finally:
            A.ara_batch_release(b)
        b = A.ara_batch_create(gpu_ctx, [])
        A.ara_batch_run(b)
        A.ara_batch_release(b)
    finally:
        an.release()
        other.release()


def test_batched_portfolio_matches_oracle(A, S, gpu_ctx):
    """The batched portfolio (one YET, 64 layers of 1-32 ELTs from a 256-ELT pool,
    binary32 tables): every layer's YLT within the binary32 bound of the FP64 oracle
    and equal to its plain launch."""
    import torch
    pf = synth.portfolio_batched()
    h = S.open_portfolio(gpu_ctx, pf.event_ids, pf.trial_offsets, pf.catalog_size, pf.pool, pf.layers)
    try:
        outs = [torch.empty(pf.n_trials, dtype=torch.float64, device="cuda") for _ in pf.layers]
        port = torch.empty(pf.n_trials, dtype=torch.float64, device="cuda")
        b = A.ara_batch_create(gpu_ctx, [(h.yet, layer, 0, pf.n_trials, o) for layer, o in zip(h.layers, outs)])
        try:
            A.ara_batch_run(b)
            A.ara_batch_run(b)
            A.ara_batch_portfolio(b, port)
            A.ara_sync(gpu_ctx)
            pml, tvar = A.ara_batch_risk(b, pf.return_periods)
        finally:
            A.ara_batch_release(b)
        # portfolio YLT: the layers' YLTs added per trial in layer order from +0.0
        want = np.zeros(pf.n_trials)
        for o in outs:
            want = want + o.cpu().numpy()
        assert port.cpu().numpy().tobytes() == want.tobytes()
        port_tol = np.zeros(pf.n_trials)
        port_ref = np.zeros(pf.n_trials)
        threads = oracle.max_threads()
        for j in range(len(pf.layers)):
            _say(f"portfolio layer {j}")
            got = outs[j].cpu().numpy()
            assert got.tobytes() == _plain(A, gpu_ctx, h.yet, h.layers[j], 0, pf.n_trials).tobytes(), j
            w = pf.layer_workload(j)
            ref = oracle.analyze_workload(w, threads=threads)
            gross = ref["gross_total"]
            tol = 2.0 ** -23 * 1.0001 * gross + 1e-12 * np.maximum(np.abs(ref["ylt"]), ref["occ_total"])
            assert np.all(np.abs(got - ref["ylt"]) <= tol), j
            port_ref = port_ref + ref["ylt"]
            port_tol = port_tol + tol
            ranks = [A.ara_return_period_rank(pf.n_trials, rp) for rp in pf.return_periods]
            srt = np.sort(got)[::-1]
            assert pml[j].tolist() == [srt[k - 1] for k in ranks]
        # the portfolio against the sum of the oracle's layer YLTs (64 terms of rounding added)
        assert np.all(np.abs(port.cpu().numpy() - port_ref) <= port_tol + 64 * 2.0 ** -52 * np.abs(port_ref))
    finally:
        h.release()


def test_uneven_analyses_batch_equals_plain(A, S, gpu_ctx):
    """Independent analyses of different YETs, catalogs (100k-1M: LDS filter), trial
    counts and lengths in one batch: each YLT equals its plain launch bit for bit,
    and the oracle within tolerance (first trials of each)."""
    import torch
    ws = synth.uneven_analyses(n=10, trials=(1_000, 20_000))
    opened = []
    try:
        for w in ws:
            opened.append(S.open_analysis(gpu_ctx, w.event_ids, w.trial_offsets, w.catalog_size, w.elts,
                                          w.layer_terms))
        outs = [torch.empty(w.n_trials, dtype=torch.float64, device="cuda") for w in ws]
        b = A.ara_batch_create(gpu_ctx, [(an.yet, an.layer, 0, w.n_trials, o) for an, w, o in zip(opened, ws, outs)])
        try:
            A.ara_batch_run(b)
            A.ara_batch_run(b)
            A.ara_sync(gpu_ctx)
        finally:
            A.ara_batch_release(b)
        for an, w, o in zip(opened, ws, outs):
            _say(f"uneven {w.name}")
            got = o.cpu().numpy()
            assert got.tobytes() == _plain(A, gpu_ctx, an.yet, an.layer, 0, w.n_trials).tobytes(), w.name
            ref = oracle.analyze(w.event_ids, w.trial_offsets, w.catalog_size, w.elts, w.layer_terms, t_end=200,
                                 threads=oracle.max_threads())
            tol = 1e-12 * np.maximum(np.abs(ref["ylt"]), ref["occ_total"])
            assert np.all(np.abs(got[:200] - ref["ylt"]) <= tol), w.name
    finally:
        for an in opened:
            an.release()


def test_batch_risk_every_lds_sort_size(A, S, gpu_ctx):
    """Batched PML/TVaR sort each short YLT in one workgroup's LDS; the sort's register
    stages depend on the padded length (2^k for k <= 14).  Lengths on both sides of
    each power of two, up to one past the LDS limit (the radix sort): the same bits
    as ara_risk_measures on the plain YLT."""
    import torch
    w = synth.workload_paper_scale(n_trials=20_000)
    lengths = [1, 2, 3, 1000, 1024, 1025, 2047, 2048, 2049, 4095, 4096, 4097, 8191, 8192, 8193, 16383, 16384, 16385]
    an = S.open_analysis(gpu_ctx, w.event_ids, w.trial_offsets, w.catalog_size, w.elts, (1e5, 5e6, 1.5e8, math.inf))
    try:
        outs = [torch.full((n,), math.nan, dtype=torch.float64, device="cuda") for n in lengths]
        b = A.ara_batch_create(gpu_ctx, [(an.yet, an.layer, 7, 7 + n, o) for n, o in zip(lengths, outs)])
        try:
            _say("batch risk LDS sort sizes")
            A.ara_batch_run(b)
            A.ara_sync(gpu_ctx)
            rps = [1.0, 1.5, 10.0, 100.0, 250.0, 1e4]
            pml, tvar = A.ara_batch_risk(b, rps)
            for k, (n, o) in enumerate(zip(lengths, outs)):
                p1, v1 = A.ara_risk_measures(gpu_ctx, o, rps)
                assert pml[k].tobytes() == np.asarray(p1).tobytes(), n
                assert tvar[k].tobytes() == np.asarray(v1).tobytes(), n
                # and the sorted order is right: PML at the rank rule's k
                y = np.sort(o.cpu().numpy())[::-1]
                for r, rp in enumerate(rps):
                    assert pml[k][r] == y[A.ara_return_period_rank(n, rp) - 1], (n, rp)
        finally:
            A.ara_batch_release(b)
    finally:
        an.release()


def test_second_batch_of_a_tuned_shape_computes_on_its_first_run(A, S, gpu_ctx):
    """Two batches of the same shape on one context: the second takes the first's tuned
    schedule (no tuning runs) and still writes every YLT on its first run."""
    import torch
    rng = np.random.default_rng(11)
    w = _edge(rng, list(rng.integers(50, 900, size=700)), catalog=7000)
    an = S.open_analysis(gpu_ctx, w.event_ids, w.trial_offsets, w.catalog_size, w.elts, w.layer_terms)
    try:
        specs = [(0, w.n_trials), (5, 333)]
        want = [_plain(A, gpu_ctx, an.yet, an.layer, t0, t1) for t0, t1 in specs]
        for rep in range(2):
            _say(f"same-shape batch {rep}")
            outs = [torch.full((t1 - t0,), math.nan, dtype=torch.float64, device="cuda") for t0, t1 in specs]
            b = A.ara_batch_create(gpu_ctx, [(an.yet, an.layer, t0, t1, o) for (t0, t1), o in zip(specs, outs)])
            try:
                A.ara_batch_run(b)
                A.ara_sync(gpu_ctx)
                for k, o in enumerate(outs):
                    assert o.cpu().numpy().tobytes() == want[k].tobytes(), (rep, k)
            finally:
                A.ara_batch_release(b)
    finally:
        an.release()


def test_set_terms_between_batch_runs(A, S, gpu_ctx):
    """Re-pricing a member layer (ara_layer_set_terms) between runs of a batch: the next
    run uses the new occurrence and aggregate terms, for a dense-table job and a tiled
    job alike (each equal to a plain launch with the new terms, bit for bit)."""
    import torch
    small = synth.workload_plain_small()
    big = synth.workload_paper_scale(n_trials=6_000, catalog=200_000, n_elts=4, nnz=30_000)
    a1 = S.open_analysis(gpu_ctx, small.event_ids, small.trial_offsets, small.catalog_size, small.elts,
                         small.layer_terms)
    a2 = S.open_analysis(gpu_ctx, big.event_ids, big.trial_offsets, big.catalog_size, big.elts,
                         (1e5, 5e6, 1e8, math.inf))
    try:
        assert A.ara_yet_info(a2.yet)[2] == 2, "the second job should take the tiled kernel"
        specs = [(a1, 0, small.n_trials), (a2, 0, big.n_trials), (a2, 17, 4000)]
        outs = [torch.full((t1 - t0,), math.nan, dtype=torch.float64, device="cuda") for _, t0, t1 in specs]
        b = A.ara_batch_create(gpu_ctx, [(an.yet, an.layer, t0, t1, o) for (an, t0, t1), o in zip(specs, outs)])
        try:
            terms_seq = [None, ((2e4, 2e6, 1e5, 4e6), (5e4, 1e7, 3e8, 2e8)), ((0.0, math.inf, 0.0, math.inf),) * 2]
            for rep, terms in enumerate(terms_seq):
                _say(f"batch re-priced {rep}")
                if terms is not None:
                    A.ara_layer_set_terms(gpu_ctx, a1.layer, terms[0])
                    A.ara_layer_set_terms(gpu_ctx, a2.layer, terms[1])
                for o in outs:
                    o.fill_(math.nan)
                A.ara_batch_run(b)
                A.ara_sync(gpu_ctx)
                for k, ((an, t0, t1), o) in enumerate(zip(specs, outs)):
                    assert o.cpu().numpy().tobytes() == _plain(A, gpu_ctx, an.yet, an.layer, t0, t1).tobytes(), (rep, k)
            # the last terms pass everything through: the YLT is the summed gross losses
            ref = oracle.analyze_workload(big.with_terms((0.0, math.inf, 0.0, math.inf)), threads=oracle.max_threads())
            got = outs[1].cpu().numpy()
            assert np.all(np.abs(got - ref["ylt"]) <= 1e-12 * np.maximum(np.abs(ref["ylt"]), ref["occ_total"]))
        finally:
            A.ara_batch_release(b)
    finally:
        a1.release()
        a2.release()


def test_rebuilt_layer_in_lds_bitmap_batch(A, S, gpu_ctx):
    """Jobs on the LDS-bitmap placement read their layer's ranks and compacted values,
    which a rebuild (ara_layer_build, ara_layer_set_terms) leaves to the first call that
    needs them: ara_batch_run builds them before its kernels, so each run equals a
    plain launch of the same placement after the same rebuild, bit for bit."""
    import torch
    big = synth.workload_paper_scale(n_trials=5_000, catalog=200_000, n_elts=4, nnz=30_000)
    A.ara_set_option(gpu_ctx, A.ARA_OPT_PLACEMENT, A.ARA_PLACE_LDS_BITMAP)
    an = S.open_analysis(gpu_ctx, big.event_ids, big.trial_offsets, big.catalog_size, big.elts,
                         (1e5, 5e6, 1e8, math.inf))
    try:
        specs = [(0, big.n_trials), (123, 3_456)]
        outs = [torch.full((t1 - t0,), math.nan, dtype=torch.float64, device="cuda") for t0, t1 in specs]
        b = A.ara_batch_create(gpu_ctx, [(an.yet, an.layer, t0, t1, o) for (t0, t1), o in zip(specs, outs)])
        try:
            steps = [None, ("terms", (3e5, 2e6, 1e6, 4e6)), ("build", None), ("terms", (0.0, math.inf, 0.0, math.inf))]
            for rep, step in enumerate(steps):
                _say(f"LDS-bitmap batch after rebuild {rep}")
                if step is not None and step[0] == "terms":
                    A.ara_layer_set_terms(gpu_ctx, an.layer, step[1])
                elif step is not None:
                    A.ara_layer_build(gpu_ctx, an.layer, A.ARA_BUILD_TABLES)
                for o in outs:
                    o.fill_(math.nan)
                A.ara_batch_run(b)
                A.ara_sync(gpu_ctx)
                got = [o.cpu().numpy() for o in outs]
                for k, ((t0, t1), g) in enumerate(zip(specs, got)):
                    assert g.tobytes() == _plain(A, gpu_ctx, an.yet, an.layer, t0, t1).tobytes(), (rep, k)
            ref = oracle.analyze_workload(big.with_terms((0.0, math.inf, 0.0, math.inf)), threads=oracle.max_threads())
            assert np.all(np.abs(got[0] - ref["ylt"]) <= 1e-12 * np.maximum(np.abs(ref["ylt"]), ref["occ_total"]))
        finally:
            A.ara_batch_release(b)
    finally:
        an.release()
        A.ara_set_option(gpu_ctx, A.ARA_OPT_PLACEMENT, 0)


def test_tuning_cache_round_trip(A, S, gpu_ctx, tmp_path):
    """A batch shape tuned on one context, its schedule saved to a file and loaded into
    a fresh context: the fresh context's batch of that shape takes the saved schedule
    (no tuning runs), writes every YLT on its first run, and equals plain launches."""
    import torch
    rng = np.random.default_rng(23)
    w = _edge(rng, list(rng.integers(40, 700, size=900)), catalog=6000)
    path = str(tmp_path / "schedules.txt")
    specs = [(0, w.n_trials), (11, 500)]
    schedules = []
    for ctx_rep in range(2):
        ctx = gpu_ctx if ctx_rep == 0 else A.ara_ctx_create(0)
        an = S.open_analysis(ctx, w.event_ids, w.trial_offsets, w.catalog_size, w.elts, w.layer_terms)
        try:
            if ctx_rep == 1:
                A.ara_tune_cache_load(ctx, path)
            _say(f"tuning cache context {ctx_rep}")
            want = [_plain(A, ctx, an.yet, an.layer, t0, t1) for t0, t1 in specs]
            outs = [torch.full((t1 - t0,), math.nan, dtype=torch.float64, device="cuda") for t0, t1 in specs]
            b = A.ara_batch_create(ctx, [(an.yet, an.layer, t0, t1, o) for (t0, t1), o in zip(specs, outs)])
            try:
                A.ara_batch_run(b)
                A.ara_sync(ctx)
                for k, o in enumerate(outs):
                    assert o.cpu().numpy().tobytes() == want[k].tobytes(), (ctx_rep, k)
                schedules.append(A.ara_batch_info(b))
            finally:
                A.ara_batch_release(b)
            if ctx_rep == 0:
                A.ara_tune_cache_save(ctx, path)
        finally:
            an.release()
            if ctx_rep == 1:
                A.ara_ctx_destroy(ctx)
    assert schedules[0] == schedules[1]
    lines = [ln for ln in open(path) if not ln.startswith("#")]
    assert len(lines) >= 1
    bad = tmp_path / "bad.txt"
    bad.write_text("not a schedule\n")
    with pytest.raises(A.AraError):
        A.ara_tune_cache_load(gpu_ctx, str(bad))
