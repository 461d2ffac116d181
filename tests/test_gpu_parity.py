"""Parity of the HIP path (through the C-ABI) with the CPU oracle.

Bars:
  * event lookups (combined and occurrence-net loss per event): bit-exact;
  * integer-valued inputs (every intermediate exact in binary64): bit-exact;
  * binary64 YLT: |gpu - oracle| <= 1e-12 * max(|oracle|, P_k), P_k the trial's
    total of occurrence-net losses (both sides sum the same non-negative terms in
    different orders, each within (k-1)u P_k of the exact value, and the aggregate
    clamp is 1-Lipschitz; the max() keeps the bound meaningful where the clamp
    cancels, P_k close to AggR);
  * PML/TVaR: identical ranks; values within the YLT bound (order statistics are
    1-Lipschitz in the sup norm) plus the TVaR summation bound;
  * binary32 tables: |gpu - oracle64| <= 2^-23 * 1.0001 * G_t + 1e-12 * P_k, G_t the
    trial's gross loss (two binary32 roundings per looked-up loss, each <= 2^-24
    relative, propagated through 1-Lipschitz clamps).
"""
from __future__ import annotations

import json
import math
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from exact_ara import rank_exact

pytestmark = pytest.mark.gpu

INF = math.inf
GOLD = os.path.join(os.path.dirname(__file__), "golden", "hand_worked_small.json")


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


def analyze(A, S, ctx, w, placement=0, precision=0, t0=0, t1=None, terms=None, block=0, grid_per_cu=0,
            packing=1, mode=0, binning=1):
    import torch
    A.ara_set_option(ctx, A.ARA_OPT_PLACEMENT, placement)
    A.ara_set_option(ctx, A.ARA_OPT_TRIAL_MODE, mode)
    A.ara_set_option(ctx, A.ARA_OPT_BLOCK_THREADS, block)
    A.ara_set_option(ctx, A.ARA_OPT_GRID_PER_CU, grid_per_cu)
    A.ara_set_option(ctx, A.ARA_OPT_YET_PACKING, packing)
    A.ara_set_option(ctx, A.ARA_OPT_YET_BINNING, binning)
    try:
        an = S.open_analysis(ctx, w.event_ids, w.trial_offsets, w.catalog_size, w.elts,
                             terms if terms is not None else w.layer_terms, w.elt_terms, precision)
    finally:
        A.ara_set_option(ctx, A.ARA_OPT_YET_PACKING, 1)
        A.ara_set_option(ctx, A.ARA_OPT_YET_BINNING, 1)
    try:
        # 2-byte binned copy where it applies (large catalogs), else 3-byte packed, else int32
        ib = A.ara_yet_info(an.yet)[2]
        plain = 3 if packing and w.n_events > 0 and w.catalog_size <= 1 << 24 else 4
        assert ib == plain or (binning and ib == 2 and w.catalog_size > 20480), (ib, plain)
        t1 = w.n_trials if t1 is None else t1
        ylt = torch.empty(max(t1 - t0, 1), dtype=torch.float64, device="cuda")
        A.ara_analyze(ctx, an.yet, an.layer, t0, t1, ylt)
        A.ara_sync(ctx)
        return ylt[: t1 - t0].cpu().numpy()
    finally:
        an.release()
        A.ara_set_option(ctx, A.ARA_OPT_PLACEMENT, 0)
        A.ara_set_option(ctx, A.ARA_OPT_BLOCK_THREADS, 0)
        A.ara_set_option(ctx, A.ARA_OPT_GRID_PER_CU, 0)
        A.ara_set_option(ctx, A.ARA_OPT_TRIAL_MODE, 0)


def analyze_events(A, S, ctx, w, placement=0, precision=0):
    import torch
    A.ara_set_option(ctx, A.ARA_OPT_PLACEMENT, placement)
    an = S.open_analysis(ctx, w.event_ids, w.trial_offsets, w.catalog_size, w.elts, w.layer_terms, w.elt_terms,
                         precision)
    try:
        n, ne = w.n_trials, max(w.n_events, 1)
        out = {k: torch.full((n if k == "ylt" else ne,), math.nan, dtype=torch.float64, device="cuda")
               for k in ("ylt", "gross", "occ", "cum", "ceded")}
        A.ara_analyze_events(ctx, an.yet, an.layer, 0, n, out["ylt"], out["gross"], out["occ"], out["cum"],
                             out["ceded"])
        A.ara_sync(ctx)
        res = {k: v.cpu().numpy() for k, v in out.items()}
        for k in ("gross", "occ", "cum", "ceded"):
            res[k] = res[k][: w.n_events]
        return res
    finally:
        an.release()
        A.ara_set_option(ctx, A.ARA_OPT_PLACEMENT, 0)


def assert_ylt_close(got, ref, rel=1e-12, what=""):
    y, P = ref["ylt"], ref["occ_total"]
    tol = rel * np.maximum(np.abs(y), P)
    err = np.abs(got - y)
    bad = np.nonzero(~(err <= tol))[0]
    assert bad.size == 0, (f"{what}: {bad.size} trials off; first {bad[:5]} got {got[bad[:5]]} "
                           f"want {y[bad[:5]]} tol {tol[bad[:5]]}")


PLACEMENTS = [1, 2, 3]   # LDS bitmap, LDS dense, global dense


def _gold_workload(terms=None):
    g = json.load(open(GOLD))
    elts = [(np.array(e["ids"], np.int32), np.array(e["losses"], np.float64)) for e in g["elts"]]
    trials = g["trials"]
    offs = np.zeros(len(trials) + 1, np.int64)
    offs[1:] = np.cumsum([len(t) for t in trials])
    ids = np.array([e for t in trials for e in t], np.int32)
    lt = tuple(INF if v == "inf" else float(v) for v in (terms or g["layer_terms"]))
    return g, synth.Workload("hand", ids, offs, g["catalog_size"], elts, lt, None, (1, 2, 3, 4, 6, 250), 0)


# ----------------------------------------------------------------------------- hand-worked example
@pytest.mark.parametrize("placement", PLACEMENTS)
def test_hand_worked_example(A, S, gpu_ctx, placement):
    _say(f"hand-worked example placement={placement}")
    g, w = _gold_workload()
    ex = g["expected"]
    ylt = analyze(A, S, gpu_ctx, w, placement)
    assert ylt.tolist() == [float(v) for v in ex["ylt"]]
    ev = analyze_events(A, S, gpu_ctx, w, placement)
    flat = lambda k: [float(v) for t in ex[k] for v in t]
    assert ev["gross"].tolist() == flat("gross")
    assert ev["occ"].tolist() == flat("occ")
    assert ev["cum"].tolist() == flat("cum")
    assert ev["ceded"].tolist() == flat("ceded")
    assert ev["ylt"].tolist() == [float(v) for v in ex["ylt"]]
    import torch
    pml, tvar = A.ara_risk_measures(gpu_ctx, torch.tensor(ex["ylt"], dtype=torch.float64, device="cuda"),
                                    ex["return_periods"])
    from fractions import Fraction as Fr
    assert pml.tolist() == [float(v) for v in ex["pml"]]
    assert tvar.tolist() == [float(Fr(v)) for v in ex["tvar"]]
    for key in ("pass_through_terms", "uncapped_aggregate"):
        _, w2 = _gold_workload(g["variants"][key]["layer_terms"])
        y2 = analyze(A, S, gpu_ctx, w2, placement)
        if key == "pass_through_terms":
            assert y2.tolist() == [float(v) for v in g["variants"][key]["ylt"]]
        else:
            assert y2[0] == g["variants"][key]["ylt_T0"]


# ----------------------------------------------------------------------------- exact tiny cases
@pytest.mark.parametrize("placement", PLACEMENTS)
def test_random_tiny_integer_bit_exact(A, S, gpu_ctx, placement):
    rng = np.random.default_rng(100 + placement)
    for i in range(60):
        w = synth.random_tiny(rng, integer_losses=True, financial_terms=(i % 2 == 1), events_max=40)
        _say(f"tiny integer case {i} placement={placement} C={w.catalog_size} elts={len(w.elts)} trials={w.n_trials}")
        ref = oracle.analyze_workload(w, per_event=True)
        got = analyze(A, S, gpu_ctx, w, placement)
        assert got.tolist() == ref["ylt"].tolist(), i
        if w.n_events:
            ev = analyze_events(A, S, gpu_ctx, w, placement)
            assert ev["gross"].tolist() == ref["gross"].tolist()
            assert ev["occ"].tolist() == ref["occ"].tolist()
            assert ev["cum"].tolist() == ref["cum"].tolist()
            assert ev["ceded"].tolist() == ref["ceded"].tolist()
            assert ev["ylt"].tolist() == ref["ylt"].tolist()


def test_random_tiny_real_losses(A, S, gpu_ctx):
    rng = np.random.default_rng(7)
    for i in range(40):
        w = synth.random_tiny(rng, integer_losses=False, financial_terms=(i % 3 == 0), events_max=60)
        _say(f"tiny real case {i}")
        ref = oracle.analyze_workload(w)
        for pl in PLACEMENTS:
            got = analyze(A, S, gpu_ctx, w, pl)
            assert_ylt_close(got, ref, what=f"case {i} placement {pl}")


# ----------------------------------------------------------------------------- plain 10k-trial configuration
@pytest.fixture(scope="module")
def small():
    return synth.workload_plain_small()


@pytest.mark.parametrize("placement", [0] + PLACEMENTS)
def test_plain_small_ylt(A, S, gpu_ctx, small, placement):
    _say(f"plain 10k trials placement={placement}")
    ref = oracle.analyze_workload(small, threads=oracle.max_threads())
    got = analyze(A, S, gpu_ctx, small, placement)
    assert_ylt_close(got, ref, what="plain small")
    got32 = analyze(A, S, gpu_ctx, small, placement, packing=0)
    assert got32.tobytes() == got.tobytes()   # same events, same summation order


@pytest.mark.parametrize("placement", [2, 3])
def test_lane_per_trial_is_the_sequential_sum(A, S, gpu_ctx, small, placement):
    """A lane adds its trial's occurrence-net values in time order from +0.0, exactly
    the oracle's cumulative total: the YLT equals the oracle's f(P_k) bit for bit.
    The wave-per-trial form sums in another order (within tolerance)."""
    rng = np.random.default_rng(77)
    edge = _edge_workload(rng, [0, 1, 3, 4, 5, 255, 256, 257, 1023, 1025, 2049, 0, 7, 4099, 1, 2])
    for w, name in [(small, "plain small"), (edge, "edge lengths")]:
        _say(f"lane mode {name} placement={placement}")
        ref = oracle.analyze_workload(w, threads=oracle.max_threads())
        lane = analyze(A, S, gpu_ctx, w, placement, mode=2)
        assert lane.tobytes() == ref["ylt_closed"].tobytes(), name
        wave = analyze(A, S, gpu_ctx, w, placement, mode=1)
        assert_ylt_close(wave, ref, what=name)
        for block in (256, 1024):
            assert analyze(A, S, gpu_ctx, w, placement, mode=2, block=block).tobytes() == lane.tobytes()


def test_occurrence_maximum_bit_exact(A, S, gpu_ctx, small, paper_reduced):
    """Largest occurrence-net loss per trial: a maximum of bit-exact table values, so
    it equals the oracle's bit for bit in every placement (ragged and empty trials
    included); occurrence PML comes from ara_risk_measures on it."""
    import torch
    rng = np.random.default_rng(31)
    edge = _edge_workload(rng, [0, 1, 3, 4, 5, 255, 256, 257, 1023, 1025, 2049, 0, 7, 4099, 1, 2])
    for w, pls in [(small, [1, 2, 3]), (edge, [1, 2, 3]), (paper_reduced, [1, 3, 4])]:
        ref = oracle.analyze_workload(w, threads=oracle.max_threads())["occ_max"]
        for pl in pls:
            _say(f"occurrence maxima {w.name} placement={pl}")
            A.ara_set_option(gpu_ctx, A.ARA_OPT_PLACEMENT, pl)
            an = S.open_analysis(gpu_ctx, w.event_ids, w.trial_offsets, w.catalog_size, w.elts, w.layer_terms,
                                 w.elt_terms)
            try:
                out = torch.full((w.n_trials,), math.nan, dtype=torch.float64, device="cuda")
                A.ara_analyze_occ_max(gpu_ctx, an.yet, an.layer, 0, w.n_trials, out)
                A.ara_sync(gpu_ctx)
                got = out.cpu().numpy()
                assert got.tobytes() == ref.tobytes(), (w.name, pl)
                sub = torch.empty(5, dtype=torch.float64, device="cuda")
                A.ara_analyze_occ_max(gpu_ctx, an.yet, an.layer, 3, 8, sub)
                A.ara_sync(gpu_ctx)
                assert sub.cpu().numpy().tobytes() == ref[3:8].tobytes()
            finally:
                an.release()
                A.ara_set_option(gpu_ctx, A.ARA_OPT_PLACEMENT, 0)
        pml, _ = A.ara_risk_measures(gpu_ctx, torch.from_numpy(ref).cuda(), [10.0, 100.0])
        pml_o, _, _, _ = oracle.risk(ref, [10.0, 100.0])
        assert np.asarray(pml).tobytes() == np.asarray(pml_o).tobytes()


def test_bitmap_queue_overflow_all_events_flagged(A, S, gpu_ctx):
    """Every catalog event has a nonzero occurrence-net loss, so every 256-event load
    flags more events than the per-wave queue holds: the queue is resolved early,
    slot by slot.  Checked against the oracle, with both ID encodings."""
    rng = np.random.default_rng(97)
    C = 40_000                                   # > 20,480 events: the LDS filter placement
    ids_all = np.arange(C, dtype=np.int32)
    elts = [(ids_all, rng.lognormal(8.0, 1.0, size=C)), (ids_all[::3].copy(), rng.lognormal(9.0, 1.0, size=len(ids_all[::3])))]
    lengths = [2000, 1, 0, 1023, 1024, 1025, 4100, 3, 257, 2048] * 8
    counts = np.asarray(lengths, np.int64)
    offs = np.zeros(len(counts) + 1, np.int64)
    np.cumsum(counts, out=offs[1:])
    ids = rng.integers(0, C, size=int(offs[-1])).astype(np.int32)
    w = synth.Workload("all-flagged", ids, offs, C, elts, (0.0, INF, 0.0, INF), None, (2.0,), 0)
    _say("bitmap queue overflow")
    ref = oracle.analyze_workload(w, threads=oracle.max_threads())
    got = analyze(A, S, gpu_ctx, w, 1)
    assert_ylt_close(got, ref, what="all flagged")
    assert analyze(A, S, gpu_ctx, w, 1, packing=0).tobytes() == got.tobytes()


def _catalog_lookup_reference(w, precision_f32=False):
    ids = np.arange(w.catalog_size, dtype=np.int32)
    offs = np.array([0, w.catalog_size], np.int64)
    r = oracle.analyze(ids, offs, w.catalog_size, w.elts, w.layer_terms, elt_terms=w.elt_terms,
                       per_event=True, dat_f32=precision_f32)
    return r["gross"], r["occ"]


@pytest.mark.parametrize("placement", PLACEMENTS)
def test_lookups_bit_exact_small(A, S, gpu_ctx, small, placement):
    import torch
    _say(f"lookups plain small placement={placement}")
    gross, occ = _catalog_lookup_reference(small)
    A.ara_set_option(gpu_ctx, A.ARA_OPT_PLACEMENT, placement)
    an = S.open_analysis(gpu_ctx, small.event_ids, small.trial_offsets, small.catalog_size, small.elts,
                         small.layer_terms)
    try:
        ids = torch.arange(small.catalog_size, dtype=torch.int32, device="cuda")
        g = torch.empty(small.catalog_size, dtype=torch.float64, device="cuda")
        o = torch.empty_like(g)
        A.ara_lookup(gpu_ctx, an.layer, ids, g, o)
        A.ara_sync(gpu_ctx)
        assert np.array_equal(g.cpu().numpy(), gross)
        assert np.array_equal(o.cpu().numpy(), occ)
        nz, pl, lds = A.ara_layer_stats(gpu_ctx, an.layer)
        assert nz == int(np.count_nonzero(occ))
        assert pl == placement
    finally:
        an.release()
        A.ara_set_option(gpu_ctx, A.ARA_OPT_PLACEMENT, 0)


@pytest.mark.parametrize("precision", [0, 1])
def test_rebuild_after_records_move_to_other_events(A, S, gpu_ctx, precision):
    """An ELT's table holds values only where its seen bits are set.  The caller moves
    every record of each ELT (borrowed device records, changed in place) to events it
    did not list before and rebuilds with ARA_BUILD_TABLES: the events listed before
    read 0 again.  Catalog lookups equal the oracle's for the new records bit for bit,
    and the YLT (tiled kernel: a 50,000-event catalog) matches the oracle."""
    import torch
    _say(f"rebuild with moved records precision={precision}")
    rng = np.random.default_rng(20251)
    C = 50_000
    ids, offs = synth.yet_poisson(rng, 3_000, 100.0, C)
    elts = [synth.elt_sparse(rng, 5_000, C, 10.0, 2.0) for _ in range(3)]
    et = [(1.0, 0.0, INF), (0.8, 2e3, 3e5), (1.0, 0.0, INF)]
    terms = (5e4, 1e6, 2e5, 5e6)
    moved = []
    for e_ids, _ in elts:
        free = np.setdiff1d(np.arange(C, dtype=np.int32), e_ids)
        moved.append((rng.permutation(rng.choice(free, size=e_ids.size, replace=False)).astype(np.int32),
                      rng.lognormal(10.0, 2.0, size=e_ids.size)))
    an = S.open_analysis(gpu_ctx, ids, offs, C, elts, terms, et, precision)
    try:
        assert A.ara_yet_info(an.yet)[2] == 2   # the catalog-binned copy: the tiled kernel runs
        for h, (m_ids, m_loss) in zip(an.elts, moved):
            h._keep[0].copy_(torch.from_numpy(m_ids))
            h._keep[1].copy_(torch.from_numpy(m_loss))
        A.ara_layer_build(gpu_ctx, an.layer, A.ARA_BUILD_TABLES)
        w = synth.Workload("moved", ids, offs, C, moved, terms, et, (10.0, 100.0), 0)
        gross, occ = _catalog_lookup_reference(w, precision_f32=precision == 1)
        if precision == 1:   # the binary32 combined table, then the occurrence terms in binary64
            gross = gross.astype(np.float32).astype(np.float64)
            occ = np.minimum(np.maximum(gross - terms[0], 0.0), terms[1])
        cat = torch.arange(C, dtype=torch.int32, device="cuda")
        g = torch.empty(C, dtype=torch.float64, device="cuda")
        o = torch.empty_like(g)
        A.ara_lookup(gpu_ctx, an.layer, cat, g, o)
        ylt = torch.empty(w.n_trials, dtype=torch.float64, device="cuda")
        A.ara_analyze(gpu_ctx, an.yet, an.layer, 0, w.n_trials, ylt)
        A.ara_sync(gpu_ctx)
        g, o = g.cpu().numpy(), o.cpu().numpy()
        assert np.array_equal(g, gross)
        assert np.array_equal(o, occ)
        old = np.setdiff1d(np.concatenate([e_ids for e_ids, _ in elts]), np.concatenate([m for m, _ in moved]))
        assert old.size > 0 and np.all(g[old] == 0.0)

        def check(got, ref, what):
            if precision == 0:
                assert_ylt_close(got, ref, what=what)
            else:
                bound = 2.0 ** -23 * 1.0001 * ref["gross_total"] + 1e-12 * ref["occ_total"]
                assert np.all(np.abs(got - ref["ylt"]) <= bound), what

        def bitmap_ylt():
            # the LDS-bitmap kernel reads the layer's ranks and compacted values, which a
            # rebuild leaves to the first call that needs them
            A.ara_set_option(gpu_ctx, A.ARA_OPT_PLACEMENT, A.ARA_PLACE_LDS_BITMAP)
            try:
                out = torch.full((w.n_trials,), math.nan, dtype=torch.float64, device="cuda")
                A.ara_analyze(gpu_ctx, an.yet, an.layer, 0, w.n_trials, out)
                A.ara_sync(gpu_ctx)
                return out.cpu().numpy()
            finally:
                A.ara_set_option(gpu_ctx, A.ARA_OPT_PLACEMENT, 0)

        ref = oracle.analyze_workload(w)
        check(ylt.cpu().numpy(), ref, "moved records, tiled")
        check(bitmap_ylt(), ref, "moved records, LDS bitmap")
        assert A.ara_layer_stats(gpu_ctx, an.layer)[0] == int(np.count_nonzero(occ))
        # new occurrence terms: the filter again, its ranks on first use
        terms2 = (2e5, 5e5, 1e5, 3e6)
        A.ara_layer_set_terms(gpu_ctx, an.layer, terms2)
        w2 = w.with_terms(terms2)
        ref2 = oracle.analyze_workload(w2)
        check(bitmap_ylt(), ref2, "new terms, LDS bitmap")
        occ2 = np.minimum(np.maximum(gross - terms2[0], 0.0), terms2[1])
        assert A.ara_layer_stats(gpu_ctx, an.layer)[0] == int(np.count_nonzero(occ2))
    finally:
        an.release()


def test_rebuild_detects_records_made_invalid_in_place(A, S, gpu_ctx, small):
    """A rebuild re-checks the records: an event listed twice, a negative loss or an ID
    outside the catalog, written into an ELT's borrowed device records, is reported by
    the next blocking call; restoring the records and rebuilding gives the first
    lookups and YLT again, bit for bit (every build starts from cleared seen bits)."""
    import torch
    _say("rebuild with records made invalid in place")
    an = S.open_analysis(gpu_ctx, small.event_ids, small.trial_offsets, small.catalog_size, small.elts,
                         small.layer_terms)
    try:
        cat = torch.arange(small.catalog_size, dtype=torch.int32, device="cuda")

        def outputs():
            g = torch.empty(small.catalog_size, dtype=torch.float64, device="cuda")
            ylt = torch.empty(small.n_trials, dtype=torch.float64, device="cuda")
            A.ara_lookup(gpu_ctx, an.layer, cat, g, None)
            A.ara_analyze(gpu_ctx, an.yet, an.layer, 0, small.n_trials, ylt)
            A.ara_sync(gpu_ctx)
            return g.cpu().numpy().tobytes(), ylt.cpu().numpy().tobytes()

        first = outputs()
        ids, losses = an.elts[2]._keep
        id_copy, loss_copy = ids.clone(), losses.clone()
        for what, code in [("dup", A.ARA_E_DUP_EVENT), ("loss", A.ARA_E_BAD_LOSS),
                           ("range", A.ARA_E_EVENT_ID_RANGE)]:
            if what == "dup":
                ids[7] = ids[1500]
            elif what == "loss":
                losses[11] = -1.0
            else:
                ids[13] = small.catalog_size
            A.ara_layer_build(gpu_ctx, an.layer, A.ARA_BUILD_TABLES)
            with pytest.raises(A.AraError) as e:
                A.ara_sync(gpu_ctx)
            assert e.value.status == code, what
            ids.copy_(id_copy)
            losses.copy_(loss_copy)
            A.ara_layer_build(gpu_ctx, an.layer, A.ARA_BUILD_TABLES)
            assert outputs() == first, what
    finally:
        an.release()


def test_layer_of_40_mixed_precision_elts(A, S, gpu_ctx):
    """A layer of 40 ELTs (more than the 32 whose seen bits one load brings in) whose
    tables alternate binary64 and binary32, half of them with financial terms.  A
    binary32 table stores each loss rounded to binary32, so the oracle takes those
    ELTs' losses rounded beforehand: the combined table (binary64, as the layer mixes
    precisions) then equals it bit for bit, and the YLT (tiled kernel) matches."""
    import torch
    from paper_1308_2066_amd import ara
    _say("layer of 40 ELTs, mixed precision")
    rng = np.random.default_rng(40_32)
    C = 50_000
    ids, offs = synth.yet_poisson(rng, 2_000, 100.0, C)
    elts, et, precs = [], [], []
    for j in range(40):
        e_ids, e_loss = synth.elt_sparse(rng, 3_000, C, 10.0, 2.0)
        elts.append((e_ids, e_loss))
        et.append((0.9, 1e3, 4e5) if j % 4 >= 2 else (1.0, 0.0, INF))
        precs.append(ara.ARA_F32 if j % 2 else ara.ARA_F64)
    terms = (5e4, 1e6, 2e5, 5e6)
    yet = ara.ara_yet_create(gpu_ctx, torch.from_numpy(ids).cuda(), torch.from_numpy(offs).cuda(), C)
    handles = [ara.ara_elt_create(gpu_ctx, torch.from_numpy(e_ids).cuda(), torch.from_numpy(e_loss).cuda(), C,
                                  terms=t, precision=pr)
               for (e_ids, e_loss), t, pr in zip(elts, et, precs)]
    layer = ara.ara_layer_create(gpu_ctx, handles, C, terms)
    try:
        assert A.ara_yet_info(yet)[2] == 2   # the catalog-binned copy: the tiled kernel runs
        rounded = [(e_ids, e_loss.astype(np.float32).astype(np.float64) if pr == ara.ARA_F32 else e_loss)
                   for (e_ids, e_loss), pr in zip(elts, precs)]
        w = synth.Workload("mixed-40", ids, offs, C, rounded, terms, et, (10.0, 100.0), 0)
        gross, occ = _catalog_lookup_reference(w)
        cat = torch.arange(C, dtype=torch.int32, device="cuda")
        g = torch.empty(C, dtype=torch.float64, device="cuda")
        o = torch.empty_like(g)
        A.ara_lookup(gpu_ctx, layer, cat, g, o)
        ylt = torch.full((w.n_trials,), math.nan, dtype=torch.float64, device="cuda")
        A.ara_analyze(gpu_ctx, yet, layer, 0, w.n_trials, ylt)
        A.ara_sync(gpu_ctx)
        assert np.array_equal(g.cpu().numpy(), gross)
        assert np.array_equal(o.cpu().numpy(), occ)
        assert_ylt_close(ylt.cpu().numpy(), oracle.analyze_workload(w), what="40 mixed ELTs")
    finally:
        ara.ara_layer_release(layer)
        for h in handles:
            ara.ara_elt_release(h)
        ara.ara_yet_release(yet)


def test_largest_catalog(A, S, gpu_ctx):
    """The largest catalog the library accepts, 2^28 events (byte offsets into its
    binary64 tables reach 2^31; no packed or binned YET copy, so the global-table
    kernel runs): events at both ends of the catalog, a binary32 ELT beside binary64
    ones.  Lookups bit-exact with the oracle, the YLT within the bound; a catalog of
    one event more is rejected."""
    import torch
    from paper_1308_2066_amd import ara
    _say("largest catalog, 2^28 events")
    C = 1 << 28
    rng = np.random.default_rng(1 << 28)
    hot = np.unique(np.concatenate([np.arange(C - 3000, C), np.arange(0, 3000),
                                    rng.choice(C, 6000, replace=False)])).astype(np.int32)
    precs = [ara.ARA_F64, ara.ARA_F32, ara.ARA_F64]
    elts, rounded = [], []
    for pr in precs:
        ids = np.unique(np.concatenate([[0, C - 2, C - 1], rng.choice(hot, 2000, replace=False)])).astype(np.int32)
        loss = rng.lognormal(10.0, 2.0, ids.size)
        elts.append((ids, loss))
        rounded.append((ids, loss.astype(np.float32).astype(np.float64) if pr == ara.ARA_F32 else loss))
    counts = rng.poisson(40.0, 300).astype(np.int64)
    offs = np.zeros(counts.size + 1, np.int64)
    np.cumsum(counts, out=offs[1:])
    ev = rng.choice(hot, int(offs[-1])).astype(np.int32)
    terms = (5e3, 1e6, 2e4, 5e6)
    with pytest.raises(A.AraError) as e:
        A.ara_elt_create(gpu_ctx, torch.from_numpy(elts[0][0]).cuda(), torch.from_numpy(elts[0][1]).cuda(), C + 1)
    assert e.value.status == A.ARA_E_INVALID_ARG
    yet = ara.ara_yet_create(gpu_ctx, torch.from_numpy(ev).cuda(), torch.from_numpy(offs).cuda(), C)
    handles = [ara.ara_elt_create(gpu_ctx, torch.from_numpy(i).cuda(), torch.from_numpy(l).cuda(), C, precision=pr)
               for (i, l), pr in zip(elts, precs)]
    layer = ara.ara_layer_create(gpu_ctx, handles, C, terms)
    try:
        assert A.ara_yet_info(yet)[2] == 4   # int32 IDs only
        q = torch.from_numpy(hot).cuda()
        g = torch.full((hot.size,), math.nan, dtype=torch.float64, device="cuda")
        o = torch.full_like(g, math.nan)
        A.ara_lookup(gpu_ctx, layer, q, g, o)
        ylt = torch.full((counts.size,), math.nan, dtype=torch.float64, device="cuda")
        A.ara_analyze(gpu_ctx, yet, layer, 0, counts.size, ylt)
        A.ara_sync(gpu_ctx)
        look = oracle.analyze(hot, np.array([0, hot.size], np.int64), C, rounded, terms, per_event=True)
        assert np.array_equal(g.cpu().numpy(), look["gross"])
        assert np.array_equal(o.cpu().numpy(), look["occ"])
        w = synth.Workload("largest-catalog", ev, offs, C, rounded, terms, None, (10.0, 100.0), 0)
        assert_ylt_close(ylt.cpu().numpy(), oracle.analyze_workload(w), what="2^28-event catalog")
    finally:
        ara.ara_layer_release(layer)
        for h in handles:
            ara.ara_elt_release(h)
        ara.ara_yet_release(yet)


def test_kernel_timing(A, S, gpu_ctx, small):
    """ARA_OPT_KERNEL_TIMING = n: ara_kernel_ms reports the mean trial-kernel time of the
    last min(k, n) timed ara_analyze calls, for the tiled kernel (events attached to its
    launch) and another placement (events around its launches): positive, and no longer
    than torch events recorded around the same calls; without the option, or before a
    timed call, it is an error."""
    import torch
    _say("kernel timing")
    rng = np.random.default_rng(77)
    C = 50_000
    ids, offs = synth.yet_poisson(rng, 4_000, 200.0, C)
    elts = [synth.elt_sparse(rng, 5_000, C, 10.0, 2.0) for _ in range(3)]
    tiled = S.open_analysis(gpu_ctx, ids, offs, C, elts, (5e4, 1e6, 2e5, 5e6))
    plain = S.open_analysis(gpu_ctx, small.event_ids, small.trial_offsets, small.catalog_size, small.elts,
                            small.layer_terms)
    stream = torch.cuda.current_stream()
    try:
        assert A.ara_yet_info(tiled.yet)[2] == 2
        with pytest.raises(A.AraError) as e:
            A.ara_kernel_ms(gpu_ctx)
        assert e.value.status == A.ARA_E_INVALID_ARG
        for bad in (-1, 4097):
            with pytest.raises(A.AraError):
                A.ara_set_option(gpu_ctx, A.ARA_OPT_KERNEL_TIMING, bad)
        for an in (tiled, plain):
            for ring, calls in ((1, 3), (4, 3), (2, 5)):
                A.ara_set_option(gpu_ctx, A.ARA_OPT_KERNEL_TIMING, ring)
                with pytest.raises(A.AraError):
                    A.ara_kernel_ms(gpu_ctx)          # nothing timed yet
                n = an.n_trials
                ylt = torch.empty(n, dtype=torch.float64, device="cuda")
                around = []
                for _ in range(calls):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    A.ara_analyze(gpu_ctx, an.yet, an.layer, 0, n, ylt)
                    e1.record(stream)
                    A.ara_sync(gpu_ctx)
                    around.append(e0.elapsed_time(e1))
                ms = A.ara_kernel_ms(gpu_ctx)
                last = around[-min(ring, calls):]
                assert 0.0 < ms <= float(np.mean(last)) * 1.001 + 1e-3, (ring, calls, ms, last)
        A.ara_set_option(gpu_ctx, A.ARA_OPT_KERNEL_TIMING, 0)
        with pytest.raises(A.AraError):
            A.ara_kernel_ms(gpu_ctx)
    finally:
        A.ara_set_option(gpu_ctx, A.ARA_OPT_KERNEL_TIMING, 0)
        tiled.release()
        plain.release()


def test_plain_small_events_mode(A, S, gpu_ctx, small):
    _say("events mode plain small")
    ref = oracle.analyze_workload(small, per_event=True, threads=oracle.max_threads())
    ev = analyze_events(A, S, gpu_ctx, small)
    assert np.array_equal(ev["gross"], ref["gross"])
    assert np.array_equal(ev["occ"], ref["occ"])
    Pk = np.repeat(ref["occ_total"], np.diff(small.trial_offsets))
    assert np.all(np.abs(ev["cum"] - ref["cum"]) <= 1e-12 * Pk)
    assert np.all(np.abs(ev["ceded"] - ref["ceded"]) <= 2e-12 * Pk)
    assert_ylt_close(ev["ylt"], ref, what="events-mode ylt")


@pytest.mark.parametrize("terms", [(5e4, 1e6, 2e5, 5e6), (5e4, 1e6, 2e5, INF), (5e4, 1e6, 3e6, INF)])
def test_plain_small_risk_measures(A, S, gpu_ctx, small, terms):
    import torch
    _say(f"risk measures plain small terms={terms}")
    w = small.with_terms(terms)
    ref = oracle.analyze_workload(w, threads=oracle.max_threads())
    got = analyze(A, S, gpu_ctx, w)
    assert_ylt_close(got, ref)
    rps = [1.0, 2.0, 10.0, 100.0, 250.0, 1000.0, 10_000.0]
    pml_o, tvar_o, ranks_o, _ = oracle.risk(ref["ylt"], rps)
    pml, tvar = A.ara_risk_measures(gpu_ctx, torch.from_numpy(got).cuda(), rps)
    ranks = [A.ara_return_period_rank(len(got), rp) for rp in rps]
    assert ranks == ranks_o.tolist()
    # the GPU's PML is exactly its own k-th order statistic
    srt = np.sort(got)[::-1]
    assert pml.tolist() == [srt[k - 1] for k in ranks]
    ytol = float(np.max(1e-12 * np.maximum(np.abs(ref["ylt"]), ref["occ_total"])))
    assert np.all(np.abs(pml - pml_o) <= ytol)
    k = np.array(ranks, dtype=np.float64)
    assert np.all(np.abs(tvar - tvar_o) <= ytol + 2 * k * 2.0 ** -53 * np.abs(tvar_o))


# ----------------------------------------------------------------------------- edge cases
def _edge_workload(rng, lengths, catalog=5000, n_elts=3, lead=0):
    lengths = np.asarray(lengths, np.int64)
    offs = np.zeros(len(lengths) + 1, np.int64)
    offs[1:] = np.cumsum(lengths)
    ids = rng.integers(0, catalog, size=int(offs[-1])).astype(np.int32)
    elts = [synth.elt_sparse(rng, catalog // 3, catalog, 10.0, 2.0) for _ in range(n_elts)]
    return synth.Workload("edge", ids, offs, catalog, elts, (5e4, 1e6, 2e5, INF), None, (10.0,), 0)


@pytest.mark.parametrize("placement", PLACEMENTS)
def test_edge_trial_lengths(A, S, gpu_ctx, placement):
    rng = np.random.default_rng(55)
    # the tail: lengths about the half of a 256-occurrence chunk in the per-occurrence kernel
    lengths = [0, 1, 3, 4, 5, 255, 256, 257, 1023, 1024, 1025, 2047, 2049, 3000, 0, 0, 7, 4099, 1, 2,
               127, 128, 129, 131]
    w = _edge_workload(rng, lengths)
    assert w.n_events % 4 != 0
    _say(f"edge lengths placement={placement} n_events={w.n_events}")
    ref = oracle.analyze_workload(w, per_event=True)
    got = analyze(A, S, gpu_ctx, w, placement)
    assert_ylt_close(got, ref)
    assert analyze(A, S, gpu_ctx, w, placement, packing=0).tobytes() == got.tobytes()
    ev = analyze_events(A, S, gpu_ctx, w, placement)
    assert np.array_equal(ev["gross"], ref["gross"]) and np.array_equal(ev["occ"], ref["occ"])
    Pk = np.repeat(ref["occ_total"], np.diff(w.trial_offsets))
    assert np.all(np.abs(ev["cum"] - ref["cum"]) <= 1e-12 * Pk)
    assert np.all(np.abs(ev["ceded"] - ref["ceded"]) <= 2e-12 * Pk)
    assert_ylt_close(ev["ylt"], ref, what="events-mode ylt")
    # sub-ranges of trials
    for t0, t1 in [(0, 1), (3, 11), (13, 20), (5, 5), (19, 20)]:
        sub = analyze(A, S, gpu_ctx, w, placement, t0=t0, t1=t1)
        assert np.array_equal(sub, got[t0:t1])


def test_single_trial_and_last_partial_group(A, S, gpu_ctx):
    rng = np.random.default_rng(9)
    for n in [1, 2, 3, 5, 6, 7, 1021, 1022, 1023, 4097]:
        w = _edge_workload(rng, [n])
        _say(f"single trial n={n}")
        ref = oracle.analyze_workload(w)
        for pl in PLACEMENTS:
            for pk in (1, 0):
                assert_ylt_close(analyze(A, S, gpu_ctx, w, pl, packing=pk), ref, what=f"n={n} pl={pl} pk={pk}")


def test_many_short_trials_and_empty_layer(A, S, gpu_ctx):
    rng = np.random.default_rng(21)
    w = _edge_workload(rng, rng.integers(0, 9, size=5000))
    _say("many short trials")
    ref = oracle.analyze_workload(w)
    for pl in PLACEMENTS:
        assert_ylt_close(analyze(A, S, gpu_ctx, w, pl), ref)
    w0 = synth.Workload("empty-layer", w.event_ids, w.trial_offsets, w.catalog_size, [], w.layer_terms)
    for pl in PLACEMENTS:
        assert not np.any(analyze(A, S, gpu_ctx, w0, pl))


def test_schedule_independence_and_determinism(A, S, gpu_ctx, small):
    _say("schedule independence")
    base = analyze(A, S, gpu_ctx, small)
    for block, gpc in [(256, 1), (512, 2), (1024, 1), (256, 8), (1024, 0)]:
        again = analyze(A, S, gpu_ctx, small, block=block, grid_per_cu=gpc)
        assert again.tobytes() == base.tobytes(), (block, gpc)


# ----------------------------------------------------------------------------- sort
@pytest.mark.parametrize("n", [1, 2, 63, 2047, 2049, 4095, 4096, 4097, 100_003, 1_000_000, 4_500_001])
def test_sort_bit_exact(A, gpu_ctx, n):
    import torch
    _say(f"sort n={n}")
    rng = np.random.default_rng(n)
    x = rng.lognormal(10, 3, size=n)
    x[rng.random(n) < 0.2] = 0.0
    x[rng.random(n) < 0.05] = -0.0
    x[rng.random(n) < 0.1] = 5e6          # ties
    x[rng.random(n) < 0.01] = 1e-300
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    A.ara_sort_desc(gpu_ctx, torch.from_numpy(x).cuda(), out)
    A.ara_sync(gpu_ctx)
    got = out.cpu().numpy()
    want = np.sort(x + 0.0)[::-1]
    assert got.tobytes() == want.tobytes()


@pytest.mark.parametrize("n,kind", [(300_001, "mixed"), (1_000_000, "constant"), (70_000, "mixed")])
def test_risk_measures_large_k(A, gpu_ctx, n, kind):
    """PML/TVaR with k up to n (chunked top-k sums): ranks identical, PML bit-exact,
    TVaR within the summation bound of a k-term sum of non-negative values."""
    import torch
    _say(f"risk large k n={n} kind={kind}")
    rng = np.random.default_rng(n + 17)
    if kind == "constant":
        y = np.full(n, 5e7)
    else:
        y = rng.lognormal(12, 2, size=n)
        y[rng.random(n) < 0.3] = 0.0
        y[rng.random(n) < 0.05] = 5e7
    rps = [1.0, 1.5, 2.0, 10.0, 100.0, float(n), 2.0 * n]
    pml_o, tvar_o, ranks_o, _ = oracle.risk(y, rps)
    pml, tvar = A.ara_risk_measures(gpu_ctx, torch.from_numpy(y).cuda(), rps)
    assert [A.ara_return_period_rank(n, rp) for rp in rps] == list(ranks_o)
    assert np.asarray(pml).tobytes() == np.asarray(pml_o).tobytes()
    k = np.asarray(ranks_o, dtype=np.float64)
    bound = 2.0 * k * 2.0 ** -53 * np.asarray(tvar_o) + 1e-300
    assert np.all(np.abs(np.asarray(tvar) - tvar_o) <= bound), (tvar, tvar_o)


@pytest.mark.parametrize("n,kind", [(16_384, "distinct"), (16_385, "distinct"), (50_000, "ties_at_k"),
                                    (200_000, "tie_block"), (1_000_000, "distinct"), (123_457, "two_values")])
def test_risk_measures_selection_paths(A, gpu_ctx, n, kind):
    """PML/TVaR against the oracle on YLTs that take each path of the selection: the
    one-workgroup sort (n <= 16384), buckets copied out and sorted with ties at the
    k-th loss, a tie block larger than any bucket that can be copied (every digit
    picked from counts), and two values only; ranks identical, PML bit-exact, TVaR
    within the summation bound, and the same bits on a second call."""
    import torch
    _say(f"risk selection paths n={n} kind={kind}")
    rng = np.random.default_rng(n * 7 + len(kind))
    rps = [1.0, 2.0, 3.0, 10.0, 100.0, 250.0, 1000.0, float(n)]
    y = rng.lognormal(13, 2.2, size=n)
    if kind == "ties_at_k":
        for rp in (10.0, 100.0):   # 300 copies of the loss at each rank
            k = A.ara_return_period_rank(n, rp)
            v = np.sort(y)[::-1][k - 1]
            y[rng.choice(n, 300, replace=False)] = v
    elif kind == "tie_block":
        y[rng.random(n) < 0.4] = float(np.quantile(y, 0.9))
    elif kind == "two_values":
        y = np.where(rng.random(n) < 0.25, 7.5e6, 1.25e6)
    pml_o, tvar_o, ranks_o, _ = oracle.risk(y, rps)
    yt = torch.from_numpy(y).cuda()
    pml, tvar = A.ara_risk_measures(gpu_ctx, yt, rps)
    assert [A.ara_return_period_rank(n, rp) for rp in rps] == list(ranks_o)
    assert np.asarray(pml).tobytes() == np.asarray(pml_o).tobytes()
    k = np.asarray(ranks_o, dtype=np.float64)
    bound = 2.0 * k * 2.0 ** -53 * np.asarray(tvar_o) + 1e-300
    assert np.all(np.abs(np.asarray(tvar) - tvar_o) <= bound), (tvar, tvar_o)
    pml2, tvar2 = A.ara_risk_measures(gpu_ctx, yt, rps)   # the same bits on a second call
    assert np.asarray(pml2).tobytes() == np.asarray(pml).tobytes()
    assert np.asarray(tvar2).tobytes() == np.asarray(tvar).tobytes()


def test_packed_copy_only_below_2_24(A, gpu_ctx):
    import torch
    _say("packed copy catalog limit")
    ids = torch.zeros(8, dtype=torch.int32, device="cuda")
    offs = torch.tensor([0, 5, 8], dtype=torch.int64, device="cuda")
    for cat, want in [(1 << 24, 3), ((1 << 24) + 1, 4), (1, 3)]:
        y = A.ara_yet_create(gpu_ctx, ids, offs, cat)
        try:
            assert A.ara_yet_info(y) == (8, 2, want)
        finally:
            A.ara_yet_release(y)
    A.ara_set_option(gpu_ctx, A.ARA_OPT_YET_PACKING, 0)
    try:
        y = A.ara_yet_create(gpu_ctx, ids, offs, 100)
        assert A.ara_yet_info(y)[2] == 4
        A.ara_yet_release(y)
    finally:
        A.ara_set_option(gpu_ctx, A.ARA_OPT_YET_PACKING, 1)


# ----------------------------------------------------------------------------- errors
def test_input_errors(A, S, gpu_ctx):
    import torch
    _say("input errors")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    with pytest.raises(A.AraError) as e:
        A.ara_yet_create(gpu_ctx, dev(np.array([0, 5, 9], np.int32)), dev(np.array([0, 3], np.int64)), 9)
    assert e.value.status == A.ARA_E_EVENT_ID_RANGE
    with pytest.raises(A.AraError) as e:
        A.ara_yet_create(gpu_ctx, dev(np.array([0, 5, 8], np.int32)), dev(np.array([0, 2, 1, 3], np.int64)), 9)
    assert e.value.status == A.ARA_E_BAD_OFFSETS
    with pytest.raises(A.AraError) as e:
        A.ara_yet_create(gpu_ctx, dev(np.array([0, 5, 8], np.int32)), dev(np.array([0, 2], np.int64)), 9)
    assert e.value.status == A.ARA_E_BAD_OFFSETS
    for ids, losses, code in [([1, 1], [1.0, 2.0], A.ARA_E_DUP_EVENT), ([9], [1.0], A.ARA_E_EVENT_ID_RANGE),
                              ([1], [-1.0], A.ARA_E_BAD_LOSS), ([1], [math.nan], A.ARA_E_BAD_LOSS),
                              ([2], [math.inf], A.ARA_E_BAD_LOSS)]:
        with pytest.raises(A.AraError) as e:
            A.ara_elt_create(gpu_ctx, dev(np.array(ids, np.int32)), dev(np.array(losses)), 9)
        assert e.value.status == code
    with pytest.raises(A.AraError) as e:
        A.ara_elt_create(gpu_ctx, dev(np.array([1], np.int32)), dev(np.array([1.0])), 9, terms=(-1.0, 0.0, 1.0))
    assert e.value.status == A.ARA_E_BAD_TERMS
    elt = A.ara_elt_create(gpu_ctx, dev(np.array([1], np.int32)), dev(np.array([1.0])), 9)
    with pytest.raises(A.AraError) as e:
        A.ara_layer_create(gpu_ctx, [elt], 10, (0, 1, 0, 1))
    assert e.value.status == A.ARA_E_INVALID_ARG
    with pytest.raises(A.AraError) as e:
        A.ara_layer_create(gpu_ctx, [elt], 9, (0, 1, -1, 1))
    assert e.value.status == A.ARA_E_BAD_TERMS
    layer = A.ara_layer_create(gpu_ctx, [elt], 9, (0, 1, 0, 1))
    with pytest.raises(A.AraError) as e:
        A.ara_elt_release(elt)
    assert e.value.status == A.ARA_E_BUSY
    yet = A.ara_yet_create(gpu_ctx, dev(np.array([0, 5, 8], np.int32)), dev(np.array([0, 3], np.int64)), 9)
    y = torch.empty(1, dtype=torch.float64, device="cuda")
    with pytest.raises(A.AraError) as e:
        A.ara_analyze(gpu_ctx, yet, layer, 0, 2, torch.empty(2, dtype=torch.float64, device="cuda"))
    assert e.value.status == A.ARA_E_INVALID_ARG
    with pytest.raises(A.AraError) as e:
        A.ara_risk_measures(gpu_ctx, torch.empty(0, dtype=torch.float64, device="cuda"), [10.0])
    assert e.value.status == A.ARA_E_EMPTY
    with pytest.raises(A.AraError) as e:
        A.ara_risk_measures(gpu_ctx, y, [0.5])
    assert e.value.status == A.ARA_E_INVALID_ARG
    with pytest.raises(A.AraError) as e:
        A.ara_set_option(gpu_ctx, A.ARA_OPT_BLOCK_THREADS, 100)
    assert e.value.status == A.ARA_E_INVALID_ARG
    A.ara_analyze(gpu_ctx, yet, layer, 0, 1, y)
    A.ara_sync(gpu_ctx)
    A.ara_layer_release(layer)
    A.ara_elt_release(elt)
    A.ara_yet_release(yet)


# ----------------------------------------------------------------------------- paper-scale shape
@pytest.fixture(scope="module")
def paper_reduced():
    return synth.workload_paper_scale(n_trials=20_000)


def _twin_terms(w, ref_occ_total):
    # aggregate terms that do not saturate: retention near the median occurrence-net total, no limit
    return (w.layer_terms[0], w.layer_terms[1], float(np.median(ref_occ_total)), INF)


def test_paper_shape_reduced_f64(A, S, gpu_ctx, paper_reduced):
    w = paper_reduced
    _say("paper shape 20k x 1000 f64")
    ref = oracle.analyze_workload(w, threads=oracle.max_threads())
    got = analyze(A, S, gpu_ctx, w)
    assert_ylt_close(got, ref, what="saturating terms")
    twin = _twin_terms(w, ref["occ_total"])
    ref2 = oracle.analyze_workload(w.with_terms(twin), threads=oracle.max_threads())
    assert np.count_nonzero(ref2["ylt"]) > w.n_trials // 3
    for pl in [1, 3]:
        got2 = analyze(A, S, gpu_ctx, w, pl, terms=twin)
        assert_ylt_close(got2, ref2, what=f"twin placement {pl}")
        assert analyze(A, S, gpu_ctx, w, pl, terms=twin, packing=0).tobytes() == got2.tobytes()
    # a 1M-event catalog does not fit LDS as a dense table: forcing it is refused
    with pytest.raises(A.AraError) as e:
        analyze(A, S, gpu_ctx, w, 2, terms=twin)
    assert e.value.status == A.ARA_E_UNSUPPORTED


def test_paper_shape_lookups_bit_exact(A, S, gpu_ctx, paper_reduced):
    import torch
    w = paper_reduced
    _say("paper shape lookups")
    gross, occ = _catalog_lookup_reference(w)
    for pl in [1, 3]:
        A.ara_set_option(gpu_ctx, A.ARA_OPT_PLACEMENT, pl)
        an = S.open_analysis(gpu_ctx, w.event_ids[:4], np.array([0, 4], np.int64), w.catalog_size, w.elts,
                             w.layer_terms)
        try:
            ids = torch.arange(w.catalog_size, dtype=torch.int32, device="cuda")
            g = torch.empty(w.catalog_size, dtype=torch.float64, device="cuda")
            o = torch.empty_like(g)
            A.ara_lookup(gpu_ctx, an.layer, ids, g, o)
            A.ara_sync(gpu_ctx)
            assert np.array_equal(g.cpu().numpy(), gross)
            assert np.array_equal(o.cpu().numpy(), occ)
        finally:
            an.release()
            A.ara_set_option(gpu_ctx, A.ARA_OPT_PLACEMENT, 0)


def test_paper_shape_reduced_f32_tables(A, S, gpu_ctx, paper_reduced):
    import torch
    w = paper_reduced
    _say("paper shape 20k x 1000 f32 tables")
    twin = None
    ref = oracle.analyze_workload(w, threads=oracle.max_threads())
    twin = _twin_terms(w, ref["occ_total"])
    for terms in [w.layer_terms, twin]:
        ref = oracle.analyze_workload(w.with_terms(terms), threads=oracle.max_threads())
        got = analyze(A, S, gpu_ctx, w, precision=1, terms=terms)
        bound = 2.0 ** -23 * 1.0001 * ref["gross_total"] + 1e-12 * ref["occ_total"]
        assert np.all(np.abs(got - ref["ylt"]) <= bound)
    # the binary32 combined table equals the binary32 rounding of the oracle's sum of binary32 losses
    gross32, _ = _catalog_lookup_reference(w, precision_f32=True)
    an = S.open_analysis(gpu_ctx, w.event_ids[:4], np.array([0, 4], np.int64), w.catalog_size, w.elts,
                         w.layer_terms, None, 1)
    try:
        ids = torch.arange(w.catalog_size, dtype=torch.int32, device="cuda")
        g = torch.empty(w.catalog_size, dtype=torch.float64, device="cuda")
        A.ara_lookup(gpu_ctx, an.layer, ids, g, None)
        A.ara_sync(gpu_ctx)
        assert np.array_equal(g.cpu().numpy(), gross32.astype(np.float32).astype(np.float64))
    finally:
        an.release()
    # per-occurrence gross losses through the binary32 tables (the events kernel reads
    # the combined table only where its nonzero bit is set): the same table values
    nt = 500
    e1 = int(w.trial_offsets[nt])
    an = S.open_analysis(gpu_ctx, w.event_ids[:e1], w.trial_offsets[: nt + 1], w.catalog_size, w.elts,
                         w.layer_terms, None, 1)
    try:
        gev = torch.full((e1,), math.nan, dtype=torch.float64, device="cuda")
        A.ara_analyze_events(gpu_ctx, an.yet, an.layer, 0, nt, None, gev, None, None, None)
        A.ara_sync(gpu_ctx)
        want = gross32.astype(np.float32).astype(np.float64)[w.event_ids[:e1]]
        assert np.array_equal(gev.cpu().numpy(), want)
    finally:
        an.release()
