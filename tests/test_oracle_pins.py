"""Pins for the CPU oracle: checks that tie it to the paper and to mathematics,
not to itself.  CPU only.

* a hand-worked example (tests/golden/hand_worked_small.json);
* exact rational brute force on random tiny inputs (bit-exact where every
  intermediate is representable, within a rounding bound otherwise);
* closed forms: pass-through terms give the summed losses, a single
  occurrence reduces to the composition of the two clamps, the aggregate
  differences telescope to f(P_k);
* invariants: monotone in limits, antitone in retentions, exact scaling by 2,
  trial permutation, event permutation within a trial;
* brute-force order statistics for PML/TVaR and the rank rule.
"""
from __future__ import annotations

import json
import math
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
import synth
from exact_ara import rank_exact, trial_exact, workload_exact

GOLD = os.path.join(os.path.dirname(__file__), "golden", "hand_worked_small.json")
INF = math.inf


def _gold():
    with open(GOLD) as f:
        g = json.load(f)
    elts = [(np.array(e["ids"], np.int32), np.array(e["losses"], np.float64)) for e in g["elts"]]
    trials = g["trials"]
    offs = np.zeros(len(trials) + 1, np.int64)
    offs[1:] = np.cumsum([len(t) for t in trials])
    ids = np.array([e for t in trials for e in t], np.int32)
    return g, elts, ids, offs


def _terms(lst):
    return tuple(INF if v == "inf" else float(v) for v in lst)


# ----------------------------------------------------------------------------- hand-worked example
def test_hand_worked_example_per_event_and_ylt():
    g, elts, ids, offs = _gold()
    r = oracle.analyze(ids, offs, g["catalog_size"], elts, _terms(g["layer_terms"]), per_event=True)
    ex = g["expected"]
    flat = lambda key: np.array([v for t in ex[key] for v in t], np.float64)
    assert np.array_equal(r["gross"], flat("gross"))
    assert np.array_equal(r["occ"], flat("occ"))
    assert np.array_equal(r["cum"], flat("cum"))
    assert np.array_equal(r["ceded"], flat("ceded"))
    assert np.array_equal(r["ylt"], np.array(ex["ylt"], np.float64))
    assert np.array_equal(r["ylt_closed"], np.array(ex["ylt"], np.float64))


def test_hand_worked_example_pml_tvar():
    g, elts, ids, offs = _gold()
    ex = g["expected"]
    pml, tvar, ranks, srt = oracle.risk(np.array(ex["ylt"], np.float64), ex["return_periods"])
    assert ranks.tolist() == ex["ranks"]
    assert pml.tolist() == [float(v) for v in ex["pml"]]
    assert tvar.tolist() == [float(Fr(v)) for v in ex["tvar"]]
    assert srt.tolist() == sorted(map(float, ex["ylt"]), reverse=True)


def test_hand_worked_variants():
    g, elts, ids, offs = _gold()
    v = g["variants"]
    t0 = np.array(v["reordered_T0"]["trial"], np.int32)
    r = oracle.analyze(t0, np.array([0, len(t0)], np.int64), 5, elts, _terms(g["layer_terms"]), per_event=True)
    assert r["ceded"].tolist() == v["reordered_T0"]["ceded"]
    assert r["ylt"].tolist() == [v["reordered_T0"]["ylt"]]
    r = oracle.analyze(ids, offs, 5, elts, _terms(v["pass_through_terms"]["layer_terms"]))
    assert r["ylt"].tolist() == v["pass_through_terms"]["ylt"]
    r = oracle.analyze(ids, offs, 5, elts, _terms(v["uncapped_aggregate"]["layer_terms"]))
    assert r["ylt"][0] == v["uncapped_aggregate"]["ylt_T0"]


# ----------------------------------------------------------------------------- exact brute force
@pytest.mark.parametrize("financial", [False, True])
def test_exact_bruteforce_integer_inputs_bit_exact(financial):
    """Integer losses/terms with dyadic fx: every intermediate is exact in binary64,
    so the oracle must equal the rational brute force bit for bit."""
    rng = np.random.default_rng(11 + financial)
    for _ in range(300):
        w = synth.random_tiny(rng, integer_losses=True, financial_terms=financial)
        r = oracle.analyze_workload(w, per_event=True)
        ex = workload_exact(w)
        assert r["ylt"].tolist() == [float(e["lr"]) for e in ex]
        assert r["ylt_closed"].tolist() == [float(e["lr_closed"]) for e in ex]
        assert r["occ_total"].tolist() == [float(e["P"]) for e in ex]
        assert r["gross"].tolist() == [float(v) for e in ex for v in e["gross"]]
        assert r["occ"].tolist() == [float(v) for e in ex for v in e["occ"]]
        assert r["ceded"].tolist() == [float(v) for e in ex for v in e["ceded"]]
        assert r["occ_max"].tolist() == [float(e["occ_max"]) for e in ex]


@pytest.mark.parametrize("financial", [False, True])
def test_exact_bruteforce_real_losses_within_rounding(financial):
    """Lognormal losses: the oracle is within a small multiple of the unit
    roundoff of the exact result, scaled by the trial's loss magnitude."""
    rng = np.random.default_rng(23 + financial)
    for _ in range(200):
        w = synth.random_tiny(rng, integer_losses=False, financial_terms=financial)
        r = oracle.analyze_workload(w, per_event=True)
        ex = workload_exact(w)
        for t, e in enumerate(ex):
            scale = float(sum(e["gross"], Fr(0))) + float(e["P"]) + 1.0
            assert abs(r["ylt"][t] - float(e["lr"])) <= 1e-13 * scale
            assert abs(r["ylt_closed"][t] - float(e["lr_closed"])) <= 1e-13 * scale
            # the largest occurrence-net loss: a max of values each within a few ulps
            assert abs(r["occ_max"][t] - float(e["occ_max"])) <= 1e-14 * 8 * (float(e["occ_max"]) + 1e-300)
        # looked-up per-event gross is a short sum: within a few ulps
        g_ex = np.array([float(v) for e in ex for v in e["gross"]])
        assert np.all(np.abs(r["gross"] - g_ex) <= 1e-14 * (np.abs(g_ex) + 1e-300) * 8)


def test_f32_dat_storage_matches_rounded_losses():
    rng = np.random.default_rng(5)
    for _ in range(100):
        w = synth.random_tiny(rng)
        r = oracle.analyze_workload(w, per_event=True, dat_f32=True)
        ex = workload_exact(w, f32_losses=True)
        g_ex = np.array([float(v) for e in ex for v in e["gross"]])
        assert np.all(np.abs(r["gross"] - g_ex) <= 1e-14 * 8 * np.abs(g_ex))
        # f32 rounding really happened: with f32 storage the gross equals sums of float32 values
        assert np.all(np.abs(r["gross"] - g_ex) <= np.abs(g_ex) * 2.0 ** -50)


# ----------------------------------------------------------------------------- closed forms
def test_pass_through_terms_equal_summed_losses():
    """OccR = AggR = 0, limits infinite: the trial loss is the sum over its
    occurrences of the losses summed across ELTs (independent numpy formulation)."""
    w = synth.workload_plain_small().with_terms((0.0, INF, 0.0, INF))
    r = oracle.analyze_workload(w)
    comb = np.zeros(w.catalog_size)
    for ids, losses in w.elts:                 # ELTs in layer order, starting from +0.0
        add = np.zeros(w.catalog_size)
        add[ids] = losses
        comb = comb + add
    x = comb[w.event_ids]
    trial = np.repeat(np.arange(w.n_trials), np.diff(w.trial_offsets))
    expect = np.bincount(trial, weights=x, minlength=w.n_trials)   # sequential in event order
    assert np.array_equal(r["ylt_closed"], expect)
    assert np.array_equal(r["occ_total"], expect)
    assert np.allclose(r["ylt"], expect, rtol=1e-12, atol=0)


def test_single_occurrence_reduces_to_composed_clamps():
    rng = np.random.default_rng(3)
    w = synth.workload_plain_small()
    n = 5000
    ids = rng.integers(0, w.catalog_size, n).astype(np.int32)
    offs = np.arange(n + 1, dtype=np.int64)
    occR, occL, aggR, aggL = 5e4, 1e6, 2e5, 5e6
    for terms in [(occR, occL, aggR, aggL), (occR, occL, 0.0, INF), (0.0, INF, aggR, aggL), (1e5, 3e5, 1e4, 1e5)]:
        r = oracle.analyze(ids, offs, w.catalog_size, w.elts, terms, per_event=True)
        x = r["gross"]
        occ = np.minimum(np.maximum(x - terms[0], 0.0), terms[1])
        expect = np.minimum(np.maximum(occ - terms[2], 0.0), terms[3])
        assert np.array_equal(r["ylt"], expect)


def test_occurrence_maximum_bounds_and_single_occurrence():
    """The largest occurrence-net loss is at most the trial's total and at most OccL,
    equals the total for one-occurrence trials, and is 0 exactly for empty trials."""
    rng = np.random.default_rng(41)
    for _ in range(100):
        w = synth.random_tiny(rng, integer_losses=False)
        r = oracle.analyze_workload(w, per_event=True)
        counts = np.diff(w.trial_offsets)
        assert np.all(r["occ_max"] <= r["occ_total"])
        assert np.all(r["occ_max"] <= w.layer_terms[1])
        assert np.all(r["occ_max"][counts == 0] == 0.0)
        assert np.array_equal(r["occ_max"][counts == 1], r["occ_total"][counts == 1])
        for t in range(w.n_trials):
            ev = r["occ"][w.trial_offsets[t] - w.trial_offsets[0]:w.trial_offsets[t + 1] - w.trial_offsets[0]]
            assert r["occ_max"][t] == (ev.max() if ev.size else 0.0)


def test_aggregate_differences_telescope():
    """lr (sum of differences) equals f(P_k) up to rounding of the k differences."""
    w = synth.workload_plain_small()
    for terms in [w.layer_terms, (5e4, 1e6, 2e5, INF), (5e4, 1e6, 3e6, 2e6)]:
        r = oracle.analyze_workload(w.with_terms(terms))
        k = np.diff(w.trial_offsets).astype(np.float64)
        gamma = (k + 1) * 2.0 ** -53 / (1 - (k + 1) * 2.0 ** -53)
        assert np.all(np.abs(r["ylt"] - r["ylt_closed"]) <= 2 * gamma * np.maximum(r["occ_total"], r["ylt_closed"]))


# ----------------------------------------------------------------------------- invariants
def test_monotone_in_limits_antitone_in_retentions():
    w = synth.workload_plain_small()
    base = np.array(w.layer_terms)
    r0 = oracle.analyze_workload(w)["ylt_closed"]
    for i, sign in [(0, -1), (1, +1), (2, -1), (3, +1)]:
        t = base.copy()
        t[i] = t[i] * 1.7
        r1 = oracle.analyze_workload(w.with_terms(t))["ylt_closed"]
        if sign > 0:
            assert np.all(r1 >= r0)
        else:
            assert np.all(r1 <= r0)
        assert np.any(r1 != r0)


def test_bounds_zero_to_aggregate_limit():
    w = synth.workload_plain_small()
    r = oracle.analyze_workload(w)
    assert np.all(r["ylt_closed"] >= 0) and np.all(r["ylt_closed"] <= w.layer_terms[3])
    assert np.all(r["ylt"] >= -1e-9) and np.all(r["ylt"] <= w.layer_terms[3] * (1 + 1e-12))


def test_exact_scaling_by_two():
    w = synth.workload_plain_small()
    r1 = oracle.analyze_workload(w, per_event=True)
    w2 = synth.Workload(w.name, w.event_ids, w.trial_offsets, w.catalog_size,
                        [(i, l * 2.0) for i, l in w.elts], tuple(2.0 * t for t in w.layer_terms))
    r2 = oracle.analyze_workload(w2, per_event=True)
    for key in ("ylt", "ylt_closed", "gross", "ceded", "cum"):
        assert np.array_equal(r2[key], 2.0 * r1[key]), key


def test_trial_permutation_permutes_ylt_and_keeps_measures():
    w = synth.workload_plain_small().with_terms((5e4, 1e6, 2e5, INF))
    r = oracle.analyze_workload(w)
    rng = np.random.default_rng(9)
    perm = rng.permutation(w.n_trials)
    lens = np.diff(w.trial_offsets)
    ids = np.concatenate([w.event_ids[w.trial_offsets[t]:w.trial_offsets[t + 1]] for t in perm])
    offs = np.zeros(w.n_trials + 1, np.int64)
    offs[1:] = np.cumsum(lens[perm])
    rp = oracle.analyze(ids, offs, w.catalog_size, w.elts, w.layer_terms)
    assert np.array_equal(rp["ylt"], r["ylt"][perm])
    a = oracle.risk(r["ylt"], w.return_periods)
    b = oracle.risk(rp["ylt"], w.return_periods)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_event_order_within_trial_changes_only_rounding():
    w = synth.workload_plain_small().with_terms((5e4, 1e6, 2e5, INF))
    r = oracle.analyze_workload(w)
    rng = np.random.default_rng(4)
    ids = w.event_ids.copy()
    for t in range(w.n_trials):
        a, b = w.trial_offsets[t], w.trial_offsets[t + 1]
        ids[a:b] = rng.permutation(ids[a:b])
    r2 = oracle.analyze(ids, w.trial_offsets, w.catalog_size, w.elts, w.layer_terms)
    assert np.allclose(r2["ylt"], r["ylt"], rtol=1e-12, atol=1e-6)


# ----------------------------------------------------------------------------- order statistics
def test_rank_rule_special_cases():
    assert oracle.rank(10_000, 10) == 1000
    assert oracle.rank(10_000, 100) == 100
    assert oracle.rank(10_000, 250) == 40
    assert oracle.rank(49, 4.9) == 10          # 49/4.9 rounds to 10.000000000000002 in binary64
    assert oracle.rank(10, 3) == 4
    assert oracle.rank(6, 4) == 2
    assert oracle.rank(5, 1) == 5
    assert oracle.rank(5, 1e9) == 1
    assert oracle.rank(5, INF) == 1
    assert oracle.rank(0, 10) == -1
    assert oracle.rank(5, 0.5) == -1
    assert oracle.rank(5, float("nan")) == -1


def test_rank_rule_matches_exact_ceiling():
    rng = np.random.default_rng(8)
    for _ in range(2000):
        n = int(rng.integers(1, 10 ** 6))
        rp = float(rng.choice([1, 2, 3, 4, 5, 7, 10, 20, 25, 50, 100, 200, 250, 500, 1000, 10_000]))
        assert oracle.rank(n, rp) == rank_exact(n, Fr(rp))


def test_pml_tvar_brute_force():
    rng = np.random.default_rng(12)
    for _ in range(300):
        n = int(rng.integers(1, 40))
        y = np.round(rng.lognormal(2, 2, n), 3)
        if rng.random() < 0.3:
            y[rng.random(n) < 0.5] = 0.0
        rps = [1.0, 1.5, 2.0, 3.0, 7.0, 100.0]
        pml, tvar, ranks, srt = oracle.risk(y, rps)
        s = sorted(y.tolist(), reverse=True)
        assert srt.tolist() == s
        for i, rp in enumerate(rps):
            k = rank_exact(n, Fr(rp))
            assert ranks[i] == k
            assert pml[i] == s[k - 1]
            exact = sum((Fr(v) for v in s[:k]), Fr(0)) / k
            assert abs(tvar[i] - float(exact)) <= 1e-15 * k * max(s[0], 1e-300)
            assert tvar[i] >= pml[i] * (1 - 1e-15)
        assert pml[0] == min(s) and pml[-1] == s[rank_exact(n, Fr(100)) - 1]
        assert list(pml) == sorted(pml)                       # non-decreasing in return period
        assert abs(tvar[0] - float(sum((Fr(v) for v in s), Fr(0)) / n)) <= 1e-15 * n * max(s[0], 1e-300)


def test_negative_zero_canonicalised():
    pml, tvar, ranks, srt = oracle.risk(np.array([-0.0, 0.0, -0.0]), [1.0])
    assert all(math.copysign(1.0, v) > 0 for v in srt)
    assert math.copysign(1.0, pml[0]) > 0


# ----------------------------------------------------------------------------- input errors
def test_rejects_invalid_inputs():
    g, elts, ids, offs = _gold()
    lt = _terms(g["layer_terms"])
    cases = [
        (dict(elts=[(np.array([0, 0], np.int32), np.array([1.0, 2.0]))]), -5),
        (dict(elts=[(np.array([5], np.int32), np.array([1.0]))]), -2),
        (dict(elts=[(np.array([1], np.int32), np.array([-1.0]))]), -4),
        (dict(elts=[(np.array([1], np.int32), np.array([np.nan]))]), -4),
        (dict(elts=[(np.array([1], np.int32), np.array([np.inf]))]), -4),
        (dict(layer_terms=(-1.0, 1.0, 0.0, 1.0)), -6),
        (dict(layer_terms=(np.nan, 1.0, 0.0, 1.0)), -6),
        (dict(layer_terms=(0.0, 1.0, INF, 1.0)), -6),
        (dict(layer_terms=(0.0, -1.0, 0.0, 1.0)), -6),
        (dict(event_ids=np.array([0, 9], np.int32), trial_offsets=np.array([0, 2], np.int64)), -2),
        (dict(event_ids=np.array([0, 1], np.int32), trial_offsets=np.array([0, 2, 1], np.int64)), -3),
    ]
    for kw, code in cases:
        args = dict(event_ids=ids, trial_offsets=offs, catalog_size=5, elts=elts, layer_terms=lt)
        args.update(kw)
        with pytest.raises(oracle.OracleError) as ei:
            oracle.analyze(**args)
        assert ei.value.code == code, kw
    with pytest.raises(oracle.OracleError):
        oracle.risk(np.zeros(0), [10.0])
    with pytest.raises(oracle.OracleError):
        oracle.risk(np.ones(3), [0.5])


def test_threads_do_not_change_results():
    w = synth.workload_plain_small()
    a = oracle.analyze_workload(w, threads=1)
    b = oracle.analyze_workload(w, threads=4)
    for k in a:
        assert np.array_equal(a[k], b[k])


def test_trial_subrange_matches_full_run():
    w = synth.workload_plain_small()
    a = oracle.analyze_workload(w, per_event=True)
    b = oracle.analyze_workload(w, t_begin=1234, t_end=4321, per_event=True)
    assert np.array_equal(a["ylt"][1234:4321], b["ylt"])
    e0, e1 = w.trial_offsets[1234], w.trial_offsets[4321]
    assert np.array_equal(a["ceded"][e0:e1], b["ceded"])
