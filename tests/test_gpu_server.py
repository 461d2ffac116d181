"""Pricing server on the GPU: requests batched by the worker give exactly the results
of the same analysis run alone (a layer of the same pool ELTs, ara_analyze,
ara_risk_measures), whether they arrive together or one by one; the served PML/TVaR
match the oracle within the binary32-table bound; iterations overlap (two in flight at
once); admission holds requests whose YLT does not fit the memory budget yet."""
from __future__ import annotations

import sys
import threading

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
def served(ara_lib, gpu_ctx):
    """The plain small YET and the batched portfolio's 256-ELT pool, resident."""
    from paper_1308_2066_amd import session
    pf = synth.portfolio_batched(n_layers=1)
    h = session.open_portfolio(gpu_ctx, pf.event_ids, pf.trial_offsets, pf.catalog_size, pf.pool, [])
    yield pf, h
    h.release()


def _requests(rng, n, pool, n_trials, long_ranges=False):
    out = []
    for _ in range(n):
        k = int(rng.integers(1, 33))
        idx = [int(i) for i in rng.choice(pool, size=k, replace=False)]
        terms = synth.loguniform_terms(rng)
        if long_ranges or rng.random() < 0.5:
            t0 = int(rng.integers(0, n_trials // 2))
            t1 = int(rng.integers(t0 + 1, n_trials + 1))
        else:
            t0 = int(rng.integers(0, n_trials - 10))
            t1 = t0 + int(rng.integers(1, 10))
        out.append((idx, terms, t0, t1))
    return out


def _alone(A, ctx, h, req, rps):
    import torch
    idx, terms, t0, t1 = req
    layer = A.ara_layer_create(ctx, [h.pool[i] for i in idx], h.yet.catalog_size, terms)
    try:
        y = torch.empty(t1 - t0, dtype=torch.float64, device="cuda")
        A.ara_analyze(ctx, h.yet, layer, t0, t1, y)
        pml, tvar = A.ara_risk_measures(ctx, y, rps)
        return np.asarray(pml), np.asarray(tvar)
    finally:
        A.ara_layer_release(layer)


def test_server_results_equal_alone(A, gpu_ctx, served):
    pf, h = served
    rps = list(pf.return_periods) + [1.0, 2.0]
    rng = np.random.default_rng(11)
    reqs = _requests(rng, 48, len(h.pool), pf.n_trials)
    srv = A.ara_server_create(gpu_ctx, h.yet, h.pool, rps, max_batch=8)
    try:
        _say("server: 48 requests at once")
        tickets = [A.ara_server_submit(srv, *r) for r in reqs]
        mixed = [A.ara_server_wait(srv, t) for t in tickets]
        st = A.ara_server_stats(srv)
        assert st["completed"] == len(reqs) and st["slots"] == 16
        assert st["iterations"] < len(reqs) and st["max_in_iteration"] > 1          # requests were batched
        _say("server: the same requests one by one")
        for r, (pml, tvar, sec) in zip(reqs, mixed):
            t = A.ara_server_submit(srv, *r)
            p1, v1, _ = A.ara_server_wait(srv, t)
            assert p1.tobytes() == pml.tobytes() and v1.tobytes() == tvar.tobytes()
            assert sec >= 0.0
        _say("server: against the plain launches")
        for r, (pml, tvar, _) in zip(reqs, mixed):
            p0, v0 = _alone(A, gpu_ctx, h, r, rps)
            assert pml.tobytes() == p0.tobytes() and tvar.tobytes() == v0.tobytes(), r
    finally:
        A.ara_server_release(srv)


def test_server_concurrent_clients(A, gpu_ctx, served):
    """Several client threads submitting and waiting at once."""
    pf, h = served
    rps = list(pf.return_periods)
    srv = A.ara_server_create(gpu_ctx, h.yet, h.pool, rps, max_batch=4)
    results, errors = {}, []

    def client(seed):
        try:
            rng = np.random.default_rng(seed)
            for r in _requests(rng, 6, len(h.pool), pf.n_trials):
                t = A.ara_server_submit(srv, *r)
                results[(seed, t)] = (r, A.ara_server_wait(srv, t))
        except Exception as e:        # reported below
            errors.append(e)

    try:
        threads = [threading.Thread(target=client, args=(s,)) for s in range(5)]
        for t in threads:
            t.start()
        for t in threads:
            t.join(timeout=120)
        assert not errors, errors
        assert len(results) == 30
        for (seed, _), (r, (pml, tvar, _)) in list(results.items())[:10]:
            p0, v0 = _alone(A, gpu_ctx, h, r, rps)
            assert pml.tobytes() == p0.tobytes() and tvar.tobytes() == v0.tobytes()
    finally:
        A.ara_server_release(srv)


def test_server_rejects_bad_requests(A, gpu_ctx, served):
    pf, h = served
    srv = A.ara_server_create(gpu_ctx, h.yet, h.pool, [10.0], max_batch=2)
    try:
        for args, status in [(([], (0, 1, 0, 1), 0, 5), A.ARA_E_INVALID_ARG),
                             (([256], (0, 1, 0, 1), 0, 5), A.ARA_E_INVALID_ARG),
                             (([1], (0, 1, 0, 1), 5, 5), A.ARA_E_INVALID_ARG),
                             (([1], (0, 1, 0, 1), 0, pf.n_trials + 1), A.ARA_E_INVALID_ARG),
                             (([1], (-1, 1, 0, 1), 0, 5), A.ARA_E_BAD_TERMS)]:
            with pytest.raises(A.AraError) as e:
                A.ara_server_submit(srv, *args)
            assert e.value.status == status, args
        with pytest.raises(A.AraError) as e:
            A.ara_server_wait(srv, 12345)
        assert e.value.status == A.ARA_E_INVALID_ARG
        t = A.ara_server_submit(srv, [3, 1], (1e4, 1e6, 0, 1e8), 0, 100)
        pml, tvar, _ = A.ara_server_wait(srv, t)
        assert pml.shape == (1,) and tvar[0] >= pml[0]
    finally:
        A.ara_server_release(srv)
    with pytest.raises(A.AraError) as e:
        A.ara_server_create(gpu_ctx, h.yet, h.pool, [0.5])
    assert e.value.status == A.ARA_E_INVALID_ARG


def _oracle_check(pf, req, rps, pml, tvar):
    """PML/TVaR of a served request against the oracle: ranks are the rank rule's,
    values within the YLT bound of binary32 tables (two binary32 roundings of each
    looked-up loss: 2^-23 * G_t) plus the binary64 summation bound."""
    idx, terms, t0, t1 = req
    r = oracle.analyze(pf.event_ids, pf.trial_offsets, pf.catalog_size, [pf.pool[i] for i in idx], terms,
                       t_begin=t0, t_end=t1, dat_f32=True, threads=oracle.max_threads())
    pml_o, tvar_o, ranks, _ = oracle.risk(r["ylt"], rps)
    tol = float(np.max(2.0 ** -23 * 1.0001 * r["gross_total"] + 1e-12 * np.maximum(np.abs(r["ylt"]), r["occ_total"])))
    assert np.all(np.abs(pml - pml_o) <= tol), (req, pml, pml_o)
    assert np.all(np.abs(tvar - tvar_o) <= tol + 2.0 * np.asarray(ranks) * 2.0 ** -53 * tvar_o), (req, tvar, tvar_o)


def test_served_results_match_oracle(A, gpu_ctx, served):
    """A sample of served requests (submitted together, so they are batched and their
    iterations overlap) against the CPU oracle."""
    pf, h = served
    rps = [1.0, 2.0, 10.0, 100.0, 250.0]
    rng = np.random.default_rng(21)
    reqs = _requests(rng, 12, len(h.pool), pf.n_trials)
    reqs.append((list(range(32)), (1e4, 1e8, 0.0, 1e12), 0, pf.n_trials))     # 32 ELTs, the whole YET
    reqs.append(([5], (0.0, float("inf"), 0.0, float("inf")), 7, 8))            # one trial, pass-through terms
    srv = A.ara_server_create(gpu_ctx, h.yet, h.pool, rps, max_batch=4)
    try:
        _say("server vs oracle: 14 requests")
        tickets = [A.ara_server_submit(srv, *r) for r in reqs]
        got = [A.ara_server_wait(srv, t) for t in tickets]
        for n in range(len(reqs)):
            assert A.ara_return_period_rank(reqs[n][3] - reqs[n][2], 10.0) == oracle.rank(reqs[n][3] - reqs[n][2], 10.0)
        for r, (pml, tvar, _) in zip(reqs, got):
            _oracle_check(pf, r, rps, pml, tvar)
    finally:
        A.ara_server_release(srv)


def test_iterations_overlap(A, gpu_ctx, served):
    """With requests queued faster than one iteration completes, the worker enqueues the
    next iteration on the other lane while the first is on the GPU: more requests are
    in flight at once than one iteration holds."""
    pf, h = served
    rps = list(pf.return_periods)
    rng = np.random.default_rng(23)
    reqs = _requests(rng, 40, len(h.pool), pf.n_trials, long_ranges=True)
    srv = A.ara_server_create(gpu_ctx, h.yet, h.pool, rps, max_batch=4)
    try:
        _say("server overlap: 40 requests, 4 per iteration")
        tickets = [A.ara_server_submit(srv, *r) for r in reqs]
        got = [A.ara_server_wait(srv, t) for t in tickets]
        st = A.ara_server_stats(srv)
        assert st["completed"] == 40 and st["max_in_iteration"] <= 4
        assert st["max_in_flight"] > st["max_in_iteration"], st
        for r, (pml, tvar, _) in list(zip(reqs, got))[:6]:
            p0, v0 = _alone(A, gpu_ctx, h, r, rps)
            assert pml.tobytes() == p0.tobytes() and tvar.tobytes() == v0.tobytes()
    finally:
        A.ara_server_release(srv)


def test_admission_by_memory_holds_and_completes(A, gpu_ctx, served):
    """A budget with room for one whole-YET YLT: requests over the whole YET are
    admitted one at a time (each waits for the previous one's completion), small ones
    share the arena; every request completes with the bits of its analysis alone.  A
    request larger than the arena is refused at submission."""
    pf, h = served
    rps = list(pf.return_periods)
    probe = A.ara_server_create(gpu_ctx, h.yet, h.pool, rps, max_batch=1)
    slot_bytes = A.ara_server_stats(probe)["slot_bytes"]
    A.ara_server_release(probe)
    n = pf.n_trials
    budget = 2 * slot_bytes + 8 * n          # two slots (one per lane) and one whole-YET YLT
    srv = A.ara_server_create(gpu_ctx, h.yet, h.pool, rps, max_batch=8, memory_budget=budget)
    try:
        st = A.ara_server_stats(srv)
        assert st["slots"] == 2 and st["arena_bytes"] == 8 * n, st
        rng = np.random.default_rng(29)
        whole = [(sorted(int(i) for i in rng.choice(len(h.pool), size=int(rng.integers(1, 33)), replace=False)),
                  synth.loguniform_terms(rng), 0, n) for _ in range(6)]
        small = [(list(r[0]), r[1], 100 * k, 100 * k + 50) for k, r in enumerate(whole)]
        reqs = [x for pair in zip(whole, small) for x in pair]
        _say("server admission: 12 requests, budget for one whole-YET YLT")
        tickets = [A.ara_server_submit(srv, *r) for r in reqs]
        got = [A.ara_server_wait(srv, t) for t in tickets]
        st = A.ara_server_stats(srv)
        assert st["completed"] == 12 and st["held"] > 0, st
        assert st["max_in_flight"] <= 2 and st["iterations"] >= 7, st
        for r, (pml, tvar, _) in zip(reqs, got):
            p0, v0 = _alone(A, gpu_ctx, h, r, rps)
            assert pml.tobytes() == p0.tobytes() and tvar.tobytes() == v0.tobytes(), r
        t = A.ara_server_submit(srv, [1], (0, 1, 0, 1), 0, n)           # exactly the arena: accepted
        A.ara_server_wait(srv, t)
    finally:
        A.ara_server_release(srv)
    tiny = A.ara_server_create(gpu_ctx, h.yet, h.pool, rps, max_batch=1, memory_budget=2 * slot_bytes + 8 * 100)
    try:
        with pytest.raises(A.AraError) as e:
            A.ara_server_submit(tiny, [1], (0, 1, 0, 1), 0, 101)
        assert e.value.status == A.ARA_E_OOM
    finally:
        A.ara_server_release(tiny)
