"""Pricing server on the GPU: requests batched by the worker give exactly the results
of the same analysis run alone (a layer of the same pool ELTs, ara_analyze,
ara_risk_measures), whether they arrive together or one by one."""
from __future__ import annotations

import sys
import threading

import numpy as np
import pytest

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
        iterations, completed, most, slots = A.ara_server_stats(srv)
        assert completed == len(reqs) and slots == 8
        assert iterations < len(reqs) and most > 1          # requests were batched
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
