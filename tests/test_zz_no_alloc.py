"""The allocation-free risk measures call (ara_risk_measures_noalloc): through the
C-ABI, its PML and TVaR equal ara_risk_measures' with a caller workspace bit for
bit, on two calls in a row (the second on a shorter YLT, so it runs on what the
first left in the shared device array), and on the largest YLT it takes; longer
YLTs are rejected."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

RPS = [1.0, 2.0, 10.0, 100.0, 250.0, 1000.0, 1e6]


def _ylt(n, seed):
    import torch
    rng = np.random.default_rng(seed)
    y = rng.lognormal(14.0, 2.0, size=n)
    y[rng.integers(0, n, size=max(1, n // 10))] = 0.0     # ties at zero, as in uncapped YLTs
    y[rng.integers(0, n, size=max(1, n // 20))] = 5e7     # ties at an aggregate limit
    return torch.from_numpy(y).cuda()


def _both(A, ctx, y):
    import torch
    ws = torch.empty(A.ara_sort_workspace_size(y.numel()), dtype=torch.uint8, device="cuda")
    ref = A.ara_risk_measures(ctx, y, RPS, ws)
    got = A.ara_risk_measures_noalloc(ctx, y, RPS)
    return ref, got


def test_noalloc_equals_workspace_call_twice_then_smaller(ara_lib, gpu_ctx):
    A = ara_lib
    for n, seed in [(1_000_000, 1), (70_001, 2), (1, 3)]:
        print(f"noalloc: n={n} seed={seed}", flush=True)
        (pml_r, tvar_r), (pml_g, tvar_g) = _both(A, gpu_ctx, _ylt(n, seed))
        assert pml_g.tobytes() == pml_r.tobytes(), n
        assert tvar_g.tobytes() == tvar_r.tobytes(), n


def test_noalloc_largest_and_too_long(ara_lib, gpu_ctx):
    A = ara_lib
    n = A.ARA_NOALLOC_MAX_N
    (pml_r, tvar_r), (pml_g, tvar_g) = _both(A, gpu_ctx, _ylt(n, 4))
    assert pml_g.tobytes() == pml_r.tobytes() and tvar_g.tobytes() == tvar_r.tobytes()
    import torch
    y = torch.zeros(n + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(A.AraError) as ei:
        A.ara_risk_measures_noalloc(gpu_ctx, y, RPS)
    assert ei.value.status == A.ARA_E_INVALID_ARG
    with pytest.raises(A.AraError) as ei:
        A.ara_risk_measures_noalloc(gpu_ctx, y[:0], RPS)
    assert ei.value.status == A.ARA_E_EMPTY
    # the context still works after the rejected calls
    (pml_r, tvar_r), (pml_g, tvar_g) = _both(A, gpu_ctx, _ylt(1000, 5))
    assert pml_g.tobytes() == pml_r.tobytes() and tvar_g.tobytes() == tvar_r.tobytes()
