"""Exact (rational) brute force of the analysis on tiny inputs -- a pin for the oracle.

Every loss and term is converted to ``fractions.Fraction`` (exact for binary64
values) and the analysis of Section II-B is evaluated without rounding, by a
plain dictionary lookup per ELT (no direct access tables) and two independent
formulations of the aggregate step:

* ``literal``: the cumulative sum, aggregate terms and differences, as the
  paper's step 4 describes them;
* ``closed``: min(max(P_k - AggR, 0), AggL) with P_k the trial's total of
  occurrence-net losses.  Because every occurrence-net loss is >= 0, the
  cumulative sum is non-decreasing and the aggregate clamp f is non-decreasing
  with f(0) = 0, so the differences telescope to f(P_k).

Infinite limits are represented by ``None`` (no cap).
"""
from __future__ import annotations

import math
from fractions import Fraction as Fr
from typing import Dict, List, Optional, Sequence, Tuple


def _q(x: float) -> Optional[Fr]:
    return None if math.isinf(x) else Fr(x)


def excess(x: Fr, retention: Fr, limit: Optional[Fr]) -> Fr:
    v = x - retention
    if v < 0:
        v = Fr(0)
    if limit is not None and v > limit:
        v = limit
    return v


def trial_exact(events: Sequence[int], elts: List[Dict[int, Fr]], elt_terms, layer_terms,
                f32_losses: bool = False):
    """Exact analysis of one trial.  Returns dict(lr, lr_closed, P, gross, occ, cum, ceded,
    occ_max), occ_max being the largest occurrence-net loss (0 for an empty trial)."""
    occR, occL, aggR, aggL = (_q(layer_terms[0]), _q(layer_terms[1]), _q(layer_terms[2]), _q(layer_terms[3]))
    gross = []
    for e in events:
        s = Fr(0)
        for j, table in enumerate(elts):
            l = table.get(int(e), Fr(0))
            if elt_terms is not None:
                fx, r, lim = elt_terms[j]
                l = excess(Fr(fx) * l, Fr(r), _q(lim))
            s += l
        gross.append(s)
    occ = [excess(x, occR, occL) for x in gross]
    cum, run = [], Fr(0)
    for v in occ:
        run += v
        cum.append(run)
    F = [excess(p, aggR, aggL) for p in cum]
    ceded = [F[i] - (F[i - 1] if i else Fr(0)) for i in range(len(F))]
    lr = sum(ceded, Fr(0))
    closed = excess(run, aggR, aggL)
    occ_max = max(occ, default=Fr(0))
    return dict(lr=lr, lr_closed=closed, P=run, gross=gross, occ=occ, cum=cum, ceded=ceded, occ_max=occ_max)


def workload_exact(w, f32_losses: bool = False):
    """Exact per-trial results for an object with the fields of ``synth.Workload``."""
    import numpy as np
    elts = []
    for ids, losses in w.elts:
        d = {}
        for i, l in zip(ids.tolist(), losses.tolist()):
            d[int(i)] = Fr(float(np.float32(l))) if f32_losses else Fr(l)
        elts.append(d)
    out = []
    offs = w.trial_offsets
    for t in range(w.n_trials):
        ev = w.event_ids[offs[t]:offs[t + 1]].tolist()
        out.append(trial_exact(ev, elts, w.elt_terms, w.layer_terms))
    return out


def rank_exact(n: int, rp: Fr) -> int:
    """ceil(n / rp) clamped to [1, n], in exact arithmetic."""
    q = Fr(n) / rp
    k = -((-q.numerator) // q.denominator)
    return max(1, min(n, k))
