"""The C-ABI from a plain C program (tests/ara_c_client.c, no Python or torch in the
process): a hand-worked four-trial example through ara_analyze, ara_analyze_occ_max and
ara_risk_measures, checked against the oracle and against values worked out by hand.

The example: catalog of 5 events; ELT 1 = {0: 40, 2: 100, 3: 5}, ELT 2 = {0: 15,
1: 70, 3: 2} (identity financial terms), so the combined table is
[55, 70, 100, 7, 0]; occurrence terms retention 10, limit 50 give occurrence-net
losses [45, 50, 50, 0, 0]; trials [3,0,2,0,4], [1], [], [2,2] have P = 140, 50, 0,
100; aggregate retention 30, limit 100 give YLT = [100, 20, 0, 70]; occurrence maxima
[50, 50, 0, 50].  Ranks for N = 4 at return periods 1, 2, 4 are k = 4, 2, 1:
PML = [0, 70, 100], TVaR = [47.5, 85, 100]."""
from __future__ import annotations

import os
import subprocess

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLIENT = os.path.join(ROOT, "tests", "_build", "ara_c_client")


def _run_client():
    if not os.path.exists(CLIENT):
        raise RuntimeError(f"{CLIENT} is missing: run __graft_entry__.build() first")
    print(f"[case] C client {CLIENT}", flush=True)
    r = subprocess.run([CLIENT], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    out = {}
    for ln in r.stdout.splitlines():
        name, idx, val = ln.split()
        out.setdefault(name, {})[int(idx)] = float(val)
    return {k: np.array([v[i] for i in range(len(v))]) for k, v in out.items()}


def test_c_client_hand_example():
    got = _run_client()
    ids = np.array([3, 0, 2, 0, 4, 1, 2, 2], np.int32)
    offs = np.array([0, 5, 6, 6, 8], np.int64)
    elts = [(np.array([0, 2, 3], np.int32), np.array([40.0, 100.0, 5.0])),
            (np.array([0, 1, 3], np.int32), np.array([15.0, 70.0, 2.0]))]
    ref = oracle.analyze(ids, offs, 5, elts, (10.0, 50.0, 30.0, 100.0))
    rps = [1.0, 2.0, 4.0]
    pml_o, tvar_o, _, _ = oracle.risk(ref["ylt"], rps)
    # small integers: every step is exact in binary64, so equality is the bar
    assert got["ylt"].tolist() == ref["ylt"].tolist() == [100.0, 20.0, 0.0, 70.0]
    assert got["occ_max"].tolist() == ref["occ_max"].tolist() == [50.0, 50.0, 0.0, 50.0]
    assert got["pml"].tolist() == list(pml_o) == [0.0, 70.0, 100.0]
    assert got["tvar"].tolist() == list(tvar_o) == [47.5, 85.0, 100.0]
