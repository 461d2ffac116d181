"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of oracle/ara_oracle.c (a dropped term, a
wrong sign or index, a transposed operand, an exclusive instead of inclusive
prefix, ...), builds the copy with the oracle's own compiler flags, and runs
tests/test_oracle_pins.py against it in a subprocess (the oracle binding loads the
copy named by ARA_ORACLE_LIB).  The pins must fail for every mutant, and pass for
an unmodified copy built the same way.  CPU only: nothing here touches a GPU.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ara_oracle.c")
PINS = os.path.join(ROOT, "tests", "test_oracle_pins.py")

# (name, text in the oracle source, replacement).  Each text occurs exactly once.
MUTATIONS = [
    ("exclusive prefix (step 4 sum bounds)",
     "{ run += lo[d]; P[d] = run; }", "{ P[d] = run; run += lo[d]; }"),
    ("occurrence limit dropped (step 3)",
     "lo[d] = clamp_excess(lo[d], OccR, OccL);", "lo[d] = clamp_excess(lo[d], OccR, INFINITY);"),
    ("occurrence retention and limit transposed (step 3)",
     "lo[d] = clamp_excess(lo[d], OccR, OccL);", "lo[d] = clamp_excess(lo[d], OccL, OccR);"),
    ("aggregate retention dropped (step 4)",
     "F[d] = clamp_excess(P[d], AggR, AggL);", "F[d] = clamp_excess(P[d], 0.0, AggL);"),
    ("difference against the occurrence before last",
     "c[d] = F[d] - (d > 0 ? F[d - 1] : 0.0);", "c[d] = F[d] - (d > 1 ? F[d - 2] : 0.0);"),
    ("difference with the wrong sign",
     "c[d] = F[d] - (d > 0 ? F[d - 1] : 0.0);", "c[d] = (d > 0 ? F[d - 1] : 0.0) - F[d];"),
    ("first ELT of the layer skipped (steps 1-2)",
     "for (int32_t j = 0; j < n_elts; ++j) {\n                    const double *tab",
     "for (int32_t j = 1; j < n_elts; ++j) {\n                    const double *tab"),
    ("ELT losses overwritten instead of accumulated (step 2)",
     "for (int64_t d = 0; d < k; ++d) lo[d] += x[d];", "for (int64_t d = 0; d < k; ++d) lo[d] = x[d];"),
    ("financial terms: fx dropped",
     "x[d] = clamp_excess(fx * x[d], fr, fl);", "x[d] = clamp_excess(x[d], fr, fl);"),
    ("financial terms: retention and limit transposed",
     "x[d] = clamp_excess(fx * x[d], fr, fl);", "x[d] = clamp_excess(fx * x[d], fl, fr);"),
    ("binary32 table rounding dropped",
     "dat[id] = dat_f32 ? (double)(float)l : l;", "dat[id] = l;"),
    ("rank rule: floor instead of ceiling",
     "double k = (fabs(q - r) <= 4.0 * ulp) ? r : ceil(q);", "double k = (fabs(q - r) <= 4.0 * ulp) ? r : floor(q);"),
    ("PML one rank too far",
     "pml[i] = y[k - 1];", "pml[i] = y[k < n ? k : k - 1];"),
    ("TVaR divided by k + 1",
     "tvar[i] = s / (double)k;", "tvar[i] = s / (double)(k + 1);"),
    ("ascending instead of descending order",
     "return (x < y) - (x > y);", "return (x > y) - (x < y);"),
    ("-0.0 not canonicalised",
     "y[i] = ylt[i] + 0.0;", "y[i] = ylt[i];"),
    ("occurrence maximum of the gross losses",
     "m = lo[d] > m ? lo[d] : m;", "m = x[d] > m ? x[d] : m;"),
    ("duplicate events accepted",
     "if (seen[id]) return OR_E_DUP_EVENT;", ""),
]


def _build(src_text: str, out_dir: str, tag: str) -> str:
    c = os.path.join(out_dir, f"oracle_{tag}.c")
    so = os.path.join(out_dir, f"liboracle_{tag}.so")
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                           "-shared", "-w", "-o", so, c, "-lm"])
    return so


def _run_pins(so: str) -> subprocess.CompletedProcess:
    env = dict(os.environ, ARA_ORACLE_LIB=so, OMP_NUM_THREADS="2")
    return subprocess.run([sys.executable, "-m", "pytest", PINS, "-x", "-q", "-p", "no:cacheprovider"],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


def test_every_mutation_fails_the_pins(tmp_path):
    with open(SRC) as f:
        src = f.read()
    jobs = [("control", src)]
    for k, (name, old, new) in enumerate(MUTATIONS):
        assert src.count(old) == 1, f"mutation {name!r}: its text must occur exactly once"
        jobs.append((f"m{k}", src.replace(old, new)))

    def one(job):
        tag, text = job
        return tag, _run_pins(_build(text, str(tmp_path), tag))

    with ThreadPoolExecutor(max_workers=4) as ex:
        results = dict(ex.map(one, jobs))
    control = results.pop("control")
    assert control.returncode == 0, "unmodified copy must pass the pins:\n" + control.stdout[-2000:]
    survived = []
    for k, (name, _, _) in enumerate(MUTATIONS):
        r = results[f"m{k}"]
        # 1 = tests ran and failed; anything else (collection error, crash) would not show a pin catching it
        if r.returncode != 1:
            survived.append(f"{name} (pytest exit {r.returncode})\n{r.stdout[-800:]}")
    assert not survived, "mutations the pins did not catch:\n" + "\n".join(survived)
