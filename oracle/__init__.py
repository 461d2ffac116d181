"""CPU oracle for aggregate risk analysis -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls it, and the two share no
code.

The arithmetic lives in ``ara_oracle.c`` (plain C, binary64, no contraction),
which follows the paper's basic sequential algorithm (Section II-B) literally,
with per-ELT direct access tables (Section III-B) and the layer terms of
Table I.  This module only marshals numpy arrays to it and builds it with gcc
when the shared object is missing or older than its source.

Every function here is pinned by the CPU tests in ``tests/test_oracle_pins.py``
(hand-worked example, exact rational brute force, closed forms, invariants,
brute-force quantiles).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ara_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# The mutation test (tests/test_oracle_mutations.py) points this at a build of a copy
# of ara_oracle.c with one planted mistake, to show that the pins catch it.
_ALT_LIB = os.environ.get("ARA_ORACLE_LIB")
_lock = threading.Lock()
_lib = None

ERRORS = {0: "ok", -1: "invalid argument", -2: "event id out of range", -3: "bad trial offsets",
          -4: "bad loss", -5: "duplicate event in an ELT", -6: "bad terms", -7: "empty", -8: "out of memory"}


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}: {ERRORS.get(code, '?')}")
        self.code = code


def build(force: bool = False) -> str:
    """Compile ara_oracle.c into liboracle.so (gcc, -O2, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if _ALT_LIB:
                lib = ctypes.CDLL(_ALT_LIB)
            else:
                build()
                lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            lib.oracle_analyze.restype = ctypes.c_int
            lib.oracle_analyze.argtypes = [P, P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                           P, P, P, P, ctypes.c_int, P, P, P, P, P, P, P, P, P, P, ctypes.c_int]
            lib.oracle_rank.restype = ctypes.c_int64
            lib.oracle_rank.argtypes = [ctypes.c_int64, ctypes.c_double]
            lib.oracle_risk.restype = ctypes.c_int
            lib.oracle_risk.argtypes = [P, ctypes.c_int64, P, ctypes.c_int32, P, P, P, P]
            lib.oracle_check_layer_terms.restype = ctypes.c_int
            lib.oracle_check_layer_terms.argtypes = [P]
            lib.oracle_max_threads.restype = ctypes.c_int
            lib.oracle_max_threads.argtypes = []
            _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def analyze(event_ids, trial_offsets, catalog_size: int, elts, layer_terms, elt_terms=None,
            t_begin: int = 0, t_end: Optional[int] = None, dat_f32: bool = False,
            per_event: bool = False, threads: int = 1) -> dict:
    """Run the literal analysis over trials [t_begin, t_end).

    ``elts`` is a list of (ids int32, losses float64) pairs in the layer's order;
    ``elt_terms`` an optional list of (fx, retention, limit); ``layer_terms`` is
    (OccR, OccL, AggR, AggL).  Returns a dict with per-trial ``ylt``,
    ``occ_total`` (P_k), ``gross_total``, ``ylt_closed`` and ``occ_max`` (the largest
    occurrence-net loss); with ``per_event``
    also ``gross``, ``occ``, ``cum`` and ``ceded`` per occurrence.
    """
    lib = _load()
    ids = np.ascontiguousarray(event_ids, dtype=np.int32)
    offs = np.ascontiguousarray(trial_offsets, dtype=np.int64)
    n_trials = offs.shape[0] - 1
    t_end = n_trials if t_end is None else int(t_end)
    t_begin = int(t_begin)
    if not (0 <= t_begin <= t_end <= n_trials):
        raise ValueError("bad trial range")
    n_elts = len(elts)
    eoff = np.zeros(n_elts + 1, dtype=np.int64)
    for j, (ei, _) in enumerate(elts):
        eoff[j + 1] = eoff[j] + len(ei)
    pid = np.ascontiguousarray(np.concatenate([np.asarray(e[0], dtype=np.int32) for e in elts])
                               if n_elts else np.zeros(0, np.int32), dtype=np.int32)
    plo = np.ascontiguousarray(np.concatenate([np.asarray(e[1], dtype=np.float64) for e in elts])
                               if n_elts else np.zeros(0, np.float64), dtype=np.float64)
    et = None
    if elt_terms is not None:
        et = np.ascontiguousarray(np.asarray(elt_terms, dtype=np.float64).reshape(n_elts, 3))
    lt = np.ascontiguousarray(np.asarray(layer_terms, dtype=np.float64).reshape(4))
    nt = t_end - t_begin
    out = {k: np.empty(nt, dtype=np.float64) for k in ("ylt", "occ_total", "gross_total", "ylt_closed", "occ_max")}
    nev = int(offs[t_end] - offs[t_begin]) if n_trials >= 0 and nt > 0 else 0
    ev = {k: (np.empty(nev, dtype=np.float64) if per_event else None) for k in ("gross", "occ", "cum", "ceded")}
    rc = lib.oracle_analyze(_ptr(ids), _ptr(offs), t_begin, t_end, int(catalog_size), n_elts, _ptr(eoff),
                            _ptr(pid), _ptr(plo), _ptr(et), 1 if dat_f32 else 0, _ptr(lt),
                            _ptr(out["ylt"]), _ptr(out["occ_total"]), _ptr(out["gross_total"]),
                            _ptr(out["ylt_closed"]), _ptr(out["occ_max"]), _ptr(ev["gross"]), _ptr(ev["occ"]),
                            _ptr(ev["cum"]),
                            _ptr(ev["ceded"]), int(threads))
    if rc != 0:
        raise OracleError(rc)
    if per_event:
        out.update(ev)
    return out


def analyze_workload(w, **kw) -> dict:
    """``analyze`` on an object with the fields of ``synth.Workload``."""
    return analyze(w.event_ids, w.trial_offsets, w.catalog_size, w.elts, w.layer_terms,
                   elt_terms=w.elt_terms, **kw)


def rank(n: int, return_period: float) -> int:
    """k such that PML(RP) is the k-th largest of n year losses (see oracle_rank in the C source)."""
    return int(_load().oracle_rank(int(n), float(return_period)))


def risk(ylt, return_periods: Sequence[float]):
    """(pml, tvar, ranks, sorted_descending) of a YLT."""
    lib = _load()
    y = np.ascontiguousarray(ylt, dtype=np.float64)
    rp = np.ascontiguousarray(np.asarray(return_periods, dtype=np.float64))
    n_rp = rp.shape[0]
    pml = np.empty(n_rp, dtype=np.float64)
    tvar = np.empty(n_rp, dtype=np.float64)
    ranks = np.empty(n_rp, dtype=np.int64)
    srt = np.empty(y.shape[0], dtype=np.float64)
    rc = lib.oracle_risk(_ptr(y), y.shape[0], _ptr(rp), n_rp, _ptr(pml), _ptr(tvar), _ptr(ranks), _ptr(srt))
    if rc != 0:
        raise OracleError(rc)
    return pml, tvar, ranks, srt


def check_layer_terms(terms) -> int:
    t = np.ascontiguousarray(np.asarray(terms, dtype=np.float64).reshape(4))
    return int(_load().oracle_check_layer_terms(_ptr(t)))
