"""C-ABI checks that need no GPU: the library loads, exports every entry point
that include/ara.h declares, and its host-only logic behaves as documented."""
from __future__ import annotations

import ctypes
import math
import os
import re
from fractions import Fraction as Fr

import numpy as np
import pytest

from exact_ara import rank_exact

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ara.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ara_[a-z_]+)\s*\(", text)))


def test_header_declarations_exported(ara_lib):
    lib = ctypes.CDLL(ara_lib.LIB_PATH)
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(ara_lib.EXPORTED)


def test_status_strings(ara_lib):
    codes = [0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10, -11]
    strs = [ara_lib.ara_status_str(c) for c in codes]
    assert strs[0] == "ok"
    assert len(set(strs)) == len(strs)
    assert ara_lib.ara_status_str(-999) == "unknown status"
    assert ara_lib.ara_version() >= 100


def test_return_period_rank(ara_lib):
    r = ara_lib.ara_return_period_rank
    assert r(10_000, 10) == 1000 and r(10_000, 100) == 100 and r(10_000, 250) == 40
    assert r(49, 4.9) == 10 and r(6, 4) == 2 and r(5, 1) == 5 and r(5, math.inf) == 1
    rng = np.random.default_rng(1)
    for _ in range(3000):
        n = int(rng.integers(1, 10 ** 7))
        rp = float(rng.choice([1, 1.5, 2, 3, 7, 10, 20, 50, 100, 200, 250, 500, 1000, 1e4]))
        assert r(n, rp) == rank_exact(n, Fr(rp))
    for bad in [(0, 10.0), (5, 0.5), (5, float("nan")), (-1, 2.0)]:
        with pytest.raises(ara_lib.AraError):
            r(*bad)


def test_layer_terms_validation(ara_lib):
    ok = [(0, math.inf, 0, math.inf), (5e4, 1e6, 2e5, 5e6), (0, 0, 0, 0)]
    bad = [(-1, 1, 0, 1), (math.nan, 1, 0, 1), (math.inf, 1, 0, 1), (0, -1, 0, 1), (0, 1, 0, math.nan),
           (0, 1, math.inf, 1)]
    for t in ok:
        assert ara_lib.ara_check_layer_terms(t) == 0
    for t in bad:
        assert ara_lib.ara_check_layer_terms(t) == ara_lib.ARA_E_BAD_TERMS


def test_sort_workspace_size(ara_lib):
    prev = 0
    for n in [0, 1, 4095, 4096, 4097, 10 ** 6]:
        b = ara_lib.ara_sort_workspace_size(n)
        assert b >= 2 * 8 * n and b >= prev
        prev = b


def test_no_device_is_reported_cleanly(ara_lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    lib = ctypes.CDLL(ara_lib.LIB_PATH)
    out = ctypes.c_void_p()
    assert lib.ara_ctx_create(0, None, ctypes.byref(out)) == ara_lib.ARA_E_DEVICE
    assert out.value is None


def test_c_client_compiles_against_header(ara_lib, tmp_path):
    """A plain C11 program using only include/ara.h links against libara.so (gcc,
    -Wall -Werror) and resolves it through its rpath: the boundary needs no Python."""
    import subprocess
    import __graft_entry__ as g
    exe = g.build_c_client(str(tmp_path / "ara_c_client"))
    r = subprocess.run(["ldd", exe], capture_output=True, text=True, check=True)
    line = [ln for ln in r.stdout.splitlines() if "libara.so" in ln]
    assert line and "not found" not in line[0], r.stdout


def test_noalloc_scratch_holds_the_largest_sort(ara_lib):
    """The allocation-free risk call's device array holds the sort workspace of its
    largest YLT, and the binding's limits are the header's."""
    text = open(HEADER).read()
    max_n = re.search(r"#define ARA_NOALLOC_MAX_N \(1 << (\d+)\)", text)
    scratch = re.search(r"#define ARA_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", text)
    assert max_n and scratch
    assert ara_lib.ARA_NOALLOC_MAX_N == 1 << int(max_n.group(1))
    assert ara_lib.ARA_NOALLOC_SCRATCH_BYTES == int(scratch.group(1)) << int(scratch.group(2))
    assert ara_lib.ara_sort_workspace_size(ara_lib.ARA_NOALLOC_MAX_N) <= ara_lib.ARA_NOALLOC_SCRATCH_BYTES
