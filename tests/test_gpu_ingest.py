"""YET ingest: the catalog-binned copy against its definition, bit for bit.

Definition (the layout the tiled trial kernel reads): the catalog is cut into bins
of 2^14 events; region b holds, trial after trial, each trial's occurrences of bin-b
events in time order, each as its ID minus 2^14 b; boff[b][t] is where trial t's run
starts in region b, boff[b][n_trials] the region's length.  The expected copy below
is that definition computed with numpy's stable sort (integer work: bit-exact)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
BIN_SHIFT = 14


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _expected(ids: np.ndarray, offs: np.ndarray, catalog: int):
    n_trials = len(offs) - 1
    n_bins = (catalog + (1 << BIN_SHIFT) - 1) >> BIN_SHIFT
    trial = np.repeat(np.arange(n_trials, dtype=np.int64), np.diff(offs))
    b = ids.astype(np.int64) >> BIN_SHIFT
    order = np.argsort(b * (n_trials + 1) + trial, kind="stable")
    counts = np.bincount(b * n_trials + trial, minlength=n_bins * n_trials).reshape(n_bins, n_trials)
    boff = np.zeros((n_bins, n_trials + 1), np.int64)
    boff[:, 1:] = np.cumsum(counts, axis=1)
    local = (ids[order] & ((1 << BIN_SHIFT) - 1)).astype(np.uint16)
    per_bin = np.split(local, np.cumsum(boff[:, -1])[:-1])
    return n_bins, boff, per_bin


def _check_copy(A, y, ids, offs, catalog):
    got = A.ara_yet_binned(y)
    assert got is not None, "expected a binned copy"
    region, boff, ids16 = got
    n_bins, boff_x, per_bin = _expected(ids, offs, catalog)
    assert len(region) == n_bins + 1 and region[0] == 0
    assert np.all(region[:-1] % 8 == 0)
    assert np.array_equal(boff.astype(np.int64), boff_x)
    for b in range(n_bins):
        assert region[b] + boff_x[b, -1] <= region[b + 1]
        assert np.array_equal(ids16[region[b]:region[b] + boff_x[b, -1]], per_bin[b]), f"bin {b}"


@pytest.mark.parametrize("run_bytes", [4, 3])
@pytest.mark.parametrize("case", ["poisson", "ragged_long_trial", "one_bin_heavy", "many_trials"])
def test_binned_copy_matches_definition(ara_lib, gpu_ctx, case, run_bytes):
    import torch
    A = ara_lib
    rng = np.random.default_rng({"poisson": 11, "ragged_long_trial": 12, "one_bin_heavy": 13, "many_trials": 14}[case])
    catalog = 200_003   # 13 bins, the last one partial
    if case == "many_trials":
        # more 64-trial blocks per bin (17,188) than the block-total scan takes in one
        # round (16,384), and a trial count that is not a multiple of 4
        catalog = 30_001   # 2 bins
        lens = rng.poisson(20, size=1_100_003)
    elif case == "poisson":
        lens = rng.poisson(300, size=5000)
        lens[::97] = 0   # empty trials
    elif case == "ragged_long_trial":
        # a block of trials with more occurrences than one workgroup stages in LDS
        lens = rng.poisson(80, size=3000)
        lens[1234] = 90_000
        lens[2999] = 70_001
    else:
        lens = rng.poisson(500, size=800)
    offs = np.zeros(len(lens) + 1, np.int64)
    offs[1:] = np.cumsum(lens)
    ids = rng.integers(0, catalog, size=int(offs[-1]), dtype=np.int32)
    if case == "one_bin_heavy":   # most occurrences in bin 3, so runs of one bin are long
        heavy = rng.random(len(ids)) < 0.8
        ids[heavy] = (3 << BIN_SHIFT) + rng.integers(0, 1 << BIN_SHIFT, size=int(heavy.sum()), dtype=np.int32)
    _say(f"binned copy {case}, {run_bytes}-byte run starts: {len(lens)} trials, {len(ids)} occurrences")
    A.ara_set_option(gpu_ctx, A.ARA_OPT_YET_RUN_BYTES, run_bytes)
    try:
        y = A.ara_yet_create(gpu_ctx, torch.from_numpy(ids).cuda(), torch.from_numpy(offs).cuda(), catalog)
    finally:
        A.ara_set_option(gpu_ctx, A.ARA_OPT_YET_RUN_BYTES, 4)
    try:
        assert A.ara_yet_info(y)[2] == 2
        assert A.ara_yet_memory(y)[1] == run_bytes
        _check_copy(A, y, ids, offs, catalog)
    finally:
        A.ara_yet_release(y)


@pytest.mark.parametrize("run_bytes", [4, 3])
@pytest.mark.parametrize("shape", ["one_trial", "63_trials", "65_trials", "mostly_empty", "smallest_catalog"])
def test_binned_copy_edge_shapes(ara_lib, gpu_ctx, shape, run_bytes):
    """Trial counts either side of a 64-trial block, a single trial, trials that are
    nearly all empty, and the smallest catalog that gets a binned copy (one event more
    than a dense binary64 table in 160 KB of LDS): the copy against its definition."""
    import torch
    A = ara_lib
    rng = np.random.default_rng({"one_trial": 21, "63_trials": 22, "65_trials": 23, "mostly_empty": 24,
                                 "smallest_catalog": 25}[shape])
    catalog = 20_481 if shape == "smallest_catalog" else 50_000
    if shape == "one_trial":
        lens = np.array([777])
    elif shape == "63_trials":
        lens = rng.integers(100, 300, size=63)
    elif shape == "65_trials":
        lens = rng.integers(100, 300, size=65)
    elif shape == "mostly_empty":
        lens = np.zeros(640, np.int64)
        lens[[0, 63, 64, 639]] = [12_000, 1, 9_000, 16_000]
    else:
        lens = rng.integers(50, 150, size=200)
    offs = np.zeros(len(lens) + 1, np.int64)
    offs[1:] = np.cumsum(lens)
    ids = rng.integers(0, catalog, size=int(offs[-1]), dtype=np.int32)
    _say(f"binned copy edge shape {shape}, {run_bytes}-byte run starts: {len(lens)} trials, {len(ids)} occurrences")
    A.ara_set_option(gpu_ctx, A.ARA_OPT_YET_RUN_BYTES, run_bytes)
    try:
        y = A.ara_yet_create(gpu_ctx, torch.from_numpy(ids).cuda(), torch.from_numpy(offs).cuda(), catalog)
    finally:
        A.ara_set_option(gpu_ctx, A.ARA_OPT_YET_RUN_BYTES, 4)
    try:
        assert A.ara_yet_info(y)[2] == 2, "binned copy expected"
        assert A.ara_yet_memory(y)[1] == run_bytes
        _check_copy(A, y, ids, offs, catalog)
    finally:
        A.ara_yet_release(y)


def test_paper_scale_binned_copy(ara_lib, gpu_ctx):
    """The paper-scale YET (10^6 trials x 1000 events, 10^6-event catalog) with 3-byte
    run starts: at most 2.2 GB added to the caller's arrays, per-bin totals over every
    occurrence, and every run of 2,000 sampled trials."""
    import torch
    A = ara_lib
    w = synth.workload_paper_scale()
    _say("paper-scale binned copy, 3-byte run starts")
    A.ara_set_option(gpu_ctx, A.ARA_OPT_YET_RUN_BYTES, 3)
    try:
        y = A.ara_yet_create(gpu_ctx, torch.from_numpy(w.event_ids).cuda(), torch.from_numpy(w.trial_offsets).cuda(),
                             w.catalog_size)
    finally:
        A.ara_set_option(gpu_ctx, A.ARA_OPT_YET_RUN_BYTES, 4)
    try:
        assert A.ara_yet_info(y)[2] == 2
        extra, run_bytes = A.ara_yet_memory(y)
        assert run_bytes == 3, "every bin is shorter than 2^24: 3-byte run starts"
        assert extra <= 2.2e9, f"{extra} bytes added to the caller's arrays"
        region, boff, ids16 = A.ara_yet_binned(y)
        n_bins = len(region) - 1
        totals = np.bincount(w.event_ids >> BIN_SHIFT, minlength=n_bins)
        assert np.array_equal(boff[:, -1].astype(np.int64), totals)
        assert np.all(np.diff(boff.astype(np.int64), axis=1) >= 0)
        rng = np.random.default_rng(5)
        for t in np.sort(rng.choice(w.n_trials, size=2000, replace=False)):
            tid = w.event_ids[w.trial_offsets[t]:w.trial_offsets[t + 1]]
            tb = tid >> BIN_SHIFT
            for b in range(n_bins):
                run = ids16[region[b] + boff[b, t]:region[b] + boff[b, t + 1]]
                want = (tid[tb == b] & ((1 << BIN_SHIFT) - 1)).astype(np.uint16)
                assert np.array_equal(run, want), f"trial {t} bin {b}"
    finally:
        A.ara_yet_release(y)


@pytest.mark.parametrize("run_bytes", [4, 3])
@pytest.mark.parametrize("bad", [-1, 1_000_000, 2_000_000_000])
def test_binned_yet_rejects_bad_ids_and_offsets(ara_lib, gpu_ctx, bad, run_bytes):
    """A YET whose size takes the binned copy is checked in the copy's count pass:
    one ID outside [0, catalog) anywhere (first trial, last trial, middle) fails the
    creation with ARA_E_EVENT_ID_RANGE, bad offsets with ARA_E_BAD_OFFSETS, and the
    context works afterwards; with either run-start form."""
    A = ara_lib
    A.ara_set_option(gpu_ctx, A.ARA_OPT_YET_RUN_BYTES, run_bytes)
    try:
        _rejects_bad_ids_and_offsets(A, gpu_ctx, bad, run_bytes)
    finally:
        A.ara_set_option(gpu_ctx, A.ARA_OPT_YET_RUN_BYTES, 4)


def _rejects_bad_ids_and_offsets(A, gpu_ctx, bad, run_bytes):
    import torch
    rng = np.random.default_rng(abs(bad) % 97)
    n_trials, per = 3000, 600
    C = 1_000_000
    ids = rng.integers(0, C, size=n_trials * per).astype(np.int32)
    offs = np.arange(0, n_trials * per + 1, per, dtype=np.int64)
    for where in (0, ids.size - 1, ids.size // 2 + 13):
        print(f"[case] binned yet bad id {bad} at {where}", flush=True)
        bad_ids = ids.copy()
        bad_ids[where] = bad
        with pytest.raises(A.AraError) as e:
            A.ara_yet_create(gpu_ctx, torch.from_numpy(bad_ids).cuda(), torch.from_numpy(offs).cuda(), C)
        assert e.value.status == A.ARA_E_EVENT_ID_RANGE
    for name, o in [("decreasing", np.concatenate([offs[:10], offs[9:10] - 1, offs[11:]])),
                    ("last short", np.concatenate([offs[:-1], offs[-1:] - 1])),
                    ("first not 0", offs + np.int64(1)), ("negative", np.concatenate([offs[:5], [-7], offs[6:]]))]:
        print(f"[case] binned yet bad offsets: {name}", flush=True)
        with pytest.raises(A.AraError) as e:
            A.ara_yet_create(gpu_ctx, torch.from_numpy(ids).cuda(), torch.from_numpy(np.ascontiguousarray(o)).cuda(), C)
        assert e.value.status == A.ARA_E_BAD_OFFSETS, name
    yet = A.ara_yet_create(gpu_ctx, torch.from_numpy(ids).cuda(), torch.from_numpy(offs).cuda(), C)
    try:
        assert A.ara_yet_info(yet)[2] == 2, "this YET should keep a binned copy"
        assert A.ara_yet_memory(yet)[1] == run_bytes
    finally:
        A.ara_yet_release(yet)
