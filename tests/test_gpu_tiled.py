"""The tiled YLT kernel (catalog-binned YET copy, one catalog bin's occurrence-net
values in LDS at a time, a lane per trial) against the oracle and against the
LDS-bitmap kernel.

Bar: binary64 YLT within 1e-12 * max(|y|, P_k) of the oracle (the tiled kernel adds a
trial's occurrence-net losses grouped by catalog bin, another order of the same
non-negative terms); the same bits on every run; batched jobs equal plain launches
bit for bit."""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

INF = math.inf
TILES = 4          # ARA_PLACE_LDS_TILES
BITMAP = 1         # ARA_PLACE_LDS_BITMAP
GLOBAL_DENSE = 3   # ARA_PLACE_GLOBAL_DENSE


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def A(ara_lib):
    return ara_lib


@pytest.fixture(scope="module")
def S():
    from paper_1308_2066_amd import session
    return session


def _open(A, S, ctx, w, terms=None, binning=1, precision=0, run_bytes=4):
    A.ara_set_option(ctx, A.ARA_OPT_YET_BINNING, binning)
    A.ara_set_option(ctx, A.ARA_OPT_YET_RUN_BYTES, run_bytes)
    try:
        return S.open_analysis(ctx, w.event_ids, w.trial_offsets, w.catalog_size, w.elts,
                               terms if terms is not None else w.layer_terms, w.elt_terms, precision)
    finally:
        A.ara_set_option(ctx, A.ARA_OPT_YET_BINNING, 1)
        A.ara_set_option(ctx, A.ARA_OPT_YET_RUN_BYTES, 4)


def _run(A, ctx, an, placement, t0=0, t1=None):
    import torch
    t1 = an_trials(A, an) if t1 is None else t1
    A.ara_set_option(ctx, A.ARA_OPT_PLACEMENT, placement)
    try:
        y = torch.full((max(t1 - t0, 1),), math.nan, dtype=torch.float64, device="cuda")
        if t1 > t0:
            A.ara_analyze(ctx, an.yet, an.layer, t0, t1, y)
        A.ara_sync(ctx)
        return y[: t1 - t0].cpu().numpy()
    finally:
        A.ara_set_option(ctx, A.ARA_OPT_PLACEMENT, 0)


def an_trials(A, an):
    return A.ara_yet_info(an.yet)[1]


def _close(got, ref, what=""):
    y, P = ref["ylt"], ref["occ_total"]
    tol = 1e-12 * np.maximum(np.abs(y), P)
    bad = np.nonzero(~(np.abs(got - y) <= tol))[0]
    assert bad.size == 0, f"{what}: {bad.size} trials off; first {bad[:5]} got {got[bad[:5]]} want {y[bad[:5]]}"


def _workload(rng, lengths, catalog, n_elts=4, nnz=None, mu=10.0, sigma=2.0, terms=(5e4, 1e6, 2e5, INF),
              id_sampler=None):
    lengths = np.asarray(lengths, np.int64)
    offs = np.zeros(len(lengths) + 1, np.int64)
    offs[1:] = np.cumsum(lengths)
    n = int(offs[-1])
    ids = (id_sampler(n) if id_sampler else rng.integers(0, catalog, size=n)).astype(np.int32)
    nnz = nnz or catalog // 3
    elts = [synth.elt_sparse(rng, nnz, catalog, mu, sigma) for _ in range(n_elts)]
    return synth.Workload("tiled", ids, offs, catalog, elts, terms, None, (10.0,), 0)


def _occ_max(A, ctx, an, placement, t0, t1):
    import torch
    A.ara_set_option(ctx, A.ARA_OPT_PLACEMENT, placement)
    try:
        out = torch.full((max(t1 - t0, 1),), math.nan, dtype=torch.float64, device="cuda")
        if t1 > t0:
            A.ara_analyze_occ_max(ctx, an.yet, an.layer, t0, t1, out)
        A.ara_sync(ctx)
        return out[: t1 - t0].cpu().numpy()
    finally:
        A.ara_set_option(ctx, A.ARA_OPT_PLACEMENT, 0)


def _check_occ_max(A, ctx, an, ref, what, sub_ranges=(), f32=False):
    """Occurrence maxima through the tiled kernel (a maximum of table values): with
    binary64 tables the oracle's bits, whole and on sub-ranges.  With binary32 tables
    the combined table is rounded to binary32 before the occurrence terms (the oracle
    rounds each ELT's table only): the bits of the LDS-filter kernel, which reads the
    same tables, and the oracle's values within that rounding."""
    n = an_trials(A, an)
    got = _occ_max(A, ctx, an, TILES, 0, n)
    want = _occ_max(A, ctx, an, BITMAP, 0, n) if f32 else ref["occ_max"]
    assert got.tobytes() == want.tobytes(), f"{what}: occurrence maxima differ"
    if f32:
        bound = 2.0 ** -23 * 1.0001 * ref["gross_total"]
        assert np.all(np.abs(got - ref["occ_max"]) <= bound), what
    assert _occ_max(A, ctx, an, 0, 0, n).tobytes() == got.tobytes(), "auto placement must pick the tiled kernel"
    for t0, t1 in sub_ranges:
        assert _occ_max(A, ctx, an, 0, t0, t1).tobytes() == want[t0:t1].tobytes(), (what, t0, t1)


def _tiles_vs_oracle_and_bitmap(A, S, ctx, w, what, sub_ranges=()):
    an = _open(A, S, ctx, w)
    try:
        assert A.ara_yet_info(an.yet)[2] == 2, "binned copy expected"
        got = _run(A, ctx, an, 0)
        assert A.ara_layer_stats(ctx, an.layer)[1] in (BITMAP, TILES)
        again = _run(A, ctx, an, TILES)
        assert again.tobytes() == got.tobytes(), "auto placement must pick the tiled kernel here"
        ref = oracle.analyze_workload(w, threads=oracle.max_threads())
        _close(got, ref, what)
        _close(_run(A, ctx, an, BITMAP), ref, what + " (bitmap)")
        for t0, t1 in sub_ranges:
            sub = _run(A, ctx, an, 0, t0, t1)
            _close(sub, {k: v[t0:t1] for k, v in ref.items()}, f"{what} [{t0}, {t1})")
        _check_occ_max(A, ctx, an, ref, what, sub_ranges)
        return got
    finally:
        an.release()


def test_paper_shape_many_tiles(A, S, gpu_ctx):
    """1M-event catalog, 16 ELTs: 62 bins staged in turn; unsaturated aggregate terms
    so every YLT value is checked."""
    w = synth.workload_paper_scale(n_trials=8_000)
    w = w.with_terms((1e5, 5e6, 1.5e8, INF))
    _say("tiled paper shape 8k x 1000")
    _tiles_vs_oracle_and_bitmap(A, S, gpu_ctx, w, "paper shape", sub_ranges=[(0, 1), (17, 4113), (7999, 8000)])


def test_dense_layer_splits_bins(A, S, gpu_ctx):
    """Every event flagged (no zero in any bin's values), trials of 0 to 4099
    occurrences: runs longer than the prefetched 32 IDs read the rest when reached,
    odd-starting runs drop the previous run's last ID."""
    rng = np.random.default_rng(301)
    C = 100_003                                  # not a multiple of the bin size
    ids_all = np.arange(C, dtype=np.int32)
    elts = [(ids_all, rng.lognormal(8.0, 1.0, size=C))]
    lengths = list(rng.integers(200, 1500, size=600)) + [0, 1, 4099, 2, 0]
    w = _workload(rng, lengths, C)
    w = synth.Workload("dense", w.event_ids, w.trial_offsets, C, elts, (0.0, INF, 0.0, INF), None, (2.0,), 0)
    _say("tiled dense layer")
    _tiles_vs_oracle_and_bitmap(A, S, gpu_ctx, w, "dense", sub_ranges=[(3, 299), (600, 605)])


def test_ragged_and_empty_runs(A, S, gpu_ctx):
    """Ragged trial lengths, empty trials, long runs of trials without occurrences in
    a bin (IDs concentrated in a few bins), a catalog that ends inside a bin."""
    rng = np.random.default_rng(302)
    C = 70_001
    lengths = [0] * 70 + list(rng.integers(0, 400, size=500)) + [0] * 200 + [5000, 1, 1, 3000] + [0] * 64 + [7]

    def concentrated(n):
        # most occurrences in bins 0 and 2, a few in the partial last bin
        pick = rng.random(n)
        out = rng.integers(0, 32768, size=n)
        out = np.where(pick < 0.5, out, rng.integers(65536, 70_001, size=n))
        return out

    w = _workload(rng, lengths, C, n_elts=3, nnz=20_000, id_sampler=concentrated)
    _say("tiled ragged runs")
    _tiles_vs_oracle_and_bitmap(A, S, gpu_ctx, w, "ragged", sub_ranges=[(0, 70), (69, 71), (560, 839)])


def test_single_tile_and_determinism(A, S, gpu_ctx):
    """A 60,000-event catalog (four bins); runs repeat bit for bit; without the binned
    copy the bitmap kernel gives the same values within the bound."""
    rng = np.random.default_rng(303)
    w = _workload(rng, rng.integers(500, 1500, size=3000), 60_000, nnz=3_000)
    _say("tiled single tile")
    got = _tiles_vs_oracle_and_bitmap(A, S, gpu_ctx, w, "one tile")
    an = _open(A, S, gpu_ctx, w)
    try:
        for _ in range(3):
            assert _run(A, gpu_ctx, an, 0).tobytes() == got.tobytes()
    finally:
        an.release()
    an = _open(A, S, gpu_ctx, w, binning=0)
    try:
        assert A.ara_yet_info(an.yet)[2] == 3
        with pytest.raises(A.AraError) as e:
            _run(A, gpu_ctx, an, TILES)
        assert e.value.status == A.ARA_E_UNSUPPORTED
        _close(_run(A, gpu_ctx, an, 0), oracle.analyze_workload(w, threads=oracle.max_threads()), "no binned copy")
    finally:
        an.release()


def test_batch_with_tiled_jobs_equals_plain(A, S, gpu_ctx):
    """Tiled jobs inside a batch (beside dense-table jobs) give the plain launch's bits."""
    import torch
    rng = np.random.default_rng(304)
    w1 = _workload(rng, rng.integers(300, 1200, size=2000), 200_000)
    w2 = synth.workload_plain_small()
    a1, a2 = _open(A, S, gpu_ctx, w1), _open(A, S, gpu_ctx, w2)
    try:
        specs = [(a1, 0, w1.n_trials), (a1, 11, 1500), (a2, 0, w2.n_trials)]
        want = [_run(A, gpu_ctx, an, 0, t0, t1) for an, t0, t1 in specs]
        outs = [torch.full((t1 - t0,), math.nan, dtype=torch.float64, device="cuda") for _, t0, t1 in specs]
        b = A.ara_batch_create(gpu_ctx, [(an.yet, an.layer, t0, t1, o) for (an, t0, t1), o in zip(specs, outs)])
        try:
            for rep in range(3):
                _say(f"tiled batch run {rep}")
                for o in outs:
                    o.fill_(math.nan)
                A.ara_batch_run(b)
                A.ara_sync(gpu_ctx)
                for k, o in enumerate(outs):
                    assert o.cpu().numpy().tobytes() == want[k].tobytes(), (rep, k)
        finally:
            A.ara_batch_release(b)
    finally:
        a1.release()
        a2.release()


def test_several_passes_per_workgroup(A, S, gpu_ctx):
    """1,200,000 short trials: each persistent workgroup owns more trials than one pass
    (4032) holds, so the per-trial sums are reset and the bins restaged per pass;
    a 70,000-event catalog in five bins (the last cut short), binary32 tables (too
    large for the dense LDS table) and non-identity ELT terms."""
    rng = np.random.default_rng(305)
    C = 70_000
    n = 1_200_000
    lengths = rng.integers(40, 61, size=n)
    w = _workload(rng, lengths, C, n_elts=3, nnz=12_000)
    w = synth.Workload("passes", w.event_ids, w.trial_offsets, C, w.elts, w.layer_terms,
                       [(1.1, 100.0, 2e6), (1.0, 0.0, INF), (0.9, 0.0, INF)], (10.0,), 0)
    _say("tiled several passes")
    an = _open(A, S, gpu_ctx, w, precision=A.ARA_F32)
    try:
        assert A.ara_yet_info(an.yet)[2] == 2
        got = _run(A, gpu_ctx, an, 0)
        assert A.ara_layer_stats(gpu_ctx, an.layer)[1] in (BITMAP, TILES)
        assert _run(A, gpu_ctx, an, TILES).tobytes() == got.tobytes(), "auto placement must pick the tiled kernel"
        ref = oracle.analyze_workload(w, threads=oracle.max_threads(), dat_f32=True)
        tol = 2.0 ** -23 * 1.0001 * ref["gross_total"] + 1e-12 * np.maximum(np.abs(ref["ylt"]), ref["occ_total"])
        bad = np.nonzero(~(np.abs(got - ref["ylt"]) <= tol))[0]
        assert bad.size == 0, (bad[:5], got[bad[:5]], ref["ylt"][bad[:5]])
        assert _run(A, gpu_ctx, an, 0).tobytes() == got.tobytes()
        sub = _run(A, gpu_ctx, an, 0, 123_457, 1_199_999)
        assert sub.tobytes() == _run(A, gpu_ctx, an, 0, 123_457, 1_199_999).tobytes()
        bad = np.nonzero(~(np.abs(sub - ref["ylt"][123_457:1_199_999]) <= tol[123_457:1_199_999]))[0]
        assert bad.size == 0
        _check_occ_max(A, gpu_ctx, an, ref, "several passes", [(123_457, 1_199_999)], f32=True)
    finally:
        an.release()


def test_large_catalog_many_bins_and_rank_chunks(A, S, gpu_ctx):
    """A 3,000,003-event catalog: 184 bins (a last bin cut short) and 23,438 filter
    blocks, which the rank kernel takes in three chunks of 8192; the flagged count
    equals the one computed here from the ELTs, and the YLT matches the oracle and the
    global dense-table kernel.  2000 occurrences per trial, so that the per-(bin,
    trial) offsets stay within a quarter of the binned IDs and the copy is kept."""
    w = synth.workload_paper_scale(n_trials=20_000, per_trial=2000, catalog=3_000_003, n_elts=8, nnz=200_000)
    w = w.with_terms((1e5, 5e6, 1.5e8, INF))
    _say("tiled large catalog 3M, 20k x 2000")
    an = _open(A, S, gpu_ctx, w)
    try:
        assert A.ara_yet_info(an.yet)[2] == 2, "binned copy expected"
        got = _run(A, gpu_ctx, an, 0)
        assert _run(A, gpu_ctx, an, TILES).tobytes() == got.tobytes(), "auto placement must pick the tiled kernel"
        ref = oracle.analyze_workload(w, threads=oracle.max_threads())
        _close(got, ref, "large catalog")
        _close(_run(A, gpu_ctx, an, GLOBAL_DENSE), ref, "large catalog (global dense table)")
        comb = np.zeros(w.catalog_size)
        for ids, loss in w.elts:   # layer order, binary64, from +0.0: the combined table
            comb[ids] += loss
        assert A.ara_layer_stats(gpu_ctx, an.layer)[0] == int(np.count_nonzero(comb > w.layer_terms[0]))
        _check_occ_max(A, gpu_ctx, an, ref, "large catalog", [(5, 19_999)])
        # per-occurrence outputs: the catalog's nonzero bits (366 KB) exceed LDS, so the
        # kernel reads the combined table for every occurrence; gross and occurrence-net
        # losses are table values (bit-exact), the cumulative sums within the summation bound
        import torch
        t0, t1 = 100, 1100
        e0, e1 = int(w.trial_offsets[t0]), int(w.trial_offsets[t1])
        ev = {k: torch.full((e1 - e0,), math.nan, dtype=torch.float64, device="cuda")
              for k in ("gross", "occ", "cum", "ceded")}
        ylt = torch.full((t1 - t0,), math.nan, dtype=torch.float64, device="cuda")
        A.ara_analyze_events(gpu_ctx, an.yet, an.layer, t0, t1, ylt, ev["gross"], ev["occ"], ev["cum"], ev["ceded"])
        A.ara_sync(gpu_ctx)
        ref_ev = oracle.analyze_workload(w, t_begin=t0, t_end=t1, per_event=True, threads=oracle.max_threads())
        assert np.array_equal(ev["gross"].cpu().numpy(), ref_ev["gross"])
        assert np.array_equal(ev["occ"].cpu().numpy(), ref_ev["occ"])
        cum = ev["cum"].cpu().numpy()
        assert np.all(np.abs(cum - ref_ev["cum"]) <= 1e-12 * np.maximum(np.abs(ref_ev["cum"]), 1.0))
        _close(ylt.cpu().numpy(), ref_ev, "large catalog events")
    finally:
        an.release()


def test_largest_binned_catalog(A, S, gpu_ctx):
    """A 2^23-event catalog: 512 bins, the most a binned copy holds (the scatter's
    9-bit bin numbers, every lane of the region kernel); the YLT and the occurrence
    maxima of the tiled kernel match the oracle.  One event more (513 bins) keeps no
    binned copy, and the analysis still matches the oracle."""
    rng = np.random.default_rng(306)
    C = 1 << 23
    lengths = rng.integers(3500, 5500, size=1500)
    w = _workload(rng, lengths, C, n_elts=2, nnz=200_000)
    w = w.with_terms((5e4, 1e6, 2e8, INF))
    _say("tiled largest binned catalog 2^23")
    an = _open(A, S, gpu_ctx, w)
    try:
        assert A.ara_yet_info(an.yet)[2] == 2, "binned copy expected"
        assert A.ara_yet_binned_count(an.yet) == 512
        got = _run(A, gpu_ctx, an, 0)
        assert _run(A, gpu_ctx, an, TILES).tobytes() == got.tobytes(), "auto placement must pick the tiled kernel"
        ref = oracle.analyze_workload(w, threads=oracle.max_threads())
        _close(got, ref, "2^23 catalog")
        _check_occ_max(A, gpu_ctx, an, ref, "2^23 catalog", [(1, 1499)])
    finally:
        an.release()
    w2 = synth.Workload("tiled", w.event_ids, w.trial_offsets, C + 1, w.elts, w.layer_terms, None, (10.0,), 0)
    _say("catalog 2^23 + 1: no binned copy")
    an = _open(A, S, gpu_ctx, w2)
    try:
        assert A.ara_yet_info(an.yet)[2] != 2
        _close(_run(A, gpu_ctx, an, 0), oracle.analyze_workload(w2, threads=oracle.max_threads()), "2^23 + 1 catalog")
    finally:
        an.release()


def test_long_bin_keeps_four_byte_run_starts(A, S, gpu_ctx):
    """Asked for 3-byte run starts, a YET with a catalog bin of more than 2^24
    occurrences gets 4-byte ones (the 3-byte build flags the bin and is redone), the
    readout still gives the definition's bin lengths, and the tiled kernel on that
    form matches the oracle (YLT and maxima)."""
    rng = np.random.default_rng(307)
    C = 100_000   # 7 bins
    lengths = rng.integers(800, 1000, size=20_000)

    def mostly_bin0(n):   # 97% of the occurrences in bin 0: about 17.5M > 2^24
        x = rng.integers(0, C, size=n)
        heavy = rng.random(n) < 0.97
        x[heavy] = rng.integers(0, 1 << 14, size=int(heavy.sum()))
        return x

    w = _workload(rng, lengths, C, n_elts=2, id_sampler=mostly_bin0)
    w = w.with_terms((5e4, 1e6, 2e8, INF))
    _say(f"tiled long bin: {len(w.event_ids)} occurrences")
    an = _open(A, S, gpu_ctx, w, run_bytes=3)
    try:
        assert A.ara_yet_info(an.yet)[2] == 2, "binned copy expected"
        assert A.ara_yet_memory(an.yet)[1] == 4
        region, boff, _ = A.ara_yet_binned(an.yet)
        totals = np.bincount(w.event_ids >> 14, minlength=len(region) - 1)
        assert totals[0] >= 1 << 24
        assert np.array_equal(boff[:, -1].astype(np.int64), totals)
        got = _run(A, gpu_ctx, an, 0)
        assert _run(A, gpu_ctx, an, TILES).tobytes() == got.tobytes()
        ref = oracle.analyze_workload(w, threads=oracle.max_threads())
        _close(got, ref, "long bin")
        _check_occ_max(A, gpu_ctx, an, ref, "long bin", [(0, 20_000), (7, 9_001)])
    finally:
        an.release()


def test_three_byte_run_starts_same_bits(A, S, gpu_ctx):
    """The same YET with 3-byte run starts (ARA_OPT_YET_RUN_BYTES = 3): less memory, the
    same binned copy on readout, and the bits of the 4-byte form for the YLT and the
    occurrence maxima -- on the paper's shape and on ragged runs, whole, on sub-ranges,
    and in one batch holding both forms."""
    import torch
    rng = np.random.default_rng(308)
    paper = synth.workload_paper_scale(n_trials=6_000).with_terms((1e5, 5e6, 1.5e8, INF))
    lengths = [0] * 40 + list(rng.integers(0, 900, size=700)) + [4000, 1, 0, 2500] + [0] * 70 + [3]
    ragged = _workload(rng, lengths, 150_001, n_elts=3, nnz=40_000)
    for w, what in ((paper, "paper shape"), (ragged, "ragged")):
        _say(f"3-byte run starts: {what}")
        a4, a3 = _open(A, S, gpu_ctx, w), _open(A, S, gpu_ctx, w, run_bytes=3)
        try:
            (m4, r4), (m3, r3) = A.ara_yet_memory(a4.yet), A.ara_yet_memory(a3.yet)
            assert (r4, r3) == (4, 3) and m3 < m4, (m4, r4, m3, r3)
            (g4, b4, i4), (g3, b3, i3) = A.ara_yet_binned(a4.yet), A.ara_yet_binned(a3.yet)
            assert np.array_equal(g4, g3) and np.array_equal(b4, b3), what
            for b in range(len(g4) - 1):   # the runs (regions are padded to 8 IDs with unused slots)
                assert np.array_equal(i4[g4[b]:g4[b] + b4[b, -1]], i3[g3[b]:g3[b] + b3[b, -1]]), (what, b)
            n = w.n_trials
            y4 = _run(A, gpu_ctx, a4, 0)
            assert _run(A, gpu_ctx, a3, 0).tobytes() == y4.tobytes(), what
            assert _run(A, gpu_ctx, a3, TILES).tobytes() == y4.tobytes(), what
            for t0, t1 in ((0, 1), (13, n // 2 + 7), (n - 1, n)):
                assert _run(A, gpu_ctx, a3, 0, t0, t1).tobytes() == y4[t0:t1].tobytes(), (what, t0, t1)
            assert _occ_max(A, gpu_ctx, a3, TILES, 0, n).tobytes() == _occ_max(A, gpu_ctx, a4, TILES, 0, n).tobytes()
            specs = [(a4, 0, n), (a3, 0, n), (a3, 5, n - 3)]
            outs = [torch.full((t1 - t0,), math.nan, dtype=torch.float64, device="cuda") for _, t0, t1 in specs]
            b = A.ara_batch_create(gpu_ctx, [(an.yet, an.layer, t0, t1, o) for (an, t0, t1), o in zip(specs, outs)])
            try:
                A.ara_batch_run(b)
                A.ara_sync(gpu_ctx)
                for (an, t0, t1), o in zip(specs, outs):
                    assert o.cpu().numpy().tobytes() == y4[t0:t1].tobytes(), (what, t0, t1)
            finally:
                A.ara_batch_release(b)
        finally:
            a4.release()
            a3.release()
