"""Seeded synthetic inputs for aggregate risk analysis.

This module only draws input data: Year Event Tables (trials of time-ordered
event IDs), sparse Event Loss Tables and layer terms (Section II-A of the
paper, "Inputs"; layer terms per Table I).  It holds none of the analysis
arithmetic and imports neither the oracle nor the HIP binding, so both sides
can consume exactly the same arrays.

Workload shapes follow the paper: trials of hundreds to ~1500 events, ELTs of
10K-30K event losses, 3-30 ELTs per layer, a catalog of up to a few million
events, and the headline run of 1M trials x 1000 events (Section III-C).  The
concrete recipes (counts, distributions, terms) are the ones named below; the
paper's industrial inputs are not public, so these stand in for them.

Layout produced (the boundary's input layout):
  * ``event_ids``: int32, all trials concatenated, each trial in time order.
  * ``trial_offsets``: int64 CSR offsets, ``len = n_trials + 1``,
    ``offsets[0] == 0`` and ``offsets[-1] == len(event_ids)``.
  * an ELT: ``(ids int32, losses float64)`` with distinct ids in [0, catalog).
  * layer terms: ``(occ_retention, occ_limit, agg_retention, agg_limit)``.
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import List, Optional, Sequence, Tuple

import numpy as np

SEED_BASE = 13082066

__all__ = [
    "SEED_BASE", "Workload", "Portfolio", "portfolio_batched", "serving_yet", "serving_requests", "uneven_analyses",
    "uniform_ids", "yet_poisson", "yet_fixed", "yet_fixed_block",
    "elt_sparse", "workload_plain_small", "workload_paper_scale", "random_tiny",
    "loguniform_terms",
]


@dataclasses.dataclass
class Workload:
    """One analysis: a YET, the ELTs of one layer and the layer's terms."""
    name: str
    event_ids: np.ndarray            # int32 [n_events]
    trial_offsets: np.ndarray        # int64 [n_trials + 1]
    catalog_size: int
    elts: List[Tuple[np.ndarray, np.ndarray]]   # [(ids int32, losses f64)]
    layer_terms: Tuple[float, float, float, float]
    elt_terms: Optional[List[Tuple[float, float, float]]] = None  # (fx, retention, limit) per ELT
    return_periods: Tuple[float, ...] = (10.0, 100.0, 250.0)
    seed: int = SEED_BASE

    @property
    def n_trials(self) -> int:
        return int(self.trial_offsets.shape[0] - 1)

    @property
    def n_events(self) -> int:
        return int(self.event_ids.shape[0])

    def with_terms(self, layer_terms, name_suffix="") -> "Workload":
        return dataclasses.replace(self, layer_terms=tuple(float(x) for x in layer_terms),
                                   name=self.name + name_suffix)


def _threads() -> int:
    n = os.cpu_count() or 1
    return max(1, min(16, n))


def uniform_ids(rng: np.random.Generator, n: int, catalog: int) -> np.ndarray:
    """n event IDs drawn exactly uniformly from [0, catalog) as int32.

    Multiply-shift of 32-bit raw draws with rejection of the biased low region
    (Lemire, "Fast random integer generation in an interval", 2019), vectorised.
    """
    if not (1 <= catalog <= 2 ** 31 - 1):
        raise ValueError("catalog must be in [1, 2^31)")
    out = np.empty(n, dtype=np.int32)
    thresh = (2 ** 32 - catalog) % catalog   # == 2^32 mod catalog
    c64 = np.uint64(catalog)
    pos = np.arange(n, dtype=np.int64)
    while pos.size:
        raw = rng.bit_generator.random_raw((pos.size + 1) // 2).view(np.uint32)[: pos.size]
        m = raw.astype(np.uint64) * c64
        ok = (m & np.uint64(0xFFFFFFFF)) >= np.uint64(thresh)
        out[pos[ok]] = (m[ok] >> np.uint64(32)).astype(np.int32)
        pos = pos[~ok]
    return out


def yet_poisson(rng: np.random.Generator, n_trials: int, mean: float, catalog: int):
    """YET whose trial lengths are Poisson(mean), IDs uniform over the catalog, and
    each trial ordered by ascending uniform(0,1) timestamps (Section II-A, item 1).

    Equal timestamps (probability ~0) keep draw order (stable sort)."""
    counts = rng.poisson(mean, size=n_trials).astype(np.int64)
    offsets = np.zeros(n_trials + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    n = int(offsets[-1])
    ids = uniform_ids(rng, n, catalog)
    ts = rng.random(n)
    trial_of = np.repeat(np.arange(n_trials, dtype=np.int64), counts)
    order = np.lexsort((ts, trial_of))      # by trial, then by timestamp
    return ids[order], offsets


def yet_fixed_block(seed: int, block: int, trials_in_block: int, per_trial: int, catalog: int) -> np.ndarray:
    """IDs of one block of a fixed-length YET; block b has its own stream, so any
    block can be regenerated alone."""
    rng = np.random.default_rng([seed, 0x5945, block])
    return uniform_ids(rng, trials_in_block * per_trial, catalog)


def yet_fixed(seed: int, n_trials: int, per_trial: int, catalog: int, trial_block: int = 16384,
              out: Optional[np.ndarray] = None):
    """YET with exactly ``per_trial`` events per trial, IDs iid uniform.

    Timestamps are not drawn: for iid uniform IDs, ordering a trial by iid
    uniform timestamps leaves the distribution of the ID sequence unchanged, so
    the draw order is taken as the time order.
    """
    n = n_trials * per_trial
    ids = np.empty(n, dtype=np.int32) if out is None else out
    nblk = (n_trials + trial_block - 1) // trial_block

    def work(b):
        t0 = b * trial_block
        nt = min(trial_block, n_trials - t0)
        ids[t0 * per_trial:(t0 + nt) * per_trial] = yet_fixed_block(seed, b, nt, per_trial, catalog)

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(work, range(nblk)))
    offsets = np.arange(n_trials + 1, dtype=np.int64) * per_trial
    return ids, offsets


def elt_sparse(rng: np.random.Generator, n_nonzero: int, catalog: int, mu: float, sigma: float):
    """One ELT: ``n_nonzero`` distinct event IDs (sampled without replacement)
    with lognormal(mu, sigma) losses; every other catalog event has loss 0."""
    ids = np.sort(rng.choice(catalog, size=n_nonzero, replace=False)).astype(np.int32)
    losses = rng.lognormal(mu, sigma, size=n_nonzero).astype(np.float64)
    return ids, losses


def loguniform_terms(rng: np.random.Generator, lo: float = 1e4, hi: float = 1e8):
    """Occurrence and aggregate (retention, limit) pairs: two log-uniform draws
    per pair, retention = the smaller, limit = the larger."""
    v = np.exp(rng.uniform(math.log(lo), math.log(hi), size=4))
    occ = sorted(v[:2])
    agg = sorted(v[2:])
    return (float(occ[0]), float(occ[1]), float(agg[0]), float(agg[1]))


def workload_plain_small(seed: int = SEED_BASE + 0) -> Workload:
    """Plain FP64 analysis: 10,000 trials, Poisson(100) events per trial over a
    10,000-event catalog, one layer of 4 ELTs x 2,000 distinct events with
    lognormal(10, 2) losses; occurrence R/L 5e4/1e6, aggregate R/L 2e5/5e6;
    PML at return periods 10/100/250, TVaR at 1% (return period 100)."""
    rng = np.random.default_rng(seed)
    C = 10_000
    ids, offs = yet_poisson(rng, 10_000, 100.0, C)
    elts = [elt_sparse(rng, 2_000, C, 10.0, 2.0) for _ in range(4)]
    return Workload("plain-10k-trials-poisson100-4elt", ids, offs, C, elts,
                    (5e4, 1e6, 2e5, 5e6), None, (10.0, 100.0, 250.0), seed)


def workload_paper_scale(seed: int = SEED_BASE + 1, n_trials: int = 1_000_000, per_trial: int = 1000,
                         catalog: int = 1_000_000, n_elts: int = 16, nnz: int = 20_000) -> Workload:
    """Paper-scale analysis: 1M trials x exactly 1000 events, IDs uniform over a
    1M-event catalog, one layer of 16 ELTs x 20,000 lognormal(11, 2.5) losses;
    occurrence R/L 1e5/5e6, aggregate R/L 1e6/5e7.  ``n_trials`` may be reduced
    for parity runs of the same shape."""
    rng = np.random.default_rng([seed, 0xE17])
    elts = [elt_sparse(rng, nnz, catalog, 11.0, 2.5) for _ in range(n_elts)]
    ids, offs = yet_fixed(seed, n_trials, per_trial, catalog)
    return Workload(f"paper-scale-{n_trials}x{per_trial}-{n_elts}elt-cat{catalog}", ids, offs, catalog, elts,
                    (1e5, 5e6, 1e6, 5e7), None, (10.0, 100.0, 250.0), seed)


@dataclasses.dataclass
class Portfolio:
    """One YET analysed against many layers drawn from a shared pool of ELTs."""
    name: str
    event_ids: np.ndarray
    trial_offsets: np.ndarray
    catalog_size: int
    pool: List[Tuple[np.ndarray, np.ndarray]]
    layers: List[Tuple[List[int], Tuple[float, float, float, float]]]   # (pool indices, layer terms)
    return_periods: Tuple[float, ...]
    seed: int

    @property
    def n_trials(self) -> int:
        return int(self.trial_offsets.shape[0] - 1)

    @property
    def n_events(self) -> int:
        return int(self.event_ids.shape[0])

    def layer_workload(self, j: int) -> Workload:
        idx, terms = self.layers[j]
        return Workload(f"{self.name}-layer{j}", self.event_ids, self.trial_offsets, self.catalog_size,
                        [self.pool[i] for i in idx], terms, None, self.return_periods, self.seed)


def portfolio_batched(seed: int = SEED_BASE + 2, n_layers: int = 64, pool_size: int = 256,
                      max_elts: int = 32) -> Portfolio:
    """Batched portfolio: the plain small YET (10,000 trials, Poisson(100) events,
    10,000-event catalog) shared by n_layers layers; each layer takes U{1..max_elts}
    distinct ELTs of a pool of pool_size ELTs that are dense over the catalog (every
    event has a loss) with lognormal(11, 2.5) losses; each layer's occurrence and
    aggregate (retention, limit) pairs are log-uniform on [1e4, 1e8], the smaller
    value being the retention."""
    base = workload_plain_small()
    rng = np.random.default_rng([seed, 0xC3])
    C = base.catalog_size
    all_ids = np.arange(C, dtype=np.int32)
    pool = [(all_ids, rng.lognormal(11.0, 2.5, size=C)) for _ in range(pool_size)]
    layers = []
    for _ in range(n_layers):
        k = int(rng.integers(1, max_elts + 1))
        idx = sorted(int(i) for i in rng.choice(pool_size, size=k, replace=False))
        layers.append((idx, loguniform_terms(rng)))
    return Portfolio(f"portfolio-{n_layers}x-pool{pool_size}", base.event_ids, base.trial_offsets, C, pool, layers,
                     base.return_periods, seed)


def _ids_blocks(key, n: int, catalog: int, block: int = 1 << 22) -> np.ndarray:
    """n uniform IDs over the catalog, drawn in blocks of `block` with independent
    streams default_rng(key + [block index]) on a thread pool."""
    ids = np.empty(n, dtype=np.int32)

    def work(b):
        lo = b * block
        hi = min(n, lo + block)
        ids[lo:hi] = uniform_ids(np.random.default_rng(list(key) + [b]), hi - lo, catalog)

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(work, range((n + block - 1) // block)))
    return ids


def serving_yet(seed: int = SEED_BASE + 4, n_trials: int = 1_000_000):
    """Resident YET of the serving workload: the plain small statistics (Poisson(100)
    events per trial, IDs uniform over a 10,000-event catalog) at 10^6 trials.  With
    iid uniform IDs, ordering a trial by iid uniform timestamps does not change the
    distribution of its ID sequence, so the draw order is taken as the time order."""
    rng = np.random.default_rng(seed)
    counts = rng.poisson(100.0, size=n_trials).astype(np.int64)
    offs = np.zeros(n_trials + 1, dtype=np.int64)
    np.cumsum(counts, out=offs[1:])
    return _ids_blocks([seed, 0x5E], int(offs[-1]), 10_000), offs, 10_000


def serving_requests(n: int, n_trials: int, pool_size: int = 256, rate: float = 50.0, seed: int = SEED_BASE + 4,
                     min_trials: int = 100_000, max_trials: int = 1_000_000):
    """Pricing requests: Poisson arrivals at `rate` per second (times in seconds from
    0); each takes U{1..32} distinct pool ELTs, log-uniform occurrence and aggregate
    terms, and a contiguous range of U[min_trials, max_trials] trials with a uniform
    start."""
    rng = np.random.default_rng([seed, 0xC5])
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    out = []
    for i in range(n):
        k = int(rng.integers(1, 33))
        idx = sorted(int(j) for j in rng.choice(pool_size, size=k, replace=False))
        terms = loguniform_terms(rng)
        length = int(rng.integers(min_trials, min(max_trials, n_trials) + 1))
        t0 = int(rng.integers(0, n_trials - length + 1))
        out.append((float(t[i]), idx, terms, t0, t0 + length))
    return out


def uneven_analyses(n: int = 256, seed: int = SEED_BASE + 3, trials=(10_000, 500_000), mean=(200.0, 2000.0),
                    catalog=(100_000, 1_000_000), max_elts: int = 16, nnz: int = 20_000) -> List[Workload]:
    """Independent analyses of uneven shapes: trials log-uniform in `trials`, events
    per trial Poisson with a mean uniform in `mean`, catalogs uniform in `catalog`,
    U{1..max_elts} ELTs of `nnz` distinct events with lognormal(10, 2) losses; layer
    terms occurrence 1e5/5e6, aggregate 1e6/5e7.  With iid uniform IDs the draw order
    is taken as the time order (ordering by iid timestamps leaves the distribution of
    the ID sequence unchanged)."""
    return list(iter_uneven_analyses(n, seed, trials, mean, catalog, max_elts, nnz))


def iter_uneven_analyses(n: int = 256, seed: int = SEED_BASE + 3, trials=(10_000, 500_000), mean=(200.0, 2000.0),
                         catalog=(100_000, 1_000_000), max_elts: int = 16, nnz: int = 20_000):
    """uneven_analyses one analysis at a time (analysis a depends only on seed and a)."""
    for a in range(n):
        rng = np.random.default_rng([seed, 0xC4, a])
        n_t = int(round(math.exp(rng.uniform(math.log(trials[0]), math.log(trials[1])))))
        mu = float(rng.uniform(*mean))
        C = int(rng.integers(catalog[0], catalog[1] + 1))
        k = int(rng.integers(1, max_elts + 1))
        counts = rng.poisson(mu, size=n_t).astype(np.int64)
        offs = np.zeros(n_t + 1, dtype=np.int64)
        np.cumsum(counts, out=offs[1:])
        ids = _ids_blocks([seed, 0xC4, a], int(offs[-1]), C)
        elts = [elt_sparse(rng, min(nnz, C), C, 10.0, 2.0) for _ in range(k)]
        yield Workload(f"uneven-{a}-{n_t}x{mu:.0f}-cat{C}-{k}elt", ids, offs, C, elts, (1e5, 5e6, 1e6, 5e7), None,
                       (10.0, 100.0, 250.0), seed)


def random_tiny(rng: np.random.Generator, catalog_max: int = 8, elts_max: int = 6, trials_max: int = 8,
                events_max: int = 12, integer_losses: bool = False, allow_inf: bool = True,
                financial_terms: bool = False) -> Workload:
    """A random tiny analysis for brute-force checks: small catalog, a few ELTs
    (possibly none), trials that may be empty or repeat an event, and terms
    that may be zero or infinite."""
    C = int(rng.integers(1, catalog_max + 1))
    n_elts = int(rng.integers(0, elts_max + 1))
    elts = []
    for _ in range(n_elts):
        k = int(rng.integers(0, C + 1))
        ids = np.sort(rng.choice(C, size=k, replace=False)).astype(np.int32)
        if integer_losses:
            losses = rng.integers(0, 100, size=k).astype(np.float64)
        else:
            losses = rng.lognormal(3.0, 1.5, size=k)
        elts.append((ids, losses))
    n_trials = int(rng.integers(1, trials_max + 1))
    counts = rng.integers(0, events_max + 1, size=n_trials)
    offs = np.zeros(n_trials + 1, dtype=np.int64)
    np.cumsum(counts, out=offs[1:])
    ids = rng.integers(0, C, size=int(offs[-1])).astype(np.int32)

    def term(kind):
        r = rng.random()
        if kind == "ret":
            return 0.0 if r < 0.25 else float(rng.integers(0, 150)) if integer_losses else float(rng.lognormal(3, 1.5))
        if allow_inf and r < 0.25:
            return math.inf
        return 0.0 if r < 0.3 else float(rng.integers(0, 300)) if integer_losses else float(rng.lognormal(4, 1.5))

    lt = (term("ret"), term("lim"), term("ret"), term("lim"))
    et = None
    if financial_terms and n_elts:
        et = []
        for _ in range(n_elts):
            fx = float(rng.choice([1.0, 0.5, 2.0, 1.25])) if integer_losses else float(rng.uniform(0.5, 2.0))
            et.append((fx, term("ret"), term("lim")))
    return Workload("tiny", ids, offs, C, elts, lt, et, (1.0, 2.0, 3.0), 0)
