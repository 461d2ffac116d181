"""Uploads an analysis' numpy inputs to the GPU and creates its libara handles.

Marshalling only: every step of the analysis runs in libara's kernels.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import ara


@dataclasses.dataclass
class Analysis:
    ctx: ara.Ctx
    yet: ara.Yet
    elts: List[ara.Elt]
    layer: ara.Layer
    n_trials: int
    n_events: int

    def release(self):
        if self.layer.ptr:
            ara.ara_layer_release(self.layer)
        for e in self.elts:
            if e.ptr:
                ara.ara_elt_release(e)
        if self.yet.ptr:
            ara.ara_yet_release(self.yet)


def to_device(a: np.ndarray, device: int = 0):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(f"cuda:{device}")


def open_analysis(ctx: ara.Ctx, event_ids: np.ndarray, trial_offsets: np.ndarray, catalog_size: int,
                  elts: Sequence[Tuple[np.ndarray, np.ndarray]], layer_terms: Sequence[float],
                  elt_terms: Optional[Sequence[Sequence[float]]] = None, precision: int = ara.ARA_F64,
                  yet: Optional[ara.Yet] = None) -> Analysis:
    """Creates the YET (unless one is given), the ELTs and the layer on ctx's device."""
    if yet is None:
        yet = ara.ara_yet_create(ctx, to_device(np.asarray(event_ids, np.int32), ctx.device),
                                 to_device(np.asarray(trial_offsets, np.int64), ctx.device), catalog_size)
    handles = []
    for j, (ids, losses) in enumerate(elts):
        t = None if elt_terms is None else elt_terms[j]
        handles.append(ara.ara_elt_create(ctx, to_device(np.asarray(ids, np.int32), ctx.device),
                                          to_device(np.asarray(losses, np.float64), ctx.device), catalog_size,
                                          terms=t, precision=precision))
    layer = ara.ara_layer_create(ctx, handles, catalog_size, layer_terms)
    return Analysis(ctx, yet, handles, layer, yet.n_trials, yet.n_events)


@dataclasses.dataclass
class PortfolioHandles:
    ctx: ara.Ctx
    yet: ara.Yet
    pool: List[ara.Elt]
    layers: List[ara.Layer]

    def release(self):
        for layer in self.layers:
            if layer.ptr:
                ara.ara_layer_release(layer)
        for e in self.pool:
            if e.ptr:
                ara.ara_elt_release(e)
        if self.yet.ptr:
            ara.ara_yet_release(self.yet)


def open_portfolio(ctx: ara.Ctx, event_ids: np.ndarray, trial_offsets: np.ndarray, catalog_size: int,
                   pool: Sequence[Tuple[np.ndarray, np.ndarray]],
                   layers: Sequence[Tuple[Sequence[int], Sequence[float]]],
                   precision: int = ara.ARA_F32) -> PortfolioHandles:
    """Creates one YET, the ELTs of a pool and layers that each take some of them
    (pool indices, layer terms)."""
    yet = ara.ara_yet_create(ctx, to_device(np.asarray(event_ids, np.int32), ctx.device),
                             to_device(np.asarray(trial_offsets, np.int64), ctx.device), catalog_size)
    elts = [ara.ara_elt_create(ctx, to_device(np.asarray(ids, np.int32), ctx.device),
                               to_device(np.asarray(losses, np.float64), ctx.device), catalog_size,
                               precision=precision) for ids, losses in pool]
    made = [ara.ara_layer_create(ctx, [elts[i] for i in idx], catalog_size, terms) for idx, terms in layers]
    return PortfolioHandles(ctx, yet, elts, made)
