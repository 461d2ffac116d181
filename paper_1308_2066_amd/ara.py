"""Python binding of libara's C-ABI (include/ara.h): same names, argument
marshalling only.

Device buffers are torch tensors on the GPU; the binding passes their data
pointers and the current torch stream, keeps a reference to every borrowed
tensor inside the handle object, and raises ``AraError`` on a non-zero status.
Every computation runs in libara's HIP kernels: there is no CPU fallback, and
importing this module fails loudly when libara.so has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libara.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1308_2066_amd.build` "
                      "(or __graft_entry__.build()); there is no fallback implementation")

# torch ships its own HIP runtime under the same soname as ROCm's; loading torch
# first makes libara bind to that one runtime (torch provides the device memory
# and streams libara works on).
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

# ---------------------------------------------------------------------------- constants (ara.h)
ARA_OK = 0
ARA_E_INVALID_ARG = -1
ARA_E_EVENT_ID_RANGE = -2
ARA_E_BAD_OFFSETS = -3
ARA_E_BAD_LOSS = -4
ARA_E_DUP_EVENT = -5
ARA_E_BAD_TERMS = -6
ARA_E_EMPTY = -7
ARA_E_OOM = -8
ARA_E_DEVICE = -9
ARA_E_BUSY = -10
ARA_E_UNSUPPORTED = -11

ARA_F64 = 0
ARA_F32 = 1
ARA_MEM_HOST = 0
ARA_MEM_DEVICE = 1

ARA_PLACE_AUTO = 0
ARA_PLACE_LDS_BITMAP = 1
ARA_PLACE_LDS_DENSE = 2
ARA_PLACE_GLOBAL_DENSE = 3
ARA_PLACE_LDS_TILES = 4

ARA_OPT_PLACEMENT = 1
ARA_OPT_BLOCK_THREADS = 2
ARA_OPT_GRID_PER_CU = 3
ARA_OPT_YET_PACKING = 4
ARA_OPT_TRIAL_MODE = 5
ARA_OPT_YET_BINNING = 6
ARA_OPT_YET_RUN_BYTES = 7
ARA_OPT_KERNEL_TIMING = 8

ARA_BUILD_TABLES = 1

PLACEMENT_NAMES = {ARA_PLACE_LDS_BITMAP: "lds_bitmap", ARA_PLACE_LDS_DENSE: "lds_dense",
                   ARA_PLACE_GLOBAL_DENSE: "global_dense", ARA_PLACE_LDS_TILES: "lds_tiles"}


class ara_layer_terms(ctypes.Structure):
    _fields_ = [("occ_retention", ctypes.c_double), ("occ_limit", ctypes.c_double),
                ("agg_retention", ctypes.c_double), ("agg_limit", ctypes.c_double)]


class ara_elt_terms(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_double), ("retention", ctypes.c_double), ("limit", ctypes.c_double)]


class ara_job(ctypes.Structure):
    _fields_ = [("yet", ctypes.c_void_p), ("layer", ctypes.c_void_p), ("trial_begin", ctypes.c_int64),
                ("trial_end", ctypes.c_int64), ("ylt", ctypes.c_void_p)]


class ara_server_stats_t(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("completed", ctypes.c_int64), ("held", ctypes.c_int64),
                ("max_in_iteration", ctypes.c_int32), ("max_in_flight", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("slot_bytes", ctypes.c_int64), ("arena_bytes", ctypes.c_int64)]


class ara_server_config(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("memory_budget", ctypes.c_int64), ("n_rp", ctypes.c_int32),
                ("return_periods", ctypes.c_void_p)]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double
_ST = ctypes.c_int

_SIGS = {
    "ara_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "ara_last_error": (ctypes.c_char_p, [_P]),
    "ara_version": (ctypes.c_int, []),
    "ara_return_period_rank": (_ST, [_I64, _D, ctypes.POINTER(_I64)]),
    "ara_check_layer_terms": (_ST, [ctypes.POINTER(ara_layer_terms)]),
    "ara_ctx_create": (_ST, [ctypes.c_int, _P, ctypes.POINTER(_P)]),
    "ara_ctx_destroy": (_ST, [_P]),
    "ara_ctx_set_stream": (_ST, [_P, _P]),
    "ara_set_option": (_ST, [_P, ctypes.c_int, _I64]),
    "ara_sync": (_ST, [_P]),
    "ara_kernel_ms": (_ST, [_P, ctypes.POINTER(ctypes.c_float)]),
    "ara_yet_create": (_ST, [_P, _P, _I64, _P, _I64, _I32, ctypes.c_int, ctypes.POINTER(_P)]),
    "ara_yet_release": (_ST, [_P]),
    "ara_yet_info": (_ST, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I32)]),
    "ara_yet_binned": (_ST, [_P, ctypes.POINTER(_I32), _P, _P, _P]),
    "ara_yet_memory": (_ST, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I32)]),
    "ara_elt_create": (_ST, [_P, _P, _P, _I64, _I32, ctypes.POINTER(ara_elt_terms), ctypes.c_int, ctypes.c_int,
                             ctypes.POINTER(_P)]),
    "ara_elt_release": (_ST, [_P]),
    "ara_layer_create": (_ST, [_P, ctypes.POINTER(_P), _I32, _I32, ctypes.POINTER(ara_layer_terms),
                               ctypes.POINTER(_P)]),
    "ara_layer_set_terms": (_ST, [_P, _P, ctypes.POINTER(ara_layer_terms)]),
    "ara_layer_build": (_ST, [_P, _P, ctypes.c_int]),
    "ara_layer_stats": (_ST, [_P, _P, ctypes.POINTER(_I64), ctypes.POINTER(_I32), ctypes.POINTER(_I64)]),
    "ara_layer_release": (_ST, [_P]),
    "ara_analyze": (_ST, [_P, _P, _P, _I64, _I64, _P, ctypes.c_int]),
    "ara_analyze_events": (_ST, [_P, _P, _P, _I64, _I64, _P, _P, _P, _P, _P, ctypes.c_int]),
    "ara_lookup": (_ST, [_P, _P, _P, _I64, _P, _P, ctypes.c_int]),
    "ara_sort_workspace_size": (_ST, [_I64, ctypes.POINTER(ctypes.c_size_t)]),
    "ara_sort_desc": (_ST, [_P, _P, _I64, _P, _P, ctypes.c_size_t]),
    "ara_risk_measures": (_ST, [_P, _P, _I64, ctypes.c_int, _P, _I32, _P, _P, _P, ctypes.c_size_t]),
    "ara_risk_measures_noalloc": (_ST, [_P, _P, _I64, _P, _I32, _P, _P]),
    "ara_batch_create": (_ST, [_P, ctypes.POINTER(ara_job), _I32, ctypes.POINTER(_P)]),
    "ara_batch_run": (_ST, [_P]),
    "ara_batch_risk": (_ST, [_P, _P, _I32, _P, _P]),
    "ara_batch_portfolio": (_ST, [_P, _P]),
    "ara_analyze_occ_max": (_ST, [_P, _P, _P, _I64, _I64, _P, ctypes.c_int]),
    "ara_batch_info": (_ST, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I64),
                             ctypes.POINTER(_I32)]),
    "ara_batch_release": (_ST, [_P]),
    "ara_tune_cache_save": (_ST, [_P, ctypes.c_char_p]),
    "ara_tune_cache_load": (_ST, [_P, ctypes.c_char_p]),
    "ara_server_create": (_ST, [_P, _P, ctypes.POINTER(_P), _I32, ctypes.POINTER(ara_server_config),
                                ctypes.POINTER(_P)]),
    "ara_server_submit": (_ST, [_P, _P, _I32, ctypes.POINTER(ara_layer_terms), _I64, _I64,
                                ctypes.POINTER(ctypes.c_uint64)]),
    "ara_server_wait": (_ST, [_P, ctypes.c_uint64, _P, _P, ctypes.POINTER(_D)]),
    "ara_server_stats": (_ST, [_P, _P]),
    "ara_server_release": (_ST, [_P]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


class AraError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        msg = f"{where}: {_lib.ara_status_str(status).decode()} ({status})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)
        self.status = status


def ara_status_str(status: int) -> str:
    return _lib.ara_status_str(int(status)).decode()


def ara_version() -> int:
    return int(_lib.ara_version())


def ara_return_period_rank(n: int, rp: float) -> int:
    k = _I64(0)
    st = _lib.ara_return_period_rank(int(n), float(rp), ctypes.byref(k))
    if st:
        raise AraError(st, "ara_return_period_rank")
    return int(k.value)


def _terms(t: Sequence[float]) -> ara_layer_terms:
    return ara_layer_terms(float(t[0]), float(t[1]), float(t[2]), float(t[3]))


def ara_check_layer_terms(t: Sequence[float]) -> int:
    return int(_lib.ara_check_layer_terms(ctypes.byref(_terms(t))))


# ---------------------------------------------------------------------------- handles
class Ctx:
    def __init__(self, ptr, device):
        self.ptr = ptr
        self.device = device

    def last_error(self) -> str:
        return _lib.ara_last_error(self.ptr).decode()


class Yet:
    def __init__(self, ptr, ctx, keep, n_trials, n_events, catalog):
        self.ptr, self.ctx, self._keep = ptr, ctx, keep
        self.n_trials, self.n_events, self.catalog_size = n_trials, n_events, catalog


class Elt:
    def __init__(self, ptr, ctx, keep, catalog, precision):
        self.ptr, self.ctx, self._keep = ptr, ctx, keep
        self.catalog_size, self.precision = catalog, precision


class Layer:
    def __init__(self, ptr, ctx, elts, catalog):
        self.ptr, self.ctx, self.elts, self.catalog_size = ptr, ctx, list(elts), catalog


class Batch:
    def __init__(self, ptr, ctx, keep, n_jobs):
        self.ptr, self.ctx, self._keep, self.n_jobs = ptr, ctx, keep, n_jobs


def _check(st: int, ctx: Optional[Ctx], where: str):
    if st:
        detail = ctx.last_error() if ctx is not None and ctx.ptr else _lib.ara_last_error(None).decode()
        raise AraError(st, where, detail)


def _dev_ptr(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def ara_ctx_create(device: int = 0, stream=None) -> Ctx:
    import torch
    torch.cuda.set_device(device)
    out = _P()
    _check(_lib.ara_ctx_create(int(device), _stream_ptr(stream), ctypes.byref(out)), None, "ara_ctx_create")
    return Ctx(out, device)


def ara_ctx_destroy(ctx: Ctx):
    _check(_lib.ara_ctx_destroy(ctx.ptr), ctx, "ara_ctx_destroy")
    ctx.ptr = None


def ara_ctx_set_stream(ctx: Ctx, stream=None):
    _check(_lib.ara_ctx_set_stream(ctx.ptr, _stream_ptr(stream)), ctx, "ara_ctx_set_stream")


def ara_set_option(ctx: Ctx, option: int, value: int):
    _check(_lib.ara_set_option(ctx.ptr, int(option), int(value)), ctx, "ara_set_option")


def ara_sync(ctx: Ctx):
    _check(_lib.ara_sync(ctx.ptr), ctx, "ara_sync")


def ara_kernel_ms(ctx: Ctx) -> float:
    """Duration of the last ara_analyze trial kernel timed under ARA_OPT_KERNEL_TIMING."""
    ms = ctypes.c_float()
    _check(_lib.ara_kernel_ms(ctx.ptr, ctypes.byref(ms)), ctx, "ara_kernel_ms")
    return float(ms.value)


def ara_yet_create(ctx: Ctx, event_ids, trial_offsets, catalog_size: int) -> Yet:
    """event_ids: int32 GPU tensor (16-byte aligned); trial_offsets: int64 GPU tensor."""
    import torch
    pi = _dev_ptr(event_ids, torch.int32, "event_ids")
    po = _dev_ptr(trial_offsets, torch.int64, "trial_offsets")
    n_trials = trial_offsets.numel() - 1
    out = _P()
    _check(_lib.ara_yet_create(ctx.ptr, pi, event_ids.numel(), po, n_trials, int(catalog_size), ARA_MEM_DEVICE,
                               ctypes.byref(out)), ctx, "ara_yet_create")
    return Yet(out, ctx, (event_ids, trial_offsets), n_trials, event_ids.numel(), int(catalog_size))


def ara_yet_release(y: Yet):
    _check(_lib.ara_yet_release(y.ptr), y.ctx, "ara_yet_release")
    y.ptr, y._keep = None, None


def ara_yet_info(y: Yet):
    """(n_events, n_trials, id_bytes): id_bytes is 2 when the handle has a catalog-binned
    copy (read by the tiled kernel for layers whose table does not fit in LDS), else 3
    with a packed copy of the event IDs, else 4."""
    ne, nt, b = _I64(), _I64(), _I32()
    _check(_lib.ara_yet_info(y.ptr, ctypes.byref(ne), ctypes.byref(nt), ctypes.byref(b)), y.ctx, "ara_yet_info")
    return int(ne.value), int(nt.value), int(b.value)


def ara_yet_binned_count(y: Yet) -> int:
    """Number of catalog bins of the YET's binned copy (0 without one)."""
    nb = _I32()
    _check(_lib.ara_yet_binned(y.ptr, ctypes.byref(nb), None, None, None), y.ctx, "ara_yet_binned")
    return int(nb.value)


def ara_yet_memory(y: Yet):
    """(device_bytes, run_bytes): device memory the handle holds (its packed or binned
    copy, plus its own copies of host arrays) and the bytes per run start of its binned
    copy (3 or 4; 0 without one)."""
    nb, rb = _I64(), _I32()
    _check(_lib.ara_yet_memory(y.ptr, ctypes.byref(nb), ctypes.byref(rb)), y.ctx, "ara_yet_memory")
    return int(nb.value), int(rb.value)


def ara_yet_binned(y: Yet):
    """The YET's catalog-binned copy as numpy arrays (region int64[n_bins + 1], boff
    uint32[n_bins, n_trials + 1], ids16 uint16[region[-1]]), or None without one."""
    import numpy as np
    nb = _I32()
    _check(_lib.ara_yet_binned(y.ptr, ctypes.byref(nb), None, None, None), y.ctx, "ara_yet_binned")
    if nb.value == 0:
        return None
    region = np.zeros(nb.value + 1, np.int64)
    _check(_lib.ara_yet_binned(y.ptr, ctypes.byref(nb), region.ctypes.data, None, None), y.ctx, "ara_yet_binned")
    boff = np.zeros((nb.value, y.n_trials + 1), np.uint32)
    ids16 = np.zeros(int(region[-1]), np.uint16)
    _check(_lib.ara_yet_binned(y.ptr, ctypes.byref(nb), region.ctypes.data, boff.ctypes.data, ids16.ctypes.data),
           y.ctx, "ara_yet_binned")
    return region, boff, ids16


def ara_elt_create(ctx: Ctx, event_ids, losses, catalog_size: int, terms: Optional[Sequence[float]] = None,
                   precision: int = ARA_F64) -> Elt:
    """event_ids: int32 GPU tensor; losses: float64 GPU tensor; terms: (fx, retention, limit) or None."""
    import torch
    pi = _dev_ptr(event_ids, torch.int32, "event_ids")
    pl = _dev_ptr(losses, torch.float64, "losses")
    if event_ids.numel() != losses.numel():
        raise ValueError("event_ids and losses differ in length")
    et = None
    if terms is not None:
        et = ctypes.byref(ara_elt_terms(float(terms[0]), float(terms[1]), float(terms[2])))
    out = _P()
    _check(_lib.ara_elt_create(ctx.ptr, pi, pl, event_ids.numel(), int(catalog_size), et, int(precision),
                               ARA_MEM_DEVICE, ctypes.byref(out)), ctx, "ara_elt_create")
    return Elt(out, ctx, (event_ids, losses), int(catalog_size), int(precision))


def ara_elt_release(e: Elt):
    _check(_lib.ara_elt_release(e.ptr), e.ctx, "ara_elt_release")
    e.ptr, e._keep = None, None


def ara_layer_create(ctx: Ctx, elts: Sequence[Elt], catalog_size: int, terms: Sequence[float]) -> Layer:
    arr = (_P * max(1, len(elts)))(*[e.ptr for e in elts])
    out = _P()
    _check(_lib.ara_layer_create(ctx.ptr, arr, len(elts), int(catalog_size), ctypes.byref(_terms(terms)),
                                 ctypes.byref(out)), ctx, "ara_layer_create")
    return Layer(out, ctx, elts, int(catalog_size))


def ara_layer_set_terms(ctx: Ctx, layer: Layer, terms: Sequence[float]):
    _check(_lib.ara_layer_set_terms(ctx.ptr, layer.ptr, ctypes.byref(_terms(terms))), ctx, "ara_layer_set_terms")


def ara_layer_build(ctx: Ctx, layer: Layer, flags: int = 0):
    _check(_lib.ara_layer_build(ctx.ptr, layer.ptr, int(flags)), ctx, "ara_layer_build")


def ara_layer_stats(ctx: Ctx, layer: Layer):
    """(n_occ_nonzero, placement, lds_bytes)."""
    n = _I64(0)
    p = _I32(0)
    b = _I64(0)
    _check(_lib.ara_layer_stats(ctx.ptr, layer.ptr, ctypes.byref(n), ctypes.byref(p), ctypes.byref(b)), ctx,
           "ara_layer_stats")
    return int(n.value), int(p.value), int(b.value)


def ara_layer_release(layer: Layer):
    _check(_lib.ara_layer_release(layer.ptr), layer.ctx, "ara_layer_release")
    layer.ptr = None


def ara_analyze(ctx: Ctx, yet: Yet, layer: Layer, trial_begin: int, trial_end: int, ylt):
    """ylt: float64 GPU tensor with trial_end - trial_begin elements (asynchronous)."""
    import torch
    p = _dev_ptr(ylt, torch.float64, "ylt")
    if ylt.numel() < trial_end - trial_begin:
        raise ValueError("ylt too small")
    _check(_lib.ara_analyze(ctx.ptr, yet.ptr, layer.ptr, int(trial_begin), int(trial_end), p, ARA_MEM_DEVICE), ctx,
           "ara_analyze")


def ara_analyze_occ_max(ctx: Ctx, yet: Yet, layer: Layer, t0: int, t1: int, out):
    """Largest occurrence-net loss per trial of [t0, t1) into a float64 GPU tensor (asynchronous)."""
    import torch
    _check(_lib.ara_analyze_occ_max(ctx.ptr, yet.ptr, layer.ptr, int(t0), int(t1), _dev_ptr(out, torch.float64, "out"),
                                    ARA_MEM_DEVICE), ctx, "ara_analyze_occ_max")


def ara_analyze_events(ctx: Ctx, yet: Yet, layer: Layer, trial_begin: int, trial_end: int, ylt=None,
                       ev_gross=None, ev_occ=None, ev_cum=None, ev_ceded=None):
    """Per-occurrence outputs (float64 GPU tensors or None), asynchronous."""
    import torch
    ptrs = [None if t is None else _dev_ptr(t, torch.float64, n)
            for t, n in ((ylt, "ylt"), (ev_gross, "ev_gross"), (ev_occ, "ev_occ"), (ev_cum, "ev_cum"),
                         (ev_ceded, "ev_ceded"))]
    _check(_lib.ara_analyze_events(ctx.ptr, yet.ptr, layer.ptr, int(trial_begin), int(trial_end), *ptrs,
                                   ARA_MEM_DEVICE), ctx, "ara_analyze_events")


def ara_lookup(ctx: Ctx, layer: Layer, event_ids, gross=None, occ=None):
    import torch
    pi = _dev_ptr(event_ids, torch.int32, "event_ids")
    pg = None if gross is None else _dev_ptr(gross, torch.float64, "gross")
    po = None if occ is None else _dev_ptr(occ, torch.float64, "occ")
    _check(_lib.ara_lookup(ctx.ptr, layer.ptr, pi, event_ids.numel(), pg, po, ARA_MEM_DEVICE), ctx, "ara_lookup")


def ara_sort_workspace_size(n: int) -> int:
    b = ctypes.c_size_t(0)
    _check(_lib.ara_sort_workspace_size(int(n), ctypes.byref(b)), None, "ara_sort_workspace_size")
    return int(b.value)


def _workspace(values, workspace):
    """The caller's sort workspace, or a torch allocation of ara_sort_workspace_size
    bytes (the library then allocates nothing)."""
    import torch
    if workspace is None:
        workspace = torch.empty(max(1, ara_sort_workspace_size(values.numel())), dtype=torch.uint8,
                                device=values.device)
    return workspace, _dev_ptr(workspace, torch.uint8, "workspace")


def ara_sort_desc(ctx: Ctx, values, out, workspace=None):
    """Descending sort of a float64 GPU tensor into out.  Asynchronous with a caller
    workspace; with none, the binding allocates one through torch and waits for the
    sort before it is released."""
    import torch
    pv = _dev_ptr(values, torch.float64, "values")
    po = _dev_ptr(out, torch.float64, "out")
    own = workspace is None
    workspace, pw = _workspace(values, workspace)
    _check(_lib.ara_sort_desc(ctx.ptr, pv, values.numel(), po, pw, workspace.numel()), ctx, "ara_sort_desc")
    if own:
        ara_sync(ctx)


def ara_risk_measures(ctx: Ctx, ylt, return_periods: Sequence[float], workspace=None):
    """(pml, tvar) numpy arrays for a float64 GPU tensor YLT (blocking).  Without a
    workspace the binding allocates one through torch."""
    import torch
    py = _dev_ptr(ylt, torch.float64, "ylt")
    rp = np.ascontiguousarray(np.asarray(return_periods, dtype=np.float64))
    pml = np.empty(rp.shape[0], np.float64)
    tvar = np.empty(rp.shape[0], np.float64)
    workspace, pw = _workspace(ylt, workspace)     # blocking call: a torch workspace may go after it
    _check(_lib.ara_risk_measures(ctx.ptr, py, ylt.numel(), ARA_MEM_DEVICE, rp.ctypes.data_as(_P), rp.shape[0],
                                  pml.ctypes.data_as(_P), tvar.ctypes.data_as(_P), pw, workspace.numel()), ctx,
           "ara_risk_measures")
    return pml, tvar


ARA_NOALLOC_MAX_N = 1 << 20
ARA_NOALLOC_SCRATCH_BYTES = 17 << 20


def ara_risk_measures_noalloc(ctx: Ctx, ylt, return_periods: Sequence[float]):
    """(pml, tvar) as ara_risk_measures, with the sort workspace in the library's own
    device array (no allocation by the library or the binding; blocking)."""
    import torch
    py = _dev_ptr(ylt, torch.float64, "ylt")
    rp = np.ascontiguousarray(np.asarray(return_periods, dtype=np.float64))
    pml = np.empty(rp.shape[0], np.float64)
    tvar = np.empty(rp.shape[0], np.float64)
    _check(_lib.ara_risk_measures_noalloc(ctx.ptr, py, ylt.numel(), rp.ctypes.data_as(_P), rp.shape[0],
                                          pml.ctypes.data_as(_P), tvar.ctypes.data_as(_P)), ctx,
           "ara_risk_measures_noalloc")
    return pml, tvar


# ---------------------------------------------------------------------------- host-memory forms
def ara_yet_create_host(ctx: Ctx, event_ids: np.ndarray, trial_offsets: np.ndarray, catalog_size: int) -> Yet:
    """As ara_yet_create, from host arrays (copied to the device by the library)."""
    ids = np.ascontiguousarray(event_ids, dtype=np.int32)
    offs = np.ascontiguousarray(trial_offsets, dtype=np.int64)
    out = _P()
    _check(_lib.ara_yet_create(ctx.ptr, ids.ctypes.data_as(_P), ids.shape[0], offs.ctypes.data_as(_P),
                               offs.shape[0] - 1, int(catalog_size), ARA_MEM_HOST, ctypes.byref(out)), ctx,
           "ara_yet_create")
    return Yet(out, ctx, None, offs.shape[0] - 1, ids.shape[0], int(catalog_size))


def ara_elt_create_host(ctx: Ctx, event_ids: np.ndarray, losses: np.ndarray, catalog_size: int,
                        terms: Optional[Sequence[float]] = None, precision: int = ARA_F64) -> Elt:
    ids = np.ascontiguousarray(event_ids, dtype=np.int32)
    ls = np.ascontiguousarray(losses, dtype=np.float64)
    et = None if terms is None else ctypes.byref(ara_elt_terms(float(terms[0]), float(terms[1]), float(terms[2])))
    out = _P()
    _check(_lib.ara_elt_create(ctx.ptr, ids.ctypes.data_as(_P), ls.ctypes.data_as(_P), ids.shape[0],
                               int(catalog_size), et, int(precision), ARA_MEM_HOST, ctypes.byref(out)), ctx,
           "ara_elt_create")
    return Elt(out, ctx, None, int(catalog_size), int(precision))


def ara_analyze_host(ctx: Ctx, yet: Yet, layer: Layer, trial_begin: int, trial_end: int) -> np.ndarray:
    out = np.empty(trial_end - trial_begin, np.float64)
    _check(_lib.ara_analyze(ctx.ptr, yet.ptr, layer.ptr, int(trial_begin), int(trial_end), out.ctypes.data_as(_P),
                            ARA_MEM_HOST), ctx, "ara_analyze")
    return out


# ----------------------------------------------------------------------------- batches
def ara_batch_create(ctx: Ctx, jobs) -> Batch:
    """jobs: sequence of (Yet, Layer, trial_begin, trial_end, ylt) with ylt a float64
    GPU tensor of trial_end - trial_begin elements."""
    import torch
    arr = (ara_job * max(len(jobs), 1))()
    keep = []
    for i, (y, layer, t0, t1, ylt) in enumerate(jobs):
        py = _dev_ptr(ylt, torch.float64, "ylt")
        if ylt.numel() < t1 - t0:
            raise ValueError("ylt shorter than the job's trial range")
        arr[i] = ara_job(y.ptr, layer.ptr, int(t0), int(t1), py.value)
        keep.append((y, layer, ylt))
    out = _P()
    _check(_lib.ara_batch_create(ctx.ptr, arr, len(jobs), ctypes.byref(out)), ctx, "ara_batch_create")
    return Batch(out, ctx, keep, len(jobs))


def ara_batch_run(b: Batch):
    _check(_lib.ara_batch_run(b.ptr), b.ctx, "ara_batch_run")


def ara_batch_risk(b: Batch, return_periods: Sequence[float]):
    """(pml, tvar) numpy arrays of shape (n_jobs, n_rp) (blocking)."""
    rp = np.ascontiguousarray(np.asarray(return_periods, dtype=np.float64))
    pml = np.empty((b.n_jobs, rp.shape[0]), np.float64)
    tvar = np.empty_like(pml)
    _check(_lib.ara_batch_risk(b.ptr, rp.ctypes.data_as(_P), rp.shape[0], pml.ctypes.data_as(_P),
                               tvar.ctypes.data_as(_P)), b.ctx, "ara_batch_risk")
    return pml, tvar


def ara_batch_portfolio(b: Batch, out):
    """Portfolio YLT (sum of the jobs' YLTs per trial, job order) into a float64 GPU tensor."""
    import torch
    _check(_lib.ara_batch_portfolio(b.ptr, _dev_ptr(out, torch.float64, "out")), b.ctx, "ara_batch_portfolio")


def ara_batch_info(b: Batch):
    """(n_items, grid, events_per_item, graph)."""
    n, g, e, gr = _I32(), _I32(), _I64(), _I32()
    _check(_lib.ara_batch_info(b.ptr, ctypes.byref(n), ctypes.byref(g), ctypes.byref(e), ctypes.byref(gr)), b.ctx,
           "ara_batch_info")
    return int(n.value), int(g.value), int(e.value), int(gr.value)


def ara_tune_cache_save(ctx: Ctx, path: str):
    """Writes the context's tuned batch schedules to a text file."""
    _check(_lib.ara_tune_cache_save(ctx.ptr, os.fsencode(path)), ctx, "ara_tune_cache_save")


def ara_tune_cache_load(ctx: Ctx, path: str):
    """Reads tuned batch schedules from a file written by ara_tune_cache_save."""
    _check(_lib.ara_tune_cache_load(ctx.ptr, os.fsencode(path)), ctx, "ara_tune_cache_load")


def ara_batch_release(b: Batch):
    _check(_lib.ara_batch_release(b.ptr), b.ctx, "ara_batch_release")
    b.ptr, b._keep = None, None


# ----------------------------------------------------------------------------- serving
class Server:
    def __init__(self, ptr, ctx, keep, n_rp):
        self.ptr, self.ctx, self._keep, self.n_rp = ptr, ctx, keep, n_rp


def ara_server_create(ctx: Ctx, yet: Yet, pool: Sequence[Elt], return_periods: Sequence[float], max_batch: int = 32,
                      memory_budget: int = 0) -> Server:
    rp = np.ascontiguousarray(np.asarray(return_periods, dtype=np.float64))
    arr = (_P * len(pool))(*[e.ptr for e in pool])
    cfg = ara_server_config(int(max_batch), int(memory_budget), rp.shape[0], rp.ctypes.data_as(_P).value)
    out = _P()
    _check(_lib.ara_server_create(ctx.ptr, yet.ptr, arr, len(pool), ctypes.byref(cfg), ctypes.byref(out)), ctx,
           "ara_server_create")
    return Server(out, ctx, (yet, list(pool), rp), rp.shape[0])


def ara_server_submit(s: Server, elt_index: Sequence[int], terms: Sequence[float], trial_begin: int,
                      trial_end: int) -> int:
    idx = np.ascontiguousarray(np.asarray(elt_index, dtype=np.int32))
    t = ctypes.c_uint64()
    _check(_lib.ara_server_submit(s.ptr, idx.ctypes.data_as(_P), idx.shape[0], ctypes.byref(_terms(terms)),
                                  int(trial_begin), int(trial_end), ctypes.byref(t)), s.ctx, "ara_server_submit")
    return int(t.value)


def ara_server_wait(s: Server, ticket: int):
    """(pml, tvar, seconds from submission to completion); blocks (the GIL is released)."""
    pml = np.empty(s.n_rp, np.float64)
    tvar = np.empty(s.n_rp, np.float64)
    sec = _D()
    _check(_lib.ara_server_wait(s.ptr, ctypes.c_uint64(int(ticket)), pml.ctypes.data_as(_P), tvar.ctypes.data_as(_P),
                                ctypes.byref(sec)), s.ctx, "ara_server_wait")
    return pml, tvar, float(sec.value)


def ara_server_stats(s: Server) -> dict:
    """Counters and sizes: iterations, completed, held, max_in_iteration, max_in_flight,
    slots, slot_bytes, arena_bytes."""
    st = ara_server_stats_t()
    _check(_lib.ara_server_stats(s.ptr, ctypes.byref(st)), s.ctx, "ara_server_stats")
    return {k: int(getattr(st, k)) for k, _ in ara_server_stats_t._fields_ if k != "pad_"}


def ara_server_release(s: Server):
    _check(_lib.ara_server_release(s.ptr), s.ctx, "ara_server_release")
    s.ptr, s._keep = None, None
