// C-ABI of libara: handle lifetimes, argument validation, table placement and the
// launches of the analysis path.  Declarations and contracts: include/ara.h.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ara_internal.h"

using namespace ara;

struct ara_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int n_cu = 0;
    int lds_max = 0;
    uint32_t *d_err = nullptr;       // device error bits
    double *d_out = nullptr;         // small device result staging
    double *h_out = nullptr;         // pinned host mirror of d_out
    uint32_t *h_err = nullptr;       // pinned host error word
    int placement = ARA_PLACE_AUTO;
    int block_threads = 0;           // 0 = automatic
    int grid_per_cu = 0;             // 0 = automatic
    int yet_packing = 1;             // keep a packed copy of YET IDs where they fit 24 bits
    int live = 0;                    // handles alive on this context
    std::string msg;
};

struct ara_yet {
    ara_ctx *ctx;
    const int32_t *ids;
    const int64_t *offs;
    int64_t n_events, n_trials;
    int32_t catalog;
    bool owns;
    uint8_t *ids24;    // packed copy (owned), or null
};

struct ara_elt {
    ara_ctx *ctx;
    int32_t catalog;
    ara_precision prec;
    const int32_t *pair_ids;
    const double *pair_losses;
    int64_t n_pairs;
    bool owns_pairs;
    void *dat;
    uint32_t *seen;
    EltDesc *d_desc;     // this ELT alone, for its own builds
    EltDesc desc;
    int users;           // live layers referencing this ELT
};

struct ara_layer {
    ara_ctx *ctx;
    std::vector<ara_elt *> elts;
    ara_layer_terms terms;
    int32_t catalog;
    bool f32;
    EltDesc *d_descs;    // device copy of the member ELTs' descriptors
    int64_t max_pairs;
    LayerTables t;
};

static constexpr size_t kStageDoubles = 512;   // 2 x 256 return periods
static constexpr int32_t kMaxCatalog = 1 << 28; // byte offsets into catalog tables stay below 2^31
static constexpr int32_t kMaxElts = 65535;      // ELT index is a grid dimension of the table builds
static constexpr int32_t kMaxPackedCatalog = 1 << 24;   // IDs of a packed YET copy take 3 bytes

// ------------------------------------------------------------------ helpers
// Message of the last error that had no context to hold it (ara_ctx_create).
static thread_local std::string g_msg;

static ara_status fail(ara_ctx *c, ara_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->msg = buf;
    else g_msg = buf;
    return s;
}

static ara_status hip_fail(ara_ctx *c, hipError_t e, const char *what) {
    if (e == hipErrorOutOfMemory) return fail(c, ARA_E_OOM, "%s: out of device memory", what);
    return fail(c, ARA_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_OR_RETURN(ctx, expr, what)                  \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
    } while (0)

static bool bad_retention(double r) { return !(r >= 0.0) || std::isinf(r); }
static bool bad_limit(double l) { return !(l >= 0.0); }

static ara_status err_bits_status(uint32_t bits) {
    if (bits & ERR_ID_RANGE) return ARA_E_EVENT_ID_RANGE;
    if (bits & ERR_OFFSETS) return ARA_E_BAD_OFFSETS;
    if (bits & ERR_LOSS) return ARA_E_BAD_LOSS;
    if (bits & ERR_DUP) return ARA_E_DUP_EVENT;
    return ARA_OK;
}

// Waits for the context stream, then reads and clears the device error word.
static ara_status sync_and_check(ara_ctx *c) {
    HIP_OR_RETURN(c, hipMemcpyAsync(c->h_err, c->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream),
                  "read error word");
    HIP_OR_RETURN(c, hipStreamSynchronize(c->stream), "stream synchronize");
    const uint32_t bits = *c->h_err;
    if (bits) {
        HIP_OR_RETURN(c, launch_fill_u32(c->d_err, 1, 0u, c->stream), "clear error word");
        HIP_OR_RETURN(c, hipStreamSynchronize(c->stream), "stream synchronize");
        ara_status s = err_bits_status(bits);
        return fail(c, s, "device-detected input error (bits 0x%x): %s", bits, ara_status_str(s));
    }
    return ARA_OK;
}

template <typename T>
static ara_status dev_alloc(ara_ctx *c, T **p, size_t bytes, const char *what) {
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return hip_fail(c, e, what);
    }
    return ARA_OK;
}

static void dev_free(void *p) {
    if (p) (void)hipFree(p);
}

// The bitmap trial kernel keeps the filter tables and its per-wave event queues
// (16 waves x kQueueCapMax events) in static LDS.  Returns the queue capacity for a
// workgroup of wpb waves, or 0 if the catalog's tables do not fit.
static int bitmap_qcap(int32_t catalog, int wpb, int lds_max) {
    const size_t table = bitmap_table_bytes(bitmap_blocks(catalog));
    if (wpb > 16 || lds_max < kLdsMaxBytes || table > trial_bitmap_table_capacity()) return 0;
    return kQueueCapMax;
}

// Chooses where the layer's table lives during the trial kernel and the launch shape.
static ara_status plan_trial(ara_ctx *c, const ara_layer *L, int64_t n_trials, TrialLaunch &tl) {
    int pl = c->placement;
    const int64_t dense = int64_t(L->catalog) * 8;
    const int block_bitmap = c->block_threads ? c->block_threads : 1024;
    const int qcap = bitmap_qcap(L->catalog, block_bitmap / 64, c->lds_max);
    if (pl == ARA_PLACE_AUTO) {
        if (dense <= c->lds_max) pl = ARA_PLACE_LDS_DENSE;
        else if (qcap > 0) pl = ARA_PLACE_LDS_BITMAP;
        else pl = ARA_PLACE_GLOBAL_DENSE;
    }
    int64_t lds = 0;
    if (pl == ARA_PLACE_LDS_DENSE) {
        lds = dense;
        if (lds > c->lds_max)
            return fail(c, ARA_E_UNSUPPORTED, "dense LDS table needs %lld bytes, device allows %d", (long long)lds, c->lds_max);
    } else if (pl == ARA_PLACE_LDS_BITMAP) {
        if (qcap == 0)
            return fail(c, ARA_E_UNSUPPORTED, "LDS bitmap of a %d-event catalog leaves no room for the event queues",
                        L->catalog);
        lds = int64_t(bitmap_table_bytes(bitmap_blocks(L->catalog)));   // lookup kernel: dynamic LDS table
    }
    tl.placement = pl;
    tl.f32 = L->f32;
    tl.lds_bytes = size_t(lds);
    tl.qcap = pl == ARA_PLACE_LDS_BITMAP ? qcap : 0;
    tl.block = c->block_threads ? c->block_threads : (pl == ARA_PLACE_GLOBAL_DENSE ? 256 : 1024);
    int per_cu = c->grid_per_cu;
    if (per_cu == 0) {
        const int by_threads = 2048 / tl.block;
        const int64_t lds_all = pl == ARA_PLACE_LDS_BITMAP ? int64_t(kLdsMaxBytes) : lds;   // static LDS = all of it
        const int by_lds = lds_all > 0 ? int(c->lds_max / lds_all) : by_threads;
        per_cu = std::max(1, std::min(by_threads, by_lds));
    }
    int64_t grid = int64_t(c->n_cu) * per_cu;
    const int64_t wpb = tl.block / 64;                      // one wave per trial at a time
    grid = std::min<int64_t>(grid, std::max<int64_t>(1, (n_trials + wpb - 1) / wpb));
    tl.grid = int(grid);
    return ARA_OK;
}

// ------------------------------------------------------------------ misc
extern "C" const char *ara_status_str(int s) {
    switch (s) {
    case ARA_OK: return "ok";
    case ARA_E_INVALID_ARG: return "invalid argument";
    case ARA_E_EVENT_ID_RANGE: return "event id outside the catalog";
    case ARA_E_BAD_OFFSETS: return "trial offsets are not CSR";
    case ARA_E_BAD_LOSS: return "loss negative, NaN or infinite";
    case ARA_E_DUP_EVENT: return "event listed twice in an ELT";
    case ARA_E_BAD_TERMS: return "invalid terms";
    case ARA_E_EMPTY: return "empty year loss table";
    case ARA_E_OOM: return "out of device memory";
    case ARA_E_DEVICE: return "device or HIP runtime error";
    case ARA_E_BUSY: return "handle in use";
    case ARA_E_UNSUPPORTED: return "unsupported table placement";
    default: return "unknown status";
    }
}

extern "C" const char *ara_last_error(const ara_ctx *c) { return c ? c->msg.c_str() : g_msg.c_str(); }

extern "C" int ara_version(void) { return 100; }

extern "C" ara_status ara_return_period_rank(int64_t n, double rp, int64_t *k) {
    if (!k || n < 1 || !(rp >= 1.0)) return ARA_E_INVALID_ARG;
    const double q = double(n) / rp;
    const double r = std::nearbyint(q);
    const double ulp = std::nextafter(q, INFINITY) - q;
    double kk = (std::fabs(q - r) <= 4.0 * ulp) ? r : std::ceil(q);
    kk = kk < 1.0 ? 1.0 : (kk > double(n) ? double(n) : kk);
    *k = int64_t(kk);
    return ARA_OK;
}

extern "C" ara_status ara_check_layer_terms(const ara_layer_terms *t) {
    if (!t) return ARA_E_INVALID_ARG;
    if (bad_retention(t->occ_retention) || bad_limit(t->occ_limit) || bad_retention(t->agg_retention) ||
        bad_limit(t->agg_limit))
        return ARA_E_BAD_TERMS;
    return ARA_OK;
}

static ara_status check_elt_terms(const ara_elt_terms *t) {
    if (!t) return ARA_OK;
    if (!(t->fx >= 0.0) || std::isinf(t->fx) || bad_retention(t->retention) || bad_limit(t->limit))
        return ARA_E_BAD_TERMS;
    return ARA_OK;
}

// ------------------------------------------------------------------ context
extern "C" ara_status ara_ctx_create(int device, void *hip_stream, ara_ctx **out) {
    if (!out) return fail(nullptr, ARA_E_INVALID_ARG, "ctx: NULL output");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return fail(nullptr, ARA_E_DEVICE, "ctx: no HIP device (%s)", hipGetErrorString(e));
    }
    if (device < 0 || device >= n) return fail(nullptr, ARA_E_INVALID_ARG, "ctx: device %d of %d", device, n);
    hipDeviceProp_t p;
    e = hipGetDeviceProperties(&p, device);
    if (e != hipSuccess) return fail(nullptr, ARA_E_DEVICE, "ctx: device properties: %s", hipGetErrorString(e));
    if (std::strncmp(p.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, ARA_E_DEVICE, "ctx: device %d is %s, this library is built for gfx950", device, p.gcnArchName);
    e = hipSetDevice(device);
    if (e != hipSuccess) return fail(nullptr, ARA_E_DEVICE, "ctx: set device: %s", hipGetErrorString(e));
    ara_ctx *c = new (std::nothrow) ara_ctx();
    if (!c) return fail(nullptr, ARA_E_OOM, "ctx: host allocation");
    c->device = device;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->n_cu = p.multiProcessorCount;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) lds = 65536;
    c->lds_max = std::min(lds, kLdsMaxBytes);
    const char *step = "kernel attributes";
    e = prepare_trial_kernels();
    if (e == hipSuccess) { step = "error word"; e = hipMalloc(&c->d_err, 256); }
    if (e == hipSuccess) { step = "result staging"; e = hipMalloc(&c->d_out, kStageDoubles * sizeof(double)); }
    if (e == hipSuccess) {
        step = "pinned staging";
        e = hipHostMalloc(reinterpret_cast<void **>(&c->h_out), kStageDoubles * sizeof(double), hipHostMallocDefault);
    }
    if (e == hipSuccess) {
        step = "pinned error word";
        e = hipHostMalloc(reinterpret_cast<void **>(&c->h_err), 64, hipHostMallocDefault);
    }
    if (e == hipSuccess) { step = "clear error word"; e = launch_fill_u32(c->d_err, 64, 0u, c->stream); }
    if (e == hipSuccess) { step = "synchronize"; e = hipStreamSynchronize(c->stream); }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(nullptr, ARA_E_DEVICE, "ctx: %s: %s", step, hipGetErrorString(e));
        dev_free(c->d_err);
        dev_free(c->d_out);
        if (c->h_out) (void)hipHostFree(c->h_out);
        if (c->h_err) (void)hipHostFree(c->h_err);
        delete c;
        return ARA_E_DEVICE;
    }
    *out = c;
    return ARA_OK;
}

extern "C" ara_status ara_ctx_destroy(ara_ctx *c) {
    if (!c) return ARA_E_INVALID_ARG;
    if (c->live > 0) return fail(c, ARA_E_BUSY, "%d handles still alive on this context", c->live);
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    dev_free(c->d_err);
    dev_free(c->d_out);
    if (c->h_out) (void)hipHostFree(c->h_out);
    if (c->h_err) (void)hipHostFree(c->h_err);
    delete c;
    return ARA_OK;
}

extern "C" ara_status ara_ctx_set_stream(ara_ctx *c, void *hip_stream) {
    if (!c) return ARA_E_INVALID_ARG;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return ARA_OK;
}

extern "C" ara_status ara_set_option(ara_ctx *c, int option, int64_t v) {
    if (!c) return ARA_E_INVALID_ARG;
    switch (option) {
    case ARA_OPT_PLACEMENT:
        if (v < ARA_PLACE_AUTO || v > ARA_PLACE_GLOBAL_DENSE) return fail(c, ARA_E_INVALID_ARG, "bad placement %lld", (long long)v);
        c->placement = int(v);
        return ARA_OK;
    case ARA_OPT_BLOCK_THREADS:
        if (v != 0 && v != 256 && v != 512 && v != 1024) return fail(c, ARA_E_INVALID_ARG, "bad block size %lld", (long long)v);
        c->block_threads = int(v);
        return ARA_OK;
    case ARA_OPT_GRID_PER_CU:
        if (v < 0 || v > 64) return fail(c, ARA_E_INVALID_ARG, "bad workgroups per CU %lld", (long long)v);
        c->grid_per_cu = int(v);
        return ARA_OK;
    case ARA_OPT_YET_PACKING:
        if (v != 0 && v != 1) return fail(c, ARA_E_INVALID_ARG, "bad packing flag %lld", (long long)v);
        c->yet_packing = int(v);
        return ARA_OK;
    default:
        return fail(c, ARA_E_INVALID_ARG, "unknown option %d", option);
    }
}

extern "C" ara_status ara_sync(ara_ctx *c) {
    if (!c) return ARA_E_INVALID_ARG;
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    return sync_and_check(c);
}

// ------------------------------------------------------------------ YET
extern "C" ara_status ara_yet_create(ara_ctx *c, const int32_t *ids, int64_t n_events, const int64_t *offs,
                                    int64_t n_trials, int32_t catalog, ara_mem mem, ara_yet **out) {
    if (!c || !out) return ARA_E_INVALID_ARG;
    *out = nullptr;
    if (n_events < 0 || n_trials < 0 || catalog < 1 || catalog > kMaxCatalog || !offs || (n_events > 0 && !ids) ||
        (mem != ARA_MEM_HOST && mem != ARA_MEM_DEVICE))
        return fail(c, ARA_E_INVALID_ARG, "yet: bad sizes or pointers");
    if (mem == ARA_MEM_DEVICE && (reinterpret_cast<uintptr_t>(ids) & 15u))
        return fail(c, ARA_E_INVALID_ARG, "yet: event_ids must be 16-byte aligned");
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    ara_yet *y = new (std::nothrow) ara_yet();
    if (!y) return ARA_E_OOM;
    *y = ara_yet{c, ids, offs, n_events, n_trials, catalog, mem == ARA_MEM_HOST, nullptr};
    if (y->owns) {
        int32_t *di = nullptr;
        int64_t *doff = nullptr;
        ara_status s = dev_alloc(c, &di, size_t(n_events) * 4, "yet ids");
        if (s == ARA_OK) s = dev_alloc(c, &doff, size_t(n_trials + 1) * 8, "yet offsets");
        if (s != ARA_OK) {
            dev_free(di);
            delete y;
            return s;
        }
        hipError_t e = hipMemcpy(di, ids, size_t(n_events) * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(doff, offs, size_t(n_trials + 1) * 8, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            dev_free(di);
            dev_free(doff);
            delete y;
            return hip_fail(c, e, "yet upload");
        }
        y->ids = di;
        y->offs = doff;
    }
    hipError_t e = launch_validate_yet(y->ids, n_events, y->offs, n_trials, catalog, c->d_err, c->stream);
    ara_status s = e == hipSuccess ? sync_and_check(c) : hip_fail(c, e, "validate yet");
    if (s == ARA_OK && c->yet_packing && n_events > 0 && catalog <= kMaxPackedCatalog) {
        s = dev_alloc(c, &y->ids24, yet_packed_bytes(n_events), "packed yet ids");
        if (s == ARA_OK) {
            e = launch_yet_pack(y->ids, n_events, y->ids24, c->stream);
            s = e == hipSuccess ? sync_and_check(c) : hip_fail(c, e, "pack yet");
        }
    }
    if (s != ARA_OK) {
        if (y->owns) {
            dev_free(const_cast<int32_t *>(y->ids));
            dev_free(const_cast<int64_t *>(y->offs));
        }
        dev_free(y->ids24);
        delete y;
        return s;
    }
    c->live++;
    *out = y;
    return ARA_OK;
}

extern "C" ara_status ara_yet_release(ara_yet *y) {
    if (!y) return ARA_E_INVALID_ARG;
    (void)hipSetDevice(y->ctx->device);
    (void)hipStreamSynchronize(y->ctx->stream);
    if (y->owns) {
        dev_free(const_cast<int32_t *>(y->ids));
        dev_free(const_cast<int64_t *>(y->offs));
    }
    dev_free(y->ids24);
    y->ctx->live--;
    delete y;
    return ARA_OK;
}

extern "C" ara_status ara_yet_info(const ara_yet *y, int64_t *n_events, int64_t *n_trials, int32_t *id_bytes) {
    if (!y) return ARA_E_INVALID_ARG;
    if (n_events) *n_events = y->n_events;
    if (n_trials) *n_trials = y->n_trials;
    if (id_bytes) *id_bytes = y->ids24 ? 3 : 4;
    return ARA_OK;
}

// ------------------------------------------------------------------ ELT
static void elt_free(ara_elt *t) {
    if (t->owns_pairs) {
        dev_free(const_cast<int32_t *>(t->pair_ids));
        dev_free(const_cast<double *>(t->pair_losses));
    }
    dev_free(t->dat);
    dev_free(t->seen);
    dev_free(t->d_desc);
    delete t;
}

extern "C" ara_status ara_elt_create(ara_ctx *c, const int32_t *ids, const double *losses, int64_t n_pairs,
                                    int32_t catalog, const ara_elt_terms *terms, ara_precision prec, ara_mem mem,
                                    ara_elt **out) {
    if (!c || !out) return ARA_E_INVALID_ARG;
    *out = nullptr;
    if (n_pairs < 0 || catalog < 1 || catalog > kMaxCatalog || (n_pairs > 0 && (!ids || !losses)) || (prec != ARA_F64 && prec != ARA_F32) ||
        (mem != ARA_MEM_HOST && mem != ARA_MEM_DEVICE))
        return fail(c, ARA_E_INVALID_ARG, "elt: bad sizes, pointers, precision or memory kind");
    if (check_elt_terms(terms) != ARA_OK) return fail(c, ARA_E_BAD_TERMS, "elt: invalid financial terms");
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    ara_elt *t = new (std::nothrow) ara_elt();
    if (!t) return ARA_E_OOM;
    t->ctx = c;
    t->catalog = catalog;
    t->prec = prec;
    t->n_pairs = n_pairs;
    t->pair_ids = ids;
    t->pair_losses = losses;
    t->owns_pairs = mem == ARA_MEM_HOST;
    t->users = 0;
    ara_status s = ARA_OK;
    if (t->owns_pairs) {
        int32_t *di = nullptr;
        double *dl = nullptr;
        s = dev_alloc(c, &di, size_t(n_pairs) * 4, "elt ids");
        if (s == ARA_OK) s = dev_alloc(c, &dl, size_t(n_pairs) * 8, "elt losses");
        t->pair_ids = di;
        t->pair_losses = dl;
        if (s == ARA_OK && n_pairs > 0) {
            hipError_t e = hipMemcpy(di, ids, size_t(n_pairs) * 4, hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(dl, losses, size_t(n_pairs) * 8, hipMemcpyHostToDevice);
            if (e != hipSuccess) s = hip_fail(c, e, "elt upload");
        }
    }
    const size_t vbytes = prec == ARA_F32 ? 4 : 8;
    if (s == ARA_OK) s = dev_alloc(c, &t->dat, size_t(catalog) * vbytes, "elt table");
    if (s == ARA_OK) s = dev_alloc(c, &t->seen, (size_t(catalog) + 31) / 32 * 4, "elt seen bits");
    if (s == ARA_OK) s = dev_alloc(c, &t->d_desc, sizeof(EltDesc), "elt descriptor");
    if (s != ARA_OK) {
        elt_free(t);
        return s;
    }
    EltDesc &d = t->desc;
    d.pair_ids = t->pair_ids;
    d.pair_losses = t->pair_losses;
    d.n_pairs = n_pairs;
    d.dat = t->dat;
    d.seen = t->seen;
    d.f32 = prec == ARA_F32;
    d.identity = terms ? 0 : 1;
    d.fx = terms ? terms->fx : 1.0;
    d.retention = terms ? terms->retention : 0.0;
    d.limit = terms ? terms->limit : INFINITY;
    hipError_t e = hipMemcpy(t->d_desc, &d, sizeof(EltDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_elt_clear(t->d_desc, 1, catalog, c->stream);
    if (e == hipSuccess) e = launch_elt_scatter(t->d_desc, 1, n_pairs, catalog, c->d_err, c->stream);
    s = e == hipSuccess ? sync_and_check(c) : hip_fail(c, e, "elt build");
    if (s != ARA_OK) {
        elt_free(t);
        return s;
    }
    c->live++;
    *out = t;
    return ARA_OK;
}

extern "C" ara_status ara_elt_release(ara_elt *t) {
    if (!t) return ARA_E_INVALID_ARG;
    if (t->users > 0) return fail(t->ctx, ARA_E_BUSY, "elt used by %d live layers", t->users);
    ara_ctx *c = t->ctx;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    elt_free(t);
    c->live--;
    return ARA_OK;
}

// ------------------------------------------------------------------ layer
static ara_status layer_enqueue_filter(ara_layer *L) {
    ara_ctx *c = L->ctx;
    hipError_t e = launch_layer_filter(L->catalog, L->f32, L->terms.occ_retention, L->terms.occ_limit, L->t, c->stream);
    return e == hipSuccess ? ARA_OK : hip_fail(c, e, "layer filter");
}

static ara_status layer_enqueue_build(ara_layer *L, int flags) {
    ara_ctx *c = L->ctx;
    const int n = int(L->elts.size());
    hipError_t e = hipSuccess;
    if ((flags & ARA_BUILD_TABLES) && n > 0) {
        e = launch_elt_clear(L->d_descs, n, L->catalog, c->stream);
        if (e == hipSuccess) e = launch_elt_scatter(L->d_descs, n, L->max_pairs, L->catalog, c->d_err, c->stream);
    }
    if (e == hipSuccess) e = launch_layer_combine(L->d_descs, n, L->catalog, L->f32, 0.0, 0.0, L->t, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "layer build");
    return layer_enqueue_filter(L);
}

static void layer_free(ara_layer *L) {
    dev_free(L->d_descs);
    dev_free(L->t.comb);
    dev_free(L->t.occ);
    dev_free(L->t.bitmap);
    dev_free(L->t.rank);
    dev_free(L->t.rel16);
    dev_free(L->t.base32);
    dev_free(L->t.vals);
    dev_free(L->t.n_flagged);
    delete L;
}

extern "C" ara_status ara_layer_create(ara_ctx *c, ara_elt *const *elts, int32_t n_elts, int32_t catalog,
                                      const ara_layer_terms *terms, ara_layer **out) {
    if (!c || !out) return ARA_E_INVALID_ARG;
    *out = nullptr;
    if (n_elts < 0 || n_elts > kMaxElts || (n_elts > 0 && !elts) || catalog < 1 || catalog > kMaxCatalog) return fail(c, ARA_E_INVALID_ARG, "layer: bad ELT list or catalog");
    if (ara_check_layer_terms(terms) != ARA_OK) return fail(c, ARA_E_BAD_TERMS, "layer: invalid layer terms");
    bool all_f32 = n_elts > 0;
    for (int32_t j = 0; j < n_elts; ++j) {
        if (!elts[j] || elts[j]->ctx != c) return fail(c, ARA_E_INVALID_ARG, "layer: ELT %d is NULL or from another context", j);
        if (elts[j]->catalog != catalog) return fail(c, ARA_E_INVALID_ARG, "layer: ELT %d catalog %d != %d", j, elts[j]->catalog, catalog);
        all_f32 = all_f32 && elts[j]->prec == ARA_F32;
    }
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    ara_layer *L = new (std::nothrow) ara_layer();
    if (!L) return ARA_E_OOM;
    L->ctx = c;
    L->elts.assign(elts, elts + n_elts);
    L->terms = *terms;
    L->catalog = catalog;
    L->f32 = all_f32;
    L->max_pairs = 0;
    std::vector<EltDesc> d(static_cast<size_t>(n_elts));
    for (int32_t j = 0; j < n_elts; ++j) {
        d[size_t(j)] = elts[j]->desc;
        L->max_pairs = std::max(L->max_pairs, elts[j]->n_pairs);
    }
    const int32_t nblk = bitmap_blocks(catalog);
    L->t.nblk = nblk;
    ara_status s = dev_alloc(c, &L->d_descs, sizeof(EltDesc) * size_t(n_elts), "layer descriptors");
    if (s == ARA_OK) s = dev_alloc(c, &L->t.comb, size_t(catalog) * (all_f32 ? 4 : 8), "layer combined table");
    if (s == ARA_OK) s = dev_alloc(c, &L->t.occ, size_t(catalog) * 8, "layer occurrence table");
    if (s == ARA_OK) s = dev_alloc(c, &L->t.bitmap, size_t(nblk) * 16, "layer bitmap");
    if (s == ARA_OK) s = dev_alloc(c, &L->t.rank, size_t(nblk) * 4, "layer ranks");
    if (s == ARA_OK) s = dev_alloc(c, &L->t.rel16, align16(size_t(nblk) * 2), "layer relative ranks");
    if (s == ARA_OK) s = dev_alloc(c, &L->t.base32, align16(size_t(bitmap_supers(nblk)) * 4), "layer rank bases");
    if (s == ARA_OK) s = dev_alloc(c, &L->t.vals, size_t(catalog) * 8, "layer values");
    if (s == ARA_OK) s = dev_alloc(c, &L->t.n_flagged, 16, "layer count");
    if (s == ARA_OK && n_elts > 0) {
        hipError_t e = hipMemcpy(L->d_descs, d.data(), sizeof(EltDesc) * size_t(n_elts), hipMemcpyHostToDevice);
        if (e != hipSuccess) s = hip_fail(c, e, "layer descriptors upload");
    }
    if (s == ARA_OK) s = layer_enqueue_build(L, 0);
    if (s != ARA_OK) {
        layer_free(L);
        return s;
    }
    for (auto *t : L->elts) t->users++;
    c->live++;
    *out = L;
    return ARA_OK;
}

extern "C" ara_status ara_layer_set_terms(ara_ctx *c, ara_layer *L, const ara_layer_terms *terms) {
    if (!c || !L || L->ctx != c) return ARA_E_INVALID_ARG;
    if (ara_check_layer_terms(terms) != ARA_OK) return fail(c, ARA_E_BAD_TERMS, "layer: invalid layer terms");
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    L->terms = *terms;
    return layer_enqueue_filter(L);
}

extern "C" ara_status ara_layer_build(ara_ctx *c, ara_layer *L, int flags) {
    if (!c || !L || L->ctx != c || (flags & ~ARA_BUILD_TABLES)) return ARA_E_INVALID_ARG;
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    return layer_enqueue_build(L, flags);
}

extern "C" ara_status ara_layer_stats(ara_ctx *c, const ara_layer *L, int64_t *n_flagged, int32_t *placement,
                                     int64_t *lds_bytes) {
    if (!c || !L || L->ctx != c) return ARA_E_INVALID_ARG;
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    TrialLaunch tl{};
    ara_status s = plan_trial(c, L, 1 << 20, tl);
    if (s != ARA_OK) return s;
    if (placement) *placement = tl.placement;
    if (lds_bytes) *lds_bytes = int64_t(tl.lds_bytes);
    if (n_flagged) {
        HIP_OR_RETURN(c, hipMemcpyAsync(c->h_err + 1, L->t.n_flagged, 4, hipMemcpyDeviceToHost, c->stream), "read count");
        HIP_OR_RETURN(c, hipStreamSynchronize(c->stream), "stream synchronize");
        *n_flagged = int64_t(c->h_err[1]);
    }
    return ARA_OK;
}

extern "C" ara_status ara_layer_release(ara_layer *L) {
    if (!L) return ARA_E_INVALID_ARG;
    ara_ctx *c = L->ctx;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto *t : L->elts) t->users--;
    layer_free(L);
    c->live--;
    return ARA_OK;
}

// ------------------------------------------------------------------ analysis
static TrialArgs trial_args(const ara_yet *y, const ara_layer *L, int64_t t0, int64_t t1, double *ylt) {
    TrialArgs a{};
    if (y) {
        a.ids = y->ids;
        a.ids24 = y->ids24;
        a.n_events = y->n_events;
        a.offs = y->offs;
    }
    a.t_begin = t0;
    a.t_end = t1;
    a.catalog = L->catalog;
    a.nblk = L->t.nblk;
    a.comb = L->t.comb;
    a.occ = L->t.occ;
    a.bitmap = L->t.bitmap;
    a.rel16 = L->t.rel16;
    a.base32 = L->t.base32;
    a.vals = L->t.vals;
    a.occ_r = L->terms.occ_retention;
    a.occ_l = L->terms.occ_limit;
    a.agg_r = L->terms.agg_retention;
    a.agg_l = L->terms.agg_limit;
    a.ylt = ylt;
    a.err = L->ctx->d_err;
    return a;
}

static ara_status check_analysis(ara_ctx *c, const ara_yet *y, const ara_layer *L, int64_t t0, int64_t t1) {
    if (!c || !y || !L || y->ctx != c || L->ctx != c) return ARA_E_INVALID_ARG;
    if (t0 < 0 || t1 < t0 || t1 > y->n_trials) return fail(c, ARA_E_INVALID_ARG, "trial range [%lld, %lld) outside [0, %lld)",
                                                           (long long)t0, (long long)t1, (long long)y->n_trials);
    if (y->catalog != L->catalog) return fail(c, ARA_E_INVALID_ARG, "YET catalog %d != layer catalog %d", y->catalog, L->catalog);
    return ARA_OK;
}

extern "C" ara_status ara_analyze(ara_ctx *c, const ara_yet *y, const ara_layer *L, int64_t t0, int64_t t1, double *ylt,
                                 ara_mem mem) {
    ara_status s = check_analysis(c, y, L, t0, t1);
    if (s != ARA_OK) return s;
    if ((t1 > t0 && !ylt) || (mem != ARA_MEM_HOST && mem != ARA_MEM_DEVICE)) return fail(c, ARA_E_INVALID_ARG, "analyze: bad output");
    if (t1 == t0) return ARA_OK;
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    TrialLaunch tl{};
    s = plan_trial(c, L, t1 - t0, tl);
    if (s != ARA_OK) return s;
    double *dst = ylt;
    if (mem == ARA_MEM_HOST) {
        s = dev_alloc(c, &dst, size_t(t1 - t0) * 8, "ylt staging");
        if (s != ARA_OK) return s;
    }
    // trial indices inside a launch are 32-bit: split very long ranges
    constexpr int64_t kMaxTrialsPerLaunch = int64_t(1) << 30;
    hipError_t e = hipSuccess;
    for (int64_t tb = t0; tb < t1 && e == hipSuccess; tb += kMaxTrialsPerLaunch) {
        const int64_t te = std::min(t1, tb + kMaxTrialsPerLaunch);
        TrialArgs a = trial_args(y, L, tb, te, dst + (tb - t0));
        a.qcap = tl.qcap;
        e = launch_trial_ylt(a, tl, c->stream);
    }
    if (e != hipSuccess) s = hip_fail(c, e, "trial kernel");
    if (s == ARA_OK && mem == ARA_MEM_HOST) {
        e = hipMemcpyAsync(ylt, dst, size_t(t1 - t0) * 8, hipMemcpyDeviceToHost, c->stream);
        s = e == hipSuccess ? sync_and_check(c) : hip_fail(c, e, "ylt download");
    }
    if (mem == ARA_MEM_HOST) {
        (void)hipStreamSynchronize(c->stream);
        dev_free(dst);
    }
    return s;
}

extern "C" ara_status ara_analyze_events(ara_ctx *c, const ara_yet *y, const ara_layer *L, int64_t t0, int64_t t1,
                                        double *ylt, double *g, double *o, double *cu, double *ce, ara_mem mem) {
    ara_status s = check_analysis(c, y, L, t0, t1);
    if (s != ARA_OK) return s;
    if (mem != ARA_MEM_HOST && mem != ARA_MEM_DEVICE) return fail(c, ARA_E_INVALID_ARG, "analyze_events: bad memory kind");
    if (t1 == t0) return ARA_OK;
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    // number of occurrences in the range, from the device offsets
    HIP_OR_RETURN(c, hipMemcpyAsync(c->h_out, y->offs + t0, 8, hipMemcpyDeviceToHost, c->stream), "read offsets");
    HIP_OR_RETURN(c, hipMemcpyAsync(c->h_out + 1, y->offs + t1, 8, hipMemcpyDeviceToHost, c->stream), "read offsets");
    HIP_OR_RETURN(c, hipStreamSynchronize(c->stream), "stream synchronize");
    int64_t e0, e1;
    std::memcpy(&e0, c->h_out, 8);
    std::memcpy(&e1, c->h_out + 1, 8);
    const int64_t nev = e1 - e0;
    if (nev < 0) return fail(c, ARA_E_BAD_OFFSETS, "analyze_events: offsets decrease");
    double *host[5] = {ylt, g, o, cu, ce};
    double *dev[5] = {ylt, g, o, cu, ce};
    const size_t len[5] = {size_t(t1 - t0), size_t(nev), size_t(nev), size_t(nev), size_t(nev)};
    if (mem == ARA_MEM_HOST) {
        for (int k = 0; k < 5; ++k) {
            dev[k] = nullptr;
            if (host[k] && len[k] > 0) {
                s = dev_alloc(c, &dev[k], len[k] * 8, "event output staging");
                if (s != ARA_OK) {
                    for (int j = 0; j < k; ++j) dev_free(dev[j]);
                    return s;
                }
            }
        }
    }
    TrialArgs a = trial_args(y, L, t0, t1, dev[0]);
    a.ev_gross = dev[1];
    a.ev_occ = dev[2];
    a.ev_cum = dev[3];
    a.ev_ceded = dev[4];
    const int64_t waves = t1 - t0;
    const int grid = int(std::min<int64_t>(int64_t(c->n_cu) * 8, (waves + 3) / 4));
    hipError_t e = launch_trial_events(a, L->f32, std::max(grid, 1), c->stream);
    s = e == hipSuccess ? ARA_OK : hip_fail(c, e, "event kernel");
    if (mem == ARA_MEM_HOST) {
        for (int k = 0; k < 5 && s == ARA_OK; ++k)
            if (dev[k]) {
                e = hipMemcpyAsync(host[k], dev[k], len[k] * 8, hipMemcpyDeviceToHost, c->stream);
                if (e != hipSuccess) s = hip_fail(c, e, "event output download");
            }
        ara_status s2 = sync_and_check(c);
        if (s == ARA_OK) s = s2;
        for (int k = 0; k < 5; ++k) dev_free(dev[k]);
    }
    return s;
}

extern "C" ara_status ara_lookup(ara_ctx *c, const ara_layer *L, const int32_t *ids, int64_t n, double *g, double *o,
                                ara_mem mem) {
    if (!c || !L || L->ctx != c || n < 0 || (n > 0 && !ids) || (mem != ARA_MEM_HOST && mem != ARA_MEM_DEVICE))
        return ARA_E_INVALID_ARG;
    if (n == 0) return ARA_OK;
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    TrialLaunch tl{};
    ara_status s = plan_trial(c, L, 1 << 20, tl);
    if (s != ARA_OK) return s;
    const int32_t *di = ids;
    double *dg = g, *dout = o;
    if (mem == ARA_MEM_HOST) {
        int32_t *ti = nullptr;
        s = dev_alloc(c, &ti, size_t(n) * 4, "lookup ids");
        if (s == ARA_OK) s = dev_alloc(c, &dg, size_t(n) * 8, "lookup gross");
        if (s == ARA_OK) s = dev_alloc(c, &dout, size_t(n) * 8, "lookup occ");
        if (s == ARA_OK) {
            hipError_t e = hipMemcpy(ti, ids, size_t(n) * 4, hipMemcpyHostToDevice);
            if (e != hipSuccess) s = hip_fail(c, e, "lookup upload");
        }
        di = ti;
        if (s != ARA_OK) {
            dev_free(ti);
            dev_free(dg);
            dev_free(dout);
            return s;
        }
    }
    hipError_t e = launch_lookup(trial_args(nullptr, L, 0, 0, nullptr), tl, di, n,
                                 mem == ARA_MEM_HOST ? dg : g, mem == ARA_MEM_HOST ? dout : o, c->stream);
    s = e == hipSuccess ? ARA_OK : hip_fail(c, e, "lookup kernel");
    if (mem == ARA_MEM_HOST) {
        if (s == ARA_OK && g) {
            e = hipMemcpyAsync(g, dg, size_t(n) * 8, hipMemcpyDeviceToHost, c->stream);
            if (e != hipSuccess) s = hip_fail(c, e, "lookup download");
        }
        if (s == ARA_OK && o) {
            e = hipMemcpyAsync(o, dout, size_t(n) * 8, hipMemcpyDeviceToHost, c->stream);
            if (e != hipSuccess) s = hip_fail(c, e, "lookup download");
        }
        ara_status s2 = sync_and_check(c);
        if (s == ARA_OK) s = s2;
        dev_free(const_cast<int32_t *>(di));
        dev_free(dg);
        dev_free(dout);
    }
    return s;
}

// ------------------------------------------------------------------ order statistics
extern "C" ara_status ara_sort_workspace_size(int64_t n, size_t *bytes) {
    if (!bytes || n < 0) return ARA_E_INVALID_ARG;
    *bytes = sort_workspace_bytes(n);
    return ARA_OK;
}

static ara_status workspace_for(ara_ctx *c, int64_t n, void *ws, size_t ws_bytes, void **use, bool *owned) {
    *owned = false;
    *use = ws;
    const size_t need = sort_workspace_bytes(n);
    if (ws) {
        if (ws_bytes < need) return fail(c, ARA_E_INVALID_ARG, "workspace %zu bytes < %zu needed", ws_bytes, need);
        return ARA_OK;
    }
    ara_status s = dev_alloc(c, use, need, "sort workspace");
    *owned = s == ARA_OK;
    return s;
}

extern "C" ara_status ara_sort_desc(ara_ctx *c, const double *in, int64_t n, double *out, void *ws, size_t ws_bytes) {
    if (!c || n < 0 || (n > 0 && (!in || !out))) return ARA_E_INVALID_ARG;
    if (n == 0) return ARA_OK;
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    void *w = nullptr;
    bool owned = false;
    ara_status s = workspace_for(c, n, ws, ws_bytes, &w, &owned);
    if (s != ARA_OK) return s;
    hipError_t e = launch_sort_desc_keys(in, n, w, c->stream);
    if (e == hipSuccess) e = launch_sort_decode(w, n, out, c->stream);
    s = e == hipSuccess ? ARA_OK : hip_fail(c, e, "sort");
    if (owned) {
        (void)hipStreamSynchronize(c->stream);
        dev_free(w);
    }
    return s;
}

extern "C" ara_status ara_risk_measures(ara_ctx *c, const double *ylt, int64_t n, ara_mem mem, const double *rps,
                                       int32_t n_rp, double *pml, double *tvar, void *ws, size_t ws_bytes) {
    if (!c || n < 0 || n_rp < 0 || (n_rp > 0 && (!rps || !pml || !tvar)) || (mem != ARA_MEM_HOST && mem != ARA_MEM_DEVICE))
        return ARA_E_INVALID_ARG;
    if (n == 0) return fail(c, ARA_E_EMPTY, "risk measures of an empty YLT");
    if (!ylt) return ARA_E_INVALID_ARG;
    if (size_t(n_rp) * 2 > kStageDoubles) return fail(c, ARA_E_INVALID_ARG, "at most %zu return periods", kStageDoubles / 2);
    std::vector<int64_t> ks(static_cast<size_t>(n_rp));
    for (int32_t i = 0; i < n_rp; ++i)
        if (ara_return_period_rank(n, rps[i], &ks[size_t(i)]) != ARA_OK)
            return fail(c, ARA_E_INVALID_ARG, "return period %g invalid (must be >= 1)", rps[i]);
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    const double *dy = ylt;
    double *tmp = nullptr;
    ara_status s = ARA_OK;
    if (mem == ARA_MEM_HOST) {
        s = dev_alloc(c, &tmp, size_t(n) * 8, "ylt upload");
        if (s != ARA_OK) return s;
        hipError_t e = hipMemcpy(tmp, ylt, size_t(n) * 8, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            dev_free(tmp);
            return hip_fail(c, e, "ylt upload");
        }
        dy = tmp;
    }
    void *w = nullptr;
    bool owned = false;
    s = workspace_for(c, n, ws, ws_bytes, &w, &owned);
    if (s == ARA_OK) {
        hipError_t e = launch_sort_desc_keys(dy, n, w, c->stream);
        if (e == hipSuccess && n_rp > 0) e = launch_risk(w, n, ks.data(), n_rp, c->d_out, c->stream);
        if (e == hipSuccess && n_rp > 0)
            e = hipMemcpyAsync(c->h_out, c->d_out, size_t(2 * n_rp) * 8, hipMemcpyDeviceToHost, c->stream);
        s = e == hipSuccess ? sync_and_check(c) : hip_fail(c, e, "risk measures");
        if (s == ARA_OK) {
            for (int32_t base = 0; base < n_rp; base += 16) {
                const int32_t m = std::min<int32_t>(16, n_rp - base);
                for (int32_t i = 0; i < m; ++i) {
                    pml[base + i] = c->h_out[2 * base + i];
                    tvar[base + i] = c->h_out[2 * base + m + i];
                }
            }
        }
    }
    if (owned || tmp) (void)hipStreamSynchronize(c->stream);
    if (owned) dev_free(w);
    dev_free(tmp);
    return s;
}
