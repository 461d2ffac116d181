// C-ABI of libara: handle lifetimes, argument validation, table placement and the
// launches of the analysis path.  Declarations and contracts: include/ara.h.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ara_internal.h"

using namespace ara;

struct ara_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int n_cu = 0;
    int lds_max = 0;
    uint32_t *d_err = nullptr;       // device error bits (word 0), then d_out
    double *d_out = nullptr;         // small device result staging
    double *h_out = nullptr;         // pinned host mirror of d_out
    uint32_t *h_err = nullptr;       // pinned host error word
    uint32_t *h_plan = nullptr;      // pinned copy of a radix sort's pass plan
    void *scratch = nullptr;         // device address of this device's `scratch` array
    int placement = ARA_PLACE_AUTO;
    int block_threads = 0;           // 0 = automatic
    int grid_per_cu = 0;             // 0 = automatic
    int yet_packing = 1;             // keep a packed copy of YET IDs where they fit 24 bits
    int yet_binning = 1;             // keep a catalog-binned copy of YET IDs where it applies
    int yet_run_bytes = 4;           // bytes per run start of the binned copy (3 or 4)
    int trial_mode = 0;              // 0 = by trial length, 1 = wave per trial, 2 = lane per trial
    std::vector<hipEvent_t> k_ev;    // ARA_OPT_KERNEL_TIMING: a ring of (start, stop) event pairs
    int64_t k_count = 0;             // trial kernels timed since the option was set
    std::map<std::string, std::pair<int64_t, bool>> tuned;   // batch shape -> (events per item, interleave)
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
    // catalog-binned copy (owned), or null ids16
    uint16_t *ids16 = nullptr;
    uint32_t *boff = nullptr;     // run starts: n_bins rows of `stride` entries, 4 bytes each,
    uint8_t *boff24 = nullptr;    // or 3 bytes each (one of the two)
    int64_t *region = nullptr;    // n_bins + 1 element offsets
    int64_t stride = 0;
    int32_t n_bins = 0;
    int64_t copy_bytes = 0;       // device memory of the packed or binned copy
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
    uint64_t terms_gen = 0;   // incremented by every ara_layer_set_terms
    // t.rank, rel16, base32, n_flagged and vals match the current tables: rebuilds
    // leave them to the first call whose kernel reads them (layer_ranks)
    mutable bool ranks_ready = false;
};

static constexpr size_t kStageDoubles = 512;   // 2 x 256 return periods
static constexpr int64_t kMaxTimedLaunches = 4096;   // ARA_OPT_KERNEL_TIMING ring size
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

constexpr size_t kErrBytes = 16;   // the error word and spare words before the result staging

static ara_status err_bits_status(uint32_t bits) {
    if (bits & ERR_ID_RANGE) return ARA_E_EVENT_ID_RANGE;
    if (bits & ERR_OFFSETS) return ARA_E_BAD_OFFSETS;
    if (bits & ERR_LOSS) return ARA_E_BAD_LOSS;
    if (bits & ERR_DUP) return ARA_E_DUP_EVENT;
    return ARA_OK;
}

// Waits for the context stream, then reads and clears the device error word.  With
// `wide`, the ERR_BIN_WIDE bit (not an input error) is returned there.  `copied`: the
// caller has already queued the error word's copy to h_err.
static ara_status sync_and_check(ara_ctx *c, bool *wide = nullptr, bool copied = false) {
    if (!copied)
        HIP_OR_RETURN(c, hipMemcpyAsync(c->h_err, c->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream),
                      "read error word");
    HIP_OR_RETURN(c, hipStreamSynchronize(c->stream), "stream synchronize");
    uint32_t bits = *c->h_err;
    if (bits) {
        HIP_OR_RETURN(c, launch_fill_u32(c->d_err, 1, 0u, c->stream), "clear error word");
        HIP_OR_RETURN(c, hipStreamSynchronize(c->stream), "stream synchronize");
        if (wide) *wide = (bits & ERR_BIN_WIDE) != 0;
        bits &= ~ERR_BIN_WIDE;
        if (bits) {
            ara_status s = err_bits_status(bits);
            return fail(c, s, "device-detected input error (bits 0x%x): %s", bits, ara_status_str(s));
        }
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
// mean_len: mean occurrences per trial of the YET (decides lane or wave per trial);
// tiles: kNoTiles for paths without a tiled kernel (a forced tiled placement runs them
// with the LDS bitmap), else whether the YET has a catalog-binned copy.
enum { kNoTiles = -1 };
static ara_status plan_trial(ara_ctx *c, const ara_layer *L, int64_t n_trials, double mean_len, TrialLaunch &tl,
                             int tiles = kNoTiles) {
    int pl = c->placement;
    const bool binned = tiles > 0;
    if (pl == ARA_PLACE_LDS_TILES && tiles == kNoTiles) pl = ARA_PLACE_LDS_BITMAP;
    const int64_t dense = int64_t(L->catalog) * 8;
    const int block_bitmap = c->block_threads ? c->block_threads : 1024;
    const int qcap = bitmap_qcap(L->catalog, block_bitmap / 64, c->lds_max);
    if (pl == ARA_PLACE_AUTO) {
        if (dense <= c->lds_max) pl = ARA_PLACE_LDS_DENSE;
        else if (binned && c->lds_max >= kLdsMaxBytes) pl = ARA_PLACE_LDS_TILES;
        else if (qcap > 0) pl = ARA_PLACE_LDS_BITMAP;
        else pl = ARA_PLACE_GLOBAL_DENSE;
    }
    if (pl == ARA_PLACE_LDS_TILES) {
        if (!binned || c->lds_max < kLdsMaxBytes)
            return fail(c, ARA_E_UNSUPPORTED, "tiled placement needs a YET with a binned copy and %d bytes of LDS",
                        kLdsMaxBytes);
        tl.placement = pl;
        tl.f32 = L->f32;
        tl.lds_bytes = size_t(kLdsMaxBytes);
        tl.qcap = 0;
        tl.lane = false;
        tl.block = kTiledWaves * 64;
        tl.grid = int(std::max<int64_t>(1, std::min<int64_t>(c->n_cu, (n_trials + 63) / 64)));
        return ARA_OK;
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
    tl.lane = pl != ARA_PLACE_LDS_BITMAP &&
              (c->trial_mode == 2 || (c->trial_mode == 0 && mean_len <= double(kLaneModeMaxMean)));
    tl.block = c->block_threads ? c->block_threads : (pl == ARA_PLACE_GLOBAL_DENSE || tl.lane ? 256 : 1024);
    int per_cu = c->grid_per_cu;
    if (per_cu == 0) {
        const int by_threads = 2048 / tl.block;
        const int64_t lds_all = pl == ARA_PLACE_LDS_BITMAP ? int64_t(kLdsMaxBytes) : lds;   // static LDS = all of it
        const int by_lds = lds_all > 0 ? int(c->lds_max / lds_all) : by_threads;
        per_cu = std::max(1, std::min(by_threads, by_lds));
    }
    int64_t grid = int64_t(c->n_cu) * per_cu;
    const int64_t tpb = tl.lane ? tl.block : tl.block / 64;   // trials in flight per workgroup
    grid = std::min<int64_t>(grid, std::max<int64_t>(1, (n_trials + tpb - 1) / tpb));
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
// Sort workspace of ara_risk_measures_noalloc: one file-scope device array, so
// that the call allocates nothing.  Every GPU the library runs on holds its own
// copy until the process ends.  In host code `scratch` only names the array; its
// device address on each device comes from hipGetSymbolAddress, taken once per
// device when the first context is created there, and is what kernels receive.
static_assert(ARA_NOALLOC_MAX_N > 0, "maximum YLT length of the allocation-free call");
constexpr size_t kScratchBytes = ARA_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kScratchDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_addr[kScratchDevices];

// Device address of `scratch` on `device`, which must be the current device.
static hipError_t scratch_address(int device, void **out) {
    if (device < 0 || device >= kScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_addr[device] = p;
    }
    *out = g_scratch_addr[device];
    return hipSuccess;
}

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
    if (e == hipSuccess) { step = "scratch address"; e = scratch_address(device, &c->scratch); }
    // the error word (and a spare word) followed by the result staging, on the device and
    // pinned on the host, so one copy brings back results and error bits together
    const size_t blk = kErrBytes + kStageDoubles * sizeof(double);
    if (e == hipSuccess) { step = "error word and result staging"; e = hipMalloc(&c->d_err, blk); }
    if (e == hipSuccess) c->d_out = reinterpret_cast<double *>(reinterpret_cast<char *>(c->d_err) + kErrBytes);
    if (e == hipSuccess) {
        step = "pinned error word and staging";
        e = hipHostMalloc(reinterpret_cast<void **>(&c->h_err), blk, hipHostMallocDefault);
    }
    if (e == hipSuccess) c->h_out = reinterpret_cast<double *>(reinterpret_cast<char *>(c->h_err) + kErrBytes);
    if (e == hipSuccess) {
        step = "pinned sort plan";
        e = hipHostMalloc(reinterpret_cast<void **>(&c->h_plan), 32 * sizeof(uint32_t), hipHostMallocDefault);
    }
    if (e == hipSuccess) { step = "clear error word"; e = launch_fill_u32(c->d_err, kErrBytes / 4, 0u, c->stream); }
    if (e == hipSuccess) { step = "synchronize"; e = hipStreamSynchronize(c->stream); }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(nullptr, ARA_E_DEVICE, "ctx: %s: %s", step, hipGetErrorString(e));
        dev_free(c->d_err);
        if (c->h_err) (void)hipHostFree(c->h_err);
        if (c->h_plan) (void)hipHostFree(c->h_plan);
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
    dev_free(c->d_err);   // with d_out
    for (hipEvent_t ev : c->k_ev) (void)hipEventDestroy(ev);
    if (c->h_err) (void)hipHostFree(c->h_err);   // with h_out
    if (c->h_plan) (void)hipHostFree(c->h_plan);
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
        if (v < ARA_PLACE_AUTO || v > ARA_PLACE_LDS_TILES) return fail(c, ARA_E_INVALID_ARG, "bad placement %lld", (long long)v);
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
    case ARA_OPT_TRIAL_MODE:
        if (v < 0 || v > 2) return fail(c, ARA_E_INVALID_ARG, "bad trial mode %lld", (long long)v);
        c->trial_mode = int(v);
        return ARA_OK;
    case ARA_OPT_YET_PACKING:
        if (v != 0 && v != 1) return fail(c, ARA_E_INVALID_ARG, "bad packing flag %lld", (long long)v);
        c->yet_packing = int(v);
        return ARA_OK;
    case ARA_OPT_YET_BINNING:
        if (v != 0 && v != 1) return fail(c, ARA_E_INVALID_ARG, "bad binning flag %lld", (long long)v);
        c->yet_binning = int(v);
        return ARA_OK;
    case ARA_OPT_YET_RUN_BYTES:
        if (v != 3 && v != 4) return fail(c, ARA_E_INVALID_ARG, "bad run start size %lld", (long long)v);
        c->yet_run_bytes = int(v);
        return ARA_OK;
    case ARA_OPT_KERNEL_TIMING: {
        if (v < 0 || v > kMaxTimedLaunches) return fail(c, ARA_E_INVALID_ARG, "bad timing ring size %lld", (long long)v);
        HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
        (void)hipStreamSynchronize(c->stream);
        for (hipEvent_t ev : c->k_ev) (void)hipEventDestroy(ev);
        c->k_ev.clear();
        c->k_count = 0;
        for (int64_t i = 0; i < 2 * v; ++i) {
            hipEvent_t ev = nullptr;
            const hipError_t e = hipEventCreate(&ev);
            if (e != hipSuccess) {
                for (hipEvent_t x : c->k_ev) (void)hipEventDestroy(x);
                c->k_ev.clear();
                return hip_fail(c, e, "timing event");
            }
            c->k_ev.push_back(ev);
        }
        return ARA_OK;
    }
    default:
        return fail(c, ARA_E_INVALID_ARG, "unknown option %d", option);
    }
}

extern "C" ara_status ara_kernel_ms(ara_ctx *c, float *ms) {
    if (!c || !ms) return ARA_E_INVALID_ARG;
    if (c->k_ev.empty() || c->k_count == 0) return fail(c, ARA_E_INVALID_ARG, "no trial kernel timed since timing was set");
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    const int64_t n = int64_t(c->k_ev.size() / 2), m = std::min(c->k_count, n);
    double sum = 0.0;
    for (int64_t k = c->k_count - m; k < c->k_count; ++k) {
        const size_t i = size_t(k % n);
        float one = 0.0f;
        HIP_OR_RETURN(c, hipEventSynchronize(c->k_ev[2 * i + 1]), "timing event");
        HIP_OR_RETURN(c, hipEventElapsedTime(&one, c->k_ev[2 * i], c->k_ev[2 * i + 1]), "timing event");
        sum += double(one);
    }
    *ms = float(sum / double(m));
    return ARA_OK;
}

extern "C" ara_status ara_sync(ara_ctx *c) {
    if (!c) return ARA_E_INVALID_ARG;
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    return sync_and_check(c);
}

// ------------------------------------------------------------------ YET
static void yet_free_binned(ara_yet *y) {
    dev_free(y->ids16);
    dev_free(y->boff);
    dev_free(y->boff24);
    dev_free(y->region);
    y->ids16 = nullptr;
    y->boff = nullptr;
    y->boff24 = nullptr;
    y->region = nullptr;
    y->n_bins = 0;
}

// Whether a YET of these sizes gets a catalog-binned copy (see ara_yet_create).
static bool yet_binning_applies(const ara_ctx *c, const ara_yet *y) {
    const int32_t nb = catalog_bins(y->catalog);
    const int64_t n = y->n_trials;
    return c->yet_binning && y->n_events > 0 && n > 0 && int64_t(y->catalog) * 8 > int64_t(c->lds_max) &&
           y->catalog <= kMaxPackedCatalog && nb <= kMaxBins && (n + 1 + 4095) / 4096 <= 65535 &&
           4.0 * double(nb) * double(n) <= 0.25 * 2.0 * double(y->n_events);
}

// Builds the catalog-binned copy when it applies; the YET is usable without it, so
// running out of device memory only skips it.  Its count pass checks the offsets and
// every event ID: *ids_checked tells whether it ran.  A YET of fewer than 2^31
// occurrences has fewer than that in every bin: its copy is then sized from the
// occurrence count (each region rounded up to 8 elements), the region starts are
// computed on the device and the passes run back to back, with one wait at the end
// (a bad ID or offset found by the count pass stops the later passes on the device).
// Larger YETs read the bins' lengths back first to check them.  Asked for 3-byte run
// starts, a one-wait build of at most 64 bins writes them; if a bin turns out to hold
// 2^24 occurrences or more (flagged on the device) it is built again with 4-byte ones.
static ara_status yet_build_binned(ara_ctx *c, ara_yet *y, bool *ids_checked) {
    const int32_t nb = catalog_bins(y->catalog);
    const int64_t n = y->n_trials;
    *ids_checked = false;
    if (!yet_binning_applies(c, y)) return ARA_OK;
    y->stride = (n + 2 + 7) & ~int64_t(7);   // see ara_yet: a multiple of 8, at least n + 2
    const bool one_wait = y->n_events < (int64_t(1) << 31);
    // 3-byte run starts when asked for, unless a bin turns out too long for them
    bool b24 = c->yet_run_bytes == 3 && one_wait && nb <= 64;
    uint32_t *sums = nullptr;
    size_t ids16_bytes = size_t(y->n_events + 8 * int64_t(nb)) * 2 + 16;
    ara_status s = dev_alloc(c, &sums, bin_offsets_scratch_words(n, nb) * 4, "binned yet scan");
    if (s == ARA_OK) s = dev_alloc(c, &y->region, size_t(nb + 1) * 8, "binned yet regions");
    if (s == ARA_OK && one_wait) s = dev_alloc(c, &y->ids16, ids16_bytes, "binned yet ids");
    while (s == ARA_OK) {
        // 3-byte form: 16 bytes of slack after the last row (the tiled kernel reads the
        // aligned words around an entry, up to 2 bytes past its row)
        if (b24) s = dev_alloc(c, &y->boff24, size_t(nb) * size_t(y->stride) * 3 + 16, "binned yet run starts");
        else s = dev_alloc(c, &y->boff, size_t(nb) * size_t(y->stride) * 4, "binned yet run starts");
        if (s != ARA_OK) break;
        const RunStarts r{y->boff, y->boff24, y->stride};
        hipError_t e = launch_bin_offsets(y->ids, y->offs, y->n_events, n, nb, r, y->catalog, sums, c->d_err,
                                          c->stream);
        if (e == hipSuccess) e = launch_bin_regions(r, n, nb, y->region, c->d_err, c->stream);
        if (one_wait) {
            if (e == hipSuccess)
                e = launch_bin_scatter(y->ids, y->offs, y->n_events, n, nb, r, y->region, y->ids16, c->d_err, c->stream);
            bool wide = false;
            s = e == hipSuccess ? sync_and_check(c, &wide) : hip_fail(c, e, "binned yet");
            *ids_checked = e == hipSuccess;   // an ID outside the catalog shows in s
            if (s == ARA_OK && wide) {   // a bin of 2^24 occurrences or more: again with 4-byte run starts
                dev_free(y->boff24);
                y->boff24 = nullptr;
                b24 = false;
                continue;
            }
            break;
        }
        std::vector<uint32_t> len(static_cast<size_t>(nb));
        int64_t total = 0;
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(len.data(), 4, y->boff + n, size_t(y->stride) * 4, 4, size_t(nb),
                                 hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(&total, y->region + nb, 8, hipMemcpyDeviceToHost, c->stream);
        s = e == hipSuccess ? sync_and_check(c) : hip_fail(c, e, "binned yet offsets");
        *ids_checked = e == hipSuccess;
        bool fits = true;
        for (int32_t b = 0; s == ARA_OK && b < nb; ++b) fits = fits && len[size_t(b)] < (1u << 31);
        if (s == ARA_OK && !fits) {
            dev_free(sums);
            yet_free_binned(y);
            return ARA_OK;
        }
        ids16_bytes = size_t(total) * 2 + 16;
        if (s == ARA_OK) s = dev_alloc(c, &y->ids16, ids16_bytes, "binned yet ids");
        if (s == ARA_OK) {
            e = launch_bin_scatter(y->ids, y->offs, y->n_events, n, nb, r, y->region, y->ids16, c->d_err, c->stream);
            s = e == hipSuccess ? sync_and_check(c) : hip_fail(c, e, "binned yet scatter");
        }
        break;
    }
    dev_free(sums);
    if (s == ARA_OK) {
        y->n_bins = nb;
        y->copy_bytes = int64_t(ids16_bytes) + int64_t(nb + 1) * 8 + int64_t(nb) * y->stride * (y->boff24 ? 3 : 4) +
                        (y->boff24 ? 16 : 0);
        return ARA_OK;
    }
    yet_free_binned(y);
    if (s == ARA_E_OOM) {
        c->msg.clear();
        return ARA_OK;
    }
    return s;
}

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
    // the binned copy's count pass checks the offsets and IDs; without it (or if it is
    // skipped before that pass) the check runs on its own.  The binned copy serves the
    // tiled kernel; the packed copy the kernels that stream a whole trial's IDs.  A YET
    // keeps one of them: with a binned copy the others stream the int32 IDs as given
    bool checked = false;
    ara_status s = yet_binning_applies(c, y) ? yet_build_binned(c, y, &checked) : ARA_OK;
    hipError_t e = hipSuccess;
    if (s == ARA_OK && !checked) {
        e = launch_validate_yet(y->ids, n_events, y->offs, n_trials, catalog, c->d_err, c->stream, true);
        s = e == hipSuccess ? sync_and_check(c) : hip_fail(c, e, "validate yet");
    }
    if (s == ARA_OK && !y->ids16 && c->yet_packing && n_events > 0 && catalog <= kMaxPackedCatalog) {
        s = dev_alloc(c, &y->ids24, yet_packed_bytes(n_events), "packed yet ids");
        if (s == ARA_OK) {
            y->copy_bytes = int64_t(yet_packed_bytes(n_events));
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
        yet_free_binned(y);
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
    yet_free_binned(y);
    y->ctx->live--;
    delete y;
    return ARA_OK;
}

extern "C" ara_status ara_yet_info(const ara_yet *y, int64_t *n_events, int64_t *n_trials, int32_t *id_bytes) {
    if (!y) return ARA_E_INVALID_ARG;
    if (n_events) *n_events = y->n_events;
    if (n_trials) *n_trials = y->n_trials;
    if (id_bytes) *id_bytes = y->ids16 ? 2 : (y->ids24 ? 3 : 4);
    return ARA_OK;
}

extern "C" ara_status ara_yet_memory(const ara_yet *y, int64_t *device_bytes, int32_t *run_bytes) {
    if (!y) return ARA_E_INVALID_ARG;
    if (device_bytes) *device_bytes = y->copy_bytes + (y->owns ? y->n_events * 4 + (y->n_trials + 1) * 8 : 0);
    if (run_bytes) *run_bytes = y->ids16 ? (y->boff24 ? 3 : 4) : 0;
    return ARA_OK;
}

extern "C" ara_status ara_yet_binned(const ara_yet *y, int32_t *n_bins, int64_t *region, uint32_t *boff,
                                    uint16_t *ids16) {
    if (!y || !n_bins) return ARA_E_INVALID_ARG;
    ara_ctx *c = y->ctx;
    *n_bins = y->ids16 ? y->n_bins : 0;
    if (!y->ids16) return ARA_OK;
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    HIP_OR_RETURN(c, hipStreamSynchronize(c->stream), "binned copy");
    const size_t nb = size_t(y->n_bins), cols = size_t(y->n_trials + 1);
    std::vector<int64_t> reg(nb + 1);
    HIP_OR_RETURN(c, hipMemcpy(reg.data(), y->region, (nb + 1) * 8, hipMemcpyDeviceToHost), "binned copy");
    if (region) std::copy(reg.begin(), reg.end(), region);
    if (boff && y->boff) {
        HIP_OR_RETURN(c, hipMemcpy2D(boff, cols * 4, y->boff, size_t(y->stride) * 4, cols * 4, nb, hipMemcpyDeviceToHost),
                      "binned copy");
    } else if (boff) {   // 3-byte run starts, widened
        std::vector<uint8_t> b24(nb * cols * 3);
        HIP_OR_RETURN(c, hipMemcpy2D(b24.data(), cols * 3, y->boff24, size_t(y->stride) * 3, cols * 3, nb,
                                     hipMemcpyDeviceToHost), "binned copy");
        for (size_t i = 0; i < nb * cols; ++i)
            boff[i] = uint32_t(b24[3 * i]) | (uint32_t(b24[3 * i + 1]) << 8) | (uint32_t(b24[3 * i + 2]) << 16);
    }
    if (ids16) HIP_OR_RETURN(c, hipMemcpy(ids16, y->ids16, size_t(reg[nb]) * 2, hipMemcpyDeviceToHost), "binned copy");
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
    // whole 8-byte pairs: the combined-table build reads binary32 tables two entries at a time
    if (s == ARA_OK) s = dev_alloc(c, &t->dat, (size_t(catalog) * vbytes + 7) & ~size_t(7), "elt table");
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
    L->ranks_ready = false;
    hipError_t e = launch_layer_filter(L->catalog, L->f32, L->terms.occ_retention, L->terms.occ_limit, L->t, c->stream,
                                       false);
    return e == hipSuccess ? ARA_OK : hip_fail(c, e, "layer filter");
}

// The filter-based kernels (LDS bitmap, lookups, events, occurrence maxima outside the
// tiled path, batches) read the layer's ranks and compacted values; the tiled kernel
// reads its occurrence values only.  Enqueued on the context's stream, before the
// caller's kernels.
static ara_status layer_ranks(const ara_layer *L) {
    if (L->ranks_ready) return ARA_OK;
    ara_ctx *c = L->ctx;
    hipError_t e = launch_layer_ranks(L->catalog, L->t, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "layer ranks");
    L->ranks_ready = true;
    return ARA_OK;
}

static ara_status layer_enqueue_build(ara_layer *L, int flags, bool ranks) {
    ara_ctx *c = L->ctx;
    const int n = int(L->elts.size());
    hipError_t e = hipSuccess;
    if ((flags & ARA_BUILD_TABLES) && n > 0) {
        e = launch_elt_clear(L->d_descs, n, L->catalog, c->stream);
        if (e == hipSuccess) e = launch_elt_scatter(L->d_descs, n, L->max_pairs, L->catalog, c->d_err, c->stream);
    }
    L->ranks_ready = false;
    if (e == hipSuccess)
        e = launch_layer_tables(L->d_descs, n, L->catalog, L->f32, L->terms.occ_retention, L->terms.occ_limit, L->t,
                                c->stream, ranks);
    if (e != hipSuccess) return hip_fail(c, e, "layer build");
    L->ranks_ready = ranks;
    return ARA_OK;
}

static void layer_free(ara_layer *L) {
    dev_free(L->d_descs);
    dev_free(L->t.comb);
    dev_free(L->t.occ);
    dev_free(L->t.bitmap);
    dev_free(L->t.nz);
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
    if (s == ARA_OK) s = dev_alloc(c, &L->t.nz, size_t(nblk) * 16, "layer nonzero bitmap");
    if (s == ARA_OK) s = dev_alloc(c, &L->t.rank, size_t(nblk) * 4, "layer ranks");
    if (s == ARA_OK) s = dev_alloc(c, &L->t.rel16, align16(size_t(nblk) * 2), "layer relative ranks");
    if (s == ARA_OK) s = dev_alloc(c, &L->t.base32, align16(size_t(bitmap_supers(nblk)) * 4), "layer rank bases");
    if (s == ARA_OK) s = dev_alloc(c, &L->t.vals, size_t(catalog) * 8, "layer values");
    if (s == ARA_OK) s = dev_alloc(c, &L->t.n_flagged, 16, "layer count");
    if (s == ARA_OK && n_elts > 0) {
        hipError_t e = hipMemcpy(L->d_descs, d.data(), sizeof(EltDesc) * size_t(n_elts), hipMemcpyHostToDevice);
        if (e != hipSuccess) s = hip_fail(c, e, "layer descriptors upload");
    }
    if (s == ARA_OK) s = layer_enqueue_build(L, 0, true);
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
    L->terms_gen++;
    return layer_enqueue_filter(L);
}

extern "C" ara_status ara_layer_build(ara_ctx *c, ara_layer *L, int flags) {
    if (!c || !L || L->ctx != c || (flags & ~ARA_BUILD_TABLES)) return ARA_E_INVALID_ARG;
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    return layer_enqueue_build(L, flags, false);
}

extern "C" ara_status ara_layer_stats(ara_ctx *c, const ara_layer *L, int64_t *n_flagged, int32_t *placement,
                                     int64_t *lds_bytes) {
    if (!c || !L || L->ctx != c) return ARA_E_INVALID_ARG;
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    TrialLaunch tl{};
    ara_status s = plan_trial(c, L, 1 << 20, 1e9, tl);
    if (s != ARA_OK) return s;
    if (placement) *placement = tl.placement;
    if (lds_bytes) *lds_bytes = int64_t(tl.lds_bytes);
    if (n_flagged) {
        s = layer_ranks(L);
        if (s != ARA_OK) return s;
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
    a.nz = L->t.nz;
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

// Arguments of the tiled trial kernel for trials [t0, t1) over `grid` workgroups.
static TiledArgs tiled_args(const ara_yet *y, const ara_layer *L, int64_t t0, int64_t t1, double *ylt, int grid) {
    TiledArgs a{};
    a.ids16 = y->ids16;
    a.region = y->region;
    a.boff = y->boff;
    a.boff24 = y->boff24;
    a.stride = y->stride;
    a.t_begin = t0;
    a.t_end = t1;
    a.per_wg = (t1 - t0 + grid - 1) / std::max(1, grid);
    a.occ = L->t.occ;
    a.catalog = L->catalog;
    a.n_bins = y->n_bins;
    a.agg_r = L->terms.agg_retention;
    a.agg_l = L->terms.agg_limit;
    a.ylt = ylt;
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
    s = plan_trial(c, L, t1 - t0, y->n_trials ? double(y->n_events) / double(y->n_trials) : 0.0, tl,
                   y->ids16 ? 1 : 0);
    if (s == ARA_OK && tl.placement != ARA_PLACE_LDS_TILES) s = layer_ranks(L);
    if (s != ARA_OK) return s;
    double *dst = ylt;
    if (mem == ARA_MEM_HOST) {
        s = dev_alloc(c, &dst, size_t(t1 - t0) * 8, "ylt staging");
        if (s != ARA_OK) return s;
    }
    // trial indices inside a launch are 32-bit: split very long ranges
    constexpr int64_t kMaxTrialsPerLaunch = int64_t(1) << 30;
    const bool timing = !c->k_ev.empty(), tiles = tl.placement == ARA_PLACE_LDS_TILES;
    const size_t slot = timing ? size_t(c->k_count % int64_t(c->k_ev.size() / 2)) : 0;
    hipEvent_t t_start = timing ? c->k_ev[2 * slot] : nullptr, t_stop = timing ? c->k_ev[2 * slot + 1] : nullptr;
    hipError_t e = timing && !tiles ? hipEventRecord(t_start, c->stream) : hipSuccess;
    for (int64_t tb = t0; tb < t1 && e == hipSuccess; tb += kMaxTrialsPerLaunch) {
        const int64_t te = std::min(t1, tb + kMaxTrialsPerLaunch);
        if (tiles) {
            // timed: events attached to the first launch's start and the last one's end
            const bool first = tb == t0, last = te == t1;
            e = launch_trial_tiled(tiled_args(y, L, tb, te, dst + (tb - t0), tl.grid), tl.grid, c->stream, false,
                                   first ? t_start : nullptr, last ? t_stop : nullptr);
            continue;
        }
        TrialArgs a = trial_args(y, L, tb, te, dst + (tb - t0));
        a.qcap = tl.qcap;
        e = launch_trial_ylt(a, tl, c->stream);
    }
    if (e == hipSuccess && timing && !tiles) e = hipEventRecord(t_stop, c->stream);
    if (e == hipSuccess && timing) c->k_count++;
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

extern "C" ara_status ara_analyze_occ_max(ara_ctx *c, const ara_yet *y, const ara_layer *L, int64_t t0, int64_t t1,
                                         double *out, ara_mem mem) {
    ara_status s = check_analysis(c, y, L, t0, t1);
    if (s != ARA_OK) return s;
    if ((t1 > t0 && !out) || (mem != ARA_MEM_HOST && mem != ARA_MEM_DEVICE))
        return fail(c, ARA_E_INVALID_ARG, "occurrence maxima: bad output");
    if (t1 == t0) return ARA_OK;
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    TrialLaunch tl{};
    s = plan_trial(c, L, t1 - t0, 1e9, tl, y->ids16 ? 1 : 0);
    if (s == ARA_OK && tl.placement != ARA_PLACE_LDS_TILES) s = layer_ranks(L);
    if (s != ARA_OK) return s;
    const int by_lds = tl.lds_bytes > 0 ? std::max(1, int(c->lds_max / int64_t(tl.lds_bytes))) : 8;
    const int64_t grid = std::min<int64_t>(int64_t(c->n_cu) * std::min(8, by_lds), (t1 - t0 + 255) / 256);
    double *dst = out;
    if (mem == ARA_MEM_HOST) {
        s = dev_alloc(c, &dst, size_t(t1 - t0) * 8, "occurrence maxima staging");
        if (s != ARA_OK) return s;
    }
    hipError_t e = hipSuccess;
    if (tl.placement == ARA_PLACE_LDS_TILES) {
        // the tiled kernel with a maximum in place of the sum (trial indices inside a
        // launch are 32-bit: very long ranges are split)
        constexpr int64_t kMaxTrialsPerLaunch = int64_t(1) << 30;
        for (int64_t tb = t0; tb < t1 && e == hipSuccess; tb += kMaxTrialsPerLaunch) {
            const int64_t te = std::min(t1, tb + kMaxTrialsPerLaunch);
            e = launch_trial_tiled(tiled_args(y, L, tb, te, dst + (tb - t0), tl.grid), tl.grid, c->stream, true);
        }
    } else {
        const TrialArgs a = trial_args(y, L, t0, t1, nullptr);
        e = launch_trial_occ_max(a, tl, int(std::max<int64_t>(1, grid)), dst, c->stream);
    }
    if (e != hipSuccess) s = hip_fail(c, e, "occurrence maxima");
    if (s == ARA_OK && mem == ARA_MEM_HOST) {
        e = hipMemcpyAsync(out, dst, size_t(t1 - t0) * 8, hipMemcpyDeviceToHost, c->stream);
        s = e == hipSuccess ? sync_and_check(c) : hip_fail(c, e, "occurrence maxima download");
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
    s = layer_ranks(L);
    if (s != ARA_OK) return s;
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
    hipError_t e = launch_trial_events(a, L->f32, c->n_cu, c->lds_max, c->stream);
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
    ara_status s = plan_trial(c, L, 1 << 20, 1e9, tl);
    if (s == ARA_OK) s = layer_ranks(L);
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
    hipError_t e = launch_sort_desc_keys(in, n, w, c->stream);   // stays asynchronous
    if (e == hipSuccess) e = launch_sort_decode(w, n, out, c->stream);
    s = e == hipSuccess ? ARA_OK : hip_fail(c, e, "sort");
    if (owned) {
        (void)hipStreamSynchronize(c->stream);
        dev_free(w);
    }
    return s;
}

constexpr int32_t kMaxReturnPeriods = int32_t(kStageDoubles / 2);

// Ranks ks[0 .. n_rp) of the return periods for n losses (host, no allocation);
// ARA_E_INVALID_ARG for too many or a bad period.
static ara_status risk_ranks(ara_ctx *c, int64_t n, const double *rps, int32_t n_rp, int64_t *ks) {
    if (n_rp > kMaxReturnPeriods) return fail(c, ARA_E_INVALID_ARG, "at most %d return periods", kMaxReturnPeriods);
    for (int32_t i = 0; i < n_rp; ++i)
        if (ara_return_period_rank(n, rps[i], &ks[i]) != ARA_OK)
            return fail(c, ARA_E_INVALID_ARG, "return period %g invalid (must be >= 1)", rps[i]);
    return ARA_OK;
}

// PML/TVaR of the n_rp ranks ks of the device YLT dy (radix selection in workspace
// w), results to the host (blocking).  Allocates nothing.
static ara_status risk_on_device(ara_ctx *c, const double *dy, int64_t n, const int64_t *ks, int32_t n_rp, double *pml,
                                 double *tvar, void *w) {
    hipError_t e = launch_risk_select(dy, n, w, ks, n_rp, c->d_out, c->stream);
    // the error word and the results in one copy (they are adjacent)
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->h_err, c->d_err, kErrBytes + size_t(2 * n_rp) * 8, hipMemcpyDeviceToHost, c->stream);
    ara_status s = e == hipSuccess ? sync_and_check(c, nullptr, true) : hip_fail(c, e, "risk measures");
    if (s != ARA_OK) return s;
    for (int32_t base = 0; base < n_rp; base += 16) {
        const int32_t m = std::min<int32_t>(16, n_rp - base);
        for (int32_t i = 0; i < m; ++i) {
            pml[base + i] = c->h_out[2 * base + i];
            tvar[base + i] = c->h_out[2 * base + m + i];
        }
    }
    return ARA_OK;
}

extern "C" ara_status ara_risk_measures(ara_ctx *c, const double *ylt, int64_t n, ara_mem mem, const double *rps,
                                       int32_t n_rp, double *pml, double *tvar, void *ws, size_t ws_bytes) {
    if (!c || n < 0 || n_rp < 0 || (n_rp > 0 && (!rps || !pml || !tvar)) || (mem != ARA_MEM_HOST && mem != ARA_MEM_DEVICE))
        return ARA_E_INVALID_ARG;
    if (n == 0) return fail(c, ARA_E_EMPTY, "risk measures of an empty YLT");
    if (!ylt) return ARA_E_INVALID_ARG;
    int64_t ks[kMaxReturnPeriods];
    ara_status s = risk_ranks(c, n, rps, n_rp, ks);
    if (s != ARA_OK) return s;
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    const double *dy = ylt;
    double *tmp = nullptr;
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
    if (s == ARA_OK) s = risk_on_device(c, dy, n, ks, n_rp, pml, tvar, w);
    if (owned || tmp) (void)hipStreamSynchronize(c->stream);
    if (owned) dev_free(w);
    dev_free(tmp);
    return s;
}

extern "C" ara_status ara_risk_measures_noalloc(ara_ctx *c, const double *ylt, int64_t n, const double *rps,
                                               int32_t n_rp, double *pml, double *tvar) {
    if (!c || n < 0 || n_rp < 0 || (n_rp > 0 && (!rps || !pml || !tvar))) return ARA_E_INVALID_ARG;
    if (n == 0) return fail(c, ARA_E_EMPTY, "risk measures of an empty YLT");
    if (!ylt) return ARA_E_INVALID_ARG;
    if (n > int64_t(ARA_NOALLOC_MAX_N))
        return fail(c, ARA_E_INVALID_ARG, "allocation-free risk measures: %lld losses, at most %lld", (long long)n,
                    (long long)ARA_NOALLOC_MAX_N);
    if (sort_workspace_bytes(n) > kScratchBytes || !c->scratch)
        return fail(c, ARA_E_DEVICE, "allocation-free risk measures: scratch of %zu bytes too small for %lld losses",
                    kScratchBytes, (long long)n);
    int64_t ks[kMaxReturnPeriods];
    ara_status s = risk_ranks(c, n, rps, n_rp, ks);
    if (s != ARA_OK) return s;
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    return risk_on_device(c, ylt, n, ks, n_rp, pml, tvar, c->scratch);
}

// ------------------------------------------------------------------ batches
struct ara_batch {
    ara_ctx *ctx;
    std::vector<ara_job> jobs;
    std::vector<BatchJob> hjobs;
    std::vector<int64_t> mean_len;   // per job: occurrences per trial of its YET (at least 1)
    std::vector<TiledArgs> tjobs;    // jobs run by the tiled kernel: their arguments
    std::vector<int32_t> tiled_job;  // the job of each entry of `tjobs`
    std::vector<TiledItem> titems;   // their passes (tjobs indices), one launch for all
    TiledArgs *d_tjobs = nullptr;
    TiledItem *d_titems = nullptr;
    uint32_t *d_next = nullptr;      // the tiled launch's item counter
    std::vector<uint64_t> terms_gen; // per job: its layer's terms generation when last uploaded
    std::string shape;               // key of the tuning cache
    BatchJob *d_jobs = nullptr;
    BatchItem *d_items = nullptr;
    int32_t n_items = 0, grid = 0;   // grid: the largest of the per-mode launches
    int32_t mode_off[kBatchModes] = {}, mode_cnt[kBatchModes] = {};
    int64_t events_per_item = 0;
    bool interleave = false;         // workgroups take every G-th item (else contiguous runs)
    hipStream_t cap = nullptr;       // private stream the launch is captured on
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // risk measures
    const double **d_ylts = nullptr;
    int64_t *d_ns = nullptr, *d_ks = nullptr;
    double *d_risk = nullptr;
    int32_t risk_cap = 0;            // return periods d_ks/d_risk hold
    void *ws = nullptr;              // sort workspace for YLTs too long for one workgroup
    size_t ws_bytes = 0;
    bool counted = false;            // counted in ctx->live
};

// Work items of job j (trials [tb, te), mean_len occurrences per trial) of about
// `events` occurrences each: whole trials, at least one per lane (lane mode) or wave.
static void split_items(int32_t j, int32_t mode, int64_t tb, int64_t te, int64_t mean_len, int64_t events,
                        std::vector<BatchItem> &items) {
    const int64_t unit = mode == kModeLaneLds || mode == kModeLaneGlobal ? 1024 : 16;
    int64_t per = std::max<int64_t>(1, events / std::max<int64_t>(1, mean_len));
    per = (per + unit - 1) / unit * unit;
    for (int64_t t = tb; t < te; t += per) items.push_back(BatchItem{j, 0, t, std::min(te, t + per)});
}

// Work items of many jobs grouped by mode (kernel), then by job in job order; off/cnt
// give each mode's range of the list.
static std::vector<BatchItem> group_items(const std::vector<BatchJob> &hjobs, const int64_t *tb, const int64_t *te,
                                          const std::vector<int64_t> &mean_len, int64_t events, int32_t *off,
                                          int32_t *cnt) {
    std::vector<BatchItem> items;
    for (int m = 0; m < kBatchModes; ++m) {
        off[m] = int32_t(items.size());
        for (size_t j = 0; j < hjobs.size(); ++j)
            if (hjobs[j].mode == m) split_items(int32_t(j), m, tb[j], te[j], mean_len[j], events, items);
        cnt[m] = int32_t(items.size()) - off[m];
    }
    return items;
}

// Workgroups and items per workgroup for n items (at most one workgroup per CU).
static void batch_shape(int32_t n_items, int n_cu, int32_t &grid, int32_t &per_wg) {
    grid = std::max(1, std::min(n_items, n_cu));
    per_wg = (n_items + grid - 1) / grid;
    grid = n_items > 0 ? (n_items + per_wg - 1) / std::max(1, per_wg) : 1;
}

// One persistent launch per mode present, in mode order; interleave: workgroups take
// every G-th item instead of a contiguous run.  Jobs of the tiled kernel follow, one
// launch each.
struct TiledBatch {
    const TiledArgs *jobs = nullptr;
    const TiledItem *items = nullptr;
    int32_t n_items = 0;
    uint32_t *next = nullptr;
};

static hipError_t launch_grouped(const BatchJob *d_jobs, const BatchItem *d_items, const int32_t *off,
                                 const int32_t *cnt, int n_cu, bool interleave, hipStream_t s,
                                 const std::vector<std::pair<TiledArgs, int>> &tiled, const TiledBatch &tb = TiledBatch()) {
    for (int m = 0; m < kBatchModes; ++m) {
        if (cnt[m] == 0) continue;
        int32_t grid = 1, per_wg = 0;
        batch_shape(cnt[m], n_cu, grid, per_wg);
        if (interleave) {
            grid = std::max(1, std::min(cnt[m], n_cu));
            per_wg = 0;
        }
        const hipError_t e = launch_batch(m, d_jobs, d_items + off[m], cnt[m], per_wg, grid, s);
        if (e != hipSuccess) return e;
    }
    for (const auto &ta : tiled) {
        const hipError_t e = launch_trial_tiled(ta.first, ta.second, s);
        if (e != hipSuccess) return e;
    }
    if (tb.n_items > 0)
        return launch_trial_tiled_items(tb.jobs, tb.items, tb.n_items, tb.next, std::min(tb.n_items, n_cu), s);
    return hipSuccess;
}

static TiledBatch batch_tiled(const ara_batch *b) {
    TiledBatch t;
    t.jobs = b->d_tjobs;
    t.items = b->d_titems;
    t.n_items = int32_t(b->titems.size());
    t.next = b->d_next;
    return t;
}

// A tiled job's trials [tb, te) as work items of job index k: passes of nearly equal
// size, as few as kTiledPassTrials allows (each pass stages every bin of the catalog
// once), with each one's cost (occurrences, plus the staging).  A trial's YLT does not
// depend on the pass that holds it (its lane adds the bins in order and each run's
// occurrences in order), so the items give the plain launch's bits.
static void tiled_passes(int32_t k, int64_t tb, int64_t te, double mean_len, double stage,
                         std::vector<std::pair<double, TiledItem>> &out) {
    const int64_t n = te - tb;
    const int64_t passes = (n + kTiledPassTrials - 1) / kTiledPassTrials;
    const int64_t per = (n + passes - 1) / std::max<int64_t>(1, passes);
    for (int64_t p = tb; p < te; p += per) {
        TiledItem it{};
        it.job = k;
        it.t0 = p;
        it.t1 = std::min(p + per, te);
        out.emplace_back(double(it.t1 - it.t0) * mean_len + stage, it);
    }
}

static ara_status batch_set_items(ara_batch *b, int64_t events) {
    ara_ctx *c = b->ctx;
    std::vector<int64_t> tb, te;
    for (const ara_job &j : b->jobs) {
        tb.push_back(j.trial_begin);
        te.push_back(j.trial_end);
    }
    const std::vector<BatchItem> items = group_items(b->hjobs, tb.data(), te.data(), b->mean_len, events, b->mode_off,
                                                     b->mode_cnt);
    dev_free(b->d_items);
    b->d_items = nullptr;
    b->n_items = int32_t(items.size());
    if (b->n_items > 0) {
        ara_status s = dev_alloc(c, &b->d_items, items.size() * sizeof(BatchItem), "batch items");
        if (s != ARA_OK) return s;
        HIP_OR_RETURN(c, hipMemcpy(b->d_items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice),
                      "batch items upload");
    }
    b->grid = 0;
    for (int m = 0; m < kBatchModes; ++m) {
        int32_t g = 1, per = 0;
        if (b->mode_cnt[m]) batch_shape(b->mode_cnt[m], c->n_cu, g, per);
        if (b->mode_cnt[m]) b->grid = std::max(b->grid, g);
    }
    b->events_per_item = events;
    return ARA_OK;
}

extern "C" ara_status ara_batch_create(ara_ctx *c, const ara_job *jobs, int32_t n_jobs, ara_batch **out) {
    if (!c || !out || n_jobs < 0 || (n_jobs > 0 && !jobs)) return ARA_E_INVALID_ARG;
    *out = nullptr;
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    ara_batch *b = new (std::nothrow) ara_batch();
    if (!b) return ARA_E_OOM;
    b->ctx = c;
    char key[160];
    std::vector<std::pair<double, TiledItem>> titems;
    for (int32_t j = 0; j < n_jobs; ++j) {
        const ara_job &jb = jobs[j];
        ara_status s = check_analysis(c, jb.yet, jb.layer, jb.trial_begin, jb.trial_end);
        if (s == ARA_OK && jb.trial_end > jb.trial_begin && !jb.ylt) s = fail(c, ARA_E_INVALID_ARG, "job %d: no YLT", j);
        TrialLaunch tl{};
        const double mean = jb.yet && jb.yet->n_trials ? double(jb.yet->n_events) / double(jb.yet->n_trials) : 0.0;
        if (s == ARA_OK) s = plan_trial(c, jb.layer, jb.trial_end - jb.trial_begin, mean, tl, jb.yet->ids16 ? 1 : 0);
        if (s != ARA_OK) {
            delete b;
            return s;
        }
        BatchJob h{};
        h.a = trial_args(jb.yet, jb.layer, jb.trial_begin, jb.trial_end, jb.ylt);
        h.a.qcap = tl.qcap;
        h.mode = batch_mode(tl, h.a.ids24 != nullptr);
        h.placement = tl.placement;
        if (h.mode == kModeTiled && jb.trial_end > jb.trial_begin) {
            b->tjobs.push_back(tiled_args(jb.yet, jb.layer, jb.trial_begin, jb.trial_end, jb.ylt, tl.grid));
            b->tiled_job.push_back(j);
            tiled_passes(int32_t(b->tjobs.size() - 1), jb.trial_begin, jb.trial_end, mean,
                         kTiledStageCost * double(jb.layer->catalog), titems);
        }
        b->terms_gen.push_back(jb.layer->terms_gen);
        b->jobs.push_back(jb);
        b->hjobs.push_back(h);
        b->mean_len.push_back(std::max<int64_t>(1, int64_t(std::llround(mean))));
        std::snprintf(key, sizeof key, "%d:%lld:%lld:%d;", h.mode, (long long)(jb.trial_end - jb.trial_begin),
                      (long long)b->mean_len.back(), jb.layer->catalog);
        b->shape += key;
    }
    ara_status s = ARA_OK;
    if (n_jobs > 0) {
        s = dev_alloc(c, &b->d_jobs, b->hjobs.size() * sizeof(BatchJob), "batch jobs");
        if (s == ARA_OK) {
            hipError_t e = hipMemcpy(b->d_jobs, b->hjobs.data(), b->hjobs.size() * sizeof(BatchJob), hipMemcpyHostToDevice);
            if (e != hipSuccess) s = hip_fail(c, e, "batch jobs upload");
        }
    }
    if (s == ARA_OK && !titems.empty()) {
        // costliest passes first, so that the last ones taken are short
        std::stable_sort(titems.begin(), titems.end(),
                         [](const std::pair<double, TiledItem> &x, const std::pair<double, TiledItem> &y) {
                             return x.first > y.first;
                         });
        for (const auto &it : titems) b->titems.push_back(it.second);
        s = dev_alloc(c, &b->d_tjobs, b->tjobs.size() * sizeof(TiledArgs), "batch tiled jobs");
        if (s == ARA_OK) s = dev_alloc(c, &b->d_titems, b->titems.size() * sizeof(TiledItem), "batch tiled items");
        if (s == ARA_OK) s = dev_alloc(c, &b->d_next, 256, "batch tiled counter");
        if (s == ARA_OK) {
            hipError_t e = hipMemcpy(b->d_tjobs, b->tjobs.data(), b->tjobs.size() * sizeof(TiledArgs), hipMemcpyHostToDevice);
            if (e == hipSuccess)
                e = hipMemcpy(b->d_titems, b->titems.data(), b->titems.size() * sizeof(TiledItem), hipMemcpyHostToDevice);
            if (e != hipSuccess) s = hip_fail(c, e, "batch tiled upload");
        }
    }
    if (s != ARA_OK) {
        ara_batch_release(b);
        return s;
    }
    c->live++;
    b->counted = true;
    *out = b;
    return ARA_OK;
}

// First run: time each candidate split (every candidate computes the same results),
// keep the fastest for this batch shape, then capture the launch in a graph that
// later runs replay on the context's stream.  *computed: whether the timed runs
// wrote every job's YLT (not so when the shape was already tuned on this context).
constexpr int kTuneReps = 3;   // timings of each candidate (the fastest counts)

static ara_status batch_tune(ara_batch *b, bool *computed) {
    ara_ctx *c = b->ctx;
    *computed = false;
    auto it = c->tuned.find(b->shape);
    if (it != c->tuned.end()) {
        b->interleave = it->second.second;
        return batch_set_items(b, it->second.first);
    }
    static const int64_t kEvents[] = {int64_t(1) << 16, int64_t(1) << 18, int64_t(1) << 20, int64_t(1) << 22};
    {
        ara_status s0 = batch_set_items(b, kEvents[0]);
        if (s0 != ARA_OK) return s0;
        int32_t persistent = 0;
        for (int m = 0; m < kBatchModes; ++m) persistent += b->mode_cnt[m];
        if (persistent == 0) {   // only tiled jobs: nothing to choose
            c->tuned[b->shape] = {kEvents[0], false};
            b->interleave = false;
            return ARA_OK;
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_OR_RETURN(c, hipEventCreate(&e0), "event");
    hipError_t e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(c, e, "event");
    }
    std::pair<int64_t, bool> best{kEvents[0], false};
    float best_ms = 1e30f;
    ara_status s = ARA_OK;
    for (int64_t ev : kEvents) {
        s = batch_set_items(b, ev);
        if (s != ARA_OK) break;
        for (bool inter : {false, true}) {
            for (int rep = 0; rep < kTuneReps && e == hipSuccess; ++rep) {
                e = hipEventRecord(e0, c->stream);
                if (e == hipSuccess)
                    e = launch_grouped(b->d_jobs, b->d_items, b->mode_off, b->mode_cnt, c->n_cu, inter, c->stream, {},
                                       batch_tiled(b));
                if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e == hipSuccess && ms < best_ms) {
                    best_ms = ms;
                    best = {ev, inter};
                }
            }
            if (e != hipSuccess) break;
        }
        if (e != hipSuccess) {
            s = hip_fail(c, e, "batch tuning run");
            break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != ARA_OK) return s;
    s = sync_and_check(c);
    if (s != ARA_OK) return s;
    *computed = true;
    c->tuned[b->shape] = best;
    b->interleave = best.second;
    return batch_set_items(b, best.first);
}

static ara_status batch_capture(ara_batch *b) {
    ara_ctx *c = b->ctx;
    HIP_OR_RETURN(c, hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking), "capture stream");
    HIP_OR_RETURN(c, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal), "begin capture");
    hipError_t e = launch_grouped(b->d_jobs, b->d_items, b->mode_off, b->mode_cnt, c->n_cu, b->interleave, b->cap, {},
                                  batch_tiled(b));
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->cap, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) b->graph = g;
    else if (g) (void)hipGraphDestroy(g);
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    return e == hipSuccess ? ARA_OK : hip_fail(c, e, "batch graph");
}

// Layer terms are copied into the job descriptors and the tiled jobs' arguments, both
// in device memory that the captured launches read: after ara_layer_set_terms on a
// member layer, upload them again.
static ara_status batch_refresh_terms(ara_batch *b) {
    ara_ctx *c = b->ctx;
    bool changed = false;
    for (size_t j = 0; j < b->jobs.size(); ++j) {
        const ara_layer *L = b->jobs[j].layer;
        if (L->terms_gen == b->terms_gen[j]) continue;
        changed = true;
        b->terms_gen[j] = L->terms_gen;
        TrialArgs &a = b->hjobs[j].a;
        a.occ_r = L->terms.occ_retention;
        a.occ_l = L->terms.occ_limit;
        a.agg_r = L->terms.agg_retention;
        a.agg_l = L->terms.agg_limit;
    }
    if (!changed) return ARA_OK;
    for (size_t k = 0; k < b->tjobs.size(); ++k) {
        const ara_layer *L = b->jobs[size_t(b->tiled_job[k])].layer;
        b->tjobs[k].agg_r = L->terms.agg_retention;
        b->tjobs[k].agg_l = L->terms.agg_limit;
    }
    // earlier runs on the stream may still read the descriptors
    HIP_OR_RETURN(c, hipStreamSynchronize(c->stream), "stream synchronize");
    HIP_OR_RETURN(c, hipMemcpy(b->d_jobs, b->hjobs.data(), b->hjobs.size() * sizeof(BatchJob), hipMemcpyHostToDevice),
                  "batch jobs upload");
    if (!b->tjobs.empty())
        HIP_OR_RETURN(c, hipMemcpy(b->d_tjobs, b->tjobs.data(), b->tjobs.size() * sizeof(TiledArgs), hipMemcpyHostToDevice),
                      "batch tiled jobs upload");
    return ARA_OK;
}

extern "C" ara_status ara_batch_run(ara_batch *b) {
    if (!b) return ARA_E_INVALID_ARG;
    ara_ctx *c = b->ctx;
    if (b->jobs.empty()) return ARA_OK;
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    ara_status s = batch_refresh_terms(b);
    for (size_t j = 0; j < b->jobs.size() && s == ARA_OK; ++j) s = layer_ranks(b->jobs[j].layer);
    if (s != ARA_OK) return s;
    if (!b->exec) {
        bool computed = false;
        s = batch_tune(b, &computed);
        if (s != ARA_OK) return s;
        s = batch_capture(b);
        if (s != ARA_OK) return s;
        if (computed) return ARA_OK;   // the tuning runs already computed every job
    }
    HIP_OR_RETURN(c, hipGraphLaunch(b->exec, c->stream), "batch graph launch");
    return ARA_OK;
}

extern "C" ara_status ara_tune_cache_save(const ara_ctx *c, const char *path) {
    if (!c || !path) return ARA_E_INVALID_ARG;
    FILE *f = std::fopen(path, "w");
    if (!f) return ARA_E_INVALID_ARG;
    std::fprintf(f, "# libara batch schedules: events per item, interleave, batch shape\n");
    for (const auto &kv : c->tuned)
        std::fprintf(f, "%lld %d %s\n", (long long)kv.second.first, kv.second.second ? 1 : 0, kv.first.c_str());
    const bool ok = std::fflush(f) == 0;
    std::fclose(f);
    return ok ? ARA_OK : ARA_E_INVALID_ARG;
}

extern "C" ara_status ara_tune_cache_load(ara_ctx *c, const char *path) {
    if (!c || !path) return ARA_E_INVALID_ARG;
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(c, ARA_E_INVALID_ARG, "tuning cache %s: cannot open", path);
    std::map<std::string, std::pair<int64_t, bool>> got;
    char line[8192];
    ara_status s = ARA_OK;
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        long long ev = 0;
        int inter = 0, used = 0;
        if (std::sscanf(line, "%lld %d %n", &ev, &inter, &used) != 2 || ev < 1 || (inter != 0 && inter != 1)) {
            s = fail(c, ARA_E_INVALID_ARG, "tuning cache %s: bad line", path);
            break;
        }
        std::string key(line + used);
        while (!key.empty() && (key.back() == '\n' || key.back() == '\r')) key.pop_back();
        if (key.empty()) {
            s = fail(c, ARA_E_INVALID_ARG, "tuning cache %s: line without a shape", path);
            break;
        }
        got[key] = {int64_t(ev), inter != 0};
    }
    std::fclose(f);
    if (s != ARA_OK) return s;
    for (const auto &kv : got) c->tuned[kv.first] = kv.second;
    return ARA_OK;
}

extern "C" ara_status ara_batch_info(const ara_batch *b, int32_t *n_items, int32_t *grid, int64_t *events_per_item,
                                    int32_t *graph) {
    if (!b) return ARA_E_INVALID_ARG;
    if (n_items) *n_items = b->n_items;
    if (grid) *grid = b->grid;
    if (events_per_item) *events_per_item = b->events_per_item;
    if (graph) *graph = (b->exec ? 1 : 0) | (b->interleave ? 2 : 0);
    return ARA_OK;
}

// Device list of the jobs' YLT pointers and lengths (built once).
static ara_status batch_ylt_list(ara_batch *b) {
    if (b->d_ylts) return ARA_OK;
    ara_ctx *c = b->ctx;
    const size_t nj = b->jobs.size();
    std::vector<const double *> yp(nj);
    std::vector<int64_t> ns(nj);
    for (size_t j = 0; j < nj; ++j) {
        yp[j] = b->jobs[j].ylt;
        ns[j] = b->jobs[j].trial_end - b->jobs[j].trial_begin;
    }
    ara_status s = dev_alloc(c, &b->d_ylts, nj * sizeof(double *), "batch ylt list");
    if (s == ARA_OK) s = dev_alloc(c, &b->d_ns, nj * 8, "batch sizes");
    if (s != ARA_OK) return s;
    HIP_OR_RETURN(c, hipMemcpy(b->d_ylts, yp.data(), nj * sizeof(double *), hipMemcpyHostToDevice), "upload");
    HIP_OR_RETURN(c, hipMemcpy(b->d_ns, ns.data(), nj * 8, hipMemcpyHostToDevice), "upload");
    return ARA_OK;
}

extern "C" ara_status ara_batch_portfolio(ara_batch *b, double *out) {
    if (!b || !out) return ARA_E_INVALID_ARG;
    ara_ctx *c = b->ctx;
    if (b->jobs.empty()) return fail(c, ARA_E_INVALID_ARG, "portfolio of an empty batch");
    const int64_t n = b->jobs[0].trial_end - b->jobs[0].trial_begin;
    for (const ara_job &j : b->jobs)
        if (j.trial_end - j.trial_begin != n) return fail(c, ARA_E_INVALID_ARG, "portfolio: jobs cover different trial counts");
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    ara_status s = batch_ylt_list(b);
    if (s != ARA_OK) return s;
    const hipError_t e = launch_sum_ylts(b->d_ylts, int32_t(b->jobs.size()), n, out, c->stream);
    return e == hipSuccess ? ARA_OK : hip_fail(c, e, "portfolio sum");
}

extern "C" ara_status ara_batch_risk(ara_batch *b, const double *rps, int32_t n_rp, double *pml, double *tvar) {
    if (!b || n_rp < 0 || (n_rp > 0 && (!rps || !pml || !tvar))) return ARA_E_INVALID_ARG;
    ara_ctx *c = b->ctx;
    const int32_t nj = int32_t(b->jobs.size());
    if (nj == 0 || n_rp == 0) return ARA_OK;
    if (size_t(n_rp) * 2 > kStageDoubles) return fail(c, ARA_E_INVALID_ARG, "at most %zu return periods", kStageDoubles / 2);
    for (int32_t j = 0; j < nj; ++j)
        if (b->jobs[size_t(j)].trial_end == b->jobs[size_t(j)].trial_begin)
            return fail(c, ARA_E_EMPTY, "job %d: risk measures of an empty YLT", j);
    std::vector<int64_t> ks(size_t(nj) * size_t(n_rp));
    for (int32_t j = 0; j < nj; ++j) {
        const int64_t n = b->jobs[size_t(j)].trial_end - b->jobs[size_t(j)].trial_begin;
        for (int32_t r = 0; r < n_rp; ++r)
            if (ara_return_period_rank(n, rps[r], &ks[size_t(j) * n_rp + r]) != ARA_OK)
                return fail(c, ARA_E_INVALID_ARG, "return period %g invalid (must be >= 1)", rps[r]);
    }
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    {
        ara_status s = batch_ylt_list(b);
        if (s != ARA_OK) return s;
    }
    if (b->risk_cap < n_rp) {
        dev_free(b->d_ks);
        dev_free(b->d_risk);
        b->d_ks = nullptr;
        b->d_risk = nullptr;
        ara_status s = dev_alloc(c, &b->d_ks, ks.size() * 8, "batch ranks");
        if (s == ARA_OK) s = dev_alloc(c, &b->d_risk, size_t(nj) * 2 * size_t(n_rp) * 8, "batch risk");
        if (s != ARA_OK) return s;
        b->risk_cap = n_rp;
    }
    HIP_OR_RETURN(c, hipMemcpyAsync(b->d_ks, ks.data(), ks.size() * 8, hipMemcpyHostToDevice, c->stream), "upload ranks");
    // short YLTs: one workgroup each, all in one launch; long ones: radix selection,
    // one after another in the workspace, each into its own results
    hipError_t e = launch_risk_batch(b->d_ylts, b->d_ns, b->d_ks, nj, n_rp, b->d_risk, c->stream);
    for (int32_t j = 0; j < nj && e == hipSuccess; ++j) {
        const int64_t n = b->jobs[size_t(j)].trial_end - b->jobs[size_t(j)].trial_begin;
        if (n <= kRiskLdsKeys) continue;
        const size_t need = sort_workspace_bytes(n);
        if (b->ws_bytes < need) {
            e = hipStreamSynchronize(c->stream);
            dev_free(b->ws);
            b->ws = nullptr;
            b->ws_bytes = 0;
            if (e == hipSuccess) e = hipMalloc(&b->ws, need);
            if (e != hipSuccess) break;
            b->ws_bytes = need;
        }
        // groups of 16 return periods: pml[m] then tvar[m] per group
        e = launch_risk_select(b->jobs[size_t(j)].ylt, n, b->ws, &ks[size_t(j) * n_rp], n_rp,
                               b->d_risk + size_t(j) * 2 * n_rp, c->stream);
    }
    if (e != hipSuccess) return hip_fail(c, e, "batch risk measures");
    std::vector<double> small(size_t(nj) * 2 * size_t(n_rp));
    HIP_OR_RETURN(c, hipMemcpyAsync(small.data(), b->d_risk, small.size() * 8, hipMemcpyDeviceToHost, c->stream),
                  "download risk");
    ara_status s = sync_and_check(c);
    if (s != ARA_OK) return s;
    for (int32_t j = 0; j < nj; ++j) {
        const int64_t n = b->jobs[size_t(j)].trial_end - b->jobs[size_t(j)].trial_begin;
        const double *src = &small[size_t(j) * 2 * n_rp];
        for (int32_t r = 0; r < n_rp; ++r) {
            if (n <= kRiskLdsKeys) {   // the batched kernel: pml[n_rp], then tvar[n_rp]
                pml[size_t(j) * n_rp + r] = src[r];
                tvar[size_t(j) * n_rp + r] = src[n_rp + r];
            } else {                   // the selection: per group of 16, pml[m] then tvar[m]
                const int32_t base = r / 16 * 16, m = std::min<int32_t>(16, n_rp - base), i = r - base;
                pml[size_t(j) * n_rp + r] = src[2 * base + i];
                tvar[size_t(j) * n_rp + r] = src[2 * base + m + i];
            }
        }
    }
    return ARA_OK;
}

extern "C" ara_status ara_batch_release(ara_batch *b) {
    if (!b) return ARA_E_INVALID_ARG;
    ara_ctx *c = b->ctx;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    dev_free(b->d_jobs);
    dev_free(b->d_items);
    dev_free(b->d_tjobs);
    dev_free(b->d_titems);
    dev_free(b->d_next);
    dev_free(b->d_ylts);
    dev_free(b->d_ns);
    dev_free(b->d_ks);
    dev_free(b->d_risk);
    dev_free(b->ws);
    if (b->counted) c->live--;
    delete b;
    return ARA_OK;
}

// ------------------------------------------------------------------ serving
// The worker keeps two lanes -- a private context (stream, error word, staging) with its
// own slot layers, job and item arrays and sort workspace each -- and launches an
// iteration on a free lane as soon as requests are queued, without waiting for the
// other lane's iteration: requests that arrive while one iteration runs on the GPU are
// admitted into the next one, whose work is enqueued (and runs) alongside it.  A
// request's YLT lives in an arena shared by the lanes; it is admitted, in arrival
// order, when a slot of the lane is free and its YLT fits in the arena.  Iterations
// complete in launch order (the worker waits on each lane's completion event), so the
// arena works as a ring: requests take ranges at its head and give them back in the
// order they took them.
namespace {

struct ServerRequest {
    std::vector<int32_t> elts;
    ara_layer_terms terms;
    int64_t t0 = 0, t1 = 0;
    int64_t ylt_off = 0;        // its YLT: arena[ylt_off .. ylt_off + t1 - t0)
    std::vector<double> pml, tvar;
    ara_status status = ARA_OK;
    bool done = false;
    std::chrono::steady_clock::time_point submitted, finished;
};

// Contiguous ranges of doubles taken at the head of a ring and given back oldest first.
struct YltRing {
    int64_t cap = 0, head = 0, used = 0;
    std::deque<int64_t> spans;   // per live range: its length plus the end-of-ring gap skipped for it
    bool take(int64_t n, int64_t &off) {
        if (n > cap) return false;
        if (used == 0) head = 0;
        const int64_t skip = head + n > cap ? cap - head : 0;
        if (used + skip + n > cap) return false;
        off = skip ? 0 : head;
        head = off + n == cap ? 0 : off + n;
        used += skip + n;
        spans.push_back(skip + n);
        return true;
    }
    void give_oldest() {
        used -= spans.front();
        spans.pop_front();
    }
};

struct ServerLane {
    ara_ctx *pc = nullptr;            // private context: stream, error word, staging, options
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;        // recorded once the lane's results and error word are on the host
    std::vector<ara_layer *> slots;   // one request's tables each (member list: every pool ELT)
    BatchJob *d_jobs = nullptr, *h_jobs = nullptr;
    BatchItem *d_items = nullptr, *h_items = nullptr;
    int32_t item_cap = 0;
    int32_t mode_off[kBatchModes] = {}, mode_cnt[kBatchModes] = {};
    EltDesc *h_descs = nullptr;       // pinned: every slot's descriptors
    const double **d_ylts = nullptr, **h_ylts = nullptr;
    int64_t *d_ns = nullptr, *d_ks = nullptr, *h_nks = nullptr;   // h_nks: ns then ks, pinned
    double *d_res = nullptr, *h_res = nullptr;                    // [slot][2 * n_rp]
    void *ws = nullptr;               // radix sort workspace for the YET's length
    std::vector<ServerRequest *> reqs;   // the iteration in flight (empty: the lane is free)
    ara_status launch_status = ARA_OK;   // an error while enqueueing it (then its event is not waited on)
};

}  // namespace

struct ara_server {
    ara_ctx *ctx = nullptr;           // the caller's context (handles, slot layers)
    const ara_yet *yet = nullptr;
    std::vector<ara_elt *> pool;
    std::vector<double> rps;
    ServerLane lanes[2];
    std::deque<int> busy;             // lanes in flight, in launch order
    double *arena = nullptr;          // YLTs of admitted requests
    YltRing ring;
    int32_t slots_per_lane = 0;
    int64_t slot_bytes = 0;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::pair<uint64_t, ServerRequest *>> queue;
    std::map<uint64_t, ServerRequest *> live;
    uint64_t next_ticket = 1;
    bool stopping = false;
    int64_t iterations = 0, completed = 0, held = 0;
    int32_t max_seen = 0, in_flight = 0, max_in_flight = 0;
};

static constexpr int64_t kServerEventsPerItem = int64_t(1) << 18;

// Enqueues one iteration of requests `take` on lane `ln`: their layers' tables, one
// batched launch of their YLTs, their PML/TVaR, the copies of results and error word to
// the host, and the lane's completion event.  Nothing here waits for the device.
static ara_status server_launch(ara_server *sv, ServerLane &ln, const std::vector<ServerRequest *> &take) {
    ara_ctx *pc = ln.pc;
    const int32_t nr = int32_t(sv->rps.size());
    const size_t np = sv->pool.size();
    const int32_t nj = int32_t(take.size());
    const double mean_len = double(sv->yet->n_events) / double(std::max<int64_t>(1, sv->yet->n_trials));
    std::vector<std::pair<TiledArgs, int>> tiled;
    for (int32_t i = 0; i < nj; ++i) {
        ServerRequest *r = take[size_t(i)];
        ara_layer *L = ln.slots[size_t(i)];
        EltDesc *hd = ln.h_descs + size_t(i) * np;
        // the slot layer keeps its member list (every pool ELT, for the ELTs' user
        // counts); its descriptors, precision and terms become the request's
        bool all_f32 = !r->elts.empty();
        for (size_t k = 0; k < r->elts.size(); ++k) {
            const ara_elt *e = sv->pool[size_t(r->elts[k])];
            hd[k] = e->desc;
            all_f32 = all_f32 && e->prec == ARA_F32;
        }
        L->f32 = all_f32;
        L->terms = r->terms;
        const int n = int(r->elts.size());
        hipError_t e = hipMemcpyAsync(L->d_descs, hd, sizeof(EltDesc) * size_t(n), hipMemcpyHostToDevice, ln.stream);
        if (e == hipSuccess)
            e = launch_layer_tables(L->d_descs, n, L->catalog, L->f32, r->terms.occ_retention, r->terms.occ_limit, L->t,
                                    ln.stream);
        if (e != hipSuccess) return hip_fail(pc, e, "server layer build");
        TrialLaunch tl{};
        ara_status s = plan_trial(pc, L, r->t1 - r->t0, mean_len, tl, sv->yet->ids16 ? 1 : 0);
        if (s != ARA_OK) return s;
        double *ylt = sv->arena + r->ylt_off;
        BatchJob &h = ln.h_jobs[i];
        h.a = trial_args(sv->yet, L, r->t0, r->t1, ylt);
        h.a.err = pc->d_err;
        h.a.qcap = tl.qcap;
        h.mode = batch_mode(tl, h.a.ids24 != nullptr);
        h.placement = tl.placement;
        if (h.mode == kModeTiled) tiled.emplace_back(tiled_args(sv->yet, L, r->t0, r->t1, ylt, tl.grid), tl.grid);
        ln.h_ylts[i] = ylt;
    }
    std::vector<BatchItem> items;
    {
        std::vector<BatchJob> hj(ln.h_jobs, ln.h_jobs + nj);
        std::vector<int64_t> tb, te, ml(size_t(nj), std::max<int64_t>(1, int64_t(std::llround(mean_len))));
        for (ServerRequest *r : take) {
            tb.push_back(r->t0);
            te.push_back(r->t1);
        }
        items = group_items(hj, tb.data(), te.data(), ml, kServerEventsPerItem, ln.mode_off, ln.mode_cnt);
    }
    if (int32_t(items.size()) > ln.item_cap) return fail(pc, ARA_E_OOM, "server: %zu work items", items.size());
    std::copy(items.begin(), items.end(), ln.h_items);
    hipError_t e = hipMemcpyAsync(ln.d_jobs, ln.h_jobs, sizeof(BatchJob) * size_t(nj), hipMemcpyHostToDevice, ln.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ln.d_items, ln.h_items, sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice, ln.stream);
    if (e == hipSuccess)
        e = launch_grouped(ln.d_jobs, ln.d_items, ln.mode_off, ln.mode_cnt, pc->n_cu, true, ln.stream, tiled);
    // risk measures: ranks per request, short YLTs in one launch, long ones by radix
    // selection (nothing waits on the host here)
    int64_t *hn = ln.h_nks, *hk = ln.h_nks + sv->slots_per_lane;
    for (int32_t i = 0; i < nj; ++i) {
        const int64_t n = take[size_t(i)]->t1 - take[size_t(i)]->t0;
        hn[i] = n;
        for (int32_t r = 0; r < nr; ++r) (void)ara_return_period_rank(n, sv->rps[size_t(r)], &hk[size_t(i) * nr + r]);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(ln.d_ylts, ln.h_ylts, sizeof(double *) * size_t(nj), hipMemcpyHostToDevice, ln.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ln.d_ns, hn, 8 * size_t(nj), hipMemcpyHostToDevice, ln.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ln.d_ks, hk, 8 * size_t(nj) * nr, hipMemcpyHostToDevice, ln.stream);
    if (e == hipSuccess) e = launch_risk_batch(ln.d_ylts, ln.d_ns, ln.d_ks, nj, nr, ln.d_res, ln.stream);
    for (int32_t i = 0; i < nj && e == hipSuccess; ++i) {
        if (hn[i] <= kRiskLdsKeys) continue;
        e = launch_risk_select(ln.h_ylts[i], hn[i], ln.ws, &hk[size_t(i) * nr], nr, ln.d_res + size_t(i) * 2 * nr,
                               ln.stream);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(ln.h_res, ln.d_res, sizeof(double) * 2 * size_t(nr) * nj, hipMemcpyDeviceToHost, ln.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(pc->h_err, pc->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, ln.stream);
    if (e == hipSuccess) e = hipEventRecord(ln.done, ln.stream);
    return e == hipSuccess ? ARA_OK : hip_fail(pc, e, "server iteration");
}

// Completes lane ln's iteration (the oldest in flight; its event has completed, or
// enqueueing it failed): results to the requests, arena ranges back, the lane free.
static void server_finish(ara_server *sv, ServerLane &ln) {
    ara_ctx *pc = ln.pc;
    const int32_t nr = int32_t(sv->rps.size());
    ara_status s = ln.launch_status;
    if (s == ARA_OK) {
        const hipError_t e = hipEventSynchronize(ln.done);
        if (e != hipSuccess) s = hip_fail(pc, e, "server iteration");
    } else {
        (void)hipStreamSynchronize(ln.stream);
    }
    if (s == ARA_OK && *pc->h_err) s = sync_and_check(pc);   // reports and clears the device error word
    for (size_t i = 0; i < ln.reqs.size(); ++i) {
        ServerRequest *r = ln.reqs[i];
        if (s == ARA_OK) {
            r->pml.assign(ln.h_res + i * 2 * nr, ln.h_res + i * 2 * nr + nr);
            r->tvar.assign(ln.h_res + i * 2 * nr + nr, ln.h_res + i * 2 * nr + 2 * nr);
        }
    }
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        const auto now = std::chrono::steady_clock::now();
        for (ServerRequest *r : ln.reqs) {
            r->status = s;
            r->done = true;
            r->finished = now;
            sv->ring.give_oldest();
        }
        sv->iterations++;
        sv->completed += int64_t(ln.reqs.size());
        sv->in_flight -= int32_t(ln.reqs.size());
    }
    ln.reqs.clear();
    sv->cv_done.notify_all();
}

static void server_loop(ara_server *sv) {
    (void)hipSetDevice(sv->ctx->device);
    for (;;) {
        bool progressed = false;
        // the oldest iteration in flight, if its results are on the host (iterations are
        // completed in launch order: the arena's ranges return in the order taken)
        if (!sv->busy.empty()) {
            ServerLane &old = sv->lanes[sv->busy.front()];
            if (old.launch_status != ARA_OK || hipEventQuery(old.done) != hipErrorNotReady) {
                server_finish(sv, old);
                sv->busy.pop_front();
                progressed = true;
            }
        }
        int lane = -1;
        for (int k = 0; k < 2 && lane < 0; ++k)
            if (sv->lanes[k].reqs.empty()) lane = k;
        bool head_held = false;
        std::vector<ServerRequest *> take;
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            if (sv->stopping && sv->queue.empty() && sv->busy.empty()) return;
            // admission in arrival order: a free slot of the lane and room for the YLT
            while (lane >= 0 && !sv->queue.empty() && int32_t(take.size()) < sv->slots_per_lane) {
                ServerRequest *r = sv->queue.front().second;
                if (!sv->ring.take(r->t1 - r->t0, r->ylt_off)) {
                    head_held = true;
                    sv->held++;
                    break;
                }
                take.push_back(r);
                sv->queue.pop_front();
            }
            sv->in_flight += int32_t(take.size());
            sv->max_in_flight = std::max(sv->max_in_flight, sv->in_flight);
            sv->max_seen = std::max(sv->max_seen, int32_t(take.size()));
        }
        if (!take.empty()) {
            ServerLane &ln = sv->lanes[lane];
            ln.reqs = take;
            ln.launch_status = server_launch(sv, ln, take);
            sv->busy.push_back(lane);
            progressed = true;
        }
        if (progressed) continue;
        if (!sv->busy.empty()) {
            if (lane >= 0 && !head_held) {
                // a lane is free and nothing is queued: a new request wakes the worker at
                // once; otherwise look at the iteration in flight again shortly
                std::unique_lock<std::mutex> lk(sv->mu);
                sv->cv_work.wait_for(lk, std::chrono::microseconds(50),
                                     [&] { return sv->stopping || !sv->queue.empty(); });
            } else {
                // both lanes busy, or the next request waits for arena space: only the
                // oldest iteration's completion can let work proceed
                const ServerLane &old = sv->lanes[sv->busy.front()];
                if (old.launch_status == ARA_OK) (void)hipEventSynchronize(old.done);
            }
        } else {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_work.wait(lk, [&] { return sv->stopping || !sv->queue.empty(); });
        }
    }
}

static void server_free(ara_server *sv) {
    for (ServerLane &ln : sv->lanes) {
        for (ara_layer *L : ln.slots)
            if (L) ara_layer_release(L);
        dev_free(ln.d_jobs);
        dev_free(ln.d_items);
        dev_free(ln.d_ylts);
        dev_free(ln.d_ns);
        dev_free(ln.d_ks);
        dev_free(ln.d_res);
        dev_free(ln.ws);
        if (ln.h_jobs) (void)hipHostFree(ln.h_jobs);
        if (ln.h_items) (void)hipHostFree(ln.h_items);
        if (ln.h_descs) (void)hipHostFree(ln.h_descs);
        if (ln.h_ylts) (void)hipHostFree(ln.h_ylts);
        if (ln.h_nks) (void)hipHostFree(ln.h_nks);
        if (ln.h_res) (void)hipHostFree(ln.h_res);
        if (ln.done) (void)hipEventDestroy(ln.done);
        if (ln.pc) (void)ara_ctx_destroy(ln.pc);
        if (ln.stream) (void)hipStreamDestroy(ln.stream);
    }
    dev_free(sv->arena);
    for (auto &p : sv->live) delete p.second;
    delete sv;
}

// Device bytes of one slot: a layer's tables over the catalog and a descriptor per pool ELT.
static int64_t server_slot_bytes(int32_t C, int32_t n_pool) {
    const int64_t nblk = bitmap_blocks(C);
    return int64_t(C) * 8 * 3 + nblk * (16 + 16 + 4) + int64_t(align16(size_t(nblk) * 2)) +
           int64_t(align16(size_t(bitmap_supers(int32_t(nblk))) * 4)) + 64 +
           int64_t(n_pool) * int64_t(sizeof(EltDesc));
}

static ara_status server_lane_create(ara_ctx *c, ara_server *sv, ServerLane &ln, int32_t n_pool,
                                     const ara_server_config *cfg) {
    const ara_yet *y = sv->yet;
    const int32_t ns = sv->slots_per_lane;
    HIP_OR_RETURN(c, hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking), "server stream");
    HIP_OR_RETURN(c, hipEventCreateWithFlags(&ln.done, hipEventDisableTiming), "server event");
    ara_status s = ara_ctx_create(c->device, ln.stream, &ln.pc);
    if (s != ARA_OK) return fail(c, s, "server context: %s", ara_last_error(nullptr));
    ln.pc->placement = c->placement;
    ln.pc->block_threads = c->block_threads;
    ln.pc->grid_per_cu = c->grid_per_cu;
    ln.pc->trial_mode = c->trial_mode;
    ln.pc->yet_packing = c->yet_packing;
    const ara_layer_terms none{0.0, INFINITY, 0.0, INFINITY};
    ln.slots.assign(size_t(ns), nullptr);
    for (int32_t i = 0; i < ns && s == ARA_OK; ++i)
        s = ara_layer_create(c, sv->pool.data(), n_pool, y->catalog, &none, &ln.slots[size_t(i)]);
    if (s != ARA_OK) return s;
    // a worst case of work items: every slot with the YET's longest possible range
    const int64_t per_slot_items = y->n_trials / 16 + 2;
    ln.item_cap = int32_t(std::min<int64_t>(int64_t(ns) * per_slot_items, int64_t(1) << 30));
    const size_t nr = size_t(cfg->n_rp);
    s = dev_alloc(c, &ln.d_jobs, sizeof(BatchJob) * size_t(ns), "server jobs");
    if (s == ARA_OK) s = dev_alloc(c, &ln.d_items, sizeof(BatchItem) * size_t(ln.item_cap), "server items");
    if (s == ARA_OK) s = dev_alloc(c, &ln.d_ylts, sizeof(double *) * size_t(ns), "server ylt list");
    if (s == ARA_OK) s = dev_alloc(c, &ln.d_ns, 8 * size_t(ns), "server sizes");
    if (s == ARA_OK) s = dev_alloc(c, &ln.d_ks, 8 * size_t(ns) * nr, "server ranks");
    if (s == ARA_OK) s = dev_alloc(c, &ln.d_res, 16 * size_t(ns) * nr, "server results");
    if (s == ARA_OK) s = dev_alloc(c, &ln.ws, sort_workspace_bytes(y->n_trials), "server sort workspace");
    if (s != ARA_OK) return s;
    hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&ln.h_jobs), sizeof(BatchJob) * size_t(ns), hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&ln.h_items), sizeof(BatchItem) * size_t(ln.item_cap),
                          hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&ln.h_descs), sizeof(EltDesc) * size_t(ns) * sv->pool.size(),
                          hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&ln.h_ylts), sizeof(double *) * size_t(ns), hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&ln.h_nks), 8 * size_t(ns) * (1 + nr), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&ln.h_res), 16 * size_t(ns) * nr, hipHostMallocDefault);
    return e == hipSuccess ? ARA_OK : hip_fail(c, e, "server pinned staging");
}

extern "C" ara_status ara_server_create(ara_ctx *c, const ara_yet *y, ara_elt *const *pool, int32_t n_pool,
                                       const ara_server_config *cfg, ara_server **out) {
    if (!c || !out || !y || !cfg || !pool || n_pool < 1 || y->ctx != c) return ARA_E_INVALID_ARG;
    *out = nullptr;
    if (cfg->max_batch < 1 || cfg->n_rp < 1 || cfg->n_rp > 16 || !cfg->return_periods || cfg->memory_budget < 0)
        return fail(c, ARA_E_INVALID_ARG, "server: bad configuration");
    if (y->n_trials < 1) return fail(c, ARA_E_EMPTY, "server: the YET has no trials");
    for (int32_t r = 0; r < cfg->n_rp; ++r) {
        int64_t k = 0;
        if (ara_return_period_rank(1, cfg->return_periods[r], &k) != ARA_OK)
            return fail(c, ARA_E_INVALID_ARG, "server: return period %g invalid", cfg->return_periods[r]);
    }
    for (int32_t j = 0; j < n_pool; ++j)
        if (!pool[j] || pool[j]->ctx != c || pool[j]->catalog != y->catalog)
            return fail(c, ARA_E_INVALID_ARG, "server: pool ELT %d is NULL, of another context or catalog", j);
    HIP_OR_RETURN(c, hipSetDevice(c->device), "set device");
    // the budget: slots' tables (at most half of it) and the YLT arena (the rest)
    int64_t budget = cfg->memory_budget;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        HIP_OR_RETURN(c, hipMemGetInfo(&fr, &tot), "memory info");
        budget = int64_t(fr / 4);
    }
    const int64_t slot_bytes = server_slot_bytes(y->catalog, n_pool);
    const int32_t per_lane = int32_t(std::max<int64_t>(1, std::min<int64_t>(cfg->max_batch, budget / 2 / (2 * slot_bytes))));
    const int64_t arena = (budget - 2 * int64_t(per_lane) * slot_bytes) / 8;
    if (arena < 1)
        return fail(c, ARA_E_OOM, "server: two slots need %lld bytes, budget %lld", (long long)(2 * slot_bytes),
                    (long long)budget);
    ara_server *sv = new (std::nothrow) ara_server();
    if (!sv) return ARA_E_OOM;
    sv->ctx = c;
    sv->yet = y;
    sv->pool.assign(pool, pool + n_pool);
    sv->rps.assign(cfg->return_periods, cfg->return_periods + cfg->n_rp);
    sv->slots_per_lane = per_lane;
    sv->slot_bytes = slot_bytes;
    sv->ring.cap = arena;
    ara_status s = dev_alloc(c, &sv->arena, size_t(arena) * 8, "server ylt arena");
    for (int k = 0; k < 2 && s == ARA_OK; ++k) s = server_lane_create(c, sv, sv->lanes[k], n_pool, cfg);
    if (s == ARA_OK) {
        const hipError_t e = hipStreamSynchronize(c->stream);   // the slot layers' first builds
        if (e != hipSuccess) s = hip_fail(c, e, "server slot layers");
    }
    if (s != ARA_OK) {
        server_free(sv);
        return s;
    }
    try {
        sv->worker = std::thread(server_loop, sv);
    } catch (...) {
        server_free(sv);
        return fail(c, ARA_E_OOM, "server: cannot start the worker thread");
    }
    c->live++;
    *out = sv;
    return ARA_OK;
}

extern "C" ara_status ara_server_submit(ara_server *sv, const int32_t *idx, int32_t n_elts, const ara_layer_terms *terms,
                                       int64_t t0, int64_t t1, uint64_t *ticket) {
    if (!sv || !ticket || n_elts < 1 || !idx) return ARA_E_INVALID_ARG;
    if (n_elts > int32_t(sv->pool.size())) return ARA_E_INVALID_ARG;
    for (int32_t k = 0; k < n_elts; ++k)
        if (idx[k] < 0 || idx[k] >= int32_t(sv->pool.size())) return ARA_E_INVALID_ARG;
    if (ara_check_layer_terms(terms) != ARA_OK) return ARA_E_BAD_TERMS;
    if (t0 < 0 || t1 <= t0 || t1 > sv->yet->n_trials) return ARA_E_INVALID_ARG;
    if (t1 - t0 > sv->ring.cap) return ARA_E_OOM;   // its YLT alone exceeds the server's budget
    ServerRequest *r = new (std::nothrow) ServerRequest();
    if (!r) return ARA_E_OOM;
    r->elts.assign(idx, idx + n_elts);
    r->terms = *terms;
    r->t0 = t0;
    r->t1 = t1;
    r->submitted = std::chrono::steady_clock::now();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stopping) {
            delete r;
            return ARA_E_BUSY;
        }
        *ticket = sv->next_ticket++;
        sv->live[*ticket] = r;
        sv->queue.emplace_back(*ticket, r);
    }
    sv->cv_work.notify_one();
    return ARA_OK;
}

extern "C" ara_status ara_server_wait(ara_server *sv, uint64_t ticket, double *pml, double *tvar, double *seconds) {
    if (!sv) return ARA_E_INVALID_ARG;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->live.find(ticket);
    if (it == sv->live.end()) return ARA_E_INVALID_ARG;
    ServerRequest *r = it->second;
    sv->cv_done.wait(lk, [&] { return r->done; });
    sv->live.erase(it);
    lk.unlock();
    const ara_status s = r->status;
    if (s == ARA_OK) {
        if (pml) std::copy(r->pml.begin(), r->pml.end(), pml);
        if (tvar) std::copy(r->tvar.begin(), r->tvar.end(), tvar);
    }
    if (seconds) *seconds = std::chrono::duration<double>(r->finished - r->submitted).count();
    delete r;
    return s;
}

extern "C" ara_status ara_server_stats(ara_server *sv, ara_server_stats_t *st) {
    if (!sv || !st) return ARA_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(sv->mu);
    st->iterations = sv->iterations;
    st->completed = sv->completed;
    st->held = sv->held;
    st->max_in_iteration = sv->max_seen;
    st->max_in_flight = sv->max_in_flight;
    st->slots = 2 * sv->slots_per_lane;
    st->slot_bytes = sv->slot_bytes;
    st->arena_bytes = sv->ring.cap * 8;
    return ARA_OK;
}

extern "C" ara_status ara_server_release(ara_server *sv) {
    if (!sv) return ARA_E_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stopping = true;
    }
    sv->cv_work.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    ara_ctx *c = sv->ctx;
    (void)hipSetDevice(c->device);
    server_free(sv);
    c->live--;
    return ARA_OK;
}
