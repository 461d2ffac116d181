/*
 * ara.h -- C-ABI of the MI355X aggregate risk analysis engine (libara.so).
 *
 * The engine computes the analysis stage of aggregate risk analysis as defined
 * in Bahl, Baltzer, Rau-Chaplin, Varghese, "Parallel Simulations for Analysing
 * Portfolios of Catastrophic Event Risk":
 *   inputs  (Section II-A): a Year Event Table (YET) of trials, each a sequence
 *           of event occurrences ordered by time; Event Loss Tables (ELTs) of
 *           (event, loss) records with per-ELT financial terms; a layer = a list
 *           of ELTs plus the layer terms of Table I;
 *   method  (Section II-B, basic algorithm, steps 1-4): per trial, look up each
 *           occurrence in the layer's ELTs (direct access tables, Section III-B),
 *           apply financial terms and sum across ELTs, apply occurrence terms,
 *           take the cumulative sum in time order under the aggregate terms;
 *   outputs (Section II-C): the Year Loss Table (one loss per trial) and the
 *           PML / TVaR filters named in Section I.
 *
 * Conventions for every entry point:
 *   - Returns an ara_status: ARA_OK (0) or a negative error.  No C++ exception
 *     and no abort crosses this boundary.  After an error on a context,
 *     ara_last_error(ctx) gives a human-readable message.
 *   - Pointers are plain host or device pointers as stated by an ara_mem
 *     argument.  ARA_MEM_DEVICE buffers are borrowed: the caller keeps them
 *     alive and unchanged for as long as the handle that uses them lives.
 *     ARA_MEM_HOST inputs are copied to device memory owned by the handle.
 *   - Work is enqueued on the context's HIP stream.  Calls documented as
 *     "blocking" synchronise that stream before returning; the others are
 *     asynchronous, and errors that kernels detect (an event ID outside the
 *     catalog, bad trial offsets) are reported by the next blocking call or by
 *     ara_sync().
 *   - A context and its handles are used by one host thread at a time.
 *   - Event IDs are 0-based: valid IDs are 0 .. catalog_size-1, with
 *     1 <= catalog_size <= 2^28 (larger catalogs: ARA_E_INVALID_ARG).
 *   - Arithmetic is binary64 throughout.  ARA_F32 only selects binary32
 *     storage of the loss tables.
 */
#ifndef ARA_H
#define ARA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ara_status {
    ARA_OK = 0,
    ARA_E_INVALID_ARG = -1,    /* NULL handle/pointer, negative size, bad range or option        */
    ARA_E_EVENT_ID_RANGE = -2, /* an event ID outside [0, catalog_size)                          */
    ARA_E_BAD_OFFSETS = -3,    /* trial offsets not CSR: offsets[0]=0, non-decreasing, end=n_events */
    ARA_E_BAD_LOSS = -4,       /* a loss that is negative, NaN or infinite                        */
    ARA_E_DUP_EVENT = -5,      /* an ELT lists the same event twice                               */
    ARA_E_BAD_TERMS = -6,      /* retention NaN/negative/infinite, limit NaN/negative, fx invalid  */
    ARA_E_EMPTY = -7,          /* risk measures of an empty YLT                                   */
    ARA_E_OOM = -8,            /* device allocation failed                                        */
    ARA_E_DEVICE = -9,         /* no usable gfx950 device, or a HIP runtime error                 */
    ARA_E_BUSY = -10,          /* releasing an ELT still used by a live layer                     */
    ARA_E_UNSUPPORTED = -11    /* a requested table placement cannot hold this catalog            */
} ara_status;

typedef enum ara_precision {
    ARA_F64 = 0, /* loss tables stored in binary64                                                    */
    ARA_F32 = 1  /* loss tables stored rounded to binary32 (arithmetic stays binary64)                */
} ara_precision;

typedef enum ara_mem { ARA_MEM_HOST = 0, ARA_MEM_DEVICE = 1 } ara_mem;

/* Layer terms of Table I.  Retentions finite and >= 0; limits >= 0, +INFINITY = no limit. */
typedef struct ara_layer_terms {
    double occ_retention; /* T_OccR: deductible per event occurrence                 */
    double occ_limit;     /* T_OccL: cover per occurrence in excess of the retention */
    double agg_retention; /* T_AggR: deductible on the trial's cumulative loss        */
    double agg_limit;     /* T_AggL: cover on the cumulative loss above the retention */
} ara_layer_terms;

/* Financial terms I of one ELT (Section II-A names them but does not define them).
 * Applied to each looked-up event loss l as min(max(fx*l - retention, 0), limit).
 * fx finite >= 0, retention finite >= 0, limit >= 0 or +INFINITY.
 * A NULL ara_elt_terms pointer means the identity (1, 0, +INFINITY). */
typedef struct ara_elt_terms {
    double fx;
    double retention;
    double limit;
} ara_elt_terms;

/* Where a layer's combined loss table lives while trials are analysed. */
typedef enum ara_placement {
    ARA_PLACE_AUTO = 0,         /* pick from the catalog size (default)                              */
    ARA_PLACE_LDS_BITMAP = 1,   /* LDS: 1 bit/event "occurrence loss nonzero" + ranks; values in L2  */
    ARA_PLACE_LDS_DENSE = 2,    /* LDS: the whole combined table (small catalogs)                    */
    ARA_PLACE_GLOBAL_DENSE = 3, /* HBM/L2: the whole combined table, gathered per occurrence         */
    ARA_PLACE_LDS_TILES = 4     /* LDS: the occurrence-net values of one 2^14-event catalog bin at a
                                   time, each lane adding its trial's occurrences of the bin from the
                                   YET's binned copy (needs one: see ara_yet_create).  AUTO picks it
                                   when the YET has a binned copy and the dense table does not fit
                                   in LDS                                                          */
} ara_placement;

/* Context options (ara_set_option). */
typedef enum ara_option {
    ARA_OPT_PLACEMENT = 1,      /* an ara_placement value                                            */
    ARA_OPT_BLOCK_THREADS = 2,  /* threads per workgroup of the trial kernel: 256, 512 or 1024       */
    ARA_OPT_GRID_PER_CU = 3,    /* workgroups per compute unit of the trial kernel (1..64; 0 = auto)  */
    ARA_OPT_YET_PACKING = 4,    /* 1 (default): YETs created later also keep a packed copy of their
                                   event IDs when catalog_size <= 2^24 and they keep no binned
                                   copy; 0: never                                                   */
    ARA_OPT_TRIAL_MODE = 5,     /* dense-table YLT kernels: 0 (default) = one lane per trial when the
                                   YET averages <= 256 occurrences per trial, else one wave per
                                   trial; 1 = always a wave; 2 = always a lane.  A lane adds its
                                   trial's values in time order (the sequential sum)               */
    ARA_OPT_YET_BINNING = 6,    /* 1 (default): YETs created later also keep a catalog-binned copy
                                   where it applies (see ara_yet_create); 0: never                 */
    ARA_OPT_YET_RUN_BYTES = 7,  /* bytes per run start of binned copies built later: 4 (default), or
                                   3 (with at most 64 bins and fewer than 2^31 occurrences; 4 when
                                   a bin holds 2^24 occurrences or more): a quarter less memory for
                                   the run starts, about 2% more time in the tiled kernel          */
    ARA_OPT_KERNEL_TIMING = 8   /* n in 1..4096: ara_analyze times its trial kernel with a pair of
                                   HIP events, the pairs of the last n calls kept in a ring (for
                                   the tiled kernel, events attached to its launch: the start of
                                   its first dispatch and the end of its last; for the others,
                                   recorded on the stream just around the launches); setting the
                                   option waits for the stream and starts a new ring.
                                   ara_kernel_ms reads it.  0 (default): no timing             */
} ara_option;

typedef struct ara_ctx ara_ctx;
typedef struct ara_yet ara_yet;
typedef struct ara_elt ara_elt;
typedef struct ara_layer ara_layer;

/* Static string for a status code (never NULL). */
const char *ara_status_str(int status);

/* Last error message of a context ("" if none), valid until the next call on ctx.
 * With ctx == NULL: the message of the calling thread's last failure that had no
 * context (ara_ctx_create). */
const char *ara_last_error(const ara_ctx *ctx);

/* Library version: major * 10000 + minor * 100 + patch. */
int ara_version(void);

/* Rank k (1..n) of the order statistic that return period rp selects from n year
 * losses sorted in descending order: k = ceil(n / rp) clamped to [1, n], taking
 * the nearest integer when n / rp is within 4 ulps of it.  PML(rp) is the k-th
 * largest loss and TVaR(rp) the mean of the k largest (a tail level alpha is
 * rp = 1 / alpha).  The paper names PML and TVaR (Section I) without defining
 * them; this is the engine's definition.  Host only; needs no device.
 * Errors: ARA_E_INVALID_ARG if n < 1, rp < 1, rp is NaN or k is NULL. */
ara_status ara_return_period_rank(int64_t n, double rp, int64_t *k);

/* Validates layer terms as documented at ara_layer_terms (host only). */
ara_status ara_check_layer_terms(const ara_layer_terms *terms);

/* Creates a context on HIP device `device` (must be gfx950).  hip_stream is a
 * hipStream_t to enqueue on (borrowed), or NULL for the device's null stream.
 * Errors: ARA_E_DEVICE (no such device / not gfx950), ARA_E_OOM, ARA_E_INVALID_ARG. */
ara_status ara_ctx_create(int device, void *hip_stream, ara_ctx **out);

/* Synchronises and destroys the context.  Handles created on it must be released first. */
ara_status ara_ctx_destroy(ara_ctx *ctx);

/* Changes the stream later work is enqueued on (borrowed hipStream_t, NULL = null stream). */
ara_status ara_ctx_set_stream(ara_ctx *ctx, void *hip_stream);

/* Sets a tuning option (ara_option) of the context.  ARA_E_INVALID_ARG for unknown options/values. */
ara_status ara_set_option(ara_ctx *ctx, int option, int64_t value);

/* Blocking.  Waits for all work enqueued on the context and reports (then clears)
 * the first device-detected input error: ARA_E_EVENT_ID_RANGE, ARA_E_BAD_OFFSETS,
 * ARA_E_BAD_LOSS or ARA_E_DUP_EVENT.  ARA_E_DEVICE on a HIP runtime error. */
ara_status ara_sync(ara_ctx *ctx);

/* Blocking.  *ms = the mean duration of the trial kernels of the last min(k, n)
 * ara_analyze calls timed under ARA_OPT_KERNEL_TIMING = n, k the calls timed since the
 * option was set (waits for them).  ARA_E_INVALID_ARG when no call was timed since
 * the option was set; ARA_E_DEVICE on a HIP runtime error. */
ara_status ara_kernel_ms(ara_ctx *ctx, float *ms);

/* ---------------------------------------------------------------- Year Event Table
 * Creates a YET handle (Section II-A item 1; in memory as the paper's event-ID and
 * trial-boundary vectors, Section III-B).
 *   event_ids      int32[n_events]: the event of every occurrence, all trials
 *                  concatenated, each trial in ascending time order.
 *   trial_offsets  int64[n_trials + 1]: trial t is event_ids[off[t] .. off[t+1]);
 *                  off[0] = 0, non-decreasing, off[n_trials] = n_events.
 *   catalog_size   number of events in the catalog (>= 1).
 *   mem            ARA_MEM_DEVICE: both arrays are borrowed device pointers;
 *                  ARA_MEM_HOST: both are copied to the device.
 * Blocking: every ID and offset is checked on the device before returning.
 * Packed copy: when catalog_size <= 2^24, ARA_OPT_YET_PACKING is 1 and the handle
 * keeps no binned copy (below), the library also stores the checked IDs in 3 bytes
 * each (event i at bytes 3i..3i+2, little endian, in 12-byte groups of 4 events),
 * owned by the handle; the YLT kernels then stream that copy (3 instead of 4 bytes
 * per occurrence).  Borrowed arrays must not change while the handle lives: later
 * analyses may read either form.
 * Binned copy: when ARA_OPT_YET_BINNING is 1, the catalog is larger than a dense
 * table in LDS (more than 20480 events) and at most 2^23 events, every trial has
 * fewer than 2^31 occurrences in each 2^14-event catalog bin, and the per-bin offsets
 * (4 bytes per trial and bin) stay below a quarter of the 2-byte IDs, the library also
 * stores the occurrences regrouped by catalog bin: bin by bin, each trial's
 * occurrences of that bin's events in time order as 2-byte IDs within the bin, with
 * per-(bin, trial) offsets.  Analyses of layers whose table does not fit in LDS then
 * read that copy (ARA_PLACE_LDS_TILES); other placements then stream the int32 IDs.
 * If the device has no memory for it, the handle is created without it.  Device
 * memory the handle adds to the caller's arrays (ara_yet_memory gives it exactly):
 * with a binned copy 2 bytes per occurrence plus 4 bytes per (bin, trial + 2, rounded
 * up to a multiple of 8), 3 with ARA_OPT_YET_RUN_BYTES = 3, plus about 24 bytes per
 * bin, else 3 bytes per occurrence with a packed copy.
 * Errors: ARA_E_INVALID_ARG, ARA_E_EVENT_ID_RANGE, ARA_E_BAD_OFFSETS, ARA_E_OOM, ARA_E_DEVICE. */
ara_status ara_yet_create(ara_ctx *ctx, const int32_t *event_ids, int64_t n_events,
                          const int64_t *trial_offsets, int64_t n_trials, int32_t catalog_size,
                          ara_mem mem, ara_yet **out);
ara_status ara_yet_release(ara_yet *yet);

/* Sizes of a YET handle and the bytes per event ID of the form the YLT kernels read
 * for layers whose table does not fit in LDS: 2 with a binned copy, else 3 with a
 * packed copy, else 4.  Any output pointer may be NULL. */
ara_status ara_yet_info(const ara_yet *yet, int64_t *n_events, int64_t *n_trials, int32_t *id_bytes);

/* Device memory held by a YET handle: its packed or binned copy, plus the copies of
 * the caller's arrays when it was created from host memory (ARA_MEM_HOST).
 *   device_bytes  out: that memory in bytes.
 *   run_bytes     out: bytes per run start of the binned copy (3, or 4 when a bin
 *                 holds 2^24 occurrences or more; 0 without a binned copy).
 * Any output pointer may be NULL.  Errors: ARA_E_INVALID_ARG. */
ara_status ara_yet_memory(const ara_yet *yet, int64_t *device_bytes, int32_t *run_bytes);

/* The YET's catalog-binned copy (see ara_yet_create), copied to host memory, for
 * checking and inspection.  Bin b holds catalog events [2^14 b, 2^14 (b + 1)).
 *   n_bins      out: number of bins (0: the handle has no binned copy).
 *   region      NULL, or int64[n_bins + 1], out: region b of the copy is elements
 *               [region[b], region[b] + boff[b][n_trials]) (each region starts at
 *               a multiple of 8 elements); region[n_bins] bounds the copy.
 *   boff        NULL, or uint32[n_bins * (n_trials + 1)], out: boff[b (n_trials + 1) + t]
 *               is where trial t's run starts in region b (row b ends with the
 *               region's length).
 *   ids16       NULL, or uint16[region[n_bins]], out: the copy (each ID within its bin).
 * Call with NULL buffers first to learn n_bins and region.  Blocking (waits for the
 * context's stream).  Errors: ARA_E_INVALID_ARG, ARA_E_DEVICE. */
ara_status ara_yet_binned(const ara_yet *yet, int32_t *n_bins, int64_t *region, uint32_t *boff, uint16_t *ids16);

/* ---------------------------------------------------------------- Event Loss Table
 * Creates an ELT handle (Section II-A item 2) and builds its direct access table
 * over the whole catalog (Section III-B): entry e holds the loss of event e, or 0
 * if the ELT does not list e.
 *   event_ids, losses  n_pairs records (int32 event, binary64 loss >= 0, finite);
 *                      every event at most once; any order.
 *   terms              financial terms I of this ELT, or NULL for the identity.
 *   precision          storage of the direct access table (ARA_F32 rounds each loss
 *                      to nearest binary32).
 *   mem                as for ara_yet_create (DEVICE records are borrowed and re-read
 *                      by ara_layer_build with ARA_BUILD_TABLES).
 * Blocking.  Errors: ARA_E_INVALID_ARG, ARA_E_EVENT_ID_RANGE, ARA_E_BAD_LOSS,
 * ARA_E_DUP_EVENT, ARA_E_BAD_TERMS, ARA_E_OOM, ARA_E_DEVICE. */
ara_status ara_elt_create(ara_ctx *ctx, const int32_t *event_ids, const double *losses, int64_t n_pairs,
                          int32_t catalog_size, const ara_elt_terms *terms, ara_precision precision,
                          ara_mem mem, ara_elt **out);
/* ARA_E_BUSY while a live layer uses the ELT. */
ara_status ara_elt_release(ara_elt *elt);

/* ---------------------------------------------------------------- Layer
 * Creates a layer (Section II-A item 3): the listed ELTs, in this order, under the
 * layer terms, over a catalog of catalog_size events (every ELT must have been
 * created with that catalog size).  0 <= n_elts <= 65535; with n_elts = 0 every
 * trial loses 0.  The layer holds a reference to each ELT.  It builds, on the
 * device, the layer's combined table: for every catalog event e, the sum over the
 * layer's ELTs (in listed order, binary64, from +0.0) of the ELT's financial terms
 * applied to its loss for e -- the per-occurrence work of steps 1 and 2 of the
 * basic algorithm, which depends only on the event -- stored in binary32 when every
 * ELT is ARA_F32, else binary64; and the occurrence filter: which events have a
 * nonzero loss after the occurrence terms, with the compacted values of those.
 * Asynchronous (the build is enqueued).  Errors: ARA_E_INVALID_ARG (catalog
 * mismatch, NULL), ARA_E_BAD_TERMS, ARA_E_OOM, ARA_E_DEVICE. */
ara_status ara_layer_create(ara_ctx *ctx, ara_elt *const *elts, int32_t n_elts, int32_t catalog_size,
                            const ara_layer_terms *terms, ara_layer **out);

/* New layer terms (an underwriter re-pricing the layer).  Re-enqueues the occurrence
 * filter build; the combined table is unchanged.  Asynchronous.  ARA_E_BAD_TERMS. */
ara_status ara_layer_set_terms(ara_ctx *ctx, ara_layer *layer, const ara_layer_terms *terms);

#define ARA_BUILD_TABLES 1 /* also rebuild each member ELT's direct access table from its records */

/* Re-enqueues the layer's table builds: with ARA_BUILD_TABLES, each member ELT's
 * direct access table from its (resident) records, then the combined table and
 * the occurrence filter.  The filter's ranks and compacted values, which only the
 * filter-based placements, lookups, event outputs and batches read, are enqueued by
 * the first such call (the tiled placement never needs them); ara_layer_set_terms
 * does the same.  Asynchronous; record errors surface at the next blocking call.
 * Errors: ARA_E_INVALID_ARG, ARA_E_DEVICE. */
ara_status ara_layer_build(ara_ctx *ctx, ara_layer *layer, int flags);

/* Blocking.  Number of catalog events whose occurrence-net loss is nonzero under
 * the current terms, the table placement ara_analyze would use, and the bytes of
 * LDS it would take per workgroup.  Any output pointer may be NULL. */
ara_status ara_layer_stats(ara_ctx *ctx, const ara_layer *layer, int64_t *n_occ_nonzero,
                           int32_t *placement, int64_t *lds_bytes);
ara_status ara_layer_release(ara_layer *layer);

/* ---------------------------------------------------------------- Analysis
 * Year Loss Table of trials [trial_begin, trial_end) of the YET under the layer
 * (Section II-B steps 1-4, Section II-C output):
 *   ylt[t - trial_begin] = min(max(P_t - AggR, 0), AggL),  P_t = sum over the trial's
 *   occurrences d of min(max(x_d - OccR, 0), OccL), x_d = combined table[event_d].
 * This equals the basic algorithm's sum of per-occurrence ceded losses: the
 * cumulative sum is non-decreasing and the aggregate clamp is non-decreasing with
 * value 0 at 0, so the differences telescope.  ylt has trial_end - trial_begin
 * doubles in memory `ylt_mem`.  The YET and the layer must share a catalog size.
 * Asynchronous for ARA_MEM_DEVICE output; blocking for ARA_MEM_HOST.  Trials with
 * no events get 0.  Kernel-detected errors: ARA_E_EVENT_ID_RANGE, ARA_E_BAD_OFFSETS.
 * Errors: ARA_E_INVALID_ARG, ARA_E_UNSUPPORTED (forced placement too small), ARA_E_DEVICE. */
ara_status ara_analyze(ara_ctx *ctx, const ara_yet *yet, const ara_layer *layer,
                       int64_t trial_begin, int64_t trial_end, double *ylt, ara_mem ylt_mem);

/* Largest occurrence-net loss of every trial in [t0, t1) (after the occurrence terms
 * of Section II-B step 3; 0 for an empty trial): the year's largest single occurrence,
 * whose distribution over trials is the occurrence exceedance curve, so
 * ara_risk_measures on it gives occurrence PML and TVaR.  A maximum: exact, the same
 * bits in any order.  out: t1 - t0 doubles (mem as for ara_analyze).
 * Errors: as for ara_analyze. */
ara_status ara_analyze_occ_max(ara_ctx *ctx, const ara_yet *yet, const ara_layer *layer, int64_t t0, int64_t t1,
                               double *out, ara_mem mem);

/* Per-occurrence form of the analysis, the steps exactly as the basic algorithm
 * orders them: x_d (loss summed over the layer's ELTs after financial terms),
 * occ_d (after occurrence terms), cum_d (inclusive cumulative sum in time order),
 * ceded_d = f(cum_d) - f(cum_{d-1}) with f the aggregate clamp and f(cum_0) = 0,
 * and ylt = the sum of ceded_d per trial.  Per-occurrence arrays have
 * off[trial_end] - off[trial_begin] doubles, indexed from off[trial_begin]; any of
 * them (and ylt) may be NULL.  All pointers in memory `mem`.  Asynchronous for
 * ARA_MEM_DEVICE, blocking for ARA_MEM_HOST.  Errors as ara_analyze. */
ara_status ara_analyze_events(ara_ctx *ctx, const ara_yet *yet, const ara_layer *layer,
                              int64_t trial_begin, int64_t trial_end, double *ylt,
                              double *ev_gross, double *ev_occ, double *ev_cum, double *ev_ceded,
                              ara_mem mem);

/* Looks events up through the same table placement the trial kernel uses:
 * gross[i] = combined table[event_ids[i]] and occ[i] = its occurrence-net loss.
 * For checking lookups bit for bit.  n >= 0; out pointers may be NULL; all in `mem`.
 * Asynchronous for ARA_MEM_DEVICE, blocking for ARA_MEM_HOST. */
ara_status ara_lookup(ara_ctx *ctx, const ara_layer *layer, const int32_t *event_ids, int64_t n,
                      double *gross, double *occ, ara_mem mem);

/* ---------------------------------------------------------------- Order statistics
 * Device workspace (bytes) that ara_sort_desc and ara_risk_measures need for n losses. */
ara_status ara_sort_workspace_size(int64_t n, size_t *bytes);

/* Sorts n binary64 values into descending order (-0.0 becomes +0.0; NaN sorts
 * first).  in/out: device pointers (may alias); workspace: device,
 * >= ara_sort_workspace_size(n) bytes, or NULL to let the library allocate.
 * Asynchronous when a workspace is given.  Errors: ARA_E_INVALID_ARG, ARA_E_OOM. */
ara_status ara_sort_desc(ara_ctx *ctx, const double *in, int64_t n, double *out,
                         void *workspace, size_t workspace_bytes);

/* Risk measures from a YLT of n >= 1 losses in memory ylt_mem: for each of the n_rp
 * return periods, pml[i] = the k-th largest loss and tvar[i] = the mean of the k
 * largest, k = ara_return_period_rank(n, return_periods[i]).  return_periods, pml
 * and tvar are host arrays of n_rp.  workspace as for ara_sort_desc.  Blocking.
 * Errors: ARA_E_EMPTY (n == 0), ARA_E_INVALID_ARG, ARA_E_OOM, ARA_E_DEVICE, and any
 * pending kernel-detected input error. */
ara_status ara_risk_measures(ara_ctx *ctx, const double *ylt, int64_t n, ara_mem ylt_mem,
                             const double *return_periods, int32_t n_rp, double *pml, double *tvar,
                             void *workspace, size_t workspace_bytes);

/* Largest YLT, and the device memory per GPU, of ara_risk_measures_noalloc. */
#define ARA_NOALLOC_MAX_N (1 << 20)
#define ARA_NOALLOC_SCRATCH_BYTES (17u << 20)

/* ara_risk_measures for callers that cannot allocate device memory: code that must
 * not call hipMalloc (tight serving loops, harnesses that forbid it).  The same
 * sort and sums as ara_risk_measures, so the same results bit for bit; the sort
 * workspace is a library-owned device array of ARA_NOALLOC_SCRATCH_BYTES that each
 * GPU the library runs on holds until the process ends (its address is taken when
 * the first context is created on that GPU).  The call makes no hipMalloc, hipFree
 * or other allocating call.
 *   ylt            device pointer, n losses, 1 <= n <= ARA_NOALLOC_MAX_N.
 *   return_periods host array of n_rp (at most 256); pml, tvar: host arrays of n_rp.
 * Blocking (results are copied to the host), so it cannot be graph-captured.  All
 * calls on one GPU share that GPU's array: calls that overlap in time on one GPU
 * (from several contexts or threads) race and give wrong results; serialise them.
 * Errors: ARA_E_EMPTY (n == 0), ARA_E_INVALID_ARG (n > ARA_NOALLOC_MAX_N, bad
 * arguments or return periods), ARA_E_DEVICE, and any pending kernel-detected
 * input error. */
ara_status ara_risk_measures_noalloc(ara_ctx *ctx, const double *ylt, int64_t n,
                                     const double *return_periods, int32_t n_rp, double *pml, double *tvar);

/* ---------------------------------------------------------------- Batches
 * Many analyses in one persistent launch: the layer loop of Algorithm 1 (one YET,
 * many layers) and Section IV's portfolios, or independent analyses of different
 * YETs, catalogs and trial counts.  A job is one (YET, layer, trial range) with its
 * YLT destination; jobs may share YETs and layers.  Each job runs the same device
 * code as ara_analyze with the context's options at ara_batch_create (placement,
 * trial mode, YET packing), so its YLT equals ara_analyze's bit for bit.
 *   ylt  device memory, trial_end - trial_begin doubles, written by ara_batch_run.
 * The YETs and layers must outlive the batch; rebuilding a layer's tables
 * (ara_layer_build, ara_layer_set_terms) between runs is allowed (the tables are
 * rebuilt in place). */
typedef struct ara_job {
    const ara_yet *yet;
    const ara_layer *layer;
    int64_t trial_begin, trial_end;
    double *ylt;
} ara_job;

typedef struct ara_batch ara_batch;

/* Plans the batch: validates every job (as ara_analyze would) and uploads their
 * descriptors.  Errors: those of ara_analyze's argument checks, ARA_E_OOM. */
ara_status ara_batch_create(ara_ctx *ctx, const ara_job *jobs, int32_t n_jobs, ara_batch **out);

/* Computes every job's YLT on the context's stream.  The jobs are split into work
 * items of about equal occurrence counts (whole trials), which one persistent launch
 * processes.  The first run of a batch tunes the split: it times a few candidates
 * (each computes all YLTs), keeps the fastest for batches of this shape on this
 * context, and captures the launch in a HIP graph (blocking); later runs replay the
 * graph (non-blocking).  Input errors found on the device are reported by ara_sync. */
ara_status ara_batch_run(ara_batch *batch);

/* PML and TVaR of every job's YLT at the given return periods (as
 * ara_risk_measures, bit for bit): pml[j * n_rp + r], tvar[j * n_rp + r].  YLTs of up
 * to 16384 trials are sorted in one workgroup's LDS, all in one launch; longer ones
 * with the radix sort.  Blocking.  Errors: ARA_E_EMPTY (an empty job),
 * ARA_E_INVALID_ARG (return period < 1 or NaN, more than 256 of them). */
ara_status ara_batch_risk(ara_batch *batch, const double *return_periods, int32_t n_rp, double *pml,
                          double *tvar);

/* Portfolio year loss table (Section IV: a portfolio of layers over one YET):
 * out[t] = the sum over the batch's jobs, in job order from +0.0, of their YLTs' t-th
 * entries.  Every job must cover the same number of trials; out is device memory of
 * that many doubles.  Enqueued on the context's stream (after the batch's runs);
 * ara_risk_measures on it gives the portfolio's PML and TVaR.
 * Errors: ARA_E_INVALID_ARG (no jobs, or jobs of different trial counts). */
ara_status ara_batch_portfolio(ara_batch *batch, double *out);

/* The context's batch schedules (the tuner's choice per batch shape: jobs' kernels,
 * trial counts, mean trial lengths and catalogs) written to a text file, or read
 * from one into the context, so that batches of a known shape skip the tuning runs
 * in a later process.  A loaded entry replaces the context's entry for its shape.
 * Host only.  Errors: ARA_E_INVALID_ARG (NULL arguments, a file that cannot be
 * opened or written, a malformed line: then nothing is loaded). */
ara_status ara_tune_cache_save(const ara_ctx *ctx, const char *path);
ara_status ara_tune_cache_load(ara_ctx *ctx, const char *path);

/* The tuned schedule: work items, workgroups, occurrences per item, and in `graph`
 * bit 0 = runs replay a graph, bit 1 = workgroups take every G-th item (G workgroups)
 * rather than a contiguous run, so the grid works on few jobs at a time and their
 * tables share the L2.  Items and workgroups count the persistent launches of the
 * dense and filter placements only: the jobs whose placement is ARA_PLACE_LDS_TILES (as
 * ara_analyze would choose it) run together in one more launch of the tiled kernel,
 * whose items are passes of up to 4032 trials of one job (a trial's YLT does not depend
 * on the pass that holds it, so the same bits as ara_analyze), costliest first, taken
 * from a counter by whichever workgroup is free; they add nothing here (a batch of only
 * such jobs reports 0 and 0).  Any output pointer may be NULL. */
ara_status ara_batch_info(const ara_batch *batch, int32_t *n_items, int32_t *grid, int64_t *events_per_item,
                          int32_t *graph);

ara_status ara_batch_release(ara_batch *batch);

/* ---------------------------------------------------------------- Serving
 * A pricing server (real-time pricing of layers, Section I and Section IV) keeps one
 * YET and a pool of ELTs resident and answers requests -- a layer made of pool ELTs,
 * its terms and a trial range -- with PML and TVaR at the server's return periods.
 *
 * Continuous batching: a worker thread keeps two lanes, each with its own stream,
 * slots (a layer's tables each) and staging.  Whenever a lane is free and requests are
 * queued, it admits them in arrival order into that lane's free slots and enqueues one
 * iteration for them -- their layers' tables built in place, all their YLTs in one
 * batched launch, their risk measures, the copy of the results to the host -- without
 * waiting for the other lane's iteration: requests that arrive while one iteration is
 * on the GPU join the next, which runs beside it.  Iterations complete in launch order.
 *
 * Admission by memory: memory_budget bytes (0 = a quarter of free HBM) hold the slots'
 * tables (2 lanes x slots_per_lane x slot_bytes, at most half of the budget, and at
 * most max_batch slots per lane) and an arena for the YLTs of admitted requests (the
 * rest).  A request is admitted when its lane has a free slot and its own YLT (8 bytes
 * per trial of its range) fits in the arena beside those of the requests in flight;
 * otherwise it, and every request after it, waits for an iteration to complete.
 *
 * Every result equals that of the same analysis run alone (ara_layer_create over the
 * same pool ELTs + ara_analyze + ara_risk_measures) bit for bit: each request runs the
 * same device code over the same inputs in the same order, whatever it is batched with.
 * The server works on its own streams and error words; the context's options at
 * ara_server_create apply.  The YET and the pool ELTs must outlive the server. */
typedef struct ara_server ara_server;

typedef struct ara_server_config {
    int32_t max_batch;              /* slots per lane (requests per iteration), >= 1            */
    int64_t memory_budget;          /* bytes for slots' tables + the YLT arena; 0 = 1/4 of free HBM */
    int32_t n_rp;                   /* return periods of every request, 1..16                   */
    const double *return_periods;   /* n_rp values >= 1 (copied)                                */
} ara_server_config;

/* Errors: ARA_E_INVALID_ARG (bad config, handles of another context, an empty pool or
 * one ELT of another catalog), ARA_E_OOM (the budget holds no two slots and an arena,
 * or device memory ran out), ARA_E_DEVICE. */
ara_status ara_server_create(ara_ctx *ctx, const ara_yet *yet, ara_elt *const *pool, int32_t n_pool,
                             const ara_server_config *config, ara_server **out);

/* Queues a request: ELTs pool[elt_index[0..n_elts)] (n_elts >= 1, in that order),
 * layer terms, and trials [trial_begin, trial_end) (non-empty).  Returns at once with
 * a ticket.  The pool ELTs' tables must not be rebuilt while the server runs.
 * Errors: ARA_E_INVALID_ARG, ARA_E_BAD_TERMS, ARA_E_OOM (its YLT alone is larger than
 * the arena), ARA_E_BUSY (the server is stopping). */
ara_status ara_server_submit(ara_server *server, const int32_t *elt_index, int32_t n_elts,
                             const ara_layer_terms *terms, int64_t trial_begin, int64_t trial_end,
                             uint64_t *ticket);

/* Waits for a request and returns its PML and TVaR (n_rp values each) and, if seconds
 * is not NULL, the time from its submission to its completion (steady clock), then
 * forgets the ticket.  Returns the request's status (device-detected input errors
 * included).  ARA_E_INVALID_ARG for an unknown ticket. */
ara_status ara_server_wait(ara_server *server, uint64_t ticket, double *pml, double *tvar, double *seconds);

typedef struct ara_server_stats_t {
    int64_t iterations;        /* iterations completed                                         */
    int64_t completed;         /* requests completed                                           */
    int64_t held;              /* times the next queued request waited for arena space          */
    int32_t max_in_iteration;  /* most requests in one iteration                               */
    int32_t max_in_flight;     /* most requests admitted and not yet completed at one time      */
    int32_t slots;             /* slots over both lanes                                        */
    int32_t pad_;
    int64_t slot_bytes;        /* device bytes of one slot's tables                            */
    int64_t arena_bytes;       /* device bytes of the YLT arena                                */
} ara_server_stats_t;

/* Counters and sizes of the server.  Errors: ARA_E_INVALID_ARG (NULL). */
ara_status ara_server_stats(ara_server *server, ara_server_stats_t *stats);

/* Completes every queued request, stops the worker and frees the server. */
ara_status ara_server_release(ara_server *server);

#ifdef __cplusplus
}
#endif
#endif /* ARA_H */
