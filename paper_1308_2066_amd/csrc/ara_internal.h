// Internal declarations shared by the HIP sources of libara (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "ara.h"

namespace ara {

// Error bits a kernel may set in the context's device error word.
enum : uint32_t { ERR_ID_RANGE = 1u, ERR_OFFSETS = 2u, ERR_LOSS = 4u, ERR_DUP = 8u };
// Not an input error: a bin of the binned copy is too long for 3-byte run starts (the
// copy then keeps 4-byte ones).
constexpr uint32_t ERR_BIN_WIDE = 16u;

// Device-side description of one ELT: its sparse records, its direct access
// table over the catalog, and its financial terms.
struct EltDesc {
    const int32_t *pair_ids;
    const double *pair_losses;
    int64_t n_pairs;
    void *dat;          // catalog entries, binary64 or binary32 (f32 != 0); defined where seen
    uint32_t *seen;     // one bit per catalog event: listed by the ELT (also detects duplicates)
    int32_t f32;
    int32_t identity;   // financial terms are (1, 0, +inf)
    double fx, retention, limit;
};

// Combined table of a layer and its occurrence filter.
//   comb    catalog values: the loss per event summed over the layer's ELTs
//   bitmap  one bit per event: occurrence-net loss of comb[e] is nonzero;
//           grouped in blocks of 128 events = 4 words
//   rank    per 128-event block: number of flagged events in earlier blocks
//   rel16   the same count relative to the first block of its 256-block superblock
//   base32  per superblock (32768 events): number of flagged events before it
//   occ     catalog binary64 values: occurrence-net loss min(max(comb[e]-OccR,0),OccL)
//   vals    occ values of the flagged events, in event order (binary64)
struct LayerTables {
    void *comb = nullptr;
    double *occ = nullptr;
    uint32_t *bitmap = nullptr;
    uint32_t *nz = nullptr;         // one bit per event: combined loss nonzero (bitmap's layout)
    uint32_t *rank = nullptr;
    uint16_t *rel16 = nullptr;
    uint32_t *base32 = nullptr;
    double *vals = nullptr;
    uint32_t *n_flagged = nullptr;
    int32_t nblk = 0;
};

constexpr int kEventsPerBlock = 128;        // events per bitmap block
constexpr int kBlocksPerSuper = 256;        // bitmap blocks per rank superblock (32768 events)
constexpr int kLdsMaxBytes = 160 * 1024;    // LDS per workgroup on gfx950
constexpr int kBufWord3 = 0x00020000;       // raw buffer descriptor word 3 (32-bit data format)
constexpr int kQueueRow = 64;               // queued events are processed one wave-row at a time
constexpr int kQueueCapMax = 192;           // per-wave queue capacity (events), a multiple of kQueueRow
constexpr int kQueueCapMin = 128;
constexpr int kQueueWords = 16 * kQueueCapMax;  // static LDS of the bitmap trial kernel (16 waves)

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }
__host__ __device__ inline int32_t bitmap_blocks(int32_t catalog) { return (catalog + kEventsPerBlock - 1) / kEventsPerBlock; }
__host__ __device__ inline int32_t bitmap_supers(int32_t nblk) { return (nblk + kBlocksPerSuper - 1) / kBlocksPerSuper; }
// LDS layout of the bitmap placement: bits | rel16 | base32 | per-wave queues.
__host__ __device__ inline size_t bitmap_rel_offset(int32_t nblk) { return size_t(nblk) * 16; }
__host__ __device__ inline size_t bitmap_base_offset(int32_t nblk) { return bitmap_rel_offset(nblk) + align16(size_t(nblk) * 2); }
__host__ __device__ inline size_t bitmap_table_bytes(int32_t nblk) { return bitmap_base_offset(nblk) + align16(size_t(bitmap_supers(nblk)) * 4); }

// Arguments of the trial kernels.
struct TrialArgs {
    const int32_t *ids;
    const uint8_t *ids24;    // packed copy of ids (3 bytes each), or null
    int64_t n_events;
    const int64_t *offs;
    int64_t t_begin, t_end;
    int32_t catalog;
    int32_t nblk;
    const void *comb;        // combined table (binary64, or binary32 when f32)
    const double *occ;       // occurrence-net table over the catalog
    const uint32_t *bitmap;  // occurrence filter (see LayerTables)
    const uint32_t *nz;      // combined loss nonzero, one bit per event (see LayerTables)
    const uint16_t *rel16;
    const uint32_t *base32;
    const double *vals;
    int32_t qcap;            // per-wave queue capacity (bitmap placement)
    int32_t pad_;
    double occ_r, occ_l, agg_r, agg_l;
    double *ylt;
    double *ev_gross, *ev_occ, *ev_cum, *ev_ceded;
    uint32_t *err;
};

// ---- launchers (each enqueues on `s` and returns the launch status)
hipError_t launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t s);
hipError_t launch_validate_yet(const int32_t *ids, int64_t n_events, const int64_t *offs, int64_t n_trials,
                               int32_t catalog, uint32_t *err, hipStream_t s,
                               bool check_ids = true);
size_t yet_packed_bytes(int64_t n_events);
hipError_t launch_yet_pack(const int32_t *ids, int64_t n_events, uint8_t *packed, hipStream_t s);
hipError_t launch_elt_clear(const EltDesc *d, int n_elts, int32_t catalog, hipStream_t s);
hipError_t launch_elt_scatter(const EltDesc *d, int n_elts, int64_t max_pairs, int32_t catalog, uint32_t *err,
                              hipStream_t s);
// combined table, occurrence values and bitmaps of a layer; with `ranks`, also its
// ranks, flagged count and compacted values (launch_layer_ranks)
hipError_t launch_layer_tables(const EltDesc *d, int n_elts, int32_t catalog, bool f32, double occ_r, double occ_l,
                               const LayerTables &t, hipStream_t s, bool ranks = true);
// the same from an existing combined table (new occurrence terms)
hipError_t launch_layer_filter(int32_t catalog, bool f32, double occ_r, double occ_l, const LayerTables &t,
                               hipStream_t s, bool ranks = true);
// ranks (rank, rel16, base32), flagged count and compacted values from the bitmap and
// occurrence values: what the filter-based kernels read; the tiled kernel reads occ only
hipError_t launch_layer_ranks(int32_t catalog, const LayerTables &t, hipStream_t s);

struct TrialLaunch {
    int placement;      // ara_placement (resolved)
    bool f32;
    int block;          // threads per workgroup
    int grid;           // workgroups
    size_t lds_bytes;
    int qcap;           // per-wave queue capacity (bitmap placement)
    bool lane;          // one lane per trial (short trials, dense tables) instead of one wave
};

// Trials with at most this many occurrences on average go one per lane (dense tables).
constexpr int kLaneModeMaxMean = 256;
hipError_t launch_trial_ylt(const TrialArgs &a, const TrialLaunch &l, hipStream_t s);
hipError_t launch_trial_events(const TrialArgs &a, bool f32, int n_cu, int lds_max, hipStream_t s);
hipError_t launch_trial_occ_max(const TrialArgs &a, const TrialLaunch &l, int grid, double *out, hipStream_t s);
hipError_t launch_lookup(const TrialArgs &a, const TrialLaunch &l, const int32_t *ids, int64_t n, double *gross,
                         double *occ, hipStream_t s);
hipError_t prepare_trial_kernels();

// ---- batched analyses: jobs (a trial kernel's arguments + how they run) and work
// items (a job's trial range), processed by one persistent launch
enum BatchMode : int32_t {
    kModeLaneLds = 0,      // lane per trial, dense table in LDS
    kModeLaneGlobal = 1,   // lane per trial, dense table in HBM/L2
    kModeWaveLds = 2,      // wave per trial, dense table in LDS
    kModeWaveGlobal = 3,   // wave per trial, dense table in HBM/L2
    kModeWaveBitmap = 4,   // wave per trial, LDS filter, int32 IDs
    kModeWaveBitmap24 = 5, // wave per trial, LDS filter, packed IDs
    kModeTiled = 6         // the tiled kernel, launched on its own (not part of k_batch)
};
struct BatchJob {
    TrialArgs a;           // t_begin/t_end/ylt: the job's whole range
    int32_t mode;          // BatchMode
    int32_t placement;     // ara_placement of the table
};
struct BatchItem {
    int32_t job;
    int32_t pad_;
    int64_t t0, t1;        // trials [t0, t1) of the job's YET
};
constexpr int kBatchModes = 6;
hipError_t launch_batch(int32_t mode, const BatchJob *jobs, const BatchItem *items, int32_t n_items, int32_t per_wg,
                        int grid, hipStream_t s);
int32_t batch_mode(const TrialLaunch &l, bool packed);
hipError_t launch_sum_ylts(const double *const *ylts, int32_t n_jobs, int64_t n, double *out, hipStream_t s);
constexpr int kRiskLdsKeys = 16384;   // YLTs up to this length are sorted in one workgroup's LDS
hipError_t launch_risk_batch(const double *const *ylts, const int64_t *ns, const int64_t *ks, int n_jobs, int n_k,
                             double *out, hipStream_t s);
// bitmap placement (static LDS: filter tables up to trial_bitmap_table_capacity() bytes + event queues)
hipError_t launch_trial_ylt_bitmap(const TrialArgs &a, int grid, int block, hipStream_t s);
size_t trial_bitmap_table_capacity();

// ---- catalog-binned YET copy and the tiled trial kernel
// The catalog is cut into bins of 2^14 events (a bin's binary64 values fill most of
// a workgroup's LDS).  The binned copy holds, bin by bin (bin-major), every trial's
// occurrences of that bin's events in trial order (time order within a trial) as
// 14-bit IDs local to the bin, one uint16 each.  Region b
// starts at element region[b] (a multiple of 8); boff[b * stride + t] is where trial
// t's run starts inside region b (trial t's occurrences of bin b are
// [boff[b][t], boff[b][t + 1])), t = 0..n_trials.  Asked for (ARA_OPT_YET_RUN_BYTES)
// and with at most 64 bins the run starts are 3 bytes each (little-endian, row b at
// byte 3 b stride) unless a bin holds 2^24 occurrences or more: a quarter less memory,
// read as an unaligned 4-byte word whose top byte is dropped.  stride is a multiple of 8 and at least n_trials + 2, so
// that word stays inside its row; the array has 16 bytes of slack after its last row.
constexpr int kBinShift = 14;
constexpr int32_t kBinEvents = 1 << kBinShift;
constexpr int kMaxBins = 512;                                 // catalogs up to 2^23 events
inline int32_t catalog_bins(int32_t catalog) { return (catalog + kBinEvents - 1) / kBinEvents; }

// Run starts as the build writes them: 4 bytes each (abs), or 3 bytes each (b24, row
// b at byte 3 b stride; at most 64 bins).  stride: a multiple of 8, at least
// n_trials + 2.
struct RunStarts {
    uint32_t *abs;
    uint8_t *b24;
    int64_t stride;
};
__device__ __forceinline__ uint32_t run_at(const RunStarts &r, int64_t b, int64_t t) {
    if (r.abs) return r.abs[b * r.stride + t];
    uint32_t w;   // an unaligned word: this entry and the next one's first byte
    __builtin_memcpy(&w, r.b24 + 3 * (b * r.stride + t), 4);
    return w & 0xFFFFFFu;
}

// Run starts for t = 0..n_trials: the exclusive prefix sums over trials of each
// trial's occurrence count in bin b, so run(b, n_trials) is bin b's length.  In the
// 3-byte form a bin of 2^24 occurrences or more sets ERR_BIN_WIDE (its entries are
// then not usable).  sums: bin_offsets_scratch_words(n_trials, n_bins) words of
// scratch.  Also checks the YET (ERR_OFFSETS, ERR_ID_RANGE in err; bad offsets or IDs
// are not followed or counted): the count pass doubles as ingest's check.
hipError_t launch_bin_offsets(const int32_t *ids, const int64_t *offs, int64_t n_events, int64_t n_trials,
                              int32_t n_bins, const RunStarts &r, int32_t catalog, uint32_t *sums, uint32_t *err,
                              hipStream_t s);
size_t bin_offsets_scratch_words(int64_t n_trials, int32_t n_bins);
// Region starts (n_bins + 1, int64, multiples of 8) from the bins' lengths.
hipError_t launch_bin_regions(const RunStarts &r, int64_t n_trials, int32_t n_bins, int64_t *region,
                              const uint32_t *err, hipStream_t s);
// Both skip their work when *err is nonzero (the count pass found a bad ID or offset,
// or a bin too long for the 3-byte form).
hipError_t launch_bin_scatter(const int32_t *ids, const int64_t *offs, int64_t n_events, int64_t n_trials,
                              int32_t n_bins, const RunStarts &r, const int64_t *region, uint16_t *ids16,
                              const uint32_t *err, hipStream_t s);

constexpr int kTiledWaves = 16;                 // waves per workgroup of the tiled kernel
constexpr int kTiledWaveTrials = 252;           // trials per wave and pass (their sums are in LDS)
constexpr int kTiledPassTrials = kTiledWaveTrials * kTiledWaves;   // trials per workgroup pass
constexpr double kTiledStageCost = 0.5;         // a pass's bin staging, in occurrences per catalog event
                                                // (orders a batch's passes; results do not depend on it)
static_assert(size_t(kBinEvents + 2) * 8 + size_t(kTiledWaves) * kTiledWaveTrials * 8 + 16 <= size_t(kLdsMaxBytes),
              "a bin's binary64 values, the zero slot and the per-trial sums fit in LDS");

struct TiledArgs {
    const uint16_t *ids16;      // the YET's catalog-binned copy (see ara_yet)
    const int64_t *region;      // n_bins + 1 element offsets (multiples of 8)
    const uint32_t *boff;       // run starts, 4 bytes each, or null
    const uint8_t *boff24;      // or 3 bytes each (row b at byte 3 b stride)
    int64_t stride;             // entries per boff row
    int64_t t_begin, t_end;
    int64_t per_wg;             // trials per workgroup
    const double *occ;          // the layer's occurrence-net values, one per catalog event
    int32_t catalog;
    int32_t n_bins;
    double agg_r, agg_l;
    double *ylt;
};
// occ_max: each trial's largest occurrence-net loss into a.ylt instead of the YLT;
// start/stop (or null): HIP events attached to the launch (its dispatch's start and end)
hipError_t launch_trial_tiled(const TiledArgs &a, int grid, hipStream_t s, bool occ_max = false,
                              hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
// A pass of the tiled kernel as a work item: analysis `job`, trials [t0, t1).
struct TiledItem {
    int32_t job;
    int32_t pad_;
    int64_t t0, t1;
};
static_assert(sizeof(TiledItem) == 24, "six words");
// The YLTs of many analyses' passes in one launch (device arrays; `next`: one word of
// device memory, cleared by a fill kernel first, so the launch can be graph-captured).
hipError_t launch_trial_tiled_items(const TiledArgs *jobs, const TiledItem *items, int32_t n_items, uint32_t *next,
                                    int grid, hipStream_t s);

// ---- order statistics
size_t sort_workspace_bytes(int64_t n);
hipError_t launch_sort_desc_keys(const double *in, int64_t n, void *ws, hipStream_t s,
                                 uint32_t *host_plan = nullptr);   // sorted keys -> ws
hipError_t launch_sort_decode(const void *ws, int64_t n, double *out, hipStream_t s);
// PML/TVaR of the n losses y (device) at ranks ks[0, n_k) by radix selection (no
// sort): out holds, per group of up to 16 ranks, pml[m] then tvar[m].  ws: a sort
// workspace for n.  Asynchronous; no host waits.
hipError_t launch_risk_select(const double *y, int64_t n, void *ws, const int64_t *ks, int n_k, double *out_pml_tvar,
                              hipStream_t s);

}  // namespace ara
