// Output filters (Section II-C): the YLT sorted in descending order, then
// PML = the k-th largest loss and TVaR = the mean of the k largest, with k set by
// the return period (the paper names both measures, Section I, but does not define
// them; the engine's rank rule is ara_return_period_rank).
//
// PML and TVaR need no full sort (risk measures by selection, below); the sort is
// kept for ara_sort_desc.
//
// LSD radix sort of 64-bit keys, 8-bit digits, 8 passes.  A binary64 value maps to
// an unsigned key whose order is the value order (sign flip for non-negatives,
// complement for negatives, -0.0 canonicalised to +0.0); descending order sorts the
// complemented key ascending.  The encoding pass also finds the digits in which
// keys differ; a pass in which every key has the same digit is skipped on the device
// (capped YLTs often hold one value many times).  Each other pass: per-tile digit
// counts, exclusive offsets per (digit, tile), and a stable scatter in which every
// wave ranks its keys by matching digits across lanes with 8 ballots; the tile's keys
// are placed in LDS in output order first, so a store instruction writes runs of
// consecutive output positions.
#include "ara_internal.h"

namespace ara {

constexpr int kSortThreads = 1024;
constexpr int kSortPerThread = 2;
constexpr int kSortTile = kSortThreads * kSortPerThread;   // 2048 keys
constexpr int kWavesPerTile = kSortThreads / 64;            // 16
constexpr int kWaveKeys = 64 * kSortPerThread;              // consecutive keys a wave owns
constexpr int kPasses = 8;
static_assert(kSortThreads >= 256 && kSortThreads % 64 == 0, "the first 256 threads take one digit each");

__device__ __forceinline__ uint64_t desc_key(double d) {
    uint64_t u = __builtin_bit_cast(uint64_t, d + 0.0);   // -0.0 + 0.0 == +0.0
    u = (u >> 63) ? ~u : (u | 0x8000000000000000ull);       // ascending order key
    return ~u;                                             // descending
}

__device__ __forceinline__ double key_value(uint64_t k) {
    uint64_t u = ~k;
    u = (u >> 63) ? (u & 0x7FFFFFFFFFFFFFFFull) : ~u;
    return __builtin_bit_cast(double, u);
}

static inline int64_t sort_tiles(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

// Workspace: two key buffers, per-(digit, tile) counts, the encoding's digit
// differences (one 64-bit word per workgroup), and the pass plan (which buffer holds
// the keys before each pass, and which passes leave the order unchanged because
// every key has the same digit).
struct SortWs {
    uint64_t *a, *b;
    uint32_t *counts;   // [256][tiles]
    uint32_t *hist;     // 8 KB: the encoding's per-workgroup digit differences (uint64)
    uint32_t *dtotal;   // [256] keys per digit in the current pass (in the second half of hist)
    uint32_t *plan;     // plan[p]: keys before pass p are in b (1) or a (0), p = 0..8;
                        // plan[16 + p]: pass p is skipped
    double *part;       // kRiskGroup * kRiskMaxBlocks doubles: the selection's digit counts
};

constexpr int kRiskGroup = 16;        // return periods per launch
constexpr int kRiskMaxBlocks = 1024;  // partial sums per return period

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t sort_workspace_bytes(int64_t n) {
    return 2 * align256(size_t(n) * 8) + align256(size_t(sort_tiles(n)) * 256 * 4) + align256(8 * 256 * 4) + 256 +
           size_t(kRiskGroup) * kRiskMaxBlocks * 8;
}

static SortWs sort_ws(void *ws, int64_t n) {
    char *p = reinterpret_cast<char *>(ws);
    const size_t keys = align256(size_t(n) * 8);
    const size_t counts = align256(size_t(sort_tiles(n)) * 256 * 4);
    SortWs w;
    w.a = reinterpret_cast<uint64_t *>(p);
    w.b = reinterpret_cast<uint64_t *>(p + keys);
    w.counts = reinterpret_cast<uint32_t *>(p + 2 * keys);
    w.hist = reinterpret_cast<uint32_t *>(p + 2 * keys + counts);
    w.dtotal = w.hist + 1024;   // after 512 64-bit slots of encoding differences
    w.plan = reinterpret_cast<uint32_t *>(p + 2 * keys + counts + align256(8 * 256 * 4));
    w.part = reinterpret_cast<double *>(p + 2 * keys + counts + align256(8 * 256 * 4) + 256);
    return w;
}

__device__ __forceinline__ const uint64_t *cur_keys(const SortWs &w, int pass) {
    return w.plan[pass] ? w.b : w.a;
}

// Encode values into descending-order keys.  A pass leaves the order unchanged when
// every key has the same digit in it; so each workgroup also ORs key ^ (the first
// key) over its keys, and a pass is skipped when that digit of the OR over all
// workgroups is zero.  A wave reads 8 rows of 64 values at a time.
constexpr int kEncodeBlocks = 256;   // workgroups of k_sort_encode (one OR slot each)
static_assert(kEncodeBlocks <= 512, "the OR slots end where the digit totals start");

__global__ __launch_bounds__(1024) void k_sort_encode(const double *__restrict__ in, int64_t n,
                                                     uint64_t *__restrict__ keys, uint64_t *__restrict__ diff) {
    constexpr int kRows = 8;
    __shared__ uint64_t wdiff[16];
    const uint64_t k0 = desc_key(in[0]);
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    uint64_t d = 0;
    for (int64_t i0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i0 < n; i0 += kRows * stride) {
        uint64_t k[kRows];
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const int64_t i = i0 + r * stride;
            k[r] = i < n ? desc_key(in[i]) : k0;
        }
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const int64_t i = i0 + r * stride;
            if (i < n) keys[i] = k[r];
            d |= k[r] ^ k0;
        }
    }
    for (int o = 32; o >= 1; o >>= 1) d |= __shfl_xor(d, o, 64);
    if ((threadIdx.x & 63) == 0) wdiff[threadIdx.x >> 6] = d;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t o = 0;
        for (int k = 0; k < 16; ++k) o |= wdiff[k];
        diff[blockIdx.x] = o;
    }
}

// The plan: which buffer holds the keys before each pass, and which passes are skipped.
__global__ __launch_bounds__(64) void k_sort_plan(const uint64_t *__restrict__ diff, int n_slots,
                                                  uint32_t *__restrict__ plan) {
    uint64_t d = 0;
    for (int i = threadIdx.x; i < n_slots; i += 64) d |= diff[i];
    for (int o = 32; o >= 1; o >>= 1) d |= __shfl_xor(d, o, 64);
    if (threadIdx.x != 0) return;
    uint32_t sel = 0;
    plan[0] = 0;
    for (int p = 0; p < kPasses; ++p) {
        const uint32_t triv = ((d >> (8 * p)) & 255u) == 0 ? 1u : 0u;
        plan[16 + p] = triv;
        sel = triv ? sel : 1u - sel;
        plan[p + 1] = sel;
    }
}

// Lanes whose digit equals this lane's digit (among lanes with `valid`).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const uint64_t bb = __ballot((d >> b) & 1u);
        m &= ((d >> b) & 1u) ? bb : ~bb;
    }
    return m;
}

__device__ __forceinline__ uint64_t lanes_below(int lane) { return lane ? (~0ull >> (64 - lane)) : 0ull; }

// counts[d * tiles + tile] = number of keys of the tile with digit d
__global__ __launch_bounds__(kSortThreads) void k_sort_count(SortWs w, int64_t n, int pass, int64_t tiles) {
    if (w.plan[16 + pass]) return;
    __shared__ uint32_t hist[256];
    const uint64_t *keys = cur_keys(w, pass);
    const int shift = 8 * pass;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x < 256) hist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = int64_t(blockIdx.x) * kSortTile + wv * kWaveKeys;
    uint32_t d[kSortPerThread];
#pragma unroll
    for (int r = 0; r < kSortPerThread; ++r) {
        const int64_t i = base + r * 64 + lane;
        d[r] = i < n ? uint32_t(keys[i] >> shift) & 255u : 0u;
    }
#pragma unroll
    for (int r = 0; r < kSortPerThread; ++r) {
        if (base + r * 64 + lane < n) atomicAdd(&hist[d[r]], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 256) w.counts[int64_t(threadIdx.x) * tiles + blockIdx.x] = hist[threadIdx.x];
}

// Exclusive offsets within each digit's row of tile counts: one workgroup per digit
// scans its row in place, in chunks of 1024 (four consecutive counts per thread), and
// stores the row's total in w.dtotal.  The scatter adds the prefix of the totals over
// the smaller digits, so the offset of (d, t) is that of the flat digit-major array.
__global__ __launch_bounds__(256) void k_sort_rowscan(SortWs w, int pass, int64_t tiles) {
    if (w.plan[16 + pass]) return;
    __shared__ uint32_t wsum[4];
    uint32_t *c = w.counts + int64_t(blockIdx.x) * tiles;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    uint32_t carry = 0;
    for (int64_t base = 0; base < tiles; base += 1024) {
        uint32_t v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t i = base + 4 * tid + j;
            v[j] = i < tiles ? c[i] : 0u;
        }
        const uint32_t t = v[0] + v[1] + v[2] + v[3];
        uint32_t inc = t;   // inclusive wave scan of the threads' sums
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        if (lane == 63) wsum[wv] = inc;
        __syncthreads();
        uint32_t before = 0;
        for (int k = 0; k < wv; ++k) before += wsum[k];
        const uint32_t total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        uint32_t run = carry + before + inc - t;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t i = base + 4 * tid + j;
            if (i < tiles) c[i] = run;
            run += v[j];
        }
        carry += total;
        __syncthreads();
    }
    if (tid == 0) w.dtotal[blockIdx.x] = carry;
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(SortWs w, int64_t n, int pass, int64_t tiles) {
    if (w.plan[16 + pass]) return;
    __shared__ uint32_t whist[kWavesPerTile][256];
    __shared__ uint32_t woff[kWavesPerTile][256];   // tile-local start of (wave, digit)
    __shared__ uint32_t lstart[256];                // tile-local start of each digit
    __shared__ uint32_t gstart[256];                // output index of the tile's first key of each digit
    __shared__ uint64_t stage[kSortTile];           // the tile's keys in output order
    __shared__ uint32_t wtot[4], ltot[4];
    const uint64_t *in = cur_keys(w, pass);
    uint64_t *out = w.plan[pass] ? w.a : w.b;
    const int shift = 8 * pass;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < kWavesPerTile * 256; i += kSortThreads) whist[i >> 8][i & 255] = 0;
    // keys in the smaller digits: exclusive scan of the digit totals (first four waves)
    uint32_t dt = 0, dinc = 0;
    if (threadIdx.x < 256) {
        dt = w.dtotal[threadIdx.x];
        dinc = dt;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(dinc, o, 64);
            if (lane >= o) dinc += y;
        }
        if (lane == 63) wtot[wv] = dinc;
    }
    __syncthreads();
    uint32_t dbase = dinc - dt;
    for (int k = 0; k < wv && k < 4; ++k) dbase += wtot[k];
    const int64_t tile0 = int64_t(blockIdx.x) * kSortTile;
    const int64_t base = tile0 + wv * kWaveKeys;
    uint64_t key[kSortPerThread];
    uint32_t rank[kSortPerThread];
#pragma unroll
    for (int r = 0; r < kSortPerThread; ++r) {
        const int64_t i = base + r * 64 + lane;
        key[r] = i < n ? in[i] : 0ull;
    }
#pragma unroll
    for (int r = 0; r < kSortPerThread; ++r) {
        const bool valid = base + r * 64 + lane < n;
        const uint32_t d = uint32_t(key[r] >> shift) & 255u;
        const uint64_t m = match_digit(d, valid);
        const uint64_t below = m & lanes_below(lane);
        rank[r] = whist[wv][d] + uint32_t(__popcll(below));   // read before this round's update
        if (valid && below == 0) whist[wv][d] += uint32_t(__popcll(m));
    }
    __syncthreads();
    // tile-local start of each digit: exclusive scan of the tile's digit counts
    uint32_t tt = 0, tinc = 0;
    if (threadIdx.x < 256) {
        for (int k = 0; k < kWavesPerTile; ++k) tt += whist[k][threadIdx.x];
        tinc = tt;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(tinc, o, 64);
            if (lane >= o) tinc += y;
        }
        if (lane == 63) ltot[wv] = tinc;
    }
    __syncthreads();
    if (threadIdx.x < 256) {
        const int d = threadIdx.x;
        uint32_t run = tinc - tt;
        for (int k = 0; k < wv; ++k) run += ltot[k];
        lstart[d] = run;
        gstart[d] = dbase + w.counts[int64_t(d) * tiles + blockIdx.x];
        for (int k = 0; k < kWavesPerTile; ++k) {
            woff[k][d] = run;
            run += whist[k][d];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortPerThread; ++r) {
        if (base + r * 64 + lane < n) {
            const uint32_t d = uint32_t(key[r] >> shift) & 255u;
            stage[woff[wv][d] + rank[r]] = key[r];
        }
    }
    __syncthreads();
    // consecutive threads write consecutive keys of a digit's run
    const int tile_n = int(std::min<int64_t>(kSortTile, n - tile0));
    for (int i = threadIdx.x; i < tile_n; i += kSortThreads) {
        const uint64_t k = stage[i];
        const uint32_t d = uint32_t(k >> shift) & 255u;
        out[gstart[d] + uint32_t(i) - lstart[d]] = k;
    }
}

__global__ __launch_bounds__(256) void k_sort_decode(SortWs w, int64_t n, double *__restrict__ out) {
    const uint64_t *keys = cur_keys(w, kPasses);
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        out[i] = key_value(keys[i]);
}

// Sorted descending keys of `in` end in the workspace key buffer the plan names.
// host_plan: pinned host memory of 32 words, or null.  With it, the host reads the
// pass plan (one small copy and a wait) and launches only the passes that reorder
// keys; without it every pass is launched and trivial ones return at once (for
// callers that must not block).
hipError_t launch_sort_desc_keys(const double *in, int64_t n, void *ws, hipStream_t s, uint32_t *host_plan) {
    if (n <= 0) return hipSuccess;
    SortWs w = sort_ws(ws, n);
    const int64_t tiles = sort_tiles(n);
    const unsigned eb = unsigned(std::min<int64_t>((n + 255) / 256, kEncodeBlocks));
    uint64_t *diff = reinterpret_cast<uint64_t *>(w.hist);
    hipLaunchKernelGGL(k_sort_encode, dim3(eb), dim3(1024), 0, s, in, n, w.a, diff);
    hipLaunchKernelGGL(k_sort_plan, dim3(1), dim3(64), 0, s, diff, int(eb), w.plan);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    bool skip[kPasses] = {};
    if (host_plan) {
        e = hipMemcpyAsync(host_plan, w.plan, 32 * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        for (int p = 0; p < kPasses; ++p) skip[p] = host_plan[16 + p] != 0;
    }
    for (int pass = 0; pass < kPasses; ++pass) {
        if (skip[pass]) continue;
        hipLaunchKernelGGL(k_sort_count, dim3(unsigned(tiles)), dim3(kSortThreads), 0, s, w, n, pass, tiles);
        hipLaunchKernelGGL(k_sort_rowscan, dim3(256), dim3(256), 0, s, w, pass, tiles);
        hipLaunchKernelGGL(k_sort_scatter, dim3(unsigned(tiles)), dim3(kSortThreads), 0, s, w, n, pass, tiles);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_sort_decode(const void *ws, int64_t n, double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    SortWs w = sort_ws(const_cast<void *>(ws), n);
    const unsigned eb = unsigned(std::min<int64_t>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k_sort_decode, dim3(eb), dim3(256), 0, s, w, n, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Risk measures by radix selection.  PML(rp) = the k-th largest loss and TVaR(rp) =
// the mean of the k largest, k = ara_return_period_rank(n, rp).  In descending-order
// keys PML is the k-th smallest key K.  K is found digit by digit from the most
// significant 8 bits down: pass p counts, for every rank, digit p of the keys that
// share the digits chosen so far (the rank's bucket); the next kernel (every
// workgroup of it, from the complete counts) picks the digit where the running count
// reaches the rank, and the rank left within that digit carries on.  A digit in which
// every key agrees (the OR of key ^ first key is zero there) is not counted.  Once
// every rank's bucket holds at most kCollect keys, that pass copies the buckets out
// instead of counting, and one workgroup per rank sorts its bucket in LDS for K; the
// later passes do nothing.  The k largest losses are the losses whose key is below K,
// plus (k - their number) copies of PML, so
//   TVaR = (sum of the losses whose key is below K + r * PML) / k,
// r = the copies of K among the k largest.  That sum is taken in a fixed order: per
// tile of 2048 losses in index order, 256 slots (slot t adds the tile's losses t,
// t + 256, ..., t + 1792 in turn; the others add +0.0) and a fixed tree over the
// slots; then the tile sums, slot t adding tiles t, t + 256, ... in turn, and the same
// tree.  A YLT of at most kRiskLdsKeys losses is sorted whole in one workgroup's LDS
// instead (k_risk_lds), with the same sums, so every path gives the same bits.
// Kernel boundaries order every step: no workgroup waits on another.
constexpr int kSelPerThread = 4;
constexpr int kSelThreads = 1024;
constexpr int kSelBlocks = 256;                         // most workgroups of a counting pass
constexpr int kSelChunk = kSelThreads * kSelPerThread;  // keys per workgroup and round
constexpr int kSelTile = 2048;                          // losses per tile of the TVaR sum
constexpr int kCollect = 2048;                          // largest bucket sorted in LDS
static_assert(kSelTile == 8 * 256, "a tile is 8 losses for each of 256 slots");
static_assert(kPasses * kRiskGroup * 256 * 4 <= kRiskGroup * kRiskMaxBlocks * 8, "selection counts fit the part region");
static_assert(kSelTile == kSortTile && kRiskGroup * 8 <= 256 * 4, "tile sums fit the sort's per-tile counts");
static_assert(int64_t(kRiskGroup) * kCollect * 8 <= 2 * 8 * int64_t(kRiskLdsKeys + 1),
              "the buckets fit the key buffers of YLTs longer than kRiskLdsKeys");

struct SelWs {
    uint64_t *slots;    // [kSelBlocks]: OR over a workgroup's keys of key ^ (key of the first loss)
    uint64_t *prefix;   // [kPasses + 1][kRiskGroup]: digits chosen before pass p (where keys differ);
                        // [kPasses]: K
    int64_t *left;      // [kPasses + 1][kRiskGroup]: rank left among the keys of the bucket;
                        // [kPasses]: copies of K among the k largest
    uint32_t *bcount;   // [kPasses + 1][kRiskGroup]: keys in the bucket before pass p
    uint32_t *ncand;    // [kRiskGroup]: keys copied out of each bucket
    uint32_t *collected;// the pass that copied the buckets out (0: none)
    uint32_t *count;    // [kPasses][kRiskGroup][256] digit counts
    uint64_t *cand;     // [kRiskGroup][kCollect] the buckets copied out (in the key buffers)
    double *tile_sum;   // [kRiskGroup][tiles]
};

// The selection's tables in the sort workspace.
static SelWs sel_ws(void *ws, int64_t n) {
    const SortWs w = sort_ws(ws, n);
    SelWs q;
    q.slots = reinterpret_cast<uint64_t *>(w.hist);
    q.prefix = reinterpret_cast<uint64_t *>(w.hist + 1280);
    q.left = reinterpret_cast<int64_t *>(w.hist + 1280 + 2 * kRiskGroup * (kPasses + 1));
    q.bcount = w.hist + 1280 + 4 * kRiskGroup * (kPasses + 1);
    q.ncand = q.bcount + kRiskGroup * (kPasses + 1);
    q.collected = q.ncand + kRiskGroup;
    q.count = reinterpret_cast<uint32_t *>(w.part);
    q.cand = w.a;
    q.tile_sum = reinterpret_cast<double *>(w.counts);
    return q;
}
static_assert(1280 + 5 * kRiskGroup * (kPasses + 1) + kRiskGroup + 1 <= 2048, "selection state fits the 8 KB table");

struct SelKs {
    int64_t k[kRiskGroup];
    int m;              // ranks in this group
    int n_slots;        // workgroups of the counting passes (OR slots written)
};

// Digits (8 bits each) in which some key differs from the first: 0xFF in every such digit.
__device__ __forceinline__ uint64_t varying_digits(uint64_t d) {
    uint64_t m = 0;
#pragma unroll
    for (int p = 0; p < kPasses; ++p)
        if ((d >> (8 * p)) & 255u) m |= 0xFFull << (8 * p);
    return m;
}

// OR of the workgroups' slots (d: this thread's share), in every thread (after a barrier).
__device__ __forceinline__ uint64_t slots_or(uint64_t d, uint64_t *lds) {
    for (int o = 32; o >= 1; o >>= 1) d |= __shfl_xor(d, o, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = d;
    __syncthreads();
    uint64_t r = 0;
    for (int k = 0; k < int(blockDim.x >> 6); ++k) r |= lds[k];
    return r;
}

// The selection state before pass p into pre/left/bc (LDS, m ranks), and the digits in
// which keys vary: p = 0 is the start (no digit chosen, the ranks themselves, every key
// in the bucket); for p >= 1, the state before pass p - 1 with digit p - 1 picked from
// its complete counts (unchanged when every key has the same digit there).  Every load
// is issued first, so the workgroup waits for one round trip.  pre/left/bc hold
// 2 kRiskGroup entries (the upper half is scratch).  Whole workgroup (>= 256 threads);
// ends with a barrier.
__device__ __forceinline__ uint64_t sel_state(const SelWs &q, const SelKs &ks, int64_t n, int p, uint64_t *pre,
                                              int64_t *left, uint32_t *bc, uint64_t *lds, uint32_t (*wsum)[4]) {
    const int tid = threadIdx.x, lane = tid & 63, m = ks.m;
    const uint64_t slot = tid < ks.n_slots ? q.slots[tid] : 0ull;
    uint64_t pr = 0;
    int64_t lf = 0;
    uint32_t bn = 0;
    if (tid < m) {
        pr = p > 0 ? q.prefix[(p - 1) * kRiskGroup + tid] : 0ull;
        lf = p > 0 ? q.left[(p - 1) * kRiskGroup + tid] : ks.k[tid];
        bn = p > 0 ? q.bcount[(p - 1) * kRiskGroup + tid] : uint32_t(n);
    }
    uint32_t c[kRiskGroup];
    const uint32_t *cnt = q.count + size_t(p > 0 ? p - 1 : 0) * kRiskGroup * 256;
#pragma unroll
    for (int r = 0; r < kRiskGroup; ++r) c[r] = p > 0 && r < m && tid < 256 ? cnt[r * 256 + tid] : 0u;
    if (tid < m) {
        pre[tid] = pr;
        left[tid] = lf;
        bc[tid] = bn;
        pre[kRiskGroup + tid] = 0ull;   // the digit picked (every count row has one)
        left[kRiskGroup + tid] = lf;
        bc[kRiskGroup + tid] = bn;
    }
    const uint64_t vary = varying_digits(slots_or(slot, lds));   // its barrier also publishes pre/left
    const int shift = 56 - 8 * (p - 1);
    if (p == 0 || ((vary >> shift) & 255u) == 0) {
        __syncthreads();
        return vary;
    }
    // inclusive scans of the m count rows over the digits (threads 0..255), then the pick
    uint32_t inc[kRiskGroup];
#pragma unroll
    for (int r = 0; r < kRiskGroup; ++r) {
        inc[r] = c[r];
        if (r >= m) continue;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(inc[r], o, 64);
            if (lane >= o) inc[r] += t;
        }
        if (lane == 63 && tid < 256) wsum[r][tid >> 6] = inc[r];
    }
    __syncthreads();
    if (tid < 256) {
#pragma unroll
        for (int r = 0; r < kRiskGroup; ++r) {
            if (r >= m) continue;
            uint32_t before = inc[r] - c[r];
            for (int k = 0; k < (tid >> 6); ++k) before += wsum[r][k];
            const int64_t l = left[r];
            if (int64_t(before) < l && l <= int64_t(before) + int64_t(c[r])) {   // one digit per rank
                pre[kRiskGroup + r] = uint64_t(tid);
                left[kRiskGroup + r] = l - int64_t(before);
                bc[kRiskGroup + r] = c[r];
            }
        }
    }
    __syncthreads();
    if (tid < m) {
        pre[tid] |= pre[kRiskGroup + tid] << shift;
        left[tid] = left[kRiskGroup + tid];
        bc[tid] = bc[kRiskGroup + tid];
    }
    __syncthreads();
    return vary;
}

// Clears the counts and the bucket copies' state and writes each workgroup's OR slot.
__global__ __launch_bounds__(kSelThreads) void k_sel_prep(const double *__restrict__ y, int64_t n, SelWs q, SelKs ks) {
    __shared__ uint64_t wdiff[kSelThreads / 64];
    const int tid = threadIdx.x;
    for (int i = blockIdx.x * kSelThreads + tid; i < kPasses * kRiskGroup * 256; i += gridDim.x * kSelThreads)
        q.count[i] = 0u;
    if (blockIdx.x == 0) {
        if (tid < kRiskGroup) q.ncand[tid] = 0u;
        if (tid == 0) *q.collected = 0u;
    }
    const uint64_t k0 = desc_key(y[0]);
    uint64_t d = 0;
    for (int64_t i = int64_t(blockIdx.x) * kSelThreads + tid; i < n; i += int64_t(gridDim.x) * kSelThreads)
        d |= desc_key(y[i]) ^ k0;
    for (int o = 32; o >= 1; o >>= 1) d |= __shfl_xor(d, o, 64);
    if ((tid & 63) == 0) wdiff[tid >> 6] = d;
    __syncthreads();
    if (tid == 0) {
        uint64_t o = 0;
        for (int k = 0; k < kSelThreads / 64; ++k) o |= wdiff[k];
        q.slots[blockIdx.x] = o;
    }
}

// Pass p: with the state before it (workgroup 0 records it), either copies every
// rank's bucket out (all of them small), or counts digit p of the bucket's keys;
// nothing once the buckets have been copied out.
__global__ __launch_bounds__(kSelThreads) void k_sel_pass(const double *__restrict__ y, int64_t n, SelWs q, SelKs ks,
                                                        int pass) {
    __shared__ uint32_t hist[kRiskGroup][256];
    __shared__ uint64_t lds[kSelThreads / 64];
    __shared__ uint64_t pre[2 * kRiskGroup];
    __shared__ int64_t left[2 * kRiskGroup];
    __shared__ uint32_t bc[2 * kRiskGroup];
    __shared__ uint32_t wsum[kRiskGroup][4];
    const int tid = threadIdx.x, lane = tid & 63;
    const int m = ks.m;
    {
        // the pass that copied the buckets out, if an earlier one did (this pass's own
        // workgroup 0 may set it while the others run)
        const uint32_t c = *q.collected;
        if (c != 0u && c < uint32_t(pass)) return;
    }
    const uint64_t vary = sel_state(q, ks, n, pass, pre, left, bc, lds, wsum);
    if (blockIdx.x == 0 && tid < m) {
        q.prefix[pass * kRiskGroup + tid] = pre[tid];
        q.left[pass * kRiskGroup + tid] = left[tid];
        q.bcount[pass * kRiskGroup + tid] = bc[tid];
    }
    bool small = pass > 0;
    for (int r = 0; r < m; ++r) small = small && bc[r] <= uint32_t(kCollect);
    // compare keys on the chosen digits that vary (the others agree everywhere)
    const int shift = 56 - 8 * pass;
    const uint64_t above = shift == 56 ? 0ull : ~0ull << (shift + 8);
    const uint64_t cmp = above & vary;
    if (small) {
        if (blockIdx.x == 0 && tid == 0) *q.collected = uint32_t(pass);
        for (int64_t i = int64_t(blockIdx.x) * kSelThreads + tid; i < n; i += int64_t(gridDim.x) * kSelThreads) {
            const uint64_t key = desc_key(y[i]);
            for (int r = 0; r < m; ++r) {
                if (((key ^ pre[r]) & cmp) == 0) {
                    const uint32_t at = atomicAdd(&q.ncand[r], 1u);
                    q.cand[int64_t(r) * kCollect + at] = key;   // at < bucket size <= kCollect
                }
            }
        }
        return;
    }
    if (((vary >> shift) & 255u) == 0) return;   // every key has the same digit here
    for (int i = tid; i < kRiskGroup * 256; i += kSelThreads) hist[i >> 8][i & 255] = 0u;
    __syncthreads();
    for (int64_t b0 = int64_t(blockIdx.x) * kSelChunk; b0 < n; b0 += int64_t(gridDim.x) * kSelChunk) {
        uint64_t key[kSelPerThread];
        bool ok[kSelPerThread];
#pragma unroll
        for (int u = 0; u < kSelPerThread; ++u) {
            const int64_t i = b0 + u * kSelThreads + tid;
            ok[u] = i < n;
            key[u] = ok[u] ? desc_key(y[i]) : 0ull;
        }
#pragma unroll
        for (int u = 0; u < kSelPerThread; ++u) {
            const uint32_t dg = uint32_t(key[u] >> shift) & 255u;
            for (int r = 0; r < m; ++r) {
                const bool match = ok[u] && ((key[u] ^ pre[r]) & cmp) == 0;
                const uint64_t mm = __ballot(match);
                if (mm == 0) continue;
                const int lead = __ffsll(static_cast<unsigned long long>(mm)) - 1;
                const uint32_t d0 = uint32_t(__builtin_amdgcn_readlane(int(dg), lead));
                if (__ballot(match && dg != d0) == 0) {   // one digit in the wave: one add
                    if (lane == lead) atomicAdd(&hist[r][d0], uint32_t(__popcll(mm)));
                } else if (match) {
                    atomicAdd(&hist[r][dg], 1u);
                }
            }
        }
    }
    __syncthreads();
    uint32_t *cnt = q.count + size_t(pass) * kRiskGroup * 256;
    for (int i = tid; i < m * 256; i += kSelThreads)
        if (hist[i >> 8][i & 255]) atomicAdd(&cnt[i], hist[i >> 8][i & 255]);
}

// 256-slot sum of one tile's losses below key K: v and kv are the slot's 8 losses
// (+0.0 past the end) and their keys.
__device__ __forceinline__ double slot_sum_below(const double (&v)[8], const uint64_t (&kv)[8], uint64_t K) {
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) s += kv[u] < K ? v[u] : 0.0;
    return s;
}

// Fixed tree over 256 slot values (threads >= 256 only keep the barriers).
__device__ __forceinline__ double tree256(double s, double *part) {
    if (threadIdx.x < 256) part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (int(threadIdx.x) < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    const double r = part[0];
    __syncthreads();
    return r;
}

// Loads slot t's 8 losses of tile [lo, lo + 2048) (canonical +0.0 for -0.0; +0.0 past n).
__device__ __forceinline__ void tile_slot(const double *y, int64_t n, int64_t lo, double (&v)[8], uint64_t (&kv)[8]) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int64_t i = lo + int64_t(threadIdx.x) + 256 * u;
        v[u] = i < n && threadIdx.x < 256 ? y[i] + 0.0 : 0.0;
        kv[u] = desc_key(v[u]);
    }
}

// Each tile's sum of the losses below each rank's K (one 256-thread workgroup per tile).
__global__ __launch_bounds__(256) void k_sel_sum(const double *__restrict__ y, int64_t n, SelWs q, SelKs ks) {
    __shared__ double part[256];
    __shared__ uint64_t K[kRiskGroup];
    const int tid = threadIdx.x, m = ks.m;
    const int64_t tiles = (n + kSelTile - 1) / kSelTile;
    double v[8];
    uint64_t kv[8];
    tile_slot(y, n, int64_t(blockIdx.x) * kSelTile, v, kv);
    if (tid < m) K[tid] = q.prefix[kPasses * kRiskGroup + tid];
    __syncthreads();
    for (int r = 0; r < m; ++r) {
        const double s = tree256(slot_sum_below(v, kv, K[r]), part);
        if (tid == 0) q.tile_sum[int64_t(r) * tiles + blockIdx.x] = s;
    }
}

// PML and TVaR of each rank from K, its copies and the tile sums (one workgroup).
__global__ __launch_bounds__(256) void k_sel_final(int64_t n, SelWs q, SelKs ks, double *__restrict__ out) {
    __shared__ double part[256];
    const int tid = threadIdx.x, m = ks.m;
    const int64_t tiles = (n + kSelTile - 1) / kSelTile;
    for (int r = 0; r < m; ++r) {
        double s = 0.0;
        for (int64_t t = tid; t < tiles; t += 256) s += q.tile_sum[int64_t(r) * tiles + t];
        s = tree256(s, part);
        if (tid == 0) {
            const double pml = key_value(q.prefix[kPasses * kRiskGroup + r]);
            out[r] = pml;
            out[m + r] = (s + double(q.left[kPasses * kRiskGroup + r]) * pml) / double(ks.k[r]);
        }
    }
}

// Ascending bitonic sort of key[0, np) in LDS by a workgroup of 1024 threads; np is a
// power of two, equal to 1024 E when E > 1 (else at most 1024).  Stages whose pairs
// lie within a thread's E consecutive keys run in registers without barriers; the
// others go through LDS, each thread taking whole pairs (q-th pair: bit log2(h) of
// its lower index is 0).
template <int E>
__device__ __forceinline__ void bitonic_sort_lds(uint64_t *key, int np) {
    const int tid = threadIdx.x;
    for (int k = 2; k <= np; k <<= 1) {
        for (int h = k >> 1; h >= E; h >>= 1) {
            for (int q = tid; q < np / 2; q += 1024) {
                const int i = ((q & ~(h - 1)) << 1) | (q & (h - 1));
                const int p = i | h;
                const uint64_t a = key[i], b = key[p];
                if ((a > b) == ((i & k) == 0)) {
                    key[i] = b;
                    key[p] = a;
                }
            }
            __syncthreads();
        }
        if (E > 1) {
            const int base = E * tid;
            uint64_t r[E];
#pragma unroll
            for (int e = 0; e < E; ++e) r[e] = key[base + e];
#pragma unroll
            for (int hh = E / 2; hh > 0; hh >>= 1) {
                if (hh > (k >> 1)) continue;   // the merge of size k has no stage hh
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if (e & hh) continue;
                    const bool asc = ((base + e) & k) == 0;
                    const uint64_t a = r[e], b = r[e | hh];
                    const bool sw = (a > b) == asc;
                    r[e] = sw ? b : a;
                    r[e | hh] = sw ? a : b;
                }
            }
#pragma unroll
            for (int e = 0; e < E; ++e) key[base + e] = r[e];
            __syncthreads();
        }
    }
}

// The same sort for np = 16384 (16 keys per thread) with the stages on index bits >= 4
// taken four bits at a time: a thread loads the 16 keys whose indices differ only in
// a 4-bit field at bit lo (the other 10 bits from its thread index), runs the stages
// on those bits in registers and writes them back: one barrier per group instead of
// one per stage.
__device__ __forceinline__ void bitonic_sort_lds_16k(uint64_t *key) {
    constexpr int np = 16384;
    const int tid = threadIdx.x;
    for (int k = 2; k <= np; k <<= 1) {
        int hb = 31 - __builtin_clz(uint32_t(k)) - 1;   // the merge's highest stage bit
        while (hb >= 4) {
            const int lo = hb - 3 > 4 ? hb - 3 : 4;        // group: bits [lo, hb], field [lo, lo + 3]
            const int base = ((tid >> lo) << (lo + 4)) | (tid & ((1 << lo) - 1));
            uint64_t r[16];
#pragma unroll
            for (int e = 0; e < 16; ++e) r[e] = key[base | (e << lo)];
#pragma unroll
            for (int d = 3; d >= 0; --d) {
                if (lo + d > hb) continue;
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    if (e & (1 << d)) continue;
                    const int f = e | (1 << d);
                    const bool asc = ((base | (e << lo)) & k) == 0;
                    const uint64_t a = r[e], b = r[f];
                    const bool sw = (a > b) == asc;
                    r[e] = sw ? b : a;
                    r[f] = sw ? a : b;
                }
            }
#pragma unroll
            for (int e = 0; e < 16; ++e) key[base | (e << lo)] = r[e];
            __syncthreads();
            hb = lo - 1;
        }
        // bits 3..0: the thread's 16 consecutive keys
        const int base = 16 * tid;
        uint64_t r[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) r[e] = key[base + e];
#pragma unroll
        for (int hh = 8; hh > 0; hh >>= 1) {
            if (hh > (k >> 1)) continue;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                if (e & hh) continue;
                const bool asc = ((base + e) & k) == 0;
                const uint64_t a = r[e], b = r[e | hh];
                const bool sw = (a > b) == asc;
                r[e] = sw ? b : a;
                r[e | hh] = sw ? a : b;
            }
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) key[base + e] = r[e];
        __syncthreads();
    }
}

// K and its copies among the k largest (final state) for rank blockIdx.x: from its
// bucket copied out (sorted in LDS), else from the last digit's counts.
__global__ __launch_bounds__(1024) void k_sel_finish(const double *__restrict__ y, int64_t n, SelWs q, SelKs ks) {
    __shared__ uint64_t key[kCollect];
    __shared__ uint64_t lds[16];
    __shared__ uint64_t pre[2 * kRiskGroup];
    __shared__ int64_t left[2 * kRiskGroup];
    __shared__ uint32_t bc[2 * kRiskGroup];
    __shared__ uint32_t wsum[kRiskGroup][4];
    __shared__ int below;
    const int tid = threadIdx.x, r = blockIdx.x;
    const uint32_t p = *q.collected;
    if (p == 0) {   // every digit picked from counts: the state after the last digit
        const uint64_t vary = sel_state(q, ks, n, kPasses, pre, left, bc, lds, wsum);
        if (tid == 0) {
            const uint64_t k0 = desc_key(y[0]);
            q.prefix[kPasses * kRiskGroup + r] = (pre[r] & vary) | (k0 & ~vary);
            q.left[kPasses * kRiskGroup + r] = left[r];
        }
        return;
    }
    const uint32_t nc = min(q.ncand[r], uint32_t(kCollect));
    const int64_t lf = q.left[int64_t(p) * kRiskGroup + r];   // rank within the bucket
    int np = 1;
    while (np < int(nc)) np <<= 1;
    for (int i = tid; i < np; i += 1024) key[i] = i < int(nc) ? q.cand[int64_t(r) * kCollect + i] : ~0ull;
    __syncthreads();
    if (np == 2048) bitonic_sort_lds<2>(key, np);
    else bitonic_sort_lds<1>(key, np);
    if (tid == 0) {
        const uint64_t K = key[lf - 1];
        int lo = 0, hi = int(lf) - 1;   // keys of the bucket below K: the first index holding K
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (key[mid] < K) lo = mid + 1;
            else hi = mid;
        }
        below = lo;
        q.prefix[kPasses * kRiskGroup + r] = K;
        q.left[kPasses * kRiskGroup + r] = lf - below;
    }
}

// PML/TVaR of the losses y[0, n) (n <= kRiskLdsKeys) at ranks k(0..n_k-1), sorted whole
// in LDS by one workgroup of 1024 threads: out[r] = PML, out[n_k + r] = TVaR.
template <typename RankAt>
__device__ __forceinline__ void risk_lds(const double *y, int n, int n_k, RankAt k_at, double *out, uint64_t *key,
                                         double *part, double *tile_s, int *below) {
    int np = 1;
    while (np < n) np <<= 1;
    for (int i = threadIdx.x; i < np; i += blockDim.x) key[i] = i < n ? desc_key(y[i]) : ~0ull;
    __syncthreads();
    switch (np) {
    case 16384: bitonic_sort_lds_16k(key); break;
    case 8192: bitonic_sort_lds<8>(key, np); break;
    case 4096: bitonic_sort_lds<4>(key, np); break;
    case 2048: bitonic_sort_lds<2>(key, np); break;
    default: bitonic_sort_lds<1>(key, np); break;
    }
    const int nt = (n + kSelTile - 1) / kSelTile;   // <= kRiskLdsKeys / kSelTile
    for (int r = 0; r < n_k; ++r) {
        const int64_t k = k_at(r);
        const uint64_t K = key[k - 1];
        if (threadIdx.x == 0) {   // keys below K: the first index holding K
            int lo = 0, hi = int(k) - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (key[mid] < K) lo = mid + 1;
                else hi = mid;
            }
            *below = lo;
        }
        for (int b = 0; b < nt; ++b) {
            double v[8];
            uint64_t kv[8];
            tile_slot(y, n, int64_t(b) * kSelTile, v, kv);
            const double s = tree256(slot_sum_below(v, kv, K), part);
            if (threadIdx.x == 0) tile_s[b] = s;
            __syncthreads();
        }
        double s = 0.0;
        if (threadIdx.x < 256)
            for (int b = threadIdx.x; b < nt; b += 256) s += tile_s[b];
        s = tree256(s, part);
        if (threadIdx.x == 0) {
            const double pml = key_value(K);
            out[r] = pml;
            out[n_k + r] = (s + double(k - *below) * pml) / double(k);
        }
        __syncthreads();
    }
}

// One YLT of at most kRiskLdsKeys losses, ranks from the kernel arguments.
__global__ __launch_bounds__(1024) void k_risk_lds(const double *__restrict__ y, int n, SelKs ks,
                                                   double *__restrict__ out) {
    __shared__ uint64_t key[kRiskLdsKeys];
    __shared__ double part[256];
    __shared__ double tile_s[kRiskLdsKeys / kSelTile];
    __shared__ int below;
    risk_lds(y, n, ks.m, [&](int r) { return ks.k[r]; }, out, key, part, tile_s, &below);
}

hipError_t launch_risk_select(const double *y, int64_t n, void *ws, const int64_t *ks, int n_k, double *out,
                              hipStream_t s) {
    if (n <= 0 || n_k <= 0) return hipSuccess;
    const SelWs q = sel_ws(ws, n);
    const int blocks = int(std::min<int64_t>(kSelBlocks, (n + kSelChunk - 1) / kSelChunk));
    const unsigned tiles = unsigned((n + kSelTile - 1) / kSelTile);
    for (int base = 0; base < n_k; base += kRiskGroup) {
        SelKs g{};
        g.m = std::min(kRiskGroup, n_k - base);
        g.n_slots = blocks;
        for (int i = 0; i < g.m; ++i) g.k[i] = ks[base + i];
        // out layout per group: pml[m], tvar[m]
        if (n <= kRiskLdsKeys) {
            hipLaunchKernelGGL(k_risk_lds, dim3(1), dim3(1024), 0, s, y, int(n), g, out + 2 * base);
        } else {
            hipLaunchKernelGGL(k_sel_prep, dim3(unsigned(blocks)), dim3(kSelThreads), 0, s, y, n, q, g);
            for (int p = 0; p < kPasses; ++p)
                hipLaunchKernelGGL(k_sel_pass, dim3(unsigned(blocks)), dim3(kSelThreads), 0, s, y, n, q, g, p);
            hipLaunchKernelGGL(k_sel_finish, dim3(unsigned(g.m)), dim3(1024), 0, s, y, n, q, g);
            hipLaunchKernelGGL(k_sel_sum, dim3(tiles), dim3(256), 0, s, y, n, q, g);
            hipLaunchKernelGGL(k_sel_final, dim3(1), dim3(256), 0, s, n, q, g, out + 2 * base);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------------
// Batched risk measures of many small YLTs (n <= kRiskLdsKeys each): one workgroup
// per YLT, risk_lds, so the results equal those of ara_risk_measures on the same YLT
// bit for bit.
__global__ __launch_bounds__(1024) void k_risk_batch(const double *const *__restrict__ ylts,
                                                     const int64_t *__restrict__ ns, const int64_t *__restrict__ ks,
                                                     int n_k, double *__restrict__ out) {
    __shared__ uint64_t key[kRiskLdsKeys];
    __shared__ double part[256];
    __shared__ double tile_s[kRiskLdsKeys / kSelTile];
    __shared__ int below;
    const int j = blockIdx.x;
    if (ns[j] < 1 || ns[j] > kRiskLdsKeys) return;   // longer YLTs take the radix selection
    risk_lds(ylts[j], int(ns[j]), n_k, [&](int r) { return ks[int64_t(j) * n_k + r]; }, out + int64_t(j) * 2 * n_k,
             key, part, tile_s, &below);
}

hipError_t launch_risk_batch(const double *const *ylts, const int64_t *ns, const int64_t *ks, int n_jobs, int n_k,
                             double *out, hipStream_t s) {
    if (n_jobs <= 0 || n_k <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_risk_batch, dim3(unsigned(n_jobs)), dim3(1024), 0, s, ylts, ns, ks, n_k, out);
    return hipGetLastError();
}

}  // namespace ara
