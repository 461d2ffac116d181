// Output filters (Section II-C): the YLT sorted in descending order, then
// PML = the k-th largest loss and TVaR = the mean of the k largest, with k set by
// the return period (the paper names both measures, Section I, but does not define
// them; the engine's rank rule is ara_return_period_rank).
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
    double *part;       // [kRiskGroup][kRiskMaxBlocks] partial sums of the top-k keys
};

constexpr int kRiskGroup = 16;        // return periods per launch
constexpr int kRiskMaxBlocks = 1024;  // partial sums per return period
constexpr int kRiskChunk = 2048;      // keys per partial sum, at least (8 per thread)

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

// PML = the k-th largest, TVaR = the mean of the k largest.  The top k keys are
// summed in fixed chunks (one workgroup each, fixed stride and LDS tree), then the
// chunk sums in chunk order: the result does not depend on scheduling.
struct RiskKs {
    int64_t k[kRiskGroup];
    int64_t chunk[kRiskGroup];
};

__device__ __forceinline__ double block_sum(double s, double *part) {
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o >= 1; o >>= 1) {
        if (int(threadIdx.x) < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    return part[0];
}

__global__ __launch_bounds__(256) void k_risk_part(SortWs w, RiskKs ks) {
    __shared__ double part[256];
    const uint64_t *keys = cur_keys(w, kPasses);
    const int r = blockIdx.y;
    const int64_t k = ks.k[r], chunk = ks.chunk[r];
    const int64_t lo = int64_t(blockIdx.x) * chunk;
    const int64_t hi = lo + chunk < k ? lo + chunk : k;
    // each thread adds its keys lo + t, lo + t + 256, ... in that order; 8 are read
    // before they are added.  Slots past hi add +0.0, which changes no sum here: the
    // running sum starts at +0.0 and round-to-nearest addition never makes it -0.0.
    constexpr int kAhead = 8;
    double s = 0.0;
    for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += kAhead * blockDim.x) {
        double v[kAhead];
#pragma unroll
        for (int u = 0; u < kAhead; ++u) {
            const int64_t i = i0 + int64_t(u) * blockDim.x;
            v[u] = i < hi ? key_value(keys[i]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kAhead; ++u) s += v[u];
    }
    s = block_sum(s, part);
    if (threadIdx.x == 0) w.part[r * kRiskMaxBlocks + blockIdx.x] = s;   // 0 past k
}

__global__ __launch_bounds__(256) void k_risk_final(SortWs w, RiskKs ks, int n_k, int nb, double *__restrict__ out) {
    __shared__ double part[256];
    const uint64_t *keys = cur_keys(w, kPasses);
    const int r = blockIdx.x;
    const int64_t k = ks.k[r];
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += w.part[r * kRiskMaxBlocks + b];
    s = block_sum(s, part);
    if (threadIdx.x == 0) {
        out[r] = key_value(keys[k - 1]);
        out[n_k + r] = s / double(k);
    }
}

hipError_t launch_risk(const void *ws, int64_t n, const int64_t *ks, int n_k, double *out, hipStream_t s) {
    SortWs w = sort_ws(const_cast<void *>(ws), n);
    for (int base = 0; base < n_k; base += kRiskGroup) {
        RiskKs r{};
        const int m = std::min(kRiskGroup, n_k - base);
        int64_t nb = 1;
        for (int i = 0; i < m; ++i) {
            const int64_t k = ks[base + i];
            int64_t chunk = (k + kRiskMaxBlocks - 1) / kRiskMaxBlocks;
            chunk = chunk < kRiskChunk ? kRiskChunk : chunk;
            r.k[i] = k;
            r.chunk[i] = chunk;
            nb = std::max(nb, (k + chunk - 1) / chunk);
        }
        // out layout per group: pml[m], tvar[m]
        hipLaunchKernelGGL(k_risk_part, dim3(unsigned(nb), unsigned(m)), dim3(256), 0, s, w, r);
        hipLaunchKernelGGL(k_risk_final, dim3(unsigned(m)), dim3(256), 0, s, w, r, m, int(nb), out + 2 * base);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------------
// Batched risk measures of many small YLTs (n <= kRiskLdsKeys each): one workgroup
// per YLT sorts its keys in LDS (bitonic network; the array is padded to a power of
// two with the largest key, which sorts last) and then forms PML and TVaR from the
// sorted keys with exactly the chunks and sums of k_risk_part/k_risk_final, so the
// results equal those of ara_risk_measures on the same YLT bit for bit.
__device__ __forceinline__ double sum256(double s, double *part) {
    // the 256-thread tree of block_sum, threads >= 256 only keep the barriers
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

__global__ __launch_bounds__(1024) void k_risk_batch(const double *const *__restrict__ ylts,
                                                     const int64_t *__restrict__ ns, const int64_t *__restrict__ ks,
                                                     int n_k, double *__restrict__ out) {
    __shared__ uint64_t key[kRiskLdsKeys];
    __shared__ double part[256];
    __shared__ double chunk_sum[kRiskLdsKeys / kRiskChunk];
    const int j = blockIdx.x;
    if (ns[j] < 1 || ns[j] > kRiskLdsKeys) return;   // longer YLTs take the radix sort
    const int n = int(ns[j]);
    const double *y = ylts[j];
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
    for (int r = 0; r < n_k; ++r) {
        const int64_t k = ks[int64_t(j) * n_k + r];
        int64_t chunk = (k + kRiskMaxBlocks - 1) / kRiskMaxBlocks;
        chunk = chunk < kRiskChunk ? kRiskChunk : chunk;
        const int nb = int((k + chunk - 1) / chunk);   // <= kRiskLdsKeys / kRiskChunk here
        for (int b = 0; b < nb; ++b) {
            const int64_t lo = b * chunk, hi = lo + chunk < k ? lo + chunk : k;
            double s = 0.0;
            if (threadIdx.x < 256)
                for (int64_t i = lo + threadIdx.x; i < hi; i += 256) s += key_value(key[i]);
            s = sum256(s, part);
            if (threadIdx.x == 0) chunk_sum[b] = s;
            __syncthreads();
        }
        double s = 0.0;
        if (threadIdx.x < 256)
            for (int b = threadIdx.x; b < nb; b += 256) s += chunk_sum[b];
        s = sum256(s, part);
        if (threadIdx.x == 0) {
            out[int64_t(j) * 2 * n_k + r] = key_value(key[k - 1]);
            out[int64_t(j) * 2 * n_k + n_k + r] = s / double(k);
        }
    }
}

hipError_t launch_risk_batch(const double *const *ylts, const int64_t *ns, const int64_t *ks, int n_jobs, int n_k,
                             double *out, hipStream_t s) {
    if (n_jobs <= 0 || n_k <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_risk_batch, dim3(unsigned(n_jobs)), dim3(1024), 0, s, ylts, ns, ks, n_k, out);
    return hipGetLastError();
}

}  // namespace ara
