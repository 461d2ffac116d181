// Output filters (Section II-C): the YLT sorted in descending order, then
// PML = the k-th largest loss and TVaR = the mean of the k largest, with k set by
// the return period (the paper names both measures, Section I, but does not define
// them; the engine's rank rule is ara_return_period_rank).
//
// LSD radix sort of 64-bit keys, 8-bit digits, 8 passes.  A binary64 value maps to
// an unsigned key whose order is the value order (sign flip for non-negatives,
// complement for negatives, -0.0 canonicalised to +0.0); descending order sorts the
// complemented key ascending.  Each pass: per-tile digit counts, one exclusive scan
// over (digit, tile), and a stable scatter in which every wave ranks its keys by
// matching digits across lanes with 8 ballots.
#include "ara_internal.h"

namespace ara {

constexpr int kSortThreads = 256;
constexpr int kSortPerThread = 16;
constexpr int kSortTile = kSortThreads * kSortPerThread;   // 4096 keys
constexpr int kWavesPerTile = kSortThreads / 64;            // 4, each owns 1024 consecutive keys

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

size_t sort_workspace_bytes(int64_t n) {
    const size_t keys = (size_t(n) * 8 + 255) & ~size_t(255);
    const size_t counts = (size_t(sort_tiles(n)) * 256 * 4 + 255) & ~size_t(255);
    return 2 * keys + counts + 256;
}

struct SortWs {
    uint64_t *a, *b;
    uint32_t *counts;
};

static SortWs sort_ws(void *ws, int64_t n) {
    const size_t keys = (size_t(n) * 8 + 255) & ~size_t(255);
    char *p = reinterpret_cast<char *>(ws);
    return SortWs{reinterpret_cast<uint64_t *>(p), reinterpret_cast<uint64_t *>(p + keys),
                  reinterpret_cast<uint32_t *>(p + 2 * keys)};
}

__global__ __launch_bounds__(256) void k_sort_encode(const double *__restrict__ in, int64_t n,
                                                     uint64_t *__restrict__ keys) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        keys[i] = desc_key(in[i]);
}

__global__ __launch_bounds__(256) void k_sort_decode(const uint64_t *__restrict__ keys, int64_t n,
                                                     double *__restrict__ out) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        out[i] = key_value(keys[i]);
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
__global__ __launch_bounds__(kSortThreads) void k_sort_count(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                                            uint32_t *__restrict__ counts, int64_t tiles) {
    __shared__ uint32_t hist[256];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    hist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = int64_t(blockIdx.x) * kSortTile + w * 1024;
    for (int r = 0; r < kSortPerThread; ++r) {
        const int64_t i = base + r * 64 + lane;
        const bool valid = i < n;
        const uint32_t d = valid ? uint32_t(keys[i] >> shift) & 255u : 0u;
        const uint64_t m = match_digit(d, valid);
        if (valid && (m & lanes_below(lane)) == 0) atomicAdd(&hist[d], uint32_t(__popcll(m)));
    }
    __syncthreads();
    counts[int64_t(threadIdx.x) * tiles + blockIdx.x] = hist[threadIdx.x];
}

// In-place exclusive scan of len counters (one workgroup of 1024).
__global__ __launch_bounds__(1024) void k_sort_scan(uint32_t *__restrict__ c, int64_t len) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (len + 1023) / 1024;
    const int64_t b = t * per, e = (b + per < len) ? b + per : len;
    uint32_t s = 0;
    for (int64_t i = b; i < e; ++i) s += c[i];
    part[t] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {   // inclusive Hillis-Steele scan of the partial sums
        const uint32_t v = t >= o ? part[t - o] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - s;
    for (int64_t i = b; i < e; ++i) {
        const uint32_t v = c[i];
        c[i] = run;
        run += v;
    }
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(const uint64_t *__restrict__ in,
                                                              uint64_t *__restrict__ out, int64_t n, int shift,
                                                              const uint32_t *__restrict__ offs, int64_t tiles) {
    __shared__ uint32_t whist[kWavesPerTile][256];
    __shared__ uint32_t woff[kWavesPerTile][256];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int k = 0; k < kWavesPerTile; ++k) whist[k][threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = int64_t(blockIdx.x) * kSortTile + w * 1024;
    uint64_t key[kSortPerThread];
    uint32_t rank[kSortPerThread];
    for (int r = 0; r < kSortPerThread; ++r) {
        const int64_t i = base + r * 64 + lane;
        const bool valid = i < n;
        key[r] = valid ? in[i] : 0ull;
        const uint32_t d = uint32_t(key[r] >> shift) & 255u;
        const uint64_t m = match_digit(d, valid);
        const uint64_t below = m & lanes_below(lane);
        rank[r] = whist[w][d] + uint32_t(__popcll(below));   // read before this round's update
        if (valid && below == 0) whist[w][d] += uint32_t(__popcll(m));
    }
    __syncthreads();
    {
        const int d = threadIdx.x;
        uint32_t run = offs[int64_t(d) * tiles + blockIdx.x];
        for (int k = 0; k < kWavesPerTile; ++k) {
            woff[k][d] = run;
            run += whist[k][d];
        }
    }
    __syncthreads();
    for (int r = 0; r < kSortPerThread; ++r) {
        const int64_t i = base + r * 64 + lane;
        if (i < n) {
            const uint32_t d = uint32_t(key[r] >> shift) & 255u;
            out[woff[w][d] + rank[r]] = key[r];
        }
    }
}

// Sorted descending keys of `in` end in the first key buffer of the workspace.
hipError_t launch_sort_desc_keys(const double *in, int64_t n, void *ws, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    SortWs w = sort_ws(ws, n);
    const int64_t tiles = sort_tiles(n);
    const unsigned eb = unsigned(std::min<int64_t>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k_sort_encode, dim3(eb), dim3(256), 0, s, in, n, w.a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint64_t *src = w.a, *dst = w.b;
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = pass * 8;
        hipLaunchKernelGGL(k_sort_count, dim3(unsigned(tiles)), dim3(kSortThreads), 0, s, src, n, shift, w.counts, tiles);
        hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, s, w.counts, tiles * 256);
        hipLaunchKernelGGL(k_sort_scatter, dim3(unsigned(tiles)), dim3(kSortThreads), 0, s, src, dst, n, shift, w.counts,
                           tiles);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint64_t *t = src;
        src = dst;
        dst = t;
    }
    return hipSuccess;   // 8 passes: result back in w.a
}

hipError_t launch_sort_decode(const void *ws, int64_t n, double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    SortWs w = sort_ws(const_cast<void *>(ws), n);
    const unsigned eb = unsigned(std::min<int64_t>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k_sort_decode, dim3(eb), dim3(256), 0, s, w.a, n, out);
    return hipGetLastError();
}

// One workgroup per return period: PML = k-th largest, TVaR = mean of the k largest,
// summed with a fixed per-thread stride and a fixed LDS tree (deterministic).
struct RiskKs {
    int64_t k[16];
};

__global__ __launch_bounds__(1024) void k_risk(const uint64_t *__restrict__ keys, RiskKs ks, int n_k,
                                               double *__restrict__ out) {
    __shared__ double part[1024];
    const int64_t k = ks.k[blockIdx.x];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < k; i += 1024) s += key_value(keys[i]);
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 512; o >= 1; o >>= 1) {
        if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[blockIdx.x] = key_value(keys[k - 1]);
        out[n_k + blockIdx.x] = part[0] / double(k);
    }
}

hipError_t launch_risk(const void *ws, int64_t n, const int64_t *ks, int n_k, double *out, hipStream_t s) {
    SortWs w = sort_ws(const_cast<void *>(ws), n);
    for (int base = 0; base < n_k; base += 16) {
        RiskKs r{};
        const int m = std::min(16, n_k - base);
        for (int i = 0; i < m; ++i) r.k[i] = ks[base + i];
        // out layout per group: pml[m], tvar[m]
        hipLaunchKernelGGL(k_risk, dim3(unsigned(m)), dim3(1024), 0, s, w.a, r, m, out + 2 * base);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace ara
