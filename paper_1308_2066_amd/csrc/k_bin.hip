// Catalog-binned copy of a YET (built once, at YET creation).
//
// The trial kernel of Section III-B looks every occurrence up in a table over the
// whole catalog.  When the layer's table does not fit in LDS, the tiled trial
// kernel instead walks the catalog in LDS-sized tiles and, for each tile, streams
// only the occurrences of that tile's events.  To make those occurrences contiguous
// the YET is regrouped by catalog bin (2^15 events): region b holds, for every
// trial in order, the trial's occurrences of bin-b events in time order, each as
// its 15-bit ID within the bin.  boff[b][t] gives where trial t's run starts in
// region b, so a tile's occurrences of any trial range are one contiguous span per
// bin.  The regrouping only changes which occurrences are read together; each
// trial still has exactly its own occurrences.
#include "ara_internal.h"

namespace ara {

// boff[b][t] = number of trial t's occurrences in bin b; boff[b][n_trials] = 0.
// One wave per trial, counting in an LDS histogram.
__global__ __launch_bounds__(64) void k_bin_count(const int32_t *__restrict__ ids, const int64_t *__restrict__ offs,
                                                  int64_t n_trials, int32_t n_bins, uint32_t *__restrict__ boff,
                                                  int64_t stride) {
    __shared__ uint32_t hist[kMaxBins];
    const int lane = threadIdx.x;
    if (blockIdx.x == 0)
        for (int32_t b = lane; b < n_bins; b += 64) boff[b * stride + n_trials] = 0u;
    for (int64_t t = blockIdx.x; t < n_trials; t += gridDim.x) {
        for (int32_t b = lane; b < n_bins; b += 64) hist[b] = 0u;
        __syncthreads();
        const int64_t o0 = offs[t], o1 = offs[t + 1];
        for (int64_t i = o0 + lane; i < o1; i += 64) atomicAdd(&hist[uint32_t(ids[i]) >> kBinShift], 1u);
        __syncthreads();
        for (int32_t b = lane; b < n_bins; b += 64) boff[b * stride + t] = hist[b];
        __syncthreads();
    }
}

hipError_t launch_bin_count(const int32_t *ids, const int64_t *offs, int64_t n_trials, int32_t n_bins,
                            uint32_t *boff, int64_t stride, hipStream_t s) {
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(n_trials, 65536));
    hipLaunchKernelGGL(k_bin_count, dim3(unsigned(grid)), dim3(64), 0, s, ids, offs, n_trials, n_bins, boff, stride);
    return hipGetLastError();
}

// Exclusive prefix sums along each boff row (entries 0..n_entries-1), in three
// steps: per 4096-entry block (local scan, block total), per row (scan of the block
// totals), per block (add the block's offset).
constexpr int kScanBlock = 4096;

size_t bin_scan_scratch_words(int64_t n_entries, int32_t n_bins) {
    return size_t((n_entries + kScanBlock - 1) / kScanBlock) * size_t(n_bins);
}

__global__ __launch_bounds__(1024) void k_bin_scan_local(uint32_t *__restrict__ boff, int64_t stride,
                                                         int64_t n_entries, uint32_t *__restrict__ sums) {
    __shared__ uint32_t wsum[16];
    const int64_t nblk = (n_entries + kScanBlock - 1) / kScanBlock;
    uint32_t *row = boff + int64_t(blockIdx.y) * stride;
    const int64_t i0 = int64_t(blockIdx.x) * kScanBlock + 4 * threadIdx.x;
    uint32_t v[4], own = 0;
    for (int k = 0; k < 4; ++k) {
        v[k] = i0 + k < n_entries ? row[i0 + k] : 0u;
        own += v[k];
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = own;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int k = 0; k < 16; ++k) {
        if (k < w) before += wsum[k];
        total += wsum[k];
    }
    uint32_t run = before + inc - own;
    for (int k = 0; k < 4; ++k) {
        if (i0 + k < n_entries) row[i0 + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) sums[int64_t(blockIdx.y) * nblk + blockIdx.x] = total;
}

__global__ void k_bin_scan_top(uint32_t *__restrict__ sums, int64_t nblk, int32_t n_bins) {
    const int32_t b = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= n_bins) return;
    uint32_t run = 0;
    for (int64_t k = 0; k < nblk; ++k) {
        const uint32_t x = sums[int64_t(b) * nblk + k];
        sums[int64_t(b) * nblk + k] = run;
        run += x;
    }
}

__global__ __launch_bounds__(1024) void k_bin_scan_add(uint32_t *__restrict__ boff, int64_t stride,
                                                       int64_t n_entries, const uint32_t *__restrict__ sums) {
    const int64_t nblk = (n_entries + kScanBlock - 1) / kScanBlock;
    const uint32_t add = sums[int64_t(blockIdx.y) * nblk + blockIdx.x];
    if (add == 0) return;
    uint32_t *row = boff + int64_t(blockIdx.y) * stride;
    const int64_t i0 = int64_t(blockIdx.x) * kScanBlock;
    for (int k = threadIdx.x; k < kScanBlock; k += blockDim.x)
        if (i0 + k < n_entries) row[i0 + k] += add;
}

hipError_t launch_bin_scan(uint32_t *boff, int64_t stride, int64_t n_entries, int32_t n_bins, uint32_t *sums,
                           hipStream_t s) {
    const int64_t nblk = (n_entries + kScanBlock - 1) / kScanBlock;
    if (nblk > 65535 || n_bins > 65535) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(nblk), static_cast<unsigned>(n_bins));
    hipLaunchKernelGGL(k_bin_scan_local, grid, dim3(1024), 0, s, boff, stride, n_entries, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_scan_top, dim3(unsigned((n_bins + 63) / 64)), dim3(64), 0, s, sums, nblk, n_bins);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_scan_add, grid, dim3(1024), 0, s, boff, stride, n_entries, sums);
    return hipGetLastError();
}

// Writes each occurrence at region[b] + boff[b][t] + (its rank among trial t's
// earlier occurrences of bin b): one wave per trial, 64 occurrences at a time; the
// lanes of a chunk that share a bin are placed in lane order (stable).
__global__ __launch_bounds__(64) void k_bin_scatter(const int32_t *__restrict__ ids, const int64_t *__restrict__ offs,
                                                    int64_t n_trials, int32_t n_bins, const uint32_t *__restrict__ boff,
                                                    int64_t stride, const int64_t *__restrict__ region,
                                                    uint16_t *__restrict__ ids16) {
    __shared__ int64_t cur[kMaxBins];   // next write position of the trial's run in each bin
    const int lane = threadIdx.x;
    for (int64_t t = blockIdx.x; t < n_trials; t += gridDim.x) {
        for (int32_t b = lane; b < n_bins; b += 64) cur[b] = region[b] + int64_t(boff[b * stride + t]);
        __syncthreads();
        const int64_t o0 = offs[t], o1 = offs[t + 1];
        for (int64_t base = o0; base < o1; base += 64) {
            const int64_t i = base + lane;
            const bool valid = i < o1;
            const uint32_t id = valid ? uint32_t(ids[i]) : 0u;
            const int32_t b = int32_t(id >> kBinShift);
            uint64_t todo = __ballot(valid);
            while (todo) {
                const int leader = __builtin_ctzll(todo);
                const int32_t bl = __builtin_amdgcn_readlane(b, leader);
                const uint64_t m = __ballot(valid && b == bl);
                const int64_t at = cur[bl];
                if (valid && b == bl) {
                    const uint32_t r = __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
                    ids16[at + r] = uint16_t(id & uint32_t(kBinEvents - 1));
                }
                __syncthreads();
                if (lane == leader) cur[bl] = at + __popcll(m);
                __syncthreads();
                todo &= ~m;
            }
        }
        __syncthreads();
    }
}

hipError_t launch_bin_scatter(const int32_t *ids, const int64_t *offs, int64_t n_trials, int32_t n_bins,
                              const uint32_t *boff, int64_t stride, const int64_t *region, uint16_t *ids16,
                              hipStream_t s) {
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(n_trials, 65536));
    hipLaunchKernelGGL(k_bin_scatter, dim3(unsigned(grid)), dim3(64), 0, s, ids, offs, n_trials, n_bins, boff, stride,
                       region, ids16);
    return hipGetLastError();
}

}  // namespace ara
