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
#include <type_traits>

#include "ara_internal.h"

namespace ara {

// boff[b][t] = number of trial t's occurrences in bin b; boff[b][n_trials] = 0.
// One wave per trial (four per workgroup), counting in the wave's own LDS
// histogram; a wave's LDS operations complete in order, so it needs no barrier.
// The YET is checked on the way, as ara_yet_create states: a trial's offsets must lie
// in [0, n_events] in order, the first be 0 and the last n_events (else ERR_OFFSETS
// and the trial's IDs are not read), every ID be in [0, catalog) (else ERR_ID_RANGE
// and the ID is not counted).
constexpr int kCountWaves = 4;

__global__ __launch_bounds__(kCountWaves * 64) void k_bin_count(const int32_t *__restrict__ ids,
                                                                const int64_t *__restrict__ offs, int64_t n_events,
                                                                int64_t n_trials, int32_t n_bins,
                                                                uint32_t *__restrict__ boff, int64_t stride,
                                                                int32_t catalog, uint32_t *err) {
    __shared__ uint32_t hist[kCountWaves][kMaxBins];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t cat = uint32_t(catalog);
    uint32_t *h = hist[wave];
    bool bad = false, bad_offs = false;
    if (blockIdx.x == 0)
        for (int32_t b = threadIdx.x; b < n_bins; b += kCountWaves * 64) boff[b * stride + n_trials] = 0u;
    for (int64_t t = int64_t(blockIdx.x) * kCountWaves + wave; t < n_trials; t += int64_t(gridDim.x) * kCountWaves) {
        for (int32_t b = lane; b < n_bins; b += 64) h[b] = 0u;
        __builtin_amdgcn_wave_barrier();
        int64_t o0 = offs[t], o1 = offs[t + 1];
        if (o0 < 0 || o1 < o0 || o1 > n_events || (t == 0 && o0 != 0) || (t == n_trials - 1 && o1 != n_events)) {
            bad_offs = true;
            o1 = o0;   // read none of this trial's IDs
        }
        constexpr int kAhead = 16;   // loads in flight per lane (4 KB per wave: enough to keep HBM busy)
        for (int64_t base = o0; base < o1; base += 64 * kAhead) {
            uint32_t v[kAhead];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) {
                const int64_t i = base + 64 * u + lane;
                v[u] = i < o1 ? uint32_t(ids[i]) : 0u;
            }
#pragma unroll
            for (int u = 0; u < kAhead; ++u) {
                if (base + 64 * u + lane >= o1) continue;
                if (v[u] < cat) atomicAdd(&h[v[u] >> kBinShift], 1u);
                else bad = true;
            }
        }
        __builtin_amdgcn_wave_barrier();
        for (int32_t b = lane; b < n_bins; b += 64) boff[b * stride + t] = h[b];
        __builtin_amdgcn_wave_barrier();
    }
    const uint32_t flags = (__builtin_amdgcn_ballot_w64(bad) ? ERR_ID_RANGE : 0u) |
                           (__builtin_amdgcn_ballot_w64(bad_offs) ? ERR_OFFSETS : 0u);
    if (flags && lane == 0) atomicOr(err, flags);
}

hipError_t launch_bin_count(const int32_t *ids, const int64_t *offs, int64_t n_events, int64_t n_trials, int32_t n_bins,
                            uint32_t *boff, int64_t stride, int32_t catalog, uint32_t *err, hipStream_t s) {
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>((n_trials + kCountWaves - 1) / kCountWaves, 65536));
    hipLaunchKernelGGL(k_bin_count, dim3(unsigned(grid)), dim3(kCountWaves * 64), 0, s, ids, offs, n_events, n_trials,
                       n_bins, boff, stride, catalog, err);
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

// Region starts from the scanned offsets: region[0] = 0, region[b + 1] = region[b] +
// (bin b's length rounded up to 8), bin b's length being boff[b][n_trials] after the
// scan.  One wave, up to 512 bins (8 per lane).  Skipped when the count pass found a
// bad ID or offset (err set): the scatter is skipped then too.
__global__ __launch_bounds__(64) void k_bin_regions(const uint32_t *__restrict__ boff, int64_t stride, int64_t n_trials,
                                                    int32_t n_bins, int64_t *__restrict__ region,
                                                    const uint32_t *__restrict__ err) {
    if (*err != 0u) return;
    const int lane = threadIdx.x;
    int64_t v[8], own = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int32_t b = lane * 8 + k;
        v[k] = b < n_bins ? (int64_t(boff[int64_t(b) * stride + n_trials]) + 7) & ~int64_t(7) : 0;
        own += v[k];
    }
    int64_t inc = own;
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    int64_t run = inc - own;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int32_t b = lane * 8 + k;
        if (b < n_bins) region[b] = run;
        run += v[k];
    }
    if (lane == 63) region[n_bins] = inc;   // the total
}

hipError_t launch_bin_regions(const uint32_t *boff, int64_t stride, int64_t n_trials, int32_t n_bins, int64_t *region,
                              const uint32_t *err, hipStream_t s) {
    if (n_bins > kMaxBins || kMaxBins > 8 * 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bin_regions, dim3(1), dim3(64), 0, s, boff, stride, n_trials, n_bins, region, err);
    return hipGetLastError();
}

// Writes each occurrence at region[b] + boff[b][t] + (its rank among trial t's
// earlier occurrences of bin b).  A workgroup takes `per_block` consecutive trials;
// their occurrences of bin b form one contiguous span of region b, so when the
// block's occurrences fit in LDS they are placed there first (a counting sort by
// bin) and each bin's span is then written with consecutive stores.  A block with
// more occurrences than the LDS holds writes every occurrence to its place directly.
// Either way a wave takes one trial at a time, 64 occurrences per step in time
// order; lanes of a step that share a bin are ranked in lane order, so each run keeps
// the trial's time order.  The mask of lanes with the same bin comes from LDS when
// the bins fit a wave's table (at most 64: every lane ORs its bit into its bin's
// word, reads the word back and clears it; ORs do not depend on the order the lanes
// are taken in), else from one ballot per bit of the bin number (six ballots per
// step cost 1.6 ms of a 10^9-occurrence ingest, the LDS masks 0.5 ms).
constexpr int kScatterWaves = 16;
constexpr int kScatterCap = 61440;   // occurrences staged per workgroup (120 KB)

int64_t bin_scatter_block_trials(int64_t n_events, int64_t n_trials) {
    const double mean = n_trials > 0 ? double(n_events) / double(n_trials) : 0.0;
    const double by_cap = mean > 0.0 ? 0.75 * double(kScatterCap) / mean : 4096.0;
    return std::max<int64_t>(1, std::min<int64_t>(4096, int64_t(by_cap)));
}

// Rank of this lane among the lanes of `valid` whose bin equals its own, and their
// number; NBITS = bits needed for the largest bin number.
template <int NBITS>
__device__ __forceinline__ void same_bin_rank(uint32_t b, uint64_t valid, uint32_t &rank, uint32_t &count) {
    uint64_t m = valid;
#pragma unroll
    for (int k = 0; k < NBITS; ++k) {
        const bool bit = (b >> k) & 1u;
        const uint64_t ones = __builtin_amdgcn_ballot_w64(bit);
        m &= bit ? ones : ~ones;
    }
    rank = __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
    count = uint32_t(__popcll(m));
}

template <int NBITS, bool STAGED>
__global__ __launch_bounds__(kScatterWaves * 64) void k_bin_scatter(const int32_t *__restrict__ ids,
                                                                    const int64_t *__restrict__ offs, int64_t n_trials,
                                                                    int32_t n_bins, const uint32_t *__restrict__ boff,
                                                                    int64_t stride, const int64_t *__restrict__ region,
                                                                    uint16_t *__restrict__ ids16, int64_t per_block,
                                                                    const uint32_t *__restrict__ err) {
    constexpr int kBins = NBITS <= 6 ? 64 : kMaxBins;   // bins the LDS tables hold
    __shared__ uint16_t stage[STAGED ? kScatterCap : 2];
    __shared__ uint32_t cur[kScatterWaves][kBins];      // next position of the wave's trial's run, per bin
    __shared__ uint32_t lbase[kBins + 1];               // start of bin b's span in `stage`
    __shared__ uint32_t bstart[kBins];                  // boff[b][t0]
    __shared__ uint64_t lanes_of[NBITS <= 6 ? kScatterWaves : 1][NBITS <= 6 ? 64 : 1];   // per wave and bin: its lanes
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t t0 = int64_t(blockIdx.x) * per_block;
    if (t0 >= n_trials) return;
    // the count pass found a bad ID or offset: the counts do not describe the input
    if (*err != 0u) return;
    const int64_t t1 = min(t0 + per_block, n_trials);
    // a block with more occurrences than the LDS holds is left to the unstaged launch
    // (and the unstaged launch leaves the others)
    if ((offs[t1] - offs[t0] <= int64_t(kScatterCap)) != STAGED) return;
    constexpr bool staged = STAGED;
    uint32_t *wc = cur[wave];
    uint64_t *lm = lanes_of[NBITS <= 6 ? wave : 0];
    if (NBITS <= 6) lm[lane] = 0;
    if (staged) {
        for (int32_t b = threadIdx.x; b < n_bins; b += kScatterWaves * 64) {
            const uint32_t s = boff[b * stride + t0];
            bstart[b] = s;
            lbase[b + 1] = boff[b * stride + t1] - s;
        }
        __syncthreads();
        if (wave == 0) {   // exclusive scan of the span lengths, 8 bins per lane
            uint32_t v[8], own = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int32_t b = lane * 8 + k;
                v[k] = b < n_bins ? lbase[b + 1] : 0u;
                own += v[k];
            }
            uint32_t inc = own;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(inc, o, 64);
                if (lane >= o) inc += y;
            }
            uint32_t run = inc - own;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int32_t b = lane * 8 + k;
                if (b < n_bins) lbase[b] = run;
                run += v[k];
            }
            if (lane == 63) lbase[n_bins] = run;
        }
        __syncthreads();
    }
    // a trial's IDs are read a chunk of kChunkSteps steps of 64 ahead of the step
    // that places them, so a wave waits for about one load per chunk rather than one
    // per step, and enough bytes are in flight to keep HBM busy
    constexpr int kChunkSteps = 16;   // 4 KB of IDs in flight per wave (a 1000-event trial at once)
    for (int64_t t = t0 + wave; t < t1; t += kScatterWaves) {
        for (int32_t b = lane; b < n_bins; b += 64)
            wc[b] = staged ? lbase[b] + boff[b * stride + t] - bstart[b] : boff[b * stride + t];
        __builtin_amdgcn_wave_barrier();
        const int64_t o0 = offs[t], o1 = offs[t + 1];
        uint32_t cur[kChunkSteps];
#pragma unroll
        for (int u = 0; u < kChunkSteps; ++u) {
            const int64_t i = o0 + 64 * u + lane;
            cur[u] = i < o1 ? uint32_t(ids[i]) : 0u;
        }
        for (int64_t base = o0; base < o1; base += 64 * kChunkSteps) {
            uint32_t nxt[kChunkSteps];
#pragma unroll
            for (int u = 0; u < kChunkSteps; ++u) {
                const int64_t i = base + 64 * (kChunkSteps + u) + lane;
                nxt[u] = i < o1 ? uint32_t(ids[i]) : 0u;
            }
#pragma unroll
            for (int u = 0; u < kChunkSteps; ++u) {
                const bool valid = base + 64 * u + lane < o1;
                const uint32_t id = cur[u];
                const uint32_t b = id >> kBinShift;
                uint32_t rank, count;
                if (NBITS <= 6) {
                    // the lanes of this step with bin b: every lane ORs its bit into its bin's
                    // mask (an OR does not depend on the order the lanes are taken in), reads the
                    // mask back and clears it
                    const uint32_t bb = valid ? b : 63u;
                    __hip_atomic_fetch_or(&lm[bb], valid ? uint64_t(1) << lane : uint64_t(0), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_WAVEFRONT);
                    const uint64_t m = lm[bb];
                    __builtin_amdgcn_wave_barrier();
                    lm[bb] = 0;
                    rank = __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
                    count = uint32_t(__popcll(m));
                } else {
                    same_bin_rank<NBITS>(b, __builtin_amdgcn_ballot_w64(valid), rank, count);
                }
                const uint32_t at = wc[b];
                const uint16_t local = uint16_t(id & uint32_t(kBinEvents - 1));
                if (valid) {
                    if (staged) stage[at + rank] = local;
                    else ids16[region[b] + int64_t(at + rank)] = local;
                    if (rank + 1 == count) wc[b] = at + count;
                }
                __builtin_amdgcn_wave_barrier();
            }
#pragma unroll
            for (int u = 0; u < kChunkSteps; ++u) cur[u] = nxt[u];
        }
    }
    if (!staged) return;
    __syncthreads();
    // each bin's span to its place in region b, consecutive lanes on consecutive IDs
    for (int32_t b = wave; b < n_bins; b += kScatterWaves) {
        const uint32_t l0 = lbase[b], len = lbase[b + 1] - l0;
        uint16_t *dst = ids16 + region[b] + int64_t(bstart[b]);
        for (uint32_t k = lane; k < len; k += 64) dst[k] = stage[l0 + k];
    }
}

hipError_t launch_bin_scatter(const int32_t *ids, const int64_t *offs, int64_t n_events, int64_t n_trials,
                              int32_t n_bins, const uint32_t *boff, int64_t stride, const int64_t *region,
                              uint16_t *ids16, const uint32_t *err, hipStream_t s) {
    if (n_trials <= 0) return hipSuccess;
    if (n_bins > kMaxBins) return hipErrorInvalidValue;
    const int64_t per = bin_scatter_block_trials(n_events, n_trials);
    const int64_t grid = (n_trials + per - 1) / per;
    if (grid > int64_t(INT32_MAX)) return hipErrorInvalidValue;
    const int nbits = n_bins > 1 ? 32 - __builtin_clz(uint32_t(n_bins - 1)) : 0;
    // one instantiation per bit count of the bin numbers (the rank's ballots unrolled),
    // each launched for the staged blocks and then for the others
    hipError_t e = hipSuccess;
    auto launch = [&](auto nb_const) {
        constexpr int NB = decltype(nb_const)::value;
        hipLaunchKernelGGL((k_bin_scatter<NB, true>), dim3(unsigned(grid)), dim3(kScatterWaves * 64), 0, s, ids, offs,
                           n_trials, n_bins, boff, stride, region, ids16, per, err);
        e = hipGetLastError();
        if (e != hipSuccess) return;
        hipLaunchKernelGGL((k_bin_scatter<NB, false>), dim3(unsigned(grid)), dim3(kScatterWaves * 64), 0, s, ids, offs,
                           n_trials, n_bins, boff, stride, region, ids16, per, err);
        e = hipGetLastError();
    };
    switch (nbits) {
    case 0: launch(std::integral_constant<int, 0>()); break;
    case 1: launch(std::integral_constant<int, 1>()); break;
    case 2: launch(std::integral_constant<int, 2>()); break;
    case 3: launch(std::integral_constant<int, 3>()); break;
    case 4: launch(std::integral_constant<int, 4>()); break;
    case 5: launch(std::integral_constant<int, 5>()); break;
    case 6: launch(std::integral_constant<int, 6>()); break;
    case 7: launch(std::integral_constant<int, 7>()); break;
    case 8: launch(std::integral_constant<int, 8>()); break;
    case 9: launch(std::integral_constant<int, 9>()); break;
    default: return hipErrorInvalidValue;
    }
    return e;
}

}  // namespace ara
