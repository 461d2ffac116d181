// Catalog-binned copy of a YET (built once, at YET creation).
//
// The trial kernel of Section III-B looks every occurrence up in a table over the
// whole catalog.  When the layer's table does not fit in LDS, the tiled trial
// kernel instead walks the catalog one 2^14-event bin at a time, with the bin's
// slice of the table in LDS, and for each bin streams only the occurrences of
// that bin's events.  To make those occurrences contiguous the YET is regrouped by
// bin: region b holds, for every trial in order, the trial's occurrences of bin-b
// events in time order, each as its 14-bit ID within the bin (2 bytes).
// The run start of trial t in region b (4 bytes, or 3 bytes when asked for and every
// bin is shorter than 2^24) gives where its run starts, so the occurrences of any
// trial range in one bin are one contiguous span.  The regrouping only changes which
// occurrences are read together; each trial still has exactly its own occurrences.
//
// The build runs count, row scans, region starts and scatter back to back on the
// stream; the count pass checks the YET, and the later passes do nothing once it
// has flagged an error.
#include <type_traits>

#include "ara_internal.h"

namespace ara {

// boff[b][t] = number of trial t's occurrences in bin b; boff[b][n_trials] = 0.
// The YET is checked on the way, as ara_yet_create states: a trial's offsets must lie
// in [0, n_events] in order, the first be 0 and the last n_events (else ERR_OFFSETS
// and the trial's IDs are not read), every ID be in [0, catalog) (else ERR_ID_RANGE
// and the ID is not counted).
//
// Up to 512 bins: one wave per trial (four per workgroup), counting in the wave's
// own LDS histogram, then writing the counts, 4 bytes into each bin's row.
constexpr int kCountWaves = 4;

// One wave adds trial t's occurrences to the LDS histogram h (a wave's LDS
// operations complete in order, so the caller needs no barrier before reading it).
__device__ __forceinline__ void count_trial(const int32_t *__restrict__ ids, const int64_t *__restrict__ offs, int64_t t,
                                            int64_t n_events, int64_t n_trials, uint32_t cat, int lane, uint32_t *h,
                                            bool &bad, bool &bad_offs) {
    int64_t o0 = offs[t], o1 = offs[t + 1];
    if (o0 < 0 || o1 < o0 || o1 > n_events || (t == 0 && o0 != 0) || (t == n_trials - 1 && o1 != n_events)) {
        bad_offs = true;
        o1 = o0;   // read none of this trial's IDs
    }
    constexpr int kAhead = 16;   // loads in flight per lane (4 KB per wave)
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
}

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
        count_trial(ids, offs, t, n_events, n_trials, cat, lane, h, bad, bad_offs);
        __builtin_amdgcn_wave_barrier();
        for (int32_t b = lane; b < n_bins; b += 64) boff[b * stride + t] = h[b];
        __builtin_amdgcn_wave_barrier();
    }
    const uint32_t flags = (__builtin_amdgcn_ballot_w64(bad) ? ERR_ID_RANGE : 0u) |
                           (__builtin_amdgcn_ballot_w64(bad_offs) ? ERR_OFFSETS : 0u);
    if (flags && lane == 0) atomicOr(err, flags);
}

// Up to 64 bins (the paper-scale catalog has 62): a workgroup takes 64 consecutive
// trials (a block) at a time and its waves count them into an LDS table, a row per
// trial.  Each bin's 64 counts then become their exclusive prefix sums within the
// block (one wave scan), written with one coalesced store (4-byte entries, or 3-byte
// ones packed 4 to 12 bytes by every fourth lane), and the block's total goes to
// sums[b][block]; the block's start is added afterwards.  In the 3-byte form the
// entries up to the row's end are written (those past n_trials are padding), so the
// entry at n_trials gets its block's prefix when it falls in the last block.  (The
// per-trial stores of the kernel above, 4 bytes at a row stride apart, cost 0.3 ms
// more of a 10^9-occurrence ingest, and scanning the counts in separate passes
// 0.2 ms more.)
constexpr int kCountBlock = 64;
typedef uint32_t u32x3b __attribute__((ext_vector_type(3)));

template <bool B24>
__global__ __launch_bounds__(kCountWaves * 64) void k_bin_count_block(const int32_t *__restrict__ ids,
                                                                      const int64_t *__restrict__ offs,
                                                                      int64_t n_events, int64_t n_trials,
                                                                      int32_t n_bins, RunStarts r, int32_t catalog,
                                                                      uint32_t *__restrict__ sums, uint32_t *err) {
    __shared__ uint32_t hist[kCountBlock][65];   // padded rows: a bin's column reads without bank conflicts
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t cat = uint32_t(catalog);
    const int64_t nblk = (n_trials + kCountBlock - 1) / kCountBlock;
    bool bad = false, bad_offs = false;
    for (int64_t t0 = int64_t(blockIdx.x) * kCountBlock; t0 < n_trials; t0 += int64_t(gridDim.x) * kCountBlock) {
        for (int i = threadIdx.x; i < kCountBlock * 65; i += kCountWaves * 64) (&hist[0][0])[i] = 0u;
        __syncthreads();
        for (int j = wave; j < kCountBlock; j += kCountWaves) {
            const int64_t t = t0 + j;
            if (t >= n_trials) break;
            count_trial(ids, offs, t, n_events, n_trials, cat, lane, hist[j], bad, bad_offs);
        }
        __syncthreads();
        const int64_t t = t0 + lane;
        for (int32_t b = wave; b < n_bins; b += kCountWaves) {
            const uint32_t x = hist[lane][b];   // 0 past the last trial
            uint32_t inc = x;
            for (int k = 1; k < 64; k <<= 1) {
                const uint32_t y = __shfl_up(inc, k, 64);
                if (lane >= k) inc += y;
            }
            const uint32_t before = inc - x;
            if (B24) {
                const uint32_t v1 = __shfl_down(before, 1, 64), v2 = __shfl_down(before, 2, 64),
                               v3 = __shfl_down(before, 3, 64);
                if ((lane & 3) == 0 && t < r.stride) {   // t + 3 < stride too: both are multiples of 4
                    const u32x3b w = {before | (v1 << 24), (v1 >> 8) | (v2 << 16), (v2 >> 16) | (v3 << 8)};
                    *reinterpret_cast<u32x3b *>(r.b24 + 3 * (b * r.stride + t)) = w;   // 4-byte aligned
                }
            } else if (t < n_trials) {
                r.abs[b * r.stride + t] = before;
            }
            if (lane == 63) sums[b * nblk + t0 / kCountBlock] = inc;
        }
        __syncthreads();
    }
    const uint32_t flags = (__builtin_amdgcn_ballot_w64(bad) ? ERR_ID_RANGE : 0u) |
                           (__builtin_amdgcn_ballot_w64(bad_offs) ? ERR_OFFSETS : 0u);
    if (flags && lane == 0) atomicOr(err, flags);
}

// The block totals of one bin (a workgroup per bin) become their exclusive prefix
// sums in place, 16 per thread and 16384 per round; the bin's length goes to its
// entry at n_trials (in the 3-byte form only when that entry starts a block of its
// own: else the add below gives it), and a length of 2^24 or more in the 3-byte form
// sets ERR_BIN_WIDE.
template <bool B24>
__global__ __launch_bounds__(1024) void k_bin_block_scan(uint32_t *__restrict__ sums, int64_t nblk, RunStarts r,
                                                         int64_t n_trials, uint32_t *err) {
    __shared__ uint32_t wsum[16];
    uint32_t *row = sums + int64_t(blockIdx.x) * nblk;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t carry = 0;
    for (int64_t c0 = 0; c0 < nblk; c0 += 1024 * 16) {
        const int64_t i0 = c0 + 16 * int64_t(threadIdx.x);
        uint32_t v[16], own = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            v[k] = i0 + k < nblk ? row[i0 + k] : 0u;
            own += v[k];
        }
        uint32_t inc = own;
        for (int k = 1; k < 64; k <<= 1) {
            const uint32_t y = __shfl_up(inc, k, 64);
            if (lane >= k) inc += y;
        }
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        uint32_t before = 0, total = 0;
        for (int k = 0; k < 16; ++k) {
            if (k < w) before += wsum[k];
            total += wsum[k];
        }
        uint32_t run = carry + before + inc - own;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (i0 + k < nblk) row[i0 + k] = run;
            run += v[k];
        }
        carry += total;
        __syncthreads();   // wsum is reused
    }
    if (threadIdx.x != 0) return;
    const int64_t at = int64_t(blockIdx.x) * r.stride + n_trials;
    if (!B24) {
        r.abs[at] = carry;
        return;
    }
    if (carry >= (1u << 24)) atomicOr(err, ERR_BIN_WIDE);
    // a whole word (3 at is a multiple of 4 here); its top byte is the next entry's, padding
    if (n_trials % kCountBlock == 0) *reinterpret_cast<uint32_t *>(r.b24 + 3 * at) = carry;
}

// Adds to each run start the start of its block in the bin (sums after the scan),
// 4 entries per thread, 4096 per workgroup: the 4-byte entries t < n_trials (the one
// at n_trials holds the length), or the 3-byte ones of every block that has trials,
// as 12-byte groups (the last group may reach into padding).
template <bool B24>
__global__ __launch_bounds__(1024) void k_bin_block_add(RunStarts r, int64_t n_trials, const uint32_t *__restrict__ sums,
                                                        int64_t nblk) {
    typedef uint32_t u32x4b __attribute__((ext_vector_type(4)));
    const int64_t t = int64_t(blockIdx.x) * 4096 + 4 * int64_t(threadIdx.x);
    const int64_t b = blockIdx.y;
    if (B24) {
        if (t >= nblk * kCountBlock || t > n_trials) return;
        const uint32_t add = sums[b * nblk + t / kCountBlock];
        u32x3b *p = reinterpret_cast<u32x3b *>(r.b24 + 3 * (b * r.stride + t));   // 12 t: 4-byte aligned
        const u32x3b w = *p;
        const uint32_t v0 = (w[0] & 0xFFFFFFu) + add, v1 = ((w[0] >> 24) | (w[1] << 8)) + add,
                       v2 = ((w[1] >> 16) | (w[2] << 16)) + add, v3 = (w[2] >> 8) + add;
        *p = u32x3b{(v0 & 0xFFFFFFu) | (v1 << 24), ((v1 >> 8) & 0xFFFFu) | (v2 << 16),
                    ((v2 >> 16) & 0xFFu) | (v3 << 8)};
        return;
    }
    if (t >= n_trials) return;
    const uint32_t add = sums[b * nblk + t / kCountBlock];
    uint32_t *row = r.abs + b * r.stride;
    if (t + 4 <= n_trials) {   // rows start 16-byte aligned (stride is a multiple of 8)
        u32x4b *p = reinterpret_cast<u32x4b *>(row + t);
        *p = *p + add;
    } else {
        for (int64_t k = t; k < n_trials; ++k) row[k] += add;   // leaves the length at n_trials
    }
}

// Exclusive prefix sums along each boff row (entries 0..n_entries-1), in three
// steps: per 4096-entry block (local scan, block total), per row (scan of the block
// totals), per block (add the block's offset).
constexpr int kScanBlock = 4096;


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

static hipError_t launch_bin_scan(uint32_t *boff, int64_t stride, int64_t n_entries, int32_t n_bins, uint32_t *sums,
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


size_t bin_offsets_scratch_words(int64_t n_trials, int32_t n_bins) {
    const int64_t per_row = n_bins <= 64 ? (n_trials + kCountBlock - 1) / kCountBlock
                                         : (n_trials + 1 + kScanBlock - 1) / kScanBlock;
    return size_t(per_row) * size_t(n_bins);
}

hipError_t launch_bin_offsets(const int32_t *ids, const int64_t *offs, int64_t n_events, int64_t n_trials,
                              int32_t n_bins, const RunStarts &r, int32_t catalog, uint32_t *sums, uint32_t *err,
                              hipStream_t s) {
    if (n_trials <= 0 || n_bins <= 0 || n_bins > kMaxBins) return hipErrorInvalidValue;
    if ((r.stride & 7) || r.stride < n_trials + 2 || (r.abs == nullptr) == (r.b24 == nullptr)) return hipErrorInvalidValue;
    if (r.b24 && n_bins > 64) return hipErrorInvalidValue;
    hipError_t e;
    if (n_bins <= 64) {
        const int64_t nblk = (n_trials + kCountBlock - 1) / kCountBlock;
        const int64_t add_blocks = (n_trials + 1 + 4095) / 4096;
        if (add_blocks > 65535) return hipErrorInvalidValue;
        const dim3 grid{unsigned(std::min<int64_t>(nblk, 65536))}, add_grid{unsigned(add_blocks), unsigned(n_bins)};
        if (r.b24) {
            hipLaunchKernelGGL(k_bin_count_block<true>, grid, dim3(kCountWaves * 64), 0, s, ids, offs, n_events,
                               n_trials, n_bins, r, catalog, sums, err);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL(k_bin_block_scan<true>, dim3(unsigned(n_bins)), dim3(1024), 0, s, sums, nblk, r,
                               n_trials, err);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL(k_bin_block_add<true>, add_grid, dim3(1024), 0, s, r, n_trials, sums, nblk);
            return hipGetLastError();
        }
        hipLaunchKernelGGL(k_bin_count_block<false>, grid, dim3(kCountWaves * 64), 0, s, ids, offs, n_events, n_trials,
                           n_bins, r, catalog, sums, err);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_bin_block_scan<false>, dim3(unsigned(n_bins)), dim3(1024), 0, s, sums, nblk, r, n_trials,
                           err);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_bin_block_add<false>, add_grid, dim3(1024), 0, s, r, n_trials, sums, nblk);
        return hipGetLastError();
    }
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>((n_trials + kCountWaves - 1) / kCountWaves, 65536));
    hipLaunchKernelGGL(k_bin_count, dim3(unsigned(grid)), dim3(kCountWaves * 64), 0, s, ids, offs, n_events, n_trials,
                       n_bins, r.abs, r.stride, catalog, err);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_bin_scan(r.abs, r.stride, n_trials + 1, n_bins, sums, s);
}

// Region starts from the scanned offsets: region[0] = 0, region[b + 1] = region[b] +
// (bin b's length rounded up to 8), bin b's length being its run start at n_trials.
// One wave, up to 512 bins (8 per lane).  Skipped when an error bit is set (a bad ID
// or offset, or a bin too long for 3-byte run starts): the scatter is skipped then
// too.
__global__ __launch_bounds__(64) void k_bin_regions(RunStarts r, int64_t n_trials, int32_t n_bins,
                                                    int64_t *__restrict__ region, const uint32_t *__restrict__ err) {
    if (*err != 0u) return;
    const int lane = threadIdx.x;
    int64_t v[8], own = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int32_t b = lane * 8 + k;
        v[k] = b < n_bins ? (int64_t(run_at(r, b, n_trials)) + 7) & ~int64_t(7) : 0;
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

hipError_t launch_bin_regions(const RunStarts &r, int64_t n_trials, int32_t n_bins, int64_t *region,
                              const uint32_t *err, hipStream_t s) {
    if (n_bins > kMaxBins || kMaxBins > 8 * 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bin_regions, dim3(1), dim3(64), 0, s, r, n_trials, n_bins, region, err);
    return hipGetLastError();
}

// Writes each occurrence at region[b] + run(b, t) + (its rank among trial t's
// earlier occurrences of bin b).  A workgroup takes `per_block` consecutive trials;
// their occurrences of bin b form one contiguous span of region b, so when the
// block's occurrences fit in LDS they are placed there first (a counting sort by
// bin) and each bin's span is then written out whole.  A block with more
// occurrences than the LDS holds writes every occurrence to its place directly.
//
// Either way a wave takes one trial at a time, 64 occurrences per step in time
// order; lanes of a step that share a bin are ranked in lane order, so each run keeps
// the trial's time order.  The mask of lanes with the same bin comes from LDS when
// the bins fit a wave's table (at most 64: every lane ORs its bit into its bin's
// word and reads the word back; ORs do not depend on the order the lanes are taken
// in), else from one ballot per bit of the bin number (six ballots per step cost
// 1.6 ms of a 10^9-occurrence ingest, the LDS masks 0.5 ms).  With at most 64 bins
// and staging, lane l keeps bin l's next position in a register (read by the other
// lanes with a cross-lane permute) and clears bin l's mask word after the step by
// exchanging it for 0, which also gives it the bin's count for the step.
//
// Staging: 72 KB of LDS per 8-wave workgroup, so two workgroups share a CU and one
// places occurrences while the other starts or writes out.  Each bin's span starts
// in LDS at the same position modulo 8 as its destination, so it goes out in
// aligned 16-byte stores with at most 7 IDs on either side (2-byte stores cost
// 0.15 ms more of a 10^9-occurrence ingest, one 16-wave workgroup per CU 0.13 ms).
constexpr int kScatterWaves = 8;
constexpr int kScatterCap = 36864;   // IDs staged per workgroup (72 KB)
constexpr int kScatterPad = 7;       // slack per bin for the alignment of its span

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

template <int NBITS>
__global__ __launch_bounds__(kScatterWaves * 64) void k_bin_scatter(const int32_t *__restrict__ ids,
                                                                    const int64_t *__restrict__ offs, int64_t n_trials,
                                                                    int32_t n_bins, RunStarts r,
                                                                    const int64_t *__restrict__ region,
                                                                    uint16_t *__restrict__ ids16, int64_t per_block,
                                                                    const uint32_t *__restrict__ err) {
    constexpr int kBins = NBITS <= 6 ? 64 : kMaxBins;   // bins the LDS tables hold
    __shared__ __attribute__((aligned(16))) uint16_t stage[kScatterCap];
    __shared__ uint32_t cur[kScatterWaves][kBins];      // next position of the wave's trial's run, per bin
    __shared__ uint32_t lbase[kBins + 1];               // start of bin b's span in `stage`
    __shared__ uint32_t bstart[kBins];                  // run(b, t0)
    __shared__ uint32_t blen[kBins];                    // bin b's span length
    __shared__ uint64_t lanes_of[NBITS <= 6 ? kScatterWaves : 1][NBITS <= 6 ? 64 : 1];   // per wave and bin: its lanes
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t0 = int64_t(blockIdx.x) * per_block;
    if (t0 >= n_trials) return;
    // the count pass found a bad ID or offset: the counts do not describe the input
    if (*err != 0u) return;
    const int64_t t1 = min(t0 + per_block, n_trials);
    // a block with more occurrences than the LDS holds writes them to their places
    // directly (the body below, compiled for each case)
    const bool fits = offs[t1] - offs[t0] + int64_t(kScatterPad) * n_bins <= int64_t(kScatterCap);
    auto body = [&](auto staged_case) {
    constexpr bool staged = decltype(staged_case)::value;
    uint32_t *wc = cur[wave];
    uint64_t *lm = lanes_of[NBITS <= 6 ? wave : 0];
    if (NBITS <= 6) lm[lane] = 0;
    if (staged) {
        for (int32_t b = threadIdx.x; b < n_bins; b += kScatterWaves * 64) {
            const uint32_t s = run_at(r, b, t0);
            bstart[b] = s;
            lbase[b + 1] = run_at(r, b, t1) - s;
        }
        __syncthreads();
        if (wave == 0) {   // exclusive scan of the padded span lengths, 8 bins per lane
            uint32_t v[8], own = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int32_t b = lane * 8 + k;
                v[k] = b < n_bins ? lbase[b + 1] + kScatterPad : 0u;
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
                if (b < n_bins) {   // the span starts at the destination's position modulo 8
                    lbase[b] = run + ((bstart[b] - run) & 7u);
                    blen[b] = v[k] - kScatterPad;
                }
                run += v[k];
            }
            if (lane == 63) lbase[n_bins] = run;
        }
        __syncthreads();
    }
    // A wave places its trials t0 + wave, t0 + wave + kScatterWaves, ... one chunk of
    // kChunkSteps steps at a time.  Before it places a chunk it issues the loads of the
    // next one, with the next trial's run starts and the offsets of the trial after
    // that, all of them whatever the path (IDs past a trial's end read as 0 from the
    // buffer record), so the count of outstanding loads is the same on every path and
    // a wave waits only for the chunk it places (conditional loads made the compiler
    // wait for every load in flight before each chunk: 0.35 ms more of a
    // 10^9-occurrence ingest).
    constexpr int kChunkSteps = 16, kChunkIds = 64 * kChunkSteps;
    constexpr int kWB = (kBins + 63) / 64;
    typedef int64_t i64x2 __attribute__((ext_vector_type(2)));
    auto load_offs = [&](int64_t tt) -> i64x2 {   // offs[tt], offs[tt + 1], tt clamped to a trial
        const int64_t tc = min(tt, n_trials - 1);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)(offs + tc), 0, 16, kBufWord3);
        return __builtin_bit_cast(i64x2, __builtin_amdgcn_raw_buffer_load_b128(rs, 0, 0, 0));
    };
    auto load_wb = [&](int64_t tt, uint32_t (&w)[kWB]) {   // run(b, tt), b = lane + 64 k
        const int64_t tc = min(tt, n_trials);
#pragma unroll
        for (int k = 0; k < kWB; ++k) w[k] = run_at(r, min(lane + 64 * k, n_bins - 1), tc);
    };
    auto load_chunk = [&](int64_t start, int64_t end, uint32_t (&c)[kChunkSteps]) {
        const int32_t avail = int32_t(max(int64_t(0), min(end - start, int64_t(kChunkIds))));
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc((void *)(ids + (avail ? start : 0)), 0, avail * 4, kBufWord3);
#pragma unroll
        for (int u = 0; u < kChunkSteps; ++u) c[u] = __builtin_amdgcn_raw_buffer_load_b32(rs, (64 * u + lane) * 4, 0, 0);
    };
    auto uniform = [](int64_t v) {   // a value the wave holds in every lane, in scalar registers
        const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v))));
        const uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(uint64_t(v) >> 32))));
        return int64_t((uint64_t(hi) << 32) | lo);
    };
    int64_t t = t0 + wave, o0 = 0, o1 = 0;
    uint32_t cv[kChunkSteps], wb[kWB];
    i64x2 pn;   // offsets of trial t + kScatterWaves
    {
        const i64x2 p = load_offs(t);
        load_wb(t, wb);
        pn = load_offs(t + kScatterWaves);
        if (t < t1) {
            o0 = uniform(p[0]);
            o1 = uniform(p[1]);
        }
        load_chunk(o0, o1, cv);
    }
    int64_t base = o0;
    uint32_t curs = 0;   // NBITS <= 6, staged: lane l holds bin l's next position
    while (t < t1) {
        if (base == o0) {
            if (NBITS <= 6 && staged) {
                curs = lane < n_bins ? lbase[lane] + wb[0] - bstart[lane] : 0u;
            } else {
#pragma unroll
                for (int k = 0; k < kWB; ++k) {
                    const int32_t b = lane + 64 * k;
                    if (b < n_bins) wc[b] = staged ? lbase[b] + wb[k] - bstart[b] : wb[k];
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        // the next chunk: the rest of trial t, else the start of trial t + kScatterWaves
        const bool same = base + kChunkIds < o1;
        const int64_t nt = same ? t : t + kScatterWaves;
        int64_t nb = same ? base + kChunkIds : uniform(pn[0]), ne = same ? o1 : uniform(pn[1]);
        if (nt >= t1) nb = ne = 0;
        uint32_t wbn[kWB], nxt[kChunkSteps];
        load_wb(nt, wbn);
        const i64x2 qn = load_offs(nt + kScatterWaves);
        load_chunk(nb, ne, nxt);
        const int32_t len = int32_t(min(o1 - base, int64_t(kChunkIds)));
#pragma unroll
        for (int u = 0; u < kChunkSteps; ++u) {
            const bool valid = 64 * u + lane < len;
            const uint32_t id = cv[u];
            const uint32_t b = id >> kBinShift;
            uint32_t rank, count;
            if (NBITS <= 6 && staged) {
                const uint32_t bb = valid ? b : 63u;
                __hip_atomic_fetch_or(&lm[bb], valid ? uint64_t(1) << lane : uint64_t(0), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WAVEFRONT);
                const uint64_t m = lm[bb];
                __builtin_amdgcn_wave_barrier();
                // lane l takes bin l's mask and clears it in one exchange
                const uint64_t ml = __hip_atomic_exchange(&lm[lane], uint64_t(0), __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_WAVEFRONT);
                rank = __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
                const uint32_t at = uint32_t(__builtin_amdgcn_ds_bpermute(int(b << 2), int(curs)));
                if (valid) stage[at + rank] = uint16_t(id & uint32_t(kBinEvents - 1));
                curs += uint32_t(__popcll(ml));
                __builtin_amdgcn_wave_barrier();
                continue;
            }
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
        for (int u = 0; u < kChunkSteps; ++u) cv[u] = nxt[u];
#pragma unroll
        for (int k = 0; k < kWB; ++k) wb[k] = wbn[k];
        if (!same) o0 = nb;
        o1 = ne;
        base = nb;
        t = nt;
        pn = qn;
    }
    if (!staged) return;
    __syncthreads();
    // each bin's span to its place in region b: up to 7 IDs to the first 16-byte
    // boundary, whole 16-byte groups (consecutive lanes on consecutive groups), the rest
    typedef uint32_t u32x4s __attribute__((ext_vector_type(4)));
    for (int32_t b = wave; b < n_bins; b += kScatterWaves) {
        const uint32_t l0 = lbase[b], len = blen[b];
        uint16_t *dst = ids16 + region[b] + int64_t(bstart[b]);
        const uint32_t head = min(len, (8u - (bstart[b] & 7u)) & 7u);
        const uint32_t n16 = (len - head) >> 3, tail = (len - head) & 7u;
        if (uint32_t(lane) < head) dst[lane] = stage[l0 + lane];
        const u32x4s *src16 = reinterpret_cast<const u32x4s *>(stage + l0 + head);
        u32x4s *dst16 = reinterpret_cast<u32x4s *>(dst + head);
        for (uint32_t k = lane; k < n16; k += 64) dst16[k] = src16[k];
        if (uint32_t(lane) < tail) dst[head + 8 * n16 + lane] = stage[l0 + head + 8 * n16 + lane];
    }
    };
    if (fits) body(std::true_type{});
    else body(std::false_type{});
}

hipError_t launch_bin_scatter(const int32_t *ids, const int64_t *offs, int64_t n_events, int64_t n_trials,
                              int32_t n_bins, const RunStarts &r, const int64_t *region, uint16_t *ids16,
                              const uint32_t *err, hipStream_t s) {
    if (n_trials <= 0) return hipSuccess;
    if (n_bins > kMaxBins) return hipErrorInvalidValue;
    const int64_t per = bin_scatter_block_trials(n_events, n_trials);
    const int64_t grid = (n_trials + per - 1) / per;
    if (grid > int64_t(INT32_MAX)) return hipErrorInvalidValue;
    const int nbits = n_bins > 1 ? 32 - __builtin_clz(uint32_t(n_bins - 1)) : 0;
    // one instantiation per bit count of the bin numbers (the rank's ballots unrolled)
    hipError_t e = hipSuccess;
    auto launch = [&](auto nb_const) {
        constexpr int NB = decltype(nb_const)::value;
        hipLaunchKernelGGL((k_bin_scatter<NB>), dim3(unsigned(grid)), dim3(kScatterWaves * 64), 0, s, ids, offs,
                           n_trials, n_bins, r, region, ids16, per, err);
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
