// Batched analyses: many jobs -- a (YET, layer, trial range) each, the layer loop of
// Algorithm 1 and the portfolios of Section IV -- in one persistent launch.
//
// The host splits every job into work items of about equal event counts (whole
// trials), groups them by mode and job, and launches one persistent kernel per mode
// present; each workgroup takes a contiguous run of items, so it stages a job's table
// into LDS once and keeps it while its items belong to that job.  An item runs exactly the device code of the plain trial kernels
// (trial_dense.h, trial_bitmap.h) on its trial range, so every trial's year loss
// is computed by the same operations in the same order as alone: a batch gives the
// plain launches' results bit for bit, whatever the split.
#include "trial_dense.h"
#include "trial_bitmap.h"

#include <algorithm>

namespace ara {

// A wave-uniform copy of a descriptor, read through the scalar data path (constant
// address space), word by word.
template <typename T>
__device__ __forceinline__ T load_uniform(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "descriptor size");
    typedef const __attribute__((address_space(4))) uint32_t *const_u32_ptr;
    const const_u32_ptr src = (const_u32_ptr)p;
    T v;
    uint32_t *dst = reinterpret_cast<uint32_t *>(&v);
#pragma unroll
    for (int i = 0; i < int(sizeof(T) / 4); ++i) dst[i] = src[i];
    return v;
}

// One kernel per mode: each carries only its own path, so registers are not shared
// with the other modes' state.  Items of one launch all have mode MODE.
// per_wg > 0: workgroup w takes items [w * per_wg, (w + 1) * per_wg) (few job changes
// per workgroup); per_wg == 0: it takes items w, w + G, w + 2G, ... (G workgroups), so
// at any moment the whole grid works on neighbouring items, i.e. on one or two jobs,
// whose tables then share the L2.
template <int MODE>
__global__ __launch_bounds__(1024) void k_batch(const BatchJob *__restrict__ jobs, const BatchItem *__restrict__ items,
                                                int32_t n_items, int32_t per_wg) {
    __shared__ __attribute__((aligned(16))) uint32_t lds[kLdsMaxBytes / 4];
    const int lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t wpb = __builtin_amdgcn_readfirstlane(blockDim.x >> 6);
    const int32_t step = per_wg > 0 ? 1 : int32_t(gridDim.x);
    const int32_t i0 = per_wg > 0 ? int32_t(blockIdx.x) * per_wg : int32_t(blockIdx.x);
    const int32_t i1 = per_wg > 0 ? (i0 + per_wg < n_items ? i0 + per_wg : n_items) : n_items;
    int32_t cur = -1;
    for (int32_t i = i0; i < i1; i += step) {
        const BatchItem it = load_uniform(items + i);
        TrialArgs a = load_uniform(&jobs[it.job].a);
        if (it.job != cur) {
            __syncthreads();   // every wave is done with the previous job's table
            if constexpr (MODE == kModeWaveBitmap || MODE == kModeWaveBitmap24) stage_bitmap(a, lds);
            else if constexpr (MODE == kModeLaneLds || MODE == kModeWaveLds) stage_lds<ARA_PLACE_LDS_DENSE>(a, lds);
            // global-table modes read HBM/L2 directly: nothing to stage
            cur = it.job;
        }
        if constexpr (MODE == kModeLaneLds) {
            a.t_end = it.t1;
            dense_lane_run<ARA_PLACE_LDS_DENSE>(a, lds, it.t0 + threadIdx.x, blockDim.x);
        } else if constexpr (MODE == kModeLaneGlobal) {
            a.t_end = it.t1;
            dense_lane_run<ARA_PLACE_GLOBAL_DENSE>(a, lds, it.t0 + threadIdx.x, blockDim.x);
        } else if constexpr (MODE == kModeWaveLds) {
            a.t_end = it.t1;
            dense_wave_run<ARA_PLACE_LDS_DENSE>(a, lds, it.t0 + wave, wpb, lane);
        } else if constexpr (MODE == kModeWaveGlobal) {
            a.t_end = it.t1;
            dense_wave_run<ARA_PLACE_GLOBAL_DENSE>(a, lds, it.t0 + wave, wpb, lane);
        } else {
            a.ylt += it.t0 - a.t_begin;
            a.t_begin = it.t0;
            a.t_end = it.t1;
            bitmap_wave_run<MODE == kModeWaveBitmap24>(a, lds, lds + kTabWords + wave * uint32_t(a.qcap), wave, wpb,
                                                       lane);
        }
    }
}

// Portfolio year losses: out[t] = sum over jobs j = 0, 1, ... (in that order) of
// ylts[j][t], one thread per trial.
__global__ __launch_bounds__(256) void k_sum_ylts(const double *const *__restrict__ ylts, int32_t n_jobs, int64_t n,
                                                  double *__restrict__ out) {
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x) {
        double s = 0.0;
        for (int32_t j = 0; j < n_jobs; ++j) s += ylts[j][t];
        out[t] = s;
    }
}

hipError_t launch_sum_ylts(const double *const *ylts, int32_t n_jobs, int64_t n, double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t grid = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_sum_ylts, dim3(unsigned(grid)), dim3(256), 0, s, ylts, n_jobs, n, out);
    return hipGetLastError();
}

int32_t batch_mode(const TrialLaunch &l, bool packed) {
    switch (l.placement) {
    case ARA_PLACE_LDS_BITMAP: return packed ? kModeWaveBitmap24 : kModeWaveBitmap;
    case ARA_PLACE_LDS_TILES: return kModeTiled;
    case ARA_PLACE_LDS_DENSE: return l.lane ? kModeLaneLds : kModeWaveLds;
    default: return l.lane ? kModeLaneGlobal : kModeWaveGlobal;
    }
}

hipError_t launch_batch(int32_t mode, const BatchJob *jobs, const BatchItem *items, int32_t n_items, int32_t per_wg,
                        int grid, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    switch (mode) {
    case kModeLaneLds: hipLaunchKernelGGL(k_batch<kModeLaneLds>, dim3(grid), dim3(1024), 0, s, jobs, items, n_items, per_wg); break;
    case kModeLaneGlobal: hipLaunchKernelGGL(k_batch<kModeLaneGlobal>, dim3(grid), dim3(1024), 0, s, jobs, items, n_items, per_wg); break;
    case kModeWaveLds: hipLaunchKernelGGL(k_batch<kModeWaveLds>, dim3(grid), dim3(1024), 0, s, jobs, items, n_items, per_wg); break;
    case kModeWaveGlobal: hipLaunchKernelGGL(k_batch<kModeWaveGlobal>, dim3(grid), dim3(1024), 0, s, jobs, items, n_items, per_wg); break;
    case kModeWaveBitmap: hipLaunchKernelGGL(k_batch<kModeWaveBitmap>, dim3(grid), dim3(1024), 0, s, jobs, items, n_items, per_wg); break;
    case kModeWaveBitmap24: hipLaunchKernelGGL(k_batch<kModeWaveBitmap24>, dim3(grid), dim3(1024), 0, s, jobs, items, n_items, per_wg); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ara
