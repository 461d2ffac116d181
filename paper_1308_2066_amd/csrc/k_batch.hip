// Batched analyses: many jobs -- a (YET, layer, trial range) each, the layer loop of
// Algorithm 1 and the portfolios of Section IV -- in one persistent launch.
//
// The host splits every job into work items of about equal event counts (whole
// trials), sorted by job, and gives each workgroup a contiguous run of items, so a
// workgroup stages a job's table into LDS once and keeps it while its items belong
// to that job.  An item runs exactly the device code of the plain trial kernels
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

__global__ __launch_bounds__(1024) void k_batch(const BatchJob *__restrict__ jobs, const BatchItem *__restrict__ items,
                                                int32_t n_items, int32_t per_wg) {
    __shared__ __attribute__((aligned(16))) uint32_t lds[kLdsMaxBytes / 4];
    const int lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t wpb = __builtin_amdgcn_readfirstlane(blockDim.x >> 6);
    const int32_t i0 = int32_t(blockIdx.x) * per_wg;
    const int32_t i1 = i0 + per_wg < n_items ? i0 + per_wg : n_items;
    int32_t cur = -1;
    for (int32_t i = i0; i < i1; ++i) {
        const BatchItem it = load_uniform(items + i);
        const BatchJob jb = load_uniform(jobs + it.job);
        const int32_t mode = jb.mode;
        TrialArgs a = jb.a;
        if (it.job != cur) {
            __syncthreads();   // every wave is done with the previous job's table
            if (mode == kModeWaveBitmap || mode == kModeWaveBitmap24) stage_bitmap(a, lds);
            else if (mode == kModeLaneLds || mode == kModeWaveLds) stage_lds<ARA_PLACE_LDS_DENSE>(a, lds);
            // global-table modes read HBM/L2 directly: nothing to stage
            cur = it.job;
        }
        switch (mode) {
        case kModeLaneLds:
            a.t_end = it.t1;
            dense_lane_run<ARA_PLACE_LDS_DENSE>(a, lds, it.t0 + threadIdx.x, blockDim.x);
            break;
        case kModeLaneGlobal:
            a.t_end = it.t1;
            dense_lane_run<ARA_PLACE_GLOBAL_DENSE>(a, lds, it.t0 + threadIdx.x, blockDim.x);
            break;
        case kModeWaveLds:
            a.t_end = it.t1;
            dense_wave_run<ARA_PLACE_LDS_DENSE>(a, lds, it.t0 + wave, wpb, lane);
            break;
        case kModeWaveGlobal:
            a.t_end = it.t1;
            dense_wave_run<ARA_PLACE_GLOBAL_DENSE>(a, lds, it.t0 + wave, wpb, lane);
            break;
        case kModeWaveBitmap:
        case kModeWaveBitmap24:
            a.ylt += it.t0 - a.t_begin;
            a.t_begin = it.t0;
            a.t_end = it.t1;
            if (mode == kModeWaveBitmap24)
                bitmap_wave_run<true>(a, lds, lds + kTabWords + wave * uint32_t(a.qcap), wave, wpb, lane);
            else
                bitmap_wave_run<false>(a, lds, lds + kTabWords + wave * uint32_t(a.qcap), wave, wpb, lane);
            break;
        default:
            break;
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
    case ARA_PLACE_LDS_DENSE: return l.lane ? kModeLaneLds : kModeWaveLds;
    default: return l.lane ? kModeLaneGlobal : kModeWaveGlobal;
    }
}

hipError_t launch_batch(const BatchJob *jobs, const BatchItem *items, int32_t n_items, int32_t per_wg, int grid,
                        hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch, dim3(grid), dim3(1024), 0, s, jobs, items, n_items, per_wg);
    return hipGetLastError();
}

}  // namespace ara
