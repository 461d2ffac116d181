// Trial kernel for catalogs whose occurrence filter fits in LDS: one persistent
// workgroup per CU stages the filter and its waves walk the trials (device code in
// trial_bitmap.h).
#include "trial_bitmap.h"

namespace ara {

template <bool P24>
__global__ __launch_bounds__(1024) void k_trial_ylt_bitmap(TrialArgs a) {
    __shared__ __attribute__((aligned(16))) uint32_t tab[kTabWords];
    __shared__ __attribute__((aligned(16))) uint32_t queues[kQueueWords];
    stage_bitmap(a, tab);
    const int lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t wpb = __builtin_amdgcn_readfirstlane(blockDim.x >> 6);
    const uint32_t stride = __builtin_amdgcn_readfirstlane(gridDim.x) * wpb;
    bitmap_wave_run<P24>(a, tab, queues + wave * uint32_t(a.qcap), blockIdx.x * wpb + wave, stride, lane);
}

size_t trial_bitmap_table_capacity() { return size_t(kTabWords) * 4; }

hipError_t launch_trial_ylt_bitmap(const TrialArgs &a, int grid, int block, hipStream_t s) {
    if (a.ids24)
        hipLaunchKernelGGL(k_trial_ylt_bitmap<true>, dim3(grid), dim3(block), 0, s, a);
    else
        hipLaunchKernelGGL(k_trial_ylt_bitmap<false>, dim3(grid), dim3(block), 0, s, a);
    return hipGetLastError();
}

}  // namespace ara
