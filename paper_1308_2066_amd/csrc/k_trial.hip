// Trial kernels: the analysis stage of Section II-B for every trial of the YET.
//
// Per trial (steps 1-4 of the basic algorithm):
//   x_d   = combined table[event_d]            (steps 1-2, the lookup, hoisted per event)
//   occ_d = min(max(x_d - OccR, 0), OccL)        (step 3, Table I occurrence terms)
//   P_d   = occ_1 + ... + occ_d                 (step 4, cumulative in time order)
//   ceded_d = f(P_d) - f(P_{d-1}),  f(P) = min(max(P - AggR, 0), AggL), f(P_0) = 0
//   lr    = sum_d ceded_d                       (the trial's year loss, Section II-C)
// Because occ_d >= 0, P is non-decreasing; f is non-decreasing with f(0) = 0, so the
// ceded losses telescope and lr = f(P_k).  k_trial_ylt computes lr that way (one
// reduction per trial).  k_trial_events runs the cumulative sum as a wave-wide
// inclusive scan and emits every per-occurrence quantity.
//
// Design for gfx950 (the paper's "chunking" of a trial into fixed-size blocks of
// events, Section III-B, taken to wave granularity):
//   * one wave64 walks one trial at a time in segments of 1024 events: four
//     16-byte non-temporal buffer loads per lane (64 lanes x 4 IDs x 4 loads), the
//     buffer's record count clipping the trial's end so no byte past it is fetched;
//   * segment i+2 is loaded while segment i is looked up (two register buffers);
//   * the occurrence-net value of an event comes from LDS when the layer's table
//     fits (this file: dense table), or from an LDS bitmap of the events whose
//     occurrence-net loss is nonzero (k_trial_bitmap.hip), or, for catalogs too
//     large for either, from the dense table in HBM/L2 (this file);
//   * persistent grid: one workgroup per LDS-sized slot of each compute unit, so the
//     table is staged into LDS once per workgroup; consecutive trials go to the waves
//     of one workgroup (same XCD), which shares their boundary cache lines.
#include "trial_dense.h"
#include "trial_bitmap.h"

namespace ara {

template <int PL>
__global__ __launch_bounds__(1024) void k_trial_ylt(TrialArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    stage_lds<PL>(a, lds);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wpb = __builtin_amdgcn_readfirstlane(blockDim.x >> 6);
    const int64_t stride = int64_t(__builtin_amdgcn_readfirstlane(gridDim.x)) * wpb;
    dense_wave_run<PL>(a, lds, a.t_begin + int64_t(blockIdx.x) * wpb + wave, stride, lane);
}

template <int PL>
__global__ __launch_bounds__(1024) void k_trial_ylt_lane(TrialArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    stage_lds<PL>(a, lds);
    dense_lane_run<PL>(a, lds, a.t_begin + int64_t(blockIdx.x) * blockDim.x + threadIdx.x,
                       int64_t(gridDim.x) * blockDim.x);
}

// ---------------------------------------------------------------------------------
// Largest occurrence-net loss of each trial (lane per trial): a maximum, so exact in
// any order.  Its distribution over trials is the occurrence exceedance curve.
template <int PL>
__device__ __forceinline__ double occ_value(const TrialArgs &a, const uint32_t *lds, uint32_t id) {
    if (PL == ARA_PLACE_LDS_BITMAP) {
        const uint32_t w = lds[id >> 5];
        return ((w >> (id & 31u)) & 1u) ? a.vals[bitmap_rank(lds, a.nblk, id)] : 0.0;
    } else if (PL == ARA_PLACE_LDS_DENSE) {
        return reinterpret_cast<const double *>(lds)[id];
    }
    return a.occ[id];
}

template <int PL>
__global__ __launch_bounds__(1024) void k_trial_occ_max(TrialArgs a, double *__restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    stage_lds<PL>(a, lds);
    const uint32_t C = uint32_t(a.catalog);
    const i32x4 *ids4 = reinterpret_cast<const i32x4 *>(a.ids);
    uint32_t bad = 0;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t t = a.t_begin + int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < a.t_end; t += stride) {
        int64_t o0 = a.offs[t], o1 = a.offs[t + 1];
        if (!(o0 >= 0 && o0 <= o1 && o1 <= a.n_events)) {
            bad |= ERR_OFFSETS;
            o0 = o1 = 0;
        }
        double m = 0.0;
        // 16 IDs (four 16-byte groups) are read before they are looked up
        for (int64_t g0 = o0 >> 2; 4 * g0 < o1; g0 += 4) {
            int32_t id16[16];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t g = g0 + u;
                if (4 * g + 4 <= a.n_events) {
                    const i32x4 x = ids4[g];
                    id16[4 * u] = x.x, id16[4 * u + 1] = x.y, id16[4 * u + 2] = x.z, id16[4 * u + 3] = x.w;
                } else {   // past the YET's last full group: no read past its end
#pragma unroll
                    for (int j = 0; j < 4; ++j) id16[4 * u + j] = 4 * g + j < a.n_events ? a.ids[4 * g + j] : 0;
                }
            }
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int64_t pos = 4 * g0 + j;
                const uint32_t id = uint32_t(id16[j]);
                if (pos < o0 || pos >= o1) continue;
                if (id >= C) {
                    bad |= ERR_ID_RANGE;
                    continue;
                }
                const double v = occ_value<PL>(a, lds, id);
                m = v > m ? v : m;
            }
        }
        out[t - a.t_begin] = m;
    }
    if (bad) atomicOr(a.err, bad);
}

// Two consecutive binary64 outputs from element pos on (8-byte aligned), if out is set;
// non-temporal, since the outputs are written once and not read back by the kernel.
typedef double f64x2_u __attribute__((ext_vector_type(2), aligned(8)));
__device__ __forceinline__ void store2(double *out, int64_t pos, double v0, double v1) {
    if (!out) return;
    __builtin_nontemporal_store(f64x2_u{v0, v1}, reinterpret_cast<f64x2_u *>(out + pos));
}

// ---------------------------------------------------------------------------------
// Per-occurrence form: every quantity of the basic algorithm, with the cumulative
// sum as wave-wide inclusive scans (lane-local over 2 consecutive events, then a
// 64-lane scan, plus the carry from the previous 128 events).  NZ: the layer's
// "combined loss nonzero" bits are staged in LDS and only events with a set bit
// read the combined table (the others' gross loss is +0.0, as the table holds).
template <typename V, bool NZ>
__global__ __launch_bounds__(1024) void k_trial_events(TrialArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint32_t nzl[];
    if (NZ) {
        const u32x4 *src = reinterpret_cast<const u32x4 *>(a.nz);
        u32x4 *dst = reinterpret_cast<u32x4 *>(nzl);
        for (int i = threadIdx.x; i < a.nblk; i += blockDim.x) dst[i] = src[i];
        __syncthreads();
    }
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wpb = __builtin_amdgcn_readfirstlane(blockDim.x >> 6);
    const int64_t stride = int64_t(__builtin_amdgcn_readfirstlane(gridDim.x)) * wpb;
    const V *comb = reinterpret_cast<const V *>(a.comb);
    const uint32_t C = uint32_t(a.catalog);
    const int64_t ev0 = uniform64(a.offs[a.t_begin]);
    uint32_t bad = 0;
    for (int64_t t = a.t_begin + int64_t(blockIdx.x) * wpb + wave; t < a.t_end; t += stride) {
        Cursor c;
        open_trial(a, t, c, bad);
        double carryP = 0.0, carryF = 0.0, lr = 0.0;
        while (true) {
            u32x4 r[kNch];
            load_seg(a, c, lane, r);
            int lo, hi;
            seg_bounds(c, lo, hi);
            for (int k = 0; k < kNch && k * kChunk < hi; ++k) {
                // lane l takes events 2l, 2l+1 and 128+2l, 129+2l of the chunk (its IDs
                // fetched from the lanes that loaded them), so that one store instruction
                // writes 64 consecutive pairs of an output array
                const bool odd = lane & 1;
                const int s0 = lane >> 1, s1 = 32 + (lane >> 1);
                uint32_t idv[4];
                {
                    const uint32_t ax = __shfl(r[k][0], s0, 64), ay = __shfl(r[k][1], s0, 64);
                    const uint32_t az = __shfl(r[k][2], s0, 64), aw = __shfl(r[k][3], s0, 64);
                    const uint32_t bx = __shfl(r[k][0], s1, 64), by = __shfl(r[k][1], s1, 64);
                    const uint32_t bz = __shfl(r[k][2], s1, 64), bw = __shfl(r[k][3], s1, 64);
                    idv[0] = odd ? az : ax;
                    idv[1] = odd ? aw : ay;
                    idv[2] = odd ? bz : bx;
                    idv[3] = odd ? bw : by;
                }
                double x[4], o[4], P[4], F[4];
                bool ok[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int rel = k * kChunk + (j < 2 ? 0 : 128) + 2 * lane + (j & 1);
                    const uint32_t id = idv[j];
                    const bool valid = rel >= lo && rel < hi;
                    const bool inr = id < C;
                    if (valid && !inr) bad |= ERR_ID_RANGE;
                    ok[j] = valid && inr;
                    const uint32_t idc = ok[j] ? id : 0u;   // lanes outside the trial read word 0
                    const bool look = NZ ? ok[j] && ((nzl[idc >> 5] >> (idc & 31u)) & 1u) : ok[j];
                    x[j] = look ? double(comb[id]) : 0.0;
                    o[j] = ok[j] ? excess(x[j], a.occ_r, a.occ_l) : 0.0;
                }
                // cumulative sums: the chunk's first 128 events, then its last 128
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const double q0 = o[2 * h], q1 = o[2 * h] + o[2 * h + 1];
                    double inc = q1;
#pragma unroll
                    for (int d = 1; d < 64; d <<= 1) {
                        const double y = __shfl_up(inc, d, 64);
                        if (lane >= d) inc += y;
                    }
                    double ex = __shfl_up(inc, 1, 64);
                    if (lane == 0) ex = 0.0;
                    const double base = carryP + ex;
                    P[2 * h] = base + q0;
                    P[2 * h + 1] = base + q1;
                    F[2 * h] = excess(P[2 * h], a.agg_r, a.agg_l);
                    F[2 * h + 1] = excess(P[2 * h + 1], a.agg_r, a.agg_l);
                    double Fprev = __shfl_up(F[2 * h + 1], 1, 64);
                    if (lane == 0) Fprev = carryF;
                    double ced[2] = {F[2 * h] - Fprev, F[2 * h + 1] - F[2 * h]};
                    if (ok[2 * h]) lr += ced[0];
                    if (ok[2 * h + 1]) lr += ced[1];
                    const int64_t pos0 = c.sbase + k * kChunk + 128 * h + 2 * lane - ev0;
                    if (ok[2 * h] && ok[2 * h + 1]) {
                        store2(a.ev_gross, pos0, x[2 * h], x[2 * h + 1]);
                        store2(a.ev_occ, pos0, o[2 * h], o[2 * h + 1]);
                        store2(a.ev_cum, pos0, P[2 * h], P[2 * h + 1]);
                        store2(a.ev_ceded, pos0, ced[0], ced[1]);
                    } else {
#pragma unroll
                        for (int j = 0; j < 2; ++j) {
                            if (!ok[2 * h + j]) continue;
                            if (a.ev_gross) a.ev_gross[pos0 + j] = x[2 * h + j];
                            if (a.ev_occ) a.ev_occ[pos0 + j] = o[2 * h + j];
                            if (a.ev_cum) a.ev_cum[pos0 + j] = P[2 * h + j];
                            if (a.ev_ceded) a.ev_ceded[pos0 + j] = ced[j];
                        }
                    }
                    carryP = __shfl(P[2 * h + 1], 63, 64);
                    carryF = __shfl(F[2 * h + 1], 63, 64);
                }
            }
            if (seg_last(c)) break;
            c.sbase += kSeg;
        }
        const double tot = wave_total(lr);
        if (lane == 0 && a.ylt) a.ylt[t - a.t_begin] = tot;
    }
    if (bad) atomicOr(a.err, bad);
}

// ---------------------------------------------------------------------------------
// Lookups through a placement, for bit-exact checks of the trial kernel's tables.
template <int PL, typename V>
__global__ __launch_bounds__(1024) void k_lookup(TrialArgs a, const int32_t *__restrict__ ids, int64_t n,
                                                 double *gross, double *occ) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    stage_lds<PL>(a, lds);
    const uint32_t C = uint32_t(a.catalog);
    uint32_t bad = 0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const uint32_t id = uint32_t(ids[i]);
        if (id >= C) {
            bad |= ERR_ID_RANGE;
            if (gross) gross[i] = __builtin_nan("");
            if (occ) occ[i] = __builtin_nan("");
            continue;
        }
        if (gross) gross[i] = double(reinterpret_cast<const V *>(a.comb)[id]);
        double o;
        if (PL == ARA_PLACE_LDS_BITMAP) {
            const uint32_t w = lds[id >> 5];
            o = 0.0;
            if ((w >> (id & 31u)) & 1u) o = a.vals[bitmap_rank(lds, a.nblk, id)];
        } else if (PL == ARA_PLACE_LDS_DENSE) {
            o = reinterpret_cast<const double *>(lds)[id];
        } else {
            o = a.occ[id];
        }
        if (occ) occ[i] = o;
    }
    if (bad) atomicOr(a.err, bad);
}

// ---------------------------------------------------------------------------------
hipError_t prepare_trial_kernels() {
    hipError_t e;
#define ARA_SET_LDS(fn)                                                                                  \
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn), hipFuncAttributeMaxDynamicSharedMemorySize, \
                            kLdsMaxBytes);                                                               \
    if (e != hipSuccess) return e;
    ARA_SET_LDS(k_trial_ylt<ARA_PLACE_LDS_DENSE>)
    ARA_SET_LDS(k_trial_ylt_lane<ARA_PLACE_LDS_DENSE>)
    ARA_SET_LDS(k_trial_occ_max<ARA_PLACE_LDS_DENSE>)
    ARA_SET_LDS(k_trial_occ_max<ARA_PLACE_LDS_BITMAP>)
    ARA_SET_LDS((k_lookup<ARA_PLACE_LDS_BITMAP, double>))
    ARA_SET_LDS((k_lookup<ARA_PLACE_LDS_DENSE, double>))
    ARA_SET_LDS((k_lookup<ARA_PLACE_LDS_BITMAP, float>))
    ARA_SET_LDS((k_lookup<ARA_PLACE_LDS_DENSE, float>))
    ARA_SET_LDS((k_trial_events<double, true>))
    ARA_SET_LDS((k_trial_events<float, true>))
#undef ARA_SET_LDS
    return hipSuccess;
}

hipError_t launch_trial_ylt(const TrialArgs &a, const TrialLaunch &l, hipStream_t s) {
    switch (l.placement) {
    case ARA_PLACE_LDS_BITMAP:
        return launch_trial_ylt_bitmap(a, l.grid, l.block, s);
    case ARA_PLACE_LDS_DENSE:
        if (l.lane)
            hipLaunchKernelGGL(k_trial_ylt_lane<ARA_PLACE_LDS_DENSE>, dim3(l.grid), dim3(l.block), l.lds_bytes, s, a);
        else
            hipLaunchKernelGGL(k_trial_ylt<ARA_PLACE_LDS_DENSE>, dim3(l.grid), dim3(l.block), l.lds_bytes, s, a);
        break;
    default:
        if (l.lane)
            hipLaunchKernelGGL(k_trial_ylt_lane<ARA_PLACE_GLOBAL_DENSE>, dim3(l.grid), dim3(l.block), 0, s, a);
        else
            hipLaunchKernelGGL(k_trial_ylt<ARA_PLACE_GLOBAL_DENSE>, dim3(l.grid), dim3(l.block), 0, s, a);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_trial_occ_max(const TrialArgs &a, const TrialLaunch &l, int grid, double *out, hipStream_t s) {
    switch (l.placement) {
    case ARA_PLACE_LDS_BITMAP:
        hipLaunchKernelGGL(k_trial_occ_max<ARA_PLACE_LDS_BITMAP>, dim3(grid), dim3(256), l.lds_bytes, s, a, out);
        break;
    case ARA_PLACE_LDS_DENSE:
        hipLaunchKernelGGL(k_trial_occ_max<ARA_PLACE_LDS_DENSE>, dim3(grid), dim3(256), l.lds_bytes, s, a, out);
        break;
    default:
        hipLaunchKernelGGL(k_trial_occ_max<ARA_PLACE_GLOBAL_DENSE>, dim3(grid), dim3(256), 0, s, a, out);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_trial_events(const TrialArgs &a, bool f32, int n_cu, int lds_max, hipStream_t s) {
    const int64_t waves = a.t_end - a.t_begin;
    const size_t nz_bytes = size_t(a.nblk) * 16;
    if (a.nz && nz_bytes <= size_t(lds_max)) {
        // one workgroup of 16 waves per CU holds the bits
        const int grid = int(std::max<int64_t>(1, std::min<int64_t>(n_cu, (waves + 15) / 16)));
        if (f32) hipLaunchKernelGGL((k_trial_events<float, true>), dim3(grid), dim3(1024), nz_bytes, s, a);
        else hipLaunchKernelGGL((k_trial_events<double, true>), dim3(grid), dim3(1024), nz_bytes, s, a);
    } else {
        const int grid = int(std::max<int64_t>(1, std::min<int64_t>(int64_t(n_cu) * 8, (waves + 3) / 4)));
        if (f32) hipLaunchKernelGGL((k_trial_events<float, false>), dim3(grid), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_trial_events<double, false>), dim3(grid), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_lookup(const TrialArgs &a, const TrialLaunch &l, const int32_t *ids, int64_t n, double *gross,
                         double *occ, hipStream_t s) {
    const int grid = 256;
#define ARA_LK(PL)                                                                                             \
    if (l.f32) hipLaunchKernelGGL((k_lookup<PL, float>), dim3(grid), dim3(1024), l.lds_bytes, s, a, ids, n, gross, occ); \
    else hipLaunchKernelGGL((k_lookup<PL, double>), dim3(grid), dim3(1024), l.lds_bytes, s, a, ids, n, gross, occ);
    switch (l.placement) {
    case ARA_PLACE_LDS_BITMAP: ARA_LK(ARA_PLACE_LDS_BITMAP) break;
    case ARA_PLACE_LDS_DENSE: ARA_LK(ARA_PLACE_LDS_DENSE) break;
    default: ARA_LK(ARA_PLACE_GLOBAL_DENSE) break;
    }
#undef ARA_LK
    return hipGetLastError();
}

}  // namespace ara
