// Tiled trial kernel: the YLT path for catalogs whose occurrence-net table does not fit
// in LDS as a whole.
//
// Per trial it computes what the bitmap kernel computes (Section II-B, steps 1-4):
//   ylt = min(max(P - AggR, 0), AggL),  P = sum over the trial's occurrences of the
//   occurrence-net loss of their event,
// which telescopes from the basic algorithm's per-occurrence ceded losses.  P is a sum
// of non-negative terms, so they may be taken in any grouping; here they are grouped
// by catalog bin.  The YET's catalog-binned copy (k_bin.hip) holds, bin after bin, the
// occurrences of each bin's 2^14 events as 2-byte bin-local IDs, trial after trial.
// A persistent workgroup owns up to kTiledPassTrials trials per pass.  For each bin it
// stages the bin's 2^14 occurrence-net values in LDS (binary64, the layer's `occ`
// table: zero for events outside the layer), then each lane adds the values of its own
// trial's run in the bin: one LDS read per occurrence, and no filter, queue, search or
// atomic.
//   Lane l of wave w, group g (< 4) holds trial T0(w) + 64 g + l.  A group's 64 runs are
//   one span of the bin; a lane reads its run 8 IDs (16 bytes) at a time from the run's
//   first even position.  An odd-starting run's first ID slot is the previous run's
//   last ID: it is redirected to a zero slot after the table.
//   Four such loads (runs of up to 32 occurrences) are issued two groups before the
//   group is added (three groups rotate through three register slots); the rest of a
//   longer run is read when reached.  Each bin's values are loaded into registers
//   while the previous bin is added, and written to LDS between two barriers.
// A trial's P is added in a fixed order (bins, then positions): the same bits on
// every run.  The per-trial sums live in LDS (one binary64 per trial of the wave).
#include <hip/hip_ext.h>

#include "trial_common.h"

namespace ara {

constexpr int kGroups = 4;                                       // groups of 64 trials per wave and pass
constexpr int kOct = 4;                                          // 8-ID loads issued ahead per run
constexpr uint32_t kZeroAddr = uint32_t(kBinEvents) * 8u;        // LDS byte address of the zero slot
constexpr uint32_t kZeroId = uint32_t(kBinEvents);               // bin-local ID that reads the zero slot
constexpr int kStageVecs = kBinEvents / (2 * kTiledWaves * 64);  // 16-byte value loads per thread per bin
static_assert(kTiledWaveTrials <= 64 * kGroups && kStageVecs * 2 * kTiledWaves * 64 == kBinEvents, "shapes");
static_assert(kTiledPassTrials == kTiledWaveTrials * kTiledWaves, "a pass fills every wave's sums");

typedef double f64x2 __attribute__((ext_vector_type(2)));

// Wave-uniform reads of tables the kernel never writes, through the scalar data path.
template <typename V>
__device__ __forceinline__ V sload(const V *p) {
    typedef const __attribute__((address_space(4))) V *cptr;
    return *(cptr)p;
}

__device__ __forceinline__ double lds_f64(const double *tab, uint32_t byte_addr) {
    return *reinterpret_cast<const double *>(reinterpret_cast<const char *>(tab) + byte_addr);
}

// LDS byte address of the value of the bin-local ID in the low / high half of w.  The
// low half is shifted from its 16-bit field directly (one instruction).
__device__ __forceinline__ uint32_t addr_lo(uint32_t w) {
    uint32_t r;
    asm("v_lshlrev_b32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_0"
        : "=v"(r) : "v"(3u), "v"(w));
    return r;
}
__device__ __forceinline__ uint32_t addr_hi(uint32_t w) { return (w >> 16) << 3; }

template <bool MAX>
__device__ __forceinline__ void fold(double &acc, double v) {
    if (MAX) acc = v > acc ? v : acc;   // occurrence-net losses are >= +0.0
    else acc += v;
}

// Bin b's span of the binned copy as a buffer (reads past it return zero).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t bin_rsrc(const TiledArgs &a, int32_t b) {
    const int64_t r0 = offset_at(a.region, b), r1 = offset_at(a.region, b + 1);
    return __builtin_amdgcn_make_buffer_rsrc((void *)(a.ids16 + r0), 0, int(uint32_t((r1 - r0) * 2)), kBufWord3);
}

// Bin b's values into registers: occ[2^14 b + i] (zero past the catalog).
__device__ __forceinline__ void stage_load(const TiledArgs &a, int32_t b, f64x2 (&st)[kStageVecs]) {
    const int64_t e0 = int64_t(b) * kBinEvents;
    const int64_t n = min(int64_t(kBinEvents), int64_t(a.catalog) - e0);
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc((void *)(a.occ + e0), 0, int(max(n, int64_t(0)) * 8), kBufWord3);
#pragma unroll
    for (int u = 0; u < kStageVecs; ++u)
        st[u] = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(
                                              r, int((threadIdx.x + u * kTiledWaves * 64) * 16), 0, 0));
}

// One lane's run in one bin.
struct Unit {
    uint32_t s;       // first position of the run, in the bin's span
    u32x4 q[kOct];    // IDs at positions (s & ~1) + 8 k .. + 7
};

// Loads with the default cache policy: a lane's four loads overlap the next lanes'
// runs, so the same lines are read several times within a group (a non-temporal hint
// made the kernel 30% slower).
__device__ __forceinline__ void unit_issue(__amdgpu_buffer_rsrc_t r, Unit &u) {
    const uint32_t s1 = u.s & ~1u;
#pragma unroll
    for (int k = 0; k < kOct; ++k) u.q[k] = __builtin_amdgcn_raw_buffer_load_b128(r, int((s1 + 8u * k) * 2u), 0, 0);
}

// 8 IDs of a run longer than kOct loads, read when reached.  The load waits for itself
// inside the asm block, so the compiler's count of the outstanding prefetch loads
// (which it uses to wait for exactly the group it adds next) stays exact.
__device__ __forceinline__ u32x4 load_ids_now(const uint16_t *p) {
    u32x4 r;
    asm volatile("global_load_dwordx4 %0, %1, off\n\ts_waitcnt vmcnt(0)" : "=v"(r) : "v"(p) : "memory");
    return r;
}

template <bool MAX>
__device__ __forceinline__ void add8(const double *tab, const u32x4 &q, double &acc) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        double v[4];
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            v[2 * d] = lds_f64(tab, addr_lo(q[2 * h + d]));
            v[2 * d + 1] = lds_f64(tab, addr_hi(q[2 * h + d]));
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) fold<MAX>(acc, v[j]);
    }
}

// The first n (1..7) IDs of q.
template <bool MAX>
__device__ __forceinline__ void add_first(const double *tab, const u32x4 &q, uint32_t n, double &acc) {
    double v[8];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        v[2 * d] = lds_f64(tab, uint32_t(2 * d) < n ? addr_lo(q[d]) : kZeroAddr);
        v[2 * d + 1] = lds_f64(tab, uint32_t(2 * d + 1) < n ? addr_hi(q[d]) : kZeroAddr);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) fold<MAX>(acc, v[j]);
}

// Adds the run [u.s, e) into acc, positions in order.  base: the bin's span.
template <bool MAX>
__device__ __forceinline__ void unit_run(const double *tab, const uint16_t *base, Unit &u, uint32_t e, double &acc) {
    const uint32_t s1 = u.s & ~1u;
    const uint32_t len = e > s1 ? e - s1 : 0u;
    const uint32_t nf = len >> 3, rest = len & 7u;
    if (u.s & 1u) u.q[0].x = (u.q[0].x & 0xFFFF0000u) | kZeroId;
#pragma unroll
    for (int k = 0; k < kOct; ++k) {
        if (__builtin_amdgcn_ballot_w64(uint32_t(k) < nf) == 0) break;
        if (uint32_t(k) < nf) add8<MAX>(tab, u.q[k], acc);
    }
    if (rest && nf < uint32_t(kOct)) {
        const u32x4 q = nf == 0 ? u.q[0] : nf == 1 ? u.q[1] : nf == 2 ? u.q[2] : u.q[3];
        add_first<MAX>(tab, q, rest, acc);
    }
    for (uint32_t k = kOct; __builtin_amdgcn_ballot_w64(k < nf || (k == nf && rest != 0)) != 0; ++k) {
        if (k < nf || (k == nf && rest != 0)) {
            const u32x4 q = load_ids_now(base + s1 + 8u * k);
            if (k < nf) add8<MAX>(tab, q, acc);
            else add_first<MAX>(tab, q, rest, acc);
        }
    }
}

// One pass of a workgroup over trials [pass, pass_end) of analysis a (at most
// kTiledPassTrials, split evenly over the waves): every bin staged once, each lane's
// trials added bin by bin, then their YLT (or maxima) written.
// MAX = false: the YLT (sums of the occurrence-net losses, then the aggregate terms);
// MAX = true: each trial's largest occurrence-net loss (0 for none).
// Units u = 4 b + g (bin b, group g) rotate through three register slots (slot u % 3):
// unit u + 3 is issued once unit u is added.  No load is issued under a condition, so
// that every wait counts only the loads issued after the one it waits for: bins past
// the last give empty runs and restage the last bin.
// B24: run starts in 3 bytes each, read as an unaligned 4-byte word (its top byte,
// the next entry's first, masked off where the value is taken).
template <bool MAX, bool B24>
__device__ __forceinline__ void tiled_pass(const TiledArgs &a, int64_t pass, int64_t pass_end, double *tab, double *ws,
                                           int lane, uint32_t wave) {
    const int64_t span = pass_end - pass;
    const int64_t per_wave = (span + kTiledWaves - 1) / kTiledWaves;
    const int64_t T0 = min(pass + int64_t(wave) * per_wave, pass_end);
    const int64_t T1 = min(T0 + per_wave, pass_end);
    const int32_t nb = a.n_bins;
#pragma unroll
    for (int g = 0; g < kGroups; ++g)
        if (64 * g + lane < kTiledWaveTrials) ws[64 * g + lane] = 0.0;
    // start of the run of trial T0 + 64 g + lane (the wave's span end past T1), and
    // the end of the group's last run (scalar)
    constexpr uint32_t kRunMask = B24 ? 0xFFFFFFu : 0xFFFFFFFFu;
    auto run_start = [&](int32_t b, int g) -> uint32_t {   // the word before masking
        const int64_t i = int64_t(b) * a.stride + min(T0 + 64 * g + lane, T1);
        if (!B24) return a.boff[i];
        uint32_t w;
        __builtin_memcpy(&w, a.boff24 + 3 * i, 4);
        return w;
    };
    auto group_end = [&](int32_t b, int g) -> uint32_t {
        const int64_t i = int64_t(b) * a.stride + min(T0 + 64 * g + 64, T1);
        if (!B24) return sload(a.boff + i);
        // the two aligned words holding bytes 3 i .. 3 i + 2
        const uint32_t *p = reinterpret_cast<const uint32_t *>(a.boff24 + ((3 * i) & ~int64_t(3)));
        const uint64_t w = uint64_t(sload(p)) | (uint64_t(sload(p + 1)) << 32);
        return uint32_t(w >> (8 * ((3 * i) & 3))) & kRunMask;
    };
    f64x2 st[kStageVecs];
    stage_load(a, 0, st);
    __amdgpu_buffer_rsrc_t rc = bin_rsrc(a, 0);
    const uint16_t *pc = a.ids16 + offset_at(a.region, 0);
    Unit U[3];
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        U[g].s = run_start(0, g) & kRunMask;
        unit_issue(rc, U[g]);
    }
    uint32_t s3 = run_start(0, 3) & kRunMask;
    uint32_t ge[kGroups];
#pragma unroll
    for (int g = 0; g < kGroups; ++g) ge[g] = group_end(0, g);
    for (int32_t b0 = 0; b0 < nb; b0 += 3) {
#pragma unroll
        for (int db = 0; db < 3; ++db) {
            const int32_t b = b0 + db;
            const bool live = b < nb, more = b + 1 < nb;
            const int32_t bn = more ? b + 1 : nb - 1;
            const __amdgpu_buffer_rsrc_t rn = bin_rsrc(a, bn);
            const uint16_t *pn = a.ids16 + offset_at(a.region, bn);
            uint32_t sn[kGroups], gn[kGroups];
#pragma unroll
            for (int g = 0; g < kGroups; ++g) {
                const uint32_t x = run_start(bn, g), y = group_end(bn, g);
                sn[g] = more ? x & kRunMask : 0u;
                gn[g] = more ? y : 0u;
            }
            __syncthreads();   // every wave is done with the previous bin
            f64x2 *dst = reinterpret_cast<f64x2 *>(tab);
#pragma unroll
            for (int u = 0; u < kStageVecs; ++u) dst[threadIdx.x + u * kTiledWaves * 64] = st[u];
            __syncthreads();
            stage_load(a, bn, st);
#pragma unroll
            for (int g = 0; g < kGroups; ++g) {
                const int slot = (db + g) % 3;
                // a run ends where the next lane's starts; lane 63's at the group end
                const uint32_t nx = uint32_t(__builtin_amdgcn_ds_bpermute(((lane + 1) & 63) * 4, int(U[slot].s)));
                const uint32_t e = lane == 63 ? ge[g] : nx;
                const int j = min(64 * g + lane, kTiledWaveTrials - 1);
                double acc = ws[j];
                unit_run<MAX>(tab, pc, U[slot], live ? e : 0u, acc);
                if (64 * g + lane < kTiledWaveTrials) ws[j] = acc;
                if (g == 0) {
                    U[slot].s = s3;
                    unit_issue(rc, U[slot]);
                } else {
                    U[slot].s = sn[g - 1];
                    unit_issue(rn, U[slot]);
                }
            }
            s3 = sn[3];
#pragma unroll
            for (int g = 0; g < kGroups; ++g) ge[g] = gn[g];
            rc = rn;
            pc = pn;
        }
    }
#pragma unroll
    for (int g = 0; g < kGroups; ++g) {
        const int64_t t = T0 + 64 * g + lane;
        if (t < T1) a.ylt[t - a.t_begin] = MAX ? ws[64 * g + lane] : excess(ws[64 * g + lane], a.agg_r, a.agg_l);
    }
}

// One analysis: workgroup w owns trials [t_begin + w per_wg, + per_wg), in passes.
template <bool MAX, bool B24>
__global__ __launch_bounds__(1024) void k_trial_tiled(TiledArgs a) {
    __shared__ __attribute__((aligned(16))) double tab[kBinEvents + 2];   // a bin's values, the zero slot
    __shared__ double sums[kTiledWaves * kTiledWaveTrials];
    const int lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (threadIdx.x == 0) tab[kBinEvents] = 0.0;
    const int64_t wg0 = a.t_begin + int64_t(blockIdx.x) * a.per_wg;
    const int64_t wg1 = min(wg0 + a.per_wg, a.t_end);
    for (int64_t pass = wg0; pass < wg1; pass += kTiledPassTrials)
        tiled_pass<MAX, B24>(a, pass, min(pass + int64_t(kTiledPassTrials), wg1), tab, sums + wave * kTiledWaveTrials,
                             lane, wave);
}

// Analysis j's arguments from device memory, through the scalar data path.
__device__ __forceinline__ TiledArgs load_args(const TiledArgs *jobs, int32_t j) {
    static_assert(sizeof(TiledArgs) % 4 == 0, "whole words");
    TiledArgs a;
    const uint32_t *src = reinterpret_cast<const uint32_t *>(jobs + j);
    uint32_t w[sizeof(TiledArgs) / 4];
#pragma unroll
    for (int i = 0; i < int(sizeof(TiledArgs) / 4); ++i) w[i] = sload(src + i);
    __builtin_memcpy(&a, w, sizeof(TiledArgs));
    return a;
}

// Many analyses in one launch (YLTs): each item is a pass over up to kTiledPassTrials
// trials of one analysis, taken in list order from a counter by whichever workgroup is
// free; a workgroup stops once the counter passes the list.  A trial's YLT does not
// depend on the pass that holds it, so these give the bits of k_trial_tiled.
__global__ __launch_bounds__(1024) void k_trial_tiled_items(const TiledArgs *__restrict__ jobs,
                                                            const TiledItem *__restrict__ items, int32_t n_items,
                                                            uint32_t *__restrict__ next) {
    __shared__ __attribute__((aligned(16))) double tab[kBinEvents + 2];
    __shared__ double sums[kTiledWaves * kTiledWaveTrials];
    __shared__ uint32_t took;
    const int lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (threadIdx.x == 0) tab[kBinEvents] = 0.0;
    for (;;) {
        if (threadIdx.x == 0) took = atomicAdd(next, 1u);
        __syncthreads();
        const uint32_t it = __builtin_amdgcn_readfirstlane(took);
        __syncthreads();   // every wave has read `took` before it is taken again
        if (it >= uint32_t(n_items)) return;
        const uint32_t *iw = reinterpret_cast<const uint32_t *>(items + it);
        const int32_t job = int32_t(sload(iw + 0));
        const int64_t t0 = int64_t(uint64_t(sload(iw + 2)) | (uint64_t(sload(iw + 3)) << 32));
        const int64_t t1 = int64_t(uint64_t(sload(iw + 4)) | (uint64_t(sload(iw + 5)) << 32));
        const TiledArgs a = load_args(jobs, job);
        if (a.boff24) tiled_pass<false, true>(a, t0, t1, tab, sums + wave * kTiledWaveTrials, lane, wave);
        else tiled_pass<false, false>(a, t0, t1, tab, sums + wave * kTiledWaveTrials, lane, wave);
    }
}

hipError_t launch_trial_tiled_items(const TiledArgs *jobs, const TiledItem *items, int32_t n_items, uint32_t *next,
                                    int grid, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    const hipError_t e = launch_fill_u32(next, 1, 0u, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_trial_tiled_items, dim3(grid), dim3(kTiledWaves * 64), 0, s, jobs, items, n_items, next);
    return hipGetLastError();
}

hipError_t launch_trial_tiled(const TiledArgs &a, int grid, hipStream_t s, bool occ_max, hipEvent_t start,
                              hipEvent_t stop) {
    const dim3 g(grid), b(kTiledWaves * 64);
    if (a.boff24) {
        if (occ_max) hipExtLaunchKernelGGL((k_trial_tiled<true, true>), g, b, 0, s, start, stop, 0, a);
        else hipExtLaunchKernelGGL((k_trial_tiled<false, true>), g, b, 0, s, start, stop, 0, a);
    } else {
        if (occ_max) hipExtLaunchKernelGGL((k_trial_tiled<true, false>), g, b, 0, s, start, stop, 0, a);
        else hipExtLaunchKernelGGL((k_trial_tiled<false, false>), g, b, 0, s, start, stop, 0, a);
    }
    return hipGetLastError();
}

}  // namespace ara
