// Device code of the YLT path for a dense occurrence-net table (in LDS, or in HBM/L2
// for catalogs too large for LDS), shared by the plain trial kernels and the
// batched kernel (internal).
#pragma once

#include "trial_common.h"

namespace ara {

// Wave-uniform position in a wave's sequence of (trial, segment).
struct Cursor {
    int64_t t;       // trial; >= t_end when the wave is done
    int64_t o0, o1;  // trial's events [o0, o1)
    int64_t sbase;   // first event of the segment, a multiple of 4
};

__device__ __forceinline__ void open_trial(const TrialArgs &a, int64_t t, Cursor &c, uint32_t &bad) {
    c.t = t;
    c.o0 = c.o1 = c.sbase = 0;
    if (t < a.t_end) {
        int64_t o0 = offset_at(a.offs, t), o1 = offset_at(a.offs, t + 1);
        if (!(o0 >= 0 && o0 <= o1 && o1 <= a.n_events)) {
            bad |= ERR_OFFSETS;
            o0 = o1 = 0;
        }
        c.o0 = o0;
        c.o1 = o1;
        c.sbase = o0 & ~int64_t(3);
    }
}

__device__ __forceinline__ bool seg_last(const Cursor &c) { return c.sbase + kSeg >= c.o1; }

// Re-asserts that a cursor is wave-uniform (keeps it in scalar registers across
// loop back-edges that the compiler cannot prove uniform).
__device__ __forceinline__ Cursor uniform_cursor(const Cursor &c) {
    Cursor u;
    u.t = uniform64(c.t);
    u.o0 = uniform64(c.o0);
    u.o1 = uniform64(c.o1);
    u.sbase = uniform64(c.sbase);
    return u;
}

__device__ __forceinline__ Cursor seg_next(const TrialArgs &a, const Cursor &c, int64_t stride, uint32_t &bad) {
    Cursor n = c;
    if (c.t >= a.t_end) return n;
    if (!seg_last(c)) {
        n.sbase = c.sbase + kSeg;
        return n;
    }
    open_trial(a, c.t + stride, n, bad);
    return n;
}

__device__ __forceinline__ void load_seg(const TrialArgs &a, const Cursor &c, int lane, u32x4 (&r)[kNch]) {
    const bool live = c.t < a.t_end;
    load_ids(a.ids, live ? c.sbase : 0, live ? seg_avail(c.sbase, c.o1, a.n_events) : 0, lane, r);
}

// Stage the layer's table into LDS (whole workgroup; ends with a barrier).
template <int PL>
__device__ __forceinline__ void stage_lds(const TrialArgs &a, uint32_t *lds) {
    if (PL == ARA_PLACE_LDS_BITMAP) {
        stage_bitmap(a, lds);
        return;
    } else if (PL == ARA_PLACE_LDS_DENSE) {
        // occurrence-net table, catalog doubles = 2*catalog words
        const uint32_t *g = reinterpret_cast<const uint32_t *>(a.occ);
        const int n = 2 * a.catalog, n4 = n >> 2;
        u32x4 *l4 = reinterpret_cast<u32x4 *>(lds);
        const u32x4 *g4 = reinterpret_cast<const u32x4 *>(g);
        for (int i = threadIdx.x; i < n4; i += blockDim.x) l4[i] = g4[i];
        for (int i = (n4 << 2) + threadIdx.x; i < n; i += blockDim.x) lds[i] = g[i];
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------------
// Look up the 16 IDs a lane holds for one segment: v[s] = occurrence-net loss of
// the event in slot s, 0 for slots outside the trial.  For the bitmap placement the
// L2 reads are issued here and consumed later (after the next prefetch is issued).
template <int PL>
__device__ __forceinline__ void seg_lookup(const TrialArgs &a, const uint32_t *lds, const u32x4 (&r)[kNch],
                                           int lane, int lo, int hi, double (&v)[kSlots], uint32_t &bad) {
    const uint32_t C = uint32_t(a.catalog);
    if (PL == ARA_PLACE_LDS_BITMAP) {
        // handled by seg_bitmap_filter / seg_bitmap_rows
    } else if (PL == ARA_PLACE_LDS_DENSE) {
        const double *tab = reinterpret_cast<const double *>(lds);
#pragma unroll
        for (int s = 0; s < kSlots; ++s) {
            const int rel = (s >> 2) * kChunk + lane * 4 + (s & 3);
            const uint32_t id = r[s >> 2][s & 3];
            const bool valid = rel >= lo && rel < hi;
            const bool inr = id < C;
            if (valid && !inr) bad |= ERR_ID_RANGE;
            v[s] = 0.0;
            if (valid && inr) v[s] = tab[id];
        }
    } else {
        const __amdgpu_buffer_rsrc_t vr =
            __builtin_amdgcn_make_buffer_rsrc((void *)a.occ, 0, int(C < 0x1FFFFFFFu ? C * 8u : 0xFFFFFFF8u), kBufWord3);
#pragma unroll
        for (int s = 0; s < kSlots; ++s) {
            const int rel = (s >> 2) * kChunk + lane * 4 + (s & 3);
            const uint32_t id = r[s >> 2][s & 3];
            const bool valid = rel >= lo && rel < hi;
            const bool inr = id < C;
            if (valid && !inr) bad |= ERR_ID_RANGE;
            // always issued (slots outside the trial read past the record: 0, no
            // memory access), so the count of loads in flight is the same on every path
            const uint32_t off = valid && inr ? id * 8u : 0xFFFFFFF8u;
            const uint2 q = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(vr, off, 0, 0));
            v[s] = __builtin_bit_cast(double, q);
        }
    }
}

__device__ __forceinline__ void seg_bounds(const Cursor &c, int &lo, int &hi) {
    const int64_t l = c.o0 - c.sbase, h = c.o1 - c.sbase;
    lo = int(l < 0 ? 0 : l);
    hi = int(h > kSeg ? kSeg : h);
}

__device__ __forceinline__ void finish_trial(const TrialArgs &a, int64_t t, double acc, int lane) {
    const double P = wave_total(acc);
    if (lane == 0) a.ylt[t - a.t_begin] = excess(P, a.agg_r, a.agg_l);
}

// One segment: look up its events (the L2 reads of the global placement are left
// in flight in v), then issue the loads of segment `nxt` into the register buffer
// just consumed, then add the values.
template <int PL>
__device__ __forceinline__ void seg_step(const TrialArgs &a, uint32_t *lds, uint32_t *q, u32x4 (&r)[kNch],
                                         const Cursor &cur, const Cursor &nxt, int lane, uint32_t &bad, double &acc) {
    int lo, hi;
    seg_bounds(cur, lo, hi);
    {
        double v[kSlots];
        seg_lookup<PL>(a, lds, r, lane, lo, hi, v, bad);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        load_seg(a, nxt, lane, r);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < kSlots; ++s) acc += v[s];
    }
}

// Wave per trial: the waves of a workgroup walk trials first, first + stride, ...
// (absolute trial indices, < a.t_end), two segments in flight per wave.
template <int PL>
__device__ __forceinline__ void dense_wave_run(const TrialArgs &a, uint32_t *lds, int64_t first, int64_t stride,
                                               int lane) {
    uint32_t *q = nullptr;   // no queue outside the bitmap placement
    uint32_t bad = 0;

    Cursor c0, c1;
    open_trial(a, first, c0, bad);
    c0 = uniform_cursor(c0);
    u32x4 A[kNch], B[kNch];
    load_seg(a, c0, lane, A);
    c1 = uniform_cursor(seg_next(a, c0, stride, bad));
    load_seg(a, c1, lane, B);

    double acc = 0.0;
    // One exit, at the top: a segment past the wave's last trial is stepped as an
    // empty one (no events) rather than leaving the loop in the middle, so the
    // compiler's wait counts at the top do not assume an empty pipeline.
    while (c0.t < a.t_end) {
        // segment c0 (in A) while c1 (in B) is in flight; A then receives c2
        const Cursor c2 = uniform_cursor(seg_next(a, c1, stride, bad));
        seg_step<PL>(a, lds, q, A, c0, c2, lane, bad, acc);
        if (seg_last(c0)) {
            finish_trial(a, c0.t, acc, lane);
            acc = 0.0;
        }
        const Cursor c3 = uniform_cursor(seg_next(a, c2, stride, bad));
        seg_step<PL>(a, lds, q, B, c1, c3, lane, bad, acc);
        if (c1.t < a.t_end && seg_last(c1)) {
            finish_trial(a, c1.t, acc, lane);
            acc = 0.0;
        }
        c0 = c2;
        c1 = c3;
    }
    if (bad) atomicOr(a.err, bad);
}

// Lane per trial, for short trials: lane i of the workgroup's wave w takes trial
// first + i, first + i + stride, ... and adds its occurrences' values in time order
// (the same sequence of additions as a sequential loop over the trial, so P is
// exactly the oracle's cumulative total).  IDs come in 16-byte groups of the lane's
// own trial; the occurrence-net values from the dense table.
template <int PL>
__device__ __forceinline__ void dense_lane_run(const TrialArgs &a, const uint32_t *lds, int64_t first, int64_t stride) {
    const uint32_t C = uint32_t(a.catalog);
    const double *tab = PL == ARA_PLACE_LDS_DENSE ? reinterpret_cast<const double *>(lds) : a.occ;
    const i32x4 *ids4 = reinterpret_cast<const i32x4 *>(a.ids);
    uint32_t bad = 0;
    for (int64_t t = first; t < a.t_end; t += stride) {
        int64_t o0 = a.offs[t], o1 = a.offs[t + 1];
        if (!(o0 >= 0 && o0 <= o1 && o1 <= a.n_events)) {
            bad |= ERR_OFFSETS;
            o0 = o1 = 0;
        }
        double P = 0.0;
        // 16 IDs (four 16-byte groups) are read before they are added, in time order
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
                const bool valid = pos >= o0 && pos < o1;
                bad |= valid && id >= C ? uint32_t(ERR_ID_RANGE) : 0u;
                const double v = tab[id < C ? id : C - 1u];
                P += valid && id < C ? v : 0.0;   // adding +0.0 leaves P's bits unchanged
            }
        }
        a.ylt[t - a.t_begin] = excess(P, a.agg_r, a.agg_l);
    }
    if (bad) atomicOr(a.err, bad);
}

}  // namespace ara
