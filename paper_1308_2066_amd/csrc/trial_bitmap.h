// Device code of the YLT path for catalogs whose occurrence filter fits in LDS
// (internal; used by the plain trial kernel and the batched kernel).
//
// The headline case (a 1M-event catalog).  Computes, per trial (Section II-B, steps 1-4),
//   ylt = min(max(P - AggR, 0), AggL),  P = sum over the trial's occurrences of the
//   occurrence-net loss of their event,
// which equals the basic algorithm's sum of per-occurrence ceded losses: the
// cumulative sum is non-decreasing and the aggregate clamp is non-decreasing with
// value 0 at 0, so the differences telescope.
//
// A wave walks its trials in segments of 1024 events (four non-temporal loads per
// lane: 16 bytes of int32 IDs, or 12 bytes of the YET's packed 3-byte copy, which
// cuts the dominant stream by a quarter).  Per segment:
//   filter  each lane tests the LDS bit of its 16 events (one LDS read each, all
//           issued together); only events whose occurrence-net loss is nonzero pass;
//   queue   passing events are appended to the wave's LDS queue in slot-then-lane
//           order (mbcnt positions), so they end up dense;
//   rows    the queue is resolved 64 events at a time: the event's rank among
//           flagged events comes from the LDS bitmap, its value from L2;
//   sum     values are added per lane in queue order, then reduced over the wave
//           at the trial's end (deterministic for a given YET layout).
// Software pipeline: the ID loads of segment i+2 are issued after the value reads of
// segment i, and the values of segment i are added one segment later.  Vector-memory
// operations complete in issue order, so waiting for values never waits for the
// newest ID loads: each ID load has two segments of time to arrive.
#pragma once

#include "trial_common.h"

namespace ara {

constexpr int kRows = kQueueCapMax / kQueueRow;                  // value reads per segment
constexpr int kTabWords = (kLdsMaxBytes - kQueueWords * 4) / 4;  // static LDS for the filter

// Wave-uniform position: trial t (relative to t_begin; t >= n when done), segment
// start sbase (multiple of 4), trial end o1, and lo = leading events before the
// trial's first event in its first segment (0..3).
struct BCur {
    uint32_t t;
    uint32_t lo;
    int64_t sbase;
    int64_t o1;
};

__device__ __forceinline__ BCur bcur_open(const TrialArgs &a, uint32_t t, uint32_t n, uint32_t &bad) {
    BCur c;
    c.t = t;
    c.lo = 0;
    c.sbase = 0;
    c.o1 = 0;
    if (t < n) {
        const int64_t r0 = uniform64(offset_at(a.offs, a.t_begin + t));
        const int64_t r1 = uniform64(offset_at(a.offs, a.t_begin + t + 1));
        const bool ok = r0 >= 0 && r0 <= r1 && r1 <= a.n_events;   // else: an empty trial, reported
        bad |= ok ? 0u : uint32_t(ERR_OFFSETS);
        const int64_t o0 = ok ? r0 : 0, o1 = ok ? r1 : 0;
        c.sbase = o0 & ~int64_t(3);
        c.lo = uint32_t(o0 - c.sbase);
        c.o1 = o1;
    }
    return c;
}

__device__ __forceinline__ bool bcur_last(const BCur &c) { return c.sbase + kSeg >= c.o1; }

// Loop-carried cursors are wave-uniform; this keeps them in scalar registers.
__device__ __forceinline__ BCur bcur_uniform(const BCur &c) {
    BCur u;
    u.t = __builtin_amdgcn_readfirstlane(c.t);
    u.lo = __builtin_amdgcn_readfirstlane(c.lo);
    u.sbase = uniform64(c.sbase);
    u.o1 = uniform64(c.o1);
    return u;
}

__device__ __forceinline__ BCur bcur_next(const TrialArgs &a, const BCur &c, uint32_t stride, uint32_t n,
                                          uint32_t &bad) {
    if (c.t >= n) return c;
    if (!bcur_last(c)) {
        BCur d = c;
        d.sbase += kSeg;
        d.lo = 0;
        return d;
    }
    return bcur_open(a, c.t + stride, n, bad);
}

// Event IDs of one segment in registers: int32 (four 16-byte loads per lane) or the
// packed copy (four 12-byte loads per lane).
template <bool P24> struct IdRegs;
template <> struct IdRegs<false> { u32x4 r[kNch]; };
template <> struct IdRegs<true> { u32x3 r[kNch]; };

template <bool P24>
__device__ __forceinline__ void bcur_load(const TrialArgs &a, const BCur &c, uint32_t n, int lane, IdRegs<P24> &g) {
    const bool live = c.t < n;
    if constexpr (P24)
        load_ids24(a.ids24, live ? c.sbase : 0, live ? seg_avail24(c.sbase, c.o1) : 0, lane, g.r);
    else
        load_ids(a.ids, live ? c.sbase : 0, live ? seg_avail(c.sbase, c.o1, a.n_events) : 0, lane, g.r);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t vals_rsrc(const TrialArgs &a) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)a.vals, 0, int(uint32_t(a.catalog) * 8u), kBufWord3);
}

__device__ __forceinline__ double load_val(__amdgpu_buffer_rsrc_t vr, uint32_t byte_off) {
    const uint2 q = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(vr, byte_off, 0, 0));
    return __builtin_bit_cast(double, q);
}

// Resolve queue entries [0, qn) now (queue overflow: many flagged events).
__device__ __forceinline__ void drain_queue(const TrialArgs &a, const uint32_t *tab, const uint32_t *q, uint32_t qn,
                                            int lane, double &acc) {
    const __amdgpu_buffer_rsrc_t vr = vals_rsrc(a);
    for (uint32_t r0 = 0; r0 < qn; r0 += kQueueRow) {
        double v = 0.0;
        if (r0 + lane < qn) v = load_val(vr, bitmap_rank(tab, a.nblk, q[r0 + lane]) * 8u);
        acc += v;
    }
}

// Filter + queue of one segment held in r; returns the queue length.  Slot s of a
// lane holds the event at position k*256 + 4*lane + j (s = 4k + j) of the segment;
// it counts if that position lies in [lo, hi) and the event's filter bit is set.
// lo < 4, so only lane 0 of the first load can hold events before the trial.
// The int32 IDs are range-checked here (mx); the packed copy was checked when built.
template <bool P24>
__device__ __forceinline__ uint32_t seg_queue(const TrialArgs &a, const uint32_t *tab, uint32_t *q,
                                              const IdRegs<P24> &g, int lane, int lo, int hi, uint32_t &mx,
                                              double &dacc) {
    const uint32_t cmax = uint32_t(a.catalog) - 1u;
    uint32_t id[kSlots], e[kSlots], w[kSlots];
#pragma unroll
    for (int k = 0; k < kNch; ++k) {
        if constexpr (P24) {
            unpack_ids24(g.r[k], id + 4 * k);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) id[4 * k + j] = g.r[k][j];
            mx = max(mx, max(max(id[4 * k], id[4 * k + 1]), max(id[4 * k + 2], id[4 * k + 3])));
        }
    }
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
        // the packed copy was checked against the catalog when it was built
        e[s] = P24 ? id[s] : min(id[s], cmax);
        w[s] = tab[e[s] >> 5];
    }
    const int l4 = lane * 4;
    bool f[kSlots];
    uint32_t total = 0;
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
        const int base = (s >> 2) * kChunk + (s & 3);
        f[s] = (__builtin_amdgcn_ubfe(w[s], e[s], 1) != 0u) & (l4 < hi - base);
        if (s < 4) f[s] = f[s] & (l4 + base >= lo);
        total += uint32_t(__popcll(__builtin_amdgcn_ballot_w64(f[s])));
    }
    uint32_t qn = 0;
    if (total <= uint32_t(a.qcap)) {
        // common case: the whole segment fits the queue
#pragma unroll
        for (int s = 0; s < kSlots; ++s) {
            const uint64_t m = __builtin_amdgcn_ballot_w64(f[s]);
            uint32_t *qs = q + qn;
            if (f[s]) qs[__builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u))] = e[s];
            qn += uint32_t(__popcll(m));
        }
        return qn;
    }
    // many flagged events: resolve the queue whenever the next slot would overflow it
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
        const uint64_t m = __builtin_amdgcn_ballot_w64(f[s]);
        const uint32_t cnt = uint32_t(__popcll(m));
        if (qn + cnt > uint32_t(a.qcap)) {
            drain_queue(a, tab, q, qn, lane, dacc);
            qn = 0;
        }
        if (f[s]) q[__builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), qn))] = e[s];
        qn += cnt;
    }
    return qn;
}

// Value reads of the queued events: always kRows 64-lane reads (lanes past the queue
// read outside the buffer record: 0, no memory access), so the number of
// outstanding vector-memory operations per segment is fixed.
__device__ __forceinline__ void seg_rows(const TrialArgs &a, const uint32_t *tab, const uint32_t *q, uint32_t qn,
                                         int lane, double (&v)[kRows]) {
    const __amdgpu_buffer_rsrc_t vr = vals_rsrc(a);
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const uint32_t r0 = uint32_t(k) * kQueueRow;
        uint32_t off = 0xFFFFFFF8u;
        if (r0 < qn) {
            const uint32_t slot = r0 + uint32_t(lane);
            const uint32_t e = slot < qn ? q[slot] : 0u;
            const uint32_t o = bitmap_rank(tab, a.nblk, e) * 8u;
            off = slot < qn ? o : 0xFFFFFFF8u;
        }
        v[k] = load_val(vr, off);
    }
}

struct Pending {
    uint32_t t;      // trial of the segment whose values are in flight (>= n: none)
    uint32_t last;   // that segment ends its trial
    double dacc;     // its values already resolved on the overflow path
};

template <bool P24>
__device__ __forceinline__ void issue(const TrialArgs &a, const uint32_t *tab, uint32_t *q, IdRegs<P24> &r,
                                      const BCur &cur, const BCur &nxt, uint32_t n, int lane, uint32_t &mx,
                                      double (&v)[kRows], Pending &p) {
    const int64_t h = cur.o1 - cur.sbase;
    const int hi = int(h > kSeg ? kSeg : h);
    p.t = cur.t;
    p.last = bcur_last(cur) ? 1u : 0u;
    p.dacc = 0.0;
    const uint32_t qn = seg_queue<P24>(a, tab, q, r, lane, int(cur.lo), hi, mx, p.dacc);
    seg_rows(a, tab, q, qn, lane, v);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    bcur_load<P24>(a, nxt, n, lane, r);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

__device__ __forceinline__ void retire(const TrialArgs &a, const Pending &p, const double (&v)[kRows], uint32_t n,
                                       int lane, double &acc) {
    if (p.t >= n) return;
    double s = p.dacc;
#pragma unroll
    for (int k = 0; k < kRows; ++k) s += v[k];
    acc += s;
    if (p.last) {
        const double P = wave_total(acc);
        if (lane == 0) a.ylt[p.t] = excess(P, a.agg_r, a.agg_l);
        acc = 0.0;
    }
}

// The waves of a workgroup walk trials first, first + stride, ... of [0, t_end -
// t_begin) (relative to a.t_begin) with the filter already in tab; q is this wave's
// queue of a.qcap entries.
template <bool P24>
__device__ __forceinline__ void bitmap_wave_run(const TrialArgs &a, const uint32_t *tab, uint32_t *q, uint32_t first,
                                                uint32_t stride, int lane) {
    const uint32_t n = uint32_t(a.t_end - a.t_begin);
    uint32_t bad = 0, mx = 0;

    BCur c0 = bcur_uniform(bcur_open(a, first, n, bad));
    BCur c1 = bcur_uniform(bcur_next(a, c0, stride, n, bad));
    // The prologue issues what a loop iteration leaves in flight (IDs, value reads of
    // an empty segment, IDs), so the waits at the loop's top are the same on entry.
    IdRegs<P24> A, B;
    double vA[kRows], vB[kRows];
    bcur_load<P24>(a, c0, n, lane, A);
    seg_rows(a, tab, q, 0u, lane, vB);
    bcur_load<P24>(a, c1, n, lane, B);

    Pending pA, pB;
    pB.t = n;
    pB.last = 0;
    pB.dacc = 0.0;
    double acc = 0.0;
    // One exit, at the top: a segment past the last trial is issued as an empty one
    // (no IDs, no queued events) rather than leaving the loop in the middle, so the
    // compiler's wait counts at the top do not assume an empty pipeline.
    while (c0.t < n) {
        pB.t = __builtin_amdgcn_readfirstlane(pB.t);
        pB.last = __builtin_amdgcn_readfirstlane(pB.last);
        const BCur c2 = bcur_uniform(bcur_next(a, c1, stride, n, bad));
        issue<P24>(a, tab, q, A, c0, c2, n, lane, mx, vA, pA);
        retire(a, pB, vB, n, lane, acc);
        const BCur c3 = bcur_uniform(bcur_next(a, c2, stride, n, bad));
        issue<P24>(a, tab, q, B, c1, c3, n, lane, mx, vB, pB);
        retire(a, pA, vA, n, lane, acc);
        c0 = c2;
        c1 = c3;
    }
    retire(a, pB, vB, n, lane, acc);
    if (mx > uint32_t(a.catalog) - 1u) bad |= ERR_ID_RANGE;
    if (bad) atomicOr(a.err, bad);
}

}  // namespace ara
