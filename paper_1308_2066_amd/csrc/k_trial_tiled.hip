// Tiled trial kernel: the YLT path for catalogs whose occurrence-net values do not
// fit in LDS as one table.
//
// Per trial it computes what the bitmap kernel computes (Section II-B, steps 1-4):
//   ylt = min(max(P - AggR, 0), AggL),  P = sum over the trial's occurrences of the
//   occurrence-net loss of their event,
// which telescopes from the basic algorithm's per-occurrence ceded losses.  P is a
// sum, so its terms may be taken in any grouping; here they are grouped by catalog
// tile.  The layer's filter (one bit per event, per-block counts) and its nonzero
// values are cut into tiles that fit in LDS together (plan_tiles).  A persistent
// workgroup owns a range of trials; for each tile it stages the tile in LDS, then
// its waves stream the occurrences of the tile's bins from the binned YET copy
// (k_bin.hip), so that every lookup is an LDS access and the only HBM traffic is
// the stream of 2-byte IDs.
//
// Per wave and bin, the occurrences of the wave's trials (up to 252) are one contiguous
// span, read in windows of up to 1024 (8 coalesced rows of 64 lanes x 2 IDs):
//   filter  each ID's LDS bit; flagged occurrences are appended to the wave's LDS
//           queue with their position in the window;
//   drain   up to three rows of 64 entries at a time: the value from LDS, the
//           trial by search over the window's trial boundaries (held one per
//           lane), and an LDS add into that trial's sum (one binary64 per trial of
//           the wave).
// A trial's P is therefore added in a fixed order (tiles, bins, windows, queue
// entries, and lanes within an instruction as the LDS unit orders its conflicting
// adds): the same bits on every run on a given device.
#include "trial_common.h"

namespace ara {

constexpr int kTileWords = kTiledLdsBytes / 4;
// trials per wave and pass: a window spans at most 63 trials (one boundary per lane),
// so 252 trials need at least four windows per bin (more where a window fills its
// 1024 positions first: about eight at 32 occurrences per trial and bin).  A
// pass of 16 waves then covers 4032 trials: one pass per workgroup for a million
// trials on 256 CUs (each pass stages every tile once)
constexpr int kPassTrials = kTiledPassTrials;   // trials per workgroup pass
static_assert(kPassTrials % kTiledWaves == 0 && kPassTrials / kTiledWaves <= kTiledWaveTrials, "per-trial sums");
constexpr int kWinRows = 8;   // 8 rows ran 1% faster than 16 (and 12 rows 3% slower)
constexpr int kWindow = kWinRows * 128;            // occurrences per window

// Wave-uniform reads of tables the kernel never writes, through the scalar data
// path (constant address space): values land in scalar registers, so buffer
// descriptors built from them stay scalar.
template <typename V>
__device__ __forceinline__ V sload(const V *p) {
    typedef const __attribute__((address_space(4))) V *cptr;
    return *(cptr)p;
}

__device__ __forceinline__ Tile load_tile(const Tile *tiles, uint32_t k) {
    const uint32_t *w = reinterpret_cast<const uint32_t *>(tiles + k);
    Tile t;
    t.blk_lo = int32_t(sload(w + 0));
    t.blk_hi = int32_t(sload(w + 1));
    t.bin_lo = int32_t(sload(w + 2));
    t.bin_hi = int32_t(sload(w + 3));
    t.rank_lo = sload(w + 4);
    t.n_vals = sload(w + 5);
    return t;
}

// Stage tile T (whole workgroup; the caller brackets it with barriers): the bits of
// its bins' blocks (zero outside the tile's own blocks), per-word counts of the
// tile's flagged events before the word, the values.  nb = blocks held.  Each thread
// issues its first values' loads (up to 8) before the filter words' and stores them
// after, so the staging waits for one round trip (two for tiles of over 8192 values).
__device__ __forceinline__ void stage_tile(const TiledArgs &a, const Tile &T, int32_t nb, uint32_t *tab) {
    constexpr uint32_t kThreads = kTiledWaves * 64, kUnroll = 8;
    double *v = reinterpret_cast<double *>(reinterpret_cast<char *>(tab) + tile_vals_offset(nb));
    const double *src = a.vals + T.rank_lo;
    double t[kUnroll];
#pragma unroll
    for (uint32_t u = 0; u < kUnroll; ++u) {
        const uint32_t i = threadIdx.x + u * kThreads;
        t[u] = i < T.n_vals ? src[i] : 0.0;
    }
    const int32_t b0 = T.bin_lo * kBlocksPerBin;
    u32x4 *l4 = reinterpret_cast<u32x4 *>(tab);
    uint16_t *r16 = reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(tab) + tile_rank_offset(nb));
    for (int i = threadIdx.x; i < nb; i += kThreads) {
        const int32_t blk = b0 + i;
        u32x4 W = {0u, 0u, 0u, 0u};
        uint32_t r0 = 0;
        if (blk >= T.blk_lo && blk < T.blk_hi) {
            W = reinterpret_cast<const u32x4 *>(a.bitmap)[blk];
            r0 = a.rank[blk] - T.rank_lo;
        }
        l4[i] = W;
        const uint32_t r1 = r0 + __popc(W.x), r2 = r1 + __popc(W.y), r3 = r2 + __popc(W.z);
        r16[4 * i + 0] = uint16_t(r0);
        r16[4 * i + 1] = uint16_t(r1);
        r16[4 * i + 2] = uint16_t(r2);
        r16[4 * i + 3] = uint16_t(r3);
    }
#pragma unroll
    for (uint32_t u = 0; u < kUnroll; ++u) {
        const uint32_t i = threadIdx.x + u * kThreads;
        if (i < T.n_vals) v[i] = t[u];
    }
    for (uint32_t i0 = threadIdx.x + kUnroll * kThreads; i0 < T.n_vals; i0 += kUnroll * kThreads) {
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) {
            const uint32_t i = i0 + u * kThreads;
            t[u] = i < T.n_vals ? src[i] : 0.0;
        }
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) {
            const uint32_t i = i0 + u * kThreads;
            if (i < T.n_vals) v[i] = t[u];
        }
    }
}

// One wave's cursor over the windows of a tile: bin b, next position ws, and jl =
// the trial (relative to the wave's first trial T0) whose run contains ws.
struct TCur {
    int32_t b;        // current bin (>= bin_hi: done)
    uint32_t ws, e;   // next position and end of the wave's span in region b
    uint32_t jl;
};

struct TWin {
    uint32_t v[kWinRows];   // IDs: row r, lane l -> positions ws2 + 128 r + 2 l, +1
    uint32_t bnd;           // boundary of trial jl + lane in region b (clamped to the span end)
};

// Open bins from b on until one has occurrences of the wave's trials.
__device__ __forceinline__ void tcur_seek(const TiledArgs &a, const Tile &T, int64_t T0, int64_t T1, TCur &c) {
    while (c.b < T.bin_hi) {
        const uint32_t *row = a.boff + int64_t(c.b) * a.stride;
        c.ws = sload(row + T0);
        c.e = sload(row + T1);
        c.jl = 0;
        if (c.ws < c.e) return;
        ++c.b;
    }
}

__device__ __forceinline__ TCur tcur_uniform(const TCur &c) {
    TCur u;
    u.b = __builtin_amdgcn_readfirstlane(c.b);
    u.ws = __builtin_amdgcn_readfirstlane(c.ws);
    u.e = __builtin_amdgcn_readfirstlane(c.e);
    u.jl = __builtin_amdgcn_readfirstlane(c.jl);
    return u;
}

// Issue the loads of the window at c (boundaries first, then IDs); a finished cursor
// issues the same loads with empty buffer records (no memory access).
__device__ __forceinline__ void twin_load(const TiledArgs &a, const Tile &T, const TCur &c, int64_t T0, int64_t T1,
                                          int lane, TWin &w) {
    const bool live = c.b < T.bin_hi;
    const int32_t b = live ? c.b : 0;
    const uint32_t *row = a.boff + int64_t(b) * a.stride;
    const int64_t nbnd = T1 - T0 + 1;   // boundaries T0 .. T1
    const __amdgpu_buffer_rsrc_t rb =
        __builtin_amdgcn_make_buffer_rsrc((void *)(row + T0), 0, live ? int(nbnd * 4) : 0, kBufWord3);
    const uint32_t jb = min(c.jl + uint32_t(lane), uint32_t(nbnd - 1));
    w.bnd = __builtin_amdgcn_raw_buffer_load_b32(rb, int(jb * 4u), 0, 0);
    const uint32_t ws2 = c.ws & ~1u;
    const uint32_t hi = min(ws2 + uint32_t(kWindow), c.e);
    const uint32_t bytes = live ? ((hi + 1u) & ~1u) * 2u : 0u;
    const __amdgpu_buffer_rsrc_t ri =
        __builtin_amdgcn_make_buffer_rsrc((void *)(a.ids16 + sload(a.region + b)), 0, int(bytes), kBufWord3);
#pragma unroll
    for (int r = 0; r < kWinRows; ++r)
        w.v[r] = __builtin_amdgcn_raw_buffer_load_b32(ri, int((ws2 + uint32_t(128 * r + 2 * lane)) * 2u), 0, kNonTemporal);
}

// Resolve N rows of queue entries from r0 on (entries below qn) of the current
// window: value, trial, add to the trial's sum.  The rows interleave their dependent
// LDS round trips.  Lane l takes entries r0 + N l + n (n < N), so the 64 adds of one
// instruction fall N entries apart, mostly in different trials (adds to one address
// in one instruction are serialised); the order of a trial's adds is fixed by the
// queue.  Every queued position lies in the window (the filter drops the others).
// Positions and boundaries are relative to the window's first row (bnd_rel).
template <bool MAX, int N>
__device__ __forceinline__ void drain_rows(const uint32_t *tab, const uint16_t *r16, const double *vals,
                                           const uint32_t *q, uint32_t r0, uint32_t qn, double *sums_jl,
                                           uint32_t id_off, uint32_t bnd_rel, int lane) {
    uint32_t p[N], i4[N];
    double v[N];
    bool in_q[N];
    // r0 + N * 64 <= 320 on every call, so the reads stay in the wave's queue and spare
    // slots; entries past qn are stale: resolved like the others (every address they
    // form is in the tile) but not added
    const uint32_t *ql = q + r0 + uint32_t(lane) * N;
#pragma unroll
    for (int n = 0; n < N; ++n) {
        in_q[n] = r0 + uint32_t(lane) * N + uint32_t(n) < qn;
        const uint32_t ent = ql[n];
        p[n] = ent >> kBinShift;
        // the value does not depend on the trial, so its reads overlap the search below
        const uint32_t x = (ent & uint32_t(kBinEvents - 1)) | id_off;
        const uint32_t wi = x >> 5;
        const uint32_t rk = uint32_t(r16[wi]) + __popc(tab[wi] & ((1u << (x & 31u)) - 1u));
        v[n] = vals[rk];
        i4[n] = 0;
    }
    // largest i with boundary(jl + i) <= p: the trial of position p.  The
    // boundaries of lanes 16, 32 and 48 are compared as scalars, then four steps
    // read other lanes' boundaries (all lanes take part); i4 = 4 i, the lane's byte
    // address.  (Seven scalar compares and three steps ran 1% slower, fifteen and
    // two 9% slower, one and five 2% slower.)
    uint32_t s16[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) s16[j] = uint32_t(__builtin_amdgcn_readlane(int(bnd_rel), 16 * (j + 1)));
#pragma unroll
    for (int n = 0; n < N; ++n) {
#pragma unroll
        for (int j = 0; j < 3; ++j) i4[n] += p[n] >= s16[j] ? 64u : 0u;
    }
#pragma unroll
    for (uint32_t step4 = 32; step4 >= 4; step4 >>= 1) {
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const uint32_t cand4 = i4[n] | step4;
            const uint32_t bc = uint32_t(__builtin_amdgcn_ds_bpermute(int(cand4), int(bnd_rel)));
            i4[n] = bc <= p[n] ? cand4 : i4[n];
        }
    }
#pragma unroll
    for (int n = 0; n < N; ++n) {
        if (in_q[n]) {
            double *dst = reinterpret_cast<double *>(reinterpret_cast<char *>(sums_jl) + 2u * i4[n]);
            if (MAX)   // occurrence-net losses are >= +0.0: their bits order as their values
                __hip_atomic_fetch_max(reinterpret_cast<uint64_t *>(dst), __builtin_bit_cast(uint64_t, v[n]),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            else
                __hip_atomic_fetch_add(dst, v[n], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        }
    }
}

// Resolve queue entries [0, qn) of the current window.
template <bool MAX>
__device__ __forceinline__ void tiled_drain(const uint32_t *tab, int32_t nb, const uint32_t *q, uint32_t qn,
                                            double *sums, uint32_t id_off, uint32_t bnd_rel, uint32_t jl, int lane) {
    const uint16_t *r16 = reinterpret_cast<const uint16_t *>(reinterpret_cast<const char *>(tab) + tile_rank_offset(nb));
    const double *vals = reinterpret_cast<const double *>(reinterpret_cast<const char *>(tab) + tile_vals_offset(nb));
    uint32_t r0 = 0;
    for (; r0 + 128 < qn; r0 += 192) drain_rows<MAX, 3>(tab, r16, vals, q, r0, qn, sums + jl, id_off, bnd_rel, lane);
    for (; r0 + 64 < qn; r0 += 128) drain_rows<MAX, 2>(tab, r16, vals, q, r0, qn, sums + jl, id_off, bnd_rel, lane);
    if (r0 < qn) drain_rows<MAX, 1>(tab, r16, vals, q, r0, qn, sums + jl, id_off, bnd_rel, lane);
}

constexpr int kHalfRows = kWinRows / 2;
static_assert(2 * kHalfRows == kWinRows, "tiled_window filters a window in two halves");
constexpr int kQueueStride = kTiledQueue + 64;   // per wave: the queue, then 64 slots that drain reads may reach

// LDS byte address of the filter word of the bin-local ID in bits LO..LO+14 of v:
// word ID >> 5 of the bin, whose words start at byte woff.
template <int LO>
__device__ __forceinline__ uint32_t word_addr(uint32_t v, uint32_t woff) {
    return __builtin_amdgcn_ubfe(v, LO + 5, 10) * 4u + woff;
}

// Lanes 0 .. c - 1 (c <= 64).
__device__ __forceinline__ uint64_t lanes_before(uint32_t c) { return c >= 64 ? ~0ull : (1ull << c) - 1ull; }

// Append one ID slot's flagged entries (lanes in m) to the queue at qn: lane l writes
// ent at qn + (lanes of m below l); the other lanes write nothing.
__device__ __forceinline__ void queue_slot(uint32_t *q, uint64_t m, uint32_t &qn, uint32_t ent) {
    const uint32_t at = __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
    uint32_t *qq = q + qn;
    if (__builtin_amdgcn_inverse_ballot_w64(m)) qq[at] = ent;
    qn += uint32_t(__popcll(m));
}

// Filter and drain one window [ws, we) of bin c.b (IDs in w), half a window at a time:
// first every row's LDS filter words are read (the reads overlap), then each ID
// slot's flagged lanes are appended to the queue.  Positions outside the window (in
// its first and last rows) are dropped from the flag masks; IDs outside the tile's
// own blocks meet zero bits.
template <bool MAX>
__device__ __forceinline__ void tiled_window(const Tile &T, int32_t nb, const uint32_t *tab, uint32_t *q,
                                             double *sums, const TCur &c, uint32_t we, const TWin &w, int lane) {
    const uint32_t id_off = uint32_t(c.b - T.bin_lo) << kBinShift;   // first tile event of the bin
    const uint32_t woff = id_off >> 3;                                // its filter word, in bytes
    const uint32_t ws2 = c.ws & ~1u;
    const uint32_t lane_rel = uint32_t(2 * lane) << kBinShift;
    const uint32_t bnd_rel = w.bnd - ws2;   // the boundary of trial jl + lane, from the first row
    const uint32_t wlen = we - ws2;         // positions of the window's rows that are in it
    uint32_t qn = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (uint32_t(128 * kHalfRows * h) >= wlen) break;   // the rest of the window is empty
        uint32_t w0[kHalfRows], w1[kHalfRows];
#pragma unroll
        for (int k = 0; k < kHalfRows; ++k) {
            const uint32_t v = w.v[h * kHalfRows + k];
            w0[k] = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(tab) + word_addr<0>(v, woff));
            w1[k] = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(tab) + word_addr<16>(v, woff));
        }
#pragma unroll
        for (int k = 0; k < kHalfRows; ++k) {
            const int r = h * kHalfRows + k;
            const uint32_t base = uint32_t(128 * r);
            if (base >= wlen) break;   // rows past the window's end hold no occurrence of it
            if (qn > uint32_t(kTiledQueue - 128)) {
                tiled_drain<MAX>(tab, nb, q, qn, sums, id_off, bnd_rel, c.jl, lane);
                qn = 0;
            }
            const uint32_t v = w.v[r];
            const uint32_t rel = lane_rel + (base << kBinShift);
            // the bit of an ID sits at ID mod 32 of its word
            uint64_t m0 = __builtin_amdgcn_ballot_w64(__builtin_amdgcn_ubfe(w0[k], v, 1) != 0u);
            uint64_t m1 = __builtin_amdgcn_ballot_w64(__builtin_amdgcn_ubfe(w1[k], v >> 16, 1) != 0u);
            if (r == 0 && (c.ws & 1u)) m0 &= ~1ull;   // position ws2 belongs to the previous window
            if (base + 128u > wlen) {                 // positions from we on belong to the next
                m0 &= lanes_before((wlen - base + 1u) >> 1);
                m1 &= lanes_before((wlen - base) >> 1);
            }
            queue_slot(q, m0, qn, rel | (v & 0xFFFFu));
            queue_slot(q, m1, qn, (rel + (1u << kBinShift)) | (v >> 16));
        }
    }
    tiled_drain<MAX>(tab, nb, q, qn, sums, id_off, bnd_rel, c.jl, lane);
}

// One window of cursor c (its IDs in cur): find where it ends, advance c to the next
// window and issue that window's loads into nxt, then filter and drain this one.
template <bool MAX>
__device__ __forceinline__ void tiled_step(const TiledArgs &a, const Tile &T, int64_t T0, int64_t T1, int32_t nb,
                                           const uint32_t *tab, uint32_t *q, double *sums, int lane, TCur &c,
                                           const TWin &cur, TWin &nxt) {
    // this window ends at the span end, after kWindow positions, or where trial jl + 63
    // starts (so its trials are jl .. jl + 62: one per boundary lane)
    const uint32_t b63 = uint32_t(__builtin_amdgcn_readlane(int(cur.bnd), 63));
    const uint32_t we = min(min((c.ws & ~1u) + uint32_t(kWindow), c.e), max(b63, c.ws));
    // next cursor: the trial containing we, or the next bin
    TCur n = c;
    const uint64_t le = __builtin_amdgcn_ballot_w64(cur.bnd <= we);
    n.jl = c.jl + uint32_t(__popcll(le)) - 1u;
    n.ws = we;
    if (we >= c.e) {
        n.b = c.b + 1;
        tcur_seek(a, T, T0, T1, n);
    }
    n = tcur_uniform(n);
    twin_load(a, T, n, T0, T1, lane, nxt);
    tiled_window<MAX>(T, nb, tab, q, sums, c, we, cur, lane);
    c = n;
}

// One pass of a workgroup over trials [pass, pass_end) of analysis a (at most
// kPassTrials, split evenly over the waves, at most 252 each): every tile staged once,
// each wave's trials streamed tile by tile, then their YLT (or maxima) written.
// MAX = false: the YLT (sums of the occurrence-net losses, then the aggregate terms);
// MAX = true: each trial's largest occurrence-net loss (0 for none).
template <bool MAX>
__device__ __forceinline__ void tiled_pass(const TiledArgs &a, int64_t pass, int64_t pass_end, uint32_t *tab,
                                           uint32_t *q, double *sums, int lane, uint32_t wave) {
    const uint32_t nt = sload(a.n_tiles);
    const int64_t span = pass_end - pass;
    const int64_t per_wave = (span + kTiledWaves - 1) / kTiledWaves;
    const int64_t T0 = min(pass + int64_t(wave) * per_wave, pass_end);
    const int64_t T1 = min(T0 + per_wave, pass_end);
#pragma unroll
    for (int k = 0; k < kTiledWaveTrials / 64; ++k) sums[lane + 64 * k] = 0.0;
    for (uint32_t k = 0; k < nt; ++k) {
        const Tile T = load_tile(a.tiles, k);
        const int32_t nb = tile_span_blocks(T.blk_lo, T.blk_hi, a.nblk);
        // the first window's loads read no LDS: they are issued before the tile is
        // staged, so their latency overlaps the staging's
        TCur c;
        c.b = T0 < T1 ? T.bin_lo : T.bin_hi;
        c.ws = c.e = c.jl = 0;
        tcur_seek(a, T, T0, T1, c);
        c = tcur_uniform(c);
        TWin A;
        twin_load(a, T, c, T0, T1, lane, A);
        __syncthreads();
        stage_tile(a, T, nb, tab);
        __syncthreads();
        while (c.b < T.bin_hi) {
            TWin B;
            tiled_step<MAX>(a, T, T0, T1, nb, tab, q, sums, lane, c, A, B);
            A = B;
        }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < kTiledWaveTrials / 64; ++k) {
        const int64_t t = T0 + lane + 64 * k;
        if (t < T1) a.ylt[t - a.t_begin] = MAX ? sums[lane + 64 * k] : excess(sums[lane + 64 * k], a.agg_r, a.agg_l);
    }
    __builtin_amdgcn_wave_barrier();
}

// One analysis: workgroup w owns trials [t_begin + w per_wg, + per_wg), in passes.
template <bool MAX>
__global__ __launch_bounds__(1024) void k_trial_tiled(TiledArgs a) {
    __shared__ __attribute__((aligned(16))) uint32_t tab[kTileWords];
    __shared__ uint32_t queues[kTiledWaves * kQueueStride];
    __shared__ double wsums[kTiledWaves * kTiledWaveTrials];
    const int lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t wg0 = a.t_begin + int64_t(blockIdx.x) * a.per_wg;
    const int64_t wg1 = min(wg0 + a.per_wg, a.t_end);
    for (int64_t pass = wg0; pass < wg1; pass += kPassTrials)
        tiled_pass<MAX>(a, pass, min(pass + int64_t(kPassTrials), wg1), tab, queues + wave * kQueueStride,
                        wsums + wave * kTiledWaveTrials, lane, wave);
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

// Many analyses in one launch (YLTs): the items are the passes that k_trial_tiled
// would run for each analysis (the same trials per pass, so the same YLT bits), taken
// in list order from a counter by whichever workgroup is free; a workgroup stops once
// the counter passes the list.
__global__ __launch_bounds__(1024) void k_trial_tiled_items(const TiledArgs *__restrict__ jobs,
                                                            const TiledItem *__restrict__ items, int32_t n_items,
                                                            uint32_t *__restrict__ next) {
    __shared__ __attribute__((aligned(16))) uint32_t tab[kTileWords];
    __shared__ uint32_t queues[kTiledWaves * kQueueStride];
    __shared__ double wsums[kTiledWaves * kTiledWaveTrials];
    // the item taken: in wave 0's first slot past its queue (a drain reads such slots
    // only as entries it does not add, and none runs while the item is taken)
    uint32_t *took = queues + kTiledQueue;
    const int lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (;;) {
        if (threadIdx.x == 0) *took = atomicAdd(next, 1u);
        __syncthreads();
        const uint32_t it = __builtin_amdgcn_readfirstlane(*took);
        __syncthreads();   // every wave has read `took` before it is taken again
        if (it >= uint32_t(n_items)) return;
        const uint32_t *iw = reinterpret_cast<const uint32_t *>(items + it);
        const int32_t job = int32_t(sload(iw + 0));
        const int64_t t0 = int64_t(uint64_t(sload(iw + 2)) | (uint64_t(sload(iw + 3)) << 32));
        const int64_t t1 = int64_t(uint64_t(sload(iw + 4)) | (uint64_t(sload(iw + 5)) << 32));
        const TiledArgs a = load_args(jobs, job);
        tiled_pass<false>(a, t0, t1, tab, queues + wave * kQueueStride, wsums + wave * kTiledWaveTrials, lane, wave);
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

hipError_t launch_trial_tiled(const TiledArgs &a, int grid, hipStream_t s, bool occ_max) {
    if (occ_max) hipLaunchKernelGGL(k_trial_tiled<true>, dim3(grid), dim3(kTiledWaves * 64), 0, s, a);
    else hipLaunchKernelGGL(k_trial_tiled<false>, dim3(grid), dim3(kTiledWaves * 64), 0, s, a);
    return hipGetLastError();
}

}  // namespace ara
