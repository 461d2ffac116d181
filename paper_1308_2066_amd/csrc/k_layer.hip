// Per-layer tables.
//
// Combined table: steps 1 and 2 of the basic algorithm (Section II-B) look each
// occurrence up in every ELT of the layer, apply that ELT's financial terms and
// accumulate across ELTs.  The result for an occurrence depends only on its event,
// so it is computed once per catalog event here, in the same order and rounding
// (ELTs in listed order, binary64, starting from +0.0); a trial's lookup of event e
// then reads comb[e].
//
// Occurrence filter: step 3 applies the occurrence terms (Table I) to each
// occurrence independently of the others, so the occurrence-net loss
// min(max(comb[e] - OccR, 0), OccL) is again a function of the event alone; it is
// computed once per catalog event (binary64, same operations as per occurrence).
// Events whose occurrence-net loss is zero contribute nothing to a trial, so the
// filter also records one bit per event ("nonzero"), per-128-event prefix counts of
// set bits, and the nonzero values compacted in event order.  A trial kernel can
// keep the bits and counts in LDS and read only the flagged values from L2.
#include "ara_internal.h"

namespace ara {

__device__ __forceinline__ double excess(double x, double retention, double limit) {
    double v = x - retention;
    v = v < 0.0 ? 0.0 : v;
    return v > limit ? limit : v;
}

template <typename V>
__global__ __launch_bounds__(256) void k_layer_bitmap(const V *__restrict__ comb, int32_t catalog, double occ_r,
                                                      double occ_l, double *__restrict__ occ,
                                                      uint32_t *__restrict__ bitmap, int64_t n_words) {
    // one thread per event slot of the bitmap; each wave covers 64 events = 2 words
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    bool flag = false;
    if (e < catalog) {
        const double o = excess(double(comb[e]), occ_r, occ_l);
        occ[e] = o;
        flag = o > 0.0;
    }
    const uint64_t m = __ballot(flag);
    const int lane = threadIdx.x & 63;
    const int64_t w0 = (e - lane) >> 5;   // even; n_words is a multiple of 4
    if (w0 >= n_words) return;
    if (lane == 0) bitmap[w0] = uint32_t(m);
    if (lane == 1) bitmap[w0 + 1] = uint32_t(m >> 32);
}

// The combined table and the occurrence filter in one pass over the catalog: per
// event, the ELTs' terms-applied losses added in listed order from +0.0 (rounded to
// the table's type), then the operations of k_layer_bitmap on the stored value.
// An ELT's loss for an event it does not list is 0 (its terms still applied, as
// for any loss): its table is read only where the event's seen bit is set, so a
// wave fetches only the table lines that hold listed events.  A wave covers 64
// consecutive events, two seen words per ELT: one load brings those words of 32
// ELTs (lane 2i + h: word h of ELT i), each ELT's 64-bit mask is then read out
// uniformly, a wave skips an ELT that lists none of its events, and the table
// loads of 8 ELTs are issued before their values are added in order.  Those loads
// are 8-byte buffer loads issued by every lane and for every ELT: a lane whose bit
// is clear reads past the record (0, no memory access), so nothing branches around
// a load.
template <typename V>
__global__ __launch_bounds__(256) void k_layer_combine_bitmap(const EltDesc *__restrict__ d, int n_elts,
                                                              int32_t catalog, V *__restrict__ comb, double occ_r,
                                                              double occ_l, double *__restrict__ occ,
                                                              uint32_t *__restrict__ bitmap,
                                                              uint32_t *__restrict__ nz, int64_t n_words) {
    constexpr int kGroup = 8;
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int64_t e0 = e - lane;                       // multiple of 64: the wave's first event
    const int64_t seen_words = (int64_t(catalog) + 31) >> 5;
    bool flag = false, nonzero = false;
    if (e0 < catalog) {                                // wave-uniform
        double s = 0.0;
        for (int jb = 0; jb < n_elts; jb += 32) {
            const int jl = jb + (lane >> 1);
            const int64_t wi = (e0 >> 5) + (lane & 1);
            uint32_t wv = 0u;
            if (jl < n_elts && wi < seen_words) wv = d[jl].seen[wi];
            const int nj = n_elts - jb < 32 ? n_elts - jb : 32;
            for (int i = 0; i < nj; i += kGroup) {   // i + k <= 31
                uint64_t raw[kGroup];
#pragma unroll
                for (int k = 0; k < kGroup; ++k) {
                    // past the last ELT: the lanes' words are 0, every lane reads past the record
                    const EltDesc &t = d[jb + i + k < n_elts ? jb + i + k : n_elts - 1];
                    const uint64_t m = uint64_t(uint32_t(__builtin_amdgcn_readlane(int(wv), 2 * (i + k)))) |
                                       uint64_t(uint32_t(__builtin_amdgcn_readlane(int(wv), 2 * (i + k) + 1))) << 32;
                    // binary32 tables: the aligned pair holding the entry (allocated in whole
                    // pairs); catalog <= 2^28 events keeps byte offsets below 2^31
                    const uint32_t rec = t.f32 ? (uint32_t(catalog) * 4u + 7u) & ~7u : uint32_t(catalog) * 8u;
                    const uint32_t at = t.f32 ? (uint32_t(e) * 4u) & ~7u : uint32_t(e) * 8u;
                    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(t.dat, 0, int(rec), kBufWord3);
                    raw[k] = __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(
                                                              r, (m >> lane) & 1u ? at : 0xFFFFFFF8u, 0, 0));
                }
#pragma unroll
                for (int k = 0; k < kGroup; ++k) {
                    if (i + k < nj) {
                        const EltDesc &t = d[jb + i + k];
                        double v = t.f32 ? double(__builtin_bit_cast(float, uint32_t(raw[k] >> ((e & 1) * 32))))
                                         : __builtin_bit_cast(double, raw[k]);
                        if (!t.identity) v = excess(t.fx * v, t.retention, t.limit);
                        s = s + v;
                    }
                }
            }
        }
        if (e < catalog) {
            const V c = V(s);
            comb[e] = c;
            nonzero = c != V(0);
            const double o = excess(double(c), occ_r, occ_l);
            occ[e] = o;
            flag = o > 0.0;
        }
    }
    const uint64_t m = __ballot(flag);
    const uint64_t z = __ballot(nonzero);
    const int64_t w0 = e0 >> 5;   // even; n_words is a multiple of 4
    if (w0 >= n_words) return;
    if (lane == 0) bitmap[w0] = uint32_t(m);
    if (lane == 1) bitmap[w0 + 1] = uint32_t(m >> 32);
    if (lane == 2) nz[w0] = uint32_t(z);
    if (lane == 3) nz[w0 + 1] = uint32_t(z >> 32);
}

// Exclusive prefix of per-block set-bit counts (rank), the same split into a 16-bit
// offset within its superblock of 256 blocks and a 32-bit base per superblock
// (rel16/base32: a smaller table to keep in LDS), and the total.  Single workgroup
// of 1024.
__global__ __launch_bounds__(1024) void k_layer_rank(const uint32_t *__restrict__ bitmap, int32_t nblk,
                                                     uint32_t *__restrict__ rank, uint32_t *__restrict__ n_flagged,
                                                     uint16_t *__restrict__ rel16, uint32_t *__restrict__ base32) {
    // each thread takes 8 consecutive blocks (their loads issued together), so a
    // catalog of up to 2^20 events is one round of loads and one scan
    constexpr int kPer = 8, kChunk = 1024 * kPer;
    static_assert(kChunk % kBlocksPerSuper == 0 && kBlocksPerSuper % kPer == 0,
                  "superblocks are whole in a chunk and start at a thread's first block");
    __shared__ uint32_t wsum[16];
    __shared__ uint32_t sbase[kChunk / kBlocksPerSuper];
    __shared__ uint32_t rk[kChunk];             // the chunk's ranks, for coalesced stores
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint32_t carry = 0;
    for (int32_t base = 0; base < nblk; base += kChunk) {
        const int32_t b0 = base + tid * kPer;
        uint4 q[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j)
            q[j] = b0 + j < nblk ? reinterpret_cast<const uint4 *>(bitmap)[b0 + j] : make_uint4(0u, 0u, 0u, 0u);
        uint32_t c[kPer], tot = 0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            c[j] = __popc(q[j].x) + __popc(q[j].y) + __popc(q[j].z) + __popc(q[j].w);
            tot += c[j];
        }
        uint32_t inc = tot;   // inclusive wave scan of the threads' totals
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        uint32_t before = 0, total = 0;
        for (int k = 0; k < 16; ++k) {
            if (k < w) before += wsum[k];
            total += wsum[k];
        }
        uint32_t r = carry + before + inc - tot;
        if (b0 % kBlocksPerSuper == 0 && b0 < nblk) {
            const int32_t sb = b0 / kBlocksPerSuper;
            sbase[(b0 - base) / kBlocksPerSuper] = r;
            base32[sb] = r;
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            rk[tid * kPer + j] = r;
            r += c[j];
        }
        __syncthreads();
        // written out from LDS by consecutive threads (one CU's stores coalesce)
        for (int k = tid; k < kChunk && base + k < nblk; k += 1024) {
            const uint32_t v = rk[k];
            rank[base + k] = v;
            rel16[base + k] = uint16_t(v - sbase[k / kBlocksPerSuper]);
        }
        carry += total;
        __syncthreads();
    }
    if (tid == 0) *n_flagged = carry;
}

__global__ __launch_bounds__(256) void k_layer_compact(const double *__restrict__ occ, int32_t catalog,
                                                       const uint32_t *__restrict__ bitmap,
                                                       const uint32_t *__restrict__ rank, double *__restrict__ vals) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= catalog) return;
    const uint32_t word = bitmap[e >> 5];
    const uint32_t bit = uint32_t(e) & 31u;
    if (!((word >> bit) & 1u)) return;
    const int64_t blk = e >> 7;
    const uint32_t k = (uint32_t(e) >> 5) & 3u;
    uint32_t idx = rank[blk] + __popc(word & ((1u << bit) - 1u));
    for (uint32_t q = 0; q < k; ++q) idx += __popc(bitmap[blk * 4 + q]);
    vals[idx] = occ[e];
}

// Ranks (with rel16/base32), the flagged count and the compacted values.
hipError_t launch_layer_ranks(int32_t catalog, const LayerTables &t, hipStream_t s) {
    hipLaunchKernelGGL(k_layer_rank, dim3(1), dim3(1024), 0, s, t.bitmap, t.nblk, t.rank, t.n_flagged, t.rel16,
                       t.base32);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned ev_blocks = unsigned((int64_t(catalog) + 255) / 256);
    hipLaunchKernelGGL(k_layer_compact, dim3(ev_blocks), dim3(256), 0, s, t.occ, catalog, t.bitmap, t.rank, t.vals);
    return hipGetLastError();
}

hipError_t launch_layer_tables(const EltDesc *d, int n_elts, int32_t catalog, bool f32, double occ_r, double occ_l,
                               const LayerTables &t, hipStream_t s, bool ranks) {
    // the bitmap covers nblk*128 event slots = nblk*2 waves; launch whole waves only
    const unsigned blocks = unsigned((int64_t(t.nblk) * kEventsPerBlock + 255) / 256);
    if (f32) {
        hipLaunchKernelGGL(k_layer_combine_bitmap<float>, dim3(blocks), dim3(256), 0, s, d, n_elts, catalog,
                           (float *)t.comb, occ_r, occ_l, t.occ, t.bitmap, t.nz, int64_t(t.nblk) * 4);
    } else {
        hipLaunchKernelGGL(k_layer_combine_bitmap<double>, dim3(blocks), dim3(256), 0, s, d, n_elts, catalog,
                           (double *)t.comb, occ_r, occ_l, t.occ, t.bitmap, t.nz, int64_t(t.nblk) * 4);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !ranks) return e;
    return launch_layer_ranks(catalog, t, s);
}

hipError_t launch_layer_filter(int32_t catalog, bool f32, double occ_r, double occ_l, const LayerTables &t,
                               hipStream_t s, bool ranks) {
    // the bitmap covers nblk*128 event slots = nblk*2 waves; launch whole waves only
    const unsigned bm_threads_blocks = unsigned((int64_t(t.nblk) * kEventsPerBlock + 255) / 256);
    if (f32) {
        hipLaunchKernelGGL(k_layer_bitmap<float>, dim3(bm_threads_blocks), dim3(256), 0, s, (const float *)t.comb,
                           catalog, occ_r, occ_l, t.occ, t.bitmap, int64_t(t.nblk) * 4);
    } else {
        hipLaunchKernelGGL(k_layer_bitmap<double>, dim3(bm_threads_blocks), dim3(256), 0, s, (const double *)t.comb,
                           catalog, occ_r, occ_l, t.occ, t.bitmap, int64_t(t.nblk) * 4);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !ranks) return e;
    return launch_layer_ranks(catalog, t, s);
}

}  // namespace ara
