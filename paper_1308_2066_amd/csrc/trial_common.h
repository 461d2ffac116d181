// Device helpers shared by the trial kernels (internal).
#pragma once

#include "ara_internal.h"

namespace ara {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

constexpr int kChunk = 256;               // events per wave-wide 16-byte load (64 lanes x 4)
constexpr int kNch = 4;                   // loads per segment
constexpr int kSeg = kChunk * kNch;       // events per segment
constexpr int kSlots = kNch * 4;          // events per lane per segment
constexpr int kNonTemporal = 2;           // cache policy of the ID stream loads

// min(max(x - retention, 0), limit): the excess-of-loss clamp of Table I.
__device__ __forceinline__ double excess(double x, double retention, double limit) {
    double v = x - retention;
    v = v < 0.0 ? 0.0 : v;
    return v > limit ? limit : v;
}

// One DPP lane permutation of a binary64 value (both halves moved the same way).
template <int Ctrl>
__device__ __forceinline__ double dpp_f64(double x) {
    const uint2 u = __builtin_bit_cast(uint2, x);
    uint2 r;
    r.x = uint32_t(__builtin_amdgcn_update_dpp(0, int(u.x), Ctrl, 0xF, 0xF, false));
    r.y = uint32_t(__builtin_amdgcn_update_dpp(0, int(u.y), Ctrl, 0xF, 0xF, false));
    return __builtin_bit_cast(double, r);
}

__device__ __forceinline__ double readlane_f64(double x, int l) {
    const uint2 u = __builtin_bit_cast(uint2, x);
    uint2 r;
    r.x = uint32_t(__builtin_amdgcn_readlane(int(u.x), l));
    r.y = uint32_t(__builtin_amdgcn_readlane(int(u.y), l));
    return __builtin_bit_cast(double, r);
}

// Sum over a full wave, returned to every lane.  Within each 16-lane row: pair lanes
// i^1, i^2, then mirror halves of 8 and of 16 (each step adds a value and its partner,
// so both end equal: a + b == b + a exactly); then the four row sums are combined in
// a fixed order.  No LDS traffic.
__device__ __forceinline__ double wave_total(double x) {
    x += dpp_f64<0xB1>(x);    // quad_perm [1,0,3,2]
    x += dpp_f64<0x4E>(x);    // quad_perm [2,3,0,1]
    x += dpp_f64<0x141>(x);   // row_half_mirror
    x += dpp_f64<0x140>(x);   // row_mirror
    return (readlane_f64(x, 0) + readlane_f64(x, 16)) + (readlane_f64(x, 32) + readlane_f64(x, 48));
}

__device__ __forceinline__ int64_t uniform64(int64_t x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(x)));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(x) >> 32));
    return int64_t((uint64_t(hi) << 32) | lo);
}

// Trial offsets are read through the scalar data path (constant address space):
// they are wave-uniform and their loads then wait on the scalar counter instead of
// joining the in-order vector-memory queue behind the event-ID prefetch.
typedef const __attribute__((address_space(4))) int64_t *const_i64_ptr;
__device__ __forceinline__ int64_t offset_at(const int64_t *offs, int64_t t) { return ((const_i64_ptr)offs)[t]; }

// Issue the four 16-byte ID loads of a segment starting at event sbase, `avail`
// events readable (0..kSeg; bytes past them are outside the buffer record and read
// as 0 without a memory access).  Always issued, so the number of outstanding
// vector-memory operations is the same on every path.
__device__ __forceinline__ void load_ids(const int32_t *ids, int64_t sbase, int avail, int lane, u32x4 (&r)[kNch]) {
    __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)(ids + sbase), 0, avail * 4, kBufWord3);
#pragma unroll
    for (int k = 0; k < kNch; ++k)
        r[k] = __builtin_amdgcn_raw_buffer_load_b128(rs, k * kChunk * 4 + lane * 16, 0, kNonTemporal);
    if (avail & 3) {
        // The YET ends inside one lane's 16-byte group: fetch that group's IDs one
        // dword at a time so a partially covered 16-byte load cannot drop them.
        const int g = (avail & ~3) - lane * 4;
#pragma unroll
        for (int k = 0; k < kNch; ++k) {
            if (g == k * kChunk) {
                const int e0 = k * kChunk + lane * 4;
                for (int j = 0; j < 4; ++j) {
                    uint32_t v = 0;
                    if (e0 + j < avail) v = __builtin_amdgcn_raw_buffer_load_b32(rs, (e0 + j) * 4, 0, 0);
                    r[k][j] = v;
                }
            }
        }
    }
}

// Packed IDs (3 bytes each, 12-byte groups of 4 events, zero-padded to whole groups):
// the same segment layout as load_ids, one 12-byte load per lane and chunk.  sbase
// and avail are multiples of 4, so each group is wholly inside or outside the record.
__device__ __forceinline__ void load_ids24(const uint8_t *ids24, int64_t sbase, int avail, int lane, u32x3 (&r)[kNch]) {
    __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)(ids24 + 3 * sbase), 0, avail * 3, kBufWord3);
#pragma unroll
    for (int k = 0; k < kNch; ++k)
        r[k] = __builtin_amdgcn_raw_buffer_load_b96(rs, k * kChunk * 3 + lane * 12, 0, kNonTemporal);
}

__device__ __forceinline__ void unpack_ids24(const u32x3 &w, uint32_t *id) {
    id[0] = w.x & 0xFFFFFFu;
    id[1] = (w.x >> 24) | ((w.y << 8) & 0xFFFF00u);
    id[2] = (w.y >> 16) | ((w.z << 16) & 0xFF0000u);
    id[3] = w.z >> 8;
}

// Packed form: readable events from sbase up to the trial's end rounded up to a
// whole group (the padded buffer always holds it), at most one segment.
__device__ __forceinline__ int seg_avail24(int64_t sbase, int64_t o1) {
    const int64_t a = ((o1 + 3) & ~int64_t(3)) - sbase;
    return int(a < 0 ? 0 : (a > kSeg ? kSeg : a));
}

// Events readable from sbase for a trial ending at o1: up to the trial's end
// rounded up to a 16-byte group, never past the YET, at most one segment.
__device__ __forceinline__ int seg_avail(int64_t sbase, int64_t o1, int64_t n_events) {
    int64_t end = (o1 + 3) & ~int64_t(3);
    if (end > n_events) end = n_events;
    int64_t a = end - sbase;
    return int(a < 0 ? 0 : (a > kSeg ? kSeg : a));
}

// Occurrence filter in LDS (layout: bits | rel16 | base32, see bitmap_*_offset):
// index among flagged events of flagged event e = rank of its superblock + rank of
// its 128-event block within the superblock + set bits before it in the block.
// Branch-free: the block's four words are read at once and selected arithmetically.
__device__ __forceinline__ uint32_t bitmap_rank(const uint32_t *tab, int32_t nblk, uint32_t e) {
    const uint32_t blk = e >> 7, q = (e >> 5) & 3u;
    const u32x4 W = reinterpret_cast<const u32x4 *>(tab)[blk];
    const uint16_t *lrel = reinterpret_cast<const uint16_t *>(reinterpret_cast<const char *>(tab) + bitmap_rel_offset(nblk));
    const uint32_t *lbase = reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(tab) + bitmap_base_offset(nblk));
    const bool q1 = (q & 1u) != 0u, q2 = (q & 2u) != 0u;
    const uint32_t word = q2 ? (q1 ? W.w : W.z) : (q1 ? W.y : W.x);
    const uint32_t c0 = __popc(W.x), c1 = c0 + __popc(W.y), c2 = c1 + __popc(W.z);
    const uint32_t before = q2 ? (q1 ? c2 : c1) : (q1 ? c0 : 0u);   // set bits in the block's earlier words
    const uint32_t below = __popc(word & ((1u << (e & 31u)) - 1u));  // set bits below e in its word
    return lbase[e >> 15] + uint32_t(lrel[blk]) + before + below;
}

// Copy the layer's occurrence filter into LDS (whole workgroup; ends with a barrier).
__device__ __forceinline__ void stage_bitmap(const TrialArgs &a, uint32_t *tab) {
    const int32_t nblk = a.nblk;
    u32x4 *l4 = reinterpret_cast<u32x4 *>(tab);
    const u32x4 *g4 = reinterpret_cast<const u32x4 *>(a.bitmap);
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) l4[i] = g4[i];
    // rel16 is allocated with 16-byte padding, so whole words can be copied
    uint32_t *lr = tab + bitmap_rel_offset(nblk) / 4;
    const uint32_t *gr = reinterpret_cast<const uint32_t *>(a.rel16);
    for (int i = threadIdx.x; i < (nblk + 1) / 2; i += blockDim.x) lr[i] = gr[i];
    uint32_t *lb = tab + bitmap_base_offset(nblk) / 4;
    for (int i = threadIdx.x; i < bitmap_supers(nblk); i += blockDim.x) lb[i] = a.base32[i];
    __syncthreads();
}

}  // namespace ara
