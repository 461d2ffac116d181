// Preprocessing stage (Section II-B: inputs are loaded into memory before the
// analysis): YET validation and ELT direct access table construction
// (Section III-B: an ELT as a dense array over the whole catalog, zero for the
// events it does not list).
#include "ara_internal.h"

namespace ara {

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

__global__ void k_fill_u32(uint32_t *__restrict__ p, size_t n, uint32_t v) {
    size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    size_t stride = size_t(gridDim.x) * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill_u32, dim3(unsigned(blocks)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// One pass over the YET: every event ID in [0, catalog), offsets in CSR form.
__global__ void k_validate_yet(const int32_t *__restrict__ ids, int64_t n_events, const int64_t *__restrict__ offs,
                               int64_t n_trials, int32_t catalog, uint32_t *err, int check_ids) {
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    uint32_t bad = 0;
    const int64_t n4 = check_ids ? n_events >> 2 : 0;
    const i32x4 *ids4 = reinterpret_cast<const i32x4 *>(ids);
    const uint32_t c = uint32_t(catalog);
    for (int64_t i = tid; i < n4; i += stride) {
        i32x4 v = __builtin_nontemporal_load(ids4 + i);
        if (uint32_t(v.x) >= c || uint32_t(v.y) >= c || uint32_t(v.z) >= c || uint32_t(v.w) >= c) bad |= ERR_ID_RANGE;
    }
    for (int64_t i = (n4 << 2) + tid; check_ids && i < n_events; i += stride)
        if (uint32_t(ids[i]) >= c) bad |= ERR_ID_RANGE;
    for (int64_t t = tid; t <= n_trials; t += stride) {
        const int64_t o = offs[t];
        if (o < 0 || o > n_events) bad |= ERR_OFFSETS;
        if (t == 0 && o != 0) bad |= ERR_OFFSETS;
        if (t == n_trials && o != n_events) bad |= ERR_OFFSETS;
        if (t < n_trials && offs[t + 1] < o) bad |= ERR_OFFSETS;
    }
    if (bad) atomicOr(err, bad);
}

hipError_t launch_validate_yet(const int32_t *ids, int64_t n_events, const int64_t *offs, int64_t n_trials,
                               int32_t catalog, uint32_t *err, hipStream_t s, bool check_ids) {
    hipLaunchKernelGGL(k_validate_yet, dim3(4096), dim3(256), 0, s, ids, n_events, offs, n_trials, catalog, err,
                       check_ids ? 1 : 0);
    return hipGetLastError();
}

// Packed copy of checked event IDs (all < 2^24): 4 IDs per 12-byte group, event i at
// bytes 3i..3i+2 little endian; the last group is zero-padded.
size_t yet_packed_bytes(int64_t n_events) { return size_t((n_events + 3) / 4) * 12; }

__global__ void k_yet_pack(const int32_t *__restrict__ ids, int64_t n_events, uint32_t *__restrict__ out) {
    const int64_t groups = (n_events + 3) / 4;
    for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < groups; g += int64_t(gridDim.x) * blockDim.x) {
        uint32_t v[4];
        if (4 * g + 4 <= n_events) {
            const i32x4 x = __builtin_nontemporal_load(reinterpret_cast<const i32x4 *>(ids) + g);
            v[0] = uint32_t(x.x), v[1] = uint32_t(x.y), v[2] = uint32_t(x.z), v[3] = uint32_t(x.w);
        } else {
            for (int j = 0; j < 4; ++j) v[j] = 4 * g + j < n_events ? uint32_t(ids[4 * g + j]) : 0u;
        }
        out[3 * g + 0] = v[0] | (v[1] << 24);
        out[3 * g + 1] = (v[1] >> 8) | (v[2] << 16);
        out[3 * g + 2] = (v[2] >> 16) | (v[3] << 8);
    }
}

hipError_t launch_yet_pack(const int32_t *ids, int64_t n_events, uint8_t *packed, hipStream_t s) {
    if (n_events <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_yet_pack, dim3(4096), dim3(256), 0, s, ids, n_events, reinterpret_cast<uint32_t *>(packed));
    return hipGetLastError();
}

// Zero each ELT's seen bits (grid.y = ELT index).  An entry of the direct access
// table is defined only where its seen bit is set: the scatter sets the bit with
// every value it writes, and readers take 0 where the bit is clear, so the table
// itself (8 or 4 bytes per catalog event) is never cleared, only its bits (one
// per event).
__global__ void k_elt_clear(const EltDesc *__restrict__ d, int32_t catalog) {
    const EltDesc e = d[blockIdx.y];
    const size_t seen_words = (size_t(catalog) + 31) / 32;
    size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const size_t stride = size_t(gridDim.x) * blockDim.x;
    for (size_t k = i; k < seen_words; k += stride) e.seen[k] = 0u;
}

hipError_t launch_elt_clear(const EltDesc *d, int n_elts, int32_t catalog, hipStream_t s) {
    if (n_elts <= 0) return hipSuccess;
    const size_t words = (size_t(catalog) + 31) / 32;
    unsigned bx = unsigned(std::min<size_t>((words + 255) / 256, 1024));
    hipLaunchKernelGGL(k_elt_clear, dim3(bx, unsigned(n_elts)), dim3(256), 0, s, d, catalog);
    return hipGetLastError();
}

// Scatter the (event, loss) records of each ELT into its table (grid.y = ELT),
// setting each written event's seen bit.  Rejects IDs outside the catalog,
// negative / NaN / infinite losses (neither written nor marked), and an event
// listed twice (the seen bit was already set).
__global__ void k_elt_scatter(const EltDesc *__restrict__ d, int32_t catalog, uint32_t *err) {
    const EltDesc e = d[blockIdx.y];
    uint32_t bad = 0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < e.n_pairs;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int32_t id = e.pair_ids[i];
        const double l = e.pair_losses[i];
        if (uint32_t(id) >= uint32_t(catalog)) { bad |= ERR_ID_RANGE; continue; }
        if (!(l >= 0.0) || __builtin_isinf(l)) { bad |= ERR_LOSS; continue; }
        const uint32_t bit = 1u << (id & 31);
        const uint32_t old = atomicOr(e.seen + (id >> 5), bit);
        if (old & bit) bad |= ERR_DUP;
        if (e.f32) reinterpret_cast<float *>(e.dat)[id] = float(l);
        else reinterpret_cast<double *>(e.dat)[id] = l;
    }
    if (bad) atomicOr(err, bad);
}

hipError_t launch_elt_scatter(const EltDesc *d, int n_elts, int64_t max_pairs, int32_t catalog, uint32_t *err,
                              hipStream_t s) {
    if (n_elts <= 0 || max_pairs <= 0) return hipSuccess;
    unsigned bx = unsigned(std::min<int64_t>((max_pairs + 255) / 256, 1024));
    hipLaunchKernelGGL(k_elt_scatter, dim3(bx, unsigned(n_elts)), dim3(256), 0, s, d, catalog, err);
    return hipGetLastError();
}

}  // namespace ara
