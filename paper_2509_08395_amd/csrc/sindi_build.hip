// gfx950 kernels of the index build on the device: the same index as the host
// build (Alg. 3: pruning of every document, then Alg. 1's lists in the tiled,
// 4-posting-aligned layout), bit for bit.
//
//   k_check_rows     structure of a device corpus (Def. 1)
//   k_prune_rows     MRP (Defs. 5-6) or VNP (Sec. 4.1), one wave per row of up
//                    to kWaveRow entries; longer rows are listed for
//   k_prune_long     the same, one workgroup per row of up to kLongRow entries
//   k_count_lists    entries per (tile, term) list, the storage range check
//                    and each term's largest stored |x|
//   k_list_offsets   per tile: 4-posting group offsets of the lists, pad counts
//   k_fill_lists     one wave per tile walks the tile's documents in order and
//                    places every kept entry at its list's cursor (LDS), so a
//                    list holds its documents in ascending order
//   k_fill_pads      the pad entries after every list
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "sindi.h"
#include "sindi_internal.h"

namespace sindi {
namespace {

constexpr int kWave = 64;
constexpr int kWaveRow = 512;     // longest row pruned by one wave
constexpr int kRowsPerWg = 4;     // waves (rows) per workgroup of k_prune_rows

// Waits for this wave's LDS operations so that every lane sees the others'.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Entry order of Def. 6: larger |x| first, equal |x| by lower term id.
// Non-entries (zero values) carry |x| = -1 and rank after every entry.
__device__ __forceinline__ bool before(float ax, int32_t ix, float ay, int32_t iy)
{
    return ax > ay || (ax == ay && ix < iy);
}

// FP16 / BF16 bits of an FP32 value, round to nearest even.
__device__ __forceinline__ uint16_t f16_bits(float x) { return __builtin_bit_cast(uint16_t, (_Float16)x); }
__device__ __forceinline__ uint16_t bf16_bits(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Kept prefix length of a row whose non-zero |x| sit in Def. 6 order in
// s[0, m) (FP64): the shortest prefix whose sum, taken in that order, reaches
// alpha times the mass (the same sum over all m); alpha = 1 keeps all.
__device__ int64_t mass_prefix(const double *s, int64_t m, double alpha)
{
    if (alpha >= 1.0) return m;
    double mass = 0.0;
    for (int64_t t = 0; t < m; ++t) mass += s[t];
    const double thr = alpha * mass;
    double run = 0.0;
    int64_t r = 0;
    while (r < m) {
        run += s[r];
        ++r;
        if (run >= thr) break;
    }
    return r;
}

// err bits: 1 row pointers, 2 term id range, 4 ids not ascending, 8 non-finite.
// One wave per row.
__global__ __launch_bounds__(256) void k_check_rows(const int64_t *ptr, const int32_t *idx,
                                                    const float *val, int64_t n_rows,
                                                    int64_t n_cols, int64_t nnz, int32_t *err)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (row >= n_rows) return;
    const int64_t a = ptr[row], b = ptr[row + 1];
    int bad = 0;
    if (a < 0 || b < a || b > nnz || (row == 0 && a != 0) || (row == n_rows - 1 && b != nnz))
        bad |= 1;
    if (!bad)
        for (int64_t e = a + lane; e < b; e += kWave) {
            const int32_t id = idx[e];
            if (id < 0 || id >= n_cols) bad |= 2;
            if (e + 1 < b && idx[e + 1] <= id) bad |= 4;
            if (!isfinite(val[e])) bad |= 8;
        }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) bad |= __shfl_xor(bad, m, kWave);
    if (bad && lane == 0) atomicOr(err, bad);
}

// One wave per row of at most kWaveRow entries.  Each lane ranks its entries
// by counting the row's entries before them in Def. 6 order (the row staged in
// the wave's LDS); MRP places |x| at its rank (FP64) and lane 0 takes the
// prefix sums in that order.  Longer rows are appended to long_rows (err bit
// 128: a row longer than kLongRow).
__global__ __launch_bounds__(kRowsPerWg * kWave) void k_prune_rows(
    const int64_t *ptr, const int32_t *idx, const float *val, int64_t n_rows, int32_t mode,
    double alpha, int32_t vn, uint8_t *keep, int32_t *long_rows, uint32_t *n_long, int32_t *err)
{
    constexpr int PER = kWaveRow / kWave;
    __shared__ float s_a[kRowsPerWg][kWaveRow];
    __shared__ int32_t s_id[kRowsPerWg][kWaveRow];
    __shared__ double s_sum[kRowsPerWg][kWaveRow];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t row = (int64_t)blockIdx.x * kRowsPerWg + w;
    if (row >= n_rows) return;
    const int64_t a = ptr[row], n = ptr[row + 1] - a;
    if (n > kWaveRow) {
        if (lane == 0) {
            if (n > kLongRow) atomicOr(err, 128);
            else long_rows[atomicAdd(n_long, 1u)] = (int32_t)row;
        }
        return;
    }
    float ax[PER];
    int32_t id[PER];
    int32_t m = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int64_t e = i * kWave + lane;
        ax[i] = -1.0f;
        id[i] = 0;
        if (e < n) {
            const float v = val[a + e];
            ax[i] = v != 0.0f ? fabsf(v) : -1.0f;  // zeros are not entries (Def. 1)
            id[i] = idx[a + e];
            s_a[w][e] = ax[i];
            s_id[w][e] = id[i];
        }
        m += __popcll(__ballot(e < n && ax[i] >= 0.0f));
    }
    wave_sync();
    int32_t rank[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        rank[i] = INT32_MAX;
        if (ax[i] < 0.0f) continue;
        int32_t r = 0;
        for (int64_t f = 0; f < n; ++f) r += before(s_a[w][f], s_id[w][f], ax[i], id[i]) ? 1 : 0;
        rank[i] = r;
    }
    int64_t keep_n;
    if (mode == SINDI_PRUNE_VNP) {
        keep_n = min((int64_t)vn, (int64_t)m);
    } else {
#pragma unroll
        for (int i = 0; i < PER; ++i)
            if (ax[i] >= 0.0f) s_sum[w][rank[i]] = (double)ax[i];
        wave_sync();
        int64_t r0 = 0;
        if (lane == 0) r0 = mass_prefix(s_sum[w], m, alpha);
        keep_n = __shfl(r0, 0, kWave);
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int64_t e = i * kWave + lane;
        if (e < n) keep[a + e] = rank[i] < keep_n ? 1 : 0;
    }
}

// One workgroup per long row (at most kLongRow entries), staged in LDS: the
// row's |x| and ids, and the |x| in rank order for the mass prefix; each
// thread keeps the ranks of its own entries in registers.
__global__ __launch_bounds__(256) void k_prune_long(const int64_t *ptr, const int32_t *idx,
                                                    const float *val, const int32_t *rows,
                                                    int32_t mode, double alpha, int32_t vn,
                                                    uint8_t *keep)
{
    extern __shared__ __align__(16) unsigned char smem[];
    float *s_a = reinterpret_cast<float *>(smem);                       // [kLongRow]
    int32_t *s_id = reinterpret_cast<int32_t *>(s_a + kLongRow);        // [kLongRow]
    double *s_sum = reinterpret_cast<double *>(s_id + kLongRow);        // [kLongRow]
    __shared__ int32_t s_m;
    __shared__ int64_t s_keep;
    const int64_t row = rows[blockIdx.x];
    const int64_t a = ptr[row], n = ptr[row + 1] - a;
    if (threadIdx.x == 0) s_m = 0;
    __syncthreads();
    int32_t mine = 0;
    for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
        const float v = val[a + e];
        s_a[e] = v != 0.0f ? fabsf(v) : -1.0f;
        s_id[e] = idx[a + e];
        mine += v != 0.0f ? 1 : 0;
    }
    atomicAdd(&s_m, mine);
    __syncthreads();
    const int64_t m = s_m;
    int32_t rk[kLongRow / 256];
    for (int64_t e = threadIdx.x, i = 0; e < n; e += blockDim.x, ++i) {
        int32_t r = INT32_MAX;
        if (s_a[e] >= 0.0f) {
            r = 0;
            for (int64_t f = 0; f < n; ++f) r += before(s_a[f], s_id[f], s_a[e], s_id[e]) ? 1 : 0;
            s_sum[r] = (double)s_a[e];
        }
        rk[i] = r;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        s_keep = mode == SINDI_PRUNE_VNP ? min((int64_t)vn, m) : mass_prefix(s_sum, m, alpha);
    __syncthreads();
    for (int64_t e = threadIdx.x, i = 0; e < n; e += blockDim.x, ++i)
        keep[a + e] = rk[i] < s_keep ? 1 : 0;
}

// One wave per row: every kept entry counts toward list (tile of the row, term);
// the largest stored |x| per term (bits of a non-negative float order like
// the floats) and the storage range check (err bit 32).
__global__ __launch_bounds__(256) void k_count_lists(const int64_t *ptr, const int32_t *idx,
                                                     const float *val, const uint8_t *keep,
                                                     int64_t n_rows, int64_t n_cols,
                                                     const int64_t *tile_doc, int64_t n_tiles,
                                                     int32_t dtype, uint32_t *cnt,
                                                     uint32_t *term_max_bits,
                                                     unsigned long long *n_kept, int32_t *err)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (row >= n_rows) return;
    // tile holding the row: tile_doc[t] <= row < tile_doc[t + 1]
    int64_t lo = 0, hi = n_tiles - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (tile_doc[mid] <= row) lo = mid; else hi = mid - 1;
    }
    uint32_t *c = cnt + (size_t)lo * (size_t)(n_cols + 1);
    const int64_t a = ptr[row], b = ptr[row + 1];
    bool bad = false;
    uint32_t kept = 0;
    for (int64_t e = a + lane; e < b; e += kWave) {
        if (!keep[e]) continue;
        ++kept;
        const int32_t j = idx[e];
        atomicAdd(&c[j], 1u);
        const float v = val[e];
        float sv = v;
        if (dtype == SINDI_F16) {
            if (fabsf(v) > 65504.0f) bad = true;
            sv = (float)__builtin_bit_cast(_Float16, f16_bits(v));
        } else if (dtype == SINDI_BF16) {
            sv = __uint_as_float((uint32_t)bf16_bits(v) << 16);
            if (isinf(sv)) bad = true;
        }
        atomicMax(&term_max_bits[j], __float_as_uint(fabsf(sv)));
    }
    if (__ballot(bad) && lane == 0) atomicOr(err, 32);
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) kept += __shfl_xor(kept, m, kWave);
    if (lane == 0 && kept) atomicAdd(n_kept, (unsigned long long)kept);
}

// One workgroup per tile: group offsets of its lists (exclusive scan of
// ceil(count / 4) over terms), pad counts in the top two bits, the tile's
// group total in goff[n_cols] and tile_groups[t]; err bit 16 if the tile holds
// more than kTileGroupsMax groups.
__global__ __launch_bounds__(256) void k_list_offsets(const uint32_t *cnt, int64_t n_cols,
                                                      uint32_t *goff, int64_t *tile_groups,
                                                      int32_t *err)
{
    __shared__ uint64_t s_part[256];
    __shared__ uint64_t s_base;
    const int64_t t = blockIdx.x;
    const uint32_t *c = cnt + (size_t)t * (size_t)(n_cols + 1);
    uint32_t *g = goff + (size_t)t * (size_t)(n_cols + 1);
    if (threadIdx.x == 0) s_base = 0;
    __syncthreads();
    for (int64_t j0 = 0; j0 < n_cols; j0 += 256) {
        const int64_t j = j0 + threadIdx.x;
        const uint32_t n = j < n_cols ? c[j] : 0u;
        const uint64_t ng = (n + 3u) / 4u;
        s_part[threadIdx.x] = ng;
        __syncthreads();
        for (int d = 1; d < 256; d <<= 1) {  // inclusive scan (Hillis-Steele)
            const uint64_t v = threadIdx.x >= d ? s_part[threadIdx.x - d] : 0ull;
            __syncthreads();
            s_part[threadIdx.x] += v;
            __syncthreads();
        }
        const uint64_t excl = s_base + s_part[threadIdx.x] - ng;
        if (j < n_cols) g[j] = (uint32_t)(excl & kGoffMask) | (((4u - (n & 3u)) & 3u) << 30);
        __syncthreads();
        if (threadIdx.x == 255) s_base += s_part[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        g[n_cols] = (uint32_t)(s_base & kGoffMask);
        tile_groups[t] = (int64_t)s_base;
        if (s_base > kTileGroupsMax) atomicOr(err, 16);
    }
}

// One wave per (tile, pass): the tile's documents in ascending order; each kept
// entry whose term falls in this pass's range takes its list's next slot.  A
// document's terms are distinct, and one wave's LDS operations complete in
// order, so every list receives its documents in ascending order.
__global__ __launch_bounds__(kWave) void k_fill_lists(
    const int64_t *ptr, const int32_t *idx, const float *val, const uint8_t *keep,
    const int64_t *tile_doc, const int64_t *tile_post, const uint32_t *goff, int64_t n_cols,
    int32_t dtype, int32_t pass_terms, uint16_t *post_doc, void *post_val)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *cur = reinterpret_cast<uint32_t *>(smem);  // [pass_terms] next slot of each list
    const int lane = threadIdx.x;
    const int64_t t = blockIdx.x;
    const int64_t j0 = (int64_t)blockIdx.y * pass_terms;
    const int64_t j1 = min(n_cols, j0 + pass_terms);
    if (j0 >= n_cols) return;
    const uint32_t *g = goff + (size_t)t * (size_t)(n_cols + 1);
    for (int64_t j = j0 + lane; j < j1; j += kWave) cur[j - j0] = 4u * (g[j] & kGoffMask);
    wave_sync();
    const int64_t d0 = tile_doc[t], d1 = tile_doc[t + 1], P0 = tile_post[t];
    for (int64_t d = d0; d < d1; ++d) {
        const int64_t a = ptr[d], b = ptr[d + 1];
        const uint16_t doc_off = (uint16_t)((d - d0) * 4);
        for (int64_t e = a + lane; e < b; e += kWave) {
            const int32_t j = idx[e];
            if (!keep[e] || j < j0 || j >= j1) continue;
            const uint32_t slot = cur[j - j0];
            cur[j - j0] = slot + 1u;
            const int64_t pos = P0 + slot;
            post_doc[pos] = doc_off;
            const float v = val[e];
            if (dtype == SINDI_F32) reinterpret_cast<float *>(post_val)[pos] = v;
            else
                reinterpret_cast<uint16_t *>(post_val)[pos] = dtype == SINDI_F16 ? f16_bits(v) : bf16_bits(v);
        }
        wave_sync();
    }
}

// One thread per (tile, term): the pad slots after the list repeat its last
// document (their values were cleared beforehand).
__global__ void k_fill_pads(const uint32_t *goff, const uint32_t *cnt, const int64_t *tile_post,
                            int64_t n_tiles, int64_t n_cols, uint16_t *post_doc)
{
    const int64_t n = n_tiles * n_cols;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = i / n_cols, j = i - t * n_cols;
        const size_t o = (size_t)t * (size_t)(n_cols + 1) + (size_t)j;
        const uint32_t pad = goff[o] >> 30;
        if (!pad) continue;
        const int64_t end = tile_post[t] + 4ll * (goff[o] & kGoffMask) + cnt[o];
        const uint16_t last = post_doc[end - 1];
        for (uint32_t k = 0; k < pad; ++k) post_doc[end + k] = last;
    }
}

template <typename F>
hipError_t set_lds(F *kernel, size_t bytes)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

inline unsigned blocks_for(int64_t threads, int per)
{
    const int64_t b = (threads + per - 1) / per;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

hipError_t build_check_rows(const int64_t *ptr, const int32_t *idx, const float *val,
                            int64_t n_rows, int64_t n_cols, int64_t nnz, int32_t *err,
                            hipStream_t s)
{
    if (n_rows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_rows, dim3(blocks_for(n_rows * kWave, 256)), dim3(256), 0, s, ptr,
                       idx, val, n_rows, n_cols, nnz, err);
    return hipGetLastError();
}

hipError_t build_prune_rows(const int64_t *ptr, const int32_t *idx, const float *val,
                            int64_t n_rows, int32_t mode, double alpha, int32_t vn, uint8_t *keep,
                            int32_t *long_rows, uint32_t *n_long, int32_t *err, hipStream_t s)
{
    if (n_rows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_prune_rows, dim3(blocks_for(n_rows, kRowsPerWg)), dim3(kRowsPerWg * kWave),
                       0, s, ptr, idx, val, n_rows, mode, alpha, vn, keep, long_rows, n_long, err);
    return hipGetLastError();
}

hipError_t build_prune_long(const int64_t *ptr, const int32_t *idx, const float *val,
                            const int32_t *rows, int32_t n_rows, int32_t mode, double alpha,
                            int32_t vn, uint8_t *keep, hipStream_t s)
{
    if (n_rows == 0) return hipSuccess;
    const size_t lds = (size_t)kLongRow * 16;
    hipError_t e = set_lds(k_prune_long, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_prune_long, dim3((unsigned)n_rows), dim3(256), lds, s, ptr, idx, val,
                       rows, mode, alpha, vn, keep);
    return hipGetLastError();
}

hipError_t build_count_lists(const int64_t *ptr, const int32_t *idx, const float *val,
                             const uint8_t *keep, int64_t n_rows, int64_t n_cols,
                             const int64_t *tile_doc, int64_t n_tiles, int32_t dtype,
                             uint32_t *cnt, uint32_t *term_max_bits, unsigned long long *n_kept,
                             int32_t *err, hipStream_t s)
{
    if (n_rows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_lists, dim3(blocks_for(n_rows * kWave, 256)), dim3(256), 0, s, ptr,
                       idx, val, keep, n_rows, n_cols, tile_doc, n_tiles, dtype, cnt,
                       term_max_bits, n_kept, err);
    return hipGetLastError();
}

hipError_t build_list_offsets(const uint32_t *cnt, int64_t n_tiles, int64_t n_cols,
                              uint32_t *goff, int64_t *tile_groups, int32_t *err, hipStream_t s)
{
    if (n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_list_offsets, dim3((unsigned)n_tiles), dim3(256), 0, s, cnt, n_cols,
                       goff, tile_groups, err);
    return hipGetLastError();
}

hipError_t build_fill_lists(const int64_t *ptr, const int32_t *idx, const float *val,
                            const uint8_t *keep, const int64_t *tile_doc, const int64_t *tile_post,
                            const uint32_t *goff, int64_t n_tiles, int64_t n_cols, int32_t dtype,
                            uint16_t *post_doc, void *post_val, hipStream_t s)
{
    if (n_tiles == 0) return hipSuccess;
    const int32_t pass_terms = (int32_t)std::min<int64_t>(n_cols, kFillTerms);
    const int64_t passes = (n_cols + pass_terms - 1) / pass_terms;
    const size_t lds = (size_t)pass_terms * 4;
    hipError_t e = set_lds(k_fill_lists, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fill_lists, dim3((unsigned)n_tiles, (unsigned)passes), dim3(kWave), lds, s,
                       ptr, idx, val, keep, tile_doc, tile_post, goff, n_cols, dtype, pass_terms,
                       post_doc, post_val);
    return hipGetLastError();
}

hipError_t build_fill_pads(const uint32_t *goff, const uint32_t *cnt, const int64_t *tile_post,
                           int64_t n_tiles, int64_t n_cols, uint16_t *post_doc, hipStream_t s)
{
    if (n_tiles == 0) return hipSuccess;
    const int64_t n = n_tiles * n_cols;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_pads, dim3((unsigned)blocks), dim3(256), 0, s, goff, cnt, tile_post,
                       n_tiles, n_cols, post_doc);
    return hipGetLastError();
}

}  // namespace sindi
