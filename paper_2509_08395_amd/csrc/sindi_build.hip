// gfx950 kernels of the index build on the device: the same index as the host
// build (Alg. 3: pruning of every document, then Alg. 1's lists in the tiled,
// 4-posting-aligned layout), bit for bit.
//
//   k_check_rows     structure of a device corpus (Def. 1)
//   k_prune_rows     MRP (Defs. 5-6) or VNP (Sec. 4.1), one wave per row of up
//                    to kWaveRow entries; longer rows are listed for
//   k_prune_long     the same, one workgroup per row of up to kLongRow entries
//   k_count_lists    entries per (tile, term) list (one workgroup per tile,
//                    counters in LDS), the storage range check and each
//                    term's largest stored |x|
//   k_list_offsets   per tile: 4-posting group offsets of the lists, pad counts
//   k_fill_lists     one wave per (tile, term pass) streams the tile's entries
//                    in order and places every kept entry of its terms at its
//                    list's cursor (LDS), so a list holds its documents in
//                    ascending order
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
constexpr int kCountThreads = 1024;  // k_count_lists workgroup
constexpr int kCountTerms = 32768;   // 16-bit list counters per pass of k_count_lists (64 KB)
constexpr int kFillRing = 8;         // chunks of 64 entries in flight per k_fill_lists wave

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
// alpha times the mass (the same sum over all m); alpha = 1 keeps all.  The
// sums run strictly in order; LDS reads go eight at a time (padding with +0.0,
// which leaves a non-negative sum unchanged).
__device__ int64_t mass_prefix(const double *s, int64_t m, double alpha)
{
    if (alpha >= 1.0) return m;
    double mass = 0.0;
    for (int64_t t = 0; t < m; t += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = t + u < m ? s[t + u] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) mass += v[u];
    }
    const double thr = alpha * mass;
    double run = 0.0;
    for (int64_t t = 0; t < m; t += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = t + u < m ? s[t + u] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (t + u >= m) break;
            run += v[u];
            if (run >= thr) return t + u + 1;
        }
    }
    return m;
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

// Def. 6 order as one unsigned 64-bit key: |x| bits (a positive finite float
// orders like its bits) above the complemented term id, so a larger key comes
// first; non-entries (zeros, slots past the row) have key 0, after every entry.
__device__ __forceinline__ uint64_t order_key(float ax, int32_t id)
{
    return ax > 0.0f ? ((uint64_t)__float_as_uint(ax) << 32) | (uint32_t)~id : 0ull;
}

// Ranks of a wave's row held in registers (key of entry i * 64 + lane in slot
// i of the lane, NC slots in use): for each slot, the number of the row's
// entries with a larger key, taking the keys one at a time by lane broadcast.
template <int NC, int PER>
__device__ __forceinline__ void rank_entries(const uint64_t (&key)[PER], int32_t (&rank)[PER])
{
#pragma unroll
    for (int i = 0; i < PER; ++i) rank[i] = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const uint32_t lo = (uint32_t)key[c], hi = (uint32_t)(key[c] >> 32);
        for (int l = 0; l < kWave; ++l) {
            const uint64_t f = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)hi, l) << 32) |
                               (uint32_t)__builtin_amdgcn_readlane((int)lo, l);
#pragma unroll
            for (int i = 0; i < NC; ++i) rank[i] += f > key[i] ? 1 : 0;
        }
    }
}

// One wave per row of at most kWaveRow entries, held in registers (entry
// i * 64 + lane in slot i of the lane).  Each lane ranks its entries by
// counting the row's entries before them in Def. 6 order (rank_entries); MRP
// places |x| at its rank (FP64, in LDS) and the prefix sums run in that order.  Longer rows are appended to
// long_rows (err bit 128: a row longer than kLongRow).
__global__ __launch_bounds__(kRowsPerWg * kWave) void k_prune_rows(
    const int64_t *ptr, const int32_t *idx, const float *val, int64_t n_rows, int32_t mode,
    double alpha, int32_t vn, uint8_t *keep, int32_t *long_rows, uint32_t *n_long, int32_t *err)
{
    constexpr int PER = kWaveRow / kWave;
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
    // non-entries (zeros, slots past the row) carry |x| = -1 and key 0
    float ax[PER];
    uint64_t key[PER];
    int32_t m = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int64_t e = i * kWave + lane;
        ax[i] = -1.0f;
        int32_t id = 0;
        if (e < n) {
            const float v = val[a + e];
            ax[i] = v != 0.0f ? fabsf(v) : -1.0f;  // zeros are not entries (Def. 1)
            id = idx[a + e];
        }
        key[i] = order_key(ax[i], id);
        m += __popcll(__ballot(ax[i] >= 0.0f));
    }
    int32_t rank[PER];
    switch ((n + kWave - 1) / kWave) {  // slots in use (wave-uniform)
    case 0: break;
    case 1: rank_entries<1>(key, rank); break;
    case 2: rank_entries<2>(key, rank); break;
    case 3: rank_entries<3>(key, rank); break;
    case 4: rank_entries<4>(key, rank); break;
    case 5: rank_entries<5>(key, rank); break;
    case 6: rank_entries<6>(key, rank); break;
    case 7: rank_entries<7>(key, rank); break;
    default: rank_entries<8>(key, rank); break;
    }
#pragma unroll
    for (int i = 0; i < PER; ++i)
        if (ax[i] < 0.0f) rank[i] = INT32_MAX;
    int64_t keep_n;
    if (mode == SINDI_PRUNE_VNP) {
        keep_n = min((int64_t)vn, (int64_t)m);
    } else {
#pragma unroll
        for (int i = 0; i < PER; ++i)
            if (ax[i] >= 0.0f) s_sum[w][rank[i]] = (double)ax[i];
        wave_sync();
        keep_n = mass_prefix(s_sum[w], m, alpha);  // the same value in every lane
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

// One workgroup per (tile, pass of pass_terms terms): the tile's entries are
// contiguous in the corpus, so the workgroup streams them and counts every
// kept entry of the pass's terms in LDS, two 16-bit counters per word (a list
// of a tile holds at most kTileMax < 2^16 entries), then writes the counts.
// Also the largest stored |x| per term (bits of a non-negative float order like
// the floats; the atomic only where the value read is smaller), the kept total
// and the storage range check (err bit 32).
__global__ __launch_bounds__(kCountThreads) void k_count_lists(
    const int64_t *ptr, const int32_t *idx, const float *val, const uint8_t *keep,
    int64_t n_cols, const int64_t *tile_doc, int32_t dtype, int32_t pass_terms, int64_t passes,
    uint32_t *cnt, uint32_t *term_max_bits, unsigned long long *n_kept, int32_t *err)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *c16 = reinterpret_cast<uint32_t *>(smem);  // [(pass_terms + 1) / 2]
    __shared__ unsigned long long s_kept;
    __shared__ int32_t s_bad;
    const int64_t t = blockIdx.x;
    const int64_t e0 = ptr[tile_doc[t]], e1 = ptr[tile_doc[t + 1]];
    uint32_t *c = cnt + (size_t)t * (size_t)(n_cols + 1);
    const int lane = threadIdx.x & (kWave - 1);
    for (int64_t pass = blockIdx.y; pass < passes; pass += gridDim.y) {
        const int64_t j0 = pass * pass_terms, j1 = min(n_cols, j0 + pass_terms);
        const int32_t nw = (int32_t)((j1 - j0 + 1) / 2);
        for (int32_t i = threadIdx.x; i < nw; i += blockDim.x) c16[i] = 0u;
        if (threadIdx.x == 0) {
            s_kept = 0ull;
            s_bad = 0;
        }
        __syncthreads();
        uint32_t kept = 0;
        bool bad = false;
        for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
            if (!keep[e]) continue;
            const int32_t j = idx[e];
            if (j < j0 || j >= j1) continue;
            ++kept;
            const uint32_t r = (uint32_t)(j - j0);
            atomicAdd(&c16[r >> 1], (r & 1u) ? 0x10000u : 1u);
            const float v = val[e];
            float sv = v;
            if (dtype == SINDI_F16) {
                if (fabsf(v) > 65504.0f) bad = true;
                sv = (float)__builtin_bit_cast(_Float16, f16_bits(v));
            } else if (dtype == SINDI_BF16) {
                sv = __uint_as_float((uint32_t)bf16_bits(v) << 16);
                if (isinf(sv)) bad = true;
            }
            const uint32_t bits = __float_as_uint(fabsf(sv));
            if (bits > term_max_bits[j]) atomicMax(&term_max_bits[j], bits);
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) kept += __shfl_xor(kept, d, kWave);
        if (lane == 0 && kept) atomicAdd(&s_kept, (unsigned long long)kept);
        if (__ballot(bad) && lane == 0) s_bad = 1;
        __syncthreads();
        for (int64_t i = threadIdx.x; i < j1 - j0; i += blockDim.x)
            c[j0 + i] = (c16[i >> 1] >> ((i & 1) * 16)) & 0xFFFFu;
        if (threadIdx.x == 0) {
            if (s_kept) atomicAdd(n_kept, s_kept);
            if (s_bad) atomicOr(err, 32);
        }
        __syncthreads();
    }
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

// One wave per (tile, pass of pass_terms terms).  The tile's entries are
// contiguous in the corpus; the wave streams them in chunks of 64 (one per
// lane), with kFillRing chunks' loads in flight.  The lanes of a chunk belong
// to consecutive documents (found from the row pointers, wave-uniform scalar
// loads); the chunk is placed one document at a time, each kept entry of the
// pass's terms taking its list's next slot by an LDS atomic.  A document's
// terms are distinct and one wave's LDS operations complete in order, so every
// list receives its documents in ascending order.
__global__ __launch_bounds__(kWave) void k_fill_lists(
    const int64_t *ptr, const int32_t *idx, const float *val, const uint8_t *keep,
    const int64_t *tile_doc, const int64_t *tile_post, const uint32_t *goff, int64_t n_cols,
    int32_t dtype, int32_t pass_terms, uint16_t *post_doc, void *post_val)
{
    constexpr int R = kFillRing;
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
    const int64_t e0 = ptr[d0], e1 = ptr[d1];
    int32_t rj[R];
    uint32_t rk[R];
    float rv[R];
    auto fetch = [&](int64_t c, int u) {  // chunk starting at entry c into ring slot u
        const int64_t e = c + lane;
        rj[u] = -1;
        rk[u] = 0u;
        rv[u] = 0.0f;
        if (e < e1) {
            rj[u] = idx[e];
            rk[u] = keep[e];
            rv[u] = val[e];
        }
    };
#pragma unroll
    for (int u = 0; u < R; ++u) fetch(e0 + (int64_t)u * kWave, u);
    int64_t dcur = d0;  // document of the current chunk's first entry
    for (int64_t c0 = e0; c0 < e1; c0 += (int64_t)R * kWave) {
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int64_t c = c0 + (int64_t)u * kWave;
            if (c < e1) {  // wave-uniform
                const int64_t e = c + lane, cend = min(c + kWave, e1);
                while (ptr[dcur + 1] <= c) ++dcur;  // skip ended and empty documents
                // lane e belongs to the last document dd with ptr[dd] <= e
                int64_t mine = dcur, dd = dcur, bnd = ptr[dcur + 1];
                while (bnd < cend) {
                    ++dd;
                    if (e >= bnd) mine = dd;
                    bnd = ptr[dd + 1];
                }
                const int32_t j = rj[u];
                const bool act0 = e < e1 && rk[u] != 0u && j >= j0 && j < j1;
                for (int64_t gd = dcur; gd <= dd; ++gd) {
                    if (act0 && mine == gd) {
                        const uint32_t slot = atomicAdd(&cur[j - j0], 1u);
                        const int64_t pos = P0 + slot;
                        post_doc[pos] = (uint16_t)((gd - d0) * 4);
                        const float v = rv[u];
                        if (dtype == SINDI_F32) reinterpret_cast<float *>(post_val)[pos] = v;
                        else
                            reinterpret_cast<uint16_t *>(post_val)[pos] =
                                dtype == SINDI_F16 ? f16_bits(v) : bf16_bits(v);
                    }
                    wave_sync();
                }
                dcur = dd;
            }
            fetch(c + (int64_t)R * kWave, u);
        }
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
    return allow_lds(reinterpret_cast<const void *>(kernel), bytes);
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
    if (n_rows == 0 || n_tiles == 0) return hipSuccess;
    const int32_t pass_terms = (int32_t)std::min<int64_t>(n_cols, kCountTerms);
    const int64_t passes = (n_cols + pass_terms - 1) / pass_terms;
    const size_t lds = (size_t)(pass_terms + 1) / 2 * 4;
    hipError_t e = set_lds(k_count_lists, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_count_lists, dim3((unsigned)n_tiles, (unsigned)std::min<int64_t>(passes, 65535)),
                       dim3(kCountThreads), lds, s, ptr, idx, val, keep, n_cols, tile_doc, dtype,
                       pass_terms, passes, cnt, term_max_bits, n_kept, err);
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
    // at most kFillTerms list cursors per wave; each pass streams the tile once
    const int64_t passes = std::min<int64_t>(65535, (n_cols + kFillTerms - 1) / kFillTerms);
    const int32_t pass_terms = (int32_t)((n_cols + passes - 1) / passes);
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
