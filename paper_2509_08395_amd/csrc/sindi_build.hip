// gfx950 kernels of the index build on the device: the same index as the host
// build (Alg. 3: pruning of every document, then Alg. 1's lists in the tiled,
// 4-posting-aligned layout), bit for bit.
//
//   k_check_rows     structure of a device corpus (Def. 1)
//   k_prune_rows     MRP (Defs. 5-6) or VNP (Sec. 4.1), one wave per row of up
//                    to kWaveRow entries sorted in registers (bitonic); longer
//                    rows are listed for
//   k_prune_long     the same, one workgroup per row of up to kLongRow entries
//   k_count_lists    entries per (tile, term) list (one workgroup per tile,
//                    counters in LDS), the storage range check and each
//                    term's largest stored |x|
//   k_list_offsets   per tile: 4-posting group offsets of the lists, pad counts
//   k_fill_lists     one workgroup per (tile, term pass) places the tile's
//                    kept entries of its terms, 16 documents at a time, each
//                    at its list's next slot plus its rank among the batch's
//                    documents holding the term (LDS), so a list holds its
//                    documents in ascending order
//   k_fill_pads      the pad entries after every list
//   k_deal_chunks    reorders every chunk of a list (kChunk groups, one per lane
//                    of a scoring wave) of two or more groups so that the adds
//                    of one scoring instruction fall in distinct LDS banks
//                    where the chunk allows (the sums do not depend on the order)
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
constexpr int kCheckRows = 16;    // rows per wave of k_check_rows
constexpr int kCountThreads = 1024;  // k_count_lists workgroup
constexpr int kCountTerms = 32768;   // 16-bit list counters per pass of k_count_lists (64 KB)
constexpr int kFillThreads = 1024;   // k_fill_lists workgroup
constexpr int kFillDocs = 16;        // documents placed together by k_fill_lists (one bit each)
constexpr int kFillPer = 2;          // entries per thread and batch of k_fill_lists
constexpr int64_t kFillCap = (int64_t)kFillThreads * kFillPer;  // entries per batch
constexpr int kDealThreads = 256;    // k_deal_chunks workgroup (one list per wave at a time)
constexpr int kLdsBanks = 32;        // words of one 32-lane LDS pass in distinct classes mod 32
                                     // fall in distinct banks (the LDS has 64 banks)

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
// One wave per kCheckRows consecutive rows: their row pointers one per lane,
// then the rows' entries swept as one range (an entry is the last of its row
// where the next one starts a row).  Entries are read only when every pointer
// of the wave's rows is in order and within the arrays.
__global__ __launch_bounds__(256) void k_check_rows(const int64_t *ptr, const int32_t *idx,
                                                    const float *val, int64_t n_rows,
                                                    int64_t n_cols, int64_t nnz, int32_t *err)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t r0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave * kCheckRows;
    if (r0 >= n_rows) return;
    const int nr = (int)min((int64_t)kCheckRows, n_rows - r0);
    const int64_t p = lane <= nr ? ptr[r0 + lane] : 0;
    const int64_t pn = __shfl_down(p, 1, kWave);
    int bad = 0;
    if (lane < nr && (p < 0 || pn < p || pn > nnz)) bad |= 1;
    if (lane == 0 && r0 == 0 && p != 0) bad |= 1;
    if (lane == nr && r0 + nr == n_rows && p != nnz) bad |= 1;
    if (__ballot(bad != 0)) {
        if (bad) atomicOr(err, bad);
        return;
    }
    __shared__ int64_t s_b[4][kCheckRows + 1];  // the row starts, per wave of the workgroup
    int64_t *rb = s_b[threadIdx.x / kWave];
    if (lane <= nr) rb[lane] = p;
    wave_sync();
    const int64_t ea = rb[0], eb = rb[nr];
    int k = 0;  // the row of the lane's current entry (entries rise through the sweep)
    for (int64_t e0 = ea + lane; e0 < eb; e0 += 4 * kWave) {
        int32_t id[4], nx[4];
        float v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t e = e0 + (int64_t)u * kWave;
            id[u] = 0;
            nx[u] = INT32_MAX;
            v[u] = 0.0f;
            if (e < eb) {
                id[u] = idx[e];
                v[u] = val[e];
                if (e + 1 < eb) nx[u] = idx[e + 1];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t e = e0 + (int64_t)u * kWave;
            if (e >= eb) continue;
            if (id[u] < 0 || id[u] >= n_cols) bad |= 2;
            if (!isfinite(v[u])) bad |= 8;
            while (rb[k + 1] <= e) ++k;  // rb[nr] = eb > e ends it
            if (rb[k + 1] != e + 1 && nx[u] <= id[u]) bad |= 4;  // e is not its row's last
        }
    }
    if (bad) atomicOr(err, bad);  // rare: every lane that found a fault
}

// Def. 6 order as one unsigned 64-bit key: |x| bits (a positive finite float
// orders like its bits) above the complemented term id, so a larger key comes
// first; non-entries (zeros, slots past the row) have key 0, after every entry.
__device__ __forceinline__ uint64_t order_key(float ax, int32_t id)
{
    return ax > 0.0f ? ((uint64_t)__float_as_uint(ax) << 32) | (uint32_t)~id : 0ull;
}

// The value of lane (lane ^ X) for X < 64, all lanes active: quad permutations
// for 1 and 2, a quad mirror then a half-row mirror for 4 (lane ^ 3 ^ 7), a
// half-row rotation for 8 (DPP, no LDS traffic); a permute through the LDS
// crossbar for 16 and 32.
template <int X>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v)
{
    const int x = (int)v;
    if constexpr (X == 1) return (uint32_t)__builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);
    else if constexpr (X == 2) return (uint32_t)__builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);
    else if constexpr (X == 4)
        return (uint32_t)__builtin_amdgcn_update_dpp(
            0, __builtin_amdgcn_update_dpp(0, x, 0x1B, 0xF, 0xF, false), 0x141, 0xF, 0xF, false);
    else if constexpr (X == 8) return (uint32_t)__builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false);
    else return (uint32_t)__shfl_xor(x, X, kWave);
}

template <int X>
__device__ __forceinline__ uint64_t lane_xor64(uint64_t v)
{
    return ((uint64_t)lane_xor<X>((uint32_t)(v >> 32)) << 32) | lane_xor<X>((uint32_t)v);
}

// One merge step (blocks of K, distance J) of a bitonic sort of the N = 64 S
// keys a wave holds, element i = lane * S + s in slot s of the lane: elements
// i and i ^ J are compared in registers for J < S and across lanes otherwise;
// the lower element of a pair takes the larger key where i & K is 0 and the
// smaller elsewhere, so the last merge (K = N) leaves the keys in descending
// order.  Equal keys are interchangeable.
template <int S, int K, int J>
__device__ __forceinline__ void bitonic_step(uint64_t (&key)[S], int lane)
{
    if constexpr (J < S) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (s & J) continue;  // s is the pair's lower slot
            const bool larger_low = (((lane * S) | s) & K) == 0;
            const uint64_t a = key[s], b = key[s | J];
            const bool a_first = (a > b) == larger_low;
            key[s] = a_first ? a : b;
            key[s | J] = a_first ? b : a;
        }
    } else {
        constexpr int X = J / S;  // partner lane: lane ^ X
        const bool take_max = ((lane & X) == 0) == (((lane * S) & K) == 0);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const uint64_t a = key[s], p = lane_xor64<X>(a);
            key[s] = (a > p) == take_max ? a : p;
        }
    }
}

template <int S, int K, int J>
__device__ __forceinline__ void bitonic_merge(uint64_t (&key)[S], int lane)
{
    bitonic_step<S, K, J>(key, lane);
    if constexpr (J > 1) bitonic_merge<S, K, J / 2>(key, lane);
}

template <int S, int K = 2>
__device__ __forceinline__ void bitonic_desc(uint64_t (&key)[S], int lane)
{
    bitonic_merge<S, K, K / 2>(key, lane);
    if constexpr (K < S * kWave) bitonic_desc<S, K * 2>(key, lane);
}

// Key of rank r (0 <= r < 64 S) of keys sorted by bitonic_desc, in every lane.
template <int S>
__device__ __forceinline__ uint64_t key_at(const uint64_t (&key)[S], int32_t r)
{
    uint64_t v = key[0];
#pragma unroll
    for (int s = 1; s < S; ++s)
        if (r % S == s) v = key[s];
    const int l = r / S;
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
}

// FP64 lane shifted down by D within rows of 16 lanes (0.0 shifted in).
template <int D>
__device__ __forceinline__ double row_shr(double v)
{
    const uint64_t b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, 0x110 + D, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), 0x110 + D, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Alg. 3 on one row of m entries (n slots read) held by a wave, S slots per
// lane: the keys sorted in Def. 6 order give every entry's rank, and the row
// keeps the entries of rank below keep_n, i.e. the keys at or above the key of
// rank keep_n - 1.  MRP's keep_n comes from the prefix sums of |x| in that
// order, taken in FP64 one after another (mass_prefix, as the host does), or,
// where the row's values make every such sum exact, by a scan: all |x| are
// integer multiples of the smallest one's unit in the last place, u, and when
// m times the largest stays below 2^53 u no partial sum, in any order of
// addition, is rounded, so the scan's sums are the sequential ones.
template <int S>
__device__ __forceinline__ void prune_row(const int32_t *ridx, const float *rval, int64_t n,
                                          int32_t mode, double alpha, int32_t vn, uint8_t *rkeep,
                                          double *s_sum)
{
    const int lane = threadIdx.x & (kWave - 1);
    uint64_t key[S], orig[S];
    int32_t m = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) {  // entry s * 64 + lane; a sort needs no particular start
        const int64_t e = s * kWave + lane;
        float ax = -1.0f;
        int32_t id = 0;
        if (e < n) {
            const float v = rval[e];
            ax = v != 0.0f ? fabsf(v) : -1.0f;  // zeros are not entries (Def. 1)
            id = ridx[e];
        }
        key[s] = orig[s] = order_key(ax, id);
        m += __popcll(__ballot(ax >= 0.0f));
    }
    bitonic_desc<S>(key, lane);  // rank lane * S + s in slot s
    int32_t keep_n = m;
    if (mode == SINDI_PRUNE_VNP) {
        keep_n = min(vn, m);
    } else if (alpha < 1.0 && m > 0) {
        const int e_max = max((int)(key_at<S>(key, 0) >> 55), 1);
        const int e_min = max((int)(key_at<S>(key, m - 1) >> 55), 1);
        const int lg = m > 1 ? 32 - __clz(m - 1) : 0;  // ceil(log2 m)
        if (e_max - e_min + lg <= 29) {
            double pre[S];
            double run = 0.0;
#pragma unroll
            for (int s = 0; s < S; ++s) {  // the lane's own ranks
                run += key[s] ? (double)__uint_as_float((uint32_t)(key[s] >> 32)) : 0.0;
                pre[s] = run;
            }
            // lanes' totals: inclusive scan in rows of 16, then the rows below
            double x = run;
            x += row_shr<1>(x);
            x += row_shr<2>(x);
            x += row_shr<4>(x);
            x += row_shr<8>(x);
            const double r0 = __shfl(x, 15, kWave), r1 = __shfl(x, 31, kWave), r2 = __shfl(x, 47, kWave);
            x += (lane >= 16 ? r0 : 0.0) + (lane >= 32 ? r1 : 0.0) + (lane >= 48 ? r2 : 0.0);
            const double before = x - run;  // exact: the lanes below this one
            const double mass = __shfl(x, kWave - 1, kWave);
            const double thr = alpha * mass;
            int first = S;  // the lane's first rank reaching thr
#pragma unroll
            for (int s = S - 1; s >= 0; --s)
                if (before + pre[s] >= thr && lane * S + s < m) first = s;
            const uint64_t hit = __ballot(first < S);
            if (hit) {
                const int l = __ffsll((long long)hit) - 1;
                keep_n = l * S + __builtin_amdgcn_readlane(first, l) + 1;
            }
        } else {
#pragma unroll
            for (int s = 0; s < S; ++s)
                if (lane * S + s < m) s_sum[lane * S + s] = (double)__uint_as_float((uint32_t)(key[s] >> 32));
            wave_sync();
            keep_n = (int32_t)mass_prefix(s_sum, m, alpha);  // the same value in every lane
        }
    }
    const uint64_t kth = keep_n > 0 ? key_at<S>(key, keep_n - 1) : ~0ull;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int64_t e = s * kWave + lane;
        if (e < n) rkeep[e] = orig[s] != 0ull && orig[s] >= kth ? 1 : 0;
    }
}

// One wave per row of at most kWaveRow entries, held in registers (entry
// s * 64 + lane in slot s of the lane; slots in use rounded up to a power of
// two).  Longer rows are appended to long_rows (err bit 128: a row longer than
// kLongRow).
__global__ __launch_bounds__(kRowsPerWg * kWave) void k_prune_rows(
    const int64_t *ptr, const int32_t *idx, const float *val, int64_t n_rows, int32_t mode,
    double alpha, int32_t vn, uint8_t *keep, int32_t *long_rows, uint32_t *n_long, int32_t *err)
{
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
    const int32_t *ri = idx + a;
    const float *rv = val + a;
    uint8_t *rk = keep + a;
    if (n <= kWave) prune_row<1>(ri, rv, n, mode, alpha, vn, rk, s_sum[w]);
    else if (n <= 2 * kWave) prune_row<2>(ri, rv, n, mode, alpha, vn, rk, s_sum[w]);
    else if (n <= 4 * kWave) prune_row<4>(ri, rv, n, mode, alpha, vn, rk, s_sum[w]);
    else prune_row<8>(ri, rv, n, mode, alpha, vn, rk, s_sum[w]);
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
        // four entries per thread at once: their loads, then the maxima read so far (a
        // stale value only lets an atomic through), then the counts and updates
        constexpr int U = 4;
        for (int64_t base = e0 + threadIdx.x; base < e1; base += (int64_t)blockDim.x * U) {
            int32_t jv[U];
            float vv[U];
            uint32_t kv[U], tm[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {  // unconditional: the lines are read either way
                const int64_t e = base + (int64_t)u * blockDim.x;
                jv[u] = -1;
                vv[u] = 0.0f;
                kv[u] = 0u;
                if (e < e1) {
                    kv[u] = keep[e];
                    jv[u] = idx[e];
                    vv[u] = val[e];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (!kv[u] || jv[u] < j0 || jv[u] >= j1) jv[u] = -1;
                tm[u] = jv[u] >= 0 ? term_max_bits[jv[u]] : 0u;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t j = jv[u];
                if (j < 0) continue;
                ++kept;
                const uint32_t r = (uint32_t)(j - j0);
                atomicAdd(&c16[r >> 1], (r & 1u) ? 0x10000u : 1u);
                const float v = vv[u];
                float sv = v;
                if (dtype == SINDI_F16) {
                    if (fabsf(v) > 65504.0f) bad = true;
                    sv = (float)__builtin_bit_cast(_Float16, f16_bits(v));
                } else if (dtype == SINDI_BF16) {
                    sv = __uint_as_float((uint32_t)bf16_bits(v) << 16);
                    if (isinf(sv)) bad = true;
                }
                const uint32_t bits = __float_as_uint(fabsf(sv));
                if (bits > tm[u]) atomicMax(&term_max_bits[j], bits);
            }
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

// One workgroup per (tile, pass of pass_terms terms) places the tile's kept
// entries of the pass's terms in their lists, each list holding its documents
// in ascending order (Alg. 1).  The documents are taken in batches: up to
// kFillDocs whole documents of at most kFillCap entries together, or a longer
// document alone, kFillCap entries at a time.  One LDS word per term holds the
// list's next slot (low 16 bits, from the list's start: a list of a tile holds
// at most kTileMax < 2^16 entries) and, while a batch is placed, one bit per
// document of the batch that holds the term (high 16 bits).  Per batch: every
// kept entry adds its document's bit; after a barrier it takes the slot the
// word gives plus the number of the batch's earlier documents holding the
// term; the entry of the last such document then adds to the word the count
// less the bits, which leaves the next slot with no bits set.  A document holds
// a term at most once, so a list's slots follow its documents' order, as in a
// one-document-at-a-time placement.  Additions commute, so each batch's slot
// advances go with the next batch's bits, two barriers per batch.  The next
// batch's entries (at most kFillCap from its first) and their lists' offsets
// are loaded while the current batch is placed.
__global__ __launch_bounds__(kFillThreads) void k_fill_lists(
    const int64_t *ptr, const int32_t *idx, const float *val, const uint8_t *keep,
    const int64_t *tile_doc, const int64_t *tile_post, const uint32_t *goff, int64_t n_cols,
    int32_t dtype, int32_t pass_terms, uint16_t *post_doc, void *post_val)
{
    constexpr int P = kFillPer;
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *word = reinterpret_cast<uint32_t *>(smem);  // [pass_terms]
    __shared__ int64_t s_bnd[2][kFillDocs + 1];           // first entries of the batch's documents
    const int tid = threadIdx.x;
    const int64_t t = blockIdx.x;
    const int64_t j0 = (int64_t)blockIdx.y * pass_terms;
    const int64_t j1 = min(n_cols, j0 + pass_terms);
    if (j0 >= n_cols) return;  // the whole workgroup
    const uint32_t *g = goff + (size_t)t * (size_t)(n_cols + 1);
    for (int64_t j = tid; j < j1 - j0; j += kFillThreads) word[j] = 0u;
    const int64_t d0 = tile_doc[t], d1 = tile_doc[t + 1], P0 = tile_post[t];
    const int64_t e1 = ptr[d1];
    int64_t d = d0, e = ptr[d0];
    int buf = 0;
    if (tid <= kFillDocs) s_bnd[0][tid] = ptr[min(d + tid, d1)];
    int32_t rj[P], nj[P];  // this batch's entries, and the next batch's (in flight)
    uint32_t rk[P], nk[P];
    float rv[P], nv[P];
    uint32_t go[P];                  // list offsets of this batch's entries
    int32_t up_j[P];                 // a slot advance of the last batch: term (or -1) ...
    uint32_t up_d[P];                // ... and the amount added to its word
    auto fetch = [&](int64_t from, int32_t (&fj)[P], uint32_t (&fk)[P], float (&fv)[P]) {
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const int64_t x = from + tid + (int64_t)u * kFillThreads;
            fj[u] = -1;
            fk[u] = 0u;
            fv[u] = 0.0f;
            if (x < e1) {
                fj[u] = idx[x];
                fk[u] = keep[x];
                fv[u] = val[x];
            }
        }
    };
    // list offsets of the entries fetched (some past their batch's end: unused)
    auto offsets = [&](const int32_t (&fj)[P], const uint32_t (&fk)[P]) {
#pragma unroll
        for (int u = 0; u < P; ++u) go[u] = fk[u] != 0u && fj[u] >= j0 && fj[u] < j1 ? g[fj[u]] : 0u;
    };
    fetch(e, rj, rk, rv);
    offsets(rj, rk);
#pragma unroll
    for (int u = 0; u < P; ++u) up_j[u] = -1;
    __syncthreads();
    while (e < e1) {
        const int64_t *bnd = s_bnd[buf];
        // documents d .. d + nb - 1 whole (entries [e, eb)), or part of document d (nb = 0)
        int nb = 0;
#pragma unroll
        for (int k = 1; k <= kFillDocs; ++k)
            if (nb == k - 1 && d + k <= d1 && bnd[k] - e <= kFillCap) nb = k;
        const int64_t eb = nb ? bnd[nb] : e + kFillCap;
        const int64_t dn = nb ? d + nb : d;
        int64_t pnext = 0;  // the next batch's row pointers, stored after this phase
        if (tid <= kFillDocs) pnext = ptr[min(dn + tid, d1)];
        fetch(eb, nj, nk, nv);
        int32_t jj[P];
        uint32_t bit[P];
#pragma unroll
        for (int u = 0; u < P; ++u) {
            if (up_j[u] >= 0) atomicAdd(&word[up_j[u] - j0], up_d[u]);
            const int64_t x = e + tid + (int64_t)u * kFillThreads;
            jj[u] = -1;
            bit[u] = 0;
            if (x < eb && rk[u] != 0u && rj[u] >= j0 && rj[u] < j1) {
                int b = 0;  // the entry's document in the batch
#pragma unroll
                for (int k = 1; k < kFillDocs; ++k) b += (k < nb && bnd[k] <= x) ? 1 : 0;
                jj[u] = rj[u];
                bit[u] = (uint32_t)b;
                atomicAdd(&word[rj[u] - j0], 1u << (16 + b));
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < P; ++u) {
            up_j[u] = -1;
            if (jj[u] < 0) continue;
            const uint32_t wd = word[jj[u] - j0];
            const uint32_t bits = wd >> 16;
            const uint32_t slot = (wd & 0xFFFFu) + (uint32_t)__popc(bits & ((1u << bit[u]) - 1u));
            const int64_t pos = P0 + 4ll * (int64_t)(go[u] & kGoffMask) + slot;
            post_doc[pos] = (uint16_t)((d + bit[u] - d0) * 4);
            const float v = rv[u];
            if (dtype == SINDI_F32) reinterpret_cast<float *>(post_val)[pos] = v;
            else
                reinterpret_cast<uint16_t *>(post_val)[pos] = dtype == SINDI_F16 ? f16_bits(v) : bf16_bits(v);
            if ((bits >> (bit[u] + 1)) == 0u) {  // the batch's last document holding the term
                up_j[u] = jj[u];
                up_d[u] = (uint32_t)__popc(bits) - (bits << 16);
            }
        }
        if (tid <= kFillDocs) s_bnd[buf ^ 1][tid] = pnext;
        offsets(nj, nk);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < P; ++u) {
            rj[u] = nj[u];
            rk[u] = nk[u];
            rv[u] = nv[u];
        }
        d = dn;
        e = eb;
        buf ^= 1;
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

// The scoring kernels hand a list chunk of c <= kChunk groups to the lanes of one wave, group
// i to lane i, and add posting p of every lane's group with one LDS instruction, which the LDS
// serves 32 lanes at a time: posting 4 i + p of the chunk lands in "bin" (p, i / 32), and the
// adds of a bin that hit the same bank are served one after another.  Score words in distinct
// classes mod 32 never share a bank.
// Each chunk of n real postings, ascending by document on entry, is reordered here: its
// postings taken by (bank, document) fill, in that order, positions 4 (32 h + r) + p for
// r = 0..31, h = 0..1, p = 0..3 (those below n), so postings of one bank go to successive bins
// and a bin holds ceil(count / bins) of them at most.  A chunk of one group (one lane) keeps its
// order, and pads stay at the list's end.  A wave takes 64 consecutive lists of tile blockIdx.x
// at a time (their offsets loaded together, a list per lane; the grid's columns stride over the
// vocabulary) and reorders those of two or more groups one after another.
__global__ __launch_bounds__(kDealThreads) void k_deal_chunks(const uint32_t *goff,
                                                              const int64_t *tile_post,
                                                              int64_t n_cols, int32_t vbytes,
                                                              uint16_t *post_doc, void *post_val)
{
    constexpr int NW = kDealThreads / kWave;
    __shared__ uint32_t s_doc[NW][4 * kChunk], s_val[NW][4 * kChunk];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t t = blockIdx.x;
    const int r = lane & 31, h = lane >> 5;
    const int64_t tile_first = tile_post[t];
    const int64_t stride = (int64_t)gridDim.y * NW * kWave;
    for (int64_t j0 = ((int64_t)blockIdx.y * NW + w) * kWave; j0 < n_cols; j0 += stride) {
        uint32_t gs_l = 0, pad_l = 0, ng_l = 0;
        if (j0 + lane < n_cols) {
            const size_t o = (size_t)t * (size_t)(n_cols + 1) + (size_t)(j0 + lane);
            const uint32_t g = goff[o];
            gs_l = g & kGoffMask;
            pad_l = g >> 30;
            ng_l = (goff[o + 1] & kGoffMask) - gs_l;
        }
        for (uint64_t todo = __ballot(ng_l > 1); todo; todo &= todo - 1) {
            const int li = __builtin_ctzll(todo);
            const uint32_t gs = (uint32_t)__builtin_amdgcn_readlane((int)gs_l, li);
            const uint32_t pad = (uint32_t)__builtin_amdgcn_readlane((int)pad_l, li);
            const uint32_t ng = (uint32_t)__builtin_amdgcn_readlane((int)ng_l, li);
            const int64_t base = tile_first + 4 * (int64_t)gs;  // the list's first slot
            for (uint32_t c0 = 0; c0 < ng; c0 += kChunk) {
                const uint32_t cg = min(ng - c0, (uint32_t)kChunk);
                if (cg == 1) break;  // the last chunk, one lane: nothing to spread
                const uint32_t n = 4 * cg - (c0 + cg == ng ? pad : 0u);
                const int64_t slot = base + 4 * (int64_t)(c0 + (uint32_t)lane);
                uint2 dw = make_uint2(0u, 0u);
                uint4 vw = make_uint4(0u, 0u, 0u, 0u);
                if ((uint32_t)lane < cg) {
                    dw = *reinterpret_cast<const uint2 *>(post_doc + slot);
                    if (vbytes == 4) {
                        vw = *reinterpret_cast<const uint4 *>(reinterpret_cast<const uint32_t *>(post_val) + slot);
                    } else {
                        const uint2 hv = *reinterpret_cast<const uint2 *>(reinterpret_cast<const uint16_t *>(post_val) + slot);
                        vw = make_uint4(hv.x & 0xFFFFu, hv.x >> 16, hv.y & 0xFFFFu, hv.y >> 16);
                    }
                }
                uint32_t doc[4] = {dw.x & 0xFFFFu, dw.x >> 16, dw.y & 0xFFFFu, dw.y >> 16};
                uint32_t val[4] = {vw.x, vw.y, vw.z, vw.w};
                bool ok[4];
                uint32_t bank[4], present = 0;
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    ok[p] = (uint32_t)(4 * lane + p) < n;
                    bank[p] = (doc[p] >> 2) & (kLdsBanks - 1);
                    if (ok[p]) present |= 1u << bank[p];
                }
                for (int m = 1; m < kWave; m <<= 1) present |= (uint32_t)__shfl_xor((int)present, m);
                present = (uint32_t)__builtin_amdgcn_readfirstlane((int)present);
                // rank of each posting under (bank, position); positions ascend with documents
                uint32_t rank[4] = {0u, 0u, 0u, 0u}, lower = 0;
                while (present) {
                    const uint32_t v = (uint32_t)__builtin_ctz(present);
                    present &= present - 1;
                    bool sel[4];
                    uint32_t acc = lower;  // + this bank's postings of the lanes below
#pragma unroll
                    for (int p = 0; p < 4; ++p) {
                        sel[p] = ok[p] && bank[p] == v;
                        const uint64_t m = __ballot(sel[p]);
                        acc = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, acc));
                        lower += (uint32_t)__popcll(m);
                    }
#pragma unroll
                    for (int p = 0; p < 4; ++p) {
                        if (sel[p]) rank[p] = acc;
                        acc += sel[p] ? 1u : 0u;
                    }
                }
#pragma unroll
                for (int p = 0; p < 4; ++p)
                    if (ok[p]) {
                        s_doc[w][rank[p]] = doc[p];
                        s_val[w][rank[p]] = val[p];
                    }
                wave_sync();
                // position 4 lane + p takes the posting of rank k: its place in the fill order
                const uint32_t r4 = 4u * (uint32_t)r;
                const uint32_t k0 = min(n, r4) + min(n > 128u ? n - 128u : 0u, r4) + 4u * (uint32_t)h;
#pragma unroll
                for (int p = 0; p < 4; ++p)
                    if (ok[p]) {
                        doc[p] = s_doc[w][k0 + (uint32_t)p];
                        val[p] = s_val[w][k0 + (uint32_t)p];
                    }
                wave_sync();
                if ((uint32_t)lane < cg) {
                    *reinterpret_cast<uint2 *>(post_doc + slot) =
                        make_uint2(doc[0] | (doc[1] << 16), doc[2] | (doc[3] << 16));
                    if (vbytes == 4)
                        *reinterpret_cast<uint4 *>(reinterpret_cast<uint32_t *>(post_val) + slot) =
                            make_uint4(val[0], val[1], val[2], val[3]);
                    else
                        *reinterpret_cast<uint2 *>(reinterpret_cast<uint16_t *>(post_val) + slot) =
                            make_uint2(val[0] | (val[1] << 16), val[2] | (val[3] << 16));
                }
            }
        }
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
    hipLaunchKernelGGL(k_check_rows, dim3(blocks_for((n_rows + kCheckRows - 1) / kCheckRows * kWave, 256)),
                       dim3(256), 0, s, ptr,
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
    hipLaunchKernelGGL(k_fill_lists, dim3((unsigned)n_tiles, (unsigned)passes), dim3(kFillThreads), lds, s,
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

hipError_t build_deal_chunks(const uint32_t *goff, const int64_t *tile_post, int64_t n_tiles,
                             int64_t n_cols, int32_t vbytes, uint16_t *post_doc, void *post_val,
                             hipStream_t s)
{
    if (n_tiles == 0 || n_cols == 0) return hipSuccess;
    if (n_tiles > 0x7FFFFFFF) return hipErrorInvalidValue;
    // 64 lists per wave
    const int64_t cols = std::min<int64_t>(65535, (n_cols + (int64_t)kDealThreads - 1) / kDealThreads);
    hipLaunchKernelGGL(k_deal_chunks, dim3((unsigned)n_tiles, (unsigned)cols), dim3(kDealThreads), 0,
                       s, goff, tile_post, n_cols, vbytes, post_doc, post_val);
    return hipGetLastError();
}

}  // namespace sindi
