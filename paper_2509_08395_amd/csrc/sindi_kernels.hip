// gfx950 kernels of the SINDI search path (arXiv 2509.08395).
//
//   k_query_prep   validate query rows; beta-mass subvector (Def. 6, Sec. 4.1)
//   k_accumulate1  stream each query term's window list I_{j,w} (Alg. 2,
//                  product + accumulate steps) into an on-chip score tile,
//                  one query per workgroup, the waves taking batches of
//                  chunks from a counter; then either sample per-thread
//                  maxima (threshold pass) or emit every tile score at or
//                  above the query's threshold (k_accumulate1_queue: the same
//                  as one persistent launch fed by a device queue)
//   k_accumulate   the same for batches of 2, 4 or 8 queries sharing lists
//   k_theta        per-query candidate threshold from the sampled maxima
//   k_finalize     exact top-gamma of the emitted candidates (Alg. 2 heap
//                  update): into the rerank pool, or sorted into the coarse
//                  top-k (Alg. 2 alone)
//   k_rerank       exact FP32 rerank of the pool from the unpruned vectors
//                  (Alg. 4), four pool entries per wave
//   k_topk         top-k of the reranked pool (Alg. 4)
//   k_score_*      delta(q, x) of listed pairs (Def. 2) and its gradient
//
// Ranking order: score descending, then document id ascending.  A candidate
// is one 64-bit key: (order-preserving score bits << 32) | (~doc id), so the
// ranking order is plain descending key order and keys are unique.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <utility>

#include "sindi_internal.h"

namespace sindi {
namespace {

constexpr int kWave = 64;
constexpr int kRerankPerWave = 4;  // pool entries one rerank wave scores at a time
constexpr int kRerankGroups = 4;   // such groups per wave (one query table per workgroup)
constexpr int kMaxSeg = kQueryHash / 2 / kWave;  // 64-term segments of the longest query

__device__ __forceinline__ uint32_t ord_f32(float f)
{
    uint32_t u = __float_as_uint(f);
    if (f == 0.0f) u = 0u;  // -0 ranks as +0
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unord_f32(uint32_t o)
{
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}
__device__ __forceinline__ uint64_t make_key(float s, uint32_t doc)
{
    return ((uint64_t)ord_f32(s) << 32) | (uint64_t)(0xFFFFFFFFu - doc);
}
__device__ __forceinline__ uint32_t key_doc(uint64_t k) { return 0xFFFFFFFFu - (uint32_t)k; }
__device__ __forceinline__ float key_score(uint64_t k) { return unord_f32((uint32_t)(k >> 32)); }

// A zero vector materialised where it is used (a plain register move the
// compiler cannot hoist out of the loop and keep live, or spill, at high
// register pressure).
__device__ __forceinline__ int4 fresh_zero4()
{
    int32_t z;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z));
    return make_int4(z, z, z, z);
}

// Wave-uniform copy of a value (scalar register).
__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
// A wave-uniform pointer to global memory, held in scalar registers, and
// loads of 8 or 16 bytes at a 32-bit byte offset from it (the scalar base +
// vector offset form of the global load).
using gbytes = const unsigned char __attribute__((address_space(1))) *;
__device__ __forceinline__ gbytes uni_ptr(const void *p)
{
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    return (gbytes)(((uint64_t)uni((uint32_t)(a >> 32)) << 32) | uni((uint32_t)a));
}
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void load_at(gbytes p, uint32_t off, uint2 &r)
{
    const u32x2 v = *(const u32x2 __attribute__((address_space(1))) *)(p + off);
    r = make_uint2(v.x, v.y);
}
__device__ __forceinline__ void load_at(gbytes p, uint32_t off, uint4 &r)
{
    const u32x4 v = *(const u32x4 __attribute__((address_space(1))) *)(p + off);
    r = make_uint4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ void lds_add(float *p, float v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Integer LDS atomics run at many times the rate of float ones on gfx950.
__device__ __forceinline__ void lds_add_i32(int32_t *p, int32_t v)
{
    __hip_atomic_fetch_add(reinterpret_cast<uint32_t *>(p), (uint32_t)v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
    return v;
}

__device__ __forceinline__ uint32_t hash_slot(int32_t id, int lg)
{
    return ((uint32_t)id * 0x9E3779B1u) >> (32 - lg);
}

// Exclusive scan of one value per thread over the block; `total` = sum.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *wsum, uint32_t &total)
{
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    if (lane == kWave - 1) wsum[wave] = x;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / kWave; ++i) {
        uint32_t s = wsum[i];
        off += (i < wave) ? s : 0u;
        tot += s;
    }
    total = tot;
    __syncthreads();
    return off + x - v;
}

// r-th largest (1-based) of n keys, by most-significant-digit radix select:
// one 256-bin histogram per byte of the key, restricted to the keys that
// share the digits chosen so far.  Requires 1 <= r <= n.
template <typename K, typename Load>
__device__ K block_select(int64_t n, int64_t r, Load load, uint32_t *hist, int *s_digit,
                          int64_t *s_need)
{
    K prefix = 0, mask = 0;
    int64_t need = r;
    for (int shift = (int)sizeof(K) * 8 - 8; shift >= 0; shift -= 8) {
        for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0u;
        __syncthreads();
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
            K key = load(i);
            if ((key & mask) == prefix) atomicAdd(&hist[(uint32_t)(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (threadIdx.x < kWave) {
            // digit of the need-th key: lane l holds digits 255 - 4l .. 252 - 4l; a prefix
            // sum over the lanes counts the keys with larger digits
            const int l = threadIdx.x;
            uint32_t h[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) h[u] = hist[255 - 4 * l - u];
            const uint32_t tot = h[0] + h[1] + h[2] + h[3];
            uint32_t incl = tot;
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const uint32_t y = __shfl_up(incl, d, kWave);
                if (l >= d) incl += y;
            }
            int64_t acc = (int64_t)(incl - tot);
            if (acc < need && (int64_t)incl >= need) {
                int u = 0;
                while (u < 3 && acc + (int64_t)h[u] < need) acc += h[u++];
                *s_digit = 255 - 4 * l - u;
                *s_need = need - acc;
            }
        }
        __syncthreads();
        prefix |= (K)(*s_digit) << shift;
        mask |= (K)0xFF << shift;
        need = *s_need;
        __syncthreads();
    }
    return prefix;
}

// ------------------------------------------------------------------ queries
// One wave per query row.  Flags malformed rows (err[0] bits: 1 row pointers,
// 2 term id out of range, 4 ids not strictly ascending, 8 non-finite value,
// 16 more than kQueryHash / 2 entries), keeps the longest row in err[1],
// and writes the coarse terms: the non-zero entries, cut to the beta-mass
// subvector when beta < 1 (entries ranked by |q| descending, ties by id;
// FP64 prefix sums in that order, the first prefix reaching beta * mass),
// with weights pre-multiplied by the query's fixed-point scale.
__global__ __launch_bounds__(256) void k_query_prep(DevQueries q, int64_t n_cols, double beta,
                                                    DevCoarse c, const float *term_max,
                                                    double *sabs, int32_t *err)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x / kWave);
    if (row >= q.n_rows) return;
    int64_t a = q.indptr[row], b = q.indptr[row + 1];
    int bad = 0;
    if (a < 0 || b < a || b > q.nnz || (row == 0 && a != 0) || (row == q.n_rows - 1 && b != q.nnz))
        bad |= 1;
    a = a < 0 ? 0 : (a > q.nnz ? q.nnz : a);
    b = b < a ? a : (b > q.nnz ? q.nnz : b);
    if (b - a > kQueryHash / 2) bad |= 16;
    for (int64_t e = a + lane; e < b; e += kWave) {
        int32_t id = q.indices[e];
        float v = q.values[e];
        if (id < 0 || id >= n_cols) bad |= 2;
        if (e + 1 < b && q.indices[e + 1] <= id) bad |= 4;
        if (!isfinite(v)) bad |= 8;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) bad |= __shfl_xor(bad, m, kWave);
    if (bad) {
        if (lane == 0) {
            atomicOr(err, bad);
            c.cn[row] = 0;
            c.qinv[row] = 1.0f;
        }
        return;
    }
    if (lane == 0) atomicMax(err + 1, (int32_t)(b - a));  // longest row: rerank table size
    int32_t r_keep = 0x7FFFFFFF;  // rank bound of kept entries
    if (beta < 1.0) {
        // rank of every non-zero entry in pi order; |x| placed at its rank
        int32_t nz = 0;
        for (int64_t e0 = a; e0 < b; e0 += kWave) {
            bool p = (e0 + lane < b) && q.values[e0 + lane] != 0.0f;
            nz += __popcll(__ballot(p));
        }
        for (int64_t e = a + lane; e < b; e += kWave) {
            float v = q.values[e];
            if (v == 0.0f) continue;
            float av = fabsf(v);
            int32_t id = q.indices[e];
            int32_t rank = 0;
            for (int64_t f = a; f < b; ++f) {
                float w = fabsf(q.values[f]);
                if (w == 0.0f) continue;
                int32_t jd = q.indices[f];
                rank += (w > av || (w == av && jd < id)) ? 1 : 0;
            }
            sabs[a + rank] = (double)av;
        }
        __threadfence();
        int32_t r = 0;
        if (lane == 0) {
            double mass = 0.0;
            for (int32_t t = 0; t < nz; ++t) mass += sabs[a + t];
            double thr = beta * mass;
            double run = 0.0;
            while (r < nz) {
                run += sabs[a + r];
                ++r;
                if (run >= thr) break;
            }
        }
        r_keep = __shfl(r, 0, kWave);
    }
    // ordered compaction of the kept entries (ascending term id preserved)
    int32_t base = 0;
    for (int64_t e0 = a; e0 < b; e0 += kWave) {
        int64_t e = e0 + lane;
        bool keep = false;
        float v = 0.0f;
        int32_t id = 0;
        if (e < b) {
            v = q.values[e];
            id = q.indices[e];
            keep = v != 0.0f;
            if (keep && r_keep != 0x7FFFFFFF) {
                float av = fabsf(v);
                int32_t rank = 0;
                for (int64_t f = a; f < b; ++f) {
                    float w = fabsf(q.values[f]);
                    if (w == 0.0f) continue;
                    int32_t jd = q.indices[f];
                    rank += (w > av || (w == av && jd < id)) ? 1 : 0;
                }
                keep = rank < r_keep;
            }
        }
        uint64_t m = __ballot(keep);
        if (keep) {
            int32_t p = base + (int32_t)lanes_below(m);
            c.ct[a + p] = id;
            c.cw[a + p] = v;
        }
        base += __popcll(m);
    }
    // fixed-point scale: the largest power of two keeping every partial
    // coarse sum of this query within 2^30 in magnitude
    float bound = 0.0f;
    for (int32_t i = lane; i < base; i += kWave)
        bound += fabsf(c.cw[a + i]) * term_max[c.ct[a + i]];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) bound += __shfl_xor(bound, m, kWave);
    int ex = 0;
    if (bound > 0.0f) {
        (void)frexpf(bound, &ex);  // bound < 2^ex
        ex = 30 - ex;
        ex = ex > 100 ? 100 : (ex < -100 ? -100 : ex);
    }
    const float scale = ldexpf(1.0f, ex);
    for (int32_t i = lane; i < base; i += kWave) c.cw[a + i] *= scale;
    if (lane == 0) {
        c.cn[row] = base;
        c.qinv[row] = ldexpf(1.0f, -ex);
    }
}

// ------------------------------------------------------------------ accumulate
// Posting values: raw bits of one aligned 4-posting group, decoded after
// every load of the step has been issued.
template <int VT> struct Val;
template <> struct Val<0> {  // FP32
    using Raw = uint4;
    static __device__ __forceinline__ Raw load(const void *p, uint64_t g)
    {
        return reinterpret_cast<const uint4 *>(p)[g];
    }
    static __device__ __forceinline__ void decode(const Raw &r, float (&v)[4])
    {
        v[0] = __uint_as_float(r.x);
        v[1] = __uint_as_float(r.y);
        v[2] = __uint_as_float(r.z);
        v[3] = __uint_as_float(r.w);
    }
    // w * x_p rounded to FP32
    static __device__ __forceinline__ float prod(const Raw &r, int p, float w)
    {
        const uint32_t b = p == 0 ? r.x : (p == 1 ? r.y : (p == 2 ? r.z : r.w));
        return w * __uint_as_float(b);
    }
};
template <> struct Val<1> {  // FP16
    using Raw = uint2;
    static __device__ __forceinline__ Raw load(const void *p, uint64_t g)
    {
        return reinterpret_cast<const uint2 *>(p)[g];
    }
    static __device__ __forceinline__ float h2f(uint32_t h)
    {
        return (float)__builtin_bit_cast(_Float16, (uint16_t)h);
    }
    static __device__ __forceinline__ void decode(const Raw &r, float (&v)[4])
    {
        v[0] = h2f(r.x & 0xFFFFu);
        v[1] = h2f(r.x >> 16);
        v[2] = h2f(r.y & 0xFFFFu);
        v[3] = h2f(r.y >> 16);
    }
    // w * x_p rounded to FP32: the FP16 value widens exactly, and a fused
    // multiply-add with a +0 addend rounds the product once, as a multiply
    // does (the sign of a zero product is lost, which the integer conversion
    // that follows ignores); one mixed-precision FMA does both steps.
    static __device__ __forceinline__ float prod(const Raw &r, int p, float w)
    {
        const uint32_t word = p < 2 ? r.x : r.y;
        const uint32_t bits = (p & 1) ? (word >> 16) : (word & 0xFFFFu);
        return __builtin_fmaf(w, h2f(bits), 0.0f);
    }
};
template <> struct Val<2> {  // BF16
    using Raw = uint2;
    static __device__ __forceinline__ Raw load(const void *p, uint64_t g)
    {
        return reinterpret_cast<const uint2 *>(p)[g];
    }
    static __device__ __forceinline__ void decode(const Raw &r, float (&v)[4])
    {
        v[0] = __uint_as_float(r.x << 16);
        v[1] = __uint_as_float(r.x & 0xFFFF0000u);
        v[2] = __uint_as_float(r.y << 16);
        v[3] = __uint_as_float(r.y & 0xFFFF0000u);
    }
    static __device__ __forceinline__ float prod(const Raw &r, int p, float w)
    {
        const uint32_t word = p < 2 ? r.x : r.y;
        return w * __uint_as_float((p & 1) ? (word & 0xFFFF0000u) : (word << 16));
    }
};

// Emit the scores of one query row segment that reach the threshold: each
// lane holds NV scores of consecutive documents starting at m0.
template <int NV>
__device__ __forceinline__ void emit_candidates(const float (&sv)[NV], const bool (&ok)[NV],
                                                int64_t doc0, uint32_t *cnt, uint64_t *out,
                                                int64_t cap)
{
    const int lane = threadIdx.x & (kWave - 1);
    uint64_t bal[NV];
    uint32_t tot = 0;
#pragma unroll
    for (int p = 0; p < NV; ++p) {
        bal[p] = __ballot(ok[p]);
        tot += (uint32_t)__popcll(bal[p]);
    }
    uint32_t b0 = 0;
    if (lane == 0) b0 = atomicAdd(cnt, tot);
    b0 = __shfl(b0, 0, kWave);
#pragma unroll
    for (int p = 0; p < NV; ++p) {
        if (ok[p]) {
            const uint64_t pos = (uint64_t)b0 + lanes_below(bal[p]);
            if (pos < (uint64_t)cap) out[pos] = make_key(sv[p], (uint32_t)(doc0 + p));
        }
        b0 += (uint32_t)__popcll(bal[p]);
    }
}

// Smallest fixed-point sum a with (float)a * qinv >= th, as an int64 (2^31 if
// no int32 sum reaches th).  (float)a * qinv is non-decreasing in a, so the
// scores at or above th are exactly the sums at or above this bound.
__device__ int64_t sum_threshold(float th, float qinv)
{
    auto reaches = [&](int64_t a) { return (float)(int32_t)a * qinv >= th; };
    if (!reaches(INT32_MAX)) return (int64_t)INT32_MAX + 1;
    int64_t lo = INT32_MIN, hi = INT32_MAX;  // invariant: reaches(hi)
    if (reaches(lo)) return lo;
    while (hi - lo > 1) {                     // invariant: !reaches(lo)
        const int64_t mid = lo + (hi - lo) / 2;
        if (reaches(mid)) hi = mid; else lo = mid;
    }
    return hi;
}

// Decode a pair-packed 64-bit score word into the two 32-bit sums it holds:
// the word is H * 2^32 + L (exactly, modulo 2^64) with |L|, |H| < 2^31.
__device__ __forceinline__ void unpack_pair(uint32_t wlo, uint32_t whi, int32_t &l, int32_t &h)
{
    l = (int32_t)wlo;
    h = (int32_t)(whi + (l < 0 ? 1u : 0u));
}

// One workgroup = a batch of B >= 2 query slots x a contiguous run of tiles.  The
// batch's (query, term) entries are first merged into one ascending list of
// distinct terms, each with a weight per query (zero where the query lacks
// the term), so a list I_{term, tile} shared by several queries of the batch
// is read once.  Then, for every tile: the score rows (the window's distance
// array of Sec. 3.3.1, one per query) are cleared in LDS; the tile's lists of
// all merged terms (each padded to whole 4-posting groups with zero values)
// are cut into chunks of up to 64 groups, and each wave takes a contiguous
// share of the chunks, several chunks in flight: one group per lane, so a
// chunk's list, weights and base address are wave-uniform (scalar registers)
// and a lane only adds its group's offset.  Every posting adds w_b * x to
// query b's score of its document (Alg. 2: product, then accumulate).
//
// Scores are 32-bit fixed point: weights arrive multiplied by the query's
// power-of-two scale and each product is truncated once to an integer, so
// the sums are exact and independent of the order of the adds; different
// terms can hit one document concurrently, so the adds are LDS atomics, and
// integer LDS atomics run many times faster than float ones on this chip.
// For B >= 2 the rows of queries 2q and 2q+1 are interleaved into one 64-bit
// word per document holding H * 2^32 + L, so one 64-bit atomic updates both
// (the sums stay within +-2^30, so both halves decode exactly).
//
// Finally each row is either sampled (per-thread maxima, for the candidate
// threshold) or every score at or above the query's threshold is appended to
// its candidate list.
template <int VT, int B, bool SAMPLE>
__global__ __launch_bounds__(kAccThreads) __attribute__((amdgpu_waves_per_eu(6))) void k_accumulate(
    DevIndex ix, DevQueries q, DevCoarse c, const int32_t *slot_q, int32_t n_slots,
    int32_t n_sample, float *maxima, const float *theta, uint32_t *count, uint64_t *cand,
    int64_t cap, int32_t tiles_per_wg, int32_t eb)
{
    constexpr int NT = kAccThreads, NW = NT / kWave;
    const int EB = eb;  // entries merged per pass: a power of two, at most NT
    constexpr int NP = B / 2;            // score words per document
    constexpr int KU = VT == 0 ? 4 : 8;  // chunks in flight per wave
    static_assert(B >= 2 && B % 2 == 0, "one query per workgroup runs in k_accumulate1");
    static_assert(kEntryBlock <= NT, "at most one merged entry per thread");
    extern __shared__ __align__(16) unsigned char smem[];
    const int T = ix.tile_stride;
    // score rows: uint64 [NP][T], B * T * 4 bytes
    unsigned char *A = smem;
    // the merged term list (u_term / u_w, EB entries)
    int32_t *u_term = reinterpret_cast<int32_t *>(smem + (size_t)B * T * 4);
    float *u_w = reinterpret_cast<float *>(u_term + EB);  // [EB][B]
    unsigned char *region = reinterpret_cast<unsigned char *>(u_w + (size_t)EB * B);
    uint64_t *keys = reinterpret_cast<uint64_t *>(region);                 // merge phase
    uint32_t *flag = reinterpret_cast<uint32_t *>(keys + EB);              // merge phase
    uint32_t *l_base = reinterpret_cast<uint32_t *>(region);               // tile phase
    uint32_t *l_end = l_base + EB;
    uint32_t *l_cp = l_end + EB;                                           // EB + 1 (+3)
    float *l_w = reinterpret_cast<float *>(l_cp + EB + 4);                 // [EB][B]
    __shared__ int64_t s_qa[B];
    __shared__ int32_t s_qpre[B + 1];
    __shared__ int32_t s_slot[B];
    __shared__ float s_qinv[B];
    __shared__ uint32_t s_wsum[NW];
    __shared__ int32_t s_nu;
    __shared__ uint32_t s_wl[NW];  // list holding each wave's first chunk
    __shared__ int32_t s_thr[B];   // per query: smallest sum at or above its threshold
    __shared__ int32_t s_none[B];  // per query: no sum reaches the threshold
    __shared__ int32_t s_imp[B];   // per query: threshold <= 0, zero sums left implicit

    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int wave = (int)uni((uint32_t)tid / kWave);  // uniform per wave: keeps chunk bookkeeping scalar
    const int32_t batch = blockIdx.x;
    if (tid == 0) {
        int32_t acc = 0;
        for (int b = 0; b < B; ++b) {
            const int32_t s = batch * B + b;
            int32_t n = 0;
            int64_t qa = 0;
            float qinv = 1.0f;
            if (s < n_slots) {
                const int32_t row = slot_q[s];
                qa = q.indptr[row];
                n = c.cn[row];
                qinv = c.qinv[row];
            }
            s_slot[b] = s < n_slots ? s : -1;
            s_qinv[b] = qinv;
            s_qa[b] = qa;
            s_qpre[b] = acc;
            acc += n;
        }
        s_qpre[B] = acc;
    }
    if (!SAMPLE && tid < B) {
        const int32_t s2 = batch * B + tid;
        const int64_t a = s2 < n_slots ? sum_threshold(theta[s2], c.qinv[slot_q[s2]])
                                       : (int64_t)INT32_MAX + 1;
        s_none[tid] = a > INT32_MAX;
        s_thr[tid] = a > INT32_MAX ? INT32_MAX : (int32_t)a;
        const float th = s2 < n_slots ? theta[s2] : 1.0f;
        s_imp[tid] = th <= 0.0f && th != -INFINITY;
    }
    __syncthreads();
    const int32_t n_e = s_qpre[B];
    const int32_t n_blocks = (n_e + EB - 1) / EB;

    // Merge entries [e0, e0 + EB) of the batch into u_term / u_w (s_nu terms).
    auto merge = [&](int32_t e0) {
        const int32_t ne = min(EB, n_e - e0);
        int P = 1;
        while (P < ne) P <<= 1;
        if (tid < P) {
            uint64_t key = ~0ull;
            if (tid < ne) {
                const int32_t e = e0 + tid;
                int b = 0;
                while (b + 1 < B && s_qpre[b + 1] <= e) ++b;
                key = ((uint64_t)(uint32_t)c.ct[s_qa[b] + (e - s_qpre[b])] << 32) | (uint32_t)tid;
            }
            keys[tid] = key;
        }
        __syncthreads();
        for (int kk = 2; kk <= P; kk <<= 1) {
            for (int j = kk >> 1; j > 0; j >>= 1) {
                if (tid < P) {
                    const int ij = tid ^ j;
                    if (ij > tid) {
                        const uint64_t x = keys[tid], y = keys[ij];
                        const bool up = (tid & kk) == 0;
                        if (up ? (x > y) : (x < y)) {
                            keys[tid] = y;
                            keys[ij] = x;
                        }
                    }
                }
                __syncthreads();
            }
        }
        const uint32_t fresh =
            (tid < ne && (tid == 0 || (keys[tid] >> 32) != (keys[tid - 1] >> 32))) ? 1u : 0u;
        uint32_t nu;
        const uint32_t ex = block_excl_scan<NT>(fresh, s_wsum, nu);
        for (int i = tid; i < (int)nu * B; i += NT) u_w[i] = 0.0f;
        if (tid < EB) flag[tid] = ex + fresh;  // 1-based merged index of this sorted entry's term
        if (tid == 0) s_nu = (int32_t)nu;
        __syncthreads();
        if (tid < ne) {
            const uint64_t key = keys[tid];
            const int32_t u = (int32_t)flag[tid] - 1;
            const int32_t e = e0 + (int32_t)(key & 0xFFFFFFFFu);
            int b = 0;
            while (b + 1 < B && s_qpre[b + 1] <= e) ++b;
            if (fresh) u_term[u] = (int32_t)(key >> 32);
            u_w[u * B + b] = c.cw[s_qa[b] + (e - s_qpre[b])];
        }
        __syncthreads();
    };

    if (n_blocks == 1) merge(0);
    const int64_t n_tile_iter = SAMPLE ? n_sample : ix.n_tiles;
    using Raw = typename Val<VT>::Raw;

    // With one merged block, each thread prefetches its term's list bounds of
    // the next tile while the current tile accumulates.
    uint32_t pre_lo = 0, pre_hi = 0;
    bool have_pre = false;
    // Workgroup y sweeps tiles [y R, (y + 1) R).  Workgroups are dispatched batch
    // fastest, so those resident together walk the same tiles at about the
    // same pace and share the tiles' lists in L2.
    const int64_t ti_beg = (int64_t)blockIdx.y * tiles_per_wg;
    const int64_t ti_end = min(n_tile_iter, ti_beg + tiles_per_wg);
    // the score rows start cleared; reading a tile's rows clears them again
    {
        int4 *A4 = reinterpret_cast<int4 *>(A);
        for (int i = tid; i < B * T / 4; i += NT) A4[i] = make_int4(0, 0, 0, 0);
    }
    __syncthreads();
    for (int64_t ti = ti_beg; ti < ti_end; ++ti) {
        const int64_t t = SAMPLE ? (ti * ix.n_tiles / n_sample) : ti;
        const int64_t d0 = ix.tile_doc[t];
        const int32_t len = (int32_t)(ix.tile_doc[t + 1] - d0);
        const uint64_t G0 = (uint64_t)ix.tile_post[t] >> 2;  // first 4-posting group of the tile
        const uint32_t *toff = ix.term_goff + (size_t)t * (size_t)(ix.n_cols + 1);

        for (int32_t blk = 0; blk < n_blocks; ++blk) {
            if (n_blocks > 1) merge(blk * EB);
            const int32_t nu = s_nu;
            // list (term, tile) = groups [gs, gs + ng) of the tile, cut into chunks
            // of kChunk groups; the non-empty lists are compacted in term order
            // with the index of their first chunk
            uint32_t gs = 0, ng = 0;
            if (tid < nu) {
                const int32_t term = u_term[tid];
                const uint32_t lo = have_pre ? pre_lo : toff[term];
                const uint32_t hi = have_pre ? pre_hi : toff[term + 1];
                gs = lo & kGoffMask;
                ng = (hi & kGoffMask) - gs;
            }
            const uint32_t nch = (ng + kChunk - 1) / kChunk;
            uint32_t total;
            // low 20 bits: chunks before this list; high bits: non-empty lists before it
            const uint32_t ex = block_excl_scan<NT>(nch | (nch ? (1u << 20) : 0u), s_wsum, total);
            // the scan's barriers order these writes after the merge-phase reads
            if (nch) {
                // chunk ci of list li covers groups [l_base + 64 ci, min(+64, l_end)) of
                // the tile (l_base wraps below zero as an unsigned number)
                const uint32_t li = ex >> 20;
                l_base[li] = gs - (ex & 0xFFFFFu) * (uint32_t)kChunk;
                l_end[li] = gs + ng;
                l_cp[li] = ex & 0xFFFFFu;
#pragma unroll
                for (int b = 0; b < B; ++b) l_w[li * B + b] = u_w[tid * B + b];
            }
            const uint32_t n_list = total >> 20, n_chunk = total & 0xFFFFFu;
            if (tid == 0) l_cp[n_list] = n_chunk;
            // wave w takes chunks [n_chunk w / NW, n_chunk (w + 1) / NW)
            if (nch) {
                const uint32_t c0l = ex & 0xFFFFFu;
#pragma unroll
                for (int w2 = 0; w2 < NW; ++w2) {
                    const uint32_t cb = (uint32_t)(((uint64_t)n_chunk * (uint32_t)w2) / NW);
                    if (cb >= c0l && cb < c0l + nch) s_wl[w2] = ex >> 20;
                }
            }
            have_pre = false;
            if (n_blocks == 1) {
                const int64_t tn = ti + 1;
                if (tn < ti_end) {
                    have_pre = true;
                    if (tid < nu) {
                        const int64_t t2 = SAMPLE ? (tn * ix.n_tiles / n_sample) : tn;
                        const uint32_t *toff2 = ix.term_goff + (size_t)t2 * (size_t)(ix.n_cols + 1);
                        const int32_t term = u_term[tid];
                        pre_lo = toff2[term];
                        pre_hi = toff2[term + 1];
                    }
                }
            }
            __syncthreads();

            // This wave's contiguous share of the chunks.  One chunk = up to 64
            // consecutive groups of one list, one group (4 postings) per lane, so a
            // chunk's list, weights and base address are wave-uniform.  The wave
            // reads the bounds of 64 consecutive lists at once (one per lane); a
            // chunk finds its list among them by a ballot over the lists' first
            // chunks and takes the list's fields by lane broadcast, so KU chunks'
            // loads leave back to back even where they cross lists.
            const uint32_t c_beg = (uint32_t)(((uint64_t)n_chunk * (uint32_t)wave) / NW);
            const uint32_t c_end = (uint32_t)(((uint64_t)n_chunk * (uint32_t)(wave + 1)) / NW);
            if (c_beg < c_end) {
                // the tile's groups, addressed by 32-bit byte offsets (a tile holds at
                // most kTileGroupsMax groups; the arrays end with kTailSlots zero postings)
                const gbytes pd_t = uni_ptr(
                    reinterpret_cast<const unsigned char *>(ix.post_doc) + G0 * sizeof(uint2));
                const gbytes pv_t = uni_ptr(
                    reinterpret_cast<const unsigned char *>(ix.post_val) + G0 * sizeof(Raw));
                uint32_t lp0 = uni(s_wl[wave]);  // list of chunk c
                for (uint32_t c = c_beg; c < c_end;) {
                    const uint32_t lw = lp0 + (uint32_t)lane;
                    const uint32_t cpn = lw + 1 <= n_list ? l_cp[lw + 1] : 0xFFFFFFFFu;
                    uint32_t basel = 0, endl = 0;
                    float wl[B];
#pragma unroll
                    for (int b = 0; b < B; ++b) wl[b] = 0.0f;
                    if (lw < n_list) {
                        basel = l_base[lw];
                        endl = l_end[lw];
#pragma unroll
                        for (int b = 0; b < B; ++b) wl[b] = l_w[lw * B + b];
                    }
                    // the window's chunks lie in lists lp0 .. lp0 + 63
                    const uint32_t c_win = min(c_end, c + (uint32_t)kWave);
                    for (uint32_t cs = c; cs < c_win; cs += KU) {
                        uint2 ids[KU];
                        Raw raw[KU];
                        uint32_t nl[KU];
                        int32_t kl[KU];
                        // Loads are unconditional, so they leave back to back: lane l reads
                        // group g0 + l even past its chunk's end (at most 63 groups past the
                        // end of a list of this tile: inside the arrays), and a slot past the
                        // window reads the tile's first groups; those lanes add nothing.
#pragma unroll
                        for (int i = 0; i < KU; ++i) {
                            const uint32_t ci = cs + (uint32_t)i;
                            uint32_t g0 = 0, n = 0;
                            int32_t k = 0;
                            if (ci < c_win) {  // wave-uniform
                                k = (int32_t)__popcll(__ballot(cpn <= ci));
                                g0 = (uint32_t)__builtin_amdgcn_readlane((int)basel, k) +
                                     ci * (uint32_t)kChunk;
                                n = min((uint32_t)kChunk,
                                        (uint32_t)__builtin_amdgcn_readlane((int)endl, k) - g0);
                            }
                            kl[i] = k;
                            nl[i] = n;
                            const uint32_t gi = g0 + (uint32_t)lane;
                            load_at(pd_t, gi * (uint32_t)sizeof(uint2), ids[i]);
                            load_at(pv_t, gi * (uint32_t)sizeof(Raw), raw[i]);
                        }
#pragma unroll
                        for (int i = 0; i < KU; ++i) {
                            if ((uint32_t)lane >= nl[i]) continue;
                            float w[B];
#pragma unroll
                            for (int b = 0; b < B; ++b)
                                w[b] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wl[b]), kl[i]));
                            // byte offsets of the documents' 32-bit score words
                            const uint32_t d4[4] = {ids[i].x & 0xFFFFu, ids[i].x >> 16,
                                                    ids[i].y & 0xFFFFu, ids[i].y >> 16};
                            float v[4];
                            Val<VT>::decode(raw[i], v);
                            unsigned char *A8 = A;
#pragma unroll
                            for (int qp = 0; qp < NP; ++qp) {
                                const float w0 = w[2 * qp], w1 = w[2 * qp + 1];
                                if (w0 == 0.0f && w1 == 0.0f) continue;
#pragma unroll
                                for (int p = 0; p < 4; ++p) {
                                    const int32_t lo = (int32_t)(w0 * v[p]);
                                    const int32_t hi = (int32_t)(w1 * v[p]);
                                    const uint32_t hw = (uint32_t)hi + (uint32_t)(lo >> 31);
                                    const uint64_t add = ((uint64_t)hw << 32) | (uint32_t)lo;
                                    uint64_t *dst = reinterpret_cast<uint64_t *>(
                                        A8 + (size_t)qp * T * 8 + 2u * d4[p]);
                                    __hip_atomic_fetch_add(dst, add, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                                }
                            }
                        }
                    }
                    // list of the next window's first chunk
                    lp0 += c_win < c_end ? (uint32_t)__popcll(__ballot(cpn <= c_win)) : 0u;
                    c = c_win;
                }
            }
            __syncthreads();
        }

        // ---- read the rows: sample maxima or emit every score at or above the
        // query's threshold, compared as the integer sum against the smallest sum
        // that reaches the threshold
        uint64_t *A64 = reinterpret_cast<uint64_t *>(A);
        for (int qp = 0; qp < NP; ++qp) {
            const int32_t sl0 = s_slot[2 * qp], sl1 = s_slot[2 * qp + 1];
            const bool any0 = sl0 >= 0 && (SAMPLE || !s_none[2 * qp]);
            const bool any1 = sl1 >= 0 && (SAMPLE || !s_none[2 * qp + 1]);
            uint64_t *row = A64 + (size_t)qp * T;
            if (!any0 && !any1) {
                for (int m = tid * 2; m < len; m += NT * 2)
                    *reinterpret_cast<int4 *>(row + m) = fresh_zero4();
                continue;
            }
            const float qi0 = s_qinv[2 * qp], qi1 = s_qinv[2 * qp + 1];
            if (SAMPLE) {
                int32_t m0 = INT32_MIN, m1 = INT32_MIN;
                for (int m = tid; m < len; m += NT) {
                    const uint64_t wd = row[m];
                    row[m] = 0ull;
                    int32_t l, h;
                    unpack_pair((uint32_t)wd, (uint32_t)(wd >> 32), l, h);
                    m0 = max(m0, l);
                    m1 = max(m1, h);
                }
                if (sl0 >= 0)
                    maxima[((size_t)sl0 * n_sample + ti) * NT + tid] = tid < len ? (float)m0 * qi0 : -INFINITY;
                if (sl1 >= 0)
                    maxima[((size_t)sl1 * n_sample + ti) * NT + tid] = tid < len ? (float)m1 * qi1 : -INFINITY;
            } else {
                const int32_t th0 = s_thr[2 * qp], th1 = s_thr[2 * qp + 1];
                const bool imp0 = s_imp[2 * qp], imp1 = s_imp[2 * qp + 1];
                for (int base = wave * 128; base < len; base += NW * 128) {
                    const int m0 = base + lane * 2;
                    int4 r = make_int4(0, 0, 0, 0);
                    if (m0 < len) {
                        r = *reinterpret_cast<const int4 *>(row + m0);
                        *reinterpret_cast<int4 *>(row + m0) = fresh_zero4();
                    }
                    int32_t l0, h0, l1, h1;
                    unpack_pair((uint32_t)r.x, (uint32_t)r.y, l0, h0);
                    unpack_pair((uint32_t)r.z, (uint32_t)r.w, l1, h1);
                    // threshold <= 0: every nonzero sum, negative ones included, so that
                    // the finalize kernel may take each document left out as a zero
                    const bool oa[2] = {any0 && m0 < len && (imp0 ? l0 != 0 : l0 >= th0),
                                        any0 && m0 + 1 < len && (imp0 ? l1 != 0 : l1 >= th0)};
                    const bool ob[2] = {any1 && m0 < len && (imp1 ? h0 != 0 : h0 >= th1),
                                        any1 && m0 + 1 < len && (imp1 ? h1 != 0 : h1 >= th1)};
                    if (__ballot(oa[0] || oa[1] || ob[0] || ob[1]) == 0) continue;
                    const float a[2] = {(float)l0 * qi0, (float)l1 * qi0};
                    const float b2[2] = {(float)h0 * qi1, (float)h1 * qi1};
                    if (sl0 >= 0)
                        emit_candidates<2>(a, oa, d0 + m0, count + sl0, cand + (size_t)sl0 * cap, cap);
                    if (sl1 >= 0)
                        emit_candidates<2>(b2, ob, d0 + m0, count + sl1, cand + (size_t)sl1 * cap, cap);
                }
            }
        }
        __syncthreads();
    }
}

// Inclusive prefix sum over the wave in lane order: within each row of 16
// lanes by four shifted adds (DPP row_shr 1, 2, 4, 8; lanes shifted in from
// outside the row read 0), then each row adds the totals of the rows below.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    const int lane = threadIdx.x & (kWave - 1);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);
    const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)x, 15);
    const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)x, 31);
    const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)x, 47);
    return x + (lane >= 16 ? r0 : 0u) + (lane >= 32 ? r1 : 0u) + (lane >= 48 ? r2 : 0u);
}

// The single-query form of k_accumulate (same grid, same scores, same
// read-out).  Every wave lays out the tile's chunks itself: the query's terms
// are taken 64 at a time (a segment, one list per lane), and a wave-wide
// prefix sum over the lists' chunk counts numbers the segment's chunks.  The
// waves then take batches of KU consecutive chunks: wave w's first batch of a
// segment is fixed (chunks w KU to w KU + KU - 1, so its loads leave at once),
// the next ones come from the segment's counter in LDS (one atomic by the
// wave's first lane, taken while the current batch's loads are in flight), so
// they finish the tile together however unevenly the lists' lengths and the
// adds' bank conflicts fall; the counters are reset between the tile's two
// barriers.  The layout needs no LDS table:
// a tile costs the two barriers around its read-out.  The first segment's
// terms, weights and list bounds (the next tile's prefetched during the
// current one) stay in registers; further segments are reloaded (cache hits).
//
// One work item: query slot `slot` over tile run `run` (tiles [run R, (run + 1) R)).  The
// score row must be all zero on entry unless clear_row (the read-out of every tile clears what
// the tile's adds touched, so it is all zero again on return).
template <int VT, bool SAMPLE>
__device__ __forceinline__ void accumulate1_item(
    const DevIndex &ix, const DevQueries &q, const DevCoarse &c, const int32_t *slot_q,
    int32_t n_sample, float *maxima, const float *theta, uint32_t *count, uint64_t *cand,
    int64_t cap, int32_t tiles_per_wg, int32_t slot, int64_t run, bool clear_row)
{
    constexpr int NT = kAccThreads, NW = NT / kWave;
    constexpr int KU = VT == 0 ? 3 : 5;  // chunks per batch of a wave
    extern __shared__ __align__(16) unsigned char smem[];
    int32_t *A32 = reinterpret_cast<int32_t *>(smem);  // the query's score row [tile_stride]
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int wave = (int)uni((uint32_t)tid / kWave);
    const int32_t row = slot_q[slot];
    const int64_t qa = q.indptr[row];
    const int32_t n = c.cn[row];
    const float qinv = c.qinv[row];
    int32_t th = 0;
    bool none = false, imp = false;
    if (!SAMPLE) {
        const int64_t a = sum_threshold(theta[slot], qinv);
        none = a > INT32_MAX;
        th = none ? INT32_MAX : (int32_t)a;
        const float tv = theta[slot];
        imp = tv <= 0.0f && tv != -INFINITY;
    }
    const int32_t nseg = (n + kWave - 1) / kWave;
    const int32_t term0 = lane < n ? c.ct[qa + lane] : 0;
    const float w0 = lane < n ? c.cw[qa + lane] : 0.0f;
    using Raw = typename Val<VT>::Raw;
    const int64_t n_tile_iter = SAMPLE ? n_sample : ix.n_tiles;
    const int64_t ti_beg = run * tiles_per_wg;
    const int64_t ti_end = min(n_tile_iter, ti_beg + tiles_per_wg);
    const size_t toff_stride = (size_t)(ix.n_cols + 1);
    auto tile_of = [&](int64_t ti) { return SAMPLE ? (ti * ix.n_tiles / n_sample) : ti; };

    // the score row starts cleared; reading a tile's row clears it again
    if (clear_row) {
        int4 *A4 = reinterpret_cast<int4 *>(smem);
        for (int i = tid; i < ix.tile_stride / 4; i += NT) A4[i] = make_int4(0, 0, 0, 0);
    }
    // Bounds of the first segment's lists in the tile (the next tile's are
    // loaded during the current one; every lane loads, lanes past the query's
    // terms read term 0's bounds and ignore them).  The grid gives every
    // workgroup at least one tile.
    uint32_t pre_lo, pre_hi;
    {
        const uint32_t *toff = ix.term_goff + (size_t)tile_of(ti_beg) * toff_stride;
        pre_lo = toff[term0];
        pre_hi = toff[term0 + 1];
    }
    // The run's tiles, one per lane (reloaded every 64 tiles): first document,
    // length, first 4-posting group and group count, so a tile starts without
    // waiting for memory.
    int64_t r_d0 = 0;
    uint64_t r_g0 = 0;
    int32_t r_len = 0;
    uint32_t r_ng = 0;
    int64_t r_base = ti_beg;
    auto load_run = [&](int64_t base) {
        const int64_t ti = base + lane;
        if (ti < ti_end) {
            const int64_t t = tile_of(ti);
            r_d0 = ix.tile_doc[t];
            r_len = (int32_t)(ix.tile_doc[t + 1] - r_d0);
            const int64_t p0 = ix.tile_post[t];
            r_g0 = (uint64_t)p0 >> 2;
            r_ng = (uint32_t)((ix.tile_post[t + 1] - p0) >> 2);
        }
    };
    load_run(r_base);
    // The waves take batches of KU chunks of a segment from the segment's counter, so that
    // they reach the tile's barrier together; wave w's first batch of a segment is chunks
    // [w KU, (w + 1) KU), so the counters start past the NW first batches.
    constexpr uint32_t kFirstTaken = (uint32_t)(NW * KU);
    __shared__ uint32_t s_next[kMaxSeg];
    for (int i = tid; i < kMaxSeg; i += NT) s_next[i] = kFirstTaken;
    __syncthreads();

    for (int64_t ti = ti_beg; ti < ti_end; ++ti) {
        if (ti - r_base == kWave) {
            r_base = ti;
            load_run(r_base);
        }
        const int j = (int)(ti - r_base);
        const int64_t t = tile_of(ti);
        const int64_t d0 = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(r_d0 >> 32), j) << 32) |
                                     (uint32_t)__builtin_amdgcn_readlane((int)r_d0, j));
        const int32_t len = __builtin_amdgcn_readlane(r_len, j);
        const uint64_t G0 = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(r_g0 >> 32), j) << 32) |
                            (uint32_t)__builtin_amdgcn_readlane((int)r_g0, j);
        const uint32_t n_groups = (uint32_t)__builtin_amdgcn_readlane((int)r_ng, j);
        const uint32_t *toff = ix.term_goff + (size_t)t * toff_stride;
        const uint32_t gs0 = pre_lo & kGoffMask;
        const uint32_t ng0 = lane < n ? (pre_hi & kGoffMask) - gs0 : 0u;
        {
            const int64_t tn = ti + 1 < ti_end ? ti + 1 : ti;
            const uint32_t *toff2 = ix.term_goff + (size_t)tile_of(tn) * toff_stride;
            pre_lo = toff2[term0];
            pre_hi = toff2[term0 + 1];
        }
        // segment s >= 1: lane l holds list 64 s + l
        auto segment = [&](int32_t s, uint32_t &gs, uint32_t &ng, float &w) {
            gs = 0;
            ng = 0;
            w = 0.0f;
            const int32_t li = s * kWave + lane;
            if (li < n) {
                const int32_t term = c.ct[qa + li];
                w = c.cw[qa + li];
                const uint32_t lo = toff[term], hi = toff[term + 1];
                gs = lo & kGoffMask;
                ng = (hi & kGoffMask) - gs;
            }
        };
        // the tile's groups, addressed by 32-bit byte offsets (a tile holds at most
        // kTileGroupsMax groups; the arrays end with kTailSlots zero postings)
        const gbytes pd_t =
            uni_ptr(reinterpret_cast<const unsigned char *>(ix.post_doc) + G0 * sizeof(uint2));
        const gbytes pv_t =
            uni_ptr(reinterpret_cast<const unsigned char *>(ix.post_val) + G0 * sizeof(Raw));
        for (int32_t s = 0; s < nseg; ++s) {
            uint32_t gs = gs0, ng = ng0;
            float wl = w0;
            if (s > 0) segment(s, gs, ng, wl);
            // chunk numbers: list l of the segment holds its chunks [incl - nch, incl)
            const uint32_t nch = (ng + kChunk - 1) / kChunk;
            const uint32_t incl = wave_incl_scan(nch);
            const uint32_t st = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
            if (st == 0) continue;
            // list of chunk ci: the lanes whose lists end at or before ci, counted
            const uint32_t cpn = incl;
            const uint32_t basel = gs - (incl - nch) * (uint32_t)kChunk;
            const uint32_t endl = gs + ng;
            auto take = [&]() {  // the first chunk of the wave's next batch
                uint32_t g = 0;
                if (lane == 0) g = atomicAdd(&s_next[s], (uint32_t)KU);
                return uni(g);
            };
            const uint32_t lb = st;
            uint32_t cs = (uint32_t)wave * (uint32_t)KU;
            // The list of the wave's last chunk: its chunks end at c_end, its chunk 0 would
            // start at group l_base, it ends at group l_end, its weight is l_w.  A wave's chunk
            // numbers only grow inside a segment, so a chunk below c_end is in that list.
            uint32_t c_end = 0, l_base = 0, l_end = 0;
            float l_w = 0.0f;
            while (cs < lb) {
                uint2 ids[KU];
                Raw raw[KU];
                uint32_t nl[KU];
                float wk[KU];
                // Loads are unconditional, so they leave back to back: lane l reads
                // group g0 + l even past its chunk's end (at most 63 groups past the
                // tile's last group: inside the arrays); those lanes add nothing.
                // The wave issues them at raised priority, so waves about to load
                // go ahead of waves adding into LDS.
                __builtin_amdgcn_s_setprio(3);
#pragma unroll
                for (int i = 0; i < KU; ++i) {
                    const uint32_t ci = cs + (uint32_t)i;
                    uint32_t g0 = 0, nn = 0;
                    if (ci < lb) {  // wave-uniform
                        if (ci >= c_end) {  // the next list holding chunks
                            const int k = (int)__popcll(__ballot(cpn <= ci));
                            c_end = (uint32_t)__builtin_amdgcn_readlane((int)cpn, k);
                            l_base = (uint32_t)__builtin_amdgcn_readlane((int)basel, k);
                            l_end = (uint32_t)__builtin_amdgcn_readlane((int)endl, k);
                            l_w = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wl), k));
                        }
                        g0 = l_base + ci * (uint32_t)kChunk;
                        nn = min((uint32_t)kChunk, l_end - g0);
                        g0 = min(g0, n_groups);
                    }
                    wk[i] = l_w;
                    nl[i] = nn;
                    const uint32_t gi = g0 + (uint32_t)lane;
                    load_at(pd_t, gi * (uint32_t)sizeof(uint2), ids[i]);
                    load_at(pv_t, gi * (uint32_t)sizeof(Raw), raw[i]);
                }
                __builtin_amdgcn_s_setprio(0);
                const uint32_t next = take();  // while this batch's loads are in flight
#pragma unroll
                for (int i = 0; i < KU; ++i) {
                    if ((uint32_t)lane >= nl[i]) continue;
                    const float w = wk[i];
                    // byte offsets of the documents' 32-bit score words
                    const uint32_t d4[4] = {ids[i].x & 0xFFFFu, ids[i].x >> 16, ids[i].y & 0xFFFFu,
                                            ids[i].y >> 16};
#pragma unroll
                    for (int p = 0; p < 4; ++p)
                        lds_add_i32(reinterpret_cast<int32_t *>(smem + d4[p]),
                                    (int32_t)Val<VT>::prod(raw[i], p, w));
                }
                // Every slot's loads are complete here, also those of slots that
                // added nothing: no load of this batch is then still in flight when
                // the next batch (or the next tile's first, behind the list-bounds
                // prefetch) reuses its registers, so those loads never wait.
#pragma unroll
                for (int i = 0; i < KU; ++i) __asm__ volatile("" ::"v"(ids[i].x), "v"(raw[i].x));
                cs = next;
            }
        }
        __syncthreads();
        if (tid < nseg) s_next[tid] = kFirstTaken;  // every wave has taken its last batch of the tile

        // ---- read the row: sample maxima or emit every score at or above the
        // query's threshold (as in k_accumulate)
        if (!SAMPLE && none) {
            for (int m = tid * 4; m < len; m += NT * 4)
                *reinterpret_cast<int4 *>(A32 + m) = fresh_zero4();
        } else if (SAMPLE) {
            int32_t mx = INT32_MIN;
            for (int m = tid; m < len; m += NT) {
                mx = max(mx, A32[m]);
                A32[m] = 0;
            }
            maxima[((size_t)slot * n_sample + ti) * NT + tid] = tid < len ? (float)mx * qinv : -INFINITY;
        } else {
            auto read_out = [&](auto imp_c) {
                constexpr bool IMP = decltype(imp_c)::value;
                const int4 zero = fresh_zero4();  // one per read-out: the loop keeps it live
                // The wave's 256 scores from base; TAIL: some of them may lie past the tile.
                auto step = [&](int base, auto tail_c) {
                    constexpr bool TAIL = decltype(tail_c)::value;
                    const int m0 = base + lane * 4;
                    int4 r = make_int4(0, 0, 0, 0);
                    if (!TAIL || m0 < len) {
                        r = *reinterpret_cast<const int4 *>(A32 + m0);
                        *reinterpret_cast<int4 *>(A32 + m0) = zero;
                    }
                    const bool look = IMP ? ((r.x | r.y | r.z | r.w) != 0)
                                          : max(max(r.x, r.y), max(r.z, r.w)) >= th;
                    if (__ballot(look) == 0) return;  // the common case
                    // threshold <= 0: every nonzero sum, negative ones included (the
                    // finalize kernel takes each document left out as a zero)
                    bool ok[4];
                    ok[0] = (IMP ? r.x != 0 : r.x >= th) && (!TAIL || m0 < len);
                    ok[1] = (IMP ? r.y != 0 : r.y >= th) && (!TAIL || m0 + 1 < len);
                    ok[2] = (IMP ? r.z != 0 : r.z >= th) && (!TAIL || m0 + 2 < len);
                    ok[3] = (IMP ? r.w != 0 : r.w >= th) && (!TAIL || m0 + 3 < len);
                    const float sv[4] = {(float)r.x * qinv, (float)r.y * qinv, (float)r.z * qinv,
                                         (float)r.w * qinv};
                    emit_candidates<4>(sv, ok, d0 + m0, count + slot, cand + (size_t)slot * cap, cap);
                };
                // whole steps without bounds checks, then at most one step across the tile's end
                int base = wave * 256;
                for (; base + 256 <= len; base += NW * 256) step(base, std::false_type{});
                if (base < len) step(base, std::true_type{});
            };
            if (imp)
                read_out(std::true_type{});
            else
                read_out(std::false_type{});
        }
        __syncthreads();
    }
}

// One workgroup per (query slot, tile run): grid (slots, runs), slots fastest, so the
// workgroups resident together score the same tiles.
template <int VT, bool SAMPLE>
__global__ __launch_bounds__(kAccThreads) __attribute__((amdgpu_waves_per_eu(6))) void k_accumulate1(
    DevIndex ix, DevQueries q, DevCoarse c, const int32_t *slot_q, int32_t n_slots,
    int32_t n_sample, float *maxima, const float *theta, uint32_t *count, uint64_t *cand,
    int64_t cap, int32_t tiles_per_wg)
{
    (void)n_slots;
    accumulate1_item<VT, SAMPLE>(ix, q, c, slot_q, n_sample, maxima, theta, count, cand, cap,
                                 tiles_per_wg, (int32_t)blockIdx.x, (int64_t)blockIdx.y, true);
}

// The same work as one persistent launch fed by a device work queue: as many workgroups as
// the device holds at once, each taking the next (slot, tile run) item from a counter until
// the queue is empty.  Items run in the grid's order (tile run major, slots in order), so the
// workgroups resident together still score the same tiles, and a caller that orders its
// slots by decreasing work starts the long queries of each run first.  Every workgroup leaves
// once the counter passes the last item; *head must be 0 at launch.
template <int VT, bool SAMPLE>
__global__ __launch_bounds__(kAccThreads) __attribute__((amdgpu_waves_per_eu(6))) void k_accumulate1_queue(
    DevIndex ix, DevQueries q, DevCoarse c, const int32_t *slot_q, int32_t n_slots,
    int32_t n_sample, float *maxima, const float *theta, uint32_t *count, uint64_t *cand,
    int64_t cap, int32_t tiles_per_wg, int64_t n_items, unsigned long long *head)
{
    __shared__ int64_t s_item;
    bool first = true;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int64_t)atomicAdd(head, 1ull);
        __syncthreads();
        const int64_t it = s_item;
        __syncthreads();  // every thread has the item before thread 0 takes the next
        if (it >= n_items) break;
        accumulate1_item<VT, SAMPLE>(ix, q, c, slot_q, n_sample, maxima, theta, count, cand, cap,
                                     tiles_per_wg, (int32_t)(it % n_slots), it / n_slots, first);
        first = false;
    }
}

// ------------------------------------------------------------------ threshold
// theta = the rank-th largest sampled maximum.  Both accumulate passes
// produce bitwise identical scores (integer sums), so every sampled document
// at or above theta is kept again by the scoring pass.  The finalize kernel
// verifies the result (at least gamma candidates kept).
__global__ __launch_bounds__(kThetaThreads) void k_theta(const float *maxima, int64_t n_m,
                                                       int64_t rank, float *theta)
{
    __shared__ uint32_t hist[256];
    __shared__ int s_digit;
    __shared__ int64_t s_need;
    const float *mx = maxima + (size_t)blockIdx.x * (size_t)n_m;
    const uint32_t key = block_select<uint32_t>(
        n_m, rank, [&](int64_t i) { return ord_f32(mx[i]); }, hist, &s_digit, &s_need);
    if (threadIdx.x == 0) {
        const float th = unord_f32(key);
        theta[blockIdx.x] = th > -INFINITY ? th : -INFINITY;
    }
}

__global__ void k_fill_f32(float *p, int64_t n, float v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_iota_i32(int32_t *p, int32_t n, int32_t first)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = first + i;
}

// Rows whose status is not kSlotOk, in order: of rows [0, n) (in_rows null)
// or of in_rows[0, n).  One workgroup; writes the count last.
__global__ __launch_bounds__(1024) void k_collect_failed(const int32_t *status,
                                                         const int32_t *in_rows, int32_t n,
                                                         int32_t *out_rows, uint32_t *count)
{
    __shared__ uint32_t s_wsum[1024 / kWave];
    uint32_t base = 0;
    for (int32_t i0 = 0; i0 < n; i0 += 1024) {
        const int32_t i = i0 + (int32_t)threadIdx.x;
        int32_t row = 0;
        uint32_t bad = 0;
        if (i < n) {
            row = in_rows ? in_rows[i] : i;
            bad = status[row] != kSlotOk ? 1u : 0u;
        }
        uint32_t tot;
        const uint32_t pos = block_excl_scan<1024>(bad, s_wsum, tot);
        if (bad) out_rows[base + pos] = row;
        base += tot;
    }
    if (threadIdx.x == 0) *count = base;
}

// ------------------------------------------------------------------ finalize
struct QueryHash {
    int32_t *id;
    float *val;
    int32_t *pos;
    int lg;
};

// Full (unpruned) query row into an open-addressing LDS table.
__device__ void build_query_hash(const DevQueries &q, int64_t a, int64_t b, QueryHash h)
{
    const int H = 1 << h.lg;
    for (int i = threadIdx.x; i < H; i += blockDim.x) h.id[i] = -1;
    __syncthreads();
    for (int64_t e = a + threadIdx.x; e < b; e += blockDim.x) {
        const int32_t id = q.indices[e];
        uint32_t s = hash_slot(id, h.lg);
        while (atomicCAS(&h.id[s], -1, id) != -1) s = (s + 1) & (uint32_t)(H - 1);
        h.val[s] = q.values[e];
        if (h.pos) h.pos[s] = (int32_t)(e - a);
    }
    __syncthreads();
}

__device__ __forceinline__ int probe(const QueryHash &h, int32_t id)
{
    const uint32_t mask = (1u << h.lg) - 1u;
    uint32_t s = hash_slot(id, h.lg);
    for (;;) {
        const int32_t k = h.id[s];
        if (k == id) return (int)s;
        if (k == -1) return -1;
        s = (s + 1) & mask;
    }
}

__host__ __device__ __forceinline__ int hash_lg(int64_t n)
{
    int lg = 6;
    while ((1ll << lg) < 2 * n) ++lg;
    return lg;
}

// delta(q, x_doc) in FP32 by one wave over the document's row.
__device__ __forceinline__ float wave_dot(const DevIndex &ix, const QueryHash &h, uint32_t doc)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t ra = ix.indptr[doc], rb = ix.indptr[doc + 1];
    float acc = 0.0f;
    for (int64_t e = ra + lane; e < rb; e += kWave) {
        const int s = probe(h, ix.indices[e]);
        if (s >= 0) acc = fmaf(h.val[s], ix.values[e], acc);
    }
    return wave_sum(acc);
}

// LDS sizes: P = the power of two at or above need keys, a rerank table of
// 2^hlg slots, hlg = hash_lg of the longest query row of the launch.
__host__ __device__ inline int32_t pow2_at_least(int32_t n)
{
    int32_t p = 1;
    while (p < n) p <<= 1;
    return p;
}

// Sort need keys (score bits, then inverted id) in LDS descending and write
// the first k as (id, score) to the query's output row, padded with (-1, -inf).
__device__ void sort_and_write(uint64_t *keys, int32_t need, int32_t k, int32_t row,
                               int64_t *out_ids, float *out_scores)
{
    constexpr int NT = kFinThreads;
    const int tid = threadIdx.x;
    const int32_t P = pow2_at_least(need);
    for (int i = need + tid; i < P; i += NT) keys[i] = 0ull;
    __syncthreads();
    for (int kk = 2; kk <= P; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < P; i += NT) {
                const int ij = i ^ j;
                if (ij > i) {
                    const uint64_t x = keys[i], y = keys[ij];
                    const bool desc = (i & kk) == 0;
                    if (desc ? (x < y) : (x > y)) {
                        keys[i] = y;
                        keys[ij] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int r = tid; r < k; r += NT) {
        const size_t o = (size_t)row * (size_t)k + r;
        if (r < need) {
            out_ids[o] = (int64_t)key_doc(keys[r]);
            out_scores[o] = key_score(keys[r]);
        } else {
            out_ids[o] = -1;
            out_scores[o] = -INFINITY;
        }
    }
}

// One workgroup per query slot: the exact top-need of its coarse candidates
// (with the zero-score documents the scoring pass left implicit).  Without a
// rerank it sorts them and writes the top k; with a rerank it writes them to
// pool[slot][need] for k_rerank and k_topk.
template <bool RERANK>
__global__ __launch_bounds__(kFinThreads) void k_finalize(
    DevIndex ix, const int32_t *slot_q, const uint32_t *count, const uint64_t *cand,
    const float *theta, int64_t cap, int32_t need, int32_t k, int32_t bm_words, uint64_t *pool,
    int64_t *out_ids, float *out_scores, int32_t *status)
{
    constexpr int NT = kFinThreads, NW = NT / kWave;
    extern __shared__ __align__(16) unsigned char smem[];
    const int32_t P = pow2_at_least(need);
    uint64_t *keys = reinterpret_cast<uint64_t *>(smem);                   // [P]
    uint32_t *bm = reinterpret_cast<uint32_t *>(keys + P);                  // [bm_words]
    __shared__ uint32_t hist[256];
    __shared__ uint32_t s_n, s_wsum[NW];
    __shared__ int s_digit;
    __shared__ int64_t s_need;
    const int tid = threadIdx.x;
    const int32_t slot = blockIdx.x;
    const int32_t row = slot_q ? slot_q[slot] : slot;
    const uint32_t cnt = count[slot];
    const float th = theta ? theta[slot] : -INFINITY;
    // threshold <= 0: the scoring pass emitted only nonzero sums; every document it did
    // not emit scores exactly 0
    const bool imp = th <= 0.0f && th != -INFINITY;
    if ((int64_t)cnt > cap || (!imp && (int64_t)cnt < (int64_t)need)) {
        if (tid == 0) status[row] = kSlotRetry;
        return;
    }
    const uint64_t *cs = cand + (size_t)slot * (size_t)cap;
    constexpr uint32_t kZeroOrd = 0x80000000u;  // ord_f32(0.0f)
    uint32_t n_pos = (uint32_t)cnt;
    if (imp) {
        uint32_t mine = 0;
        for (int64_t i = tid; i < cnt; i += NT) mine += (uint32_t)(cs[i] >> 32) > kZeroOrd ? 1u : 0u;
        (void)block_excl_scan<NT>(mine, s_wsum, n_pos);
    }
    if (tid == 0) s_n = 0;
    if (!imp || (int64_t)n_pos >= (int64_t)need) {
        // the first need candidates (all positive when zeros are implicit)
        const uint64_t kth = block_select<uint64_t>(
            cnt, need, [&](int64_t i) { return cs[i]; }, hist, &s_digit, &s_need);
        __syncthreads();
        for (int64_t i = tid; i < cnt; i += NT) {
            const uint64_t key = cs[i];
            if (key >= kth) {
                const uint32_t p = atomicAdd(&s_n, 1u);
                if (p < (uint32_t)P) keys[p] = key;
            }
        }
        __syncthreads();
    } else {
        // every positive candidate, then the lowest-id zero-score documents, then (only if
        // the zeros run out) the best emitted negatives
        const int64_t zeros_avail = ix.n_docs - (int64_t)cnt;
        const int64_t zt = min((int64_t)need - n_pos, zeros_avail);
        const int64_t nt = (int64_t)need - n_pos - zt;
        const int64_t bound = min(ix.n_docs, zt + (int64_t)cnt);  // the zt-th zero id is below
        const int32_t words = (int32_t)((bound + 31) / 32);
        if (nt > (int64_t)cnt - n_pos || words > bm_words) {
            if (tid == 0) status[row] = kSlotRetry;
            return;
        }
        __syncthreads();
        for (int64_t i = tid; i < cnt; i += NT) {
            const uint64_t key = cs[i];
            if ((uint32_t)(key >> 32) > kZeroOrd) keys[atomicAdd(&s_n, 1u)] = key;
        }
        for (int w = tid; w < words; w += NT) bm[w] = 0u;
        __syncthreads();
        for (int64_t i = tid; i < cnt; i += NT) {
            const uint32_t d = key_doc(cs[i]);
            if ((int64_t)d < bound) atomicOr(&bm[d >> 5], 1u << (d & 31));
        }
        __syncthreads();
        // zero bits in order: each thread owns a run of words
        const int32_t per = (words + NT - 1) / NT;
        const int32_t w0 = min(words, tid * per), w1 = min(words, w0 + per);
        auto free_bits = [&](int32_t w) {
            uint32_t m = ~bm[w];
            const int64_t top = bound - (int64_t)w * 32;  // valid bits in this word
            if (top < 32) m &= (1u << top) - 1u;
            return m;
        };
        uint32_t mine = 0;
        for (int32_t w = w0; w < w1; ++w) mine += (uint32_t)__popc(free_bits(w));
        uint32_t tot;
        uint32_t rank = block_excl_scan<NT>(mine, s_wsum, tot);
        for (int32_t w = w0; w < w1 && (int64_t)rank < zt; ++w) {
            uint32_t m = free_bits(w);
            while (m && (int64_t)rank < zt) {
                const int b = __ffs(m) - 1;
                m &= m - 1u;
                keys[n_pos + rank] = make_key(0.0f, (uint32_t)(w * 32 + b));
                ++rank;
            }
        }
        if (nt > 0) {
            // the nt best negatives: non-negative keys map to 0 and rank below them
            const uint64_t kthn = block_select<uint64_t>(
                cnt, nt,
                [&](int64_t i) {
                    const uint64_t key = cs[i];
                    return (uint32_t)(key >> 32) < kZeroOrd ? key : 0ull;
                },
                hist, &s_digit, &s_need);
            if (tid == 0) s_n = 0;
            __syncthreads();
            for (int64_t i = tid; i < cnt; i += NT) {
                const uint64_t key = cs[i];
                if ((uint32_t)(key >> 32) < kZeroOrd && key >= kthn)
                    keys[n_pos + zt + atomicAdd(&s_n, 1u)] = key;
            }
        }
        __syncthreads();
    }

    if (RERANK) {
        for (int i = tid; i < need; i += NT) pool[(size_t)slot * (size_t)need + i] = keys[i];
        if (tid == 0) status[row] = kSlotOk;
        return;
    }
    sort_and_write(keys, need, k, row, out_ids, out_scores);
    if (tid == 0) status[row] = kSlotOk;
}

// Exact rerank (Alg. 4): each wave scores kRerankPerWave pool entries at a
// time, kRerankGroups times, NW waves per workgroup, grid (slot, entry block);
// each workgroup builds the query's hash in LDS (2^hlg slots) once for its
// kRerankGroups x NW x kRerankPerWave entries.  The entry's key becomes (FP32
// inner product of the unpruned row with the full query, then inverted id).
// Slots not finalized are skipped.
__global__ __launch_bounds__(kFinThreads) void k_rerank(DevIndex ix, DevQueries q,
                                                        const int32_t *slot_q, int32_t need,
                                                        int32_t hlg, uint64_t *pool,
                                                        int32_t *status)
{
    constexpr int NW = kFinThreads / kWave, EPW = kRerankPerWave;
    extern __shared__ __align__(16) unsigned char smem[];
    int32_t *hid = reinterpret_cast<int32_t *>(smem);          // [2^hlg]
    float *hval = reinterpret_cast<float *>(hid + (1 << hlg));  // [2^hlg]
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int32_t slot = blockIdx.x;
    const int32_t row = slot_q ? slot_q[slot] : slot;
    if (status[row] != kSlotOk) return;
    const int64_t qa = q.indptr[row], qb = q.indptr[row + 1];
    const int lg = hash_lg(qb - qa);
    if (lg > hlg) {  // the launch was sized for shorter rows
        if (threadIdx.x == 0 && blockIdx.y == 0) status[row] = kSlotRetry;
        return;
    }
    const QueryHash h{hid, hval, nullptr, lg};
    uint64_t *e = pool + (size_t)slot * (size_t)need;
    uint32_t lo[EPW];
    int64_t ra[EPW], rb[EPW];
    // keys and row bounds of the wave's entries [c0, c0 + EPW)
    auto bounds = [&](int32_t c0) {
#pragma unroll
        for (int j = 0; j < EPW; ++j) {
            lo[j] = 0;
            ra[j] = rb[j] = 0;
            if (c0 + j < need) {
                const uint64_t key = e[c0 + j];
                lo[j] = (uint32_t)key;
                const uint32_t doc = key_doc(key);
                ra[j] = ix.indptr[doc];
                rb[j] = ix.indptr[doc + 1];
            }
        }
    };
    // The first group's keys and row bounds are loaded before the query table is
    // built, and the first two 64-entry rounds of every row of a group are loaded
    // together, so the entries' memory latencies overlap.
    const int32_t first = (int32_t)blockIdx.y * kRerankGroups * NW;
    bounds((first + wave) * EPW);
    build_query_hash(q, qa, qb, h);
    for (int g = 0; g < kRerankGroups; ++g) {
        const int32_t c0 = (first + g * NW + wave) * EPW;
        if (c0 >= need) break;  // wave-uniform; no barrier follows
        if (g > 0) bounds(c0);
        int32_t id[EPW][2];
        float xv[EPW][2];
#pragma unroll
        for (int j = 0; j < EPW; ++j)
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int64_t p = ra[j] + r * kWave + lane;
                id[j][r] = -1;
                xv[j][r] = 0.0f;
                if (p < rb[j]) {
                    id[j][r] = ix.indices[p];
                    xv[j][r] = ix.values[p];
                }
            }
        // delta(q, x_doc) in FP32, each lane over entries lane, lane + 64, ... of the
        // row in order, then summed across the wave
#pragma unroll
        for (int j = 0; j < EPW; ++j) {
            float acc = 0.0f;
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                if (id[j][r] < 0) continue;
                const int sl = probe(h, id[j][r]);
                if (sl >= 0) acc = fmaf(h.val[sl], xv[j][r], acc);
            }
            for (int64_t p = ra[j] + 2 * kWave + lane; p < rb[j]; p += kWave) {
                const int sl = probe(h, ix.indices[p]);
                if (sl >= 0) acc = fmaf(h.val[sl], ix.values[p], acc);
            }
            const float sc = wave_sum(acc);
            if (c0 + j < need && lane == 0) e[c0 + j] = ((uint64_t)ord_f32(sc) << 32) | lo[j];
        }
    }
}

// One workgroup per slot: sort the reranked pool and write the top k.
__global__ __launch_bounds__(kFinThreads) void k_topk(const int32_t *slot_q, int32_t need,
                                                      int32_t k, const uint64_t *pool,
                                                      int64_t *out_ids, float *out_scores,
                                                      const int32_t *status)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t *keys = reinterpret_cast<uint64_t *>(smem);  // [pow2_at_least(need)]
    const int32_t slot = blockIdx.x;
    const int32_t row = slot_q ? slot_q[slot] : slot;
    if (status[row] != kSlotOk) return;
    for (int i = threadIdx.x; i < need; i += kFinThreads)
        keys[i] = pool[(size_t)slot * (size_t)need + i];
    sort_and_write(keys, need, k, row, out_ids, out_scores);
}

// ------------------------------------------------------------------ pair scores
__global__ __launch_bounds__(kFinThreads) void k_score_forward(DevIndex ix, DevQueries q,
                                                               const int64_t *cand,
                                                               int32_t n_cand, float *out)
{
    constexpr int NW = kFinThreads / kWave;
    extern __shared__ __align__(16) unsigned char smem[];
    int32_t *hid = reinterpret_cast<int32_t *>(smem);
    float *hval = reinterpret_cast<float *>(hid + kQueryHash);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int64_t b = blockIdx.x;
    const int64_t qa = q.indptr[b], qb = q.indptr[b + 1];
    const QueryHash h{hid, hval, nullptr, hash_lg(qb - qa)};
    build_query_hash(q, qa, qb, h);
    for (int c = wave; c < n_cand; c += NW) {
        const int64_t d = cand[b * n_cand + c];
        float s = 0.0f;
        if (d >= 0 && d < ix.n_docs) s = wave_dot(ix, h, (uint32_t)d);
        if (lane == 0) out[b * n_cand + c] = s;
    }
}

// Gradients of s[b][c] = delta(q_b, x_c): every common dimension t adds
// G[b][c] * x_c[t] to the query entry and G[b][c] * q_b[t] to the document
// entry.  Query-side sums stay in LDS (one workgroup per query); document
// entries can be shared by several queries, so they take global atomics.
__global__ __launch_bounds__(kFinThreads) void k_score_backward(
    DevIndex ix, DevQueries q, const int64_t *cand, int32_t n_cand, const float *grad, float *gq,
    float *gx)
{
    constexpr int NW = kFinThreads / kWave;
    extern __shared__ __align__(16) unsigned char smem[];
    int32_t *hid = reinterpret_cast<int32_t *>(smem);
    float *hval = reinterpret_cast<float *>(hid + kQueryHash);
    int32_t *hpos = reinterpret_cast<int32_t *>(hval + kQueryHash);
    float *gacc = reinterpret_cast<float *>(hpos + kQueryHash);
    uint32_t *gtouch = reinterpret_cast<uint32_t *>(gacc + kQueryHash / 2);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int64_t b = blockIdx.x;
    const int64_t qa = q.indptr[b], qb = q.indptr[b + 1];
    const int n = (int)(qb - qa);
    const QueryHash h{hid, hval, hpos, hash_lg(n)};
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        gacc[i] = 0.0f;
        gtouch[i] = 0u;
    }
    build_query_hash(q, qa, qb, h);
    for (int c = wave; c < n_cand; c += NW) {
        const int64_t d = cand[b * n_cand + c];
        if (d < 0 || d >= ix.n_docs) continue;
        const float g = grad[b * n_cand + c];
        const int64_t ra = ix.indptr[d], rb = ix.indptr[d + 1];
        for (int64_t e = ra + lane; e < rb; e += kWave) {
            const int s = probe(h, ix.indices[e]);
            if (s < 0) continue;
            if (gq) {
                lds_add(&gacc[hpos[s]], g * ix.values[e]);
                gtouch[hpos[s]] = 1u;
            }
            if (gx) atomicAdd(&gx[e], g * hval[s]);
        }
    }
    __syncthreads();
    if (gq)
        for (int i = threadIdx.x; i < n; i += blockDim.x)
            if (gtouch[i]) gq[qa + i] += gacc[i];
}

template <typename F>
hipError_t set_lds(F *kernel, size_t bytes)
{
    return allow_lds(reinterpret_cast<const void *>(kernel), bytes);
}

// Workgroups of `kernel` (kAccThreads threads, `lds` bytes of dynamic LDS) the device holds
// at once, looked up once per (device, kernel, lds).
template <typename F>
hipError_t resident_workgroups(F *kernel, size_t lds, int64_t *out)
{
    static std::mutex mu;
    static std::map<std::tuple<int, const void *, size_t>, int64_t> known;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_tuple(dev, reinterpret_cast<const void *>(kernel), lds);
    auto it = known.find(key);
    if (it == known.end()) {
        int per_cu = 0, cus = 0;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kAccThreads, lds)) != hipSuccess)
            return e;
        if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
            return e;
        it = known.emplace(key, std::max<int64_t>(1, (int64_t)per_cu * cus)).first;
    }
    *out = it->second;
    return hipSuccess;
}

template <int VT, int B, bool SAMPLE>
hipError_t run_accumulate(const DevIndex &ix, const DevQueries &q, const DevCoarse &c,
                          const int32_t *slot_q, int32_t n_slots, int32_t n_sample, float *maxima,
                          const float *theta, uint32_t *count, uint64_t *cand, int64_t cap,
                          int32_t tiles_per_wg, int32_t max_terms, unsigned long long *queue,
                          hipStream_t s)
{
    const int eb = entry_block(B, max_terms);
    const size_t lds = accumulate_lds_bytes(B, ix.tile_stride, eb);
    hipError_t e;
    if constexpr (B == 1)
        e = set_lds(k_accumulate1<VT, SAMPLE>, lds);
    else
        e = set_lds(k_accumulate<VT, B, SAMPLE>, lds);
    if (e != hipSuccess) return e;
    const int64_t n_batches = (n_slots + B - 1) / B;
    const int64_t n_iter = SAMPLE ? n_sample : ix.n_tiles;
    // Contiguous tile ranges per workgroup (see the kernel); the range length
    // keeps the grid at least a few times the chip's resident workgroups.
    int64_t per = tiles_per_wg > 0 ? tiles_per_wg : 12;
    while (per > 1 && n_batches * ((n_iter + per - 1) / per) < 4096) per >>= 1;
    int64_t groups = (n_iter + per - 1) / per;
    if (groups > 65535) {
        groups = 65535;
        per = (n_iter + groups - 1) / groups;
        groups = (n_iter + per - 1) / per;
    }
    dim3 grid((unsigned)n_batches, (unsigned)groups);
    if constexpr (B == 1) {
        if (queue) {  // one persistent launch over the (slot, run) items
            if ((e = set_lds(k_accumulate1_queue<VT, SAMPLE>, lds)) != hipSuccess) return e;
            int64_t wgs = 0;
            if ((e = resident_workgroups(k_accumulate1_queue<VT, SAMPLE>, lds, &wgs)) != hipSuccess)
                return e;
            const int64_t n_items = n_batches * groups;
            hipLaunchKernelGGL((k_accumulate1_queue<VT, SAMPLE>), dim3((unsigned)std::min(wgs, n_items)),
                               dim3(kAccThreads), lds, s, ix, q, c, slot_q, n_slots, n_sample,
                               maxima, theta, count, cand, cap, (int32_t)per, n_items, queue);
            return hipGetLastError();
        }
        hipLaunchKernelGGL((k_accumulate1<VT, SAMPLE>), grid, dim3(kAccThreads), lds, s, ix, q, c,
                           slot_q, n_slots, n_sample, maxima, theta, count, cand, cap, (int32_t)per);
    } else {
        hipLaunchKernelGGL((k_accumulate<VT, B, SAMPLE>), grid, dim3(kAccThreads), lds, s, ix, q, c,
                           slot_q, n_slots, n_sample, maxima, theta, count, cand, cap, (int32_t)per,
                           (int32_t)eb);
    }
    return hipGetLastError();
}

template <int VT, bool SAMPLE>
hipError_t dispatch_b(int batch, const DevIndex &ix, const DevQueries &q, const DevCoarse &c,
                      const int32_t *slot_q, int32_t n_slots, int32_t n_sample, float *maxima,
                      const float *theta, uint32_t *count, uint64_t *cand, int64_t cap,
                      int32_t tiles_per_wg, int32_t max_terms, unsigned long long *queue,
                      hipStream_t s)
{
    switch (batch) {
    case 1: return run_accumulate<VT, 1, SAMPLE>(ix, q, c, slot_q, n_slots, n_sample, maxima, theta, count, cand, cap, tiles_per_wg, max_terms, queue, s);
    case 2: return run_accumulate<VT, 2, SAMPLE>(ix, q, c, slot_q, n_slots, n_sample, maxima, theta, count, cand, cap, tiles_per_wg, max_terms, nullptr, s);
    case 4: return run_accumulate<VT, 4, SAMPLE>(ix, q, c, slot_q, n_slots, n_sample, maxima, theta, count, cand, cap, tiles_per_wg, max_terms, nullptr, s);
    case 8: return run_accumulate<VT, 8, SAMPLE>(ix, q, c, slot_q, n_slots, n_sample, maxima, theta, count, cand, cap, tiles_per_wg, max_terms, nullptr, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t allow_lds(const void *kernel, size_t bytes)
{
    static std::mutex mu;
    static std::map<std::pair<int, const void *>, size_t> limit;  // (device, kernel) -> bytes
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    auto it = limit.find({dev, kernel});
    if (it == limit.end()) {
        int max = 0;
        hipFuncAttributes fa{};
        if ((e = hipDeviceGetAttribute(&max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess)
            return e;
        if ((e = hipFuncGetAttributes(&fa, kernel)) != hipSuccess) return e;
        const size_t lim = (size_t)max > fa.sharedSizeBytes ? (size_t)max - fa.sharedSizeBytes : 0;
        if ((e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim)) !=
            hipSuccess)
            return e;
        it = limit.emplace(std::make_pair(dev, kernel), lim).first;
    }
    return bytes <= it->second ? hipSuccess : hipErrorInvalidValue;
}

hipError_t launch_query_prep(const DevQueries &q, int64_t n_cols, double beta, DevCoarse c,
                             const float *term_max, double *scratch_abs, int32_t *err_flag,
                             hipStream_t s)
{
    if (q.n_rows == 0) return hipSuccess;
    dim3 grid((unsigned)((q.n_rows + 3) / 4));
    hipLaunchKernelGGL(k_query_prep, grid, dim3(256), 0, s, q, n_cols, beta, c, term_max,
                       scratch_abs, err_flag);
    return hipGetLastError();
}

hipError_t launch_accumulate(const DevIndex &ix, const DevQueries &q, const DevCoarse &c,
                             int batch, bool sample, const int32_t *slot_q, int32_t n_slots,
                             int32_t n_sample_tiles, float *maxima, const float *theta,
                             uint32_t *count, uint64_t *cand, int64_t cap, int32_t tiles_per_wg,
                             int32_t max_terms, unsigned long long *queue, hipStream_t s)
{
    if (n_slots == 0 || ix.n_tiles == 0) return hipSuccess;
    const int vt = ix.value_dtype;
    if (sample) {
        if (vt == 0) return dispatch_b<0, true>(batch, ix, q, c, slot_q, n_slots, n_sample_tiles, maxima, theta, count, cand, cap, tiles_per_wg, max_terms, queue, s);
        if (vt == 1) return dispatch_b<1, true>(batch, ix, q, c, slot_q, n_slots, n_sample_tiles, maxima, theta, count, cand, cap, tiles_per_wg, max_terms, queue, s);
        return dispatch_b<2, true>(batch, ix, q, c, slot_q, n_slots, n_sample_tiles, maxima, theta, count, cand, cap, tiles_per_wg, max_terms, queue, s);
    }
    if (vt == 0) return dispatch_b<0, false>(batch, ix, q, c, slot_q, n_slots, n_sample_tiles, maxima, theta, count, cand, cap, tiles_per_wg, max_terms, queue, s);
    if (vt == 1) return dispatch_b<1, false>(batch, ix, q, c, slot_q, n_slots, n_sample_tiles, maxima, theta, count, cand, cap, tiles_per_wg, max_terms, queue, s);
    return dispatch_b<2, false>(batch, ix, q, c, slot_q, n_slots, n_sample_tiles, maxima, theta, count, cand, cap, tiles_per_wg, max_terms, queue, s);
}

hipError_t launch_theta(const float *maxima, int64_t n_maxima, int64_t rank, int32_t n_slots,
                        float *theta, hipStream_t s)
{
    if (n_slots == 0) return hipSuccess;
    hipLaunchKernelGGL(k_theta, dim3((unsigned)n_slots), dim3(kThetaThreads), 0, s, maxima,
                       n_maxima, rank, theta);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_iota(int32_t *p, int32_t n, int32_t first, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int32_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_iota_i32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, first);
    return hipGetLastError();
}

hipError_t launch_collect_failed(const int32_t *status, const int32_t *in_rows, int32_t n,
                                 int32_t *out_rows, uint32_t *count, hipStream_t s)
{
    hipLaunchKernelGGL(k_collect_failed, dim3(1), dim3(1024), 0, s, status, in_rows, n, out_rows,
                       count);
    return hipGetLastError();
}

hipError_t launch_finalize(const DevIndex &ix, const DevQueries &q, const int32_t *slot_q,
                           int32_t n_slots, const uint32_t *count, const uint64_t *cand,
                           const float *theta, int64_t cap, int32_t need, int32_t k, bool rerank,
                           int32_t max_qnnz, uint64_t *pool, int64_t *out_ids, float *out_scores,
                           int32_t *status, hipStream_t s)
{
    if (n_slots == 0) return hipSuccess;
    // bitmap of candidate ids below need + cap: zero-score documents in id order
    const int64_t bm = theta ? (need + cap + 31) / 32 : 0;
    if (bm > (int64_t)1 << 20) return hipErrorInvalidValue;
    const size_t keys = (size_t)pow2_at_least(need) * 8;
    const size_t lds = keys + (size_t)bm * 4;
    hipError_t e;
    if (!rerank) {
        e = set_lds(k_finalize<false>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_finalize<false>, dim3((unsigned)n_slots), dim3(kFinThreads), lds, s,
                           ix, slot_q, count, cand, theta, cap, need, k, (int32_t)bm, nullptr,
                           out_ids, out_scores, status);
        return hipGetLastError();
    }
    if (!pool) return hipErrorInvalidValue;
    e = set_lds(k_finalize<true>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_finalize<true>, dim3((unsigned)n_slots), dim3(kFinThreads), lds, s, ix,
                       slot_q, count, cand, theta, cap, need, k, (int32_t)bm, pool, out_ids,
                       out_scores, status);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int32_t hlg = hash_lg(max_qnnz > 0 ? max_qnnz : 1);
    const size_t lds_h = ((size_t)1 << hlg) * 8;
    e = set_lds(k_rerank, lds_h);
    if (e != hipSuccess) return e;
    constexpr int PER_WG = kFinThreads / kWave * kRerankPerWave * kRerankGroups;
    hipLaunchKernelGGL(k_rerank, dim3((unsigned)n_slots, (unsigned)((need + PER_WG - 1) / PER_WG)),
                       dim3(kFinThreads), lds_h, s, ix, q, slot_q, need, hlg, pool, status);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = set_lds(k_topk, keys);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_topk, dim3((unsigned)n_slots), dim3(kFinThreads), keys, s, slot_q, need,
                       k, pool, out_ids, out_scores, status);
    return hipGetLastError();
}

hipError_t launch_score_forward(const DevIndex &ix, const DevQueries &q, const int64_t *cand,
                                int32_t n_cand, float *out, hipStream_t s)
{
    if (q.n_rows == 0 || n_cand == 0) return hipSuccess;
    const size_t lds = (size_t)kQueryHash * 8;
    hipError_t e = set_lds(k_score_forward, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_score_forward, dim3((unsigned)q.n_rows), dim3(kFinThreads), lds, s, ix,
                       q, cand, n_cand, out);
    return hipGetLastError();
}

hipError_t launch_score_backward(const DevIndex &ix, const DevQueries &q, const int64_t *cand,
                                 int32_t n_cand, const float *grad, float *gq, float *gx,
                                 hipStream_t s)
{
    if (q.n_rows == 0 || n_cand == 0) return hipSuccess;
    const size_t lds = (size_t)kQueryHash * 12 + (size_t)(kQueryHash / 2) * 8;
    hipError_t e = set_lds(k_score_backward, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_score_backward, dim3((unsigned)q.n_rows), dim3(kFinThreads), lds, s, ix,
                       q, cand, n_cand, grad, gq, gx);
    return hipGetLastError();
}

}  // namespace sindi
