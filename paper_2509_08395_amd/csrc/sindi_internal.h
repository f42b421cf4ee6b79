// Internal declarations shared by the host side and the gfx950 kernels of the
// SINDI library.  Not part of the C ABI (include/sindi.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sindi {

// Device view of a built index: the value-storing lists of Alg. 1 cut into
// score tiles (each window of Sec. 3.3.1 split into equal tiles), plus the
// unpruned corpus kept for the exact rerank of Alg. 4.
struct DevIndex {
    int64_t n_docs, n_cols, n_tiles;
    int32_t tile_stride;           // words per query row of the on-chip score tile (>= tile_max, %4 == 0)
    int32_t value_dtype;           // sindi_dtype
    const int64_t *tile_doc;       // [n_tiles + 1] first document of each tile
    const int64_t *tile_post;      // [n_tiles + 1] first posting slot of each tile (multiple of 4)
    const uint32_t *term_goff;     // [n_tiles * (n_cols + 1)] list (term, tile) starts at 4-posting
                                   // group (term_goff & kGoffMask) of the tile and ends, pads
                                   // included, where the next term's list starts; top 2 bits:
                                   // pad entries at its end
    const uint16_t *post_doc;      // [n_slots + kTailSlots] 4 * (document id - tile_doc[t]): the
                                   // byte offset of the document's score word in a row; pads
                                   // repeat the list's largest; each chunk of kChunk groups in
                                   // LDS-bank order (build_deal_chunks)
    const void *post_val;          // [n_slots + kTailSlots] value (f32 / f16 / bf16 bits); pads
                                   // and the tail hold 0
    const float *term_max;         // [n_cols] largest |stored value| in the term's lists
    const int64_t *indptr;         // unpruned corpus CSR, [n_docs + 1]
    const int32_t *indices;        // [nnz]
    const float *values;           // [nnz]
    int64_t nnz;
};

// Queries as the device kernels see them.
struct DevQueries {
    int64_t n_rows, nnz;
    const int64_t *indptr;
    const int32_t *indices;
    const float *values;
};

// Per-query coarse terms (beta-mass subvector, ascending term id), stored at
// the query row's own positions: terms ct[indptr[q] + i], weights cw[...],
// i < cn[q].  Coarse scores are accumulated as 32-bit integers in units of
// 1/scale_q, scale_q a power of two with scale_q * sum_i |q_i| max|x_i| <=
// 2^30, so no partial sum can overflow; cw holds q_i * scale_q and
// qinv[q] = 1 / scale_q.
struct DevCoarse {
    int32_t *ct;
    float *cw;
    int32_t *cn;
    float *qinv;
};

constexpr int kAccThreads = 512;       // accumulate kernel workgroup
constexpr int kFinThreads = 256;       // finalize, rerank and top-k kernels
constexpr int kThetaThreads = 1024;    // threshold kernel (one radix select per query)
constexpr int kGammaMax = 4096;        // largest reorder pool
constexpr int kQueryHash = 8192;       // rerank hash slots (query nnz <= kQueryHash / 2)
constexpr int kEntryBlock = 512;       // (query, term) entries merged per pass in the accumulate kernel
constexpr int kChunk = 64;             // 4-posting groups per list chunk (one per lane)
constexpr uint32_t kGoffMask = 0x3FFFFFFFu;
// Most 4-posting groups in one tile: a chunk addresses its groups by 32-bit
// byte offsets from the tile's first group (16 B per group for FP32 values),
// and may read up to kChunk - 1 groups past a list's end.
constexpr uint32_t kTileGroupsMax = (1u << 28) - kChunk;
// Zero postings after the last slot, so those reads stay inside the arrays.
constexpr int kTailSlots = 4 * kChunk;
constexpr int kTileMax = 16384;        // documents per tile (4 * local id fits 16 bits)
constexpr int kLongRow = 8192;         // longest corpus row of the device build
constexpr int kFillTerms = 32768;      // list cursors per pass of the device build's fill

// LDS of one accumulate workgroup: the score rows A[batch][tile_stride], for
// batch >= 2 the merged term list (ids + one weight per query, eb entries per
// merge pass) and a region that first holds the merge sort keys, then the
// tile's non-empty lists (first group, end, first chunk, weights).  A single
// query needs its score row only: its waves lay out the tile's lists in
// registers.
constexpr size_t accumulate_lds_bytes(int batch, int tile_stride, int eb = kEntryBlock)
{
    if (batch == 1) return (size_t)tile_stride * 4;
    const size_t lists = ((size_t)3 * eb + 4) * 4 + (size_t)eb * batch * 4;
    const size_t merge = (size_t)eb * 12;
    return (size_t)batch * tile_stride * 4 + (size_t)eb * 4 + (size_t)eb * batch * 4 +
           (merge > lists ? merge : lists);
}

// Entries merged per pass for a batch of `batch` queries of at most
// `max_terms` coarse terms each: a power of two in [64, kEntryBlock] (more
// entries take several passes), so short queries leave LDS for larger tiles.
inline int entry_block(int batch, int64_t max_terms)
{
    int eb = 64;
    while (eb < kEntryBlock && (int64_t)eb < (int64_t)batch * max_terms) eb <<= 1;
    return eb;
}

// Status codes written per query slot by the finalize kernel.
enum SlotStatus : int32_t { kSlotOk = 0, kSlotRetry = 1 };

// Lets `kernel` take up to the device's per-workgroup LDS (less its static
// LDS) as dynamic LDS, set once per device and kernel, so launches of any size
// from several threads never lower each other's limit; fails if `bytes` is
// beyond it.
hipError_t allow_lds(const void *kernel, size_t bytes);

// Kernel launchers (sindi_kernels.hip).  All return hipGetLastError().
// err_flag[0]: malformed-row bits, err_flag[1]: longest well-formed row (both
// must be zero on entry).
hipError_t launch_query_prep(const DevQueries &q, int64_t n_cols, double beta, DevCoarse c,
                             const float *term_max, double *scratch_abs, int32_t *err_flag,
                             hipStream_t s);

// queue: null launches one workgroup per (slot, tile run); otherwise (one query per
// workgroup only) one persistent launch of the device's resident workgroups takes the items
// from the 8-byte counter *queue, which must be zero when the launch starts.
hipError_t launch_accumulate(const DevIndex &ix, const DevQueries &q, const DevCoarse &c,
                             int batch, bool sample, const int32_t *slot_q, int32_t n_slots,
                             int32_t n_sample_tiles, float *maxima, const float *theta,
                             uint32_t *count, uint64_t *cand, int64_t cap, int32_t tiles_per_wg,
                             int32_t max_terms, unsigned long long *queue, hipStream_t s);

hipError_t launch_theta(const float *maxima, int64_t n_maxima, int64_t rank, int32_t n_slots,
                        float *theta, hipStream_t s);

hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
// p[i] = first + i for i in [0, n).
hipError_t launch_iota(int32_t *p, int32_t n, int32_t first, hipStream_t s);

// Rows whose status is not kSlotOk (of [0, n), or of in_rows[0, n)) into
// out_rows in order; their number into *count.
hipError_t launch_collect_failed(const int32_t *status, const int32_t *in_rows, int32_t n,
                                 int32_t *out_rows, uint32_t *count, hipStream_t s);

// max_qnnz: bound on the length of every finalized query row (sizes the
// rerank table; a longer row gets status kSlotRetry).  theta: the thresholds
// the candidates were emitted with (null: every document was emitted); a
// threshold <= 0 means the zero sums were left out and are supplied here.
// With rerank, pool is scratch of n_slots * need keys (select, then rerank
// with one wave per entry, then sort).
hipError_t launch_finalize(const DevIndex &ix, const DevQueries &q, const int32_t *slot_q,
                           int32_t n_slots, const uint32_t *count, const uint64_t *cand,
                           const float *theta, int64_t cap, int32_t need, int32_t k, bool rerank,
                           int32_t max_qnnz, uint64_t *pool, int64_t *out_ids, float *out_scores,
                           int32_t *status, hipStream_t s);

// Device index build (sindi_build.hip); err bits: 1 row pointers, 2 term id
// range, 4 ids not ascending, 8 non-finite, 16 a tile of more than kTileGroupsMax groups,
// 32 a kept value overflows the storage type, 128 a row longer than kLongRow.
hipError_t build_check_rows(const int64_t *ptr, const int32_t *idx, const float *val,
                            int64_t n_rows, int64_t n_cols, int64_t nnz, int32_t *err,
                            hipStream_t s);
hipError_t build_prune_rows(const int64_t *ptr, const int32_t *idx, const float *val,
                            int64_t n_rows, int32_t mode, double alpha, int32_t vn, uint8_t *keep,
                            int32_t *long_rows, uint32_t *n_long, int32_t *err, hipStream_t s);
hipError_t build_prune_long(const int64_t *ptr, const int32_t *idx, const float *val,
                            const int32_t *rows, int32_t n_rows, int32_t mode, double alpha,
                            int32_t vn, uint8_t *keep, hipStream_t s);
hipError_t build_count_lists(const int64_t *ptr, const int32_t *idx, const float *val,
                             const uint8_t *keep, int64_t n_rows, int64_t n_cols,
                             const int64_t *tile_doc, int64_t n_tiles, int32_t dtype,
                             uint32_t *cnt, uint32_t *term_max_bits, unsigned long long *n_kept,
                             int32_t *err, hipStream_t s);
hipError_t build_list_offsets(const uint32_t *cnt, int64_t n_tiles, int64_t n_cols,
                              uint32_t *goff, int64_t *tile_groups, int32_t *err, hipStream_t s);
hipError_t build_fill_lists(const int64_t *ptr, const int32_t *idx, const float *val,
                            const uint8_t *keep, const int64_t *tile_doc, const int64_t *tile_post,
                            const uint32_t *goff, int64_t n_tiles, int64_t n_cols, int32_t dtype,
                            uint16_t *post_doc, void *post_val, hipStream_t s);
hipError_t build_fill_pads(const uint32_t *goff, const uint32_t *cnt, const int64_t *tile_post,
                           int64_t n_tiles, int64_t n_cols, uint16_t *post_doc, hipStream_t s);
// Reorders every list chunk of kChunk groups (ascending by document on entry: run once, after
// the lists are filled) so that the postings one scoring instruction adds per 32-lane half fall
// in distinct LDS banks where the chunk allows; pads stay in place.  vbytes: 4 or 2.
hipError_t build_deal_chunks(const uint32_t *goff, const int64_t *tile_post, int64_t n_tiles,
                             int64_t n_cols, int32_t vbytes, uint16_t *post_doc, void *post_val,
                             hipStream_t s);

hipError_t launch_score_forward(const DevIndex &ix, const DevQueries &q, const int64_t *cand,
                                int32_t n_cand, float *out, hipStream_t s);

hipError_t launch_score_backward(const DevIndex &ix, const DevQueries &q, const int64_t *cand,
                                 int32_t n_cand, const float *grad, float *gq, float *gx,
                                 hipStream_t s);

}  // namespace sindi
