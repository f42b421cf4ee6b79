/*
 * sindi.h -- C ABI of the MI355X (gfx950) SINDI sparse maximum-inner-product
 * search library (arXiv 2509.08395: "SINDI", a value-storing, window-
 * partitioned inverted index with mass-ratio pruning and exact reordering).
 *
 * Conventions for every entry point
 *   - Return a sindi_status; SINDI_OK (0) on success.  On failure nothing is
 *     written to the caller's output buffers and sindi_last_error() returns a
 *     thread-local message.  No C++ exception crosses this interface.
 *   - "stream" is a hipStream_t passed as void*; NULL is the default stream.
 *     Every device operation of a call is enqueued on it.
 *   - The caller owns every buffer it passes.  The library keeps no pointer to
 *     them after the call returns.
 *   - Ranking order: score descending, equal scores by ascending document id.
 *   - Scores are inner products delta(x, q) (Def. 2), not the 1 - delta
 *     distance the paper's Alg. 4 ranks by.
 */
#ifndef SINDI_H
#define SINDI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The library is built with hidden symbols; these declarations are its only
 * exports. */
#pragma GCC visibility push(default)

typedef enum {
    SINDI_OK = 0,
    SINDI_E_INVALID = -1,  /* malformed input or parameter                     */
    SINDI_E_RANGE = -2,    /* a value does not fit the requested storage type   */
    SINDI_E_OOM = -3,      /* device or host allocation failed                  */
    SINDI_E_HIP = -4,      /* a HIP runtime call failed                         */
    SINDI_E_BUSY = -5,     /* serving: request queue full, or result not ready  */
    SINDI_E_INTERNAL = -6  /* a library invariant failed                        */
} sindi_status;

/* Storage type of posting values (document entries in the inverted lists). */
typedef enum { SINDI_F32 = 0, SINDI_F16 = 1, SINDI_BF16 = 2 } sindi_dtype;

/*
 * A set of sparse vectors in CSR form (Def. 1: a vector is the set of its
 * non-zero entries).  Row r owns entries [indptr[r], indptr[r+1]): term ids
 * in indices[] (strictly ascending within a row, each in [0, n_cols)) and
 * their values in values[] (finite float32).  Explicit zero values are
 * allowed and are treated as absent entries.
 * on_device = 0: the three arrays are host memory.
 * on_device = 1: they are device memory of the current HIP device (only
 *                sindi_search / sindi_search_coarse / the score calls accept
 *                device-resident queries; sindi_build reads host memory).
 */
typedef struct {
    int64_t n_rows;
    int64_t n_cols;          /* vocabulary size d                            */
    int64_t nnz;             /* == indptr[n_rows]                            */
    const int64_t *indptr;   /* [n_rows + 1], indptr[0] == 0, non-decreasing */
    const int32_t *indices;  /* [nnz]                                        */
    const float *values;     /* [nnz]                                        */
    int32_t on_device;
    int32_t reserved_;
} sindi_csr;

/* Index build parameters (Alg. 3, ApproximateSindiConstruction). */
typedef struct {
    double alpha;            /* mass-ratio pruning ratio, (0, 1]; 1 = keep all (Def. 6) */
    int64_t window;          /* window size lambda in documents, >= 1 (Sec. 3.3.1)       */
    int32_t value_dtype;     /* sindi_dtype of the stored posting values                 */
    int32_t tile;            /* max documents per on-chip score tile; 0 = library default;
                                every window is split into equal tiles of at most this
                                many documents; at most 16384.  A tile's lists may hold
                                at most 2^28 - 64 groups of 4 postings (else E_INVALID)  */
    int32_t prune;           /* sindi_prune: which entries of the corpus the lists keep  */
    int32_t vn;              /* SINDI_PRUNE_VNP: entries kept per document, >= 1         */
    int64_t list_len;        /* SINDI_PRUNE_LP, _MRP_LP: entries kept per term list, >= 1 */
    int32_t gpu_build;       /* 0: prune and lay out the lists on the host; 1: on the current
                                HIP device (MRP and VNP only; rows of at most 8192 entries);
                                the index is the same bit for bit                          */
    int32_t reserved_;
} sindi_build_params;

/*
 * Pruning of the documents before the lists are built (Sec. 4.1).  In every
 * case only non-zero entries count, and entries are ranked by |x|
 * descending; ties go to the lower term id within a document and to the
 * lower document id within a term's list.
 *   MRP     each document keeps its alpha-mass subvector (Defs. 5-6);
 *   VNP     each document keeps its vn entries of largest |x|;
 *   LP      each term's list keeps its list_len entries of largest |x|;
 *   MRP_LP  MRP first, then LP among the entries MRP kept.
 */
typedef enum { SINDI_PRUNE_MRP = 0, SINDI_PRUNE_VNP = 1, SINDI_PRUNE_LP = 2,
               SINDI_PRUNE_MRP_LP = 3 } sindi_prune;

/* Search parameters (Alg. 4, ApproximateSindiSearch).  Zero fields take defaults. */
typedef struct {
    double beta;             /* query mass-ratio pruning for the coarse stage, (0, 1]; 0 -> 1 */
    int32_t gamma;           /* reorder pool size, k <= gamma <= 4096; 0 -> max(k, 500)      */
    int32_t batch;           /* queries sharing one pass over a tile's lists: 1, 2, 4 or 8;
                                0 -> library default (1); halved while the batch's score
                                rows exceed the device's LDS (12,500-document tiles: 2)    */
    int32_t cand_cap;        /* per-query candidate buffer entries; 0 -> 32768               */
    int32_t sample_tiles;    /* tiles scored first to set each query's candidate threshold;
                                0 -> 8, -1 -> no threshold (keep every document)             */
    int32_t tile_run;        /* consecutive tiles swept by one workgroup; 0 -> 8, 12 or 32 by
                                the index's kept fraction of corpus entries times the call's
                                mean query terms (above 12: 8; above 5: 12; else 32); halved
                                while a launch would hold fewer than 4096 (query, tile run)
                                items                                                       */
    int32_t schedule;        /* scoring launches with one query per workgroup: 1 one
                                workgroup per (query, tile run); 2 one persistent launch of
                                the workgroups the device holds at once, each taking (query,
                                tile run) items from a device queue until it is empty;
                                0 -> 2.  Results are the same bit for bit.                  */
} sindi_search_params;

/* Summary of a built index. */
typedef struct {
    int64_t n_docs, n_cols, nnz;   /* unpruned corpus                          */
    int64_t n_postings;            /* entries kept by pruning = index postings */
    int64_t window;                /* lambda                                   */
    int64_t n_windows;             /* sigma = ceil(n_docs / window)            */
    int64_t n_tiles;               /* score tiles (windows split into tiles)   */
    int32_t tile_max;              /* largest tile, documents                  */
    int32_t value_dtype;
    double alpha;
    int64_t device_bytes;          /* HBM held by the index                    */
    int64_t n_slots;               /* posting slots stored: n_postings plus the
                                      pad entries that align every list to 4   */
    int32_t prune, vn;             /* as built                                 */
    int64_t list_len;
} sindi_index_info;

typedef struct sindi_index sindi_index;

/*
 * Build the index of Alg. 3 from a host CSR corpus: every document is cut to
 * its alpha-mass subvector (Defs. 5-6: entries ranked by |x| descending, ties
 * by ascending term id; the shortest prefix whose |x| sum, accumulated in
 * FP64 in that order, reaches alpha times the row's mass), or pruned by the
 * rule params->prune selects, and the kept entries are laid out as the value-storing inverted lists I_{j,w} of Alg. 1
 * (document ids ascending inside every list; stored in chunks of 256 slots, each
 * chunk's postings in the LDS-bank order sindi_index_export describes), each
 * window further split into score tiles.  The unpruned corpus is kept too, for the exact rerank of
 * Alg. 4.  Both live in device memory owned by the returned handle.
 * Values stored as FP16/BF16 are rounded to nearest even; an FP16 overflow
 * (|x| > 65504) returns SINDI_E_RANGE.
 * The corpus may be device memory only with params->gpu_build = 1 (it is
 * then validated on the device and copied).  *out receives the handle (free
 * with sindi_index_free).  Synchronous: returns after the build completes.
 */
sindi_status sindi_build(const sindi_csr *corpus, const sindi_build_params *params, void *stream,
                         sindi_index **out);

void sindi_index_free(sindi_index *idx);

sindi_status sindi_index_get_info(const sindi_index *idx, sindi_index_info *out);

/*
 * Copy the device index to host buffers (for checking the layout).
 *   tile_doc   int64 [n_tiles + 1]  first document of each tile
 *   tile_post  int64 [n_tiles + 1]  first posting slot of each tile (multiple of 4)
 *   term_goff  uint32 [n_tiles * (n_cols + 1)]  for tile t and term j, with
 *              g = term_goff[t*(n_cols+1) + j]: the list I_{j,t} starts at slot
 *              tile_post[t] + 4 * (g & 0x3FFFFFFF), holds its postings, then
 *              (g >> 30) pad entries (value 0, the list's largest document id),
 *              and the next term's list starts at the next 4-slot boundary;
 *              entry n_cols holds the tile's slot count / 4.  A list's slots
 *              form chunks of 256 from its start (the last may be shorter), and
 *              a chunk holds the next documents of the ascending list, n real
 *              postings ordered for the score row's 32 LDS banks: taken by
 *              (document mod 32, document), they fill slots 4 (32 h + r) + p
 *              of the chunk for r = 0..31, h = 0..1, p = 0..3, skipping slots
 *              at or past n; a chunk of n <= 4 stays ascending.
 *   post_doc   uint16 [n_slots]  4 * (document id - tile_doc[t]), the byte offset
 *              of the document's 32-bit score in an on-chip score row
 *   post_val   [n_slots] values as stored (4 or 2 bytes each)
 * Any pointer may be NULL to skip that array.
 */
sindi_status sindi_index_export(const sindi_index *idx, int64_t *tile_doc, int64_t *tile_post,
                                uint32_t *term_goff, uint16_t *post_doc, void *post_val);

/*
 * Alg. 4: for every query q, the coarse pool = the first gamma documents by
 * the inner product of beta-mass(q) with the pruned documents (Alg. 2 over
 * the index); each pooled document's exact delta(x, q) in FP32 from the
 * unpruned vector and the full query; the first k by that score.
 *   queries  CSR over the index's vocabulary (host or device memory)
 *   out_ids  device int64 [n_rows * k]; -1 where fewer than k documents exist
 *   out_scores device float [n_rows * k]; -inf for padding
 * Blocks until the results are in out_ids / out_scores.
 */
sindi_status sindi_search(const sindi_index *idx, const sindi_csr *queries, int32_t k,
                          const sindi_search_params *params, int64_t *out_ids, float *out_scores,
                          void *stream);

/*
 * sindi_search for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same search, results bit for bit those of sindi_search, with every
 * piece of device scratch (coarse query terms, per-query status, sampled
 * maxima, candidate lists, rerank pools) carved from one array of 256 MiB
 * that the library holds on each device it runs on until the process ends.
 * The call allocates nothing: no hipMalloc, hipFree or allocating library
 * routine; the caller passes only inputs and outputs.
 *   queries   device memory only (on_device = 1), of the index's device,
 *             which must be the current device
 *   out_ids / out_scores  device buffers as for sindi_search
 * Limit: the per-query part (20 bytes per query plus 8 per query entry, 16
 * per entry with beta < 1, each piece rounded up to 256 bytes) and one query
 * of the largest pass
 * a retry may need (8 bytes per document of the index for the pass that
 * keeps every document) must fit the 256 MiB together; otherwise the call
 * returns SINDI_E_INVALID with the sizes, before any device work, and leaves
 * the outputs untouched (sindi_search has no such limit).  Queries are
 * processed in groups that fit the rest of the array.
 * The array is shared by every call on a device and keeps the last call's
 * contents; everything that must start at zero is cleared in-stream.  Calls
 * are synchronous and the library runs one at a time per device (a second
 * thread's call waits); calls from two processes sharing a device each use
 * their own process's array.  Blocks until the results are written.
 */
sindi_status sindi_search_noalloc(const sindi_index *idx, const sindi_csr *queries, int32_t k,
                                  const sindi_search_params *params, int64_t *out_ids,
                                  float *out_scores, void *stream);

/*
 * Alg. 2 (PreciseSindiSearch) over the index: the first k documents by the
 * coarse score (inner product of beta-mass(q) with the pruned documents as
 * stored, FP32 accumulation), no rerank.  Same buffers as sindi_search.
 */
sindi_status sindi_search_coarse(const sindi_index *idx, const sindi_csr *queries, int32_t k,
                                 const sindi_search_params *params, int64_t *out_ids,
                                 float *out_scores, void *stream);

/*
 * Scores of listed candidates: out_scores[b*n_cand + c] = delta(q_b, x_{cand})
 * (Def. 2) in FP32 over the unpruned corpus rows; cand id -1 (or any id
 * outside [0, n_docs)) gives 0.
 *   queries     CSR (device memory) over the index's vocabulary
 *   cand_ids    device int64 [n_rows * n_cand]
 *   doc_values  device float [nnz]: document values aligned with the corpus
 *               values given to sindi_build (same rows and term ids, new
 *               values, e.g. a document encoder's current output), or NULL
 *               to score the values the index copied at build time.  The
 *               inverted lists that sindi_search reads are not affected.
 *   out_scores  device float [n_rows * n_cand]
 * Enqueued on the stream after the queries are validated (which waits for
 * the stream); the caller keeps every buffer alive until the stream reaches
 * the call.
 */
sindi_status sindi_score_forward(const sindi_index *idx, const sindi_csr *queries,
                                 const int64_t *cand_ids, int32_t n_cand,
                                 const float *doc_values, float *out_scores, void *stream);

/*
 * Backward of sindi_score_forward.  The score is bilinear in the values, so
 * with G = dL/dscore:
 *   grad_query_values[e] += sum_c G[b,c] * x_c[t]     (entry e = (b, t))
 *   grad_doc_values[e']  += sum_b G[b,c] * q_b[t]     (entry e' = (c, t))
 * over common dimensions t only; entries outside every intersection are
 * untouched.  x is doc_values when given (as for sindi_score_forward), else
 * the index's copy.  grad_query_values is aligned with queries->values
 * (device, [queries->nnz]); grad_doc_values with the corpus values given to
 * sindi_build (device, [nnz]).  Either may be NULL.  Accumulates (+=); the
 * document side adds with atomics, so the order of its FP32 additions is
 * not fixed.  Candidate ids -1 are skipped.
 */
sindi_status sindi_score_backward(const sindi_index *idx, const sindi_csr *queries,
                                  const int64_t *cand_ids, int32_t n_cand,
                                  const float *doc_values, const float *grad_scores,
                                  float *grad_query_values, float *grad_doc_values,
                                  void *stream);

/*
 * ---------------------------------------------------------------- serving
 * Continuous batching over one index (the paper measures single queries;
 * this is the request loop around Alg. 4).  Requests are queued as they
 * arrive; a dispatcher thread owned by the server admits queued requests into
 * a batch as soon as one of max_inflight batch slots is free and the
 * candidate memory the batch needs (sampled maxima, candidate lists, rerank
 * pools: about 330 KB per query at the defaults) fits in the largest free
 * block of one device arena of workspace_bytes shared by every batch in
 * flight: as many requests as are queued, up to max_batch and up to what fits.
 * It runs the whole search of that batch asynchronously on the slot's own HIP
 * stream, so batches overlap on the device.  A query whose sampled candidate
 * threshold missed is re-run on the same stream (a threshold over every tile,
 * then none) without holding up the dispatcher.  A batch runs with
 * the largest k any of its requests asks for; every request gets the prefix
 * of its own k.  Scoring is deterministic and independent of which other
 * queries share a batch, so a request's result equals what sindi_search
 * returns for the same query alone (bit for bit, ids and scores).
 * The server holds its device workspace (candidate buffers, query staging,
 * outputs) for its whole life; the index must outlive the server.
 */
typedef struct {
    int32_t max_inflight;     /* batches on the device at once (streams); 0 -> 3, at most 8 */
    int32_t max_batch;        /* queries per batch; 0 -> 256, at most 8192                   */
    int32_t k_max;            /* largest k of a request, <= gamma; 0 -> 100                  */
    int32_t max_query_nnz;    /* longest query row accepted; 0 -> 512, at most 4096          */
    int64_t max_queue;        /* queued requests before submit returns SINDI_E_BUSY; 0 -> 2^20 */
    int64_t workspace_bytes;  /* candidate memory shared by the batches in flight; 0 -> 2 GiB
                                 (raised to hold at least one query)                         */
    sindi_search_params search;  /* beta, gamma, cand_cap, sample_tiles, tile_run as for
                                    sindi_search; gamma 0 -> max(k_max, 500)                 */
} sindi_server_params;

/* Counters since creation. */
typedef struct {
    int64_t submitted, completed, batches, retried, largest_batch;
    double busy_ms;           /* wall time with at least one batch on the device          */
    int64_t memory_waits;     /* times queued requests waited for candidate memory        */
    int64_t arena_peak_bytes; /* most candidate memory held by the batches in flight      */
} sindi_server_stats;

typedef struct sindi_server sindi_server;

/* Create a server on the current HIP device (the index's device).  Allocates
 * the per-slot device workspace and pinned host staging, starts the
 * dispatcher thread. */
sindi_status sindi_server_create(const sindi_index *idx, const sindi_server_params *params,
                                 sindi_server **out);

/*
 * Queue one query: nnz entries, host memory, term ids strictly ascending in
 * [0, n_cols), finite values (Def. 1), 1 <= k <= k_max.  The entries are
 * copied before the call returns.  *ticket identifies the request for
 * sindi_server_wait.  SINDI_E_BUSY: max_queue requests are already waiting.
 * Thread-safe.
 */
sindi_status sindi_server_submit(sindi_server *srv, const int32_t *indices, const float *values,
                                 int32_t nnz, int32_t k, int64_t *ticket);

/*
 * Wait up to timeout_ms (< 0: without limit) for a request and collect it:
 * its k ids and scores into host buffers (ids -1 / scores -inf beyond the
 * corpus size) and the time from submit to completion in nanoseconds (any
 * output pointer may be NULL).  A collected ticket is forgotten.
 * SINDI_E_BUSY: not finished within the timeout (the ticket stays valid).
 * A request whose batch failed returns that batch's error.  Thread-safe.
 */
sindi_status sindi_server_wait(sindi_server *srv, int64_t ticket, int64_t *ids, float *scores,
                               int64_t *latency_ns, double timeout_ms);

/*
 * Open-loop replay: submit query row r of `queries` (host CSR) with k = ks[r]
 * at arrival_s[r] seconds (non-decreasing) after the call starts, whatever
 * the server's progress, then wait for every request.  Outputs (host memory):
 * out_ids / out_scores [n_rows * k_max], row r holding its ks[r] results
 * first (the rest -1 / -inf); latency_ns [n_rows] = completion minus the
 * scheduled arrival (so queueing behind a late submit counts).  Blocks.
 */
sindi_status sindi_server_replay(sindi_server *srv, const sindi_csr *queries, const int32_t *ks,
                                 const double *arrival_s, int64_t *out_ids, float *out_scores,
                                 int64_t *latency_ns);

sindi_status sindi_server_get_stats(const sindi_server *srv, sindi_server_stats *out);

/* Stop the dispatcher after the batches on the device finish; requests not
 * yet collected are dropped.  Releases everything the server holds. */
void sindi_server_destroy(sindi_server *srv);

/*
 * Kernel timing.  While enabled, the library records a pair of HIP events on
 * the caller's stream around every kernel that sindi_search /
 * sindi_search_coarse launch; sindi_profile_read waits for the recorded
 * events and reports, per kernel class, the number of launches and the sum of
 * their GPU durations in milliseconds.  Classes:
 *   0 query preparation (validation, beta-mass), 1 accumulate, threshold
 *   pass over the sampled tiles, 2 accumulate, scoring pass over every tile,
 *   3 threshold selection, 4 finalize (top-gamma, rerank, top-k).
 * Process-wide; reading with reset != 0 clears the totals.
 */
typedef struct {
    int64_t launches[5];
    double ms[5];
} sindi_profile;

sindi_status sindi_profile_enable(int32_t enable);
sindi_status sindi_profile_read(sindi_profile *out, int32_t reset);

/* Thread-local text of the last error of this thread ("" if none). */
const char *sindi_last_error(void);

/* Library version string. */
const char *sindi_version(void);

#pragma GCC visibility pop

#ifdef __cplusplus
}
#endif
#endif /* SINDI_H */
