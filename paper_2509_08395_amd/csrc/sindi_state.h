// Host-side state shared by the index/search code (sindi_host.cpp) and the
// serving loop (sindi_server.cpp).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "sindi.h"
#include "sindi_internal.h"

namespace sindi {

// Record a thread-local error message and return st.
sindi_status fail(sindi_status st, const char *fmt, ...);
// This thread's last error message.
const char *last_error();

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return ::sindi::fail(SINDI_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

int host_threads();

// Run fn(lo, hi) over [0, n) in contiguous slices on the host threads.
template <typename F>
void parallel_for(int64_t n, F fn)
{
    const int nt = (int)std::min<int64_t>(host_threads(), std::max<int64_t>(n / 1024, 1));
    if (nt <= 1) {
        fn((int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    const int64_t step = (n + nt - 1) / nt;
    for (int i = 0; i < nt; ++i) {
        const int64_t lo = i * step, hi = std::min(n, lo + step);
        if (lo >= hi) break;
        th.emplace_back([=] { fn(lo, hi); });
    }
    for (auto &t : th) t.join();
}

// Grow-only device buffer.
struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    hipError_t ensure(size_t n)
    {
        if (n <= bytes && p) return hipSuccess;
        release();
        size_t want = n < 256 ? 256 : n;
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        bytes = want;
        return hipSuccess;
    }
    template <typename T> T *as() const { return reinterpret_cast<T *>(p); }
};

// The parameters of one search, resolved against the index.
struct Plan {
    int32_t k = 0, gamma = 0, need = 0, batch = 1, n_sample = 0, tile_run = 0;
    bool queue = false;    // scoring passes as one persistent, queue-fed launch
    int32_t max_qnnz = 0;  // bound on every query row's length (rerank table size)
    int64_t cap = 0, rank = 0;
    bool keep_all = true, rerank = true;
    double beta = 1.0;
};

// Device scratch of one search as raw pointers into memory owned elsewhere (a
// Workspace, a server slot, or the library's static scratch array).  The row
// part holds one entry per query row (or per query entry) of the call; the
// arena holds, for one group of query slots at a time, what a pass keeps per
// slot: the slot's row, candidate count, threshold, sampled maxima, candidate
// list and rerank pool.
struct Scratch {
    int32_t *ct = nullptr, *cn = nullptr, *err = nullptr, *status = nullptr;
    int32_t *rows = nullptr, *rows2 = nullptr;  // failed rows, two lists for two retries
    uint32_t *n_rows = nullptr;                 // [2] lengths of rows / rows2
    float *cw = nullptr, *qinv = nullptr;
    double *sabs = nullptr;
    unsigned char *arena = nullptr;
    size_t arena_bytes = 0;
};

// Bytes of the row part of a Scratch for nq rows of nnz entries in total.
size_t scratch_row_bytes(const Plan &pl, int64_t nq, int64_t nnz);
// Lay the row part out at p (256-byte aligned pieces); the arena is left empty.
Scratch carve_rows(unsigned char *p, const Plan &pl, int64_t nq, int64_t nnz);

// How a pass finds each query's coarse candidates:
//   kPassSampled     threshold = the rank-th largest per-thread maximum over
//                    the plan's evenly spaced sample tiles (may miss: then
//                    the query is retried);
//   kPassFullSample  the same over every tile with rank = gamma, so at least
//                    gamma documents reach the threshold (misses only if more
//                    than the candidate buffer reach it);
//   kPassKeepAll     no threshold, every document is a candidate.
enum PassKind { kPassSampled = 0, kPassFullSample = 1, kPassKeepAll = 2 };
struct PassShape {
    int32_t n_sample = 0;
    int64_t n_max = 0, rank = 0, cap = 0;
    bool keep_all = false;
};
PassShape pass_shape(const sindi_index *ix, const Plan &pl, PassKind kind);
// Arena bytes of g query slots of a pass.
size_t pass_bytes(const PassShape &sh, const Plan &pl, int64_t g);
// Most query slots of a pass that an arena of `bytes` holds (0 if not one).
int64_t pass_group(const PassShape &sh, const Plan &pl, size_t bytes);

// Grow-only owner of a Scratch (sindi_search's, one per index).
struct Workspace {
    DBuf q_ptr, q_idx, q_val, row_part, arena;
    Scratch view;
};

enum { kProfPrep = 0, kProfSample = 1, kProfScore = 2, kProfTheta = 3, kProfFinal = 4 };
// Launch through `fn`, bracketed by HIP events on s while profiling is on.
hipError_t timed_launch(int cat, hipStream_t s, hipError_t (*fn)(void *), void *ctx);
template <typename F>
hipError_t timed(int cat, hipStream_t s, F f)
{
    return timed_launch(cat, s, [](void *c) { return (*static_cast<F *>(c))(); }, &f);
}

}  // namespace sindi

// ------------------------------------------------------------------ index
struct sindi_index {
    int64_t n_docs = 0, n_cols = 0, nnz = 0, n_post = 0, n_slots = 0, window = 0, n_windows = 0,
            n_tiles = 0;
    int32_t tile_max = 0, tile_stride = 0, dtype = 0, prune = 0, vn = 0;
    int64_t list_len = 0;
    double alpha = 1.0;
    int device = 0;
    int64_t max_lds = 0;
    std::vector<int64_t> h_tile_doc;
    sindi::DBuf indptr, indices, values, tile_doc, tile_post, term_goff, post_doc, post_val,
        term_max;
    std::mutex mu;        // guards ws (the workspace of sindi_search calls)
    sindi::Workspace ws;

    sindi::DevIndex dev() const;
    int64_t device_bytes() const;
};

namespace sindi {

// Resolve search parameters for nq queries (no device work).
sindi_status make_plan(const sindi_index *ix, int64_t nq, int32_t k,
                       const sindi_search_params &p, bool rerank, const char *fn, Plan &pl);
// The plan's tiles per work item: the caller's, else 8, 12 or 32 by the list postings the nq
// queries (nnz terms) read per tile, taken as the index's kept fraction times their mean
// length (the tiles the resident workgroups share through L2).
void set_tile_run(Plan &pl, const sindi_index *ix, const sindi_search_params &p, int64_t nq,
                  int64_t nnz);

// Structural check of a host CSR (Def. 1).  max_row > 0 bounds row length;
// longest (if not null) receives the longest row.
sindi_status validate_host_csr(const sindi_csr *m, const char *what, int64_t max_row,
                               int64_t *longest = nullptr);

// Enqueue on s the query preparation of rows [0, nq) of dq: beta-mass
// coarse terms, fixed-point weights and device-side validation, whose flags
// land in sc.err[0] (0: every row well formed), the longest row in sc.err[1].
sindi_status enqueue_prep(const sindi_index *ix, const Scratch &sc, const Plan &pl,
                          const DevQueries &dq, hipStream_t s);

// Enqueue on s, after enqueue_prep, passes of one kind over n query rows:
// rows [0, n) of dq when rows is null, else the rows listed in device memory
// rows[0, n).  Slots go in groups that fit sc's arena (at least one must).
// Each row's status lands in sc.status; results in the row's output rows.
sindi_status enqueue_passes(const sindi_index *ix, const Scratch &sc, const Plan &pl,
                            PassKind kind, const DevQueries &dq, const int32_t *rows, int64_t n,
                            int64_t *out_ids, float *out_scores, hipStream_t s);

// Enqueue the compaction of the rows whose status is not kSlotOk: of rows
// [0, n) (in_rows null) or of in_rows[0, n), into out_rows, the count into
// *count (device).
sindi_status enqueue_collect_failed(const Scratch &sc, const int32_t *in_rows, int64_t n,
                                    int32_t *out_rows, uint32_t *count, hipStream_t s);

// Synchronous search of validated device queries dq with the scratch sc:
// prep, sampled (or keep-all) passes, then for rows whose threshold missed a
// pass over every tile and, for rows still unresolved, a keep-all pass.  The
// arena is regrown through grow (may be null: then sc's arena must hold one
// keep-all query).  Device queries are validated on the device first.
sindi_status run_search(const sindi_index *ix, Scratch &sc, const Plan &pl, const DevQueries &dq,
                        bool device_queries, int64_t *out_ids, float *out_scores, hipStream_t s,
                        const char *fn, sindi_status (*grow)(void *, size_t, Scratch &),
                        void *grow_ctx);

}  // namespace sindi
