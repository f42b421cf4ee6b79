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

// Device scratch of one search in flight: device copies of host queries,
// coarse query terms, per-query status, the sampled maxima and thresholds,
// and the per-query candidate lists ("score windows" leaving LDS).
struct Workspace {
    DBuf q_ptr, q_idx, q_val, ct, cw, cn, qinv, sabs, err, status, slot_q, maxima, theta, count,
        cand, pool;
};

// The parameters of one search, resolved against the index.
struct Plan {
    int32_t k = 0, gamma = 0, need = 0, batch = 1, n_sample = 0, tile_run = 0;
    int32_t max_qnnz = 0;  // bound on every query row's length (rerank table size)
    int64_t cap = 0, rank = 0, n_max = 0, group = 0;
    bool keep_all = true, rerank = true;
    double beta = 1.0;
};

// Bytes of device scratch one query needs under a plan (candidates, maxima,
// rerank pool, threshold, count, status).
inline size_t plan_query_bytes(const Plan &pl)
{
    return (size_t)pl.cap * 8 + (size_t)pl.n_max * 4 + (pl.rerank ? (size_t)pl.need * 8 : 0) + 16;
}

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

// Structural check of a host CSR (Def. 1).  max_row > 0 bounds row length;
// longest (if not null) receives the longest row.
sindi_status validate_host_csr(const sindi_csr *m, const char *what, int64_t max_row,
                               int64_t *longest = nullptr);

// Size ws for nq queries of total nnz under pl (allocations; not async).
sindi_status reserve_workspace(Workspace &ws, const Plan &pl, int64_t nq, int64_t nnz);

// Enqueue on s the query preparation of rows [0, nq) of dq: beta-mass
// coarse terms, fixed-point weights and device-side validation, whose flags
// land in ws.err[0] (0: every row well formed), the longest row in ws.err[1].
// No host sync.
sindi_status enqueue_prep(const sindi_index *ix, Workspace &ws, const Plan &pl,
                          const DevQueries &dq, hipStream_t s);

// Enqueue on s, after enqueue_prep, every accumulate / threshold / finalize
// launch of the plan.  Per-query status lands in ws.status.  No host sync.
sindi_status enqueue_search(const sindi_index *ix, Workspace &ws, const Plan &pl,
                            const DevQueries &dq, int64_t *out_ids, float *out_scores,
                            hipStream_t s);

// Re-run, with every document kept, the listed query rows whose threshold
// missed (status kSlotRetry).  Synchronous.
sindi_status retry_queries(const sindi_index *ix, Workspace &ws, const Plan &pl,
                           const DevQueries &dq, const std::vector<int32_t> &rows,
                           int64_t *out_ids, float *out_scores, hipStream_t s, const char *fn);

}  // namespace sindi
