// Continuous-batching request loop over one index: the serving form of the
// search of Alg. 4.  Requests queue as they arrive; a dispatcher thread moves
// every queued request (up to max_batch) into a batch whenever one of the
// batch slots is free and runs the whole search of that batch asynchronously
// on the slot's stream.  Each slot owns its device workspace, pinned host
// staging and a completion event, so several batches overlap on the device
// and the host never waits on one batch to start the next.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sindi.h"
#include "sindi_internal.h"
#include "sindi_state.h"

using Clock = std::chrono::steady_clock;

namespace sindi {
namespace {

constexpr int32_t kMaxSlots = 8;
constexpr int32_t kMaxBatchQueries = 8192;

struct Request {
    int64_t ticket = 0;
    int32_t k = 0, nnz = 0;
    std::vector<int32_t> own_idx;  // submitted entries (copied)
    std::vector<float> own_val;
    const int32_t *idx = nullptr;  // entries to stage: own_* or a replay row
    const float *val = nullptr;
    Clock::time_point t0;          // arrival: submit time, or scheduled replay arrival
    bool done = false;
    sindi_status st = SINDI_OK;
    std::string msg;
    // results: own buffers (submit/wait) or rows of the replay caller's arrays
    std::vector<int64_t> ids;
    std::vector<float> scores;
    int64_t lat_ns = 0;
    int64_t *dst_ids = nullptr;
    float *dst_scores = nullptr;
    int64_t *dst_lat = nullptr;
};

template <typename T> struct Pinned {
    T *p = nullptr;
    Pinned() = default;
    Pinned(const Pinned &) = delete;
    Pinned &operator=(const Pinned &) = delete;
    ~Pinned()
    {
        if (p) (void)hipHostFree(p);
    }
    hipError_t alloc(size_t n) { return hipHostMalloc((void **)&p, (n ? n : 1) * sizeof(T), hipHostMallocDefault); }
};

// First-fit allocator over one device buffer: the candidate memory (sampled
// maxima, candidate lists, rerank pools) shared by every batch in flight.  A
// batch is admitted only when its share fits; used by the dispatcher thread
// alone.
struct Arena {
    DBuf buf;
    std::map<size_t, size_t> free_blocks;  // offset -> length, adjacent blocks merged
    size_t used = 0, peak = 0;
    static size_t round(size_t n) { return (n + 255) & ~(size_t)255; }
    void reset()
    {
        free_blocks.clear();
        free_blocks[0] = buf.bytes & ~(size_t)255;
        used = peak = 0;
    }
    size_t largest() const
    {
        size_t m = 0;
        for (const auto &b : free_blocks) m = std::max(m, b.second);
        return m;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = round(bytes);
        for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, at = it->first + bytes;
            free_blocks.erase(it);
            if (rest) free_blocks[at] = rest;
            used += bytes;
            peak = std::max(peak, used);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = round(bytes);
        used -= bytes;
        auto it = free_blocks.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_blocks.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_blocks.erase(next);
        }
        if (it != free_blocks.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_blocks.erase(it);
            }
        }
    }
};

// One batch slot: its stream, completion event, device scratch and pinned
// staging.  A batch moves through up to three stages, each ending with the
// slot's event: the sampled pass over every request (stage 0), a pass with a
// threshold taken over every tile for the rows whose sampled threshold missed
// (stage 1), and a pass with no threshold for rows still unresolved (stage 2).
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    DBuf q_ptr, q_idx, q_val, row_part, d_ids, d_scores;
    Scratch sc;
    size_t region_off = 0, region_bytes = 0;  // the batch's share of the arena (0: none)
    bool wants_retry_buffer = false;          // a retry waits for the server's retry buffer
    Pinned<int64_t> h_ptr, h_ids;
    Pinned<int32_t> h_idx, h_err;
    Pinned<uint32_t> h_fail;  // [2] failed-row counts of the stages
    Pinned<float> h_val, h_scores;
    std::vector<Request *> reqs;
    Plan pl;
    DevQueries dq{};
    int32_t kb = 0;
    int stage = 0;
    bool busy = false;
    sindi_status launch_st = SINDI_OK;
    std::string launch_msg;
    ~Slot()
    {
        if (stream) {
            (void)hipStreamSynchronize(stream);
            (void)hipStreamDestroy(stream);
        }
        if (done) (void)hipEventDestroy(done);
    }
};

}  // namespace
}  // namespace sindi

using namespace sindi;

struct sindi_server {
    const sindi_index *ix = nullptr;
    sindi_server_params p{};
    Plan base;                 // plan at k_max; batches differ only in k and size
    PassShape main_shape;      // the sampled pass every batch runs
    Arena arena;               // candidate memory of the batches in flight
    DBuf retry_buf;            // one query of either retry pass; one slot at a time
    Slot *retry_owner = nullptr;
    bool mem_blocked = false;  // a batch is waiting for candidate memory
    std::vector<std::unique_ptr<Slot>> slots;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> pending;
    std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
    int64_t next_ticket = 0;
    int64_t replay_left = 0;
    sindi_status replay_st = SINDI_OK;  // first failure among replayed requests
    std::string replay_msg;
    bool stop = false;
    sindi_server_stats stats{};
    int n_busy = 0;
    Clock::time_point busy_since;
    std::thread th;

    void run();
    bool launch(Slot &s, std::vector<Request *> &batch);
    sindi_status enqueue_retry(Slot &s, PassKind kind, const int32_t *rows, uint32_t n,
                               int32_t *out_rows, uint32_t *out_count, uint32_t *h_count);
    void complete(Slot &s);
    void start_retry(Slot &s);
    void finish(Slot &s, sindi_status st, const std::string &msg);
};

namespace {

sindi_status check_row(const sindi_server *srv, const int32_t *idx, const float *val, int64_t nnz,
                       int32_t k, const char *fn)
{
    if (k < 1 || k > srv->p.k_max)
        return fail(SINDI_E_INVALID, "%s: k = %d outside [1, %d]", fn, k, srv->p.k_max);
    if (nnz < 0 || nnz > srv->p.max_query_nnz)
        return fail(SINDI_E_INVALID, "%s: %lld entries (server accepts up to %d)", fn,
                    (long long)nnz, srv->p.max_query_nnz);
    if (nnz && (!idx || !val)) return fail(SINDI_E_INVALID, "%s: null entries", fn);
    for (int64_t e = 0; e < nnz; ++e) {
        if (idx[e] < 0 || idx[e] >= srv->ix->n_cols)
            return fail(SINDI_E_INVALID, "%s: term id %d out of range", fn, idx[e]);
        if (e + 1 < nnz && idx[e + 1] <= idx[e])
            return fail(SINDI_E_INVALID, "%s: term ids not strictly ascending", fn);
        if (!std::isfinite(val[e])) return fail(SINDI_E_INVALID, "%s: non-finite value", fn);
    }
    return SINDI_OK;
}

}  // namespace

// Stage a batch in pinned memory and enqueue its whole search on the slot's
// stream, ending with the copies of results and status to the host and the
// completion event.
bool sindi_server::launch(Slot &s, std::vector<Request *> &batch)
{
    // longest queries first: the scoring passes take (query, tile run) items in slot order,
    // so each run starts with its longest work (results do not depend on the order)
    std::stable_sort(batch.begin(), batch.end(),
                     [](const Request *a, const Request *b) { return a->nnz > b->nnz; });
    const int32_t nb = (int32_t)batch.size();
    int32_t kb = 1, longest = 0;
    int64_t nnz = 0;
    s.h_ptr.p[0] = 0;
    for (int32_t r = 0; r < nb; ++r) {
        const Request *q = batch[r];
        kb = std::max(kb, q->k);
        longest = std::max(longest, q->nnz);
        if (q->nnz) {
            memcpy(s.h_idx.p + nnz, q->idx, (size_t)q->nnz * 4);
            memcpy(s.h_val.p + nnz, q->val, (size_t)q->nnz * 4);
        }
        nnz += q->nnz;
        s.h_ptr.p[r + 1] = nnz;
    }
    s.reqs.swap(batch);
    s.kb = kb;
    s.pl = base;
    s.pl.k = kb;
    s.pl.max_qnnz = longest;  // sizes the kernels' per-query LDS for this batch
    set_tile_run(s.pl, ix, p.search, nb, nnz);
    s.stage = 0;
    s.dq = DevQueries{nb, nnz, s.q_ptr.as<int64_t>(), s.q_idx.as<int32_t>(), s.q_val.as<float>()};
    auto enqueue = [&]() -> sindi_status {
        const hipStream_t st = s.stream;
        HIP_TRY(hipMemcpyAsync(s.q_ptr.p, s.h_ptr.p, (size_t)(nb + 1) * 8, hipMemcpyHostToDevice, st));
        if (nnz) {
            HIP_TRY(hipMemcpyAsync(s.q_idx.p, s.h_idx.p, (size_t)nnz * 4, hipMemcpyHostToDevice, st));
            HIP_TRY(hipMemcpyAsync(s.q_val.p, s.h_val.p, (size_t)nnz * 4, hipMemcpyHostToDevice, st));
        }
        sindi_status e = enqueue_prep(ix, s.sc, s.pl, s.dq, st);
        if (e != SINDI_OK) return e;
        e = enqueue_passes(ix, s.sc, s.pl, kPassSampled, s.dq, nullptr, nb, s.d_ids.as<int64_t>(),
                           s.d_scores.as<float>(), st);
        if (e != SINDI_OK) return e;
        e = enqueue_collect_failed(s.sc, nullptr, nb, s.sc.rows, s.sc.n_rows, st);
        if (e != SINDI_OK) return e;
        HIP_TRY(hipMemcpyAsync(s.h_ids.p, s.d_ids.p, (size_t)nb * kb * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(s.h_scores.p, s.d_scores.p, (size_t)nb * kb * 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(s.h_fail.p, s.sc.n_rows, 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(s.h_err.p, s.sc.err, 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipEventRecord(s.done, st));
        return SINDI_OK;
    };
    s.launch_st = enqueue();
    s.launch_msg = s.launch_st == SINDI_OK ? std::string() : std::string(last_error());
    s.busy = true;
    return s.launch_st == SINDI_OK;
}

// Enqueue a retry stage of a slot's batch over the n device-listed rows:
// the pass, the rows it still leaves unresolved (into out_rows / out_count),
// the results and that count back to the host, then the slot's event.
sindi_status sindi_server::enqueue_retry(Slot &s, PassKind kind, const int32_t *rows, uint32_t n,
                                         int32_t *out_rows, uint32_t *out_count, uint32_t *h_count)
{
    const hipStream_t st = s.stream;
    const int32_t nb = (int32_t)s.reqs.size();
    sindi_status e = enqueue_passes(ix, s.sc, s.pl, kind, s.dq, rows, n, s.d_ids.as<int64_t>(),
                                    s.d_scores.as<float>(), st);
    if (e != SINDI_OK) return e;
    e = enqueue_collect_failed(s.sc, rows, n, out_rows, out_count, st);
    if (e != SINDI_OK) return e;
    HIP_TRY(hipMemcpyAsync(s.h_ids.p, s.d_ids.p, (size_t)nb * s.kb * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(s.h_scores.p, s.d_scores.p, (size_t)nb * s.kb * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(h_count, out_count, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(s.done, st));
    return SINDI_OK;
}

// Hand the slot's results to its requests and free the slot.
void sindi_server::finish(Slot &s, sindi_status st, const std::string &msg)
{
    const auto t1 = Clock::now();
    std::lock_guard<std::mutex> lock(mu);
    for (size_t r = 0; r < s.reqs.size(); ++r) {
        Request *q = s.reqs[r];
        q->st = st;
        q->msg = msg;
        q->lat_ns = std::chrono::duration_cast<std::chrono::nanoseconds>(t1 - q->t0).count();
        if (st == SINDI_OK) {
            const int64_t *ids = s.h_ids.p + r * s.kb;
            const float *sc = s.h_scores.p + r * s.kb;
            if (q->dst_ids) {
                memcpy(q->dst_ids, ids, (size_t)q->k * 8);
                memcpy(q->dst_scores, sc, (size_t)q->k * 4);
            } else {
                q->ids.assign(ids, ids + q->k);
                q->scores.assign(sc, sc + q->k);
            }
        }
        if (q->dst_lat) *q->dst_lat = q->lat_ns;
        q->done = true;
        if (q->dst_ids) {  // replay request: nobody collects it
            if (st != SINDI_OK && replay_st == SINDI_OK) {
                replay_st = st;
                replay_msg = msg;
            }
            --replay_left;
            reqs.erase(q->ticket);
        }
    }
    stats.completed += (int64_t)s.reqs.size();
    s.reqs.clear();
    if (s.region_bytes) arena.release(s.region_off, s.region_bytes);
    s.region_bytes = 0;
    if (retry_owner == &s) retry_owner = nullptr;
    s.wants_retry_buffer = false;
    s.busy = false;
    if (--n_busy == 0)
        stats.busy_ms += std::chrono::duration<double, std::milli>(t1 - busy_since).count();
    cv_done.notify_all();
}

// The slot's event has fired.  Rows whose candidate threshold missed are
// retried on the slot's stream (the dispatcher does not wait for them): first
// with a threshold over every tile, then with none; the batch is published
// when no row is left.
void sindi_server::complete(Slot &s)
{
    if (s.stage == 0 && s.h_err.p[0] != 0) {
        finish(s, fail(SINDI_E_INTERNAL, "sindi_server: validated queries flagged 0x%x", s.h_err.p[0]),
               last_error());
        return;
    }
    // stage 0 and 2 leave their count in h_fail[0] (rows), stage 1 in h_fail[1] (rows2)
    const uint32_t left = s.h_fail.p[s.stage == 1 ? 1 : 0];
    if (left == 0) {
        finish(s, SINDI_OK, std::string());
        return;
    }
    if (s.stage == 2) {
        finish(s, fail(SINDI_E_INTERNAL, "sindi_server: %u queries unresolved", left), last_error());
        return;
    }
    if (s.stage == 0) {
        {
            std::lock_guard<std::mutex> lock(mu);
            stats.retried += (int64_t)left;
        }
        // the sampled pass is done: its arena share goes back; retries run in the
        // server's retry buffer, one batch at a time
        arena.release(s.region_off, s.region_bytes);
        s.region_bytes = 0;
    }
    s.wants_retry_buffer = true;
    start_retry(s);
}

// Enqueue the next retry stage of a slot's batch once the retry buffer is its.
void sindi_server::start_retry(Slot &s)
{
    if (retry_owner && retry_owner != &s) return;  // the dispatcher tries again
    retry_owner = &s;
    s.wants_retry_buffer = false;
    s.sc.arena = retry_buf.as<unsigned char>();
    s.sc.arena_bytes = retry_buf.bytes;
    sindi_status e;
    if (s.stage == 0)
        e = enqueue_retry(s, kPassFullSample, s.sc.rows, s.h_fail.p[0], s.sc.rows2, s.sc.n_rows + 1,
                          s.h_fail.p + 1);
    else
        e = enqueue_retry(s, kPassKeepAll, s.sc.rows2, s.h_fail.p[1], s.sc.rows, s.sc.n_rows,
                          s.h_fail.p);
    s.stage += 1;
    if (e != SINDI_OK) {
        s.launch_st = e;  // the dispatcher drains the stream and publishes the error
        s.launch_msg = last_error();
    }
}

void sindi_server::run()
{
    (void)hipSetDevice(ix->device);
    std::vector<Request *> batch;
    for (;;) {
        // publish finished batches, and start waiting retries
        for (auto &sp : slots) {
            Slot &s = *sp;
            if (!s.busy) continue;
            if (s.wants_retry_buffer && s.launch_st == SINDI_OK) {
                start_retry(s);
                continue;
            }
            if (s.launch_st != SINDI_OK) {
                // the stream may still hold part of the batch: drain it first
                (void)hipStreamSynchronize(s.stream);
                finish(s, s.launch_st, s.launch_msg);
                continue;
            }
            const hipError_t e = hipEventQuery(s.done);
            if (e == hipErrorNotReady) continue;
            if (e != hipSuccess)
                finish(s, fail(SINDI_E_HIP, "sindi_server: batch failed: %s", hipGetErrorString(e)),
                       last_error());
            else
                complete(s);
        }
        // start the next batch on a free slot: as many queued requests as the largest
        // free block of candidate memory holds (at most max_batch)
        Slot *free_slot = nullptr;
        size_t region = 0, off = 0;
        {
            std::unique_lock<std::mutex> lock(mu);
            bool any_busy = false;
            for (auto &sp : slots) {
                if (sp->busy) any_busy = true;
                else if (!free_slot) free_slot = sp.get();
            }
            if (stop && !any_busy) return;
            int64_t fit = 0;
            if (!stop && !pending.empty() && free_slot) {
                fit = std::min<int64_t>(pass_group(main_shape, base, arena.largest()),
                                        std::min<int64_t>((int64_t)pending.size(), p.max_batch));
                if (fit < 1 && !mem_blocked) stats.memory_waits += 1;  // in-flight batches hold it
                mem_blocked = fit < 1;
            }
            if (fit < 1) {
                if (any_busy) cv_work.wait_for(lock, std::chrono::microseconds(20));
                else cv_work.wait(lock, [&] { return stop || !pending.empty(); });
                continue;
            }
            batch.clear();
            while ((int64_t)batch.size() < fit) {
                batch.push_back(pending.front());
                pending.pop_front();
            }
            region = pass_bytes(main_shape, base, fit);
            if (!arena.alloc(region, &off)) {  // cannot happen: fit came from the largest block
                for (auto it = batch.rbegin(); it != batch.rend(); ++it) pending.push_front(*it);
                continue;
            }
            stats.batches += 1;
            stats.largest_batch = std::max<int64_t>(stats.largest_batch, (int64_t)batch.size());
            stats.arena_peak_bytes = std::max<int64_t>(stats.arena_peak_bytes, (int64_t)arena.peak);
            if (n_busy++ == 0) busy_since = Clock::now();
        }
        free_slot->region_off = off;
        free_slot->region_bytes = region;
        free_slot->sc.arena = arena.buf.as<unsigned char>() + off;
        free_slot->sc.arena_bytes = region;
        launch(*free_slot, batch);
    }
}

// ------------------------------------------------------------------ C ABI
namespace {

sindi_status create_impl(const sindi_index *ix, const sindi_server_params *pp, sindi_server **out)
{
    if (!ix || !out) return fail(SINDI_E_INVALID, "sindi_server_create: null argument");
    sindi_server_params p{};
    if (pp) p = *pp;
    if (!p.max_inflight) p.max_inflight = 3;
    if (!p.max_batch) p.max_batch = 256;
    if (!p.k_max) p.k_max = 100;
    if (!p.max_query_nnz) p.max_query_nnz = 512;
    if (!p.max_queue) p.max_queue = (int64_t)1 << 20;
    if (!p.workspace_bytes) p.workspace_bytes = (int64_t)2 << 30;
    if (p.max_inflight < 1 || p.max_inflight > kMaxSlots)
        return fail(SINDI_E_INVALID, "sindi_server_create: max_inflight must be in [1, %d]", kMaxSlots);
    if (p.max_batch < 1 || p.max_batch > kMaxBatchQueries)
        return fail(SINDI_E_INVALID, "sindi_server_create: max_batch must be in [1, %d]", kMaxBatchQueries);
    if (p.max_query_nnz < 1 || p.max_query_nnz > kQueryHash / 2)
        return fail(SINDI_E_INVALID, "sindi_server_create: max_query_nnz must be in [1, %d]", kQueryHash / 2);
    if (p.max_queue < 1 || p.workspace_bytes < 1)
        return fail(SINDI_E_INVALID, "sindi_server_create: max_queue and workspace_bytes must be positive");
    if (!p.search.gamma) p.search.gamma = std::max(p.k_max, 500);

    std::unique_ptr<sindi_server> srv(new sindi_server());
    srv->ix = ix;
    srv->p = p;
    sindi_status st = make_plan(ix, p.max_batch, p.k_max, p.search, true, "sindi_server_create", srv->base);
    if (st != SINDI_OK) return st;
    srv->base.max_qnnz = p.max_query_nnz;
    // candidate memory shared by the batches in flight (at least one query), and a
    // retry buffer for one query of either retry pass
    const Plan &pl = srv->base;
    srv->main_shape = pass_shape(ix, pl, kPassSampled);
    const size_t arena = std::max<size_t>((size_t)p.workspace_bytes, pass_bytes(srv->main_shape, pl, 1));
    const size_t retry = std::max(pass_bytes(pass_shape(ix, pl, kPassFullSample), pl, 1),
                                  pass_bytes(pass_shape(ix, pl, kPassKeepAll), pl, 1));

    int prev = 0;
    HIP_TRY(hipGetDevice(&prev));
    HIP_TRY(hipSetDevice(ix->device));
    auto alloc = [&]() -> sindi_status {
        HIP_TRY(srv->arena.buf.ensure(arena));
        srv->arena.reset();
        HIP_TRY(srv->retry_buf.ensure(retry));
        const size_t mb = (size_t)p.max_batch, qn = mb * (size_t)p.max_query_nnz, kk = (size_t)p.k_max;
        for (int i = 0; i < p.max_inflight; ++i) {
            srv->slots.emplace_back(new Slot());
            Slot &s = *srv->slots.back();
            HIP_TRY(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
            HIP_TRY(hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
            HIP_TRY(s.row_part.ensure(scratch_row_bytes(pl, p.max_batch, (int64_t)qn)));
            s.sc = carve_rows(s.row_part.as<unsigned char>(), pl, p.max_batch, (int64_t)qn);
            HIP_TRY(s.q_ptr.ensure((mb + 1) * 8));
            HIP_TRY(s.q_idx.ensure(qn * 4 + 4));
            HIP_TRY(s.q_val.ensure(qn * 4 + 4));
            HIP_TRY(s.d_ids.ensure(mb * kk * 8));
            HIP_TRY(s.d_scores.ensure(mb * kk * 4));
            HIP_TRY(s.h_ptr.alloc(mb + 1));
            HIP_TRY(s.h_idx.alloc(qn));
            HIP_TRY(s.h_val.alloc(qn));
            HIP_TRY(s.h_ids.alloc(mb * kk));
            HIP_TRY(s.h_scores.alloc(mb * kk));
            HIP_TRY(s.h_fail.alloc(2));
            HIP_TRY(s.h_err.alloc(1));
        }
        return SINDI_OK;
    };
    st = alloc();
    (void)hipSetDevice(prev);
    if (st != SINDI_OK) return st;
    sindi_server *raw = srv.get();
    raw->th = std::thread([raw] { raw->run(); });
    *out = srv.release();
    return SINDI_OK;
}

sindi_status submit_impl(sindi_server *srv, const int32_t *indices, const float *values, int32_t nnz,
                         int32_t k, int64_t *ticket)
{
    if (!srv || !ticket) return fail(SINDI_E_INVALID, "sindi_server_submit: null argument");
    sindi_status st = check_row(srv, indices, values, nnz, k, "sindi_server_submit");
    if (st != SINDI_OK) return st;
    std::unique_ptr<Request> q(new Request());
    q->k = k;
    q->nnz = nnz;
    q->own_idx.assign(indices, indices + nnz);
    q->own_val.assign(values, values + nnz);
    q->idx = q->own_idx.data();
    q->val = q->own_val.data();
    q->t0 = Clock::now();
    std::lock_guard<std::mutex> lock(srv->mu);
    if (srv->stop) return fail(SINDI_E_INVALID, "sindi_server_submit: server is stopping");
    if ((int64_t)srv->pending.size() >= srv->p.max_queue)
        return fail(SINDI_E_BUSY, "sindi_server_submit: %lld requests already queued",
                    (long long)srv->pending.size());
    q->ticket = srv->next_ticket++;
    *ticket = q->ticket;
    srv->pending.push_back(q.get());
    srv->reqs.emplace(q->ticket, std::move(q));
    srv->stats.submitted += 1;
    srv->cv_work.notify_one();
    return SINDI_OK;
}

sindi_status wait_impl(sindi_server *srv, int64_t ticket, int64_t *ids, float *scores,
                       int64_t *latency_ns, double timeout_ms)
{
    if (!srv) return fail(SINDI_E_INVALID, "sindi_server_wait: null server");
    std::unique_lock<std::mutex> lock(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end() || it->second->dst_ids)
        return fail(SINDI_E_INVALID, "sindi_server_wait: unknown ticket %lld", (long long)ticket);
    Request *q = it->second.get();
    auto ready = [&] { return q->done; };
    if (timeout_ms < 0) srv->cv_done.wait(lock, ready);
    else if (!srv->cv_done.wait_for(lock, std::chrono::duration<double, std::milli>(timeout_ms), ready))
        return fail(SINDI_E_BUSY, "sindi_server_wait: ticket %lld not finished", (long long)ticket);
    const sindi_status st = q->st;
    if (st == SINDI_OK) {
        if (ids) memcpy(ids, q->ids.data(), (size_t)q->k * 8);
        if (scores) memcpy(scores, q->scores.data(), (size_t)q->k * 4);
        if (latency_ns) *latency_ns = q->lat_ns;
    } else {
        fail(st, "%s", q->msg.c_str());
    }
    srv->reqs.erase(it);
    return st;
}

sindi_status replay_impl(sindi_server *srv, const sindi_csr *qc, const int32_t *ks,
                         const double *arrival_s, int64_t *out_ids, float *out_scores,
                         int64_t *latency_ns)
{
    const char *fn = "sindi_server_replay";
    if (!srv || !qc || !out_ids || !out_scores || !latency_ns)
        return fail(SINDI_E_INVALID, "%s: null argument", fn);
    if (qc->on_device) return fail(SINDI_E_INVALID, "%s: queries must be host memory", fn);
    if (qc->n_cols != srv->ix->n_cols)
        return fail(SINDI_E_INVALID, "%s: column count mismatch", fn);
    const int64_t n = qc->n_rows;
    if (n < 0) return fail(SINDI_E_INVALID, "%s: bad query shape", fn);
    if (n == 0) return SINDI_OK;
    if (!ks || !arrival_s) return fail(SINDI_E_INVALID, "%s: null argument", fn);
    sindi_status st = validate_host_csr(qc, "queries", srv->p.max_query_nnz);
    if (st != SINDI_OK) return st;
    for (int64_t r = 0; r < n; ++r) {
        if (ks[r] < 1 || ks[r] > srv->p.k_max)
            return fail(SINDI_E_INVALID, "%s: k of row %lld outside [1, %d]", fn, (long long)r, srv->p.k_max);
        if (!std::isfinite(arrival_s[r]) || arrival_s[r] < 0 || (r && arrival_s[r] < arrival_s[r - 1]))
            return fail(SINDI_E_INVALID, "%s: arrival times must be finite, >= 0, non-decreasing", fn);
    }
    const int32_t kmax = srv->p.k_max;
    for (int64_t i = 0; i < n * kmax; ++i) {
        out_ids[i] = -1;
        out_scores[i] = -INFINITY;
    }
    for (int64_t i = 0; i < n; ++i) latency_ns[i] = -1;
    std::vector<std::unique_ptr<Request>> made((size_t)n);
    for (int64_t r = 0; r < n; ++r) {
        Request *q = new Request();
        made[r].reset(q);
        q->k = ks[r];
        q->nnz = (int32_t)(qc->indptr[r + 1] - qc->indptr[r]);
        q->idx = qc->indices + qc->indptr[r];
        q->val = qc->values + qc->indptr[r];
        q->dst_ids = out_ids + r * kmax;
        q->dst_scores = out_scores + r * kmax;
        q->dst_lat = latency_ns + r;
    }
    {
        std::lock_guard<std::mutex> lock(srv->mu);
        if (srv->stop) return fail(SINDI_E_INVALID, "%s: server is stopping", fn);
        if (srv->replay_left) return fail(SINDI_E_INVALID, "%s: another replay is running", fn);
        srv->replay_left = n;
        srv->replay_st = SINDI_OK;
    }
    const auto start = Clock::now();
    int64_t r = 0;
    while (r < n) {
        const auto due = start + std::chrono::duration_cast<Clock::duration>(
                                     std::chrono::duration<double>(arrival_s[r]));
        auto now = Clock::now();
        if (now < due) {
            if (due - now > std::chrono::microseconds(200))
                std::this_thread::sleep_until(due - std::chrono::microseconds(100));
            else
                std::this_thread::yield();
            continue;
        }
        // every request already due goes in under one lock
        std::lock_guard<std::mutex> lock(srv->mu);
        for (; r < n; ++r) {
            const auto due_r = start + std::chrono::duration_cast<Clock::duration>(
                                           std::chrono::duration<double>(arrival_s[r]));
            if (due_r > now) break;
            Request *q = made[r].release();
            q->t0 = due_r;
            q->ticket = srv->next_ticket++;
            srv->pending.push_back(q);
            srv->reqs.emplace(q->ticket, std::unique_ptr<Request>(q));
            srv->stats.submitted += 1;
        }
        srv->cv_work.notify_one();
    }
    std::unique_lock<std::mutex> lock(srv->mu);
    srv->cv_done.wait(lock, [&] { return srv->replay_left == 0; });
    if (srv->replay_st != SINDI_OK) return fail(srv->replay_st, "%s", srv->replay_msg.c_str());
    for (int64_t i = 0; i < n; ++i)
        if (latency_ns[i] < 0) return fail(SINDI_E_INTERNAL, "%s: request %lld lost", fn, (long long)i);
    return SINDI_OK;
}

}  // namespace

extern "C" {

sindi_status sindi_server_create(const sindi_index *idx, const sindi_server_params *params,
                                 sindi_server **out)
{
    try {
        return create_impl(idx, params, out);
    } catch (const std::bad_alloc &) {
        return fail(SINDI_E_OOM, "sindi_server_create: host allocation failed");
    } catch (...) {
        return fail(SINDI_E_INTERNAL, "sindi_server_create: unexpected exception");
    }
}

sindi_status sindi_server_submit(sindi_server *srv, const int32_t *indices, const float *values,
                                 int32_t nnz, int32_t k, int64_t *ticket)
{
    try {
        return submit_impl(srv, indices, values, nnz, k, ticket);
    } catch (const std::bad_alloc &) {
        return fail(SINDI_E_OOM, "sindi_server_submit: host allocation failed");
    } catch (...) {
        return fail(SINDI_E_INTERNAL, "sindi_server_submit: unexpected exception");
    }
}

sindi_status sindi_server_wait(sindi_server *srv, int64_t ticket, int64_t *ids, float *scores,
                               int64_t *latency_ns, double timeout_ms)
{
    try {
        return wait_impl(srv, ticket, ids, scores, latency_ns, timeout_ms);
    } catch (...) {
        return fail(SINDI_E_INTERNAL, "sindi_server_wait: unexpected exception");
    }
}

sindi_status sindi_server_replay(sindi_server *srv, const sindi_csr *queries, const int32_t *ks,
                                 const double *arrival_s, int64_t *out_ids, float *out_scores,
                                 int64_t *latency_ns)
{
    try {
        return replay_impl(srv, queries, ks, arrival_s, out_ids, out_scores, latency_ns);
    } catch (const std::bad_alloc &) {
        return fail(SINDI_E_OOM, "sindi_server_replay: host allocation failed");
    } catch (...) {
        return fail(SINDI_E_INTERNAL, "sindi_server_replay: unexpected exception");
    }
}

sindi_status sindi_server_get_stats(const sindi_server *srv, sindi_server_stats *out)
{
    if (!srv || !out) return fail(SINDI_E_INVALID, "sindi_server_get_stats: null argument");
    sindi_server *s = const_cast<sindi_server *>(srv);
    std::lock_guard<std::mutex> lock(s->mu);
    *out = s->stats;
    if (s->n_busy)
        out->busy_ms += std::chrono::duration<double, std::milli>(Clock::now() - s->busy_since).count();
    return SINDI_OK;
}

void sindi_server_destroy(sindi_server *srv)
{
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lock(srv->mu);
        srv->stop = true;
        srv->cv_work.notify_all();
    }
    if (srv->th.joinable()) srv->th.join();
    delete srv;
}

}  // extern "C"
