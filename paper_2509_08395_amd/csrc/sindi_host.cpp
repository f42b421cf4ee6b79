// Host side of the SINDI library: input validation, mass-ratio pruning,
// window/tile layout of the inverted lists, device upload, and the search
// pipeline that drives the gfx950 kernels.  Implements include/sindi.h
// (the serving loop is in sindi_server.cpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "sindi.h"
#include "sindi_internal.h"
#include "sindi_state.h"

namespace sindi {

// ------------------------------------------------------------------ errors
namespace {
thread_local std::string g_err;
}

sindi_status fail(sindi_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

const char *last_error() { return g_err.c_str(); }

int host_threads()
{
    const char *env = getenv("OMP_NUM_THREADS");
    int n = env ? atoi(env) : 0;
    if (n <= 0) n = (int)std::thread::hardware_concurrency();
    return n < 1 ? 1 : (n > 64 ? 64 : n);
}

// ------------------------------------------------------------------ profiling
namespace {
struct Profiler {
    std::mutex mu;
    std::atomic<bool> on{false};
    struct Rec {
        int cat;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    int64_t n[5] = {0, 0, 0, 0, 0};
    double ms[5] = {0, 0, 0, 0, 0};
};
Profiler g_prof;
}  // namespace

hipError_t timed_launch(int cat, hipStream_t s, hipError_t (*fn)(void *), void *ctx)
{
    if (!g_prof.on.load(std::memory_order_relaxed)) return fn(ctx);
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&b);
    if (e != hipSuccess) return e;
    e = hipEventRecord(a, s);
    if (e != hipSuccess) return e;
    e = fn(ctx);
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, s);
    std::lock_guard<std::mutex> lock(g_prof.mu);
    g_prof.pending.push_back({cat, a, b});
    return e;
}

sindi_status profile_enable(int32_t enable)
{
    g_prof.on.store(enable != 0);
    return SINDI_OK;
}

sindi_status profile_read(sindi_profile *out, int32_t reset)
{
    std::lock_guard<std::mutex> lock(g_prof.mu);
    sindi_status st = SINDI_OK;
    for (auto &r : g_prof.pending) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess && st == SINDI_OK)
            st = fail(SINDI_E_HIP, "sindi_profile_read: %s", hipGetErrorString(e));
        g_prof.n[r.cat] += 1;
        g_prof.ms[r.cat] += ms;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof.pending.clear();
    if (out)
        for (int i = 0; i < 5; ++i) {
            out->launches[i] = g_prof.n[i];
            out->ms[i] = g_prof.ms[i];
        }
    if (reset)
        for (int i = 0; i < 5; ++i) {
            g_prof.n[i] = 0;
            g_prof.ms[i] = 0.0;
        }
    return st;
}

namespace {

// FP32 -> FP16 / BF16, round to nearest even.
uint16_t to_f16(float x) { return __builtin_bit_cast(uint16_t, (_Float16)x); }
uint16_t to_bf16(float x)
{
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Largest tile of a window split: three 512-thread scoring workgroups (one
// query each) still share a CU's 160 KB of LDS, and fewer, larger tiles cut
// the per-tile work (list layout, barriers, read-out) per posting.  (LDS is
// allocated in 512-byte units; the kernel's static LDS is under 128 bytes.)
constexpr int32_t kDefaultTile = 12500;
static_assert(3 * ((accumulate_lds_bytes(1, kDefaultTile) + 128 + 511) / 512 * 512) <=
                  160 * 1024,
              "default tile too large");
constexpr int32_t kDefaultBatch = 1;
constexpr int32_t kDefaultCandCap = 32768;
constexpr int32_t kDefaultSampleTiles = 8;
// one persistent, queue-fed launch per scoring pass (58.7 against 58.9 ms per 7,000 queries
// with one workgroup per (query, tile run); 79.0 against 80.5 ms on the serving mix)
constexpr int32_t kDefaultSchedule = 2;
constexpr int32_t kDefaultGamma = 500;
constexpr size_t kCandBudget = size_t(4) << 30;  // candidate buffer bytes per pass

}  // namespace

// Structural check of a host CSR (Def. 1: each row a set of non-zero
// entries over [0, n_cols); ids strictly ascending; finite values).
sindi_status validate_host_csr(const sindi_csr *m, const char *what, int64_t max_row,
                               int64_t *longest)
{
    if (m->n_rows < 0 || m->n_cols < 1 || m->n_cols > INT32_MAX || m->nnz < 0)
        return fail(SINDI_E_INVALID, "%s: bad shape (rows %lld, cols %lld, nnz %lld)", what,
                    (long long)m->n_rows, (long long)m->n_cols, (long long)m->nnz);
    if (!m->indptr || (m->nnz > 0 && (!m->indices || !m->values)))
        return fail(SINDI_E_INVALID, "%s: null array", what);
    if (m->indptr[0] != 0 || m->indptr[m->n_rows] != m->nnz)
        return fail(SINDI_E_INVALID, "%s: indptr[0] must be 0 and indptr[n_rows] == nnz", what);
    std::atomic<int64_t> bad_row{-1}, long_row{0};
    std::atomic<int> bad_kind{0};
    parallel_for(m->n_rows, [&](int64_t lo, int64_t hi) {
        int64_t lr = 0;
        for (int64_t r = lo; r < hi && bad_row.load(std::memory_order_relaxed) < 0; ++r) {
            const int64_t a = m->indptr[r], b = m->indptr[r + 1];
            lr = std::max(lr, b - a);
            int kind = 0;
            if (b < a || a < 0 || b > m->nnz) kind = 1;
            else if (max_row > 0 && b - a > max_row) kind = 5;
            else
                for (int64_t e = a; e < b && !kind; ++e) {
                    const int32_t id = m->indices[e];
                    if (id < 0 || id >= m->n_cols) kind = 2;
                    else if (e + 1 < b && m->indices[e + 1] <= id) kind = 3;
                    else if (!std::isfinite(m->values[e])) kind = 4;
                }
            if (kind) {
                int64_t expect = -1;
                if (bad_row.compare_exchange_strong(expect, r)) bad_kind = kind;
            }
        }
        int64_t cur = long_row.load();
        while (lr > cur && !long_row.compare_exchange_weak(cur, lr)) {
        }
    });
    if (longest) *longest = long_row.load();
    if (bad_row >= 0) {
        static const char *msg[] = {"", "row pointers not monotone", "term id out of range",
                                    "term ids not strictly ascending (duplicate or unsorted)",
                                    "non-finite value", "row has too many entries"};
        if (bad_kind.load() == 5)
            return fail(SINDI_E_INVALID, "%s: row %lld: more than %lld entries", what,
                        (long long)bad_row.load(), (long long)max_row);
        return fail(SINDI_E_INVALID, "%s: row %lld: %s", what, (long long)bad_row.load(),
                    msg[bad_kind.load()]);
    }
    return SINDI_OK;
}

namespace {

// Def. 6 for one row: keep[e] = 1 for the entries of the alpha-mass
// subvector.  Entries ranked by |x| descending, equal |x| by ascending term
// id; prefix sums of |x| in FP64 in that order; r = first prefix reaching
// alpha * mass, mass being the full sum in the same order.  Explicit zeros
// are not entries and are never kept.
void mass_ratio_row(const int32_t *idx, const float *val, int64_t n, double alpha,
                    std::vector<int64_t> &order, uint8_t *keep)
{
    order.clear();
    for (int64_t e = 0; e < n; ++e) {
        keep[e] = 0;
        if (val[e] != 0.0f) order.push_back(e);
    }
    if (order.empty()) return;
    if (alpha >= 1.0) {
        for (int64_t e : order) keep[e] = 1;
        return;
    }
    std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
        const float ax = std::fabs(val[x]), ay = std::fabs(val[y]);
        return ax > ay || (ax == ay && idx[x] < idx[y]);
    });
    double mass = 0.0;
    for (int64_t e : order) mass += (double)std::fabs(val[e]);
    const double thr = alpha * mass;
    double run = 0.0;
    size_t r = 0;
    while (r < order.size()) {
        run += (double)std::fabs(val[order[r]]);
        ++r;
        if (run >= thr) break;
    }
    for (size_t t = 0; t < r; ++t) keep[order[t]] = 1;
}

// Vector Number Pruning (Sec. 4.1): the vn non-zero entries of largest |x|,
// ties to the lower term id (the order of Def. 6).
void vnp_row(const int32_t *idx, const float *val, int64_t n, int64_t vn,
             std::vector<int64_t> &order, uint8_t *keep)
{
    order.clear();
    for (int64_t e = 0; e < n; ++e) {
        keep[e] = 0;
        if (val[e] != 0.0f) order.push_back(e);
    }
    const size_t r = (size_t)std::min<int64_t>(vn, (int64_t)order.size());
    auto before = [&](int64_t x, int64_t y) {
        const float ax = std::fabs(val[x]), ay = std::fabs(val[y]);
        return ax > ay || (ax == ay && idx[x] < idx[y]);
    };
    if (r < order.size()) std::nth_element(order.begin(), order.begin() + r, order.end(), before);
    for (size_t t = 0; t < r; ++t) keep[order[t]] = 1;
}

// List Pruning (Sec. 4.1): every term's list keeps its lmax non-zero entries
// of largest |x|, ties to the lower document id; only entries keep already
// holds take part, and keep is narrowed in place.
void list_prune(const sindi_csr *c, int64_t lmax, std::vector<uint8_t> &keep)
{
    const int64_t nc = c->n_cols, nd = c->n_rows;
    std::vector<int64_t> start((size_t)nc + 1, 0);
    for (int64_t e = 0; e < c->nnz; ++e)
        if (keep[e]) start[(size_t)c->indices[e] + 1]++;
    for (int64_t j = 0; j < nc; ++j) start[j + 1] += start[j];
    struct Ent {
        float a;
        uint32_t doc;
        int64_t pos;
    };
    std::vector<Ent> ents((size_t)start[nc]);
    {
        std::vector<int64_t> fill(start.begin(), start.end() - 1);
        for (int64_t i = 0; i < nd; ++i)
            for (int64_t e = c->indptr[i]; e < c->indptr[i + 1]; ++e)
                if (keep[e]) ents[(size_t)fill[c->indices[e]]++] = {std::fabs(c->values[e]), (uint32_t)i, e};
    }
    parallel_for(nc, [&](int64_t lo, int64_t hi) {
        auto before = [](const Ent &x, const Ent &y) { return x.a > y.a || (x.a == y.a && x.doc < y.doc); };
        for (int64_t j = lo; j < hi; ++j) {
            Ent *b = ents.data() + start[j], *e = ents.data() + start[j + 1];
            if (e - b <= lmax) continue;
            std::nth_element(b, b + lmax, e, before);
            for (Ent *x = b + lmax; x < e; ++x) keep[(size_t)x->pos] = 0;
        }
    });
}

// The same index built on the device (sindi_build.hip): pruning, per-list
// counts, group offsets and the ordered fill run as kernels; the host only
// lays out the tiles, scans the per-tile totals and checks the flags.
sindi_status build_device(const sindi_csr *c, const sindi_build_params *p, hipStream_t s,
                          sindi_index *ix, std::vector<int64_t> &tile_doc)
{
    const int64_t nd = c->n_rows, nc = c->n_cols, nnz = c->nnz, n_tiles = ix->n_tiles;
    const hipMemcpyKind kind = c->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    auto oom = [](hipError_t e, const char *what) -> sindi_status {
        if (e == hipErrorOutOfMemory) return fail(SINDI_E_OOM, "sindi_build: device allocation of %s failed", what);
        return fail(SINDI_E_HIP, "sindi_build: %s: %s", what, hipGetErrorString(e));
    };
    hipError_t e;
#define BUILD_ALLOC(buf, bytes, what)                                                          \
    if ((e = (buf).ensure(bytes)) != hipSuccess) return oom(e, what)
    BUILD_ALLOC(ix->indptr, (size_t)(nd + 1) * 8, "indptr");
    BUILD_ALLOC(ix->indices, (size_t)nnz * 4 + 4, "indices");
    BUILD_ALLOC(ix->values, (size_t)nnz * 4 + 4, "values");
    HIP_TRY(hipMemcpyAsync(ix->indptr.p, c->indptr, (size_t)(nd + 1) * 8, kind, s));
    if (nnz) {
        HIP_TRY(hipMemcpyAsync(ix->indices.p, c->indices, (size_t)nnz * 4, kind, s));
        HIP_TRY(hipMemcpyAsync(ix->values.p, c->values, (size_t)nnz * 4, kind, s));
    }
    const int64_t *ptr = ix->indptr.as<int64_t>();
    const int32_t *idx = ix->indices.as<int32_t>();
    const float *val = ix->values.as<float>();
    DBuf err, keep, long_rows, n_long, cnt, kept, tgroups;
    BUILD_ALLOC(err, 4, "flags");
    HIP_TRY(launch_fill_u32(err.as<uint32_t>(), 1, 0u, s));
    auto flags = [&](int32_t &out_err) -> sindi_status {
        HIP_TRY(hipMemcpyAsync(&out_err, err.p, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return SINDI_OK;
    };
    int32_t ferr = 0;
    sindi_status st;
    if (c->on_device) {
        HIP_TRY(build_check_rows(ptr, idx, val, nd, nc, nnz, err.as<int32_t>(), s));
        if ((st = flags(ferr)) != SINDI_OK) return st;
        if (ferr)
            return fail(SINDI_E_INVALID,
                        "sindi_build: malformed corpus rows (flags 0x%x: 1 row pointers, 2 term "
                        "id range, 4 order, 8 non-finite)", ferr);
    }
    // Alg. 3's pruning step on the device
    BUILD_ALLOC(keep, (size_t)nnz + 4, "keep mask");
    BUILD_ALLOC(long_rows, (size_t)nd * 4 + 4, "long-row list");
    BUILD_ALLOC(n_long, 4, "counter");
    HIP_TRY(launch_fill_u32(n_long.as<uint32_t>(), 1, 0u, s));
    const int32_t mode = p->prune == SINDI_PRUNE_VNP ? SINDI_PRUNE_VNP : SINDI_PRUNE_MRP;
    HIP_TRY(build_prune_rows(ptr, idx, val, nd, mode, p->alpha, p->vn, keep.as<uint8_t>(),
                             long_rows.as<int32_t>(), n_long.as<uint32_t>(), err.as<int32_t>(), s));
    uint32_t h_long = 0;
    HIP_TRY(hipMemcpyAsync(&h_long, n_long.p, 4, hipMemcpyDeviceToHost, s));
    if ((st = flags(ferr)) != SINDI_OK) return st;
    if (ferr & 128)
        return fail(SINDI_E_INVALID, "sindi_build: a row holds more than %d entries; build it on "
                    "the host (gpu_build = 0)", kLongRow);
    HIP_TRY(build_prune_long(ptr, idx, val, long_rows.as<int32_t>(), (int32_t)h_long, mode,
                             p->alpha, p->vn, keep.as<uint8_t>(), s));
    long_rows.release();
    // Alg. 1: list sizes per (tile, term)
    const size_t stride = (size_t)nc + 1;
    BUILD_ALLOC(ix->tile_doc, tile_doc.size() * 8, "tile_doc");
    HIP_TRY(hipMemcpyAsync(ix->tile_doc.p, tile_doc.data(), tile_doc.size() * 8, hipMemcpyHostToDevice, s));
    BUILD_ALLOC(cnt, (size_t)n_tiles * stride * 4, "list counts");
    BUILD_ALLOC(ix->term_max, (size_t)nc * 4, "term maxima");
    BUILD_ALLOC(kept, 8, "counter");
    HIP_TRY(launch_fill_u32(cnt.as<uint32_t>(), (int64_t)n_tiles * (int64_t)stride, 0u, s));
    HIP_TRY(launch_fill_u32(ix->term_max.as<uint32_t>(), nc, 0u, s));
    HIP_TRY(launch_fill_u32(kept.as<uint32_t>(), 2, 0u, s));
    HIP_TRY(build_count_lists(ptr, idx, val, keep.as<uint8_t>(), nd, nc, ix->tile_doc.as<int64_t>(),
                              n_tiles, p->value_dtype, cnt.as<uint32_t>(),
                              ix->term_max.as<uint32_t>(), kept.as<unsigned long long>(),
                              err.as<int32_t>(), s));
    BUILD_ALLOC(ix->term_goff, (size_t)n_tiles * stride * 4, "term offsets");
    BUILD_ALLOC(tgroups, (size_t)n_tiles * 8 + 8, "tile totals");
    HIP_TRY(build_list_offsets(cnt.as<uint32_t>(), n_tiles, nc, ix->term_goff.as<uint32_t>(),
                               tgroups.as<int64_t>(), err.as<int32_t>(), s));
    std::vector<int64_t> tile_post((size_t)n_tiles + 1, 0);
    unsigned long long h_kept = 0;
    HIP_TRY(hipMemcpyAsync(tile_post.data() + 1, tgroups.p, (size_t)n_tiles * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&h_kept, kept.p, 8, hipMemcpyDeviceToHost, s));
    if ((st = flags(ferr)) != SINDI_OK) return st;
    if (ferr & 32) return fail(SINDI_E_RANGE, "sindi_build: a kept value overflows the storage type");
    if (ferr & 16)
        return fail(SINDI_E_INVALID, "sindi_build: a tile needs more than %u groups of 4 postings",
                    kTileGroupsMax);
    for (int64_t t = 0; t < n_tiles; ++t) tile_post[t + 1] = tile_post[t] + 4 * tile_post[t + 1];
    const int64_t n_slots = tile_post[n_tiles];
    if (n_slots >= ((int64_t)1 << 34))
        return fail(SINDI_E_INVALID, "sindi_build: more than 2^34 index postings");
    ix->n_post = (int64_t)h_kept;
    ix->n_slots = n_slots;
    BUILD_ALLOC(ix->tile_post, tile_post.size() * 8, "tile_post");
    HIP_TRY(hipMemcpyAsync(ix->tile_post.p, tile_post.data(), tile_post.size() * 8, hipMemcpyHostToDevice, s));
    const size_t vbytes = p->value_dtype == SINDI_F32 ? 4 : 2;
    BUILD_ALLOC(ix->post_doc, ((size_t)n_slots + kTailSlots) * 2, "posting ids");
    BUILD_ALLOC(ix->post_val, ((size_t)n_slots + kTailSlots) * vbytes, "posting values");
    HIP_TRY(launch_fill_u32(ix->post_val.as<uint32_t>(), (int64_t)(ix->post_val.bytes / 4), 0u, s));
    HIP_TRY(launch_fill_u32(ix->post_doc.as<uint32_t>(), (int64_t)(ix->post_doc.bytes / 4), 0u, s));
    HIP_TRY(build_fill_lists(ptr, idx, val, keep.as<uint8_t>(), ix->tile_doc.as<int64_t>(),
                             ix->tile_post.as<int64_t>(), ix->term_goff.as<uint32_t>(), n_tiles, nc,
                             p->value_dtype, ix->post_doc.as<uint16_t>(), ix->post_val.p, s));
    HIP_TRY(build_fill_pads(ix->term_goff.as<uint32_t>(), cnt.as<uint32_t>(), ix->tile_post.as<int64_t>(),
                            n_tiles, nc, ix->post_doc.as<uint16_t>(), s));
    HIP_TRY(build_deal_chunks(ix->term_goff.as<uint32_t>(), ix->tile_post.as<int64_t>(), n_tiles, nc,
                              (int32_t)vbytes, ix->post_doc.as<uint16_t>(), ix->post_val.p, s));
    HIP_TRY(hipStreamSynchronize(s));
#undef BUILD_ALLOC
    ix->h_tile_doc = std::move(tile_doc);
    return SINDI_OK;
}

sindi_status build_impl(const sindi_csr *c, const sindi_build_params *p, hipStream_t s,
                        sindi_index **out)
{
    if (!c || !p || !out) return fail(SINDI_E_INVALID, "sindi_build: null argument");
    if (c->on_device && !p->gpu_build)
        return fail(SINDI_E_INVALID, "sindi_build: a device corpus needs gpu_build = 1");
    if (p->prune < SINDI_PRUNE_MRP || p->prune > SINDI_PRUNE_MRP_LP)
        return fail(SINDI_E_INVALID, "sindi_build: unknown pruning rule %d", p->prune);
    const bool use_mrp = p->prune == SINDI_PRUNE_MRP || p->prune == SINDI_PRUNE_MRP_LP;
    const bool use_lp = p->prune == SINDI_PRUNE_LP || p->prune == SINDI_PRUNE_MRP_LP;
    if (use_mrp && !(p->alpha > 0.0 && p->alpha <= 1.0))
        return fail(SINDI_E_INVALID, "sindi_build: alpha must be in (0, 1], got %g", p->alpha);
    if (p->prune == SINDI_PRUNE_VNP && p->vn < 1)
        return fail(SINDI_E_INVALID, "sindi_build: vn must be >= 1");
    if (use_lp && p->list_len < 1) return fail(SINDI_E_INVALID, "sindi_build: list_len must be >= 1");
    if (p->gpu_build && use_lp)
        return fail(SINDI_E_INVALID, "sindi_build: list pruning is built on the host (gpu_build = 0)");
    if (p->gpu_build && c->n_rows >= (int64_t)INT32_MAX)
        return fail(SINDI_E_INVALID, "sindi_build: the device build takes fewer than 2^31 documents");
    if (p->window < 1) return fail(SINDI_E_INVALID, "sindi_build: window must be >= 1");
    if (p->value_dtype < 0 || p->value_dtype > 2)
        return fail(SINDI_E_INVALID, "sindi_build: unknown value dtype %d", p->value_dtype);
    const int32_t tile_req = p->tile ? p->tile : kDefaultTile;
    if (tile_req < 1 || tile_req > kTileMax)
        return fail(SINDI_E_INVALID, "sindi_build: tile must be in [1, %d]", kTileMax);
    if (c->n_rows >= (int64_t)0xFFFFFFFF)
        return fail(SINDI_E_INVALID, "sindi_build: too many documents");
    if (c->n_rows < 0 || c->n_cols < 1 || c->n_cols > INT32_MAX || c->nnz < 0 || !c->indptr ||
        (c->nnz > 0 && (!c->indices || !c->values)))
        return fail(SINDI_E_INVALID, "sindi_build: bad corpus shape or null array");
    sindi_status st = c->on_device ? SINDI_OK : validate_host_csr(c, "corpus", 0);
    if (st != SINDI_OK) return st;

    sindi_index *ix = new (std::nothrow) sindi_index();
    if (!ix) return fail(SINDI_E_OOM, "sindi_build: host allocation failed");
    std::unique_ptr<sindi_index> guard(ix);
    HIP_TRY(hipGetDevice(&ix->device));
    int lds = 0;
    HIP_TRY(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, ix->device));
    ix->max_lds = lds;
    const int64_t nd = c->n_rows, nc = c->n_cols;
    ix->n_docs = nd;
    ix->n_cols = nc;
    ix->nnz = c->nnz;
    ix->alpha = p->alpha;
    ix->prune = p->prune;
    ix->vn = p->vn;
    ix->list_len = p->list_len;
    ix->window = p->window;
    ix->dtype = p->value_dtype;
    ix->n_windows = nd ? (nd + p->window - 1) / p->window : 0;

    // windows of lambda documents (Sec. 3.3.1), each split into equal tiles
    std::vector<int64_t> tile_doc{0};
    int32_t tmax = 0;
    for (int64_t w = 0; w < ix->n_windows; ++w) {
        const int64_t w0 = w * p->window, wl = std::min(p->window, nd - w0);
        const int64_t nt = (wl + tile_req - 1) / tile_req;
        const int64_t base = wl / nt, extra = wl % nt;
        int64_t d = w0;
        for (int64_t i = 0; i < nt; ++i) {
            const int64_t l = base + (i < extra ? 1 : 0);
            d += l;
            tile_doc.push_back(d);
            tmax = std::max<int32_t>(tmax, (int32_t)l);
        }
    }
    const int64_t n_tiles = (int64_t)tile_doc.size() - 1;
    ix->n_tiles = n_tiles;
    ix->tile_max = tmax;
    ix->tile_stride = std::max<int32_t>(4, (tmax + 3) / 4 * 4);
    if ((int64_t)accumulate_lds_bytes(1, ix->tile_stride) > ix->max_lds)
        return fail(SINDI_E_INVALID, "sindi_build: tile of %d documents exceeds on-chip memory",
                    tmax);

    if (p->gpu_build) {
        if ((st = build_device(c, p, s, ix, tile_doc)) != SINDI_OK) return st;
        *out = guard.release();
        return SINDI_OK;
    }

    // Alg. 3's pruning step: alpha-mass subvector of every document (or the rule chosen)
    std::vector<uint8_t> keep((size_t)c->nnz);
    parallel_for(nd, [&](int64_t lo, int64_t hi) {
        std::vector<int64_t> order;
        for (int64_t r = lo; r < hi; ++r) {
            const int64_t a = c->indptr[r], n = c->indptr[r + 1] - a;
            if (use_mrp)
                mass_ratio_row(c->indices + a, c->values + a, n, p->alpha, order, keep.data() + a);
            else if (p->prune == SINDI_PRUNE_VNP)
                vnp_row(c->indices + a, c->values + a, n, p->vn, order, keep.data() + a);
            else
                for (int64_t e = 0; e < n; ++e) keep[a + e] = c->values[a + e] != 0.0f;
        }
    });
    if (use_lp) list_prune(c, p->list_len, keep);

    // Alg. 1 per tile: counts of every (tile, term) list, then offsets.  Every
    // list starts on a 4-posting boundary; the slots after its last posting up
    // to the next boundary are pad entries (value 0, the list's last document),
    // so the accumulate kernel reads whole 4-posting groups with no end masks.
    // term_goff holds group offsets relative to the tile's first group, with the
    // list's pad count in the top two bits.
    const size_t stride = (size_t)nc + 1;
    std::vector<uint32_t> term_goff((size_t)n_tiles * stride, 0u);
    std::vector<int64_t> tile_post((size_t)n_tiles + 1, 0);
    std::atomic<int> range_bad{0}, tile_big{0};
    int64_t n_post = 0;
    {
        std::mutex mx;
        parallel_for(n_tiles, [&](int64_t lo, int64_t hi) {
            int64_t kept = 0;
            for (int64_t t = lo; t < hi; ++t) {
                uint32_t *cnt = term_goff.data() + (size_t)t * stride;
                for (int64_t i = tile_doc[t]; i < tile_doc[t + 1]; ++i)
                    for (int64_t e = c->indptr[i]; e < c->indptr[i + 1]; ++e)
                        if (keep[e]) {
                            cnt[c->indices[e]]++;
                            ++kept;
                            if (p->value_dtype == SINDI_F16 && std::fabs(c->values[e]) > 65504.0f)
                                range_bad = 1;
                            if (p->value_dtype == SINDI_BF16 &&
                                std::isinf(__builtin_bit_cast(float, (uint32_t)to_bf16(c->values[e]) << 16)))
                                range_bad = 1;
                        }
                uint64_t g = 0;
                for (int64_t j = 0; j < nc; ++j) {
                    const uint32_t n = cnt[j];
                    const uint32_t pad = (4u - (n & 3u)) & 3u;
                    cnt[j] = (uint32_t)g | (pad << 30);
                    g += (n + 3u) / 4u;
                }
                if (g > kTileGroupsMax) tile_big = 1;
                cnt[nc] = (uint32_t)(g & kGoffMask);
                tile_post[t + 1] = (int64_t)g * 4;
            }
            std::lock_guard<std::mutex> lock(mx);
            n_post += kept;
        });
    }
    if (range_bad) return fail(SINDI_E_RANGE, "sindi_build: a kept value overflows the storage type");
    if (tile_big)
        return fail(SINDI_E_INVALID, "sindi_build: a tile needs more than %u groups of 4 postings",
                    kTileGroupsMax);
    for (int64_t t = 0; t < n_tiles; ++t) tile_post[t + 1] += tile_post[t];
    const int64_t n_slots = tile_post[n_tiles];
    if (n_slots >= ((int64_t)1 << 34))
        return fail(SINDI_E_INVALID, "sindi_build: more than 2^34 index postings");
    ix->n_post = n_post;
    ix->n_slots = n_slots;
    const size_t vbytes = p->value_dtype == SINDI_F32 ? 4 : 2;
    std::vector<uint16_t> post_doc((size_t)n_slots + kTailSlots, 0);
    std::vector<uint8_t> post_val(((size_t)n_slots + kTailSlots) * vbytes, 0);
    parallel_for(n_tiles, [&](int64_t lo, int64_t hi) {
        std::vector<uint64_t> fill(stride);
        for (int64_t t = lo; t < hi; ++t) {
            const uint32_t *go = term_goff.data() + (size_t)t * stride;
            for (size_t j = 0; j < stride; ++j) fill[j] = 4ull * (go[j] & kGoffMask);
            const int64_t P0 = tile_post[t], d0 = tile_doc[t];
            for (int64_t i = tile_doc[t]; i < tile_doc[t + 1]; ++i)
                for (int64_t e = c->indptr[i]; e < c->indptr[i + 1]; ++e) {
                    if (!keep[e]) continue;
                    const int64_t pos = P0 + (int64_t)fill[c->indices[e]]++;
                    post_doc[pos] = (uint16_t)((i - d0) * 4);  // byte offset of the score word
                    const float v = c->values[e];
                    if (p->value_dtype == SINDI_F32) memcpy(&post_val[pos * 4], &v, 4);
                    else {
                        const uint16_t h = p->value_dtype == SINDI_F16 ? to_f16(v) : to_bf16(v);
                        memcpy(&post_val[pos * 2], &h, 2);
                    }
                }
            // pads repeat the list's last document (value bits stay 0)
            for (int64_t j = 0; j < nc; ++j) {
                const uint32_t pad = go[j] >> 30;
                if (!pad) continue;
                const int64_t end = P0 + (int64_t)fill[j];
                for (uint32_t k = 0; k < pad; ++k) post_doc[end + k] = post_doc[end - 1];
            }
        }
    });

    // largest |stored value| per term: bounds every coarse partial sum
    std::vector<float> term_max((size_t)nc, 0.0f);
    {
        std::mutex mx;
        parallel_for(nd, [&](int64_t lo, int64_t hi) {
            std::vector<float> m((size_t)nc, 0.0f);
            for (int64_t i = lo; i < hi; ++i)
                for (int64_t e = c->indptr[i]; e < c->indptr[i + 1]; ++e) {
                    if (!keep[e]) continue;
                    float v = c->values[e];
                    if (p->value_dtype == SINDI_F16) v = (float)__builtin_bit_cast(_Float16, to_f16(v));
                    else if (p->value_dtype == SINDI_BF16)
                        v = __builtin_bit_cast(float, (uint32_t)to_bf16(v) << 16);
                    m[c->indices[e]] = std::max(m[c->indices[e]], std::fabs(v));
                }
            std::lock_guard<std::mutex> g(mx);
            for (int64_t j = 0; j < nc; ++j) term_max[j] = std::max(term_max[j], m[j]);
        });
    }

    // upload: unpruned corpus (Alg. 3 returns D too) and the tiled lists
    auto up = [&](DBuf &b, const void *src, size_t bytes) -> hipError_t {
        hipError_t e = b.ensure(bytes);
        if (e != hipSuccess) return e;
        if (bytes) e = hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, s);
        return e;
    };
    auto up_or_fail = [&](DBuf &b, const void *src, size_t bytes, const char *what) -> sindi_status {
        hipError_t e = up(b, src, bytes);
        if (e == hipErrorOutOfMemory) return fail(SINDI_E_OOM, "sindi_build: device allocation of %s failed", what);
        if (e != hipSuccess) return fail(SINDI_E_HIP, "sindi_build: upload of %s: %s", what, hipGetErrorString(e));
        return SINDI_OK;
    };
    if ((st = up_or_fail(ix->indptr, c->indptr, (size_t)(nd + 1) * 8, "indptr")) != SINDI_OK) return st;
    if ((st = up_or_fail(ix->indices, c->indices, (size_t)c->nnz * 4, "indices")) != SINDI_OK) return st;
    if ((st = up_or_fail(ix->values, c->values, (size_t)c->nnz * 4, "values")) != SINDI_OK) return st;
    if ((st = up_or_fail(ix->tile_doc, tile_doc.data(), tile_doc.size() * 8, "tile_doc")) != SINDI_OK) return st;
    if ((st = up_or_fail(ix->tile_post, tile_post.data(), tile_post.size() * 8, "tile_post")) != SINDI_OK) return st;
    if ((st = up_or_fail(ix->term_goff, term_goff.data(), term_goff.size() * 4, "term offsets")) != SINDI_OK) return st;
    if ((st = up_or_fail(ix->post_doc, post_doc.data(), post_doc.size() * 2, "posting ids")) != SINDI_OK) return st;
    if ((st = up_or_fail(ix->post_val, post_val.data(), post_val.size(), "posting values")) != SINDI_OK) return st;
    if ((st = up_or_fail(ix->term_max, term_max.data(), term_max.size() * 4, "term maxima")) != SINDI_OK) return st;
    HIP_TRY(build_deal_chunks(ix->term_goff.as<uint32_t>(), ix->tile_post.as<int64_t>(), n_tiles, nc,
                              (int32_t)vbytes, ix->post_doc.as<uint16_t>(), ix->post_val.p, s));
    HIP_TRY(hipStreamSynchronize(s));
    ix->h_tile_doc = std::move(tile_doc);
    *out = guard.release();
    return SINDI_OK;
}


}  // namespace

// ------------------------------------------------------------------ search
// Tiles per work item when the call leaves it open.  The workgroups resident together sweep
// runs of the same tiles, so the lists of a run's tiles are shared through L2 as long as the
// tiles the workgroups are spread over fit in it; the more list postings a query reads per
// tile, the shorter the run.  That load is taken as the index's kept fraction of the corpus
// entries times the mean query length.  Measured at 8.8M documents (scoring pass per 7,000
// queries): alpha 0.5 and ~35 terms (x = 7.7) fastest at 12 tiles per run (16: 2.9% slower,
// 8: 1.3%); the serving mix of 5 to 200 terms (x = 22) at 8 (12: 13% slower, 16: 29%); alpha
// 0.3 and 0.2 with ~35 terms (x = 3.5 and 1.7) at 32 (24: 0.8% and 1.2% slower, 12: 5.6% and
// 6.9%).
void set_tile_run(Plan &pl, const sindi_index *ix, const sindi_search_params &p, int64_t nq,
                  int64_t nnz)
{
    if (p.tile_run) {
        pl.tile_run = p.tile_run;
        return;
    }
    const double kept = ix->nnz > 0 ? (double)ix->n_post / (double)ix->nnz : 1.0;
    const double x = nq > 0 ? kept * (double)nnz / (double)nq : 0.0;
    pl.tile_run = x > 12.0 ? 8 : (x > 5.0 ? 12 : 32);
}

sindi_status make_plan(const sindi_index *ix, int64_t nq, int32_t k,
                       const sindi_search_params &p, bool rerank, const char *fn, Plan &pl)
{
    (void)nq;
    pl = Plan{};
    pl.rerank = rerank;
    pl.k = k;
    pl.beta = p.beta == 0.0 ? 1.0 : p.beta;
    if (!(pl.beta > 0.0 && pl.beta <= 1.0))
        return fail(SINDI_E_INVALID, "%s: beta must be in (0, 1]", fn);
    if (k < 1 || k > kGammaMax) return fail(SINDI_E_INVALID, "%s: k must be in [1, %d]", fn, kGammaMax);
    pl.gamma = rerank ? (p.gamma ? p.gamma : std::max(k, kDefaultGamma)) : k;
    if (pl.gamma < k || pl.gamma > kGammaMax)
        return fail(SINDI_E_INVALID, "%s: gamma must be in [k, %d]", fn, kGammaMax);
    int b = p.batch ? p.batch : kDefaultBatch;
    if (b != 1 && b != 2 && b != 4 && b != 8)
        return fail(SINDI_E_INVALID, "%s: batch must be 1, 2, 4 or 8", fn);
    while (b > 1 && (int64_t)accumulate_lds_bytes(b, ix->tile_stride) > ix->max_lds) b >>= 1;
    pl.batch = b;
    pl.tile_run = p.tile_run;
    if (p.schedule < 0 || p.schedule > 2)
        return fail(SINDI_E_INVALID, "%s: schedule must be 0, 1 or 2", fn);
    pl.queue = (p.schedule ? p.schedule : kDefaultSchedule) == 2;
    pl.need = (int32_t)std::min<int64_t>(pl.gamma, std::max<int64_t>(ix->n_docs, 1));
    // candidate threshold: sample tiles first, or keep every document
    int64_t cap = p.cand_cap > 0 ? p.cand_cap : kDefaultCandCap;
    cap = std::max<int64_t>(cap, pl.need);
    pl.keep_all = p.sample_tiles < 0 || ix->n_docs <= cap;
    if (pl.keep_all) cap = std::max<int64_t>(ix->n_docs, 1);
    pl.cap = cap;
    pl.n_sample = pl.keep_all ? 0
                              : (int32_t)std::min<int64_t>(
                                    ix->n_tiles, p.sample_tiles ? p.sample_tiles : kDefaultSampleTiles);
    if (!pl.keep_all) {
        int64_t sampled = 0;
        const std::vector<int64_t> &td = ix->h_tile_doc;
        for (int64_t i = 0; i < pl.n_sample; ++i) {
            const int64_t t = i * ix->n_tiles / pl.n_sample;
            sampled += td[t + 1] - td[t];
        }
        const double f = (double)sampled / (double)ix->n_docs;
        pl.rank = std::min<int64_t>((int64_t)pl.n_sample * kAccThreads,
                                    (int64_t)std::ceil(2.0 * pl.need * f) + 8);
    }
    return SINDI_OK;
}

namespace {
inline size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }
}  // namespace

size_t scratch_row_bytes(const Plan &pl, int64_t nq, int64_t nnz)
{
    const size_t e = (size_t)std::max<int64_t>(nnz, 1), q = (size_t)std::max<int64_t>(nq, 1);
    return 2 * align256(e * 4) + align256(pl.beta < 1.0 ? e * 8 : 8) + 5 * align256(q * 4) +
           2 * align256(8);
}

Scratch carve_rows(unsigned char *p, const Plan &pl, int64_t nq, int64_t nnz)
{
    const size_t e = (size_t)std::max<int64_t>(nnz, 1), q = (size_t)std::max<int64_t>(nq, 1);
    Scratch sc;
    auto take = [&](size_t bytes) {
        unsigned char *r = p;
        p += align256(bytes);
        return r;
    };
    sc.ct = reinterpret_cast<int32_t *>(take(e * 4));
    sc.cw = reinterpret_cast<float *>(take(e * 4));
    sc.sabs = reinterpret_cast<double *>(take(pl.beta < 1.0 ? e * 8 : 8));
    sc.cn = reinterpret_cast<int32_t *>(take(q * 4));
    sc.qinv = reinterpret_cast<float *>(take(q * 4));
    sc.status = reinterpret_cast<int32_t *>(take(q * 4));
    sc.rows = reinterpret_cast<int32_t *>(take(q * 4));
    sc.rows2 = reinterpret_cast<int32_t *>(take(q * 4));
    sc.err = reinterpret_cast<int32_t *>(take(8));
    sc.n_rows = reinterpret_cast<uint32_t *>(take(8));
    return sc;
}

PassShape pass_shape(const sindi_index *ix, const Plan &pl, PassKind kind)
{
    PassShape sh;
    if (kind == kPassKeepAll || (kind == kPassSampled && pl.keep_all)) {
        sh.keep_all = true;
        sh.cap = std::max<int64_t>(ix->n_docs, 1);
        return sh;
    }
    sh.cap = pl.cap;
    if (kind == kPassSampled) {
        sh.n_sample = pl.n_sample;
        sh.rank = pl.rank;
    } else {
        sh.n_sample = (int32_t)ix->n_tiles;
        sh.rank = pl.need;
    }
    sh.n_max = (int64_t)sh.n_sample * kAccThreads;
    sh.rank = std::min<int64_t>(sh.rank, sh.n_max);
    return sh;
}

size_t pass_bytes(const PassShape &sh, const Plan &pl, int64_t g)
{
    const size_t n = (size_t)g;
    return 2 * align256(n * 4) + align256(16 + n * 4) + align256(n * (size_t)sh.n_max * 4) +
           align256(n * (size_t)sh.cap * 8) + (pl.rerank ? align256(n * (size_t)pl.need * 8) : 0);
}

int64_t pass_group(const PassShape &sh, const Plan &pl, size_t bytes)
{
    // pass_bytes(g) >= g * per (alignment only adds, at most 255 bytes per array), so
    // bytes / per bounds g from above and few steps down reach the largest fit
    const size_t per = 12 + (size_t)sh.n_max * 4 + (size_t)sh.cap * 8 + (pl.rerank ? (size_t)pl.need * 8 : 0);
    int64_t g = (int64_t)(bytes / per);
    while (g > 0 && pass_bytes(sh, pl, g) > bytes) --g;
    return g;
}

sindi_status enqueue_prep(const sindi_index *ix, const Scratch &sc, const Plan &pl,
                          const DevQueries &dq, hipStream_t s)
{
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(sc.err), 2, 0u, s));
    DevCoarse dc{sc.ct, sc.cw, sc.cn, sc.qinv};
    HIP_TRY(timed(kProfPrep, s, [&] {
        return launch_query_prep(dq, ix->n_cols, pl.beta, dc, ix->term_max.as<float>(), sc.sabs,
                                 sc.err, s);
    }));
    return SINDI_OK;
}

sindi_status enqueue_passes(const sindi_index *ix, const Scratch &sc, const Plan &pl,
                            PassKind kind, const DevQueries &dq, const int32_t *rows, int64_t n,
                            int64_t *out_ids, float *out_scores, hipStream_t s)
{
    if (n <= 0) return SINDI_OK;
    if (ix->n_docs == 0) {  // every query row: k paddings
        if (rows) return fail(SINDI_E_INTERNAL, "search: a retry over an empty index");
        HIP_TRY(launch_fill_f32(out_scores, n * pl.k, -INFINITY, s));
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(out_ids), 2 * n * pl.k, 0xFFFFFFFFu, s));
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(sc.status), n, (uint32_t)kSlotOk, s));
        return SINDI_OK;
    }
    const PassShape sh = pass_shape(ix, pl, kind);
    const int64_t g = std::min<int64_t>(pass_group(sh, pl, sc.arena_bytes), n);
    if (g < 1)
        return fail(SINDI_E_INTERNAL, "search: scratch of %zu bytes holds no query of the pass",
                    sc.arena_bytes);
    unsigned char *p = sc.arena;
    auto take = [&](size_t bytes) {
        unsigned char *r = p;
        p += align256(bytes);
        return r;
    };
    int32_t *slot_q = reinterpret_cast<int32_t *>(take((size_t)g * 4));
    // the work-queue counters of the persistent scoring launches (sample, score), then the
    // per-slot candidate counts: one fill clears both
    unsigned long long *queue = reinterpret_cast<unsigned long long *>(take(16 + (size_t)g * 4));
    uint32_t *count = reinterpret_cast<uint32_t *>(queue + 2);
    float *theta = reinterpret_cast<float *>(take((size_t)g * 4));
    float *maxima = reinterpret_cast<float *>(take((size_t)g * sh.n_max * 4));
    uint64_t *cand = reinterpret_cast<uint64_t *>(take((size_t)g * sh.cap * 8));
    uint64_t *pool = pl.rerank ? reinterpret_cast<uint64_t *>(take((size_t)g * pl.need * 8)) : nullptr;
    const DevIndex dix = ix->dev();
    const DevCoarse dc{sc.ct, sc.cw, sc.cn, sc.qinv};
    // retried rows are few: one query per workgroup
    const int batch = kind == kPassSampled ? pl.batch : 1;
    for (int64_t g0 = 0; g0 < n; g0 += g) {
        const int32_t ns = (int32_t)std::min<int64_t>(g, n - g0);
        const int32_t *sq = rows ? rows + g0 : slot_q;
        if (!rows) HIP_TRY(launch_iota(slot_q, ns, (int32_t)g0, s));
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(queue), 4 + (int64_t)ns, 0u, s));
        if (sh.keep_all) {
            HIP_TRY(launch_fill_f32(theta, ns, -INFINITY, s));
        } else {
            HIP_TRY(timed(kProfSample, s, [&] {
                return launch_accumulate(dix, dq, dc, batch, true, sq, ns, sh.n_sample, maxima,
                                         nullptr, nullptr, nullptr, 0, pl.tile_run, pl.max_qnnz,
                                         pl.queue ? queue : nullptr, s);
            }));
            HIP_TRY(timed(kProfTheta, s, [&] {
                return launch_theta(maxima, sh.n_max, sh.rank, ns, theta, s);
            }));
        }
        HIP_TRY(timed(kProfScore, s, [&] {
            return launch_accumulate(dix, dq, dc, batch, false, sq, ns, 0, nullptr, theta, count,
                                     cand, sh.cap, pl.tile_run, pl.max_qnnz,
                                     pl.queue ? queue + 1 : nullptr, s);
        }));
        // without a threshold no sum is left implicit
        HIP_TRY(timed(kProfFinal, s, [&] {
            return launch_finalize(dix, dq, sq, ns, count, cand, sh.keep_all ? nullptr : theta,
                                   sh.cap, pl.need, pl.k, pl.rerank, pl.max_qnnz, pool, out_ids,
                                   out_scores, sc.status, s);
        }));
    }
    return SINDI_OK;
}

sindi_status enqueue_collect_failed(const Scratch &sc, const int32_t *in_rows, int64_t n,
                                    int32_t *out_rows, uint32_t *count, hipStream_t s)
{
    HIP_TRY(launch_collect_failed(sc.status, in_rows, (int32_t)n, out_rows, count, s));
    return SINDI_OK;
}

sindi_status run_search(const sindi_index *ix, Scratch &sc, const Plan &plan, const DevQueries &dq,
                        bool device_queries, int64_t *out_ids, float *out_scores, hipStream_t s,
                        const char *fn, sindi_status (*grow)(void *, size_t, Scratch &),
                        void *grow_ctx)
{
    Plan pl = plan;
    const int64_t nq = dq.n_rows;
    sindi_status st = enqueue_prep(ix, sc, pl, dq, s);
    if (st != SINDI_OK) return st;
    int32_t e2[2] = {0, 0};
    if (device_queries) {
        // validate before anything reaches the caller's outputs
        HIP_TRY(hipMemcpyAsync(e2, sc.err, 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (e2[0])
            return fail(SINDI_E_INVALID,
                        "%s: malformed query rows (flags 0x%x: 1 row pointers, 2 term id range, "
                        "4 order, 8 non-finite, 16 more than %d entries)",
                        fn, e2[0], kQueryHash / 2);
        pl.max_qnnz = e2[1];
    }
    if ((st = enqueue_passes(ix, sc, pl, kPassSampled, dq, nullptr, nq, out_ids, out_scores, s)) != SINDI_OK)
        return st;
    if ((st = enqueue_collect_failed(sc, nullptr, nq, sc.rows, sc.n_rows, s)) != SINDI_OK) return st;
    uint32_t n_fail = 0;
    HIP_TRY(hipMemcpyAsync(&n_fail, sc.n_rows, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(e2, sc.err, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (e2[0]) return fail(SINDI_E_INTERNAL, "%s: validated host queries flagged 0x%x", fn, e2[0]);
    // rows whose sampled threshold missed: a threshold over every tile, then no threshold
    const PassKind retry[2] = {kPassFullSample, kPassKeepAll};
    int32_t *lists[3] = {sc.rows, sc.rows2, sc.rows};
    for (int r = 0; r < 2 && n_fail > 0; ++r) {
        const size_t need = pass_bytes(pass_shape(ix, pl, retry[r]), pl, 1);
        if (sc.arena_bytes < need) {
            if (!grow) return fail(SINDI_E_INTERNAL, "%s: scratch too small for a retry", fn);
            if ((st = grow(grow_ctx, need, sc)) != SINDI_OK) return st;
        }
        if ((st = enqueue_passes(ix, sc, pl, retry[r], dq, lists[r], n_fail, out_ids, out_scores,
                                 s)) != SINDI_OK)
            return st;
        if ((st = enqueue_collect_failed(sc, lists[r], n_fail, lists[r + 1], sc.n_rows + 1, s)) != SINDI_OK)
            return st;
        HIP_TRY(hipMemcpyAsync(&n_fail, sc.n_rows + 1, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    if (n_fail) return fail(SINDI_E_INTERNAL, "%s: %u queries unresolved", fn, n_fail);
    return SINDI_OK;
}

namespace {

sindi_status grow_workspace(void *ctx, size_t bytes, Scratch &sc)
{
    Workspace &ws = *static_cast<Workspace *>(ctx);
    HIP_TRY(ws.arena.ensure(bytes));
    sc.arena = ws.arena.as<unsigned char>();
    sc.arena_bytes = ws.arena.bytes;
    return SINDI_OK;
}

sindi_status search_impl(sindi_index *ix, const sindi_csr *qc, int32_t k,
                         const sindi_search_params *pp, int64_t *out_ids, float *out_scores,
                         hipStream_t s, bool rerank, const char *fn)
{
    if (!ix || !qc || !out_ids || !out_scores) return fail(SINDI_E_INVALID, "%s: null argument", fn);
    sindi_search_params p{};
    if (pp) p = *pp;
    if (qc->n_cols != ix->n_cols)
        return fail(SINDI_E_INVALID, "%s: queries have %lld columns, index has %lld", fn,
                    (long long)qc->n_cols, (long long)ix->n_cols);
    if (qc->n_rows < 0 || qc->nnz < 0) return fail(SINDI_E_INVALID, "%s: bad query shape", fn);
    const int64_t nq = qc->n_rows;
    if (nq > INT32_MAX / 2) return fail(SINDI_E_INVALID, "%s: too many queries", fn);
    Plan pl;
    sindi_status st = make_plan(ix, nq, k, p, rerank, fn, pl);
    if (st != SINDI_OK) return st;
    if (nq == 0) return SINDI_OK;
    set_tile_run(pl, ix, p, nq, qc->nnz);
    if (qc->on_device && (!qc->indptr || (qc->nnz > 0 && (!qc->indices || !qc->values))))
        return fail(SINDI_E_INVALID, "%s: null query array", fn);
    int64_t longest = 0;
    if (!qc->on_device &&
        (st = validate_host_csr(qc, "queries", kQueryHash / 2, &longest)) != SINDI_OK)
        return st;
    pl.max_qnnz = (int32_t)longest;
    std::lock_guard<std::mutex> lock(ix->mu);
    Workspace &ws = ix->ws;
    HIP_TRY(ws.row_part.ensure(scratch_row_bytes(pl, nq, qc->nnz)));
    Scratch sc = carve_rows(ws.row_part.as<unsigned char>(), pl, nq, qc->nnz);
    // the sampled pass in groups whose candidate buffers fit kCandBudget
    const PassShape sh = pass_shape(ix, pl, kPassSampled);
    const int64_t g = std::max<int64_t>(1, std::min<int64_t>(nq, pass_group(sh, pl, kCandBudget)));
    HIP_TRY(ws.arena.ensure(pass_bytes(sh, pl, g)));
    sc.arena = ws.arena.as<unsigned char>();
    sc.arena_bytes = ws.arena.bytes;

    DevQueries dq{nq, qc->nnz, qc->indptr, qc->indices, qc->values};
    if (!qc->on_device) {
        HIP_TRY(ws.q_ptr.ensure((size_t)(nq + 1) * 8));
        HIP_TRY(ws.q_idx.ensure((size_t)qc->nnz * 4 + 4));
        HIP_TRY(ws.q_val.ensure((size_t)qc->nnz * 4 + 4));
        HIP_TRY(hipMemcpyAsync(ws.q_ptr.p, qc->indptr, (size_t)(nq + 1) * 8, hipMemcpyHostToDevice, s));
        if (qc->nnz) {
            HIP_TRY(hipMemcpyAsync(ws.q_idx.p, qc->indices, (size_t)qc->nnz * 4, hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync(ws.q_val.p, qc->values, (size_t)qc->nnz * 4, hipMemcpyHostToDevice, s));
        }
        dq.indptr = ws.q_ptr.as<int64_t>();
        dq.indices = ws.q_idx.as<int32_t>();
        dq.values = ws.q_val.as<float>();
    }
    return run_search(ix, sc, pl, dq, qc->on_device != 0, out_ids, out_scores, s, fn,
                      grow_workspace, &ws);
}

sindi_status check_dev_queries(sindi_index *ix, const sindi_csr *qc, const char *fn, hipStream_t s)
{
    if (!qc->on_device) return fail(SINDI_E_INVALID, "%s: queries must be device memory", fn);
    if (qc->n_cols != ix->n_cols) return fail(SINDI_E_INVALID, "%s: column count mismatch", fn);
    if (qc->n_rows < 0 || qc->nnz < 0) return fail(SINDI_E_INVALID, "%s: bad query shape", fn);
    if (qc->n_rows == 0) return SINDI_OK;
    if (!qc->indptr || (qc->nnz > 0 && (!qc->indices || !qc->values)))
        return fail(SINDI_E_INVALID, "%s: null query array", fn);
    Workspace &ws = ix->ws;
    Plan pl;  // beta 1: no FP64 scratch
    HIP_TRY(ws.row_part.ensure(scratch_row_bytes(pl, qc->n_rows, qc->nnz)));
    const Scratch sc = carve_rows(ws.row_part.as<unsigned char>(), pl, qc->n_rows, qc->nnz);
    DevQueries dq{qc->n_rows, qc->nnz, qc->indptr, qc->indices, qc->values};
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(sc.err), 2, 0u, s));
    DevCoarse dc{sc.ct, sc.cw, sc.cn, sc.qinv};
    HIP_TRY(launch_query_prep(dq, ix->n_cols, 1.0, dc, ix->term_max.as<float>(), nullptr, sc.err, s));
    int32_t qerr = 0;
    HIP_TRY(hipMemcpyAsync(&qerr, sc.err, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (qerr) return fail(SINDI_E_INVALID, "%s: malformed query rows (flags 0x%x)", fn, qerr);
    return SINDI_OK;
}

}  // namespace
}  // namespace sindi

sindi::DevIndex sindi_index::dev() const
{
    sindi::DevIndex d;
    d.n_docs = n_docs;
    d.n_cols = n_cols;
    d.n_tiles = n_tiles;
    d.tile_stride = tile_stride;
    d.value_dtype = dtype;
    d.tile_doc = tile_doc.as<int64_t>();
    d.tile_post = tile_post.as<int64_t>();
    d.term_goff = term_goff.as<uint32_t>();
    d.post_doc = post_doc.as<uint16_t>();
    d.post_val = post_val.p;
    d.term_max = term_max.as<float>();
    d.indptr = indptr.as<int64_t>();
    d.indices = indices.as<int32_t>();
    d.values = values.as<float>();
    d.nnz = nnz;
    return d;
}

int64_t sindi_index::device_bytes() const
{
    return (int64_t)(indptr.bytes + indices.bytes + values.bytes + tile_doc.bytes +
                     tile_post.bytes + term_goff.bytes + post_doc.bytes + post_val.bytes +
                     term_max.bytes);
}

using namespace sindi;

// ------------------------------------------------------------------ C ABI
extern "C" {

sindi_status sindi_build(const sindi_csr *corpus, const sindi_build_params *params, void *stream,
                         sindi_index **out)
{
    try {
        return build_impl(corpus, params, (hipStream_t)stream, out);
    } catch (const std::bad_alloc &) {
        return fail(SINDI_E_OOM, "sindi_build: host allocation failed");
    } catch (...) {
        return fail(SINDI_E_INTERNAL, "sindi_build: unexpected exception");
    }
}

void sindi_index_free(sindi_index *idx) { delete idx; }

sindi_status sindi_index_get_info(const sindi_index *ix, sindi_index_info *o)
{
    if (!ix || !o) return fail(SINDI_E_INVALID, "sindi_index_get_info: null argument");
    o->n_docs = ix->n_docs;
    o->n_cols = ix->n_cols;
    o->nnz = ix->nnz;
    o->n_postings = ix->n_post;
    o->n_slots = ix->n_slots;
    o->prune = ix->prune;
    o->vn = ix->vn;
    o->list_len = ix->list_len;
    o->window = ix->window;
    o->n_windows = ix->n_windows;
    o->n_tiles = ix->n_tiles;
    o->tile_max = ix->tile_max;
    o->value_dtype = ix->dtype;
    o->alpha = ix->alpha;
    o->device_bytes = ix->device_bytes();
    return SINDI_OK;
}

sindi_status sindi_index_export(const sindi_index *ix, int64_t *tile_doc, int64_t *tile_post,
                                uint32_t *term_goff, uint16_t *post_doc, void *post_val)
{
    if (!ix) return fail(SINDI_E_INVALID, "sindi_index_export: null index");
    const size_t vb = ix->dtype == SINDI_F32 ? 4 : 2;
    if (tile_doc) HIP_TRY(hipMemcpy(tile_doc, ix->tile_doc.p, (size_t)(ix->n_tiles + 1) * 8, hipMemcpyDeviceToHost));
    if (tile_post) HIP_TRY(hipMemcpy(tile_post, ix->tile_post.p, (size_t)(ix->n_tiles + 1) * 8, hipMemcpyDeviceToHost));
    if (term_goff) HIP_TRY(hipMemcpy(term_goff, ix->term_goff.p, (size_t)ix->n_tiles * (ix->n_cols + 1) * 4, hipMemcpyDeviceToHost));
    if (post_doc && ix->n_slots) HIP_TRY(hipMemcpy(post_doc, ix->post_doc.p, (size_t)ix->n_slots * 2, hipMemcpyDeviceToHost));
    if (post_val && ix->n_slots) HIP_TRY(hipMemcpy(post_val, ix->post_val.p, (size_t)ix->n_slots * vb, hipMemcpyDeviceToHost));
    return SINDI_OK;
}

sindi_status sindi_search(const sindi_index *idx, const sindi_csr *queries, int32_t k,
                          const sindi_search_params *params, int64_t *out_ids, float *out_scores,
                          void *stream)
{
    try {
        return search_impl(const_cast<sindi_index *>(idx), queries, k, params, out_ids, out_scores,
                           (hipStream_t)stream, true, "sindi_search");
    } catch (const std::bad_alloc &) {
        return fail(SINDI_E_OOM, "sindi_search: host allocation failed");
    } catch (...) {
        return fail(SINDI_E_INTERNAL, "sindi_search: unexpected exception");
    }
}

sindi_status sindi_search_coarse(const sindi_index *idx, const sindi_csr *queries, int32_t k,
                                 const sindi_search_params *params, int64_t *out_ids,
                                 float *out_scores, void *stream)
{
    try {
        return search_impl(const_cast<sindi_index *>(idx), queries, k, params, out_ids, out_scores,
                           (hipStream_t)stream, false, "sindi_search_coarse");
    } catch (const std::bad_alloc &) {
        return fail(SINDI_E_OOM, "sindi_search_coarse: host allocation failed");
    } catch (...) {
        return fail(SINDI_E_INTERNAL, "sindi_search_coarse: unexpected exception");
    }
}

sindi_status sindi_score_forward(const sindi_index *idx, const sindi_csr *queries,
                                 const int64_t *cand_ids, int32_t n_cand,
                                 const float *doc_values, float *out_scores, void *stream)
{
    if (!idx || !queries || (!cand_ids && n_cand) || (!out_scores && n_cand) || n_cand < 0)
        return fail(SINDI_E_INVALID, "sindi_score_forward: bad argument");
    sindi_index *ix = const_cast<sindi_index *>(idx);
    std::lock_guard<std::mutex> lock(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    sindi_status st = check_dev_queries(ix, queries, "sindi_score_forward", s);
    if (st != SINDI_OK) return st;
    DevQueries dq{queries->n_rows, queries->nnz, queries->indptr, queries->indices, queries->values};
    DevIndex dix = ix->dev();
    if (doc_values) dix.values = doc_values;
    HIP_TRY(launch_score_forward(dix, dq, cand_ids, n_cand, out_scores, s));
    return SINDI_OK;
}

sindi_status sindi_score_backward(const sindi_index *idx, const sindi_csr *queries,
                                  const int64_t *cand_ids, int32_t n_cand,
                                  const float *doc_values, const float *grad_scores,
                                  float *grad_query_values, float *grad_doc_values,
                                  void *stream)
{
    if (!idx || !queries || (!cand_ids && n_cand) || (!grad_scores && n_cand) || n_cand < 0)
        return fail(SINDI_E_INVALID, "sindi_score_backward: bad argument");
    sindi_index *ix = const_cast<sindi_index *>(idx);
    std::lock_guard<std::mutex> lock(ix->mu);
    hipStream_t s = (hipStream_t)stream;
    sindi_status st = check_dev_queries(ix, queries, "sindi_score_backward", s);
    if (st != SINDI_OK) return st;
    DevQueries dq{queries->n_rows, queries->nnz, queries->indptr, queries->indices, queries->values};
    DevIndex dix = ix->dev();
    if (doc_values) dix.values = doc_values;
    HIP_TRY(launch_score_backward(dix, dq, cand_ids, n_cand, grad_scores, grad_query_values,
                                  grad_doc_values, s));
    return SINDI_OK;
}

sindi_status sindi_profile_enable(int32_t enable) { return profile_enable(enable); }

sindi_status sindi_profile_read(sindi_profile *out, int32_t reset) { return profile_read(out, reset); }

const char *sindi_last_error(void) { return last_error(); }

const char *sindi_version(void) { return "sindi-mi355x 0.2 (gfx950)"; }

}  // extern "C"
