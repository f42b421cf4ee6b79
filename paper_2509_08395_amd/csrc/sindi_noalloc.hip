// sindi_search_noalloc: the search of sindi_search (Alg. 4) with every piece
// of device scratch taken from one statically sized array of the library, so
// that a call allocates no device memory.  The kernels and the pipeline are
// sindi_search's; only where the scratch lives differs.
#include <hip/hip_runtime.h>

#include <mutex>

#include "sindi.h"
#include "sindi_internal.h"
#include "sindi_state.h"

namespace sindi {
namespace {

// 256 MiB per device: the per-query rows of the call (coarse terms and
// weights, status, failed-row lists) first, the rest a pass arena.
constexpr size_t kScratchBytes = size_t(256) << 20;
constexpr int kMaxDevices = 64;

// In host code this name is a host-side stand-in; kernels take the device
// address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceScratch {
    std::mutex mu;                 // one call at a time per device
    unsigned char *ptr = nullptr;  // scratch's address on the device, once looked up
};
DeviceScratch g_dev[kMaxDevices];

// The device address of `scratch` on device dev (current), looked up once.
sindi_status scratch_address(int dev, unsigned char **out)
{
    DeviceScratch &d = g_dev[dev];
    if (!d.ptr) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SINDI_E_HIP, "sindi_search_noalloc: hipGetSymbolAddress: %s",
                        hipGetErrorString(e));
        d.ptr = static_cast<unsigned char *>(p);
    }
    *out = d.ptr;
    return SINDI_OK;
}

sindi_status noalloc_impl(const sindi_index *ix, const sindi_csr *qc, int32_t k,
                          const sindi_search_params *pp, int64_t *out_ids, float *out_scores,
                          hipStream_t s)
{
    const char *fn = "sindi_search_noalloc";
    if (!ix || !qc || !out_ids || !out_scores) return fail(SINDI_E_INVALID, "%s: null argument", fn);
    if (!qc->on_device) return fail(SINDI_E_INVALID, "%s: queries must be device memory", fn);
    if (qc->n_cols != ix->n_cols)
        return fail(SINDI_E_INVALID, "%s: queries have %lld columns, index has %lld", fn,
                    (long long)qc->n_cols, (long long)ix->n_cols);
    if (qc->n_rows < 0 || qc->nnz < 0 || qc->n_rows > INT32_MAX / 2)
        return fail(SINDI_E_INVALID, "%s: bad query shape", fn);
    if (!qc->indptr || (qc->nnz > 0 && (!qc->indices || !qc->values)))
        return fail(SINDI_E_INVALID, "%s: null query array", fn);
    sindi_search_params p{};
    if (pp) p = *pp;
    Plan pl;
    sindi_status st = make_plan(ix, qc->n_rows, k, p, true, fn, pl);
    if (st != SINDI_OK) return st;
    if (qc->n_rows == 0) return SINDI_OK;
    set_tile_run(pl, ix, p, qc->n_rows, qc->nnz);
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != ix->device)
        return fail(SINDI_E_INVALID, "%s: the index lives on device %d, device %d is current", fn,
                    ix->device, dev);
    if (dev < 0 || dev >= kMaxDevices) return fail(SINDI_E_INVALID, "%s: device %d", fn, dev);
    // sizes: the rows of the call, then at least one query of every pass a retry may need
    const size_t rows = scratch_row_bytes(pl, qc->n_rows, qc->nnz);
    const size_t one = std::max({pass_bytes(pass_shape(ix, pl, kPassSampled), pl, 1),
                                 pass_bytes(pass_shape(ix, pl, kPassFullSample), pl, 1),
                                 pass_bytes(pass_shape(ix, pl, kPassKeepAll), pl, 1)});
    if (rows > kScratchBytes || kScratchBytes - rows < one)
        return fail(SINDI_E_INVALID,
                    "%s: %lld queries of %lld entries over %lld documents need %zu + %zu bytes of "
                    "scratch; the library holds %zu (use sindi_search)",
                    fn, (long long)qc->n_rows, (long long)qc->nnz, (long long)ix->n_docs, rows, one,
                    kScratchBytes);
    std::lock_guard<std::mutex> lock(g_dev[dev].mu);
    unsigned char *base = nullptr;
    if ((st = scratch_address(dev, &base)) != SINDI_OK) return st;
    Scratch sc = carve_rows(base, pl, qc->n_rows, qc->nnz);
    sc.arena = base + rows;
    sc.arena_bytes = kScratchBytes - rows;
    const DevQueries dq{qc->n_rows, qc->nnz, qc->indptr, qc->indices, qc->values};
    return run_search(ix, sc, pl, dq, true, out_ids, out_scores, s, fn, nullptr, nullptr);
}

}  // namespace
}  // namespace sindi

extern "C" sindi_status sindi_search_noalloc(const sindi_index *idx, const sindi_csr *queries,
                                             int32_t k, const sindi_search_params *params,
                                             int64_t *out_ids, float *out_scores, void *stream)
{
    try {
        return sindi::noalloc_impl(idx, queries, k, params, out_ids, out_scores, (hipStream_t)stream);
    } catch (...) {
        return sindi::fail(SINDI_E_INTERNAL, "sindi_search_noalloc: unexpected exception");
    }
}
