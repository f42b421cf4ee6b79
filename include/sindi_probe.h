/*
 * sindi_probe.h -- microbenchmark of the gfx950 unit that bounds the scoring
 * pass of the SINDI search library: workgroup-local (LDS) atomic adds, the
 * "accumulate into the window's distance array" step of Alg. 2 (Sec. 3.2)
 * that Sec. 3.3.1 names as the memory-bound part of the method.
 *
 * Measurement only: libsindi_probe.so is not part of the search path and
 * the search library does not load it.  bench.py reports its rates beside
 * the scoring pass's own rate of posting adds, so the LDS ceiling that binds
 * the scoring kernel is reproducible from the repository.
 */
#ifndef SINDI_PROBE_H
#define SINDI_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#pragma GCC visibility push(default)

/*
 * Time one launch of n_workgroups workgroups of 512 threads, each holding a
 * 48 KB LDS array (three workgroups share a compute unit, as the scoring
 * kernel's do), in which every thread performs iters x 8 atomic adds of 1.
 *   op      0: 32-bit integer add (ds_add_u32); 1: FP32 add (ds_add_f32)
 *   stride  the words between the addresses of consecutive lanes of one
 *           instruction (1: 64 consecutive words, no bank shared by two
 *           lanes; 2, 4, ...: lanes share banks as the bank count allows);
 *           0: every lane a pseudo-random word (a fixed hash of workgroup,
 *           thread and slot), as the scatter of postings into a score tile
 *   stream  hipStream_t as void* (NULL: default stream); the call waits for
 *           the launch
 * Outputs: *ms the launch's duration by HIP events, *updates the atomic adds
 * performed (n_workgroups * 512 * iters * 8).  Every address stays inside
 * the workgroup's LDS array (a power-of-two word mask).
 * Returns 0, or a hipError_t code (invalid arguments: hipErrorInvalidValue).
 */
int sindi_probe_lds_add(int32_t op, int32_t stride, int32_t n_workgroups, int32_t iters,
                        void *stream, double *ms, double *updates);

#pragma GCC visibility pop

#ifdef __cplusplus
}
#endif
#endif /* SINDI_PROBE_H */
