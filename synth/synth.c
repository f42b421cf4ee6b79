/*
 * synth.c -- seeded synthetic sparse vectors for the SINDI workloads.
 *
 * Input generation only.  Nothing here scores, prunes, indexes or ranks: it
 * draws CSR rows of (term id, value) pairs whose shape follows the sparse
 * vector model of the paper (Def. 1: a vector is the set of its non-zero
 * entries) and the dataset statistics of its Table "datasets" (rows of a
 * SPLADE-like vocabulary, ~120 non-zeros per document, ~30-50 per query).
 * Both the CPU oracle and the GPU library consume these rows; neither shares
 * any other code.
 *
 * Randomness is counter based: every (seed, stream, row) triple keys its own
 * SplitMix64 sequence (Steele, Lea & Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014), so any row can be regenerated alone and
 * rows are generated in parallel with identical results for any thread count.
 *
 * Distributions
 *   row length : Poisson(mean) by sequential inversion, or uniform integer
 *                in [lo, hi]; then clipped to [nnz_min, nnz_max] and to vocab
 *   term ids   : Zipf(s) over ranks 1..vocab (rank r -> id r-1) or uniform,
 *                drawn without replacement by successive sampling (i.i.d.
 *                draws, repeats discarded)
 *   values     : lognormal(mu, sigma) via Box-Muller in double, or
 *                uniform(a, b); rounded to float32 (round-to-nearest-even)
 *   each row is emitted sorted by ascending term id.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int64_t vocab;
    int32_t term_dist; /* 0 = Zipf(zipf_s) by rank, 1 = uniform            */
    int32_t nnz_dist;  /* 0 = Poisson(nnz_a), 1 = uniform int [nnz_a,nnz_b] */
    double zipf_s;
    double nnz_a, nnz_b;
    int64_t nnz_min, nnz_max;
    int32_t val_dist;  /* 0 = lognormal(val_a=mu, val_b=sigma), 1 = U(a,b) */
    int32_t pad_;
    double val_a, val_b;
} synth_cfg;

/* ---- SplitMix64 ------------------------------------------------------- */
static inline uint64_t sm_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static inline uint64_t sm_next(uint64_t *s)
{
    *s += 0x9E3779B97F4A7C15ULL;
    return sm_mix(*s);
}
static inline uint64_t key3(uint64_t seed, uint64_t stream, uint64_t ctr)
{
    uint64_t k = sm_mix(seed + 0x9E3779B97F4A7C15ULL);
    k = sm_mix(k ^ (stream * 0xD1B54A32D192ED03ULL + 0x8CB92BA72F3D8DD7ULL));
    return sm_mix(k + ctr * 0x9E3779B97F4A7C15ULL);
}
/* uniform double in the open interval (0, 1) */
static inline double u01(uint64_t *s)
{
    return ((double)(sm_next(s) >> 11) + 0.5) * 0x1.0p-53;
}
static inline double std_normal(uint64_t *s)
{
    double u1 = u01(s), u2 = u01(s);
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
}

static int64_t draw_len(uint64_t *s, const synth_cfg *c)
{
    int64_t n;
    if (c->nnz_dist == 0) {
        double lam = c->nnz_a;
        if (lam <= 0) {
            n = 0;
        } else if (lam > 600.0) { /* exp(-lam) would underflow */
            n = (int64_t)llround(lam + sqrt(lam) * std_normal(s));
        } else {
            double u = u01(s), p = exp(-lam), F = p;
            int64_t k = 0, kmax = (int64_t)(lam * 20.0) + 1000;
            while (u > F && k < kmax) {
                k++;
                p *= lam / (double)k;
                F += p;
            }
            n = k;
        }
    } else {
        int64_t lo = (int64_t)c->nnz_a, hi = (int64_t)c->nnz_b;
        n = lo + (int64_t)(u01(s) * (double)(hi - lo + 1));
        if (n > hi) n = hi;
    }
    if (n < c->nnz_min) n = c->nnz_min;
    if (n > c->nnz_max) n = c->nnz_max;
    if (n > c->vocab) n = c->vocab;
    if (n < 0) n = 0;
    return n;
}

typedef struct {
    int32_t id;
    float v;
} pair_t;
static int cmp_pair(const void *a, const void *b)
{
    int32_t x = ((const pair_t *)a)->id, y = ((const pair_t *)b)->id;
    return (x > y) - (x < y);
}

static double *zipf_cdf(const synth_cfg *c)
{
    if (c->term_dist != 0) return NULL;
    double *cdf = (double *)malloc(sizeof(double) * (size_t)c->vocab);
    double acc = 0.0;
    for (int64_t r = 0; r < c->vocab; ++r) {
        acc += pow((double)(r + 1), -c->zipf_s);
        cdf[r] = acc;
    }
    for (int64_t r = 0; r < c->vocab; ++r) cdf[r] /= acc;
    cdf[c->vocab - 1] = 1.0;
    return cdf;
}

static inline int64_t draw_term(uint64_t *s, const synth_cfg *c, const double *cdf)
{
    double u = u01(s);
    if (!cdf) {
        int64_t t = (int64_t)(u * (double)c->vocab);
        return t >= c->vocab ? c->vocab - 1 : t;
    }
    int64_t lo = 0, hi = c->vocab - 1; /* first r with cdf[r] >= u */
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (cdf[mid] >= u) hi = mid; else lo = mid + 1;
    }
    return lo;
}

static inline float draw_value(uint64_t *s, const synth_cfg *c)
{
    if (c->val_dist == 0) return (float)exp(c->val_a + c->val_b * std_normal(s));
    return (float)(c->val_a + (c->val_b - c->val_a) * u01(s));
}

/* Pass 1: row lengths -> indptr[0..n_rows] (indptr[0] = 0). */
void synth_indptr(const synth_cfg *c, int64_t n_rows, uint64_t seed, uint64_t stream,
                  int64_t row0, int64_t *indptr)
{
    indptr[0] = 0;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n_rows; ++r) {
        uint64_t s = key3(seed, stream, (uint64_t)(row0 + r));
        indptr[r + 1] = draw_len(&s, c);
    }
    for (int64_t r = 0; r < n_rows; ++r) indptr[r + 1] += indptr[r];
}

/* Pass 2: fill every row; regenerates the row length from the same key. */
void synth_fill(const synth_cfg *c, int64_t n_rows, uint64_t seed, uint64_t stream,
                int64_t row0, const int64_t *indptr, int32_t *indices, float *values)
{
    double *cdf = zipf_cdf(c);
#pragma omp parallel
    {
        uint32_t *mark = (uint32_t *)calloc((size_t)c->vocab, sizeof(uint32_t));
        pair_t *buf = (pair_t *)malloc(sizeof(pair_t) * (size_t)(c->nnz_max > 0 ? c->nnz_max : 1));
        uint32_t stamp = 0;
#pragma omp for schedule(dynamic, 1024)
        for (int64_t r = 0; r < n_rows; ++r) {
            uint64_t s = key3(seed, stream, (uint64_t)(row0 + r));
            int64_t n = draw_len(&s, c);
            if (++stamp == 0) { /* stamp wrapped: clear marks */
                memset(mark, 0, sizeof(uint32_t) * (size_t)c->vocab);
                stamp = 1;
            }
            int64_t got = 0;
            while (got < n) {
                int64_t t = draw_term(&s, c, cdf);
                if (mark[t] == stamp) continue;
                mark[t] = stamp;
                buf[got].id = (int32_t)t;
                buf[got].v = draw_value(&s, c);
                ++got;
            }
            qsort(buf, (size_t)n, sizeof(pair_t), cmp_pair);
            int64_t o = indptr[r];
            for (int64_t i = 0; i < n; ++i) {
                indices[o + i] = buf[i].id;
                values[o + i] = buf[i].v;
            }
        }
        free(mark);
        free(buf);
    }
    free(cdf);
}

/* Counter-based streams of plain draws, element i keyed by (seed, stream, i0+i). */
void synth_uniform_u64(uint64_t seed, uint64_t stream, int64_t i0, int64_t n, uint64_t *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        uint64_t s = key3(seed, stream, (uint64_t)(i0 + i));
        out[i] = sm_next(&s);
    }
}
void synth_lognormal_f32(uint64_t seed, uint64_t stream, int64_t i0, int64_t n, double mu,
                         double sigma, float *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        uint64_t s = key3(seed, stream, (uint64_t)(i0 + i));
        out[i] = (float)exp(mu + sigma * std_normal(&s));
    }
}
void synth_exponential_f64(uint64_t seed, uint64_t stream, int64_t i0, int64_t n, double mean,
                           double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        uint64_t s = key3(seed, stream, (uint64_t)(i0 + i));
        out[i] = -mean * log(u01(&s));
    }
}
