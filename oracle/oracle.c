/*
 * oracle.c -- plain, slow, obviously correct CPU reference for the SINDI
 * search path (arXiv 2509.08395).  TEST INFRASTRUCTURE ONLY: it is called by
 * the test suite, by the smoke check and by the benchmark's CPU-baseline leg,
 * never by the library.  It shares no code with the GPU library.
 *
 * Arithmetic is FP64 throughout.  Inputs are FP32 values; a product of two
 * FP32 numbers is exact in FP64 (24 + 24 <= 53 significand bits), so the only
 * roundings are in the additions, which run in ascending term order.
 *
 * Ranking order everywhere: score descending, then document id ascending
 * (the ties reading of the strict ">" heap test of Alg. 2).
 *
 * Functions and the passages they follow:
 *   or_exact_topk      Defs. 2-3 (inner product over common dimensions,
 *                      Sparse-MIPS), generalised to top-k as in the Recall
 *                      definition of Sec. 5.1
 *   or_pair_scores     Def. 2, one (query, document) pair at a time
 *   or_mass_prune      Defs. 5-6 (mass of a vector, alpha-mass subvector)
 *   or_vnp_prune       Vector Number Pruning (Sec. 4.1): vn largest |x| per row
 *   or_lp_prune        List Pruning (Sec. 4.1): l' largest |x| per term list
 *   or_build_index     Alg. 1 (PreciseSindiConstruction) with the window
 *                      partition of Sec. 3.3.1
 *   or_precise_search  Alg. 2 (PreciseSindiSearch)
 *   or_approx_search   Alg. 4 (ApproximateSindiSearch): query beta-mass,
 *                      coarse top-gamma by Alg. 2, exact rerank, top-k
 *   or_score_grad      gradient of the scores delta(q_b, x_c) (Def. 2) with
 *                      respect to query and document values (bilinear form)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* a is ranked before b: higher score, or equal score and lower id */
static int ranks_before(double sa, int64_t ia, double sb, int64_t ib)
{
    return sa > sb || (sa == sb && ia < ib);
}

/* ---------------------------------------------------------------------- */
/* Bounded ranked list: the first `cap` items under the ranking order,     */
/* kept sorted; insertion by shifting (cap is small).                      */
typedef struct {
    int64_t cap, len;
    double *s;
    int64_t *id;
} ranked_t;

static void rl_init(ranked_t *r, int64_t cap)
{
    r->cap = cap;
    r->len = 0;
    r->s = (double *)malloc(sizeof(double) * (size_t)(cap > 0 ? cap : 1));
    r->id = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cap > 0 ? cap : 1));
}
static void rl_free(ranked_t *r)
{
    free(r->s);
    free(r->id);
}
static void rl_offer(ranked_t *r, double s, int64_t id)
{
    if (r->cap <= 0) return;
    if (r->len == r->cap && !ranks_before(s, id, r->s[r->len - 1], r->id[r->len - 1])) return;
    int64_t p = r->len < r->cap ? r->len : r->cap - 1;
    while (p > 0 && ranks_before(s, id, r->s[p - 1], r->id[p - 1])) {
        r->s[p] = r->s[p - 1];
        r->id[p] = r->id[p - 1];
        --p;
    }
    r->s[p] = s;
    r->id[p] = id;
    if (r->len < r->cap) r->len++;
}
static void rl_write(const ranked_t *r, int64_t k, int64_t *ids, double *scores)
{
    for (int64_t t = 0; t < k; ++t) {
        if (t < r->len) {
            ids[t] = r->id[t];
            scores[t] = r->s[t];
        } else {
            ids[t] = -1;
            scores[t] = -INFINITY;
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Column-major copy (documents ascending inside every column).            */
typedef struct {
    int64_t *ptr; /* [n_cols + 1] */
    int64_t *doc;
    float *val;
} csc_t;

static void csc_build(int64_t nd, int64_t ncols, const int64_t *ptr, const int32_t *idx,
                      const float *val, csc_t *c)
{
    int64_t nnz = ptr[nd];
    c->ptr = (int64_t *)calloc((size_t)ncols + 1, sizeof(int64_t));
    c->doc = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
    c->val = (float *)malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
    for (int64_t e = 0; e < nnz; ++e) c->ptr[idx[e] + 1]++;
    for (int64_t j = 0; j < ncols; ++j) c->ptr[j + 1] += c->ptr[j];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncols > 0 ? ncols : 1));
    memcpy(fill, c->ptr, sizeof(int64_t) * (size_t)ncols);
    for (int64_t i = 0; i < nd; ++i)
        for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
            int64_t p = fill[idx[e]]++;
            c->doc[p] = i;
            c->val[p] = val[e];
        }
    free(fill);
}
static void csc_free(csc_t *c)
{
    free(c->ptr);
    free(c->doc);
    free(c->val);
}

/* Def. 2 for one pair: sum over common dimensions, ascending term order. */
static double dot_rows(const int32_t *ia, const float *va, int64_t na, const int32_t *ib,
                       const float *vb, int64_t nb)
{
    double s = 0.0;
    int64_t a = 0, b = 0;
    while (a < na && b < nb) {
        if (ia[a] < ib[b]) {
            ++a;
        } else if (ia[a] > ib[b]) {
            ++b;
        } else {
            s += (double)va[a] * (double)vb[b];
            ++a;
            ++b;
        }
    }
    return s;
}

/* ---------------------------------------------------------------------- */
/* Exact top-k: every document's delta(x_i, q) into a dense FP64 array,     */
/* term at a time over the query's terms (ascending), then the first k     */
/* documents under the ranking order.  Untouched documents score 0.        */
void or_exact_topk(int64_t nd, int64_t ncols, const int64_t *dptr, const int32_t *didx,
                   const float *dval, int64_t nq, const int64_t *qptr, const int32_t *qidx,
                   const float *qval, int64_t k, int64_t *out_ids, double *out_scores,
                   int n_threads)
{
    csc_t c;
    csc_build(nd, ncols, dptr, didx, dval, &c);
#pragma omp parallel num_threads(n_threads > 0 ? n_threads : 1)
    {
        double *acc = (double *)malloc(sizeof(double) * (size_t)(nd > 0 ? nd : 1));
        ranked_t r;
        rl_init(&r, k < nd ? k : nd);
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < nq; ++q) {
            memset(acc, 0, sizeof(double) * (size_t)nd);
            for (int64_t e = qptr[q]; e < qptr[q + 1]; ++e) {
                int64_t j = qidx[e];
                double w = (double)qval[e];
                for (int64_t p = c.ptr[j]; p < c.ptr[j + 1]; ++p) acc[c.doc[p]] += w * (double)c.val[p];
            }
            r.len = 0;
            for (int64_t i = 0; i < nd; ++i) rl_offer(&r, acc[i], i);
            rl_write(&r, k, out_ids + q * k, out_scores + q * k);
        }
        rl_free(&r);
        free(acc);
    }
    csc_free(&c);
}

/* Def. 2 for listed (query, document) pairs. */
void or_pair_scores(const int64_t *dptr, const int32_t *didx, const float *dval,
                    const int64_t *qptr, const int32_t *qidx, const float *qval, int64_t n_pairs,
                    const int64_t *pair_q, const int64_t *pair_d, double *out)
{
    for (int64_t t = 0; t < n_pairs; ++t) {
        int64_t q = pair_q[t], d = pair_d[t];
        if (d < 0) {
            out[t] = -INFINITY;
            continue;
        }
        out[t] = dot_rows(qidx + qptr[q], qval + qptr[q], qptr[q + 1] - qptr[q], didx + dptr[d],
                          dval + dptr[d], dptr[d + 1] - dptr[d]);
    }
}

/* ---------------------------------------------------------------------- */
/* alpha-mass subvector (Defs. 5-6).  pi orders a row's entries by          */
/* non-increasing |x| (ties: lower term id first); mass is the sum of |x|   */
/* taken in that order; r is the smallest prefix length whose sum reaches   */
/* alpha * mass; the first r entries of pi are kept.  A stored value of 0   */
/* is no entry (Def. 1: a vector is the set of its non-zero entries), so it */
/* is never kept, and a row of zeros keeps nothing.                         */
typedef struct {
    double a;
    int32_t id;
    int64_t pos;
} mag_t;
static int cmp_mag(const void *x, const void *y)
{
    const mag_t *p = (const mag_t *)x, *q = (const mag_t *)y;
    if (p->a > q->a) return -1;
    if (p->a < q->a) return 1;
    return (p->id > q->id) - (p->id < q->id);
}

static int64_t mass_prune_row(const int32_t *idx, const float *val, int64_t n_stored,
                              double alpha, mag_t *tmp, uint8_t *keep)
{
    int64_t n = 0;
    for (int64_t i = 0; i < n_stored; ++i) {
        keep[i] = 0;
        if (val[i] == 0.0f) continue;  /* not an entry of the vector (Def. 1) */
        tmp[n].a = fabs((double)val[i]);
        tmp[n].id = idx[i];
        tmp[n].pos = i;
        ++n;
    }
    if (n == 0) return 0;
    qsort(tmp, (size_t)n, sizeof(mag_t), cmp_mag);
    double mass = 0.0;
    for (int64_t i = 0; i < n; ++i) mass += tmp[i].a;
    double thr = alpha * mass;
    double run = 0.0;
    int64_t r = 0;
    while (r < n) {
        run += tmp[r].a;
        ++r;
        if (run >= thr) break;
    }
    for (int64_t i = 0; i < r; ++i) keep[tmp[i].pos] = 1;
    return r;
}

void or_mass_prune(int64_t n_rows, const int64_t *ptr, const int32_t *idx, const float *val,
                   double alpha, uint8_t *keep, int n_threads)
{
#pragma omp parallel num_threads(n_threads > 0 ? n_threads : 1)
    {
        int64_t maxn = 1;
        for (int64_t i = 0; i < n_rows; ++i)
            if (ptr[i + 1] - ptr[i] > maxn) maxn = ptr[i + 1] - ptr[i];
        mag_t *tmp = (mag_t *)malloc(sizeof(mag_t) * (size_t)maxn);
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n_rows; ++i)
            mass_prune_row(idx + ptr[i], val + ptr[i], ptr[i + 1] - ptr[i], alpha, tmp, keep + ptr[i]);
        free(tmp);
    }
}

/* ---------------------------------------------------------------------- */
/* Vector Number Pruning (Sec. 4.1): each row keeps the vn non-zero entries  */
/* of largest |x|; ties in |x| go to the lower term id (the order pi of      */
/* Def. 6).                                                                  */
void or_vnp_prune(int64_t n_rows, const int64_t *ptr, const int32_t *idx, const float *val,
                  int64_t vn, uint8_t *keep, int n_threads)
{
#pragma omp parallel num_threads(n_threads > 0 ? n_threads : 1)
    {
        int64_t maxn = 1;
        for (int64_t i = 0; i < n_rows; ++i)
            if (ptr[i + 1] - ptr[i] > maxn) maxn = ptr[i + 1] - ptr[i];
        mag_t *tmp = (mag_t *)malloc(sizeof(mag_t) * (size_t)maxn);
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n_rows; ++i) {
            int64_t n = 0;
            for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
                keep[e] = 0;
                if (val[e] == 0.0f) continue;  /* not an entry (Def. 1) */
                tmp[n].a = fabs((double)val[e]);
                tmp[n].id = idx[e];
                tmp[n].pos = e;
                ++n;
            }
            qsort(tmp, (size_t)n, sizeof(mag_t), cmp_mag);
            for (int64_t t = 0; t < n && t < vn; ++t) keep[tmp[t].pos] = 1;
        }
        free(tmp);
    }
}

/* ---------------------------------------------------------------------- */
/* List Pruning (Sec. 4.1): the list of every term keeps its lmax non-zero   */
/* entries of largest |x|; ties in |x| go to the lower document id.  With    */
/* keep_in, only entries it keeps take part (the combination of MRP then     */
/* LP); keep receives the result.                                            */
typedef struct {
    double a;
    int64_t doc;
    int64_t pos;
} lent_t;
static int cmp_lent(const void *x, const void *y)
{
    const lent_t *p = (const lent_t *)x, *q = (const lent_t *)y;
    if (p->a > q->a) return -1;
    if (p->a < q->a) return 1;
    return (p->doc > q->doc) - (p->doc < q->doc);
}

void or_lp_prune(int64_t n_rows, int64_t n_cols, const int64_t *ptr, const int32_t *idx,
                 const float *val, int64_t lmax, const uint8_t *keep_in, uint8_t *keep)
{
    const int64_t nnz = ptr[n_rows];
    int64_t *cnt = (int64_t *)calloc((size_t)n_cols + 1, sizeof(int64_t));
    for (int64_t e = 0; e < nnz; ++e) {
        keep[e] = 0;
        if (val[e] != 0.0f && (!keep_in || keep_in[e])) cnt[idx[e] + 1]++;
    }
    for (int64_t j = 0; j < n_cols; ++j) cnt[j + 1] += cnt[j];
    lent_t *col = (lent_t *)malloc(sizeof(lent_t) * (size_t)(cnt[n_cols] > 0 ? cnt[n_cols] : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_cols > 0 ? n_cols : 1));
    for (int64_t j = 0; j < n_cols; ++j) fill[j] = cnt[j];
    for (int64_t i = 0; i < n_rows; ++i)
        for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
            if (val[e] == 0.0f || (keep_in && !keep_in[e])) continue;
            lent_t *c = &col[fill[idx[e]]++];
            c->a = fabs((double)val[e]);
            c->doc = i;
            c->pos = e;
        }
    for (int64_t j = 0; j < n_cols; ++j) {
        const int64_t n = cnt[j + 1] - cnt[j];
        qsort(col + cnt[j], (size_t)n, sizeof(lent_t), cmp_lent);
        for (int64_t t = 0; t < n && t < lmax; ++t) keep[col[cnt[j] + t].pos] = 1;
    }
    free(fill);
    free(col);
    free(cnt);
}

/* ---------------------------------------------------------------------- */
/* Alg. 1 on the (kept part of the) corpus.  Lists I_{j,w} are laid out in  */
/* (j, w) order; within a list, documents ascend as the loop visits them.   */
/* out_ptr has n_cols * sigma + 1 entries, sigma = ceil(nd / window).       */
void or_build_index(int64_t nd, int64_t ncols, const int64_t *ptr, const int32_t *idx,
                    const float *val, const uint8_t *keep, int64_t window, int64_t *out_ptr,
                    int32_t *out_doc, float *out_val)
{
    int64_t sigma = (nd + window - 1) / window;
    int64_t nlists = ncols * sigma;
    memset(out_ptr, 0, sizeof(int64_t) * (size_t)(nlists + 1));
    for (int64_t i = 0; i < nd; ++i)
        for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e)
            if (!keep || keep[e]) out_ptr[(int64_t)idx[e] * sigma + i / window + 1]++;
    for (int64_t l = 0; l < nlists; ++l) out_ptr[l + 1] += out_ptr[l];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nlists > 0 ? nlists : 1));
    memcpy(fill, out_ptr, sizeof(int64_t) * (size_t)nlists);
    for (int64_t i = 0; i < nd; ++i) {
        int64_t w = i / window;
        for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
            if (keep && !keep[e]) continue;
            int64_t p = fill[(int64_t)idx[e] * sigma + w]++;
            out_doc[p] = (int32_t)i;
            out_val[p] = val[e];
        }
    }
    free(fill);
}

/* ---------------------------------------------------------------------- */
/* Min-heap H of Alg. 2, ordered so that its root is the LAST entry under   */
/* the ranking order (lowest score; among equal scores, highest id).        */
typedef struct {
    int64_t len, cap;
    double *s;
    int64_t *id;
} heap_t;

static int heap_below(const heap_t *h, int64_t a, int64_t b) /* a ranks after b */
{
    return ranks_before(h->s[b], h->id[b], h->s[a], h->id[a]);
}
static void heap_swap(heap_t *h, int64_t a, int64_t b)
{
    double s = h->s[a];
    int64_t i = h->id[a];
    h->s[a] = h->s[b];
    h->id[a] = h->id[b];
    h->s[b] = s;
    h->id[b] = i;
}
static void heap_push(heap_t *h, double s, int64_t id)
{
    int64_t c = h->len++;
    h->s[c] = s;
    h->id[c] = id;
    while (c > 0) {
        int64_t p = (c - 1) / 2;
        if (!heap_below(h, c, p)) break;
        heap_swap(h, c, p);
        c = p;
    }
}
static void heap_pop(heap_t *h)
{
    h->len--;
    if (h->len == 0) return;
    h->s[0] = h->s[h->len];
    h->id[0] = h->id[h->len];
    int64_t p = 0;
    for (;;) {
        int64_t l = 2 * p + 1, r = l + 1, m = p;
        if (l < h->len && heap_below(h, l, m)) m = l;
        if (r < h->len && heap_below(h, r, m)) m = r;
        if (m == p) break;
        heap_swap(h, p, m);
        p = m;
    }
}

/* Alg. 2 for one query (its non-zero terms qi/qv, n of them) over the index */
/* from or_build_index; returns the heap contents in h (up to k entries).    */
static void precise_search_one(int64_t nd, int64_t window, int64_t sigma, const int64_t *iptr,
                               const int32_t *idoc, const float *ival, const int32_t *qi,
                               const float *qv, int64_t n, int64_t k, double *A, heap_t *h)
{
    h->len = 0;
    if (k <= 0) return;
    for (int64_t m = 0; m < window; ++m) A[m] = 0.0;
    for (int64_t w = 0; w < sigma; ++w) {
        for (int64_t t = 0; t < n; ++t) {
            int64_t l = (int64_t)qi[t] * sigma + w;
            double qj = (double)qv[t];
            for (int64_t p = iptr[l]; p < iptr[l + 1]; ++p) {
                double P = qj * (double)ival[p]; /* SimdProduct entry */
                A[idoc[p] % window] += P;
            }
        }
        int64_t wlen = nd - w * window < window ? nd - w * window : window;
        for (int64_t m = 0; m < wlen; ++m) {
            int64_t id = m + window * w;
            /* ids rise through the scan, so "ranks before the root" is Alg. 2's strict ">" */
            if (h->len < k || ranks_before(A[m], id, h->s[0], h->id[0])) heap_push(h, A[m], id);
            if (h->len > k) heap_pop(h);
            A[m] = 0.0;
        }
    }
}

static void heap_to_sorted(heap_t *h, int64_t k, int64_t *ids, double *scores)
{
    /* popping the root repeatedly yields the ranking order reversed */
    int64_t n = h->len;
    for (int64_t t = n - 1; t >= 0; --t) {
        if (t < k) {
            ids[t] = h->id[0];
            scores[t] = h->s[0];
        }
        heap_pop(h);
    }
    for (int64_t t = n; t < k; ++t) {
        ids[t] = -1;
        scores[t] = -INFINITY;
    }
}

void or_precise_search(int64_t nd, int64_t window, const int64_t *iptr, const int32_t *idoc,
                       const float *ival, int64_t nq, const int64_t *qptr, const int32_t *qidx,
                       const float *qval, int64_t k, int64_t *out_ids, double *out_scores,
                       int n_threads)
{
    int64_t sigma = (nd + window - 1) / window;
#pragma omp parallel num_threads(n_threads > 0 ? n_threads : 1)
    {
        double *A = (double *)malloc(sizeof(double) * (size_t)window);
        heap_t h = {0, k + 1, (double *)malloc(sizeof(double) * (size_t)(k + 1)),
                    (int64_t *)malloc(sizeof(int64_t) * (size_t)(k + 1))};
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < nq; ++q) {
            precise_search_one(nd, window, sigma, iptr, idoc, ival, qidx + qptr[q], qval + qptr[q],
                               qptr[q + 1] - qptr[q], k, A, &h);
            heap_to_sorted(&h, k, out_ids + q * k, out_scores + q * k);
        }
        free(A);
        free(h.s);
        free(h.id);
    }
}

/* Alg. 4: q' = beta-mass(q); H = Alg. 2 (q', I, gamma); every popped       */
/* candidate i gets the exact delta(x_i, q) from the unpruned row and the   */
/* full query; R keeps the first k under the ranking order.  Optional       */
/* outputs: the coarse pool (ids, coarse scores) in ranking order.          */
void or_approx_search(int64_t nd, int64_t window, const int64_t *iptr, const int32_t *idoc,
                      const float *ival, const int64_t *dptr, const int32_t *didx,
                      const float *dval, int64_t nq, const int64_t *qptr, const int32_t *qidx,
                      const float *qval, double beta, int64_t gamma, int64_t k, int64_t *out_ids,
                      double *out_scores, int64_t *pool_ids, double *pool_scores, int n_threads)
{
    int64_t sigma = (nd + window - 1) / window;
    int64_t maxq = 1;
    for (int64_t q = 0; q < nq; ++q)
        if (qptr[q + 1] - qptr[q] > maxq) maxq = qptr[q + 1] - qptr[q];
#pragma omp parallel num_threads(n_threads > 0 ? n_threads : 1)
    {
        double *A = (double *)malloc(sizeof(double) * (size_t)window);
        heap_t h = {0, gamma + 1, (double *)malloc(sizeof(double) * (size_t)(gamma + 1)),
                    (int64_t *)malloc(sizeof(int64_t) * (size_t)(gamma + 1))};
        mag_t *tmp = (mag_t *)malloc(sizeof(mag_t) * (size_t)maxq);
        uint8_t *keep = (uint8_t *)malloc((size_t)maxq);
        int32_t *pi = (int32_t *)malloc(sizeof(int32_t) * (size_t)maxq);
        float *pv = (float *)malloc(sizeof(float) * (size_t)maxq);
        int64_t *cid = (int64_t *)malloc(sizeof(int64_t) * (size_t)(gamma > 0 ? gamma : 1));
        double *cs = (double *)malloc(sizeof(double) * (size_t)(gamma > 0 ? gamma : 1));
        ranked_t R;
        rl_init(&R, k);
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < nq; ++q) {
            const int32_t *qi = qidx + qptr[q];
            const float *qv = qval + qptr[q];
            int64_t n = qptr[q + 1] - qptr[q];
            /* beta-mass subvector of q, kept entries in ascending term order */
            mass_prune_row(qi, qv, n, beta, tmp, keep);
            int64_t np = 0;
            for (int64_t t = 0; t < n; ++t)
                if (keep[t]) {
                    pi[np] = qi[t];
                    pv[np] = qv[t];
                    ++np;
                }
            /* coarse pool of gamma candidates (Alg. 2 over the pruned index) */
            precise_search_one(nd, window, sigma, iptr, idoc, ival, pi, pv, np, gamma, A, &h);
            int64_t nc = h.len;
            heap_to_sorted(&h, nc, cid, cs);
            if (pool_ids)
                for (int64_t t = 0; t < gamma; ++t) {
                    pool_ids[q * gamma + t] = t < nc ? cid[t] : -1;
                    pool_scores[q * gamma + t] = t < nc ? cs[t] : -INFINITY;
                }
            /* exact rerank of every candidate from the unpruned rows, keep the best k */
            R.len = 0;
            for (int64_t t = 0; t < nc; ++t) {
                int64_t i = cid[t];
                double d = dot_rows(didx + dptr[i], dval + dptr[i], dptr[i + 1] - dptr[i], qi, qv, n);
                rl_offer(&R, d, i);
            }
            rl_write(&R, k, out_ids + q * k, out_scores + q * k);
        }
        rl_free(&R);
        free(A);
        free(h.s);
        free(h.id);
        free(tmp);
        free(keep);
        free(pi);
        free(pv);
        free(cid);
        free(cs);
    }
}

/* ---------------------------------------------------------------------- */
/* Scores s[b][c] = delta(q_b, x_{cand[b][c]}) are bilinear in the values:  */
/*   ds/dq_b[t] = x_c[t]   and   ds/dx_c[t] = q_b[t]   for t in both rows.  */
/* Given G = dL/ds, accumulates dL/dq (aligned with the query values) and   */
/* dL/dx (aligned with the corpus values).  Candidates with id < 0 skip.    */
void or_score_grad(const int64_t *dptr, const int32_t *didx, const float *dval,
                   const int64_t *qptr, const int32_t *qidx, const float *qval, int64_t nq,
                   int64_t n_cand, const int64_t *cand, const double *G, double *gq, double *gx)
{
    for (int64_t b = 0; b < nq; ++b)
        for (int64_t c = 0; c < n_cand; ++c) {
            int64_t d = cand[b * n_cand + c];
            if (d < 0) continue;
            double g = G[b * n_cand + c];
            int64_t a = qptr[b], ae = qptr[b + 1], e = dptr[d], ee = dptr[d + 1];
            while (a < ae && e < ee) {
                if (qidx[a] < didx[e]) {
                    ++a;
                } else if (qidx[a] > didx[e]) {
                    ++e;
                } else {
                    if (gq) gq[a] += g * (double)dval[e];
                    if (gx) gx[e] += g * (double)qval[a];
                    ++a;
                    ++e;
                }
            }
        }
}
