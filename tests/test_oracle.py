"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Each test names the passage it pins.  None of them re-derives an expected
value by calling the oracle's own routine again; they use printed values,
closed forms, brute force, special cases and invariants.
"""
import math

import numpy as np
import pytest
from scipy.stats import norm

import oracle
import synth
from conftest import csr_from_dict_rows, dense, load_golden, rank_order


# ---------------------------------------------------------------- Def. 1 / 6
def test_sparse_vector_example_and_mass_prune():
    """Sec. 2.1 example: ||x|| = 4; Def. 6 at alpha = 0.7 keeps the two largest."""
    g = load_golden("paper_sparse_vector_example.json")
    p = g["printed_in_paper"]
    csr = synth.Csr(np.array([0, 4], np.int64), np.array(p["ids"], np.int32),
                    np.array(p["values"], np.float32), 10000)
    assert csr.nnz == p["nnz"]
    keep = oracle.mass_prune(csr, g["derived_by_def6"]["alpha"])
    assert sorted(csr.indices[keep.astype(bool)].tolist()) == g["derived_by_def6"]["kept_ids"]


def test_mass_prune_inclusive_boundary():
    """Def. 6 uses ">=": {0.5, 0.25, 0.25} at alpha 0.5 keeps one entry (dyadic, exact)."""
    csr = synth.Csr(np.array([0, 3], np.int64), np.array([0, 1, 2], np.int32),
                    np.array([0.5, 0.25, 0.25], np.float32), 3)
    assert oracle.mass_prune(csr, 0.5).tolist() == [1, 0, 0]
    # just above the boundary needs the second entry
    assert oracle.mass_prune(csr, 0.5000001).sum() == 2


def test_mass_prune_tie_break_lower_id():
    """pi sorts by |x| descending, equal |x| by ascending id: {0.25, 0.5, 0.25} at 0.75
    keeps ids {1, 0}; the tie between ids 0 and 2 goes to id 0."""
    csr = synth.Csr(np.array([0, 3], np.int64), np.array([0, 1, 2], np.int32),
                    np.array([0.25, 0.5, 0.25], np.float32), 3)
    assert oracle.mass_prune(csr, 0.75).tolist() == [1, 1, 0]


def test_mass_prune_uses_magnitude():
    """Def. 5: mass sums absolute values; a large negative entry is kept first."""
    csr = synth.Csr(np.array([0, 3], np.int64), np.array([0, 1, 2], np.int32),
                    np.array([-4.0, 1.0, 1.0], np.float32), 3)
    assert oracle.mass_prune(csr, 0.6).tolist() == [1, 0, 0]
    assert oracle.mass_prune(csr, 0.7).tolist() == [1, 1, 0]


def test_mass_prune_alpha_one_is_identity_and_empty_rows():
    rng = np.random.default_rng(1)
    csr = synth.random_csr(rng, 200, 500, 40, signed=True)
    assert oracle.mass_prune(csr, 1.0).all()
    assert (np.diff(csr.indptr) == 0).any()  # empty rows present and harmless


def test_mass_prune_never_keeps_explicit_zeros():
    """Def. 1: a sparse vector is the set of its non-zero entries, so a stored 0 is no entry
    and no alpha keeps it; a row holding only zeros keeps nothing, and the zeros do not
    change which non-zero entries a row keeps."""
    csr = synth.Csr(np.array([0, 2, 5, 6], np.int64), np.array([1, 4, 0, 2, 3, 7], np.int32),
                    np.array([0.0, 0.0, 0.5, 0.0, 0.5, 0.0], np.float32), 8)
    for alpha in (0.1, 0.5, 1.0):
        keep = oracle.mass_prune(csr, alpha)
        assert keep[[0, 1, 3, 5]].tolist() == [0, 0, 0, 0], alpha
    assert oracle.mass_prune(csr, 1.0)[[2, 4]].tolist() == [1, 1]
    # alpha 0.5 of {0.5, 0.5}: the first (lower id) reaches half the mass alone
    assert oracle.mass_prune(csr, 0.5)[[2, 4]].tolist() == [1, 0]
    rng = np.random.default_rng(3)
    c = synth.random_csr(rng, 300, 400, 30, signed=True)
    z = c.values.copy()
    z[::5] = 0.0
    cz = synth.Csr(c.indptr, c.indices, z, c.n_cols)
    stripped = oracle.apply_mask(cz, (z != 0).astype(np.uint8))
    for alpha in (0.3, 0.8, 1.0):
        keep = oracle.mass_prune(cz, alpha)
        assert not keep[z == 0].any()
        assert np.array_equal(keep[z != 0], oracle.mass_prune(stripped, alpha))


@pytest.mark.parametrize("alpha", [0.3, 0.5, 0.7])
def test_mass_prune_lognormal_closed_form(alpha):
    """For lognormal(0, s) entries the alpha-mass subvector keeps the entries above
    t with E[X; X > t] = alpha E[X]; that fraction is Phi(Phi^-1(alpha) - s)."""
    sigma = 0.8
    rows = synth.generate(40, 200_000, nnz=("uniform", 20000, 20000), clip=(1, 20000),
                          terms=("uniform",), values=("lognormal", 0.0, sigma), seed=5)
    frac = oracle.mass_prune(rows, alpha).mean()
    expect = norm.cdf(norm.ppf(alpha) - sigma)
    assert abs(frac - expect) < 3e-3, (frac, expect)


def test_mass_prune_minimal_prefix_random():
    """Kept set is the shortest prefix of pi reaching alpha * mass (checked by brute force
    over all prefixes, in exact rational arithmetic on the float32 inputs)."""
    from fractions import Fraction
    rng = np.random.default_rng(2)
    csr = synth.random_csr(rng, 60, 100, 30, signed=True, min_nnz=1)
    alpha = 0.55
    keep = oracle.mass_prune(csr, alpha).astype(bool)
    for r in range(csr.n_rows):
        i, v = csr.row(r)
        k = keep[csr.indptr[r]:csr.indptr[r + 1]]
        order = sorted(range(len(i)), key=lambda t: (-abs(float(v[t])), int(i[t])))
        mags = [Fraction(abs(float(v[t]))) for t in order]
        mass = sum(mags)
        # exact rational threshold; the FP64 rounding of alpha * mass only matters within
        # an ulp of a prefix sum, which these random magnitudes never hit
        thr = Fraction(alpha) * mass
        run, rr = Fraction(0), 0
        while rr < len(mags):
            run += mags[rr]
            rr += 1
            if run >= thr:
                break
        expect = np.zeros(len(i), bool)
        expect[order[:rr]] = True
        assert (k == expect).all(), r


# ---------------------------------------------------------------- Defs. 2-3
def test_exact_topk_matches_dense_bruteforce():
    rng = np.random.default_rng(3)
    corpus = synth.random_csr(rng, 700, 300, 25, signed=True)
    queries = synth.random_csr(rng, 40, 300, 12, signed=True)
    k = 17
    ids, sc = oracle.exact_topk(corpus, queries, k)
    S = dense(queries) @ dense(corpus).T
    for q in range(queries.n_rows):
        order = rank_order(S[q])[:k]
        np.testing.assert_allclose(sc[q], S[q][order], rtol=1e-12, atol=1e-12)
        # ids equal unless two scores are within rounding of each other
        for a, b in zip(ids[q], order):
            if a != b:
                assert abs(S[q][a] - S[q][b]) < 1e-12


def test_exact_topk_special_cases():
    rng = np.random.default_rng(4)
    corpus = synth.random_csr(rng, 50, 40, 8)
    # k larger than the corpus: complete order, padded with -1 / -inf
    q = synth.random_csr(rng, 3, 40, 5, min_nnz=1)
    ids, sc = oracle.exact_topk(corpus, q, 60)
    S = dense(q) @ dense(corpus).T
    for r in range(3):
        assert (ids[r, 50:] == -1).all() and np.isneginf(sc[r, 50:]).all()
        assert ids[r, :50].tolist() == rank_order(S[r]).tolist()
    # empty query: every score is 0, so the lowest ids win
    empty = synth.Csr(np.array([0, 0], np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32), 40)
    ids, sc = oracle.exact_topk(corpus, empty, 5)
    assert ids[0].tolist() == [0, 1, 2, 3, 4] and (sc[0] == 0).all()
    # single-term query: the top-k of that column by q * x
    j = int(corpus.indices[0])
    one = synth.Csr(np.array([0, 1], np.int64), np.array([j], np.int32), np.array([2.0], np.float32), 40)
    ids, sc = oracle.exact_topk(corpus, one, 3)
    col = dense(corpus)[:, j] * 2.0
    assert ids[0].tolist() == rank_order(col)[:3].tolist()


def test_pair_scores_products_are_exact():
    """Products of float32 values are exact in FP64: one common dimension gives x*q exactly."""
    a = np.float32(1.0000001)
    b = np.float32(3.3333333)
    c = synth.Csr(np.array([0, 1], np.int64), np.array([7], np.int32), np.array([a], np.float32), 9)
    q = synth.Csr(np.array([0, 1], np.int64), np.array([7], np.int32), np.array([b], np.float32), 9)
    from fractions import Fraction
    got = oracle.pair_scores(c, q, [0], [0])[0]
    assert Fraction(got) == Fraction(float(a)) * Fraction(float(b))


# ---------------------------------------------------------------- Sec. 3.2 example
def _paper_example():
    g = load_golden("paper_search_example.json")
    f = g["filled_in_not_printed"]
    corpus = csr_from_dict_rows(f["docs"], g["printed_in_paper"]["n_docs"], g["n_cols"])
    p, d = g["printed_in_paper"], g["derived"]
    dims = p["query_dims"]
    vals = [d["q1"], f["q5"], f["q8"]]
    return g, corpus, dims, vals


def _q(dims, vals, n_cols):
    return synth.Csr(np.array([0, len(dims)], np.int64), np.array(dims, np.int32),
                     np.array(vals, np.float32), n_cols)


def test_paper_search_example():
    g, corpus, dims, vals = _paper_example()
    p = g["printed_in_paper"]
    n_cols = g["n_cols"]
    # accumulation after I_1, after I_1 + I_5, and final A[4]
    s1 = oracle.pair_scores(corpus, _q(dims[:1], vals[:1], n_cols), [0], [4])[0]
    s15 = oracle.pair_scores(corpus, _q(dims[:2], vals[:2], n_cols), [0], [4])[0]
    q = _q(dims, vals, n_cols)
    ids, sc = oracle.exact_topk(corpus, q, 9)
    assert s1 == pytest.approx(p["q1_times_x4_dim1"], rel=1e-6)
    assert s15 == pytest.approx(p["A4_after_I1_I5"], rel=1e-6)
    assert ids[0, 0] == p["argmax_doc"]
    assert sc[0, 0] == pytest.approx(p["A4_final"], rel=1e-6)
    touched = sorted(int(i) for i, s in zip(ids[0], sc[0]) if s != 0)
    assert touched == p["touched_docs"]
    # Alg. 1 posting positions: x_4 is P[0] of I_1 and P[2] of I_5
    idx = oracle.build_index(corpus, window=9)
    assert list(idx.list(1, 0)[0]).index(4) == p["x4_dim1_position_in_I1"]
    assert list(idx.list(5, 0)[0]).index(4) == p["x4_dim5_position_in_I5"]
    # Alg. 2 finds the same argmax and value for any window size (Sec. 3.3.1)
    for lam in (1, 2, 4, 9):
        pid, ps = oracle.precise_search(oracle.build_index(corpus, window=lam), q, 1)
        assert pid[0, 0] == 4 and ps[0, 0] == pytest.approx(p["A4_final"], rel=1e-6)


# ---------------------------------------------------------------- Alg. 1
def test_index_is_exact_transpose_per_window():
    rng = np.random.default_rng(6)
    corpus = synth.random_csr(rng, 333, 50, 12, signed=True)
    keep = oracle.mass_prune(corpus, 0.6)
    kept = oracle.apply_mask(corpus, keep)
    for lam in (1, 10, 64, 333, 1000):
        idx = oracle.build_index(corpus, lam, keep)
        sigma = (333 + lam - 1) // lam
        assert idx.ptr.shape[0] == 50 * sigma + 1
        back = {}
        for j in range(50):
            for w in range(sigma):
                docs, vals = idx.list(j, w)
                assert (np.diff(docs) > 0).all()
                assert ((docs >= w * lam) & (docs < (w + 1) * lam)).all()
                for d, v in zip(docs, vals):
                    back.setdefault(int(d), []).append((j, v))
        for r in range(333):
            i, v = kept.row(r)
            got = back.get(r, [])
            assert [t for t, _ in got] == i.tolist()
            assert np.array([x for _, x in got], np.float32).tobytes() == v.tobytes()


# ---------------------------------------------------------------- Alg. 2
def test_precise_search_equals_full_sort_with_ties():
    """Alg. 2's heap keeps the first k under (score desc, id asc), ties included."""
    rng = np.random.default_rng(7)
    corpus = synth.random_csr(rng, 120, 12, 4, min_nnz=1)
    corpus = synth.Csr(corpus.indptr, corpus.indices, np.ones_like(corpus.values), 12)  # many ties
    queries = synth.random_csr(rng, 25, 12, 3)
    queries = synth.Csr(queries.indptr, queries.indices, np.ones_like(queries.values), 12)
    S = dense(queries) @ dense(corpus).T
    for lam in (1, 7, 50, 120):
        ids, sc = oracle.precise_search(oracle.build_index(corpus, lam), queries, 15)
        for q in range(25):
            assert ids[q].tolist() == rank_order(S[q])[:15].tolist()
            assert sc[q].tolist() == S[q][ids[q]].tolist()


def test_precise_search_ranks_every_document_once_with_a_short_last_window():
    """With k = n_docs Alg. 2 returns each document exactly once: the last window (here 13 of
    50 documents) is scanned only up to the corpus's end, so no id past it enters the heap, not
    even ahead of documents whose signed scores fall below zero."""
    rng = np.random.default_rng(11)
    corpus = synth.random_csr(rng, 113, 30, 8, signed=True)
    queries = synth.random_csr(rng, 6, 30, 6, signed=True, min_nnz=1)
    S = dense(queries) @ dense(corpus).T
    assert (S < 0).any(axis=1).all()
    ids, sc = oracle.precise_search(oracle.build_index(corpus, 50), queries, 113)
    for q in range(6):
        assert sorted(ids[q].tolist()) == list(range(113))
        assert ids[q].tolist() == rank_order(S[q]).tolist()


def test_coarse_scores_are_per_document_dots_of_pruned_vectors():
    """Summing postings over the query's lists equals each pruned document's dot (Sec. 3.2)."""
    rng = np.random.default_rng(8)
    corpus = synth.random_csr(rng, 400, 80, 20)
    queries = synth.random_csr(rng, 10, 80, 10, min_nnz=1)
    keep = oracle.mass_prune(corpus, 0.5)
    kept = oracle.apply_mask(corpus, keep)
    ids, sc = oracle.precise_search(oracle.build_index(corpus, 37, keep), queries, 400)
    for q in range(10):
        direct = oracle.pair_scores(kept, queries, np.full(400, q), ids[q])
        assert direct.tobytes() == sc[q].tobytes()  # same terms, same ascending order


def test_work_count_is_sum_of_list_lengths_and_window_free():
    """Thm. 3.1 / Sec. 3.3.1: postings visited = sum of the query's list lengths, any lambda."""
    rng = np.random.default_rng(9)
    corpus = synth.random_csr(rng, 300, 40, 10)
    qi = np.array([1, 5, 17], np.int32)
    lens = None
    for lam in (1, 13, 300):
        idx = oracle.build_index(corpus, lam)
        n = sum(int(idx.ptr[(j + 1) * idx.sigma] - idx.ptr[j * idx.sigma]) for j in qi)
        lens = n if lens is None else lens
        assert n == lens
    col_counts = np.bincount(corpus.indices, minlength=40)
    assert lens == int(col_counts[qi].sum())


# ---------------------------------------------------------------- Alg. 4
def test_approx_reduces_to_exact_without_pruning():
    """alpha = beta = 1 and gamma >= k: coarse scores are exact, so R = R* (Alg. 4)."""
    rng = np.random.default_rng(10)
    corpus = synth.random_csr(rng, 500, 60, 15, signed=True)
    queries = synth.random_csr(rng, 30, 60, 8)
    idx = oracle.build_index(corpus, 128)
    ex_ids, ex_sc = oracle.exact_topk(corpus, queries, 10)
    for gamma in (10, 50, 500):
        ids, sc, pid, _ = oracle.approx_search(idx, corpus, queries, 1.0, gamma, 10,
                                               want_pool=True)
        assert ids.tolist() == ex_ids.tolist()
        assert sc.tobytes() == ex_sc.tobytes()
        # the pool holds real documents only: 500 is not a multiple of the window, and a scan
        # of the last window past the corpus's end would admit ids 500..511 with coarse score 0,
        # ahead of the documents whose signed scores are negative
        assert ((pid >= 0) & (pid < 500)).all()
    assert all(sorted(row) == list(range(500)) for row in pid.tolist())


def test_approx_rerank_scores_are_exact_for_returned_ids():
    """With pruning, every returned score is delta(x_i, q) of the unpruned row (Alg. 4, its exact rerank),
    and the result is the best k of the coarse pool under exact scores."""
    wl_rng = np.random.default_rng(11)
    corpus = synth.random_csr(wl_rng, 800, 100, 30)
    queries = synth.random_csr(wl_rng, 20, 100, 12, min_nnz=1)
    keep = oracle.mass_prune(corpus, 0.4)
    idx = oracle.build_index(corpus, 100, keep)
    ids, sc, pid, ps = oracle.approx_search(idx, corpus, queries, 0.8, 40, 10, want_pool=True)
    S = dense(queries) @ dense(corpus).T
    for q in range(20):
        np.testing.assert_allclose(sc[q], S[q][ids[q]], rtol=1e-12)
        pool = pid[q][pid[q] >= 0]
        best = pool[rank_order(S[q][pool], pool)][:10]
        assert ids[q].tolist() == best.tolist()


def test_approx_beta_prunes_query_for_coarse_stage_only():
    """beta-mass(q) drives the coarse pool (Sec. 4.1), the rerank uses the full q (Alg. 4)."""
    rng = np.random.default_rng(12)
    corpus = synth.random_csr(rng, 300, 50, 20)
    queries = synth.random_csr(rng, 8, 50, 10, min_nnz=2)
    idx = oracle.build_index(corpus, 50)
    qkeep = oracle.mass_prune(queries, 0.5)
    qp = oracle.apply_mask(queries, qkeep)
    _, _, pid, ps = oracle.approx_search(idx, corpus, queries, 0.5, 30, 5, want_pool=True)
    cid, cs = oracle.precise_search(idx, qp, 30)
    assert pid.tolist() == cid.tolist() and ps.tobytes() == cs.tobytes()


# ---------------------------------------------------------------- recall, gradients
def test_recall_at_k():
    truth = np.array([[1, 2, 3, 4], [5, 6, 7, 8]])
    found = np.array([[4, 3, 9, 1], [5, 6, 7, 8]])
    assert oracle.recall_at_k(found, truth) == pytest.approx((3 / 4 + 1) / 2)


def test_score_grad_matches_finite_differences():
    """Gradient of a softmax contrastive loss over candidate scores, through the bilinear
    scores, against central differences (h = 1e-3) in FP64 on dense copies."""
    rng = np.random.default_rng(13)
    corpus = synth.random_csr(rng, 60, 30, 10, min_nnz=1)
    queries = synth.random_csr(rng, 4, 30, 8, min_nnz=2)
    cand = np.stack([rng.choice(60, size=7, replace=False) for _ in range(4)])
    pos = rng.integers(0, 7, size=4)
    tau = 3.0
    Dq, Dx = dense(queries), dense(corpus)

    def loss(Dq_, Dx_):
        S = np.einsum("bt,bct->bc", Dq_, Dx_[cand])
        return oracle.contrastive_grad(S, pos, tau)[0]

    S = np.einsum("bt,bct->bc", Dq, Dx[cand])
    _, G = oracle.contrastive_grad(S, pos, tau)
    gq, gx = oracle.score_grad(corpus, queries, cand, G)
    h = 1e-3
    for b in range(4):
        for e in range(int(queries.indptr[b]), int(queries.indptr[b + 1])):
            t = queries.indices[e]
            P, M = Dq.copy(), Dq.copy()
            P[b, t] += h
            M[b, t] -= h
            fd = (loss(P, Dx) - loss(M, Dx)) / (2 * h)
            assert gq[e] == pytest.approx(fd, rel=1e-6, abs=1e-10)
    for d in np.unique(cand)[:10]:
        for e in range(int(corpus.indptr[d]), int(corpus.indptr[d + 1])):
            t = corpus.indices[e]
            P, M = Dx.copy(), Dx.copy()
            P[d, t] += h
            M[d, t] -= h
            fd = (loss(Dq, P) - loss(Dq, M)) / (2 * h)
            assert gx[e] == pytest.approx(fd, rel=1e-6, abs=1e-10)


# ------------------------------------------------------------------ VNP and LP (Sec. 4.1)
def _transpose(csr):
    """The CSR of the transpose (rows = terms, column ids = document ids) and, for every
    entry of it, the position of the same entry in csr."""
    import synth
    rows = np.repeat(np.arange(csr.n_rows), np.diff(csr.indptr))
    order = np.lexsort((rows, csr.indices))
    counts = np.bincount(csr.indices, minlength=csr.n_cols)
    indptr = np.zeros(csr.n_cols + 1, np.int64)
    np.cumsum(counts, out=indptr[1:])
    t = synth.Csr(indptr, rows[order].astype(np.int32), csr.values[order].copy(), csr.n_rows)
    return t, order


def _vnp_invariants(csr, vn, keep):
    for r in range(csr.n_rows):
        a, b = csr.indptr[r], csr.indptr[r + 1]
        k, v, ids = keep[a:b].astype(bool), np.abs(csr.values[a:b].astype(np.float64)), csr.indices[a:b]
        nz = v > 0
        assert k.sum() == min(vn, nz.sum())
        assert not (k & ~nz).any()
        if k.any() and (nz & ~k).any():
            lo_kept, hi_drop = v[k].min(), v[nz & ~k].max()
            assert lo_kept >= hi_drop
            if lo_kept == hi_drop:  # a tie at the cut goes to the lower term id
                assert ids[k & (v == lo_kept)].max() < ids[nz & ~k & (v == hi_drop)].min()


def test_vnp_keeps_the_largest_entries_with_id_ties():
    rng = np.random.default_rng(41)
    csr = synth.random_csr(rng, 300, 80, 40, signed=True)
    csr.values[::7] = np.round(csr.values[::7])  # many exact ties in |x|
    for vn in (1, 3, 10, 100):
        _vnp_invariants(csr, vn, oracle.vnp_prune(csr, vn))


def test_vnp_with_mrp_counts_is_mrp():
    """MRP keeps a prefix of the same order pi, so VNP with each row's MRP count agrees."""
    rng = np.random.default_rng(42)
    csr = synth.random_csr(rng, 200, 500, 60)
    keep = oracle.mass_prune(csr, 0.6)
    for r in range(csr.n_rows):
        a, b = csr.indptr[r], csr.indptr[r + 1]
        row = synth.Csr(np.array([0, b - a]), csr.indices[a:b], csr.values[a:b], csr.n_cols)
        assert (oracle.vnp_prune(row, int(keep[a:b].sum())) == keep[a:b]).all()


def test_lp_is_vnp_of_the_transpose():
    """List pruning keeps, per term, what VNP keeps per row of the transposed matrix
    (there the ties in |x| go to the lower document id)."""
    rng = np.random.default_rng(43)
    csr = synth.random_csr(rng, 400, 60, 30, signed=True)
    csr.values[::5] = np.round(csr.values[::5] * 2) / 2
    t, order = _transpose(csr)
    for lmax in (1, 4, 25, 10_000):
        keep = oracle.lp_prune(csr, lmax)
        kt = oracle.vnp_prune(t, lmax)
        assert (keep[order] == kt).all()
        counts = np.bincount(csr.indices[keep.astype(bool)], minlength=csr.n_cols)
        assert (counts == np.minimum(np.bincount(csr.indices[csr.values != 0], minlength=csr.n_cols), lmax)).all()


def test_lp_after_mrp_competes_only_among_mrp_entries():
    rng = np.random.default_rng(44)
    csr = synth.random_csr(rng, 300, 50, 25)
    mrp = oracle.mass_prune(csr, 0.5)
    both = oracle.lp_prune(csr, 6, keep_in=mrp)
    assert not (both & ~mrp).any()
    sub = oracle.apply_mask(csr, mrp)
    assert (oracle.lp_prune(sub, 6) == both[mrp.astype(bool)]).all()
    assert (oracle.lp_prune(csr, 10_000, keep_in=mrp) == mrp).all()
