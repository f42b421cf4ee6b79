"""GPU parity: the HIP path through the C ABI against the CPU oracle, element by element."""
import numpy as np
import pytest

import oracle
import synth
from conftest import csr_from_dict_rows, load_golden
from parity import (check_bank_order, check_ranked, check_same_topk, check_scores, pool_margin_fn,
                    score_scale)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sindi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_08395_amd as s
    s._lib.load()
    return s


# A corpus spanning several windows and tiles, with ragged last window and tiles.
N_DOCS, VOCAB, WINDOW, TILE = 30_011, 2_000, 7_000, 2_048


@pytest.fixture(scope="module")
def small():
    corpus = synth.generate(N_DOCS, VOCAB, nnz=("poisson", 40.0), seed=11)
    queries = synth.generate(64, VOCAB, nnz=("poisson", 12.0), seed=11, stream=1)
    return corpus, queries


def _np(t):
    return t.detach().cpu().numpy()


def _tol_kth(corpus, queries, ref_ids, ref_scores, rtol):
    """Absolute near-tie tolerance at each row's last place."""
    nq, k = ref_ids.shape
    last = np.array([ref_ids[r][ref_ids[r] >= 0][-1] if (ref_ids[r] >= 0).any() else 0
                     for r in range(nq)])
    sc = score_scale(corpus, queries, np.arange(nq), last)
    return 2.0 * rtol * np.maximum(sc, 1e-30)


# ------------------------------------------------------------------ index layout
@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_index_layout_is_alg1_bit_exact(sindi, small, dtype):
    corpus, _ = small
    alpha = 0.5
    idx = sindi.Index(corpus, alpha=alpha, window=WINDOW, value_dtype=dtype, tile=TILE)
    ex = idx.export()
    info = idx.info()
    keep = oracle.mass_prune(corpus, alpha)
    ref = oracle.build_index(corpus, WINDOW, keep)
    assert info["n_postings"] == int(keep.sum())
    assert info["n_windows"] == ref.sigma
    tile_doc, tile_post, term_off = ex["tile_doc"], ex["tile_post"], ex["term_off"]
    assert tile_doc[0] == 0 and tile_doc[-1] == N_DOCS
    assert (np.diff(tile_doc) <= TILE).all() and (np.diff(tile_doc) > 0).all()
    # tiles never straddle a window boundary
    assert ((tile_doc[:-1] // WINDOW) == ((tile_doc[1:] - 1) // WINDOW)).all()
    nt = tile_doc.shape[0] - 1
    tile_of = np.repeat(np.arange(nt), np.diff(tile_post))
    term_of = np.concatenate([np.repeat(np.arange(VOCAB), np.diff(term_off[t])) for t in range(nt)])
    doc = ex["post_doc"].astype(np.int64) + tile_doc[tile_of]
    win = doc // WINDOW
    order = np.lexsort((doc, win, term_of))  # Alg. 1 order: term, window, document
    ref_docs = ref.doc.astype(np.int64)
    ref_win = ref_docs // WINDOW
    ref_term = np.repeat(np.arange(VOCAB), np.diff(ref.ptr[::ref.sigma]))
    assert (doc[order] == ref_docs).all()
    assert (win[order] == ref_win).all()
    assert (term_of[order] == ref_term).all()
    # inside every (tile, term) list the documents ascend
    same = (tile_of[1:] == tile_of[:-1]) & (term_of[1:] == term_of[:-1])
    assert (np.diff(doc)[same] > 0).all()
    # stored form: every list starts on a 4-slot boundary, each chunk of 256 slots in LDS-bank
    # order, pads hold value 0 and repeat the list's largest document
    rx = idx.export(raw=True)
    check_bank_order(rx, ex)
    goff = rx["term_goff"]
    assert (rx["tile_post"] % 4 == 0).all() and info["n_slots"] == rx["tile_post"][-1]
    assert (rx["post_doc"] % 4 == 0).all()  # stored as byte offsets of 32-bit score words
    start = 4 * (goff & 0x3FFFFFFF).astype(np.int64)
    pad = (goff >> 30).astype(np.int64)
    length = np.diff(start, axis=1) - pad[:, :-1]
    assert (length >= 0).all() and (length.sum() == info["n_postings"])
    assert ((pad[:, :-1] == (-length) % 4)).all() and (pad[:, -1] == 0).all()
    zero_bits = rx["post_val"].view(np.uint32 if dtype == "f32" else np.uint16)
    for t in range(nt):
        for j in np.nonzero(pad[t, :-1])[0][:50]:
            a = rx["tile_post"][t] + start[t, j] + length[t, j]
            assert (zero_bits[a:a + pad[t, j]] == 0).all()
    vals = ex["post_val"][order]
    if dtype == "f32":
        assert vals.view(np.uint32).tolist() == ref.val.view(np.uint32).tolist()
    elif dtype == "f16":
        assert vals.tolist() == ref.val.astype(np.float16).view(np.uint16).tolist()
    else:
        bf = torch.from_numpy(ref.val.copy()).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
        assert vals.tolist() == bf.tolist()


# ------------------------------------------------------------------ exact search
def test_exact_search_tiny_workload(sindi):
    """Plain method, exact: 10K docs, vocab 30,522, 100 queries, no pruning, top-10."""
    from synth.workloads import WORKLOADS
    wl = WORKLOADS["tiny"]
    corpus, queries = wl.corpus(), wl.queries()
    idx = sindi.Index(corpus, alpha=1.0, window=wl.window)
    ids, sc = idx.search(queries, wl.k, gamma=wl.gamma)
    ids, sc = _np(ids), _np(sc)
    ref_ids, ref_sc = oracle.exact_topk(corpus, queries, wl.k)
    check_ranked(ids, sc)
    check_scores(corpus, queries, ids, sc, rtol=1e-5)
    check_same_topk(ids, ref_ids, ref_sc, _tol_kth(corpus, queries, ref_ids, ref_sc, 1e-5))
    assert oracle.recall_at_k(ids, ref_ids) >= 0.99


def test_exact_search_signed_values_and_ragged_tiles(sindi):
    rng = np.random.default_rng(21)
    corpus = synth.random_csr(rng, 5_003, 300, 30, signed=True)
    queries = synth.random_csr(rng, 40, 300, 15, signed=True)
    idx = sindi.Index(corpus, alpha=1.0, window=1_234, tile=500)
    for k in (1, 7, 33):
        ids, sc = idx.search(queries, k, gamma=k)
        ids, sc = _np(ids), _np(sc)
        ref_ids, ref_sc = oracle.exact_topk(corpus, queries, k)
        check_ranked(ids, sc)
        check_scores(corpus, queries, ids, sc, rtol=1e-5)
        check_same_topk(ids, ref_ids, ref_sc, _tol_kth(corpus, queries, ref_ids, ref_sc, 1e-5))


def test_paper_worked_example_on_gpu(sindi):
    g = load_golden("paper_search_example.json")
    f = g["filled_in_not_printed"]
    corpus = csr_from_dict_rows(f["docs"], 9, g["n_cols"])
    q = synth.Csr(np.array([0, 3], np.int64), np.array([1, 5, 8], np.int32),
                  np.array([g["derived"]["q1"], f["q5"], f["q8"]], np.float32), g["n_cols"])
    idx = sindi.Index(corpus, alpha=1.0, window=9)
    ids, sc = idx.search(q, 9, gamma=9)
    ids, sc = _np(ids)[0], _np(sc)[0]
    assert ids[0] == g["printed_in_paper"]["argmax_doc"]
    assert sc[0] == pytest.approx(g["printed_in_paper"]["A4_final"], rel=1e-6)
    assert sorted(int(i) for i, s in zip(ids, sc) if s != 0) == g["printed_in_paper"]["touched_docs"]
    cid, csc = idx.search_coarse(q, 1)
    assert int(_np(cid)[0, 0]) == 4 and float(_np(csc)[0, 0]) == pytest.approx(36.1, rel=1e-6)


# ------------------------------------------------------------------ Alg. 2 / Alg. 4
def _pool_margin(pool_ids, pool_sc, corpus_pruned, queries_pruned, rtol):
    """Near-tie test at the rerank-pool boundary on oracle coarse scores."""
    gam = pool_ids.shape[1]

    def f(r, d):
        valid = pool_ids[r] >= 0
        last = pool_sc[r][valid][-1]
        lastid = pool_ids[r][valid][-1]
        c = oracle.pair_scores(corpus_pruned, queries_pruned, [r], [d])[0]
        sc = score_scale(corpus_pruned, queries_pruned, [r, r], [d, lastid]).max()
        return abs(c - last) <= 2 * rtol * sc + 1e-30
    return f


@pytest.mark.parametrize("dtype,coarse_rtol", [("f32", 1e-5), ("f16", 2e-3), ("bf16", 8e-3)])
def test_approximate_search_matches_alg4(sindi, small, dtype, coarse_rtol):
    corpus, queries = small
    alpha, beta, gamma, k = 0.5, 0.8, 100, 10
    idx = sindi.Index(corpus, alpha=alpha, window=WINDOW, value_dtype=dtype, tile=TILE)
    ids, sc = idx.search(queries, k, beta=beta, gamma=gamma, cand_cap=2048)
    ids, sc = _np(ids), _np(sc)
    keep = oracle.mass_prune(corpus, alpha)
    ref = oracle.build_index(corpus, WINDOW, keep)
    rid, rsc, pid, psc = oracle.approx_search(ref, corpus, queries, beta, gamma, k, want_pool=True)
    check_ranked(ids, sc)
    check_scores(corpus, queries, ids, sc, rtol=1e-5)  # FP32 rerank from unpruned rows
    cp = oracle.apply_mask(corpus, keep)
    qp = oracle.apply_mask(queries, oracle.mass_prune(queries, beta))
    check_same_topk(ids, rid, rsc, _tol_kth(corpus, queries, rid, rsc, 1e-5),
                    pool_margin=_pool_margin(pid, psc, cp, qp, coarse_rtol))


@pytest.mark.parametrize("dtype,rtol", [("f32", 1e-5), ("f16", 2e-3)])
def test_coarse_search_matches_alg2(sindi, small, dtype, rtol):
    corpus, queries = small
    alpha, k = 0.5, 50
    idx = sindi.Index(corpus, alpha=alpha, window=WINDOW, value_dtype=dtype, tile=TILE)
    ids, sc = idx.search_coarse(queries, k)
    ids, sc = _np(ids), _np(sc)
    keep = oracle.mass_prune(corpus, alpha)
    cp = oracle.apply_mask(corpus, keep)
    rid, rsc = oracle.precise_search(oracle.build_index(corpus, WINDOW, keep), queries, k)
    check_ranked(ids, sc)
    check_scores(cp, queries, ids, sc, rtol=rtol)
    check_same_topk(ids, rid, rsc, _tol_kth(cp, queries, rid, rsc, rtol))


def test_threshold_paths_agree(sindi, small):
    """Keep-all, sampled threshold and the forced retry give bit-identical results."""
    corpus, queries = small
    idx = sindi.Index(corpus, alpha=0.5, window=WINDOW, tile=TILE)
    base_ids, base_sc = map(_np, idx.search(queries, 20, gamma=200, sample_tiles=-1))
    for kw in ({"cand_cap": 4096}, {"cand_cap": 4096, "sample_tiles": 3}, {"cand_cap": 200},
               {"cand_cap": 4096, "batch": 1}):
        ids, sc = map(_np, idx.search(queries, 20, gamma=200, **kw))
        assert (ids == base_ids).all(), kw
        assert sc.tobytes() == base_sc.tobytes(), kw


@pytest.mark.parametrize("batch", [1, 2, 4, 8])
def test_batch_size_does_not_change_results(sindi, small, batch):
    """Coarse sums are integer (order free), so results are bit-identical for any batch."""
    corpus, queries = small
    idx = sindi.Index(corpus, alpha=0.5, window=WINDOW, tile=TILE)
    a_ids, a_sc = map(_np, idx.search(queries, 10, gamma=100, batch=1))
    ids, sc = map(_np, idx.search(queries, 10, gamma=100, batch=batch))
    assert (ids == a_ids).all() and sc.tobytes() == a_sc.tobytes()
    c_ids, c_sc = map(_np, idx.search_coarse(queries, 30, batch=batch))
    r_ids, r_sc = map(_np, idx.search_coarse(queries, 30, batch=1))
    assert (c_ids == r_ids).all() and c_sc.tobytes() == r_sc.tobytes()


@pytest.mark.parametrize("batch", [1, 8])
def test_long_query_in_the_call_does_not_change_results(sindi, small, batch):
    """A 300-term query beside short ones changes nothing: one query per workgroup lays out
    its terms 64 per segment (five segments for the long query), and a batch of 8 sizes its
    LDS (terms merged per pass) from the longest query of the call (64 per pass for short
    queries alone, 512 and several passes beside the long one).  Results are bit-identical,
    and the long query's own results match its search alone."""
    corpus, queries = small
    idx = sindi.Index(corpus, alpha=0.5, window=WINDOW, tile=TILE)
    long_q = synth.generate(1, VOCAB, nnz=("poisson", 300.0), clip=(300, 300), seed=12, stream=2)
    assert long_q.nnz == 300
    both = synth.Csr(np.concatenate([queries.indptr, queries.indptr[-1] + long_q.indptr[1:]]),
                     np.concatenate([queries.indices, long_q.indices]),
                     np.concatenate([queries.values, long_q.values]), VOCAB)
    a_ids, a_sc = map(_np, idx.search(queries, 10, gamma=100, batch=batch))
    b_ids, b_sc = map(_np, idx.search(both, 10, gamma=100, batch=batch))
    n = queries.n_rows
    assert (b_ids[:n] == a_ids).all() and b_sc[:n].tobytes() == a_sc.tobytes()
    l_ids, l_sc = map(_np, idx.search(long_q, 10, gamma=100, batch=batch))
    assert (b_ids[n] == l_ids[0]).all() and b_sc[n].tobytes() == l_sc[0].tobytes()
    c_ids, c_sc = map(_np, idx.search_coarse(both, 30, batch=batch))
    r_ids, r_sc = map(_np, idx.search_coarse(queries, 30, batch=batch))
    assert (c_ids[:n] == r_ids).all() and c_sc[:n].tobytes() == r_sc.tobytes()
    # the long query against the oracle's Alg. 4 on the same index
    keep = oracle.mass_prune(corpus, 0.5)
    oidx = oracle.build_index(corpus, WINDOW, keep)
    o_ids, o_sc, pid, psc = oracle.approx_search(oidx, corpus, long_q, 1.0, 100, 10, want_pool=True)
    check_same_topk(l_ids, o_ids, o_sc, _tol_kth(corpus, long_q, o_ids, o_sc, 1e-5),
                    pool_margin=_pool_margin(pid, psc, oracle.apply_mask(corpus, keep), long_q, 1e-5))


def test_tile_runs_past_the_run_table(sindi):
    """One workgroup sweeping a run of more than 64 tiles reloads its table of tile
    constants mid-run; short queries (one segment of lists) and queries of over 64 terms
    (several segments) give bit-identical results for every tile run, and match the
    oracle's Alg. 4 on the same index.  (4,096 queries: the launch keeps a requested run
    only while the grid still has 4,096 workgroups.)"""
    vocab, window = 1_000, 1_000
    corpus = synth.generate(20_000, vocab, nnz=("poisson", 30.0), seed=21)
    short = synth.generate(4_092, vocab, nnz=("poisson", 20.0), seed=21, stream=1)
    long_q = synth.generate(4, vocab, nnz=("poisson", 150.0), clip=(100, 200), seed=21, stream=2)
    queries = synth.Csr(np.concatenate([short.indptr, short.indptr[-1] + long_q.indptr[1:]]),
                        np.concatenate([short.indices, long_q.indices]),
                        np.concatenate([short.values, long_q.values]), vocab)
    idx = sindi.Index(corpus, alpha=0.5, window=window, tile=256)
    assert idx.info()["n_tiles"] == 80
    r_ids, r_sc = map(_np, idx.search(queries, 10, gamma=100, tile_run=1))
    c_ids, c_sc = map(_np, idx.search_coarse(queries, 30, tile_run=1))
    for run in (16, 65, 80, 1_000):
        ids, sc = map(_np, idx.search(queries, 10, gamma=100, tile_run=run))
        assert (ids == r_ids).all() and sc.tobytes() == r_sc.tobytes(), run
        ids, sc = map(_np, idx.search_coarse(queries, 30, tile_run=run))
        assert (ids == c_ids).all() and sc.tobytes() == c_sc.tobytes(), run
    rows = list(range(0, 4_092, 256)) + [4_092, 4_093, 4_094, 4_095]
    sub = queries.take_rows(rows)
    keep = oracle.mass_prune(corpus, 0.5)
    oidx = oracle.build_index(corpus, window, keep)
    o_ids, o_sc, pid, psc = oracle.approx_search(oidx, corpus, sub, 1.0, 100, 10, want_pool=True)
    check_same_topk(r_ids[rows], o_ids, o_sc, _tol_kth(corpus, sub, o_ids, o_sc, 1e-5),
                    pool_margin=_pool_margin(pid, psc, oracle.apply_mask(corpus, keep), sub, 1e-5))


def test_tile_size_and_query_mix_do_not_change_results(sindi, small):
    """Sec. 3.3.1: the window split only reorders the scan; here tiles are bit-invariant,
    and a query's result does not depend on which queries share its batch."""
    corpus, queries = small
    a = sindi.Index(corpus, alpha=0.5, window=WINDOW, tile=TILE)
    b = sindi.Index(corpus, alpha=0.5, window=WINDOW, tile=700)
    a_ids, a_sc = map(_np, a.search(queries, 10, gamma=100))
    b_ids, b_sc = map(_np, b.search(queries, 10, gamma=100))
    assert (a_ids == b_ids).all() and a_sc.tobytes() == b_sc.tobytes()
    for r in (0, 5, 63):
        one = queries.take_rows([r])
        o_ids, o_sc = map(_np, a.search(one, 10, gamma=100, batch=8))
        assert (o_ids[0] == a_ids[r]).all() and o_sc[0].tobytes() == a_sc[r].tobytes()


def test_device_resident_queries_match_host_queries(sindi, small):
    corpus, queries = small
    idx = sindi.Index(corpus, alpha=0.5, window=WINDOW, tile=TILE)
    h_ids, h_sc = map(_np, idx.search(queries, 10, gamma=100))
    d_ids, d_sc = map(_np, idx.search(sindi.DeviceCsr.from_host(queries), 10, gamma=100))
    assert (h_ids == d_ids).all() and h_sc.tobytes() == d_sc.tobytes()


# ------------------------------------------------------------------ edge cases
def test_empty_and_zero_queries_return_lowest_ids(sindi):
    corpus = synth.generate(3_000, 500, nnz=("poisson", 10.0), seed=3)
    q = synth.Csr(np.array([0, 0, 2, 3], np.int64), np.array([4, 9, 499], np.int32),
                  np.array([0.0, 0.0, 1.0], np.float32), 500)
    idx = sindi.Index(corpus, alpha=0.5, window=1_000, tile=300)
    ids, sc = map(_np, idx.search(q, 5, gamma=20))
    for r in (0, 1):
        assert ids[r].tolist() == [0, 1, 2, 3, 4] and (sc[r] == 0).all()
    ref_ids, ref_sc = oracle.exact_topk(corpus, q, 5)
    check_scores(corpus, q, ids, sc, rtol=1e-5)


def test_k_larger_than_corpus_pads(sindi):
    corpus = synth.generate(5, 50, nnz=("poisson", 5.0), seed=4)
    q = synth.generate(3, 50, nnz=("poisson", 5.0), seed=4, stream=1)
    idx = sindi.Index(corpus, alpha=1.0, window=2)
    ids, sc = map(_np, idx.search(q, 8, gamma=8))
    ref_ids, ref_sc = oracle.exact_topk(corpus, q, 8)
    assert (ids[:, 5:] == -1).all() and np.isneginf(sc[:, 5:]).all()
    check_ranked(ids, sc)
    check_same_topk(ids, ref_ids, ref_sc, np.full(3, 1e-5))


def test_window_of_one_document(sindi):
    corpus = synth.generate(700, 80, nnz=("poisson", 6.0), seed=5)
    q = synth.generate(10, 80, nnz=("poisson", 4.0), seed=5, stream=1)
    idx = sindi.Index(corpus, alpha=1.0, window=1)
    assert idx.info()["n_tiles"] == 700
    ids, sc = map(_np, idx.search(q, 6, gamma=6))
    ref_ids, ref_sc = oracle.exact_topk(corpus, q, 6)
    check_same_topk(ids, ref_ids, ref_sc, _tol_kth(corpus, q, ref_ids, ref_sc, 1e-5))


def test_explicit_zeros_are_absent_entries(sindi):
    corpus = synth.generate(2_000, 300, nnz=("poisson", 20.0), seed=6)
    z = corpus.values.copy()
    z[::7] = 0.0
    cz = synth.Csr(corpus.indptr, corpus.indices, z, 300)
    q = synth.generate(20, 300, nnz=("poisson", 8.0), seed=6, stream=1)
    idx = sindi.Index(cz, alpha=0.6, window=500, tile=256)
    ids, sc = map(_np, idx.search(q, 10, gamma=60))
    nz = cz.values != 0
    stripped = oracle.apply_mask(cz, nz.astype(np.uint8))
    keep_s = oracle.mass_prune(stripped, 0.6)
    ref = oracle.build_index(stripped, 500, keep_s)
    rid, rsc = oracle.approx_search(ref, stripped, q, 1.0, 60, 10)
    check_scores(stripped, q, ids, sc, rtol=1e-5)
    check_same_topk(ids, rid, rsc, _tol_kth(stripped, q, rid, rsc, 1e-5))


def test_invalid_queries_raise_and_leave_outputs(sindi):
    corpus = synth.generate(500, 100, nnz=("poisson", 8.0), seed=7)
    idx = sindi.Index(corpus, alpha=1.0, window=500)
    bad = synth.Csr(np.array([0, 2], np.int64), np.array([5, 3], np.int32),
                    np.array([1.0, 1.0], np.float32), 100)
    out = (torch.full((1, 4), 7, dtype=torch.int64, device="cuda"),
           torch.full((1, 4), 7.0, device="cuda"))
    with pytest.raises(sindi.SindiError, match="ascending"):
        idx.search(bad, 4, gamma=4, out=out)
    with pytest.raises(sindi.SindiError, match="malformed"):
        idx.search(sindi.DeviceCsr.from_host(bad), 4, gamma=4, out=out)
    assert (out[0] == 7).all() and (out[1] == 7.0).all()
    wrong_cols = synth.Csr(np.array([0, 1], np.int64), np.array([1], np.int32),
                           np.array([1.0], np.float32), 99)
    with pytest.raises(sindi.SindiError, match="columns"):
        idx.search(wrong_cols, 4)
    with pytest.raises(sindi.SindiError, match="gamma"):
        idx.search(bad, 10, gamma=5)


# ------------------------------------------------------------------ pair scores and gradients
def test_score_forward_backward_against_oracle(sindi):
    corpus = synth.generate(4_000, 3_000, nnz=("poisson", 60.0), seed=8)
    queries = synth.generate(16, 3_000, nnz=("poisson", 20.0), seed=8, stream=1)
    idx = sindi.Index(corpus, alpha=1.0, window=4_000)
    rng = np.random.default_rng(8)
    cand = np.stack([rng.choice(4_000, size=25, replace=False) for _ in range(16)]).astype(np.int64)
    cand[0, 3] = -1
    dq = sindi.DeviceCsr.from_host(queries)
    s = _np(idx.score(dq, torch.from_numpy(cand).cuda()))
    qrows = np.repeat(np.arange(16), 25)
    exact = oracle.pair_scores(corpus, queries, qrows, cand.reshape(-1)).reshape(16, 25)
    exact[0, 3] = 0.0
    np.testing.assert_allclose(s, exact, rtol=1e-5, atol=1e-6)
    G = rng.standard_normal((16, 25))
    gq = torch.zeros(queries.nnz, device="cuda")
    gx = torch.zeros(corpus.nnz, device="cuda")
    idx.score_backward(dq, torch.from_numpy(cand).cuda(), torch.from_numpy(G).float().cuda(), gq, gx)
    rq, rx = oracle.score_grad(corpus, queries, cand, G.astype(np.float32).astype(np.float64))
    np.testing.assert_allclose(_np(gq), rq, rtol=1e-5, atol=1e-5 * np.abs(rq).max())
    np.testing.assert_allclose(_np(gx), rx, rtol=1e-5, atol=1e-5 * np.abs(rx).max())


@pytest.mark.parametrize("signed", [False, True])
def test_queries_touching_fewer_documents_than_gamma(sindi, signed):
    """Most documents score exactly 0 (the query's terms are rare): the pool is every
    nonzero document, then zero-score documents by ascending id (Alg. 2 keeps filling its
    heap with zero distances), as in the oracle."""
    rng = np.random.default_rng(31 + signed)
    n, vocab = 20_000, 4_000
    corpus = synth.random_csr(rng, n, vocab, 12, signed=signed, min_nnz=1)
    # queries over the rarest terms: few documents share any of them
    cnt = np.bincount(corpus.indices, minlength=vocab)
    rare = np.argsort(cnt, kind="stable")[:200]
    rows = []
    for b in range(24):
        t = np.sort(rng.choice(rare, size=1 + b % 3, replace=False))
        v = rng.lognormal(0.0, 0.8, size=t.size) * (rng.choice([-1.0, 1.0], size=t.size) if signed else 1.0)
        rows.append(dict(zip(t.tolist(), v.astype(np.float32).tolist())))
    queries = csr_from_dict_rows(dict(enumerate(rows)), len(rows), vocab)
    idx = sindi.Index(corpus, alpha=0.7, window=5_000, tile=1_000)
    gamma, k = 300, 40
    ids, sc = idx.search(queries, k, gamma=gamma, cand_cap=1_000)
    ids, sc = _np(ids), _np(sc)
    keep = oracle.mass_prune(corpus, 0.7)
    ref = oracle.build_index(corpus, 5_000, keep)
    rid, rsc = oracle.approx_search(ref, corpus, queries, 1.0, gamma, k)
    check_ranked(ids, sc)
    check_scores(corpus, queries, ids, sc, rtol=1e-5)
    assert np.array_equal(ids, rid)



@pytest.mark.parametrize("prune,kw", [("vnp", dict(vn=20)), ("lp", dict(list_len=300)),
                                      ("mrp+lp", dict(alpha=0.5, list_len=200))])
def test_pruning_rules_layout_and_search(sindi, small, prune, kw):
    """VNP, LP and MRP-then-LP (Sec. 4.1): the lists hold exactly the oracle's kept entries
    (Alg. 1 order, values bit-exact) and the search matches the oracle's Alg. 4 over them."""
    corpus, queries = small
    idx = sindi.Index(corpus, window=WINDOW, tile=TILE, prune=prune, **kw)
    if prune == "vnp":
        keep = oracle.vnp_prune(corpus, kw["vn"])
    elif prune == "lp":
        keep = oracle.lp_prune(corpus, kw["list_len"])
    else:
        keep = oracle.lp_prune(corpus, kw["list_len"], keep_in=oracle.mass_prune(corpus, kw["alpha"]))
    info = idx.info()
    assert info["n_postings"] == int(keep.sum()) and info["prune"] == sindi._lib.PRUNE[prune]
    ex = idx.export()
    ref = oracle.build_index(corpus, WINDOW, keep)
    tile_doc, tile_post, term_off = ex["tile_doc"], ex["tile_post"], ex["term_off"]
    nt = tile_doc.shape[0] - 1
    tile_of = np.repeat(np.arange(nt), np.diff(tile_post))
    term_of = np.concatenate([np.repeat(np.arange(VOCAB), np.diff(term_off[t])) for t in range(nt)])
    doc = ex["post_doc"].astype(np.int64) + tile_doc[tile_of]
    order = np.lexsort((doc, doc // WINDOW, term_of))
    assert (doc[order] == ref.doc.astype(np.int64)).all()
    assert (term_of[order] == np.repeat(np.arange(VOCAB), np.diff(ref.ptr[::ref.sigma]))).all()
    assert ex["post_val"][order].view(np.uint32).tolist() == ref.val.view(np.uint32).tolist()
    gamma, k = 200, 20
    ids, sc = idx.search(queries, k, gamma=gamma)
    ids, sc = _np(ids), _np(sc)
    rid, rsc, pid, psc = oracle.approx_search(ref, corpus, queries, 1.0, gamma, k, want_pool=True)
    check_ranked(ids, sc)
    check_scores(corpus, queries, ids, sc, rtol=1e-5)
    cp = oracle.apply_mask(corpus, keep)
    check_same_topk(ids, rid, rsc, _tol_kth(corpus, queries, rid, rsc, 1e-5),
                    pool_margin=pool_margin_fn(pid, psc, cp, queries, 1e-5))


def test_negative_sums_below_a_zero_threshold(sindi):
    """Signed data where fewer than gamma documents score above 0 (the sampled threshold
    is 0): the lowest-id documents score below 0 and must rank after every zero-score
    document (Alg. 2's heap orders by score before id), both in the coarse top-k (Alg. 2,
    k = gamma) and in Alg. 4's pool (k = gamma), as the oracle computes them."""
    rng = np.random.default_rng(41)
    n, vocab, planted = 40_000, 2_000, 1_999
    base = synth.random_csr(rng, n, vocab - 1, 8, signed=True, min_nnz=1)
    # documents 0..59 also hold the last term, with a negative value (appended at each
    # row's end keeps the term ids ascending)
    at = base.indptr[1:61]
    indptr = base.indptr + np.minimum(np.arange(n + 1), 60)
    corpus = synth.Csr(indptr, np.insert(base.indices, at, planted),
                       np.insert(base.values, at, -(0.5 + rng.random(60)).astype(np.float32)),
                       vocab)
    cnt = np.bincount(base.indices, minlength=vocab)
    rare = np.argsort(cnt[:vocab - 1], kind="stable")[:100]
    qrows = []
    for b in range(12):
        t = np.sort(rng.choice(rare, size=1 + b % 2, replace=False))
        d = dict(zip(t.tolist(), rng.lognormal(0.0, 0.8, size=t.size).astype(np.float32).tolist()))
        d[planted] = 1.0
        qrows.append(d)
    queries = csr_from_dict_rows(dict(enumerate(qrows)), len(qrows), vocab)
    idx = sindi.Index(corpus, alpha=1.0, window=10_000, tile=2_000)
    ref = oracle.build_index(corpus, 10_000)
    for gamma in (100, 300):
        cid, csc = map(_np, idx.search_coarse(queries, gamma, cand_cap=1_000))
        rid, rsc = oracle.precise_search(ref, queries, gamma)
        assert np.array_equal(cid, rid), gamma
        # the zero-score documents start right after the planted negatives
        for r in range(queries.n_rows):
            z = cid[r][csc[r] == 0]
            assert z.size and z[0] >= 60 and not np.isin(z, np.arange(60)).any()
        ids, sc = map(_np, idx.search(queries, gamma, gamma=gamma, cand_cap=1_000))
        oid, osc = oracle.approx_search(ref, corpus, queries, 1.0, gamma, gamma)
        check_ranked(ids, sc)
        check_scores(corpus, queries, ids, sc, rtol=1e-5)
        assert np.array_equal(ids, oid), gamma


def test_every_retry_stage_gives_the_keep_all_result(sindi, small):
    """A query whose sampled threshold misses is re-run with a threshold over every tile
    (rank gamma), and, if that overflows the candidate buffer, with none.  Forced here: the
    documents of the first tile (the only one sampled) score four times higher than the
    rest, so the sampled threshold keeps fewer than gamma documents for every query; with a
    buffer of 4,096 the pass over every tile then resolves every query, with a buffer of
    gamma it overflows and the keep-all pass follows.  The kernel timing counts the passes.
    Results are bit-identical to keeping every document from the start."""
    corpus, queries = small
    vals = corpus.values.copy()
    first_tile = WINDOW // -(-WINDOW // TILE)  # windows split into equal tiles
    vals[:corpus.indptr[first_tile]] *= 4.0
    skewed = synth.Csr(corpus.indptr, corpus.indices, vals, corpus.n_cols)
    idx = sindi.Index(skewed, alpha=0.5, window=WINDOW, tile=TILE)
    assert idx.export(raw=True)["tile_doc"][1] == first_tile
    base_ids, base_sc = map(_np, idx.search(queries, 20, gamma=200, sample_tiles=-1))
    sindi.profile_enable(True)
    try:
        for cap, stages in ((4_096, 2), (200, 3)):
            sindi.profile_read(reset=True)
            ids, sc = map(_np, idx.search(queries, 20, gamma=200, sample_tiles=1, cand_cap=cap))
            prof = sindi.profile_read(reset=True)
            assert (ids == base_ids).all(), cap
            assert sc.tobytes() == base_sc.tobytes(), cap
            # threshold passes: the sampled one and the one over every tile; scoring
            # passes: one per stage that ran
            assert prof["accumulate_threshold"][0] == 2, (cap, prof)
            assert prof["accumulate_score"][0] == stages, (cap, prof)
    finally:
        sindi.profile_enable(False)


def test_scores_of_passed_document_values(sindi):
    """score / score_backward with doc_values: the document values passed are scored, not the
    index's build-time copy (doubling them doubles every score exactly), and the gradients
    follow them, against the oracle on the changed corpus."""
    corpus = synth.generate(3_000, 1_500, nnz=("poisson", 40.0), seed=9)
    queries = synth.generate(12, 1_500, nnz=("poisson", 15.0), seed=9, stream=1)
    idx = sindi.Index(corpus, alpha=0.5, window=3_000)
    rng = np.random.default_rng(9)
    cand = torch.from_numpy(np.stack([rng.choice(3_000, 30, replace=False)
                                      for _ in range(12)]).astype(np.int64)).cuda()
    dq = sindi.DeviceCsr.from_host(queries)
    xv = torch.from_numpy(corpus.values.copy()).cuda()
    s1 = idx.score(dq, cand)
    s2 = idx.score(dq, cand, doc_values=2 * xv)
    assert torch.equal(s2, 2 * s1)
    new_vals = (corpus.values * rng.uniform(0.5, 1.5, corpus.nnz)).astype(np.float32)
    changed = synth.Csr(corpus.indptr, corpus.indices, new_vals, corpus.n_cols)
    s3 = _np(idx.score(dq, cand, doc_values=torch.from_numpy(new_vals).cuda()))
    c = _np(cand)
    exact = oracle.pair_scores(changed, queries, np.repeat(np.arange(12), 30), c.reshape(-1))
    np.testing.assert_allclose(s3.reshape(-1), exact, rtol=1e-5, atol=1e-6)
    G = rng.standard_normal((12, 30)).astype(np.float32)
    gq = torch.zeros(queries.nnz, device="cuda")
    gx = torch.zeros(corpus.nnz, device="cuda")
    idx.score_backward(dq, cand, torch.from_numpy(G).cuda(), gq, gx,
                       doc_values=torch.from_numpy(new_vals).cuda())
    rq, rx = oracle.score_grad(changed, queries, c, G.astype(np.float64))
    np.testing.assert_allclose(_np(gq), rq, rtol=1e-5, atol=1e-5 * np.abs(rq).max())
    np.testing.assert_allclose(_np(gx), rx, rtol=1e-5, atol=1e-5 * np.abs(rx).max())
    # shapes the kernels would index past are refused before any device work
    E = sindi.SindiError
    with pytest.raises(E, match="doc_values"):
        idx.score(dq, cand, doc_values=xv[:-1])
    with pytest.raises(E, match="cand"):
        idx.score(dq, cand[:5])
    with pytest.raises(E, match="cand"):
        idx.score(dq, cand.int())
    with pytest.raises(E, match="grad"):
        idx.score_backward(dq, cand, torch.zeros(12, 29, device="cuda"), gq, gx)
    with pytest.raises(E, match="grad_query"):
        idx.score_backward(dq, cand, torch.from_numpy(G).cuda(), gq[:-1], gx)
    with pytest.raises(E, match="grad_doc"):
        idx.score_backward(dq, cand, torch.from_numpy(G).cuda(), gq, gx.double())


@pytest.mark.parametrize("kw", [dict(), dict(sample_tiles=1, cand_cap=200),
                                dict(sample_tiles=-1), dict(tile_run=1), dict(tile_run=65)])
def test_persistent_queue_schedule_is_bit_identical(sindi, small, kw):
    """The scoring passes as one persistent launch fed by a device work queue (schedule 2)
    give exactly the results of one workgroup per (query, tile run) (schedule 1): the same
    items run, in any order, and integer sums do not depend on it.  Also with every retry
    stage forced, with no threshold, and with runs of 1 and of more than 64 tiles."""
    corpus, queries = small
    idx = sindi.Index(corpus, alpha=0.5, window=WINDOW, tile=TILE)
    for fn, k, extra in ((idx.search, 20, dict(gamma=200)), (idx.search_coarse, 30, dict())):
        a_ids, a_sc = map(_np, fn(queries, k, schedule=1, **extra, **kw))
        b_ids, b_sc = map(_np, fn(queries, k, schedule=2, **extra, **kw))
        assert (a_ids == b_ids).all() and a_sc.tobytes() == b_sc.tobytes()


def test_largest_pool_longest_query_and_largest_tile(sindi):
    """The limits the interface states, at once: gamma = k = 4096 (the largest pool), a query
    of 4,096 terms (the longest the rerank's query table holds; 64 register segments per
    scoring wave) beside short ones, and tiles of 16,384 documents (the largest; two
    workgroups per CU) with a ragged last window and tile: Alg. 4 of the oracle on the same
    index, and one term more is refused."""
    vocab = 6_000
    corpus = synth.generate(40_003, vocab, nnz=("poisson", 30.0), seed=23)
    short = synth.generate(6, vocab, nnz=("poisson", 20.0), seed=23, stream=1)
    rng = np.random.default_rng(23)
    long_ids = np.sort(rng.choice(vocab, size=4_096, replace=False)).astype(np.int32)
    long_vals = rng.lognormal(0.0, 0.8, size=4_096).astype(np.float32)
    q = synth.Csr(np.concatenate([short.indptr, [short.indptr[-1] + 4_096]]).astype(np.int64),
                  np.concatenate([short.indices, long_ids]),
                  np.concatenate([short.values, long_vals]), vocab)
    alpha, gamma, k, window = 0.6, 4_096, 4_096, 32_768
    idx = sindi.Index(corpus, alpha=alpha, window=window, tile=16_384)
    assert idx.info()["tile_max"] == 16_384  # two tiles per window, then a ragged window of 7,235
    ids, sc = map(_np, idx.search(q, k, gamma=gamma))
    keep = oracle.mass_prune(corpus, alpha)
    ref = oracle.build_index(corpus, window, keep)
    rid, rsc, pid, psc = oracle.approx_search(ref, corpus, q, 1.0, gamma, k, want_pool=True)
    check_ranked(ids, sc)
    check_scores(corpus, q, ids, sc, rtol=1e-5)
    check_same_topk(ids, rid, rsc, _tol_kth(corpus, q, rid, rsc, 1e-5),
                    pool_margin=_pool_margin(pid, psc, oracle.apply_mask(corpus, keep), q, 1e-5))
    too_long = synth.Csr(np.array([0, 4_097], np.int64),
                         np.sort(rng.choice(vocab, size=4_097, replace=False)).astype(np.int32),
                         np.ones(4_097, np.float32), vocab)
    with pytest.raises(sindi.SindiError, match="4096"):
        idx.search(too_long, 10)
    with pytest.raises(sindi.SindiError, match="gamma"):
        idx.search(short, 10, gamma=4_097)
