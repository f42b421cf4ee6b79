"""Parity at the benchmark sizes, in the launch configuration bench.py times.

The 1M-document pruned workload is checked on every query; the 8.8M-document workload
(FP16, FP32 and BF16 postings, and the request loop over the FP16 index) on sampled queries
that the oracle computes one by one.
"""
import numpy as np
import pytest

import oracle
from parity import check_ranked, check_same_topk, check_scores, kth_tolerance, pool_margin_fn
from synth.workloads import WORKLOADS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sindi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_08395_amd as s
    s._lib.load()
    return s


def _np(t):
    return t.detach().cpu().numpy()


def _run(sindi, wl, corpus, queries, dtype):
    idx = sindi.Index(corpus, alpha=wl.alpha, window=wl.window, value_dtype=dtype)
    ids, sc = idx.search(sindi.DeviceCsr.from_host(queries), wl.k, beta=wl.beta, gamma=wl.gamma)
    return idx, _np(ids), _np(sc)


def test_pruned_1m_every_query(sindi):
    wl = WORKLOADS["pruned-1m"]
    corpus, queries = wl.corpus(), wl.queries()
    idx, ids, sc = _run(sindi, wl, corpus, queries, wl.value_dtype)
    keep = oracle.mass_prune(corpus, wl.alpha)
    ref = oracle.build_index(corpus, wl.window, keep)
    rid, rsc, pid, psc = oracle.approx_search(ref, corpus, queries, wl.beta, wl.gamma, wl.k,
                                              want_pool=True)
    check_ranked(ids, sc)
    check_scores(corpus, queries, ids, sc, rtol=1e-5)
    cp = oracle.apply_mask(corpus, keep)
    check_same_topk(ids, rid, rsc, kth_tolerance(corpus, queries, rid, 1e-5),
                    pool_margin=pool_margin_fn(pid, psc, cp, queries, 1e-5))
    truth, _ = oracle.exact_topk(corpus, queries.take_rows(np.arange(0, 1000, 10)), wl.k)
    assert oracle.recall_at_k(ids[::10], truth) >= 0.99


@pytest.fixture(scope="module")
def splade(sindi):
    """The 8.8M-document corpus and its 7,000 queries, the oracle's Alg. 3 keep mask and
    Alg. 1 index, and the pruned corpus (coarse scores are its inner products)."""
    wl = WORKLOADS["splade-8.8m"]
    corpus, queries = wl.corpus(), wl.queries()
    keep = oracle.mass_prune(corpus, wl.alpha)
    ref = oracle.build_index(corpus, wl.window, keep)
    cp = oracle.apply_mask(corpus, keep)
    del keep
    return wl, corpus, queries, ref, cp


@pytest.fixture(scope="module")
def splade_f16(sindi, splade):
    """The FP16 index bench.py times (host build), shared by the tests below."""
    wl, corpus, _, _, _ = splade
    return sindi.Index(corpus, alpha=wl.alpha, window=wl.window, value_dtype="f16")


# FP16 and BF16 round posting values (bound 2^-11 and 2^-8 relative); FP32 keeps them.
@pytest.mark.parametrize("dtype,coarse_rtol,n_sel", [("f16", 2e-3, 48), ("f32", 1e-5, 24),
                                                     ("bf16", 8e-3, 24)])
def test_splade_8_8m_sampled_queries(sindi, splade, splade_f16, dtype, coarse_rtol, n_sel):
    """All 7,000 queries searched in one call (the bench configuration), checked on evenly
    spaced queries against the oracle's Alg. 4 (near-ties at the pool boundary only within
    the storage type's coarse tolerance), every returned score against the exact FP64 inner
    product, and Recall@50 against the exact top-50."""
    wl, corpus, queries, ref, cp = splade
    if dtype == "f16":
        idx = splade_f16
    else:  # the device build (bit-identical to the host build, checked against the oracle)
        idx = sindi.Index(corpus, alpha=wl.alpha, window=wl.window, value_dtype=dtype,
                          gpu_build=True)
    ids, sc = idx.search(sindi.DeviceCsr.from_host(queries), wl.k, beta=wl.beta, gamma=wl.gamma)
    ids, sc = _np(ids), _np(sc)
    if dtype != "f16":
        idx.close()
    check_ranked(ids, sc)
    sel = np.linspace(0, wl.n_queries - 1, n_sel).astype(np.int64)
    qs = queries.take_rows(sel)
    gi, gs = ids[sel], sc[sel]
    check_scores(corpus, qs, gi, gs, rtol=1e-5)  # FP32 rerank from the FP32 unpruned rows
    rid, rsc, pid, psc = oracle.approx_search(ref, corpus, qs, wl.beta, wl.gamma, wl.k,
                                              want_pool=True)
    check_same_topk(gi, rid, rsc, kth_tolerance(corpus, qs, rid, 1e-5),
                    pool_margin=pool_margin_fn(pid, psc, cp, qs, coarse_rtol))
    truth, _ = oracle.exact_topk(corpus, qs.take_rows(np.arange(0, n_sel, 3)), wl.k)
    assert oracle.recall_at_k(gi[::3], truth) >= 0.99


def test_serving_on_the_8_8m_index(sindi, splade, splade_f16):
    """The request loop over the 8.8M-document FP16 index: serving-shaped requests (5 to
    200 terms, k in {10, 50, 100}) submitted together return exactly what a search of the
    same query alone returns, and agree with the oracle's Alg. 4."""
    wl, corpus, _, ref, cp = splade
    sw = WORKLOADS["serving"]
    n = 40
    q = sw.queries(n, row0=123_456)
    ks = sw.request_ks(n, row0=123_456)
    with sindi.Server(splade_f16, max_inflight=2, max_batch=16, k_max=100, gamma=sw.gamma) as srv:
        tickets = [srv.submit(*q.row(r), int(ks[r])) for r in range(n)]
        got = [srv.wait(t, int(ks[r])) for r, t in enumerate(tickets)]
        st = srv.stats()
    assert st["completed"] == n and st["batches"] >= 2
    for r in range(n):
        k = int(ks[r])
        a_ids, a_sc = splade_f16.search(q.take_rows([r]), k, gamma=sw.gamma)
        assert np.array_equal(got[r][0], _np(a_ids)[0]), r
        assert got[r][1].tobytes() == _np(a_sc)[0].tobytes(), r
    rows = np.arange(0, n, 4)
    qs = q.take_rows(rows)
    k = 100
    s_ids = np.stack([np.concatenate([got[r][0], np.full(k - len(got[r][0]), -1)]) for r in rows])
    rid, rsc, pid, psc = oracle.approx_search(ref, corpus, qs, 1.0, sw.gamma, k, want_pool=True)
    for i, r in enumerate(rows):
        kr = int(ks[r])
        check_scores(corpus, qs.take_rows([i]), got[r][0][None, :], got[r][1][None, :], rtol=1e-5)
        check_same_topk(s_ids[i:i + 1, :kr], rid[i:i + 1, :kr], rsc[i:i + 1, :kr],
                        kth_tolerance(corpus, qs.take_rows([i]), rid[i:i + 1, :kr], 1e-5),
                        pool_margin=pool_margin_fn(pid[i:i + 1], psc[i:i + 1], cp,
                                                   qs.take_rows([i]), 2e-3))


def test_splade_8_8m_device_build_equals_host_build(sindi, splade, splade_f16):
    """At full size the device build equals the host build bit for bit, and both keep the
    oracle's Alg. 3 entries: the same number of postings per term."""
    import time
    wl, corpus, _, ref, _ = splade
    rh = splade_f16.export(raw=True)
    t = time.time()
    g = sindi.Index(corpus, alpha=wl.alpha, window=wl.window, value_dtype=wl.value_dtype,
                    gpu_build=True)
    tg = time.time() - t
    rg = g.export(raw=True)
    print(f"device build {tg:.2f} s (upload included)")
    for key in ("tile_doc", "tile_post", "term_goff", "post_doc"):
        assert np.array_equal(rh[key], rg[key]), key
    assert np.array_equal(rh["post_val"], rg["post_val"])
    assert g.info()["n_postings"] == ref.doc.shape[0]
    assert np.array_equal(g.term_lengths(), np.diff(ref.ptr[::ref.sigma]))
