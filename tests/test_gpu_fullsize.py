"""Parity at the benchmark sizes, in the launch configuration bench.py times.

The 1M-document pruned workload is checked on every query; the 8.8M-document workload
(FP16 postings) on sampled queries that the oracle computes one by one.
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


@pytest.mark.parametrize("dtype,coarse_rtol", [("f16", 2e-3)])
def test_splade_8_8m_sampled_queries(sindi, dtype, coarse_rtol):
    wl = WORKLOADS["splade-8.8m"]
    corpus, queries = wl.corpus(), wl.queries()
    idx, ids, sc = _run(sindi, wl, corpus, queries, dtype)
    del idx
    check_ranked(ids, sc)
    sel = np.linspace(0, wl.n_queries - 1, 24).astype(np.int64)
    qs = queries.take_rows(sel)
    gi, gs = ids[sel], sc[sel]
    check_scores(corpus, qs, gi, gs, rtol=1e-5)  # FP32 rerank from the FP32 unpruned rows
    keep = oracle.mass_prune(corpus, wl.alpha)
    ref = oracle.build_index(corpus, wl.window, keep)
    rid, rsc, pid, psc = oracle.approx_search(ref, corpus, qs, wl.beta, wl.gamma, wl.k,
                                              want_pool=True)
    del ref
    cp = oracle.apply_mask(corpus, keep)
    del keep
    check_same_topk(gi, rid, rsc, kth_tolerance(corpus, qs, rid, 1e-5),
                    pool_margin=pool_margin_fn(pid, psc, cp, qs, coarse_rtol))
    truth, _ = oracle.exact_topk(corpus, qs.take_rows(np.arange(0, 24, 3)), wl.k)
    assert oracle.recall_at_k(gi[::3], truth) >= 0.99


def test_splade_8_8m_device_build_equals_host_build(sindi):
    import time
    wl = WORKLOADS["splade-8.8m"]
    corpus = wl.corpus()
    t = time.time()
    h = sindi.Index(corpus, alpha=wl.alpha, window=wl.window, value_dtype=wl.value_dtype)
    th = time.time() - t
    rh = h.export(raw=True)
    del h
    t = time.time()
    g = sindi.Index(corpus, alpha=wl.alpha, window=wl.window, value_dtype=wl.value_dtype,
                    gpu_build=True)
    tg = time.time() - t
    rg = g.export(raw=True)
    print(f"host build {th:.2f} s, device build {tg:.2f} s (upload included in both)")
    for key in ("tile_doc", "tile_post", "term_goff", "post_doc"):
        assert np.array_equal(rh[key], rg[key]), key
    assert np.array_equal(rh["post_val"], rg["post_val"])
