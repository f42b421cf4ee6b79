"""Second workload shapes at full size: short queries over a 250,000-term vocabulary
(AntSparse shape) and uniform term ids and values (RANDOM shape).  Sampled queries are
checked against the oracle's Alg. 4 (same alpha, beta, gamma) and the exact top-k."""
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


@pytest.mark.parametrize("name,n_sel,coarse_rtol", [("antsparse-1m", 250, 2e-3), ("random-1m", 48, 2e-3)])
def test_shape_against_oracle(sindi, name, n_sel, coarse_rtol):
    wl = WORKLOADS[name]
    corpus, queries = wl.corpus(), wl.queries()
    idx = sindi.Index(corpus, alpha=wl.alpha, window=wl.window, value_dtype=wl.value_dtype)
    ids, sc = idx.search(sindi.DeviceCsr.from_host(queries), wl.k, beta=wl.beta, gamma=wl.gamma)
    ids, sc = ids.cpu().numpy(), sc.cpu().numpy()
    del idx
    check_ranked(ids, sc)
    sel = np.linspace(0, queries.n_rows - 1, n_sel).astype(np.int64)
    qs = queries.take_rows(sel)
    gi, gs = ids[sel], sc[sel]
    check_scores(corpus, qs, gi, gs, rtol=1e-5)  # FP32 rerank of the unpruned rows
    keep = oracle.mass_prune(corpus, wl.alpha)
    ref = oracle.build_index(corpus, wl.window, keep)
    rid, rsc, pid, psc = oracle.approx_search(ref, corpus, qs, wl.beta, wl.gamma, wl.k,
                                              want_pool=True)
    del ref
    cp = oracle.apply_mask(corpus, keep)
    check_same_topk(gi, rid, rsc, kth_tolerance(corpus, qs, rid, 1e-5),
                    pool_margin=pool_margin_fn(pid, psc, cp, qs, coarse_rtol))
    truth, _ = oracle.exact_topk(corpus, qs, wl.k)
    r_gpu, r_ref = oracle.recall_at_k(gi, truth), oracle.recall_at_k(rid, truth)
    print(f"{name}: Recall@{wl.k} GPU {r_gpu:.4f}, oracle Alg. 4 {r_ref:.4f}")
    assert r_gpu >= r_ref - 0.005
