"""Differentiation at full size: 1M documents over a 250,002-term vocabulary (~180
non-zeros each), 256 queries (~40 non-zeros), exact top-100 candidates, one planted
positive per query, softmax contrastive loss at temperature 20.

The score of a (query, document) pair is the inner product over common dimensions
(Def. 2), so its gradient has a closed form; the oracle evaluates it in FP64."""
import numpy as np
import pytest

import oracle
from parity import check_ranked, check_scores
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


@pytest.fixture(scope="module")
def setup(sindi):
    wl = WORKLOADS["diff-1m"]
    corpus, queries = wl.corpus(), wl.queries()
    corpus, pos = wl.plant_positives(corpus, queries)
    idx = sindi.Index(corpus, alpha=wl.alpha, window=wl.window)
    ids, sc = idx.search(queries, wl.k, gamma=wl.gamma)
    cand = ids.cpu().numpy()
    # the planted positive takes the last place where the search did not find it
    at = np.argmax(cand == pos[:, None], axis=1)
    found = (cand == pos[:, None]).any(axis=1)
    cand[~found, -1] = pos[~found]
    at[~found] = wl.k - 1
    return wl, corpus, queries, idx, cand, at, ids.cpu().numpy(), sc.cpu().numpy(), found


def test_exact_candidates(sindi, setup):
    """alpha = 1 and gamma = k: the candidates are the exact top-100."""
    wl, corpus, queries, idx, cand, at, ids, sc, found = setup
    check_ranked(ids, sc)
    sel = np.arange(0, queries.n_rows, 8)
    check_scores(corpus, queries.take_rows(sel), ids[sel], sc[sel], rtol=1e-5)
    truth, _ = oracle.exact_topk(corpus, queries.take_rows(sel), wl.k)
    assert oracle.recall_at_k(ids[sel], truth) >= 0.999
    assert found.mean() > 0.5  # planted documents mostly rank in the top 100


def test_backward_kernel_matches_oracle_gradient(sindi, setup):
    wl, corpus, queries, idx, cand, at, ids, sc, found = setup
    tau = wl.extra["tau"]
    qrows = np.repeat(np.arange(queries.n_rows), wl.k)
    exact = oracle.pair_scores(corpus, queries, qrows, cand.reshape(-1)).reshape(cand.shape)
    loss, G = oracle.contrastive_grad(exact, at, tau)
    p = np.exp(exact / tau - (exact / tau).max(axis=1, keepdims=True))
    p /= p.sum(axis=1, keepdims=True)
    assert (-(p * np.log(p + 1e-300)).sum(axis=1)).mean() > 0.5  # the softmax is not saturated
    dq = sindi.DeviceCsr.from_host(queries)
    tc = torch.from_numpy(cand).cuda()
    s = idx.score(dq, tc).cpu().numpy()
    np.testing.assert_allclose(s, exact, rtol=1e-5, atol=1e-6 * np.abs(exact).max())
    G32 = G.astype(np.float32)
    gq = torch.zeros(queries.nnz, device="cuda")
    gx = torch.zeros(corpus.nnz, device="cuda")
    idx.score_backward(dq, tc, torch.from_numpy(G32).cuda(), gq, gx)
    rq, rx = oracle.score_grad(corpus, queries, cand, G32.astype(np.float64))
    gq, gx = gq.cpu().numpy(), gx.cpu().numpy()
    np.testing.assert_allclose(gq, rq, rtol=1e-5, atol=1e-6 * np.abs(rq).max())
    touched = np.nonzero(rx)[0]
    assert touched.size > 0 and not gx[np.setdiff1d(np.arange(0, corpus.nnz, 997), touched)].any()
    np.testing.assert_allclose(gx[touched], rx[touched], rtol=1e-5, atol=1e-6 * np.abs(rx).max())


def test_autograd_loss_and_gradients(sindi, setup):
    """torch.autograd through the HIP forward/backward against the FP64 closed form."""
    wl, corpus, queries, idx, cand, at, ids, sc, found = setup
    tau = wl.extra["tau"]
    qv = torch.from_numpy(queries.values.copy()).cuda().requires_grad_(True)
    xv = torch.from_numpy(corpus.values.copy()).cuda().requires_grad_(True)
    qp = torch.from_numpy(queries.indptr.astype(np.int64)).cuda()
    qi = torch.from_numpy(queries.indices.astype(np.int32)).cuda()
    tc = torch.from_numpy(cand).cuda()
    s = sindi.SindiScore.apply(qv, xv, idx, qp, qi, tc)
    z = s / tau
    rows = torch.arange(queries.n_rows, device="cuda")
    loss = (torch.logsumexp(z, dim=1) - z[rows, torch.from_numpy(at).cuda()]).mean()
    loss.backward()
    qrows = np.repeat(np.arange(queries.n_rows), wl.k)
    exact = oracle.pair_scores(corpus, queries, qrows, cand.reshape(-1)).reshape(cand.shape)
    rloss, G = oracle.contrastive_grad(exact, at, tau)
    assert abs(loss.item() - rloss) <= 1e-5 * max(1.0, abs(rloss))
    rq, rx = oracle.score_grad(corpus, queries, cand, G)
    gq, gx = qv.grad.cpu().numpy(), xv.grad.cpu().numpy()
    # FP32 softmax and scores: relative error ~1e-6 per entry of G
    np.testing.assert_allclose(gq, rq, rtol=1e-4, atol=1e-5 * np.abs(rq).max())
    touched = np.nonzero(rx)[0]
    np.testing.assert_allclose(gx[touched], rx[touched], rtol=1e-4, atol=1e-5 * np.abs(rx).max())


def _loss(scores, pos, tau):
    """Softmax contrastive loss over each query's candidates (FP64), and dL/ds."""
    z = scores.astype(np.float64) / tau
    m = z.max(axis=1, keepdims=True)
    e = np.exp(z - m)
    p = e / e.sum(axis=1, keepdims=True)
    rows = np.arange(z.shape[0])
    loss = float(np.mean(np.log(e.sum(axis=1)) + m[:, 0] - z[rows, pos]))
    G = p.copy()
    G[rows, pos] -= 1.0
    return loss, G / (tau * z.shape[0])


def test_backward_kernel_against_finite_differences_on_the_gpu(sindi, setup):
    """Central differences of the loss through the GPU forward kernel (FP32 scores, loss in
    FP64 on the host), on sampled query and document coordinates, against the GPU backward
    kernel.  Each score is linear in each coordinate and the loss is smooth in the scores, so
    the step h = 1/32 keeps the central difference's curvature error near 1e-4 while the
    rounding of the FP32 scores stays near 5e-4 of the difference (a step of 1e-3 would drown
    in that rounding; the oracle itself is checked with h = 1e-3 in FP64).  Tolerance: 1e-2
    of the gradient plus 1e-4 of the largest one.  Coordinates outside every (query,
    candidate) intersection must have a zero gradient and an exactly zero difference."""
    wl, corpus, queries, idx, cand, at, ids, sc, found = setup
    tau = wl.extra["tau"]
    dq = sindi.DeviceCsr.from_host(queries)
    tc = torch.from_numpy(cand).cuda()
    qv = torch.from_numpy(queries.values.copy()).cuda()
    xv = torch.from_numpy(corpus.values.copy()).cuda()

    def loss_at(qvals, xvals):
        s = idx.score(sindi.DeviceCsr(dq.indptr, dq.indices, qvals, queries.n_cols), tc,
                      doc_values=xvals)
        return _loss(s.cpu().numpy(), at, tau)

    L0, G = loss_at(qv, xv)
    gq = torch.zeros(queries.nnz, device="cuda")
    gx = torch.zeros(corpus.nnz, device="cuda")
    idx.score_backward(dq, tc, torch.from_numpy(G.astype(np.float32)).cuda(), gq, gx,
                       doc_values=xv)
    gq, gx = gq.cpu().numpy(), gx.cpu().numpy()
    rng = np.random.default_rng(77)
    h = 1.0 / 32
    q_nz = np.nonzero(np.abs(gq) > 1e-3 * np.abs(gq).max())[0]
    x_nz = np.nonzero(np.abs(gx) > 1e-3 * np.abs(gx).max())[0]
    # entries of candidate documents that no query shares
    rows_c = np.unique(cand)
    ents = np.concatenate([np.arange(corpus.indptr[d], corpus.indptr[d + 1]) for d in rows_c[:200]])
    x_zero = rng.choice(ents[gx[ents] == 0], 16, replace=False)
    checks = ([("q", e) for e in rng.choice(q_nz, 48, replace=False)] +
              [("x", e) for e in rng.choice(x_nz, 48, replace=False)] +
              [("x", e) for e in x_zero])
    gmax = {"q": np.abs(gq).max(), "x": np.abs(gx).max()}
    for side, e in checks:
        base = qv if side == "q" else xv
        plus, minus = base.clone(), base.clone()
        plus[e] += h
        minus[e] -= h
        if side == "q":
            fd = (loss_at(plus, xv)[0] - loss_at(minus, xv)[0]) / (2 * h)
            g = gq[e]
        else:
            fd = (loss_at(qv, plus)[0] - loss_at(qv, minus)[0]) / (2 * h)
            g = gx[e]
        if g == 0.0:
            assert fd == 0.0, (side, e, fd)
        else:
            assert abs(fd - g) <= 1e-2 * abs(g) + 1e-4 * gmax[side], (side, e, fd, g)


def test_autograd_scores_the_document_values_passed(sindi, setup):
    """SindiScore takes the document values as an input: doubling them doubles every score
    and halves nothing else (the index's build-time copy is not what it scores)."""
    wl, corpus, queries, idx, cand, at, ids, sc, found = setup
    qv = torch.from_numpy(queries.values.copy()).cuda()
    xv = torch.from_numpy(corpus.values.copy()).cuda()
    qp = torch.from_numpy(queries.indptr.astype(np.int64)).cuda()
    qi = torch.from_numpy(queries.indices.astype(np.int32)).cuda()
    tc = torch.from_numpy(cand).cuda()
    s1 = sindi.SindiScore.apply(qv, xv, idx, qp, qi, tc)
    s2 = sindi.SindiScore.apply(qv, 2 * xv, idx, qp, qi, tc)
    assert torch.equal(s2, 2 * s1)
