"""Comparison of GPU results with the oracle, tolerant only where several answers are right.

Floating-point ranking has ties within rounding: when two documents' exact
scores differ by less than the FP32 error bound, either may legitimately
take the last place of a top-k (or of the rerank pool).  The comparisons
below accept an id mismatch only when it is explained that way; everything
else must match exactly.
"""
import numpy as np

import oracle
import synth


def abs_csr(c):
    return synth.Csr(c.indptr, c.indices, np.abs(c.values), c.n_cols)


def score_scale(corpus, queries, qrows, docs):
    """sum_t |q_t x_t| per pair: the scale of the FP32 rounding error of delta."""
    return oracle.pair_scores(abs_csr(corpus), abs_csr(queries), qrows, docs)


def check_scores(corpus, queries, ids, scores, rtol):
    """Every returned id's score is delta(x_id, q) within rtol of its error scale."""
    nq, k = ids.shape
    qrows = np.repeat(np.arange(nq), k)
    flat = ids.reshape(-1)
    valid = flat >= 0
    exact = oracle.pair_scores(corpus, queries, qrows[valid], flat[valid])
    scale = score_scale(corpus, queries, qrows[valid], flat[valid])
    got = scores.reshape(-1)[valid].astype(np.float64)
    err = np.abs(got - exact)
    bad = err > rtol * np.maximum(scale, 1e-30)
    assert not bad.any(), (
        f"{bad.sum()} scores off; worst rel {np.max(err / np.maximum(scale, 1e-30)):.3g}")
    assert np.isneginf(scores.reshape(-1)[~valid]).all()
    return exact


def check_ranked(ids, scores):
    """Rows are sorted by (score desc, id asc) with ids unique; padding (-1) at the end."""
    for r in range(ids.shape[0]):
        v = ids[r] >= 0
        n = int(v.sum())
        assert v[:n].all() and not v[n:].any()
        assert len(set(ids[r, :n].tolist())) == n
        s = scores[r, :n]
        i = ids[r, :n]
        assert all((s[t] > s[t + 1]) or (s[t] == s[t + 1] and i[t] < i[t + 1]) for t in range(n - 1))


def check_same_topk(gpu_ids, ref_ids, ref_scores, tol_abs, pool_margin=None):
    """gpu top-k == reference top-k except near-ties.

    A reference id missing from the GPU row is accepted if its reference score is
    within tol_abs[row] of the reference k-th score, or, for the approximate method,
    if pool_margin(row, id) says its coarse score sat at the pool boundary.
    """
    for r in range(ref_ids.shape[0]):
        ref = [int(x) for x in ref_ids[r] if x >= 0]
        got = set(int(x) for x in gpu_ids[r] if x >= 0)
        assert len(got) == len(ref), (r, len(got), len(ref))
        kth = ref_scores[r][len(ref) - 1] if ref else 0.0
        for pos, d in enumerate(ref):
            if d in got:
                continue
            s = ref_scores[r][pos]
            if abs(s - kth) <= tol_abs[r]:
                continue
            if pool_margin is not None and pool_margin(r, d):
                continue
            raise AssertionError(f"row {r}: id {d} (score {s}, kth {kth}) missing from GPU result")


def recall(gpu_ids, truth_ids):
    return oracle.recall_at_k(gpu_ids, truth_ids)


def kth_tolerance(corpus, queries, ref_ids, rtol):
    """Per row: twice the FP32 error scale at the reference's last place."""
    nq = ref_ids.shape[0]
    last = np.array([r[r >= 0][-1] if (r >= 0).any() else 0 for r in ref_ids])
    return 2.0 * rtol * score_scale(corpus, queries, np.arange(nq), last)


def pool_margin_fn(pool_ids, pool_sc, pruned_corpus, queries, rtol):
    """Accepts a missing id whose coarse score ties the reference pool's boundary within the
    coarse tolerance (the approximate method may take either side of such a tie)."""
    def f(r, d):
        valid = pool_ids[r] >= 0
        last, lastid = pool_sc[r][valid][-1], pool_ids[r][valid][-1]
        c = oracle.pair_scores(pruned_corpus, queries, [r], [d])[0]
        sc = score_scale(pruned_corpus, queries, [r, r], [d, lastid]).max()
        return abs(c - last) <= 2 * rtol * sc
    return f


def stored_value_bits(values, dtype):
    """The bits the index must hold for FP32 values stored as dtype: FP32 copied, FP16 and
    BF16 rounded to nearest even (numpy's and torch's conversions)."""
    values = np.ascontiguousarray(values, np.float32)
    if dtype == "f32":
        return values.view(np.uint32)
    if dtype == "f16":
        return values.astype(np.float16).view(np.uint16)
    import torch
    return torch.from_numpy(values.copy()).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)


def check_layout_against_oracle(ex, ref, n_cols, window, dtype):
    """An exported index (pads dropped) holds Alg. 1's lists over the oracle's kept entries:
    per (term, window) the same documents, ascending inside every (tile, term) list, tiles
    inside windows, and each posting's value bits as stored_value_bits of the oracle's value."""
    tile_doc, tile_post, term_off = ex["tile_doc"], ex["tile_post"], ex["term_off"]
    nt = tile_doc.shape[0] - 1
    assert tile_doc[0] == 0 and tile_doc[-1] == ref.n_docs
    if nt:
        assert (np.diff(tile_doc) > 0).all()
        assert ((tile_doc[:-1] // window) == ((tile_doc[1:] - 1) // window)).all()
    tile_of = np.repeat(np.arange(nt), np.diff(tile_post))
    term_of = np.repeat(np.tile(np.arange(n_cols), nt), np.diff(term_off, axis=1).ravel())
    doc = ex["post_doc"].astype(np.int64) + tile_doc[tile_of]
    assert doc.shape[0] == ref.doc.shape[0], (doc.shape[0], ref.doc.shape[0])
    order = np.lexsort((doc, doc // window, term_of))  # Alg. 1 order: term, window, document
    assert np.array_equal(doc[order], ref.doc.astype(np.int64))
    ref_term = (np.repeat(np.arange(n_cols), np.diff(ref.ptr[::ref.sigma])) if ref.sigma
                else np.zeros(0, np.int64))
    assert np.array_equal(term_of[order], ref_term)
    same = (tile_of[1:] == tile_of[:-1]) & (term_of[1:] == term_of[:-1])
    assert (np.diff(doc)[same] > 0).all()
    got = np.ascontiguousarray(ex["post_val"])
    got = got.view(np.uint32) if dtype == "f32" else got.view(np.uint16)
    assert np.array_equal(got[order], stored_value_bits(ref.val, dtype))


def check_bank_order(raw, ex):
    """The stored lists (raw export) against the ascending ones (export()): a list's slots form
    chunks of 256 from its start; a chunk of n real postings holds the next n documents of the
    ascending list, which, taken by (document mod 32, document), fill slots 4 (32 h + r) + p
    for r = 0..31, h = 0..1, p = 0..3, skipping slots at or past n; a chunk of n <= 4 stays
    ascending.  Values move with their documents; pads (value 0, the list's largest document)
    follow the last chunk."""
    goff = raw["term_goff"]
    start = 4 * (goff & 0x3FFFFFFF).astype(np.int64)
    pad = (goff >> 30).astype(np.int64)[:, :-1]
    length = (np.diff(start, axis=1) - pad).ravel()
    first = (raw["tile_post"][:-1, None] + start[:, :-1]).ravel()   # raw slot of each list
    lid = np.repeat(np.arange(length.size), length)
    i = np.arange(lid.size) - np.repeat(np.cumsum(length) - length, length)  # rank in the list
    chunk, pos = i // 256, i % 256
    n = np.minimum(256, length[lid] - 256 * chunk)
    # sorted postings: the ascending list's items of each chunk, in (doc mod 32, doc) order
    doc = ex["post_doc"].astype(np.int64)
    key = lid * (1 << 20) + chunk
    order = np.lexsort((doc, np.where(n > 4, doc & 31, 0), key))
    # the fill order's rank of slot pos in a chunk of n postings
    lane, p = pos // 4, pos % 4
    r, h = lane & 31, lane >> 5
    k = np.minimum(n, 4 * r) + np.minimum(np.maximum(n - 128, 0), 4 * r) + 4 * h + p
    assert ((k >= 0) & (k < n)).all()
    chunk_first = i - pos                  # rank in the list of the chunk's first item
    src = order[(np.cumsum(length) - length)[lid] + chunk_first + k]
    slots = first[lid] + i
    assert np.array_equal(raw["post_doc"][slots].astype(np.int64), 4 * doc[src])
    rv, ev = raw["post_val"], ex["post_val"]
    assert np.array_equal(rv[slots].view(np.uint8), ev[src].view(np.uint8))
    # pads: value 0, the list's largest document
    ends = first + length
    has = np.nonzero(pad.ravel())[0]
    for j in has[:2000]:
        a, m = ends[j], pad.ravel()[j]
        assert (raw["post_doc"][a:a + m] == raw["post_doc"][first[j]:a].max()).all()
        assert (rv[a:a + m].view(np.uint8) == 0).all()
