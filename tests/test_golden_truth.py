"""The stored exact top-50 of the 8.8M-document bench workload (written by the oracle with
tests/golden/make_exact_truth.py) is the oracle's answer for the generated input: its
fingerprint matches the generator's output, and three queries scored against every document by
Def. 2 and ranked reproduce it."""
import os
import sys

import numpy as np
import pytest

from conftest import ROOT

sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))


@pytest.mark.slow
def test_stored_exact_topk_is_the_oracles():
    import make_exact_truth as mt
    import oracle
    from synth.workloads import WORKLOADS
    wl = WORKLOADS["splade-8.8m"]
    path = mt.truth_path(wl.name, wl.k)
    with np.load(path, allow_pickle=False) as z:
        import json
        meta = json.loads(str(z["meta"]))
        ids, scores = z["ids"], z["scores"]
    assert ids.shape == (wl.n_queries, wl.k) and scores.shape == ids.shape
    assert meta["n_docs"] == wl.n_docs and meta["seed"] == wl.seed and meta["k"] == wl.k
    corpus, queries = wl.corpus(), wl.queries()
    assert meta["fingerprint"] == mt.fingerprint(corpus, queries)
    # Recompute three queries by Def. 2 for every document (the oracle's per-pair inner
    # product: the same FP64 sums, term order ascending, as its term-at-a-time top-k) and rank
    # them, score descending then id ascending: no corpus transpose, ~10 s per query.
    docs = np.arange(wl.n_docs, dtype=np.int64)
    for q in (0, 3_500, 6_999):
        s = oracle.pair_scores(corpus, queries, np.full(wl.n_docs, q, dtype=np.int64), docs)
        top = np.lexsort((docs, -s))[:wl.k]
        assert np.array_equal(top, ids[q].astype(np.int64)), q
        assert np.array_equal(s[top].astype(np.float32), scores[q]), q
    # ranked: scores descending, ties by ascending id
    s = scores.astype(np.float64)
    assert (np.diff(s, axis=1) <= 0).all()
