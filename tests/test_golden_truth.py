"""The stored exact top-50 of the 8.8M-document bench workload (written by the oracle with
tests/golden/make_exact_truth.py) is the oracle's answer for the generated input: its
fingerprint matches the generator's output, and recomputing a few queries reproduces it."""
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
    sel = np.array([0, 6_999])  # each one scans the 1.1e9 corpus entries on one host thread
    got, sc = oracle.exact_topk(corpus, queries.take_rows(sel), wl.k)
    assert np.array_equal(got, ids[sel].astype(np.int64))
    assert np.array_equal(sc.astype(np.float32), scores[sel])
    # ranked: scores descending, ties by ascending id
    s = scores.astype(np.float64)
    assert (np.diff(s, axis=1) <= 0).all()
