"""The seeded generator: reproducible rows with the shapes the workloads state."""
import numpy as np
import pytest

import synth
from synth.workloads import WORKLOADS


def _check_canonical(csr):
    assert csr.indptr[0] == 0 and (np.diff(csr.indptr) >= 0).all()
    for r in range(csr.n_rows):
        i, v = csr.row(r)
        assert (np.diff(i) > 0).all()
        assert ((i >= 0) & (i < csr.n_cols)).all()
        assert np.isfinite(v).all() and (v != 0).all()


def test_rows_reproducible_and_independent_of_batch():
    a = synth.generate(500, 30522, seed=3, stream=1)
    b = synth.generate(100, 30522, seed=3, stream=1, row0=200)
    for r in range(100):
        ia, va = a.row(200 + r)
        ib, vb = b.row(r)
        assert ia.tolist() == ib.tolist() and va.tobytes() == vb.tobytes()
    c = synth.generate(500, 30522, seed=4, stream=1)
    assert a.indices.tobytes() != c.indices.tobytes()
    _check_canonical(a)


def test_poisson_lengths_lognormal_values_zipf_terms():
    wl = WORKLOADS["tiny"]
    c = synth.generate(20000, wl.vocab, nnz=("poisson", 120.0), seed=0)
    lens = np.diff(c.indptr)
    assert abs(lens.mean() - 120.0) < 0.5 and abs(lens.var() - 120.0) < 6.0
    logs = np.log(c.values.astype(np.float64))
    assert abs(logs.mean()) < 0.01 and abs(logs.std() - 0.8) < 0.01
    # Zipf(1.1) without replacement: the rank-1 term is in nearly every row, frequency
    # falls with rank
    df = np.bincount(c.indices, minlength=wl.vocab) / c.n_rows
    assert df[0] > 0.99 and df[0] >= df[10] >= df[100] >= df[1000]


def test_uniform_length_and_clip():
    c = synth.generate(5000, 1000, nnz=("uniform", 5, 200), seed=1)
    lens = np.diff(c.indptr)
    assert lens.min() == 5 and lens.max() == 200
    d = synth.generate(2000, 1000, nnz=("poisson", 1.0), clip=(1, 512), seed=1)
    assert np.diff(d.indptr).min() == 1
    _check_canonical(d)


def test_planted_positives_replace_only_their_rows():
    from synth.workloads import WORKLOADS
    wl = WORKLOADS["diff-1m"].scaled(3_000, 12)
    c, q = wl.corpus(), wl.queries()
    c2, pos = wl.plant_positives(c, q)
    assert len(set(pos.tolist())) == q.n_rows and (pos >= 0).all() and (pos < c.n_rows).all()
    for b, d in enumerate(pos):
        got = c2.indices[c2.indptr[d]:c2.indptr[d + 1]]
        assert (got == q.indices[q.indptr[b]:q.indptr[b + 1]]).all()
        assert (c2.values[c2.indptr[d]:c2.indptr[d + 1]] > 0).all()
    rest = np.setdiff1d(np.arange(c.n_rows), pos)
    assert (np.diff(c2.indptr)[rest] == np.diff(c.indptr)[rest]).all()
    for d in rest[::97]:
        a, e = c.indptr[d], c.indptr[d + 1]
        a2 = c2.indptr[d]
        assert (c2.indices[a2:a2 + e - a] == c.indices[a:e]).all()
        assert (c2.values[a2:a2 + e - a] == c.values[a:e]).all()
    c3, pos3 = wl.plant_positives(c, q)  # reproducible
    assert (pos3 == pos).all() and (c3.values == c2.values).all()
