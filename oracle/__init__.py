"""CPU FP64 oracle for the SINDI search path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it and the
two share no code; they meet only at the seeded inputs of :mod:`synth`.

Every function follows one passage of the paper (arXiv 2509.08395); the C
source ``oracle.c`` names them.  Python-side helpers here are plain numpy:

* :func:`recall_at_k` -- Recall = |R intersect R*| / |R*| (Sec. 5.1, metrics)
* :func:`contrastive_grad` -- softmax contrastive loss over candidate scores
  and its gradient with respect to the scores (the differentiation form's
  training loss; the paper itself has no backward pass, so this part is
  pinned by finite differences rather than by the paper).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def compile_native(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
P = ctypes.c_void_p
I64 = ctypes.c_int64


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            compile_native(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.or_exact_topk.argtypes = [I64, I64, P, P, P, I64, P, P, P, I64, P, P, ctypes.c_int]
        lib.or_pair_scores.argtypes = [P, P, P, P, P, P, I64, P, P, P]
        lib.or_mass_prune.argtypes = [I64, P, P, P, ctypes.c_double, P, ctypes.c_int]
        lib.or_build_index.argtypes = [I64, I64, P, P, P, P, I64, P, P, P]
        lib.or_precise_search.argtypes = [I64, I64, P, P, P, I64, P, P, P, I64, P, P,
                                          ctypes.c_int]
        lib.or_approx_search.argtypes = [I64, I64, P, P, P, P, P, P, I64, P, P, P,
                                         ctypes.c_double, I64, I64, P, P, P, P, ctypes.c_int]
        lib.or_score_grad.argtypes = [P, P, P, P, P, P, I64, I64, P, P, P, P]
        lib.or_vnp_prune.argtypes = [I64, P, P, P, I64, P, ctypes.c_int]
        lib.or_lp_prune.argtypes = [I64, I64, P, P, P, I64, P, P]
        for f in (lib.or_exact_topk, lib.or_pair_scores, lib.or_mass_prune, lib.or_build_index,
                  lib.or_precise_search, lib.or_approx_search, lib.or_score_grad,
                  lib.or_vnp_prune, lib.or_lp_prune):
            f.restype = None
        _lib = lib
    return _lib


def _threads(n):
    if n is not None:
        return int(n)
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _ptr(a):
    return a.ctypes.data if a is not None else None


def exact_topk(corpus, queries, k, threads=None):
    """Exact top-k by FP64 inner product (Defs. 2-3).  Returns (ids int64, scores f64)."""
    nd = corpus.n_rows
    nq = queries.n_rows
    ids = np.empty((nq, k), dtype=np.int64)
    sc = np.empty((nq, k), dtype=np.float64)
    dp, di, dv = _c(corpus.indptr, np.int64), _c(corpus.indices, np.int32), _c(corpus.values, np.float32)
    qp, qi, qv = _c(queries.indptr, np.int64), _c(queries.indices, np.int32), _c(queries.values, np.float32)
    _load().or_exact_topk(nd, corpus.n_cols, _ptr(dp), _ptr(di), _ptr(dv), nq, _ptr(qp), _ptr(qi),
                          _ptr(qv), k, _ptr(ids), _ptr(sc), _threads(threads))
    return ids, sc


def pair_scores(corpus, queries, pair_q, pair_d):
    """delta(q_{pair_q[t]}, x_{pair_d[t]}) in FP64 (Def. 2); id < 0 gives -inf."""
    pq, pd = _c(pair_q, np.int64).ravel(), _c(pair_d, np.int64).ravel()
    out = np.empty(pq.shape[0], dtype=np.float64)
    dp, di, dv = _c(corpus.indptr, np.int64), _c(corpus.indices, np.int32), _c(corpus.values, np.float32)
    qp, qi, qv = _c(queries.indptr, np.int64), _c(queries.indices, np.int32), _c(queries.values, np.float32)
    _load().or_pair_scores(_ptr(dp), _ptr(di), _ptr(dv), _ptr(qp), _ptr(qi), _ptr(qv), pq.shape[0],
                           _ptr(pq), _ptr(pd), _ptr(out))
    return out


def mass_prune(csr, alpha, threads=None):
    """Keep mask (uint8 per stored entry) of each row's alpha-mass subvector (Def. 6)."""
    keep = np.empty(csr.nnz, dtype=np.uint8)
    p, i, v = _c(csr.indptr, np.int64), _c(csr.indices, np.int32), _c(csr.values, np.float32)
    _load().or_mass_prune(csr.n_rows, _ptr(p), _ptr(i), _ptr(v), float(alpha), _ptr(keep),
                          _threads(threads))
    return keep


def vnp_prune(csr, vn, threads=None):
    """Keep mask of Vector Number Pruning: the vn entries of largest |x| per row."""
    keep = np.empty(csr.nnz, dtype=np.uint8)
    p, i, v = _c(csr.indptr, np.int64), _c(csr.indices, np.int32), _c(csr.values, np.float32)
    _load().or_vnp_prune(csr.n_rows, _ptr(p), _ptr(i), _ptr(v), int(vn), _ptr(keep),
                         _threads(threads))
    return keep


def lp_prune(csr, lmax, keep_in=None):
    """Keep mask of List Pruning: the lmax entries of largest |x| per term list (among
    the entries keep_in keeps, if given)."""
    keep = np.empty(csr.nnz, dtype=np.uint8)
    p, i, v = _c(csr.indptr, np.int64), _c(csr.indices, np.int32), _c(csr.values, np.float32)
    kin = _c(keep_in, np.uint8) if keep_in is not None else None
    _load().or_lp_prune(csr.n_rows, int(csr.n_cols), _ptr(p), _ptr(i), _ptr(v), int(lmax),
                        _ptr(kin) if kin is not None else None, _ptr(keep))
    return keep


def apply_mask(csr, keep):
    """The CSR of the kept entries (ascending term order preserved)."""
    import synth
    keep = keep.astype(bool)
    cs = np.zeros(csr.nnz + 1, dtype=np.int64)
    np.cumsum(keep, out=cs[1:])
    counts = cs[csr.indptr[1:]] - cs[csr.indptr[:-1]]
    indptr = np.zeros(csr.n_rows + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    return synth.Csr(indptr, csr.indices[keep].copy(), csr.values[keep].copy(), csr.n_cols)


class OracleIndex:
    """Alg. 1 output: lists I_{j,w} in (j, w) order; ptr has n_cols*sigma+1 entries."""

    def __init__(self, n_docs, n_cols, window, ptr, doc, val):
        self.n_docs, self.n_cols, self.window = n_docs, n_cols, window
        self.sigma = (n_docs + window - 1) // window
        self.ptr, self.doc, self.val = ptr, doc, val

    def list(self, j, w):
        l = j * self.sigma + w
        a, b = int(self.ptr[l]), int(self.ptr[l + 1])
        return self.doc[a:b], self.val[a:b]


def build_index(corpus, window, keep=None):
    """Alg. 1 (with Alg. 3's pruned corpus when a keep mask is given)."""
    nd, nc = corpus.n_rows, corpus.n_cols
    sigma = (nd + window - 1) // window
    ptr = np.empty(nc * sigma + 1, dtype=np.int64)
    n = int(corpus.nnz if keep is None else int(np.count_nonzero(keep)))
    doc = np.empty(max(n, 1), dtype=np.int32)
    val = np.empty(max(n, 1), dtype=np.float32)
    p, i, v = _c(corpus.indptr, np.int64), _c(corpus.indices, np.int32), _c(corpus.values, np.float32)
    km = None if keep is None else _c(keep, np.uint8)
    _load().or_build_index(nd, nc, _ptr(p), _ptr(i), _ptr(v), _ptr(km), window, _ptr(ptr),
                           _ptr(doc), _ptr(val))
    return OracleIndex(nd, nc, window, ptr, doc[:n], val[:n])


def precise_search(index, queries, k, threads=None):
    """Alg. 2 on an :class:`OracleIndex`.  Returns (ids, coarse scores f64)."""
    nq = queries.n_rows
    ids = np.empty((nq, k), dtype=np.int64)
    sc = np.empty((nq, k), dtype=np.float64)
    qp, qi, qv = _c(queries.indptr, np.int64), _c(queries.indices, np.int32), _c(queries.values, np.float32)
    _load().or_precise_search(index.n_docs, index.window, _ptr(index.ptr), _ptr(index.doc),
                              _ptr(index.val), nq, _ptr(qp), _ptr(qi), _ptr(qv), k, _ptr(ids),
                              _ptr(sc), _threads(threads))
    return ids, sc


def approx_search(index, corpus, queries, beta, gamma, k, threads=None, want_pool=False):
    """Alg. 4 with the unpruned ``corpus`` for the rerank.

    Returns (ids, exact scores f64) or, with ``want_pool``, also the coarse
    pool (pool ids, coarse scores), each [n_q, gamma] in ranking order.
    """
    nq = queries.n_rows
    ids = np.empty((nq, k), dtype=np.int64)
    sc = np.empty((nq, k), dtype=np.float64)
    pid = np.empty((nq, gamma), dtype=np.int64) if want_pool else None
    ps = np.empty((nq, gamma), dtype=np.float64) if want_pool else None
    dp, di, dv = _c(corpus.indptr, np.int64), _c(corpus.indices, np.int32), _c(corpus.values, np.float32)
    qp, qi, qv = _c(queries.indptr, np.int64), _c(queries.indices, np.int32), _c(queries.values, np.float32)
    _load().or_approx_search(index.n_docs, index.window, _ptr(index.ptr), _ptr(index.doc),
                             _ptr(index.val), _ptr(dp), _ptr(di), _ptr(dv), nq, _ptr(qp), _ptr(qi),
                             _ptr(qv), float(beta), gamma, k, _ptr(ids), _ptr(sc), _ptr(pid),
                             _ptr(ps), _threads(threads))
    if want_pool:
        return ids, sc, pid, ps
    return ids, sc


def score_grad(corpus, queries, cand, G):
    """dL/dq (aligned with query values) and dL/dx (aligned with corpus values), FP64."""
    cand = _c(cand, np.int64)
    G = _c(G, np.float64)
    nq, nc = cand.shape
    gq = np.zeros(queries.nnz, dtype=np.float64)
    gx = np.zeros(corpus.nnz, dtype=np.float64)
    dp, di, dv = _c(corpus.indptr, np.int64), _c(corpus.indices, np.int32), _c(corpus.values, np.float32)
    qp, qi, qv = _c(queries.indptr, np.int64), _c(queries.indices, np.int32), _c(queries.values, np.float32)
    _load().or_score_grad(_ptr(dp), _ptr(di), _ptr(dv), _ptr(qp), _ptr(qi), _ptr(qv), nq, nc,
                          _ptr(cand), _ptr(G), _ptr(gq), _ptr(gx))
    return gq, gx


def recall_at_k(found, truth):
    """Mean over queries of |R intersect R*| / |R*| (Sec. 5.1); ids < 0 are padding."""
    found = np.asarray(found)
    truth = np.asarray(truth)
    tot = 0.0
    for f, t in zip(found, truth):
        ts = set(int(x) for x in t if x >= 0)
        if not ts:
            tot += 1.0
            continue
        tot += len(ts.intersection(int(x) for x in f if x >= 0)) / len(ts)
    return tot / max(len(truth), 1)


def contrastive_grad(scores, pos, tau):
    """L = mean_b [logsumexp_c(s_bc / tau) - s_{b,pos_b} / tau] and dL/ds (FP64)."""
    s = np.asarray(scores, dtype=np.float64) / tau
    m = s.max(axis=1, keepdims=True)
    e = np.exp(s - m)
    z = e.sum(axis=1, keepdims=True)
    p = e / z
    nq = s.shape[0]
    rows = np.arange(nq)
    loss = float(np.mean(np.log(z[:, 0]) + m[:, 0] - s[rows, pos]))
    G = p.copy()
    G[rows, pos] -= 1.0
    G /= tau * nq
    return loss, G
