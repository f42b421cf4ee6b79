"""Seeded synthetic sparse-vector generator (input generation only).

This module draws the CSR corpora and query sets that both the CPU oracle and
the GPU library consume.  It contains none of the retrieval method's
arithmetic: no scoring, pruning, index construction or ranking.

Rows follow the sparse-vector model of the paper (Def. 1: a vector is the set
of its non-zero (dimension, value) entries) with the shapes of its dataset
table (Sec. 5.1, Table "datasets"): a SPLADE-sized vocabulary, Zipf-distributed
term ids, Poisson row lengths and positive lognormal weights.  The native part
(``synth.c``) is counter based: every (seed, stream, row) keys its own
SplitMix64 sequence, so any row regenerates alone and thread count does not
change the output.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")

# RNG streams: documents, queries, planted positives, serving arrivals.
STREAM_DOCS, STREAM_QUERIES, STREAM_PLANT, STREAM_ARRIVALS = 0, 1, 2, 3


def compile_native(force: bool = True) -> str:
    """Compile ``libsynth.so`` with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("vocab", ctypes.c_int64),
        ("term_dist", ctypes.c_int32),
        ("nnz_dist", ctypes.c_int32),
        ("zipf_s", ctypes.c_double),
        ("nnz_a", ctypes.c_double),
        ("nnz_b", ctypes.c_double),
        ("nnz_min", ctypes.c_int64),
        ("nnz_max", ctypes.c_int64),
        ("val_dist", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("val_a", ctypes.c_double),
        ("val_b", ctypes.c_double),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            compile_native(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.synth_indptr.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_int64, ctypes.c_uint64,
                                     ctypes.c_uint64, ctypes.c_int64, P]
        lib.synth_fill.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_int64, ctypes.c_uint64,
                                   ctypes.c_uint64, ctypes.c_int64, P, P, P]
        lib.synth_uniform_u64.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                          ctypes.c_int64, P]
        lib.synth_lognormal_f32.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                            ctypes.c_int64, ctypes.c_double, ctypes.c_double, P]
        lib.synth_exponential_f64.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                              ctypes.c_int64, ctypes.c_double, P]
        for f in (lib.synth_indptr, lib.synth_fill, lib.synth_uniform_u64,
                  lib.synth_lognormal_f32, lib.synth_exponential_f64):
            f.restype = None
        _lib = lib
    return _lib


@dataclass(frozen=True)
class Csr:
    """A host CSR matrix: row r holds indices[indptr[r]:indptr[r+1]] (ascending)."""

    indptr: np.ndarray  # int64 [n_rows + 1]
    indices: np.ndarray  # int32 [nnz]
    values: np.ndarray  # float32 [nnz]
    n_cols: int

    @property
    def n_rows(self) -> int:
        return int(self.indptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def row(self, r: int):
        a, b = int(self.indptr[r]), int(self.indptr[r + 1])
        return self.indices[a:b], self.values[a:b]

    def take_rows(self, rows) -> "Csr":
        rows = np.asarray(rows, dtype=np.int64)
        lens = self.indptr[rows + 1] - self.indptr[rows]
        indptr = np.zeros(rows.shape[0] + 1, dtype=np.int64)
        np.cumsum(lens, out=indptr[1:])
        idx = np.empty(int(indptr[-1]), dtype=np.int32)
        val = np.empty(int(indptr[-1]), dtype=np.float32)
        for i, r in enumerate(rows):
            a, b = int(self.indptr[r]), int(self.indptr[r + 1])
            idx[indptr[i]:indptr[i + 1]] = self.indices[a:b]
            val[indptr[i]:indptr[i + 1]] = self.values[a:b]
        return Csr(indptr, idx, val, self.n_cols)


def generate(n_rows: int, vocab: int, *, nnz=("poisson", 120.0), clip=(1, 512),
             terms=("zipf", 1.1), values=("lognormal", 0.0, 0.8), seed: int = 0,
             stream: int = STREAM_DOCS, row0: int = 0) -> Csr:
    """Draw ``n_rows`` sparse rows over ``vocab`` dimensions.

    nnz    : ("poisson", mean) or ("uniform", lo, hi) (inclusive), then clipped
    terms  : ("zipf", s) over ranks 1..vocab (rank r -> id r-1) or ("uniform",)
    values : ("lognormal", mu, sigma) or ("uniform", a, b)
    Row ``row0 + r`` of a (seed, stream) pair is the same whatever ``n_rows``.
    """
    lib = _load()
    c = _Cfg()
    c.vocab = int(vocab)
    if terms[0] == "zipf":
        c.term_dist, c.zipf_s = 0, float(terms[1])
    elif terms[0] == "uniform":
        c.term_dist, c.zipf_s = 1, 0.0
    else:
        raise ValueError(terms)
    if nnz[0] == "poisson":
        c.nnz_dist, c.nnz_a, c.nnz_b = 0, float(nnz[1]), 0.0
    elif nnz[0] == "uniform":
        c.nnz_dist, c.nnz_a, c.nnz_b = 1, float(nnz[1]), float(nnz[2])
    else:
        raise ValueError(nnz)
    c.nnz_min, c.nnz_max = int(clip[0]), int(clip[1])
    if values[0] == "lognormal":
        c.val_dist = 0
    elif values[0] == "uniform":
        c.val_dist = 1
    else:
        raise ValueError(values)
    c.val_a, c.val_b = float(values[1]), float(values[2])
    indptr = np.zeros(n_rows + 1, dtype=np.int64)
    lib.synth_indptr(ctypes.byref(c), n_rows, seed, stream, row0, indptr.ctypes.data)
    nnz_total = int(indptr[-1])
    indices = np.empty(nnz_total, dtype=np.int32)
    vals = np.empty(nnz_total, dtype=np.float32)
    lib.synth_fill(ctypes.byref(c), n_rows, seed, stream, row0, indptr.ctypes.data,
                   indices.ctypes.data, vals.ctypes.data)
    return Csr(indptr, indices, vals, int(vocab))


def uniform_u64(n: int, seed: int, stream: int, i0: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    _load().synth_uniform_u64(seed, stream, i0, n, out.ctypes.data)
    return out


def lognormal_f32(n: int, seed: int, stream: int, mu: float = 0.0, sigma: float = 0.8,
                  i0: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.float32)
    _load().synth_lognormal_f32(seed, stream, i0, n, mu, sigma, out.ctypes.data)
    return out


def exponential_f64(n: int, seed: int, stream: int, mean: float, i0: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    _load().synth_exponential_f64(seed, stream, i0, n, mean, out.ctypes.data)
    return out


def random_csr(rng: np.random.Generator, n_rows: int, n_cols: int, max_nnz: int,
               signed: bool = False, min_nnz: int = 0) -> Csr:
    """Small irregular CSR for tests: ragged and empty rows, optional negative values."""
    lens = rng.integers(min_nnz, max_nnz + 1, size=n_rows)
    lens = np.minimum(lens, n_cols)
    indptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(lens, out=indptr[1:])
    idx = np.empty(int(indptr[-1]), dtype=np.int32)
    val = np.empty(int(indptr[-1]), dtype=np.float32)
    for r in range(n_rows):
        a, b = int(indptr[r]), int(indptr[r + 1])
        idx[a:b] = np.sort(rng.choice(n_cols, size=b - a, replace=False))
        v = rng.lognormal(0.0, 0.8, size=b - a)
        if signed:
            v = v * rng.choice([-1.0, 1.0], size=b - a)
        val[a:b] = v.astype(np.float32)
    return Csr(indptr, idx, val, n_cols)
