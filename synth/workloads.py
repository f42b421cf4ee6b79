"""Named synthetic workloads: sizes and parameters only (no method arithmetic).

Each entry mirrors one evaluation setting of the SINDI search path on
SPLADE-shaped synthetic data: the paper's SPLADE-FULL corpus (8,841,823
documents, ~127 non-zeros each, vocabulary ~30K; Sec. 5.1, Table "datasets")
stands behind the 8.8M-document setting, and the BGE-M3-shaped AntSparse
vocabulary (250K) behind the differentiation setting.  Real datasets are not
used; every corpus here is drawn by :mod:`synth` from its seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

import synth


@dataclass(frozen=True)
class Workload:
    name: str
    n_docs: int
    vocab: int
    doc_nnz: tuple
    n_queries: int
    query_nnz: tuple
    alpha: float  # document mass-ratio pruning (1.0 = none)
    window: int  # window size lambda, documents
    gamma: int  # rerank pool
    k: int
    beta: float = 1.0  # query mass-ratio pruning (1.0 = none)
    value_dtype: str = "f32"  # posting value storage: f32 / f16 / bf16
    seed: int = 0
    terms: tuple = ("zipf", 1.1)
    values: tuple = ("lognormal", 0.0, 0.8)
    clip: tuple = (1, 512)
    extra: dict = field(default_factory=dict)

    def scaled(self, n_docs: int, n_queries: int | None = None) -> "Workload":
        return replace(self, n_docs=n_docs,
                       n_queries=self.n_queries if n_queries is None else n_queries,
                       name=f"{self.name}@{n_docs}")

    def corpus(self) -> synth.Csr:
        return synth.generate(self.n_docs, self.vocab, nnz=self.doc_nnz, clip=self.clip,
                              terms=self.terms, values=self.values, seed=self.seed,
                              stream=synth.STREAM_DOCS)

    def queries(self, n: int | None = None, row0: int = 0) -> synth.Csr:
        return synth.generate(self.n_queries if n is None else n, self.vocab,
                              nnz=self.query_nnz, clip=self.clip, terms=self.terms,
                              values=self.values, seed=self.seed,
                              stream=synth.STREAM_QUERIES, row0=row0)

    def arrivals(self, rate: float, n: int, block: int = 0) -> np.ndarray:
        """Open-loop Poisson arrival times in seconds: n requests at `rate` per second
        (exponential gaps); `block` selects an independent run of draws."""
        gaps = synth.exponential_f64(n, self.seed, synth.STREAM_ARRIVALS, 1.0 / rate,
                                     i0=block << 32)
        return np.cumsum(gaps)

    def plant_positives(self, corpus: synth.Csr, queries: synth.Csr):
        """One planted positive per query: query b's support copied into a distinct
        random document p_b, with fresh values 2 x lognormal(0, 0.8).  Returns the new
        corpus and p (int64 [n_queries])."""
        nq, nd = queries.n_rows, corpus.n_rows
        u = synth.uniform_u64(4 * nq + 64, self.seed, synth.STREAM_PLANT)
        pos, seen = [], set()
        for x in u:  # distinct documents, first come first served
            d = int(x % np.uint64(nd))
            if d not in seen:
                seen.add(d)
                pos.append(d)
            if len(pos) == nq:
                break
        pos = np.asarray(pos, np.int64)
        vals = 2.0 * synth.lognormal_f32(int(queries.nnz), self.seed, synth.STREAM_PLANT,
                                         i0=1 << 32).astype(np.float32)
        lens = np.diff(corpus.indptr).astype(np.int64)
        qlen = np.diff(queries.indptr).astype(np.int64)
        lens[pos] = qlen
        indptr = np.zeros(nd + 1, np.int64)
        np.cumsum(lens, out=indptr[1:])
        idx = np.empty(int(indptr[-1]), np.int32)
        val = np.empty(int(indptr[-1]), np.float32)
        repl = np.zeros(nd, bool)
        repl[pos] = True
        keep_rows = np.nonzero(~repl)[0]
        # untouched rows move as whole blocks
        src_len = np.diff(corpus.indptr)[keep_rows]
        src = np.repeat(corpus.indptr[keep_rows], src_len) + (
            np.arange(int(src_len.sum())) - np.repeat(np.cumsum(src_len) - src_len, src_len))
        dst = np.repeat(indptr[keep_rows], src_len) + (
            np.arange(int(src_len.sum())) - np.repeat(np.cumsum(src_len) - src_len, src_len))
        idx[dst] = corpus.indices[src]
        val[dst] = corpus.values[src]
        for b, d in enumerate(pos):
            a, e = int(queries.indptr[b]), int(queries.indptr[b + 1])
            o = int(indptr[d])
            idx[o:o + e - a] = queries.indices[a:e]
            val[o:o + e - a] = vals[a:e]
        return synth.Csr(indptr, idx, val, corpus.n_cols), pos

    def request_ks(self, n: int, choices=(10, 50, 100), row0: int = 0) -> np.ndarray:
        """k of each serving request, uniform over `choices`."""
        u = synth.uniform_u64(n, self.seed, synth.STREAM_ARRIVALS, i0=(1 << 48) + row0)
        return np.asarray(choices, np.int32)[(u % np.uint64(len(choices))).astype(np.int64)]


WORKLOADS = {
    # Plain method, exact: no pruning, one window, top-10.
    "tiny": Workload("tiny", 10_000, 30_522, ("poisson", 120.0), 100, ("poisson", 30.0),
                     alpha=1.0, window=10_000, gamma=10, k=10),
    # Mass-ratio pruned index, FP32 values, rerank pool 500, top-50.
    "pruned-1m": Workload("pruned-1m", 1_000_000, 30_522, ("poisson", 120.0), 1_000,
                          ("poisson", 30.0), alpha=0.5, window=100_000, gamma=500, k=50),
    # SPLADE-FULL-sized corpus, half-precision posting values, FP32 rerank.
    "splade-8.8m": Workload("splade-8.8m", 8_800_000, 30_522, ("poisson", 125.0), 7_000,
                            ("poisson", 35.0), alpha=0.5, window=100_000, gamma=500, k=50,
                            value_dtype="f16"),
    # Serving: same index, queries of uniform length 5..200, k in {10, 50, 100}.
    "serving": Workload("serving", 8_800_000, 30_522, ("poisson", 125.0), 20_000,
                        ("uniform", 5, 200), alpha=0.5, window=100_000, gamma=500, k=100,
                        value_dtype="f16", extra={"rates": (2e3, 5e3, 1e4, 2e4, 5e4)}),
    # Short queries over a large vocabulary (AntSparse shape: BGE-M3, ~40 non-zeros per
    # document, ~5.8 per query, 250,000 terms); the paper's alpha for it, lambda 50,000.
    "antsparse-1m": Workload("antsparse-1m", 1_000_000, 250_000, ("poisson", 40.1), 1_000,
                             ("poisson", 5.8), alpha=0.85, window=50_000, gamma=500, k=50,
                             value_dtype="f16"),
    # Uniform sparsity (RANDOM shape): term ids and values uniform, ~120 non-zeros.
    "random-1m": Workload("random-1m", 1_000_000, 30_000, ("poisson", 120.0), 1_000,
                          ("poisson", 50.0), alpha=0.5, window=100_000, gamma=500, k=50,
                          value_dtype="f16", terms=("uniform",), values=("uniform", 0.0, 1.0),
                          extra={"vocab_sweep": (10_000, 30_000, 100_000)}),
    # Differentiation: multilingual-sized vocabulary, exact top-100 candidates.
    "diff-1m": Workload("diff-1m", 1_000_000, 250_002, ("poisson", 180.0), 256,
                        ("poisson", 40.0), alpha=1.0, window=100_000, gamma=100, k=100,
                        extra={"tau": 20.0}),
}
