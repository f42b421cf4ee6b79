"""SINDI sparse maximum-inner-product search on MI355X (gfx950).

A thin Python binding over the C ABI of ``libsindi.so`` (include/sindi.h):
argument marshalling only.  Every step of the search path runs in the
library's HIP kernels; PyTorch supplies device memory and the stream.
Importing this package never falls back to CPU code: if the library is not
built, :func:`_lib.load` raises.

Method: arXiv 2509.08395 (SINDI) -- value-storing inverted lists cut into
windows (Alg. 1, Sec. 3.3.1), mass-ratio pruning of documents and queries
(Defs. 5-6, Alg. 3), coarse top-gamma over the pruned lists (Alg. 2) and an
exact rerank from the unpruned vectors (Alg. 4).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import DTYPES, SindiError  # noqa: F401

__all__ = ["Index", "Server", "DeviceCsr", "SindiScore", "SindiError", "version",
           "profile_enable", "profile_read"]


def version() -> str:
    return _lib.load().sindi_version().decode()


def profile_enable(on: bool = True) -> None:
    """Record HIP events around every search kernel (see include/sindi.h)."""
    _lib.check(_lib.load().sindi_profile_enable(1 if on else 0))


def profile_read(reset: bool = True) -> dict:
    """{kernel class: (launches, total GPU ms)} since the last reset."""
    p = _lib.SindiProfile()
    _lib.check(_lib.load().sindi_profile_read(ctypes.byref(p), 1 if reset else 0))
    return {name: (int(p.launches[i]), float(p.ms[i]))
            for i, name in enumerate(_lib.PROFILE_CLASSES)}


def _stream(stream):
    import torch
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(stream)


class _HostCsr:
    """A host CSR as the C struct (keeps the numpy arrays alive)."""

    def __init__(self, csr):
        self.indptr = np.ascontiguousarray(csr.indptr, dtype=np.int64)
        self.indices = np.ascontiguousarray(csr.indices, dtype=np.int32)
        self.values = np.ascontiguousarray(csr.values, dtype=np.float32)
        self.n_rows = self.indptr.shape[0] - 1
        self.n_cols = int(csr.n_cols)
        self.nnz = int(self.indptr[-1]) if self.n_rows >= 0 else 0

    def struct(self):
        return _lib.SindiCsr(self.n_rows, self.n_cols, self.nnz, self.indptr.ctypes.data,
                             self.indices.ctypes.data if self.nnz else None,
                             self.values.ctypes.data if self.nnz else None, 0, 0)


class DeviceCsr:
    """A CSR whose arrays are torch tensors on the GPU."""

    def __init__(self, indptr, indices, values, n_cols):
        self.indptr, self.indices, self.values, self.n_cols = indptr, indices, values, int(n_cols)

    @classmethod
    def from_host(cls, csr, device="cuda"):
        import torch
        return cls(torch.as_tensor(np.asarray(csr.indptr, np.int64)).to(device),
                   torch.as_tensor(np.asarray(csr.indices, np.int32)).to(device),
                   torch.as_tensor(np.asarray(csr.values, np.float32)).to(device), csr.n_cols)

    @property
    def n_rows(self):
        return int(self.indptr.shape[0]) - 1

    @property
    def nnz(self):
        return int(self.indices.shape[0])

    def struct(self):
        for t, dt in ((self.indptr, "int64"), (self.indices, "int32"), (self.values, "float32")):
            if not t.is_cuda or not t.is_contiguous() or str(t.dtype) != "torch." + dt:
                raise ValueError(f"DeviceCsr arrays must be contiguous CUDA {dt} tensors")
        return _lib.SindiCsr(self.n_rows, self.n_cols, self.nnz, self.indptr.data_ptr(),
                             self.indices.data_ptr(), self.values.data_ptr(), 1, 0)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _vector_arg(t, n, name):
    """None, or a contiguous float32 CUDA tensor of n elements (the kernels write or read
    exactly n)."""
    import torch
    if t is None:
        return
    if (not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32
            or not t.is_contiguous() or t.numel() != n):
        raise SindiError(_lib.SINDI_E_INVALID,
                         f"{name} must be a contiguous CUDA float32 tensor of {n} elements")


def _query_struct(queries):
    if isinstance(queries, DeviceCsr):
        return queries.struct(), queries
    h = _HostCsr(queries)
    return h.struct(), h


class Index:
    """A SINDI index in device memory (Alg. 3: pruned window lists + unpruned corpus)."""

    def __init__(self, corpus, alpha=1.0, window=100_000, value_dtype="f32", tile=0, stream=None,
                 prune="mrp", vn=0, list_len=0, gpu_build=False):
        """corpus: a host CSR, or a DeviceCsr (then gpu_build must be True)."""
        lib = _lib.load()
        if isinstance(corpus, DeviceCsr):
            h, cs = corpus, corpus.struct()
        else:
            h = _HostCsr(corpus)
            cs = h.struct()
        params = _lib.SindiBuildParams(float(alpha), int(window), DTYPES[value_dtype], int(tile),
                                       _lib.PRUNE[prune], int(vn), int(list_len),
                                       1 if gpu_build else 0, 0)
        handle = ctypes.c_void_p()
        _lib.check(lib.sindi_build(ctypes.byref(cs), ctypes.byref(params), _stream(stream),
                                   ctypes.byref(handle)))
        self._h = handle
        self.n_cols = h.n_cols
        self.nnz = h.nnz
        self.value_dtype = value_dtype

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.load().sindi_index_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        inf = _lib.SindiIndexInfo()
        _lib.check(_lib.load().sindi_index_get_info(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in inf._fields_}

    def export(self, raw: bool = False) -> dict:
        """The device layout copied to host numpy arrays.

        raw=True: the stored arrays (lists aligned to 4 slots with pad entries, the
        encoded group offsets ``term_goff``, every chunk of 64 groups in LDS-bank order).
        Otherwise the pads are dropped and every list is in ascending document order (Alg.
        1): ``tile_post`` / ``term_off`` [n_tiles, n_cols + 1] are posting offsets of the
        compacted lists and ``post_doc`` / ``post_val`` hold only real postings."""
        inf = self.info()
        nt, nc, nslot = inf["n_tiles"], inf["n_cols"], inf["n_slots"]
        tile_doc = np.empty(nt + 1, np.int64)
        tile_post = np.empty(nt + 1, np.int64)
        term_goff = np.empty(nt * (nc + 1), np.uint32)
        post_doc = np.empty(max(nslot, 1), np.uint16)
        vb = _lib.VALUE_BYTES[inf["value_dtype"]]
        post_val = np.empty(max(nslot, 1) * vb, np.uint8)
        _lib.check(_lib.load().sindi_index_export(self._h, tile_doc.ctypes.data,
                                                  tile_post.ctypes.data, term_goff.ctypes.data,
                                                  post_doc.ctypes.data, post_val.ctypes.data))
        vt = {4: np.float32, 2: np.uint16}[vb]
        post_val = post_val.view(vt)[:nslot]
        # stored: byte offsets of 32-bit score words; returned: tile-local document ids
        post_doc = post_doc[:nslot] if raw else (post_doc[:nslot] >> 2)
        goff = term_goff.reshape(nt, nc + 1)
        if raw:
            return {"tile_doc": tile_doc, "tile_post": tile_post, "term_goff": goff,
                    "post_doc": post_doc, "post_val": post_val}
        start = 4 * (goff & 0x3FFFFFFF).astype(np.int64)          # slot offsets in the tile
        pad = (goff >> 30).astype(np.int64)
        length = np.diff(start, axis=1) - pad[:, :-1]              # real postings per list
        term_off = np.zeros((nt, nc + 1), np.int64)
        np.cumsum(length, axis=1, out=term_off[:, 1:])
        # slots of the pad entries: (g >> 30) of them after every list's postings
        pads = pad[:, :-1].ravel()
        sel = np.nonzero(pads)[0]
        pad_at = (tile_post[:-1, None] + start[:, :-1]).ravel()[sel] + length.ravel()[sel]
        pad_n = pads[sel]
        rank = np.arange(int(pad_n.sum())) - np.repeat(np.cumsum(pad_n) - pad_n, pad_n)
        keep = np.ones(nslot, bool)
        keep[np.repeat(pad_at, pad_n) + rank] = False
        cpost = np.zeros(nt + 1, np.int64)
        np.cumsum(term_off[:, -1], out=cpost[1:])
        pd, pv = post_doc[keep], post_val[keep]
        # the stored chunks are in bank order: documents ascending inside each list
        order = np.lexsort((pd, np.repeat(np.arange(length.size), length.ravel())))
        return {"tile_doc": tile_doc, "tile_post": cpost, "term_off": term_off,
                "post_doc": pd[order], "post_val": pv[order]}

    def term_lengths(self) -> np.ndarray:
        """Postings per term over all tiles (int64 [n_cols]), pads excluded."""
        goff = self.export(raw=True)["term_goff"]
        start = 4 * (goff & 0x3FFFFFFF).astype(np.int64)
        return (np.diff(start, axis=1) - (goff[:, :-1] >> 30)).sum(axis=0)

    def _run(self, fn, queries, k, beta, gamma, batch, cand_cap, sample_tiles, stream, out,
             tile_run=0, schedule=0):
        import torch
        qs, keep = _query_struct(queries)
        nq = qs.n_rows
        if out is None:
            ids = torch.empty((nq, k), dtype=torch.int64, device="cuda")
            scores = torch.empty((nq, k), dtype=torch.float32, device="cuda")
        else:
            ids, scores = out
        params = _lib.SindiSearchParams(float(beta), int(gamma), int(batch), int(cand_cap),
                                        int(sample_tiles), int(tile_run), int(schedule))
        _lib.check(fn(self._h, ctypes.byref(qs), int(k), ctypes.byref(params),
                      ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(scores.data_ptr()),
                      _stream(stream)))
        del keep
        return ids, scores

    def search(self, queries, k, beta=1.0, gamma=0, batch=0, cand_cap=0, sample_tiles=0,
               stream=None, out=None, tile_run=0, schedule=0):
        """Alg. 4: (ids int64 [n, k], scores float32 [n, k]) as CUDA tensors."""
        return self._run(_lib.load().sindi_search, queries, k, beta, gamma, batch, cand_cap,
                         sample_tiles, stream, out, tile_run, schedule)

    def search_coarse(self, queries, k, beta=1.0, batch=0, cand_cap=0, sample_tiles=0,
                      stream=None, out=None, tile_run=0, schedule=0):
        """Alg. 2 over the (pruned) index: coarse top-k, no rerank."""
        return self._run(_lib.load().sindi_search_coarse, queries, k, beta, 0, batch, cand_cap,
                         sample_tiles, stream, out, tile_run, schedule)

    def _score_args(self, queries, cand, doc_values):
        """Checks the shapes the score kernels index by (they cannot see buffer sizes)."""
        import torch
        if not isinstance(queries, DeviceCsr):
            raise SindiError(_lib.SINDI_E_INVALID, "score: queries must be a DeviceCsr")
        if (not isinstance(cand, torch.Tensor) or not cand.is_cuda or cand.dtype != torch.int64
                or cand.dim() != 2 or cand.shape[0] != queries.n_rows):
            raise SindiError(_lib.SINDI_E_INVALID,
                             f"score: cand must be a CUDA int64 tensor [{queries.n_rows}, n_cand]")
        _vector_arg(doc_values, self.nnz, "doc_values")
        return queries.struct(), cand.contiguous()

    def score(self, queries: DeviceCsr, cand, doc_values=None, stream=None):
        """delta(q_b, x_c) for cand [n_q, n_cand] (int64 CUDA) -> float32 [n_q, n_cand].

        doc_values (float32 CUDA [nnz], aligned with the corpus values the index was built
        from): the document values to score; None scores the index's build-time copy."""
        import torch
        qs, cand = self._score_args(queries, cand, doc_values)
        out = torch.empty(cand.shape, dtype=torch.float32, device="cuda")
        _lib.check(_lib.load().sindi_score_forward(self._h, ctypes.byref(qs),
                                                   ctypes.c_void_p(cand.data_ptr()),
                                                   int(cand.shape[1]), _ptr(doc_values),
                                                   ctypes.c_void_p(out.data_ptr()),
                                                   _stream(stream)))
        return out

    def score_backward(self, queries: DeviceCsr, cand, grad, grad_query=None, grad_doc=None,
                       doc_values=None, stream=None):
        """Adds dL/dq into grad_query [queries.nnz] and dL/dx into grad_doc [nnz] (float32
        CUDA, either may be None) for grad = dL/dscore [n_q, n_cand]."""
        qs, cand = self._score_args(queries, cand, doc_values)
        if (not hasattr(grad, "is_cuda") or not grad.is_cuda or tuple(grad.shape) != tuple(cand.shape)):
            raise SindiError(_lib.SINDI_E_INVALID, "score_backward: grad must be a CUDA tensor "
                             f"shaped like cand {tuple(cand.shape)}")
        grad = grad.contiguous().float()
        _vector_arg(grad_query, queries.nnz, "grad_query")
        _vector_arg(grad_doc, self.nnz, "grad_doc")
        _lib.check(_lib.load().sindi_score_backward(self._h, ctypes.byref(qs), _ptr(cand),
                                                    int(cand.shape[1]), _ptr(doc_values),
                                                    _ptr(grad), _ptr(grad_query), _ptr(grad_doc),
                                                    _stream(stream)))


class Server:
    """Continuous batching over an Index (include/sindi.h, serving section).

    Requests queue as they arrive; the library's dispatcher thread runs every queued
    request (up to ``max_batch``) as one batch on one of ``max_inflight`` streams as soon
    as a stream is free.  Results are host numpy arrays.
    """

    def __init__(self, index, max_inflight=3, max_batch=256, k_max=100, max_query_nnz=512,
                 max_queue=0, workspace_bytes=0, beta=1.0, gamma=0, batch=0, cand_cap=0,
                 sample_tiles=0, tile_run=0, schedule=0):
        lib = _lib.load()
        sp = _lib.SindiSearchParams(float(beta), int(gamma), int(batch), int(cand_cap),
                                    int(sample_tiles), int(tile_run), int(schedule))
        params = _lib.SindiServerParams(int(max_inflight), int(max_batch), int(k_max),
                                        int(max_query_nnz), int(max_queue), int(workspace_bytes),
                                        sp)
        handle = ctypes.c_void_p()
        _lib.check(lib.sindi_server_create(index._h, ctypes.byref(params), ctypes.byref(handle)))
        self._h = handle
        self._index = index  # the index must outlive the server
        self.k_max = int(k_max)

    def submit(self, indices, values, k) -> int:
        """Queue one query (ascending term ids, float values); returns its ticket."""
        idx = np.ascontiguousarray(indices, dtype=np.int32)
        val = np.ascontiguousarray(values, dtype=np.float32)
        if idx.shape != val.shape:
            raise ValueError("indices and values differ in length")
        t = ctypes.c_int64()
        _lib.check(_lib.load().sindi_server_submit(self._h, idx.ctypes.data, val.ctypes.data,
                                                   int(idx.shape[0]), int(k), ctypes.byref(t)))
        return t.value

    def wait(self, ticket, k, timeout_ms=-1.0):
        """(ids int64 [k], scores float32 [k], latency in ns) of a submitted request."""
        ids = np.empty(k, np.int64)
        scores = np.empty(k, np.float32)
        lat = ctypes.c_int64()
        _lib.check(_lib.load().sindi_server_wait(self._h, int(ticket), ids.ctypes.data,
                                                 scores.ctypes.data, ctypes.byref(lat),
                                                 float(timeout_ms)))
        return ids, scores, lat.value

    def replay(self, queries, ks, arrival_s):
        """Open-loop replay: row r arrives arrival_s[r] seconds after the call starts.
        Returns ids [n, k_max], scores [n, k_max] (row r's first ks[r] entries hold its
        results) and latency_ns [n] measured from the scheduled arrival."""
        h = _HostCsr(queries)
        n = h.n_rows
        ks = np.ascontiguousarray(ks, dtype=np.int32)
        arr = np.ascontiguousarray(arrival_s, dtype=np.float64)
        if ks.shape != (n,) or arr.shape != (n,):
            raise ValueError("ks and arrival_s need one entry per query")
        ids = np.empty((n, self.k_max), np.int64)
        scores = np.empty((n, self.k_max), np.float32)
        lat = np.empty(n, np.int64)
        _lib.check(_lib.load().sindi_server_replay(self._h, ctypes.byref(h.struct()),
                                                   ks.ctypes.data, arr.ctypes.data,
                                                   ids.ctypes.data, scores.ctypes.data,
                                                   lat.ctypes.data))
        return ids, scores, lat

    def stats(self) -> dict:
        st = _lib.SindiServerStats()
        _lib.check(_lib.load().sindi_server_get_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in st._fields_}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.load().sindi_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _make_score_fn():
    import torch

    class SindiScore(torch.autograd.Function):
        """s[b, c] = delta(q_b, x_{cand[b, c]}) with hand-written HIP forward and backward.

        Inputs: query values (requires_grad), document values (requires_grad; float32
        CUDA [nnz], aligned entry for entry with the corpus the index was built from: same
        rows and term ids, values free to change, e.g. as a document encoder trains), the
        index, the query CSR structure (indptr, indices) and candidate ids [n_q, n_cand].
        The scores and both gradients use the doc_values passed, not the index's
        build-time copy; only the candidates a search returns depend on that copy.
        """

        @staticmethod
        def forward(ctx, q_values, doc_values, index, q_indptr, q_indices, cand):
            qs = DeviceCsr(q_indptr, q_indices, q_values.detach().contiguous(), index.n_cols)
            xv = doc_values.detach().contiguous()
            ctx.index, ctx.qs, ctx.cand, ctx.xv = index, qs, cand, xv
            ctx.needs = (ctx.needs_input_grad[0], ctx.needs_input_grad[1])
            return index.score(qs, cand, doc_values=xv)

        @staticmethod
        def backward(ctx, grad):
            gq = torch.zeros_like(ctx.qs.values) if ctx.needs[0] else None
            gx = torch.zeros_like(ctx.xv) if ctx.needs[1] else None
            ctx.index.score_backward(ctx.qs, ctx.cand, grad, gq, gx, doc_values=ctx.xv)
            return gq, gx, None, None, None, None

    return SindiScore


class _LazyScore:
    _fn = None

    def __getattr__(self, name):
        if _LazyScore._fn is None:
            _LazyScore._fn = _make_score_fn()
        return getattr(_LazyScore._fn, name)


SindiScore = _LazyScore()
