"""sindi_search_noalloc (the search with all device scratch in the library's static array)
against sindi_search through the C ABI: bit-identical ids and scores on two calls in a row,
the second with a smaller input (the array keeps the first call's contents), also when the
sampled threshold misses and both retry passes run inside the array; and its size limit."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sindi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_08395_amd as s
    s._lib.load()
    return s


def _noalloc(sindi, idx, dq, k, **kw):
    from paper_2509_08395_amd import _lib
    lib = _lib.load()
    n = dq.n_rows
    ids = torch.full((n, k), -7, dtype=torch.int64, device="cuda")
    sc = torch.full((n, k), 7.0, dtype=torch.float32, device="cuda")
    p = _lib.SindiSearchParams(float(kw.get("beta", 1.0)), int(kw.get("gamma", 0)),
                               int(kw.get("batch", 0)), int(kw.get("cand_cap", 0)),
                               int(kw.get("sample_tiles", 0)), 0)
    qs = dq.struct()
    rc = lib.sindi_search_noalloc(idx._h, ctypes.byref(qs), int(k), ctypes.byref(p),
                                  ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(sc.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, ids.cpu().numpy(), sc.cpu().numpy()


def _same(sindi, idx, queries, k, **kw):
    dq = sindi.DeviceCsr.from_host(queries)
    rc, ids, sc = _noalloc(sindi, idx, dq, k, **kw)
    assert rc == 0, sindi._lib.load().sindi_last_error()
    r_ids, r_sc = idx.search(dq, k, **kw)
    assert np.array_equal(ids, r_ids.cpu().numpy())
    assert sc.tobytes() == r_sc.cpu().numpy().tobytes()


def test_noalloc_equals_search_on_two_calls(sindi):
    corpus = synth.generate(60_000, 3_000, nnz=("poisson", 50.0), seed=17)
    big = synth.generate(600, 3_000, nnz=("poisson", 20.0), seed=17, stream=1)
    small = synth.generate(37, 3_000, nnz=("poisson", 9.0), seed=18, stream=1)
    idx = sindi.Index(corpus, alpha=0.5, window=20_000, value_dtype="f16", tile=4_096)
    _same(sindi, idx, big, 50, gamma=300)
    _same(sindi, idx, small, 10, gamma=100)


def test_noalloc_retry_passes_run_in_the_array(sindi):
    """One sample tile and candidate buffers of gamma entries: the sampled pass misses, the
    pass over every tile overflows, the keep-all pass resolves (all in the static array)."""
    corpus = synth.generate(30_000, 2_000, nnz=("poisson", 40.0), seed=19)
    queries = synth.generate(48, 2_000, nnz=("poisson", 12.0), seed=19, stream=1)
    idx = sindi.Index(corpus, alpha=0.5, window=7_000, tile=2_048)
    _same(sindi, idx, queries, 20, gamma=200, sample_tiles=1, cand_cap=200)
    _same(sindi, idx, queries.take_rows(np.arange(5)), 20, gamma=200, sample_tiles=1,
          cand_cap=4_096)


def test_noalloc_refuses_what_does_not_fit(sindi):
    corpus = synth.generate(5_000, 500, nnz=("poisson", 10.0), seed=20)
    idx = sindi.Index(corpus, alpha=1.0, window=5_000)
    lib = sindi._lib.load()
    # more query entries than the array holds beside one pass
    n = 9_000_000
    q = synth.Csr(np.arange(n + 1, dtype=np.int64) * 4, np.tile(np.arange(4, dtype=np.int32), n),
                  np.ones(4 * n, np.float32), 500)
    dq = sindi.DeviceCsr.from_host(q)
    rc, ids, _ = _noalloc(sindi, idx, dq, 5, gamma=5)
    assert rc == sindi._lib.SINDI_E_INVALID
    assert b"scratch" in lib.sindi_last_error()
    assert (ids == -7).all()  # outputs untouched
    # host queries are refused (the call reads device memory only)
    h = sindi._HostCsr(synth.generate(3, 500, nnz=("poisson", 5.0), seed=20, stream=1))
    qs = h.struct()
    out = torch.empty((3, 5), dtype=torch.int64, device="cuda")
    outs = torch.empty((3, 5), dtype=torch.float32, device="cuda")
    rc = lib.sindi_search_noalloc(idx._h, ctypes.byref(qs), 5, None,
                                  ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(outs.data_ptr()),
                                  None)
    assert rc == sindi._lib.SINDI_E_INVALID and b"device memory" in lib.sindi_last_error()
