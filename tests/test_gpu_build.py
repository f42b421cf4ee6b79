"""The index built on the device holds exactly the oracle's Alg. 3 pruning followed by its
Alg. 1 lists (every storage type, MRP and VNP, rows longer than one wave's 512 entries,
signed values, explicit zeros, empty rows), equals the host build bit for bit in the tiled
4-slot-aligned layout, and rejects what the host rejects."""
import numpy as np
import pytest

import oracle
import synth
from parity import check_bank_order, check_layout_against_oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sindi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_08395_amd as s
    s._lib.load()
    return s


def _same_index(a, b):
    ra, rb = a.export(raw=True), b.export(raw=True)
    for key in ("tile_doc", "tile_post", "term_goff", "post_doc"):
        assert np.array_equal(ra[key], rb[key]), key
    va, vb = ra["post_val"], rb["post_val"]
    assert np.array_equal(va.view(np.uint8), vb.view(np.uint8)), "post_val"
    ia, ib = a.info(), b.info()
    for key in ("n_postings", "n_slots", "n_tiles", "tile_max", "n_windows"):
        assert ia[key] == ib[key], key


def _same_search(a, b, queries, k=20, gamma=200):
    ia, sa = a.search(queries, k, gamma=gamma)
    ib, sb = b.search(queries, k, gamma=gamma)
    assert torch.equal(ia, ib)
    assert torch.equal(sa.view(torch.int32), sb.view(torch.int32))


def _oracle_keep(corpus, prune, kw):
    if prune == "mrp":
        return oracle.mass_prune(corpus, kw["alpha"])
    return oracle.vnp_prune(corpus, kw["vn"])


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("prune,kw", [("mrp", dict(alpha=0.5)), ("mrp", dict(alpha=1.0)),
                                      ("vnp", dict(vn=17))])
def test_device_build_equals_host_build(sindi, dtype, prune, kw):
    corpus = synth.generate(30_011, 2_000, nnz=("poisson", 40.0), seed=11)
    queries = synth.generate(32, 2_000, nnz=("poisson", 12.0), seed=11, stream=1)
    h = sindi.Index(corpus, window=7_000, value_dtype=dtype, tile=2_048, prune=prune, **kw)
    g = sindi.Index(corpus, window=7_000, value_dtype=dtype, tile=2_048, prune=prune, gpu_build=True, **kw)
    _same_index(h, g)
    check_bank_order(g.export(raw=True), g.export())
    _same_search(h, g, queries)
    # Alg. 3 then Alg. 1 as the oracle computes them
    keep = _oracle_keep(corpus, prune, kw)
    assert g.info()["n_postings"] == int(keep.sum())
    check_layout_against_oracle(g.export(), oracle.build_index(corpus, 7_000, keep), 2_000, 7_000,
                                dtype)


def test_device_build_vocabulary_over_one_pass(sindi):
    """A vocabulary of 100,000 terms (uniform term ids): the list counts and the ordered fill
    each take four passes of 32,768 terms per tile."""
    corpus = synth.generate(20_000, 100_000, nnz=("poisson", 60.0), terms=("uniform",), seed=21)
    queries = synth.generate(24, 100_000, nnz=("poisson", 20.0), terms=("uniform",), seed=21,
                             stream=1)
    assert corpus.indices.max() >= 3 * 32_768
    for dtype in ("f16", "f32"):
        h = sindi.Index(corpus, alpha=0.5, window=10_000, value_dtype=dtype, tile=5_000)
        g = sindi.Index(corpus, alpha=0.5, window=10_000, value_dtype=dtype, tile=5_000,
                        gpu_build=True)
        _same_index(h, g)
        _same_search(h, g, queries)


def test_device_build_degenerate_corpora(sindi):
    """No documents, documents with no entries, and a single document: the device build
    equals the host build, and search returns what the host-built index returns."""
    cases = {
        "no documents": synth.Csr(np.array([0]), np.zeros(0, np.int32), np.zeros(0, np.float32), 50),
        "empty rows": synth.Csr(np.zeros(6, np.int64), np.zeros(0, np.int32),
                                np.zeros(0, np.float32), 50),
        "one document": synth.Csr(np.array([0, 3]), np.array([2, 7, 40], np.int32),
                                  np.array([0.5, -1.5, 2.0], np.float32), 50),
    }
    queries = synth.Csr(np.array([0, 2, 2]), np.array([7, 40], np.int32),
                        np.array([1.0, 0.25], np.float32), 50)
    for name, c in cases.items():
        h = sindi.Index(c, alpha=0.5, window=4)
        g = sindi.Index(c, alpha=0.5, window=4, gpu_build=True)
        _same_index(h, g)
        _same_search(h, g, queries, k=3, gamma=3)
        check_layout_against_oracle(g.export(), oracle.build_index(c, 4, oracle.mass_prune(c, 0.5)),
                                    50, 4, "f32")


def test_device_build_long_rows_signed_zeros_and_empty_rows(sindi):
    """Rows up to 3,000 entries (the one-workgroup path), negative values, explicit zeros
    (not entries) and empty rows."""
    rng = np.random.default_rng(5)
    corpus = synth.random_csr(rng, 4_000, 6_000, 60, signed=True)
    long_ = synth.random_csr(rng, 40, 6_000, 3_000, signed=True, min_nnz=600)
    indptr = np.concatenate([corpus.indptr, corpus.indptr[-1] + long_.indptr[1:]])
    c = synth.Csr(indptr, np.concatenate([corpus.indices, long_.indices]),
                  np.concatenate([corpus.values, long_.values]), 6_000)
    c.values[::11] = 0.0
    lens = np.diff(c.indptr)
    assert (lens > 512).sum() >= 30 and (lens == 0).any()
    queries = synth.random_csr(rng, 24, 6_000, 40, signed=True, min_nnz=1)
    for prune, kw in (("mrp", dict(alpha=0.6)), ("vnp", dict(vn=300)), ("mrp", dict(alpha=1.0))):
        for dtype in ("f32", "bf16"):
            h = sindi.Index(c, window=1_500, tile=700, prune=prune, value_dtype=dtype, **kw)
            g = sindi.Index(c, window=1_500, tile=700, prune=prune, value_dtype=dtype,
                            gpu_build=True, **kw)
            _same_index(h, g)
            _same_search(h, g, queries)
            # against the oracle: rows over 512 entries take the one-workgroup pruning path;
            # explicit zeros are no entries and never kept; negative values rank by |x|
            keep = _oracle_keep(c, prune, kw)
            assert not keep[c.values == 0.0].any()
            assert keep[np.repeat(lens > 512, lens)].sum() > 0
            assert g.info()["n_postings"] == int(keep.sum())
            check_layout_against_oracle(g.export(), oracle.build_index(c, 1_500, keep), 6_000,
                                        1_500, dtype)


def test_device_build_from_device_corpus(sindi):
    corpus = synth.generate(12_000, 3_000, nnz=("poisson", 50.0), seed=3)
    queries = synth.generate(16, 3_000, nnz=("poisson", 10.0), seed=3, stream=1)
    h = sindi.Index(corpus, alpha=0.5, window=5_000, value_dtype="f16", tile=1_024)
    g = sindi.Index(sindi.DeviceCsr.from_host(corpus), alpha=0.5, window=5_000, value_dtype="f16",
                    tile=1_024, gpu_build=True)
    _same_index(h, g)
    _same_search(h, g, queries)
    check_layout_against_oracle(g.export(), oracle.build_index(corpus, 5_000,
                                                               oracle.mass_prune(corpus, 0.5)),
                                3_000, 5_000, "f16")


def test_device_build_rejections(sindi):
    E = sindi.SindiError
    bad = synth.Csr(np.array([0, 2, 3]), np.array([5, 1, 7], np.int32),
                    np.array([1.0, 2.0, 3.0], np.float32), 10)
    with pytest.raises(E, match="order|ascending"):
        sindi.Index(sindi.DeviceCsr.from_host(bad), alpha=0.5, window=10, gpu_build=True)
    big = synth.Csr(np.array([0, 9_000]), np.arange(9_000, dtype=np.int32),
                    np.ones(9_000, np.float32), 9_000)
    with pytest.raises(E, match="more than 8192"):
        sindi.Index(big, alpha=0.5, window=10, gpu_build=True)
    over = synth.Csr(np.array([0, 2]), np.array([0, 1], np.int32),
                     np.array([7e4, 1.0], np.float32), 4)
    with pytest.raises(E, match="overflows") as ei:
        sindi.Index(over, alpha=1.0, window=10, value_dtype="f16", gpu_build=True)
    assert ei.value.code == sindi._lib.SINDI_E_RANGE
    with pytest.raises(E, match="list pruning"):
        sindi.Index(bad, window=10, prune="lp", list_len=3, gpu_build=True)
    with pytest.raises(E, match="gpu_build"):
        sindi.Index(sindi.DeviceCsr.from_host(over), alpha=1.0, window=10)


def test_device_corpus_structure_check(sindi):
    """The device's check of a corpus in HBM (Def. 1: row pointers, term id range, ascending
    ids inside every row, finite values) over corpora of many rows, the faults placed in rows
    far from the first; ids that fall from one row to the next are no fault."""
    E = sindi.SindiError
    rng = np.random.default_rng(9)
    n_rows, n_cols = 45, 64
    rows = [np.sort(rng.choice(n_cols, size=int(rng.integers(0, 9)), replace=False)) for _ in range(n_rows)]
    rows[17] = np.array([60, 61, 62], np.int64)  # then row 18 starts low: no fault
    rows[18] = np.array([0, 1], np.int64)
    indptr = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    good = synth.Csr(indptr, np.concatenate(rows).astype(np.int32),
                     rng.lognormal(0, 0.8, size=int(indptr[-1])).astype(np.float32), n_cols)
    h = sindi.Index(good, alpha=0.5, window=20)
    g = sindi.Index(sindi.DeviceCsr.from_host(good), alpha=0.5, window=20, gpu_build=True)
    _same_index(h, g)

    def faulty(change):
        c = synth.Csr(good.indptr.copy(), good.indices.copy(), good.values.copy(), n_cols)
        change(c)
        return sindi.DeviceCsr.from_host(c)

    cases = {
        # id out of range on the last entry of a row (so the order inside the row holds)
        "0x2": lambda c: c.indices.__setitem__(
            int(c.indptr[next(r for r in range(33, n_rows) if c.indptr[r + 1] > c.indptr[r]) + 1]) - 1,
            n_cols),
        "0x8": lambda c: c.values.__setitem__(int(c.indptr[-1]) - 1, np.inf),  # non-finite
        "0x1": lambda c: c.indptr.__setitem__(30, c.indptr[31] + 1),  # pointers fall
    }
    for flag, change in cases.items():
        with pytest.raises(E, match="flags " + flag):
            sindi.Index(faulty(change), alpha=0.5, window=20, gpu_build=True)
    # ids not ascending inside a row past the first wave's 16 rows
    k = next(r for r in range(20, n_rows) if good.indptr[r + 1] - good.indptr[r] >= 2)
    c = synth.Csr(good.indptr.copy(), good.indices.copy(), good.values.copy(), n_cols)
    a = int(c.indptr[k])
    c.indices[a], c.indices[a + 1] = c.indices[a + 1], c.indices[a]
    with pytest.raises(E, match="flags 0x4"):
        sindi.Index(sindi.DeviceCsr.from_host(c), alpha=0.5, window=20, gpu_build=True)


def test_device_build_every_row_width_value_range_and_ties(sindi):
    """Rows of every width the pruning kernel sorts in registers (up to 64, 128, 256 and 512
    entries) and beyond (the one-workgroup path, and documents longer than the fill's batch of
    4,096 entries), rows whose values span more than 2^20 (their mass sums run one after
    another) beside rows of nearby values (summed by a scan that no rounding touches), and
    equal magnitudes (Def. 6: the lower term id first): the oracle's Alg. 3 and Alg. 1."""
    rng = np.random.default_rng(17)
    vocab = 20_000
    lens = np.concatenate([rng.integers(0, 65, 300), rng.integers(65, 129, 200),
                           rng.integers(129, 257, 150), rng.integers(257, 513, 120),
                           rng.integers(513, 4_000, 12), rng.integers(4_097, 8_193, 6), [0, 1, 512, 8_192]])
    rng.shuffle(lens)
    rows_i, rows_v = [], []
    for r, n in enumerate(lens):
        ids = np.sort(rng.choice(vocab, size=int(n), replace=False)).astype(np.int32)
        if r % 5 == 0:  # wide range: magnitudes from 1e-12 to 1e12
            v = 10.0 ** rng.uniform(-12, 12, size=int(n))
        elif r % 5 == 1:  # few distinct magnitudes: many ties
            v = rng.choice([0.25, 0.5, 1.0, 3.0], size=int(n))
        else:
            v = rng.lognormal(0.0, 0.8, size=int(n))
        v = (v * rng.choice([-1.0, 1.0], size=int(n))).astype(np.float32)
        rows_i.append(ids)
        rows_v.append(v)
    indptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    c = synth.Csr(indptr, np.concatenate(rows_i), np.concatenate(rows_v), vocab)
    queries = synth.random_csr(rng, 16, vocab, 30, signed=True, min_nnz=1)
    for prune, kw in (("mrp", dict(alpha=0.5)), ("mrp", dict(alpha=0.93)), ("vnp", dict(vn=200))):
        h = sindi.Index(c, window=300, tile=150, prune=prune, value_dtype="f32", **kw)
        g = sindi.Index(c, window=300, tile=150, prune=prune, value_dtype="f32", gpu_build=True, **kw)
        _same_index(h, g)
        _same_search(h, g, queries)
        keep = _oracle_keep(c, prune, kw)
        assert g.info()["n_postings"] == int(keep.sum())
        check_layout_against_oracle(g.export(), oracle.build_index(c, 300, keep), vocab, 300, "f32")
