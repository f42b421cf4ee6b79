"""bench.py's host-side contract: the counter summary it reads, and its one-GPU limit."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNELS = os.path.join(ROOT, "paper_2509_08395_amd", "csrc", "sindi_kernels.hip")
DEFAULT = {"workload": "splade-8.8m", "value_storage": "f16", "batch": 1, "tile": 12500,
           "n_queries": 7000, "n_docs": 8800000, "alpha": 0.5, "beta": 1.0}


def test_code_hash_ignores_comments_and_layout_only(tmp_path):
    a = tmp_path / "a.hip"
    a.write_text("int f(int x) {\n  return x + 1; // one\n}\n/* note */\n")
    b = tmp_path / "b.hip"
    b.write_text("int f(int x)   { return x + 1;   /* a longer\n comment */ }\n")
    c = tmp_path / "c.hip"
    c.write_text("int f(int x) { return x + 2; }\n")
    assert bench.kernel_code_sha256(a) == bench.kernel_code_sha256(b)
    assert bench.kernel_code_sha256(a) != bench.kernel_code_sha256(c)


def test_committed_counter_summary_matches_the_kernel_code():
    """The profile summary under profiles/ was taken on the kernel code as it stands, so the
    default bench run reports measured HBM traffic (retake the profile after a code change)."""
    traffic = bench.measured_traffic(DEFAULT)
    assert traffic is not None
    # beyond-L2 bytes of one scoring launch: well under the 657 GB of algorithmic list bytes
    assert 1e11 < traffic < 6.6e11


def test_counter_summary_is_not_used_for_another_configuration():
    for key, val in (("tile", 10000), ("batch", 2), ("n_queries", 1000), ("value_storage", "f32"),
                     ("alpha", 0.3), ("beta", 0.8)):
        cfg = dict(DEFAULT, **{key: val})
        assert bench.measured_traffic(cfg) is None, key


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_coarse_terms_counted_are_the_beta_mass_prefix():
    """The algorithmic bytes of a pruned-query run count the beta-mass terms (Sec. 4.1) the
    scoring pass reads: the same terms the oracle's mass pruning keeps, and every term at
    beta = 1."""
    import numpy as np
    import oracle
    import synth
    q = synth.generate(300, 5_000, nnz=("poisson", 30.0), seed=21)
    assert bench.coarse_queries(q, 1.0) is q
    rows = np.repeat(np.arange(q.n_rows), np.diff(q.indptr))
    for beta in (0.3, 0.8, 0.95):
        c = bench.coarse_queries(q, beta)
        keep = oracle.mass_prune(q, beta).astype(bool)
        assert np.array_equal(np.diff(c.indptr), np.bincount(rows[keep], minlength=q.n_rows))
        assert np.array_equal(c.indices, q.indices[keep])
