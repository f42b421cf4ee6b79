import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU cases")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def csr_from_dict_rows(rows, n_rows, n_cols):
    """CSR (float32 values) from {row: {col: value}} dicts."""
    import synth
    indptr = [0]
    idx, val = [], []
    for r in range(n_rows):
        d = rows.get(str(r), rows.get(r, {}))
        items = sorted((int(c), float(v)) for c, v in d.items())
        idx += [c for c, _ in items]
        val += [v for _, v in items]
        indptr.append(len(idx))
    return synth.Csr(np.array(indptr, np.int64), np.array(idx, np.int32),
                     np.array(val, np.float32), n_cols)


def dense(csr, dtype=np.float64):
    m = np.zeros((csr.n_rows, csr.n_cols), dtype=dtype)
    for r in range(csr.n_rows):
        i, v = csr.row(r)
        m[r, i] = v
    return m


def rank_order(scores, ids=None):
    """Indices sorted by (score desc, id asc)."""
    scores = np.asarray(scores)
    ids = np.arange(scores.shape[0]) if ids is None else np.asarray(ids)
    return np.lexsort((ids, -scores))


@pytest.fixture(scope="session")
def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False
