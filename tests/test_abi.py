"""The C ABI library: loads, exports every declared symbol, validates on the host (no GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "sindi.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sindi_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2509_08395_amd import _lib
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTS)
    assert b"gfx950" in lib.sindi_version()


def test_probe_library_exports_its_header_and_checks_arguments():
    """The LDS microbenchmark library exports exactly what include/sindi_probe.h declares
    and refuses bad arguments before any device work."""
    import ctypes as C
    from paper_2509_08395_amd import _lib
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "sindi_probe.h")).read(),
                  flags=re.S)
    names = sorted(set(re.findall(r"\b(sindi_[a-z_]+)\s*\(", text)))
    assert names == sorted(_lib.PROBE_EXPORTS)
    lib = _lib.load_probe()
    ms, upd = C.c_double(), C.c_double()
    for args in ((2, 1, 1, 1), (0, -1, 1, 1), (0, 1, 0, 1), (0, 1, 1, 0)):
        assert lib.sindi_probe_lds_add(*args, None, C.byref(ms), C.byref(upd)) != 0


def test_no_cpu_fallback_in_package():
    """The product path has no route to the oracle or to a CPU implementation."""
    pkg = os.path.join(ROOT, "paper_2509_08395_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "liboracle" not in src, f


def _csr_struct(indptr, indices, values, n_cols):
    from paper_2509_08395_amd import _lib
    indptr = np.ascontiguousarray(indptr, np.int64)
    indices = np.ascontiguousarray(indices, np.int32)
    values = np.ascontiguousarray(values, np.float32)
    s = _lib.SindiCsr(indptr.shape[0] - 1, n_cols, int(indptr[-1]), indptr.ctypes.data,
                      indices.ctypes.data, values.ctypes.data, 0, 0)
    return s, (indptr, indices, values)


@pytest.mark.parametrize("case,msg", [
    (([0, 2], [3, 1], [1.0, 1.0]), "ascending"),
    (([0, 2], [1, 1], [1.0, 1.0]), "ascending"),
    (([0, 1], [10], [1.0]), "out of range"),
    (([0, 1], [-1], [1.0]), "out of range"),
    (([0, 1], [1], [np.nan]), "non-finite"),
    (([0, 1], [1], [np.inf]), "non-finite"),
    (([0, 2, 1], [1, 2], [1.0, 1.0]), "indptr"),
])
def test_build_rejects_malformed_corpus_before_any_device_work(case, msg):
    from paper_2509_08395_amd import _lib
    lib = _lib.load()
    s, keep = _csr_struct(*case, n_cols=5)
    p = _lib.SindiBuildParams(0.5, 10, 0, 0)
    h = ctypes.c_void_p()
    rc = lib.sindi_build(ctypes.byref(s), ctypes.byref(p), None, ctypes.byref(h))
    assert rc == _lib.SINDI_E_INVALID
    err = lib.sindi_last_error().decode()
    assert msg in err or "indptr" in err or "monotone" in err, err
    assert not h.value


@pytest.mark.parametrize("alpha,window,dtype,tile", [
    (0.0, 10, 0, 0), (1.5, 10, 0, 0), (0.5, 0, 0, 0), (0.5, 10, 7, 0), (0.5, 10, 0, 70000)])
def test_build_rejects_bad_parameters(alpha, window, dtype, tile):
    from paper_2509_08395_amd import _lib
    lib = _lib.load()
    s, keep = _csr_struct([0, 1], [1], [1.0], n_cols=5)
    p = _lib.SindiBuildParams(alpha, window, dtype, tile)
    h = ctypes.c_void_p()
    assert lib.sindi_build(ctypes.byref(s), ctypes.byref(p), None, ctypes.byref(h)) == _lib.SINDI_E_INVALID


def test_null_arguments_are_errors_not_crashes():
    from paper_2509_08395_amd import _lib
    lib = _lib.load()
    assert lib.sindi_build(None, None, None, None) == _lib.SINDI_E_INVALID
    assert lib.sindi_search(None, None, 10, None, None, None, None) == _lib.SINDI_E_INVALID
    assert lib.sindi_index_get_info(None, None) == _lib.SINDI_E_INVALID
    assert lib.sindi_score_forward(None, None, None, 0, None, None, None) == _lib.SINDI_E_INVALID
    assert lib.sindi_score_backward(None, None, None, 0, None, None, None, None,
                                    None) == _lib.SINDI_E_INVALID
    lib.sindi_index_free(None)


def test_server_null_arguments_are_errors_not_crashes():
    from paper_2509_08395_amd import _lib
    lib = _lib.load()
    h = ctypes.c_void_p()
    t = ctypes.c_int64()
    assert lib.sindi_server_create(None, None, ctypes.byref(h)) == _lib.SINDI_E_INVALID
    assert lib.sindi_server_submit(None, None, None, 0, 10, ctypes.byref(t)) == _lib.SINDI_E_INVALID
    assert lib.sindi_server_wait(None, 0, None, None, None, 0.0) == _lib.SINDI_E_INVALID
    assert lib.sindi_server_replay(None, None, None, None, None, None, None) == _lib.SINDI_E_INVALID
    assert lib.sindi_server_get_stats(None, None) == _lib.SINDI_E_INVALID
    lib.sindi_server_destroy(None)


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors have the C structs' sizes and field offsets (gcc on the header)."""
    import shutil
    import subprocess
    from paper_2509_08395_amd import _lib
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    structs = {"sindi_csr": _lib.SindiCsr, "sindi_build_params": _lib.SindiBuildParams,
               "sindi_search_params": _lib.SindiSearchParams,
               "sindi_index_info": _lib.SindiIndexInfo,
               "sindi_server_params": _lib.SindiServerParams,
               "sindi_server_stats": _lib.SindiServerStats, "sindi_profile": _lib.SindiProfile}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sindi.h"', 'int main(void) {']
    for c, py in structs.items():
        lines.append(f'printf("{c} size %zu\\n", sizeof({c}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{c} {f} %zu\\n", offsetof({c}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src),
                           "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)]).decode().splitlines():
        c, f, v = line.split()
        got[(c, f)] = int(v)
    for c, py in structs.items():
        assert got[(c, "size")] == ctypes.sizeof(py), c
        for f, _ in py._fields_:
            assert got[(c, f)] == getattr(py, f).offset, (c, f)


@pytest.mark.parametrize("prune,vn,list_len", [(7, 0, 0), (-1, 0, 0), (1, 0, 0), (2, 0, 0), (3, 5, 0)])
def test_build_rejects_bad_pruning_parameters(prune, vn, list_len):
    from paper_2509_08395_amd import _lib
    lib = _lib.load()
    s, keep = _csr_struct([0, 1], [1], [1.0], n_cols=5)
    p = _lib.SindiBuildParams(0.5, 10, 0, 0, prune, vn, list_len)
    h = ctypes.c_void_p()
    assert lib.sindi_build(ctypes.byref(s), ctypes.byref(p), None, ctypes.byref(h)) == _lib.SINDI_E_INVALID
    assert not h.value


def test_score_arguments_are_checked_before_the_library_is_called():
    """The score kernels index cand, grad and the gradient buffers by the query count, the
    candidate count and the corpus size, which the C side cannot see: the binding refuses
    mis-shaped or misplaced tensors first (here CPU tensors, so nothing reaches a GPU)."""
    import torch
    import paper_2509_08395_amd as sindi
    idx = sindi.Index.__new__(sindi.Index)
    idx._h, idx.nnz, idx.n_cols = None, 10, 5
    dq = sindi.DeviceCsr(torch.zeros(3, dtype=torch.int64), torch.zeros(0, dtype=torch.int32),
                         torch.zeros(0), 5)
    E = sindi.SindiError
    with pytest.raises(E, match="DeviceCsr"):
        idx.score(object(), torch.zeros((2, 3), dtype=torch.int64))
    with pytest.raises(E, match="cand"):
        idx.score(dq, torch.zeros((2, 3), dtype=torch.int64))
    with pytest.raises(E, match="cand"):
        idx.score_backward(dq, torch.zeros((3, 3), dtype=torch.int64), torch.zeros((3, 3)))
