"""ctypes declarations of the C ABI in include/sindi.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsindi.so")

SINDI_OK, SINDI_E_INVALID, SINDI_E_RANGE, SINDI_E_OOM, SINDI_E_HIP, SINDI_E_BUSY, SINDI_E_INTERNAL = (
    0, -1, -2, -3, -4, -5, -6)
DTYPES = {"f32": 0, "f16": 1, "bf16": 2}
VALUE_BYTES = {0: 4, 1: 2, 2: 2}

P = ctypes.c_void_p


class SindiCsr(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("indptr", P), ("indices", P), ("values", P), ("on_device", ctypes.c_int32),
                ("reserved_", ctypes.c_int32)]


class SindiBuildParams(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("window", ctypes.c_int64),
                ("value_dtype", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("prune", ctypes.c_int32), ("vn", ctypes.c_int32), ("list_len", ctypes.c_int64),
                ("gpu_build", ctypes.c_int32), ("reserved_", ctypes.c_int32)]


PRUNE = {"mrp": 0, "vnp": 1, "lp": 2, "mrp+lp": 3}


class SindiSearchParams(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("gamma", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("cand_cap", ctypes.c_int32), ("sample_tiles", ctypes.c_int32),
                ("tile_run", ctypes.c_int32), ("schedule", ctypes.c_int32)]


class SindiIndexInfo(ctypes.Structure):
    _fields_ = [("n_docs", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("n_postings", ctypes.c_int64), ("window", ctypes.c_int64),
                ("n_windows", ctypes.c_int64), ("n_tiles", ctypes.c_int64),
                ("tile_max", ctypes.c_int32), ("value_dtype", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("device_bytes", ctypes.c_int64),
                ("n_slots", ctypes.c_int64), ("prune", ctypes.c_int32), ("vn", ctypes.c_int32),
                ("list_len", ctypes.c_int64)]


class SindiServerParams(ctypes.Structure):
    _fields_ = [("max_inflight", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("k_max", ctypes.c_int32), ("max_query_nnz", ctypes.c_int32),
                ("max_queue", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("search", SindiSearchParams)]


class SindiServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("retried", ctypes.c_int64),
                ("largest_batch", ctypes.c_int64), ("busy_ms", ctypes.c_double),
                ("memory_waits", ctypes.c_int64), ("arena_peak_bytes", ctypes.c_int64)]


class SindiProfile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 5), ("ms", ctypes.c_double * 5)]


PROFILE_CLASSES = ("query_prep", "accumulate_threshold", "accumulate_score", "threshold_select",
                   "finalize")

EXPORTS = ("sindi_build", "sindi_index_free", "sindi_index_get_info", "sindi_index_export",
           "sindi_search", "sindi_search_noalloc", "sindi_search_coarse", "sindi_score_forward",
           "sindi_score_backward",
           "sindi_server_create", "sindi_server_submit", "sindi_server_wait",
           "sindi_server_replay", "sindi_server_get_stats", "sindi_server_destroy",
           "sindi_profile_enable", "sindi_profile_read", "sindi_last_error", "sindi_version")


class SindiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sindi error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libsindi.so (after torch, so both share one HIP runtime).  Raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        import torch  # noqa: F401  -- loads torch's HIP runtime first
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(or python -m paper_2509_08395_amd._build)")
    lib = ctypes.CDLL(LIB_PATH)
    I32, I64 = ctypes.c_int32, ctypes.c_int64
    lib.sindi_build.argtypes = [ctypes.POINTER(SindiCsr), ctypes.POINTER(SindiBuildParams), P,
                                ctypes.POINTER(P)]
    lib.sindi_index_free.argtypes = [P]
    lib.sindi_index_free.restype = None
    lib.sindi_index_get_info.argtypes = [P, ctypes.POINTER(SindiIndexInfo)]
    lib.sindi_index_export.argtypes = [P, P, P, P, P, P]
    for f in (lib.sindi_search, lib.sindi_search_coarse, lib.sindi_search_noalloc):
        f.argtypes = [P, ctypes.POINTER(SindiCsr), I32, ctypes.POINTER(SindiSearchParams), P, P, P]
    lib.sindi_score_forward.argtypes = [P, ctypes.POINTER(SindiCsr), P, I32, P, P, P]
    lib.sindi_score_backward.argtypes = [P, ctypes.POINTER(SindiCsr), P, I32, P, P, P, P, P]
    for f in (lib.sindi_build, lib.sindi_index_get_info, lib.sindi_index_export,
              lib.sindi_search, lib.sindi_search_coarse, lib.sindi_search_noalloc,
              lib.sindi_score_forward, lib.sindi_score_backward):
        f.restype = ctypes.c_int
    lib.sindi_server_create.argtypes = [P, ctypes.POINTER(SindiServerParams), ctypes.POINTER(P)]
    lib.sindi_server_submit.argtypes = [P, P, P, I32, I32, ctypes.POINTER(I64)]
    lib.sindi_server_wait.argtypes = [P, I64, P, P, ctypes.POINTER(I64), ctypes.c_double]
    lib.sindi_server_replay.argtypes = [P, ctypes.POINTER(SindiCsr), P, P, P, P, P]
    lib.sindi_server_get_stats.argtypes = [P, ctypes.POINTER(SindiServerStats)]
    for f in (lib.sindi_server_create, lib.sindi_server_submit, lib.sindi_server_wait,
              lib.sindi_server_replay, lib.sindi_server_get_stats):
        f.restype = ctypes.c_int
    lib.sindi_server_destroy.argtypes = [P]
    lib.sindi_server_destroy.restype = None
    lib.sindi_profile_enable.argtypes = [I32]
    lib.sindi_profile_enable.restype = ctypes.c_int
    lib.sindi_profile_read.argtypes = [ctypes.POINTER(SindiProfile), I32]
    lib.sindi_profile_read.restype = ctypes.c_int
    lib.sindi_last_error.restype = ctypes.c_char_p
    lib.sindi_last_error.argtypes = []
    lib.sindi_version.restype = ctypes.c_char_p
    lib.sindi_version.argtypes = []
    _lib = lib
    return lib


PROBE_PATH = os.path.join(PKG, "libsindi_probe.so")
PROBE_EXPORTS = ("sindi_probe_lds_add",)
_probe = None


def load_probe():
    """libsindi_probe.so (include/sindi_probe.h): the LDS microbenchmark bench.py reports."""
    global _probe
    if _probe is None:
        load()  # torch's HIP runtime first, as for the search library
        if not os.path.exists(PROBE_PATH):
            raise ImportError(f"{PROBE_PATH} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(PROBE_PATH)
        lib.sindi_probe_lds_add.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32, P, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_double)]
        lib.sindi_probe_lds_add.restype = ctypes.c_int
        _probe = lib
    return _probe


def probe_lds_add(lib, op, stride, n_workgroups, iters, stream=None):
    """(milliseconds, atomic adds) of one probe launch; raises on a HIP error."""
    ms, upd = ctypes.c_double(), ctypes.c_double()
    rc = lib.sindi_probe_lds_add(int(op), int(stride), int(n_workgroups), int(iters), stream,
                                 ctypes.byref(ms), ctypes.byref(upd))
    if rc != 0:
        raise SindiError(SINDI_E_HIP, f"sindi_probe_lds_add: hipError {rc}")
    return ms.value, upd.value


def check(code):
    if code != SINDI_OK:
        raise SindiError(code, load().sindi_last_error().decode(errors="replace"))
