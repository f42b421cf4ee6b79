"""Compile the HIP library ``libsindi.so`` for gfx950 (in-tree)."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libsindi.so")
PROBE_LIB = os.path.join(PKG, "libsindi_probe.so")
BUILD = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden", "-I", os.path.join(ROOT, "include"),
          "-I", CSRC, "-Wall", "-Wno-unused-result"]
DEVICE = ["--offload-arch=gfx950", "-munsafe-fp-atomics",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def compile_native(force: bool = True, verbose: bool = False) -> str:
    if not force and os.path.exists(LIB):
        return LIB
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src, extra in (("sindi_kernels.hip", DEVICE), ("sindi_build.hip", DEVICE),
                        ("sindi_host.cpp", DEVICE), ("sindi_server.cpp", DEVICE),
                        ("sindi_noalloc.hip", DEVICE)):
        obj = os.path.join(BUILD, src + ".o")
        cmd = [HIPCC, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd))
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-o", tmp, *objs, "-pthread"])
    os.replace(tmp, LIB)
    # the LDS microbenchmark bench.py reports beside the scoring pass (not the search path)
    tmp = PROBE_LIB + ".tmp"
    cmd = [HIPCC, *COMMON, *DEVICE, "-shared", os.path.join(CSRC, "sindi_probe.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, PROBE_LIB)
    return LIB


if __name__ == "__main__":
    print(compile_native(verbose=True))
