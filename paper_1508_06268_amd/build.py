"""Build librfim.so in-tree with hipcc for gfx950.

    python -m paper_1508_06268_amd.build

Every HIP source is compiled with -ffp-contract=off (energies and exchange
decisions are evaluated exactly as written) and without packed FP32
instructions.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "librfim.so")
SOURCES = ["rfim_api.hip", "rfim_kernels.hip", "rfim_measure.hip", "rfim_noalloc.hip"]
HEADERS = [os.path.join(CSRC, "rfim_internal.h"), os.path.join(INCLUDE, "rfim.h")]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags() -> list:
    return ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-I" + INCLUDE, "-I" + CSRC]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + flags() + ["-shared", "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building librfim.so")
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    newest = max(os.path.getmtime(p) for p in [os.path.join(CSRC, s) for s in SOURCES] + HEADERS)
    return os.path.getmtime(LIB) < newest


if __name__ == "__main__":
    print(build(verbose=True))
