"""Build libntc.so for gfx950 in-tree with hipcc.

Usage: ``python -m paper_2109_09534_amd.build`` (or ``build()`` from Python).
Every call recompiles.  Host and device code are compiled together; packed
FP32 instructions are disabled for the device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libntc.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["ntc_host.cpp", "ntc_pool.cpp", "ntc_kernels.hip", "ntc_kernels_wide.hip", "ntc_aux.hip",
           "ntc_csr.hip"]


def build(verbose: bool = False, out_path: str = LIB, defines=()) -> str:
    out = out_path + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-function",
           f"-I{INCLUDE}", f"-I{CSRC}", "-o", out]
    srcs = []
    for s in SOURCES:
        p = os.path.join(CSRC, s)
        srcs += (["-x", "hip", p] if s.endswith(".cpp") else [p])
    cmd += [f"-D{d}" for d in defines]
    cmd += srcs
    cmd += ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libntc.so")
    os.replace(out, out_path)
    return out_path


if __name__ == "__main__":
    print(build(verbose=True))
