"""Build libntc.so for gfx950 in-tree with hipcc.

Usage: ``python -m paper_2109_09534_amd.build`` (or ``build()`` from Python).
Every call recompiles: each source to an object, in parallel, then one link.
Packed FP32 instructions are disabled for the device code.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libntc.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["ntc_host.cpp", "ntc_pool.cpp", "ntc_kernels.hip", "ntc_kernels_wide.hip", "ntc_aux.hip",
           "ntc_csr.hip"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libntc.so")


def build(verbose: bool = False, out_path: str = LIB, defines=()) -> str:
    """Compile every source to an object (in parallel: each file's device code
    is self-contained), then link the shared library."""
    flags = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", f"-I{INCLUDE}", f"-I{CSRC}"] + [f"-D{d}" for d in defines]
    tmp = tempfile.mkdtemp(prefix="ntc_build_")
    try:
        jobs = []
        for src in SOURCES:
            obj = os.path.join(tmp, src + ".o")
            lang = ["-x", "hip"] if src.endswith(".cpp") else []
            jobs.append(([HIPCC] + flags + ["-c"] + lang + [os.path.join(CSRC, src), "-o", obj], obj))
        workers = max(1, min(len(jobs), os.cpu_count() or 1))
        with concurrent.futures.ThreadPoolExecutor(workers) as ex:
            for f in [ex.submit(_run, cmd, verbose) for cmd, _ in jobs]:
                f.result()
        out = out_path + ".tmp"
        _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out] + [o for _, o in jobs] + ["-lrocprofiler-sdk-roctx", "-lpthread"],
             verbose)
        os.replace(out, out_path)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return out_path


if __name__ == "__main__":
    print(build(verbose=True))
