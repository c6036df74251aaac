"""The library's host code (ntc_host.cpp: argument checks, the per-mode CSR
build with its threads, the row schedule, the host sampler and the byte
counts) built with gcc's sanitizers and driven with no device by
tests/host_sanitize_driver.cpp.  The device launchers are stubs that abort,
and every array handed to the library has exactly its declared size, so an
invalid access, undefined operation, leak or data race fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2109_09534_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

SANITIZERS = {
    "address_undefined": ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"],
    "thread": ["-fsanitize=thread"],
}


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(os.path.join(ROCM, "include", "hip")),
                    reason="g++ or the HIP headers are not installed")
@pytest.mark.parametrize("kind", list(SANITIZERS))
def test_host_code_under_sanitizers(kind, tmp_path):
    san = SANITIZERS[kind] + ["-fno-omit-frame-pointer"]
    flags = ["-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", f"-I{ROOT}/include",
             f"-I{CSRC}"] + san
    objs = []
    for src in (os.path.join(CSRC, "ntc_host.cpp"), os.path.join(ROOT, "tests", "host_sanitize_driver.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = subprocess.run(["g++"] + flags + ["-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(obj)
    exe = str(tmp_path / "host_sanitized")
    libs = [f"-L{ROCM}/lib", "-lamdhip64", "-lrocprofiler-sdk-roctx", "-lpthread"]
    r = subprocess.run(["g++"] + san + objs + libs + ["-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1", LD_LIBRARY_PATH=f"{ROCM}/lib:" + os.environ.get("LD_LIBRARY_PATH", ""))
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and "sanitized host code: ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
    for marker in ("runtime error", "AddressSanitizer", "LeakSanitizer", "ThreadSanitizer"):
        assert marker not in r.stderr, r.stderr[-4000:]
