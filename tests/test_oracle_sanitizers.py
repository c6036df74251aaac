"""The FP64 oracle built with gcc's address and undefined-behaviour
sanitizers (host code only), driven through every entry point on small
seeded problems by oracle/sanitize_driver.c.  Any invalid access, leak or
undefined operation aborts the driver with a report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "ora_sanitized")
    san = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    build = ["gcc", "-std=c99", "-O1", "-g", "-fopenmp", "-fno-fast-math", "-ffp-contract=off"] + san + \
            ["-o", exe, os.path.join(ORACLE, "ntc_oracle.c"), os.path.join(ORACLE, "sanitize_driver.c"), "-lm"]
    r = subprocess.run(build, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and "sanitized oracle: ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
