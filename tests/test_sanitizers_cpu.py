"""CPU: the oracle and the library's host code under AddressSanitizer and UBSan.

The oracle is rebuilt with -fsanitize=address,undefined and every oracle pin
runs against that build (gcc's ASan runtime preloaded into a child Python).
The library is rebuilt with both sanitizers on its host code and
csrc/host_check.cpp drives every validation and error path of the C ABI
(without a GPU; on a GPU machine the same executable also runs every entry
point on small boxes).  Any sanitizer report fails the run.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_pins_under_asan_ubsan(tmp_path):
    import oracle
    lib = oracle.build_sanitized(str(tmp_path / "liboracle_san.so"))
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", MD_ORACLE_LIB=lib, OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=1200)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


def test_library_host_code_under_asan_ubsan():
    from paper_1210_3450_amd import build
    exe = build.build_host_check()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=600, cwd=str(ROOT))
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "checks" in r.stdout and "passed" in r.stdout
