"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds the sanitizer variant of the library (host code instrumented, see
paper_2106_04649_amd/build.py) and a C driver (tests/host_check.c) that calls
every entry point with arguments its validation refuses before any GPU work;
the run must end cleanly with no sanitizer report.  Needs no GPU."""

import os
import shutil
import subprocess

import pytest

from paper_2106_04649_amd import build

pytestmark = pytest.mark.slow

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _clang():
    for cand in ("/opt/rocm/llvm/bin/clang", shutil.which("clang")):
        if cand and os.path.exists(cand):
            return cand
    pytest.skip("no clang for the sanitizer build")


def test_host_paths_are_clean_under_asan_and_ubsan(tmp_path):
    clang = _clang()
    lib = build.build_sanitized()
    exe = tmp_path / "host_check"
    cmd = [clang, "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "host_check.c"),
           "-L", os.path.dirname(lib), "-lmk_asan", f"-Wl,-rpath,{os.path.dirname(lib)}", "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    out = res.stdout + res.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out
    assert res.returncode == 0, out
    assert "all checks passed" in res.stdout
