"""The CPU oracle built with gcc's AddressSanitizer and
UndefinedBehaviorSanitizer (host code only; no GPU code is built here) and
run through every entry point on small problems (oracle/sanitize_check.c):
no invalid access, leak or undefined operation."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "sanitize_check")
    src = os.path.join(ROOT, "oracle", "sanitize_check.c")
    flags = ["-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    subprocess.run(["gcc"] + flags + ["-I", os.path.join(ROOT, "oracle"), "-o", exe, src, "-lm"], check=True)
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle sanitizer run: ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
