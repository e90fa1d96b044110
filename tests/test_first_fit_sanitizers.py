"""The server arena's first-fit bookkeeping (csrc/first_fit.h, host code) under the address,
undefined-behaviour and thread sanitizers: tests/cpp/first_fit_test.cpp checks random
take/give sequences against a byte map and eight threads sharing the arena through a mutex.
CPU only; needs g++."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "cpp", "first_fit_test.cpp")
INC = os.path.join(ROOT, "paper_2510_09813_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
@pytest.mark.parametrize("san", ["address,undefined", "thread"])
def test_first_fit_under_sanitizer(tmp_path, san):
    exe = tmp_path / "first_fit_test"
    cmd = ["g++", "-std=c++17", "-O1", "-g", f"-fsanitize={san}", "-fno-omit-frame-pointer",
           f"-I{INC}", SRC, "-o", str(exe), "-pthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1", TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "first_fit ok" in r.stdout
