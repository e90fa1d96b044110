"""The host FP64 exponentials (csrc/tridiag.cpp: implicit-QR tridiagonal exponential and
its convergence-test variant; csrc/dense_expm.cpp: Pade scaling and squaring) built with the
address and undefined-behaviour sanitizers and checked against each other on random
tridiagonal matrices of 1..64 rows (tests/cpp/host_expm_test.cpp).  CPU only; needs g++ and
the HIP headers (the sources include them for their declarations)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_09813_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "cpp", "host_expm_test.cpp")
HIP_INC = "/opt/rocm/include"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(os.path.join(HIP_INC, "hip")),
                    reason="g++ or the HIP headers not available")
def test_host_exponentials_under_sanitizers(tmp_path):
    flags = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    inc = ["-D__HIP_PLATFORM_AMD__", f"-I{HIP_INC}", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
    objs = []
    for src in ("tridiag.cpp", "dense_expm.cpp"):
        obj = tmp_path / (src + ".o")
        subprocess.run(["g++", *flags, *inc, "-c", os.path.join(CSRC, src), "-o", str(obj)],
                       check=True, capture_output=True, text=True)
        objs.append(str(obj))
    exe = tmp_path / "host_expm_test"
    subprocess.run(["g++", *flags, DRIVER, *objs, "-o", str(exe)], check=True, capture_output=True,
                   text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-3000:]
    assert "host_expm ok" in r.stdout
