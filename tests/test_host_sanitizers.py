"""Host code under the sanitizers: the 1D eigensolver of EigT Step 1 (Sec. 4.1), compiled with g++ and
AddressSanitizer + UndefinedBehaviorSanitizer together with a check driver (tests/host/eig1d_check.cpp), must run
clean and decompose Lambda-bar (two-point absorbing, collocated zeta = 2 and Dirichlet closures, N = 2 ... 131) to
||Lambda V - V D|| and ||V^-1 V - I|| below 1e-9. No GPU is needed."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2602_07711_amd", "csrc")
ROCM_INC = "/opt/rocm/include"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(ROCM_INC), reason="g++ or the ROCm headers missing")
def test_eigensolver_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "eig1d_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INC, "-I" + CSRC,
           os.path.join(ROOT, "tests", "host", "eig1d_check.cpp"), os.path.join(CSRC, "eig1d.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-2000:], r.stderr[-2000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.strip().endswith("ok")
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
