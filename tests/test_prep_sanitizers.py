"""The C++ mesh preprocessing built with address and undefined-behaviour
sanitizers (host code only, g++) and run on periodic and walled lattices,
both vertex orders, with and without artificial edges, plus an invalid input
(must be an error status, not a crash)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_prep_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "prep_driver")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-pthread", f"-I{ROOT}/include",
                    f"-I{ROOT}/paper_2102_12933_amd/csrc", os.path.join(ROOT, "tests", "native", "prep_driver.cpp"),
                    os.path.join(ROOT, "paper_2102_12933_amd", "csrc", "prep.cpp"), "-o", exe],
                   check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0 and r.stdout.strip().endswith("OK")
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
