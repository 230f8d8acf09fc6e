"""Host: AddressSanitizer + UndefinedBehaviorSanitizer build of the host-only
library code (group selection, splitting) and of the C oracle, run on a small
problem and on bad arguments (tests/sanitize/driver.cpp).  The device code is
not built here: it runs only on the GPU, where these sanitizers are not used."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="needs gcc/g++")
def test_host_code_under_asan_ubsan(tmp_path):
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
    oobj = str(tmp_path / "oracle.o")
    subprocess.run(["gcc", *san, "-std=c11", "-fopenmp", "-c", os.path.join(ROOT, "oracle", "smx_oracle.c"),
                    "-o", oobj], check=True)
    exe = str(tmp_path / "driver")
    subprocess.run(["g++", *san, "-std=c++17", "-pthread", "-fopenmp", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "sanitize", "driver.cpp"),
                    os.path.join(ROOT, "paper_2004_10811_amd", "csrc", "smx_groups.cpp"), oobj, "-o", exe, "-lm"],
                   check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0 and r.stdout.strip().endswith("ok")
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
