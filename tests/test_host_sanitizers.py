"""Host code under sanitizers: the gate validation, lowering and pass planner
(plain C++, no GPU) built with g++ -fsanitize=address,undefined and driven by
random circuits of every gate kind, both precisions and random plan options."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2411_15332_amd", "csrc")


def test_planner_under_asan_ubsan():
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "fuzz")
        cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
               "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
               os.path.join(ROOT, "tests", "host", "planner_fuzz.cpp"), os.path.join(CSRC, "sv_planner.cpp"),
               os.path.join(CSRC, "sv_lower.cpp"), "-o", exe]
        b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
        if b.returncode != 0 and "asan" in b.stderr.lower():
            pytest.skip("sanitizer runtime not available")
        assert b.returncode == 0, b.stderr[-2000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe, "500"], capture_output=True, text=True, timeout=600, env=env)
        assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
        assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]
        assert r.stdout.strip().startswith("ok plans=500"), r.stdout
