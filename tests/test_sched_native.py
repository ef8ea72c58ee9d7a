"""The serving loop's scheduling pieces (arena sub-allocator, FIFO admission
by footprint, wave limits) built for the CPU alone with g++ and run under
AddressSanitizer/UBSan.  No GPU involved."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_sched_native_checks():
    src = os.path.join(ROOT, "tests", "native", "sched_check.cpp")
    inc = os.path.join(ROOT, "paper_2106_01326_amd", "csrc")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "sched_check")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=all", "-I", inc, src, "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            pytest.fail(f"build failed:\n{r.stderr}")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "all ok" in r.stdout
