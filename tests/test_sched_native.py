"""The serving loop's host side built for the CPU alone with g++, no GPU
involved: the scheduling pieces (arena sub-allocator, FIFO admission by
footprint, wave limits) under AddressSanitizer/UBSan, and the scheduler,
launcher and completion threads behind a fake executor under
ThreadSanitizer and under AddressSanitizer/UBSan."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2106_01326_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")

SANITIZERS = {"asan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
              "tsan": ["-fsanitize=thread"]}


def build_and_run(src_name, sanitizer, timeout=300):
    src = os.path.join(ROOT, "tests", "native", src_name)
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "check")
        cmd = ["g++", "-std=c++17", "-O1", "-g", *SANITIZERS[sanitizer], "-pthread",
               "-I", CSRC, "-I", INCLUDE, src, "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            pytest.fail(f"build failed:\n{r.stderr}")
        env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 second_deadlock_stack=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=timeout, env=env)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "all ok" in r.stdout
        return r.stdout


def test_sched_native_checks():
    build_and_run("sched_check.cpp", "asan")


@pytest.mark.parametrize("sanitizer", ["tsan", "asan"])
def test_serving_threads_with_fake_executor(sanitizer):
    build_and_run("serve_check.cpp", sanitizer)
