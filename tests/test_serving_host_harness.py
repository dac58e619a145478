"""The request server and the C ABI's host code under ThreadSanitizer (CPU).

serve.cpp and capi.cpp are built with g++ -fsanitize=thread against host
stand-ins of the HIP runtime calls they make (tests/serving_harness/mock:
streams are FIFOs with their own executor threads, copies and events happen
when the stream reaches them, device memory is host memory) and of the
kernel launchers (tasks that read their inputs and write their outputs on
the stream).  The driver runs the GPU serving test's pattern (six requests
alone, then mixed with up to four running), requests whose contraction fails
after its kernel was queued while others run, and a description refused on
the host.  Any buffer handed to another request or freed while a stream may
still use it shows up as a data race.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
H = os.path.join(ROOT, "tests", "serving_harness")
CSRC = os.path.join(ROOT, "paper_2405_20258_amd", "csrc")


def test_serving_loop_under_thread_sanitizer(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "harness")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=thread",
           "-I", os.path.join(H, "mock"), "-I", os.path.join(ROOT, "include"),
           os.path.join(CSRC, "capi.cpp"), os.path.join(CSRC, "serve.cpp"),
           os.path.join(H, "mock_runtime.cpp"), os.path.join(H, "stubs.cpp"),
           os.path.join(H, "main.cpp"), "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    if r.returncode != 0 and "tsan" in r.stderr.lower():
        pytest.skip("ThreadSanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([exe, "6"], capture_output=True, text=True, timeout=300,
                       env=env)
    out = r.stdout + r.stderr
    assert "ThreadSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert out.count("alone == mixed") == 6 and "OK" in r.stdout
