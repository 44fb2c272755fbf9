"""The serving loop's scheduling on the CPU: jefi_server.cpp built with the
host compiler against a host mock of the HIP runtime and of the library
calls (tests/native/server_mock.cpp), under ThreadSanitizer and under
AddressSanitizer + UBSan.  Concurrent submitters, overlapping batches with
per-session ordering, eviction and re-materialisation, a full queue,
rejections, session closing and timestamps, a session brought back into the
arena in a pass that cannot admit its request, and one ticket polled and
waited from two threads (tests/native/server_test.cpp)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "native", "server_test.cpp"), os.path.join(HERE, "native", "server_mock.cpp"),
           os.path.join(ROOT, "paper_2104_05426_amd", "csrc", "jefi_server.cpp")]
MOCK_INCLUDE = os.path.join(HERE, "native", "mock_hip")
# ThreadSanitizer needs a runtime that intercepts pthread_cond_clockwait
# (libstdc++'s timed waits); the LLVM one shipped with ROCm does.
CLANG = "/opt/rocm/llvm/bin/clang++"


def _build_and_run(tmp_path, compiler, sanitize, name):
    exe = str(tmp_path / name)
    subprocess.run([compiler, "-std=c++17", "-O1", "-g", "-pthread", sanitize, "-I", MOCK_INCLUDE, "-o", exe]
                   + SOURCES, check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=240)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "server ok" in out.stdout
    assert "WARNING" not in out.stderr, out.stderr


@pytest.mark.skipif(not os.path.exists(CLANG), reason="LLVM clang++ with a ThreadSanitizer runtime not found")
def test_server_scheduling_under_tsan(tmp_path):
    _build_and_run(tmp_path, CLANG, "-fsanitize=thread", "server_tsan")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
def test_server_scheduling_under_asan(tmp_path):
    _build_and_run(tmp_path, "g++", "-fsanitize=address,undefined", "server_asan")
