"""The serving loop's host concurrency, checked on the CPU.

server.cpp is compiled unchanged with the host compiler and ThreadSanitizer
against a data-free stub executor (tests/native/server_stub.cpp: virtual
streams and events, no kernels, no data), and driven by concurrent clients,
a progress thread, explicit progress rounds and a statistics reader
(tests/native/server_tsan.cpp).  A data race, a lost or doubled completion,
or unbalanced counters fail the test."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2402_12274_amd", "csrc")
NATIVE = os.path.join(ROOT, "tests", "native")
ROCM_INC = "/opt/rocm/include"


def _tsan_available(td):
    src = os.path.join(td, "t.cpp")
    with open(src, "w") as f:
        f.write("int main() { return 0; }\n")
    r = subprocess.run(["g++", "-fsanitize=thread", src, "-o", os.path.join(td, "t")], capture_output=True)
    return r.returncode == 0


def test_server_scheduling_under_thread_sanitizer():
    if not os.path.isdir(ROCM_INC):
        pytest.skip("HIP headers not installed")
    with tempfile.TemporaryDirectory() as td:
        if not _tsan_available(td):
            pytest.skip("no ThreadSanitizer runtime for the host compiler")
        exe = os.path.join(td, "server_tsan")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-D__HIP_PLATFORM_AMD__", "-I", ROCM_INC,
               "-I", os.path.join(ROOT, "include"), "-I", CSRC, os.path.join(CSRC, "server.cpp"), os.path.join(CSRC, "trace.cpp"),
               os.path.join(NATIVE, "server_stub.cpp"), os.path.join(NATIVE, "server_tsan.cpp"), "-o", exe, "-lpthread", "-ldl"]
        subprocess.check_call(cmd)
        env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "ThreadSanitizer" not in r.stderr, r.stderr
        assert "server tsan ok" in r.stdout
