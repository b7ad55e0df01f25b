"""The host halves of the library and the oracle under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

types.cpp and compile.cpp (constructors, layout compiler, segment queries)
are compiled unchanged with the host compiler, with tests/native/host_stub.cpp
in place of the device tables, and linked with the oracle; the test program
(tests/native/host_sanitize.cpp) builds 2000 seeded random nested types on
both sides, compares attributes, segments (one element and counts 0, 2, 3)
and iov_len budgets, runs envelope/contents, layout info and the error paths,
and packs and unpacks with the oracle.  An out-of-bounds access, a leak,
undefined behaviour or a disagreement fails the test."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2402_12274_amd", "csrc")
NATIVE = os.path.join(ROOT, "tests", "native")
ORACLE = os.path.join(ROOT, "oracle")
ROCM_INC = "/opt/rocm/include"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _sanitizers_available(td):
    src = os.path.join(td, "t.cpp")
    with open(src, "w") as f:
        f.write("int main() { return 0; }\n")
    r = subprocess.run(["g++", *SAN, src, "-o", os.path.join(td, "t")], capture_output=True)
    return r.returncode == 0


def test_host_code_under_address_and_ub_sanitizers():
    if not os.path.isdir(ROCM_INC):
        pytest.skip("HIP headers not installed")
    with tempfile.TemporaryDirectory() as td:
        if not _sanitizers_available(td):
            pytest.skip("no sanitizer runtimes for the host compiler")
        obj = os.path.join(td, "oracle.o")
        subprocess.check_call(["gcc", "-O1", "-g", *SAN, "-c", os.path.join(ORACLE, "oracle.c"), "-o", obj])
        exe = os.path.join(td, "host_sanitize")
        cmd = ["g++", "-std=c++17", "-O1", "-g", *SAN, "-D__HIP_PLATFORM_AMD__", "-I", ROCM_INC,
               "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", ORACLE,
               os.path.join(CSRC, "types.cpp"), os.path.join(CSRC, "compile.cpp"), os.path.join(CSRC, "trace.cpp"),
               os.path.join(NATIVE, "host_stub.cpp"), os.path.join(NATIVE, "host_sanitize.cpp"), obj,
               "-o", exe, "-lpthread", "-ldl"]
        subprocess.check_call(cmd)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
        assert "host sanitize ok" in r.stdout
