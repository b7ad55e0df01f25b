"""Unit checks of header-only product arithmetic, compiled with g++ (no GPU).

The magic-number division bounds every table index the kernels compute, so
it is checked against plain division on random and adversarial operands."""
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))


def test_magic_division_exact():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "magic_check")
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-o", exe, os.path.join(HERE, "native", "magic_check.cpp")])
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "bad 0" in r.stdout
