"""Host-only check of the 1D work decomposition used by the eq. (2)-(4)
kernels: tests/plan_check.cpp, built with g++ against the planner header."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_chunk_walks_cover_every_harmonic_once_in_order(tmp_path):
    exe = tmp_path / "plan_check"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-o", str(exe),
                           os.path.join(ROOT, "tests", "plan_check.cpp")])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "0 failures" in out.stdout
