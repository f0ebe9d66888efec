"""Host code under the address and undefined-behaviour sanitizers (CPU only).

Three programs are built with -fsanitize=address,undefined (host code only;
no device code is built with a sanitizer) and run:
  - tests/host_check.cpp: the runtime behind the C ABI -- validation, layout,
    the 1D planner (tile coverage of every output, queues, grids, statistics
    segments) and the no-alloc scratch layout -- with the kernel launchers
    replaced by stubs;
  - tests/plan_check.cpp: the chunk walk shared by the planner and the kernels;
  - tests/oracle_check.c: the CPU oracle on awkward sizes, every input in an
    allocation of exactly its size.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def _run(exe):
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=900, env=ENV)
    assert out.returncode == 0, out.stdout[-3000:] + out.stderr[-3000:]
    assert "ERROR: AddressSanitizer" not in out.stderr and "runtime error" not in out.stderr, \
        out.stderr[-3000:]
    return out.stdout


@pytest.mark.skipif(not os.path.exists("/opt/rocm/include/hip/hip_runtime.h"),
                    reason="HIP headers are needed to compile the runtime's host code")
def test_runtime_host_code_under_sanitizers(tmp_path):
    exe = tmp_path / "host_check"
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__",
                           "-I/opt/rocm/include", "-o", str(exe),
                           os.path.join(ROOT, "tests", "host_check.cpp"), "-L/opt/rocm/lib",
                           "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-Wno-subobject-linkage"])
    assert " 0 failures" in _run(exe)


def test_chunk_walk_under_sanitizers(tmp_path):
    exe = tmp_path / "plan_check"
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-o", str(exe),
                           os.path.join(ROOT, "tests", "plan_check.cpp")])
    assert " 0 failures" in _run(exe)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is needed")
def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_check"
    subprocess.check_call(["gcc", "-std=c11", *SAN, "-ffp-contract=off", "-o", str(exe),
                           os.path.join(ROOT, "tests", "oracle_check.c"),
                           os.path.join(ROOT, "oracle", "hrms_oracle.c"), "-lm"])
    assert " 0 failures" in _run(exe)
