"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The host-only parts of the library (box tracker, templates, work schedules,
direction shards, spherical tracker, irradiation factor) and the oracle's C
library are compiled with g++/gcc and -fsanitize=address,undefined, then
driven on small grids by the programs in tests/native/.  Any out-of-bounds
access, leak or undefined behaviour aborts the program; the drivers also
check invariants of what they compute (path lengths, schedule coverage,
direction-subset sums)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2102_01734_amd", "csrc")
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _run(cmd, exe):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_runtime_under_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_host")
    cmd = ["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
           "-I" + CSRC, os.path.join(ROOT, "tests", "native", "sanitize_host.cpp"),
           *[os.path.join(CSRC, f) for f in ("geometry.cpp", "sphere_geometry.cpp", "schedule.cpp")], "-o", exe]
    out = _run(cmd, exe)
    assert "host checks passed" in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_oracle")
    cmd = ["gcc", "-std=c11", "-D_GNU_SOURCE", *SAN, "-fopenmp", "-ffp-contract=off",
           os.path.join(ROOT, "tests", "native", "sanitize_oracle.c"), os.path.join(ROOT, "oracle", "rt_oracle.c"),
           "-lm", "-o", exe]
    out = _run(cmd, exe)
    assert "oracle checks passed" in out
