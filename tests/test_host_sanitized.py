"""Host code under the address and undefined-behaviour sanitizers (CPU only):
the library's device-memory arena (its host bookkeeping, on host arrays) and
a small run of the oracle's entry points, each built with g++/gcc and run as
a child process that must exit cleanly."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "host")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-g", "-O1"]


def _run(cmd, exe, tmp_path):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    b = subprocess.run(cmd, capture_output=True, text=True, cwd=str(tmp_path))
    assert b.returncode == 0, b.stderr[-4000:]
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the ROCm headers")
def test_arena_under_sanitizers(tmp_path):
    exe = str(tmp_path / "arena_check")
    csrc = os.path.join(ROOT, "paper_1304_4235_amd", "csrc")
    cmd = ["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), "-I" + csrc,
           os.path.join(HOST, "arena_check.cpp"), "-L/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
    assert "arena checks passed" in _run(cmd, exe, tmp_path)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    cmd = ["gcc", "-std=gnu11", *SAN, "-ffp-contract=off", "-fopenmp",
           "-I" + os.path.join(ROOT, "oracle"), os.path.join(HOST, "oracle_check.c"),
           os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", exe]
    assert "oracle checks passed" in _run(cmd, exe, tmp_path)
