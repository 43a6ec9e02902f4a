"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the CPU
oracle (oracle/pdhcg_oracle.c) and the library's host-only preparation code
(paper_2602_23967_amd/csrc/prep.cpp: validation, transpose, SpMV schedules,
box storage), each built with gcc/g++ and the sanitizers (no device code is
involved) and run by a driver under tests/sanitize/ on valid, malformed and
edge-case inputs.  A sanitizer report or a wrong result fails the test."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(exe, tmp_path, threads):
    env = dict(os.environ, OMP_NUM_THREADS=str(threads),
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    out = p.stdout + p.stderr
    assert p.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    return out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is needed")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.run(["gcc", "-std=c11", *SAN, "-ffp-contract=off", "-fopenmp", "-I", os.path.join(ROOT, "oracle"),
                    os.path.join(ROOT, "oracle", "pdhcg_oracle.c"), os.path.join(HERE, "oracle_driver.c"),
                    "-lm", "-o", exe], check=True)
    for threads in (1, 2):
        out = _run(exe, tmp_path, threads)
        assert "oracle driver: 0 failure(s)" in out


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ is needed")
def test_host_preparation_under_sanitizers(tmp_path):
    exe = str(tmp_path / "prep_san")
    csrc = os.path.join(ROOT, "paper_2602_23967_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", *SAN, "-I", csrc, os.path.join(csrc, "prep.cpp"),
                    os.path.join(HERE, "prep_driver.cpp"), "-o", exe], check=True)
    out = _run(exe, tmp_path, 1)
    assert "prep driver: 0 failure(s)" in out
