"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the CPU
oracle (oracle/etdo.c) and the plan construction (csrc/plan.cpp), each built
with gcc/g++ -fsanitize=address,undefined (host compilers only; no device
code is involved) and driven over small problems of every kind by the
drivers in tests/sanitize/.  Any sanitizer report aborts the driver."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, tmp_path, exe):
    subprocess.run(cmd, check=True, cwd=tmp_path, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(tmp_path / exe)], cwd=tmp_path, capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    out = _run(["gcc", "-std=c99", "-D_DEFAULT_SOURCE", *SAN, "-I", os.path.join(ROOT, "oracle"),
                "-o", "oracle_san", os.path.join(HERE, "sanitize", "oracle_driver.c"),
                os.path.join(ROOT, "oracle", "etdo.c"), "-lm"], tmp_path, "oracle_san")
    assert "ok" in out


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_plan_under_asan_ubsan(tmp_path):
    csrc = os.path.join(ROOT, "paper_2601_06849_amd", "csrc")
    out = _run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"), "-I", csrc,
                "-o", "plan_san", os.path.join(HERE, "sanitize", "plan_driver.cpp"),
                os.path.join(csrc, "plan.cpp")], tmp_path, "plan_san")
    assert "ok" in out
