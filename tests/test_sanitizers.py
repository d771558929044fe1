"""The CPU oracle and the host atom decomposition under AddressSanitizer and
UndefinedBehaviorSanitizer: each is compiled with gcc / g++ together with a
driver (tests/sanitize/) that calls every entry point on small inputs, edge
cases and invalid arguments; the run must exit cleanly with no report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="needs gcc and g++")


def build_and_run(cmd, exe, tmp_path):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    cmd = ["gcc", "-std=c11", "-fopenmp", *SAN, os.path.join(ROOT, "oracle", "hartree_oracle.c"),
           os.path.join(HERE, "oracle_driver.c"), "-lm", "-o", exe]
    assert "ok" in build_and_run(cmd, exe, tmp_path)


def test_partition_under_sanitizers(tmp_path):
    exe = str(tmp_path / "partition_san")
    csrc = os.path.join(ROOT, "paper_1209_4506_amd", "csrc")
    cmd = ["g++", "-std=c++17", *SAN, "-I", csrc, os.path.join(csrc, "partition.cpp"),
           os.path.join(HERE, "partition_driver.cpp"), "-o", exe]
    assert "ok" in build_and_run(cmd, exe, tmp_path)
