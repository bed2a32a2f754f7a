"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the oracle's C routines and the library's host table builders, each compiled
with a small driver (tests/sanitize/) by the host compilers and run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, exe, tmp_path):
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stdout + res.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    return out.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", *SAN, "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-o", exe,
           os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), os.path.join(ROOT, "oracle", "gs_oracle.c"),
           "-lm"]
    assert "oracle driver:" in _run(cmd, exe, tmp_path)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_tables_under_sanitizers(tmp_path):
    exe = str(tmp_path / "tables_driver")
    csrc = os.path.join(ROOT, "paper_2509_15645_amd", "csrc")
    cmd = ["g++", *SAN, "-std=c++17", "-ffp-contract=off", "-I", csrc, "-o", exe,
           os.path.join(ROOT, "tests", "sanitize", "tables_driver.cpp"), os.path.join(csrc, "gsdp_lut.cpp")]
    assert "tables driver:" in _run(cmd, exe, tmp_path)
