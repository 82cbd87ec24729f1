"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the library's host rules (argument checks, error bounds, workspace sizing and
layouts, csrc/host_rules.h) and the C sources of the oracle and of the host
CPU Simpfer, each built with gcc/g++ -fsanitize=address,undefined and run on
checks that abort at the first memory error or undefined behaviour."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _have(compiler):
    return shutil.which(compiler) is not None


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    return r.stdout


@pytest.mark.skipif(not _have("g++"), reason="g++ missing")
def test_host_rules_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_rules_check")
    subprocess.run(["g++", "-std=c++17", *SAN, "-I" + os.path.join(ROOT, "include"),
                    "-I" + os.path.join(ROOT, "paper_2110_07131_amd", "csrc"),
                    os.path.join(HERE, "host_rules_check.cpp"), "-o", exe], check=True)
    assert "host rules ok" in _run(exe)


@pytest.mark.skipif(not _have("gcc"), reason="gcc missing")
def test_oracle_and_cpu_simpfer_under_sanitizers(tmp_path):
    exe = str(tmp_path / "cpu_code_check")
    subprocess.run(["gcc", "-std=c11", *SAN, "-fopenmp", "-ffp-contract=off",
                    os.path.join(HERE, "cpu_code_check.c"), os.path.join(ROOT, "oracle", "rk_oracle.c"),
                    os.path.join(ROOT, "cpu_simpfer", "simpfer.c"), "-o", exe, "-lm"], check=True)
    assert "ok" in _run(exe)
