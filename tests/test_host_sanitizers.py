"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

Two drivers under tests/sanitize/ are built with gcc/g++ and
-fsanitize=address,undefined: one runs every oracle entry point on small
seeded inputs (products, entries, Freivalds, triangular solves, echelon forms,
PLE, error paths) and checks them against each other; the other runs the
product library's host-side field set-up (irreducibility, reduction columns,
generators, Karatsuba and folded field schedules) against definitions it
writes out.  A memory error, undefined operation or leak fails the test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="4")


def build_and_run(cmd, exe):
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "passed" in r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_checks")
    build_and_run(["gcc", "-std=c11", "-fopenmp", *FLAGS, os.path.join(HERE, "oracle_checks.c"),
                   os.path.join(ROOT, "oracle", "gf2e_oracle.c"), "-o", exe], exe)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not installed")
def test_field_setup_under_sanitizers(tmp_path):
    exe = str(tmp_path / "field_checks")
    build_and_run(["g++", "-std=c++17", *FLAGS, "-I", os.path.join(ROOT, "paper_1111_6900_amd", "csrc"),
                   os.path.join(HERE, "field_checks.cpp"), "-o", exe], exe)
