"""The oracle and the library's host-side weights-file parser built with the
address and undefined-behaviour sanitizers (gcc/g++, CPU only) and run
through drivers that reach every entry point on small inputs, valid and
invalid.  A memory error, a leak or undefined behaviour fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")


def build(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        if "sanitize" in r.stderr and ("cannot find" in r.stderr or "unrecognized" in r.stderr):
            pytest.skip("no sanitizer runtime for this compiler: " + r.stderr.strip()[:200])
        raise AssertionError(r.stderr)


def run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    build(["gcc", "-std=c99", "-fopenmp", "-ffp-contract=off"] + SAN +
          [os.path.join(ROOT, "oracle", "ccref.c"), os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
           "-lm", "-o", exe])
    assert "oracle driver OK" in run([exe])


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
def test_selector_file_parser_under_sanitizers(tmp_path):
    exe = str(tmp_path / "selfile_driver")
    build(["g++", "-std=c++17"] + SAN +
          [os.path.join(ROOT, "paper_0810_0233_amd", "csrc", "selfile.cpp"),
           os.path.join(ROOT, "tests", "sanitize", "selfile_driver.cpp"), "-o", exe])
    scratch = tmp_path / "files"
    scratch.mkdir()
    assert "selector file driver OK" in run([exe, str(scratch)])
