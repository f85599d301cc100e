"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Two CPU-only drivers are built with ``-fsanitize=address,undefined`` and
run; any invalid memory access, leak or undefined behaviour aborts them:

* ``sanitize/ptune_setfile_driver.cpp`` links the library's host-only parts:
  the portability-tuning routines (``csrc/ptune.cpp``) on random tables with
  failed entries, and the descriptor / manifest / set-file parser
  (``csrc/setfile.cpp``) on every committed set file, on every truncation
  of it and on randomly edited copies;
* ``sanitize/ref_gemm_driver.c`` links the oracle's GEMM (``oracle/ref_gemm.c``)
  with every operand in a heap block of exactly its size.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _build(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0 and "sanitizer" in p.stderr.lower() and "cannot find" in p.stderr.lower():
        pytest.skip("sanitizer runtime not installed")
    assert p.returncode == 0, p.stderr[-3000:]


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_ptune_and_setfile_under_sanitizers(tmp_path):
    exe = str(tmp_path / "ptune_setfile_driver")
    csrc = os.path.join(ROOT, "paper_2507_15277_amd", "csrc")
    _build(["g++", "-std=c++17", *SAN, "-Wall", "-o", exe, os.path.join(HERE, "ptune_setfile_driver.cpp"),
            os.path.join(csrc, "ptune.cpp"), os.path.join(csrc, "setfile.cpp")])
    p = subprocess.run([exe, os.path.join(ROOT, "paper_2507_15277_amd", "sets"),
                        os.path.join(ROOT, "paper_2507_15277_amd", "variants"), str(tmp_path)],
                       capture_output=True, text=True, env=ENV, timeout=600)
    assert p.returncode == 0 and p.stdout.strip().endswith("ok"), (p.stdout[-2000:], p.stderr[-4000:])


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_gemm_under_sanitizers(tmp_path):
    exe = str(tmp_path / "ref_gemm_driver")
    _build(["gcc", "-std=c11", "-fopenmp", *SAN, "-Wall", "-o", exe, os.path.join(HERE, "ref_gemm_driver.c"),
            os.path.join(ROOT, "oracle", "ref_gemm.c"), "-lm"])
    p = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    assert p.returncode == 0 and p.stdout.strip().endswith("ok"), (p.stdout[-2000:], p.stderr[-4000:])
