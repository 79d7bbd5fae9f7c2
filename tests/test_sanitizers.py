"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the symbolic analysis (csrc/analysis.cpp, with its invariants and the
single-writer property of the extend-add gather maps checked by
tests/native/analysis_check.cpp) and the oracle's banded LU
(oracle/band_lu.c, driven by tests/native/band_lu_check.c).  Built with the
host compilers (g++ / gcc), no GPU code involved."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, exe):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert out.returncode == 0 and out.stdout.strip().endswith("ok"), out.stdout + out.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_analysis_under_sanitizers(tmp_path):
    exe = str(tmp_path / "analysis_check")
    _run(["g++", "-std=c++17", *SAN, os.path.join(ROOT, "tests", "native", "analysis_check.cpp"),
          os.path.join(ROOT, "paper_2307_05388_amd", "csrc", "analysis.cpp"), "-o", exe], exe)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_oracle_band_lu_under_sanitizers(tmp_path):
    exe = str(tmp_path / "band_lu_check")
    _run(["gcc", "-std=c99", *SAN, os.path.join(ROOT, "tests", "native", "band_lu_check.c"),
          os.path.join(ROOT, "oracle", "band_lu.c"), "-o", exe, "-lm"], exe)
