"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code (CPU only): the oracle
(plain C, OpenMP) and the library's mesh setup (C++, threads), each driven through meshes with walls,
periodic pairing and a bottom by a small driver under tests/sanitize/.  Any sanitizer report makes
the run fail (halt_on_error, no recovery)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="halt_on_error=1:detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
           OMP_NUM_THREADS="4")


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, (" ".join(cmd), r.stdout[-3000:], r.stderr[-3000:])
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", *SAN, "-I", os.path.join(ROOT, "oracle"),
          os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), os.path.join(ROOT, "oracle", "gks_oracle.c"),
          "-lm", "-o", exe], ROOT)
    r = _run([exe], ROOT)
    assert "oracle driver: ok" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_mesh_setup_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "mesh_san")
    csrc = os.path.join(ROOT, "paper_2306_04467_amd", "csrc")
    _run(["g++", "-std=c++17", *SAN, "-pthread", "-I", csrc, os.path.join(ROOT, "tests", "sanitize", "mesh_driver.cpp"),
          os.path.join(csrc, "mesh_setup.cpp"), "-o", exe], ROOT)
    r = _run([exe], ROOT)
    assert "mesh driver: ok" in r.stdout
