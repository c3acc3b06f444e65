"""The register DFTs of csrc/dft.hpp, built for the host against the
emulation header (tests/hostemu), against the O(N^2) DFT definition in
double precision: every radix the line transforms use (1, 2, 3, 4, 6, 8, 9,
12, 16, 18, 24, 36), forward and inverse, 50 random inputs each.  A wrong sign, index or
twiddle gives an O(1) error; rounding gives ~1e-7."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EMU = os.path.join(ROOT, "tests", "hostemu")
CSRC = os.path.join(ROOT, "paper_2609_08384_amd", "csrc")


def _clang():
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if c and os.path.exists(c):
            return c
    return None


def test_register_dfts_match_definition(tmp_path):
    cxx = _clang()
    if cxx is None:
        pytest.skip("no clang++")
    exe = str(tmp_path / "dft_check")
    subprocess.run([cxx, "-x", "c++", "-std=c++17", "-O1", "-I" + EMU, "-I" + CSRC,
                    "-I" + os.path.join(ROOT, "include"), os.path.join(EMU, "dft_check.cpp"), "-o", exe],
                   check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.count(" ok") == 12, r.stdout
