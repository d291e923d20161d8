"""The build-time generator of the general-potential evaluators: its straight-line code (prefix
products kept between monomials) against the direct evaluation of the same monomials, compiled for
the host with g++ from the generated header of the last build. No device use."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1105_0542_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_1105_0542_amd", "_build")


def test_generated_evaluators_equal_direct_evaluation(tmp_path):
    gen = os.path.join(BUILD, "pimc_general_gen.hpp")
    if not os.path.exists(gen):
        pytest.skip("library not built")
    if shutil.which("g++") is None:
        pytest.skip("no host compiler")
    exe = str(tmp_path / "check")
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", CSRC, "-I", BUILD,
                    os.path.join(ROOT, "tests", "native", "check_general_codegen.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    errs = [float(x) for x in out]
    assert len(errs) == 10
    assert max(errs) < 1e-15, errs
