"""The FP64 elementary functions of the device code (tanh and exp of the non-polynomial slice
evaluators, -2 ln u, sqrt and (sin, cos)(2 pi t) of the Box-Muller step) compiled for the host with
g++ and compared with long double references over their argument ranges; the hardware estimates
they refine are replaced by perturbed exact values. No device use."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1105_0542_amd", "csrc")
NATIVE = os.path.join(ROOT, "tests", "native")


def test_device_math_within_a_few_ulp(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("no host compiler")
    exe = str(tmp_path / "check_math")
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", os.path.join(NATIVE, "stub"), "-I", CSRC,
                    os.path.join(NATIVE, "check_device_math.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    tanh_ulp, exp_ulp, log_ulp, sqrt_ulp, sincos_ulp = (float(x) for x in out)
    assert tanh_ulp < 4.0
    assert exp_ulp < 2.0
    assert log_ulp < 3.0
    assert sqrt_ulp <= 1.0
    assert sincos_ulp < 2.0
