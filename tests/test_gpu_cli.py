"""The command-line front end (argument order of the paper's program) against the library call."""
import os
import subprocess

import numpy as np
import pytest

import paper_1105_0542_amd as P

pytestmark = pytest.mark.gpu

CLI = os.path.join(os.path.dirname(P.lib_path()), "pimc")


def test_cli_prints_every_level_like_the_library():
    assert os.path.exists(CLI), "build the package first"
    args = ["-p", "8", "2.0", "0", "1", "5", "20000", "3", "0", "0", "0.5", "0", str(10 / 24)]
    out = subprocess.run([CLI] + args, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    rows = np.array([[float(v) for v in line.split()] for line in out.stdout.strip().splitlines()])
    assert rows.shape == (6, 4)
    assert list(rows[:, 0]) == [0, 1, 2, 3, 4, 5] and list(rows[:, 1]) == [1, 2, 4, 8, 16, 32]
    assert rows[0, 3] == 0.0                         # level 0: analytic, error 0
    with P.Context() as ctx:
        res, _ = ctx.amplitude([0, 0, 0.5, 0, 10 / 24], 1.0, 0.0, 1.0, 2.0, 32, 8, 20000, 3, 0, P.FLAG_HIERARCHY)
    for n in range(6):
        assert rows[n, 2] == res[n].amp and rows[n, 3] == res[n].err


def test_cli_help_and_errors():
    out = subprocess.run([CLI], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0 and "usage" in out.stdout
    bad = subprocess.run([CLI, "1", "0", "1", "4", "1"], capture_output=True, text=True, timeout=60)
    assert bad.returncode == 2


def test_cli_several_coordinates_like_the_library():
    # 2D anharmonic oscillator of Sec. 3.3 (A = 1, g = 10): V = (q.q)/2 + 10 (q.q)^2 / 24
    args = ["--dim", "2", "-p", "8", "1.0", "0", "0.5", "1", "-0.5", "4", "20000", "7", "0", "0.5", str(10 / 24)]
    out = subprocess.run([CLI] + args, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    rows = np.array([[float(v) for v in line.split()] for line in out.stdout.strip().splitlines()])
    assert rows.shape == (5, 4) and list(rows[:, 1]) == [1, 2, 4, 8, 16]
    with P.Context() as ctx:
        res, _ = ctx.amplitude_radial([0, 0.5, 10 / 24], 2, 1.0, [0.0, 0.5], [1.0, -0.5], 1.0, 16, 8, 20000, 7, 0,
                                      P.FLAG_HIERARCHY)
    for n in range(5):
        assert rows[n, 2] == res[n].amp and rows[n, 3] == res[n].err
    # four coordinates (two particles in two dimensions, isotropic): 4 + 4 endpoint coordinates
    a4, b4 = [0.1, 0.0, -0.2, 0.3], [0.4, 0.1, 0.0, -0.1]
    args4 = ["--dim", "4", "-p", "6", "-m", "1.5", "0.8"] + [str(v) for v in a4 + b4] + ["3", "5000", "2", "0.1", "0.5"]
    out4 = subprocess.run([CLI] + args4, capture_output=True, text=True, timeout=120)
    assert out4.returncode == 0, out4.stderr
    rows4 = np.array([[float(v) for v in line.split()] for line in out4.stdout.strip().splitlines()])
    assert rows4.shape == (4, 4)
    with P.Context() as ctx:
        res4, _ = ctx.amplitude_radial([0.1, 0.5], 4, 1.5, a4, b4, 0.8, 8, 6, 5000, 2, 0, P.FLAG_HIERARCHY)
    for n in range(4):
        assert rows4[n, 2] == res4[n].amp and rows4[n, 3] == res4[n].err
    bad = subprocess.run([CLI, "--dim", "5", "1", "0"], capture_output=True, text=True, timeout=60)
    assert bad.returncode == 2
    short = subprocess.run([CLI, "--dim", "2", "1.0", "0", "0", "1", "1", "4", "100", "1"], capture_output=True,
                           text=True, timeout=60)
    assert short.returncode == 2                     # no coefficient given
