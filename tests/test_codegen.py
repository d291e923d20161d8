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
    src = os.path.join(ROOT, "tests", "native", "check_general_codegen.cpp")
    parts = [None] + list(range(11, 19))           # the inline levels 1..10, then each out-of-line level
    procs = []
    for lev in parts:
        exe = str(tmp_path / f"check_{lev or 'inline'}")
        defs = [] if lev is None else [f"-DCHECK_LEVEL={lev}"]
        cmd = ["g++", "-O0", "-std=c++17", "-I", CSRC, "-I", BUILD] + defs + [src, "-o", exe]
        procs.append((exe, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    errs = []
    for exe, pr in procs:
        out, _ = pr.communicate()
        assert pr.returncode == 0, out
        errs += [float(x) for x in subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()]
    assert len(errs) == 18
    assert max(errs) < 1e-14, errs


def test_general_flop_count_of_bench_matches_generated_code():
    """The FP64 operation count per slice that the bench uses for the general mode at p = 8 is the
    count of the operations in the code generated for that level (plus the fixed per-slice work)."""
    import re
    import sys
    gen = os.path.join(BUILD, "pimc_general_gen.hpp")
    if not os.path.exists(gen):
        pytest.skip("library not built")
    src = open(gen).read()
    body = src[src.index("struct GenCompiled<8>"):]
    body = body[:body.index("};")]
    lines = [ln for ln in body.splitlines() if "for (int i" in ln]
    fma = sum(ln.count("fma(") for ln in lines)
    mul = sum(ln.count(" * ") for ln in lines)
    add = sum(ln.count(" + ") for ln in lines)
    J = 14
    poly = sum(8 - j for j in range(min(J, 8) + 1))
    expected = 2 * fma + mul + add + 2 * poly + (J + 1) + 1 + 4
    sys.path.insert(0, ROOT)
    import bench
    assert bench.GENERAL_FLOP_PER_SLICE_P8 == expected, (fma, mul, add)
    assert re.search(r"NREC = 193;", body)


def test_general_flop_count_of_bench_matches_generated_code_p18():
    """The same for the out-of-line evaluator of p = 18 (one slice, no loops over slices)."""
    import sys
    gen = os.path.join(BUILD, "pimc_general_gen_p18.hpp")
    if not os.path.exists(gen):
        pytest.skip("library not built")
    src = open(gen).read()
    body = src[src.index("struct GenCompiled<18>"):]
    one = body[body.index("eval1("):body.index("eval2(")]     # the one-slice form
    lines = [ln for ln in one.splitlines() if " = " in ln and not ln.strip().startswith(("static", "//", "const"))]
    fma = sum(ln.count("fma(") for ln in lines)
    mul = sum(ln.count(" * ") for ln in lines)
    add = sum(ln.count(" + ") for ln in lines)
    J = 34
    poly = sum(8 - j for j in range(min(J, 8) + 1))
    expected = 2 * fma + mul + add + 2 * poly + (J + 1) + 4
    sys.path.insert(0, ROOT)
    import bench
    assert bench.GENERAL_FLOP_PER_SLICE_P18 == expected, (fma, mul, add)
    assert "NREC = 24196;" in body
