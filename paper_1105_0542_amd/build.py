"""Build the HIP library libpimc.so for gfx950 in-tree with hipcc.

Usage: python -m paper_1105_0542_amd.build   (or call ``build()``).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libpimc.so")
CLI = os.path.join(PKG, "pimc")

SOURCES = ["pimc_batch_p18.hip", "pimc_batch_p12.hip", "pimc_batch_p8.hip",
           "pimc_kernels_q64.hip", "pimc_kernels_q32.hip", "pimc_kernels_tanh.hip", "pimc_kernels_batch.hip",
           "pimc_vector_d2.hip", "pimc_vector_d3.hip", "pimc_vector_d4.hip", "pimc_general_kernels.hip",
           "pimc_kernels.hip", "pimc_flow.hip", "pimc_spectrum.hip", "pimc_vector_d1.hip", "pimc_host.cpp", "pimc_flow_host.cpp", "pimc_spectrum_host.cpp",
           "pimc_general_host.cpp", "pimc_vector_host.cpp", "pimc_noalloc.cpp"]
HEADERS = ["pimc_tables.hpp", "pimc_device.hpp", "pimc_internal.hpp", "pimc_math.hpp", "pimc_walker.hpp",
           "pimc_flow.hpp", "pimc_host_common.hpp", "pimc_spectrum.hpp", "pimc_general.hpp",
           "pimc_general_device.hpp", "pimc_vector.hpp", "pimc_vector_impl.hpp", "pimc_batch.hpp"]
# Build-time generator of the general-potential evaluators: host C++ (the recursion of pimc_general.hpp)
# that writes pimc_general_gen.hpp (levels 1..10) and pimc_general_gen_p<p>.hpp (p = 11..18) into the
# object directory.
CODEGEN = "pimc_gen_codegen.cpp"
GENERATED = "pimc_general_gen.hpp"
# One translation unit per out-of-line general-mode level: (source, defines, object name).
GEN_HI_LEVELS = range(11, 19)
VARIANTS = [("pimc_general_hi.hip", [f"-DPIMC_GEN_P={p}"], f"pimc_general_hi_p{p}") for p in GEN_HI_LEVELS]
# One translation unit per dimension for the component evaluator's kernels, and one more for the
# deepest subtree of d = 3 and 4 (empty where that depth is below the split).
VARIANTS += [("pimc_vector_poly.hip", [f"-DPIMC_POLY_DIM={d}"], f"pimc_vector_poly_d{d}") for d in (1, 2, 3, 4)]
VARIANTS += [("pimc_vector_poly.hip", [f"-DPIMC_POLY_DIM={d}", "-DPIMC_POLY_DEEP=1"], f"pimc_vector_poly_d{d}_deep")
             for d in (3, 4)]

# -ffp-contract=off: every fused multiply-add in the kernels is written as fma(); no other
# expression is contracted, so the arithmetic is exactly what the source states.
# -packed-fp32-ops: packed FP32 instructions are not generated.
HIP_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


def build(verbose: bool = False, jobs: int = 4) -> str:
    """Compile every source to an object in parallel, then link libpimc.so. Always rebuilds."""
    t0 = time.time()
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", objdir]
    gen_exe = os.path.join(objdir, "pimc_gen_codegen")
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-I", CSRC, os.path.join(CSRC, CODEGEN), "-o", gen_exe],
                   check=True)
    subprocess.run([gen_exe, os.path.join(objdir, GENERATED), objdir], check=True)
    procs = []
    objs = []
    # the largest units first, so that they start before the small ones
    units = [(v[0], v[1], v[2]) for v in reversed(VARIANTS)] + [(s, [], os.path.splitext(s)[0]) for s in SOURCES]
    for src, defs, name in units:
        obj = os.path.join(objdir, name + ".o")
        objs.append(obj)
        cmd = [hipcc()] + HIP_FLAGS + defs + inc + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [hipcc(), "-x", "hip"] + HIP_FLAGS + defs + inc + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append((src, out))
        elif verbose and out.strip():
            print(out)
    if failed:
        msg = "\n".join(f"--- {s}\n{o}" for s, o in failed)
        raise RuntimeError(f"hipcc failed:\n{msg}")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    # the command-line front end: plain C++ against the C ABI, finds libpimc.so next to itself
    cli_tmp = CLI + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-Wall", "-I", os.path.join(ROOT, "include"), os.path.join(CSRC, "pimc_cli.cpp"),
           "-o", cli_tmp, "-L", PKG, "-lpimc", "-Wl,-rpath,$ORIGIN", "-Wl,-rpath-link,/opt/rocm/lib"]
    subprocess.run(cmd, check=True)
    os.replace(cli_tmp, CLI)
    if verbose:
        print(f"built {LIB} and {CLI} in {time.time() - t0:.1f}s", flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
