#!/usr/bin/env python3
"""Benchmark: FP64 slice evaluations per second of the bisection PIMC estimator at level p = 18.

Workload (one step): the p = 18 column of the convergence sweep -- the quartic oscillator
V = q^2/2 + g q^4/24 with g in {1, 10, 48} and T in {1, 2, 5}, endpoints a = 0, b = 1, 1e8 Philox
samples per point, every N = 2^1 .. 2^10 estimated (one s = 10 bisection run per point reads all
coarser levels off the same paths, as the paper's program does). Slice evaluations per sample =
sum_{n=1..10} 2^n = 2046; the N = 1 level is analytic.

Prints one JSON line with the metric, the roofline of the estimation kernel (FP64 vector ALU;
algorithmic FLOP per slice from the table size at p = 18), and the CPU oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

P_LEVEL = 18
S_DEPTH = 10
N_SAMPLES = 100_000_000
POINTS = [(g, T) for g in (1.0, 10.0, 48.0) for T in (1.0, 2.0, 5.0)]
# Algorithmic FP64 work of one slice evaluation at p = 18: E = 48 table entries -> 47 FMA (94 FLOP)
# plus mid-point (2), deviation (1), two squares (2) and the accumulation (1): 100 FLOP.
E_TABLE = {8: 16, 12: 27, 18: 48}       # quartic level-table entries per p (pimc_level_table)
FLOP_PER_SLICE = 2 * (E_TABLE[P_LEVEL] - 1) + 6
FP64_PEAK_TFLOPS = 78.6          # MI355X FP64 vector: 256 CU x 64 lanes x 2 FLOP x 2.4 GHz
CPU_SAMPLE_PATHS = 24576         # per point, for the oracle timing (about 10-20 s of the host's cores)
# Convergence sweep (every point of the configured grid): g in {1, 10, 48} x p in {1, 2, 4, 8, 12, 18} x
# T in {1, 2, 5}, 1e8 samples per point, one s = 10 run with every level per point; plus g = 0 at every p
# (T = 1) against the exact discretized Gaussian amplitude and the Mehler kernel.
C2 = dict(gs=(1.0, 10.0, 48.0), ps=(1, 2, 4, 8, 12, 18), Ts=(1.0, 2.0, 5.0), s=10, samples=100_000_000)
C3_SAMPLES = 1_000_000           # samples per task of the batched grid (the configured size)
C3_TUNE_SAMPLES = 10_000         # the same grid with fewer samples, for the autotuner
C3_REPLAY_SAMPLES = 100_000      # samples per task of one graph replay (about 12 s of device time)
# Precision workload: FP32 slice polynomials against FP64, g = 10, p = 18, N = 512, T = 1.
PREC = dict(g=10.0, p=18, s=9, T=1.0, samples=1_000_000_000, oracle_paths=1_000_000)
# Learned proposal: the anharmonic oscillator g = 10 at p = 12, N = 128, T = 2, a = 0, b = 1; 8 couplings,
# batches of 4096 fresh base paths, 2442 Adam steps (1e7 training paths), loss 0.1 log E[w^2] + 0.9 KL.
FLOW = dict(g=10.0, p=12, s=7, T=2.0, layers=8, batch=4096, lr=1e-3, beta=0.9, steps=2442,
            est_samples=1 << 24, plain_samples=1 << 26, target=1e-5,
            wide_batch=16384)   # same 1e7 training paths in 610 steps: fills the 256 CUs
# Spectrum from the space-discretized evolution operator: the two potentials of the paper's Fig. 3
# at its grid (n = 16384) and level p = 21 (short-time amplitudes, no Monte Carlo).
SPECTRUM = [dict(name="anharmonic A=1 g=48", A=1.0, g=48.0, t=0.02, L=8.0),
            dict(name="double well A=-10 g=12", A=-10.0, g=12.0, t=0.1, L=10.0)]
SPEC_N, SPEC_P, SPEC_K = 16384, 21, 10
# Several coordinates (Sec. 2.2): the 2D anharmonic oscillator of Sec. 3.3, V = r^2/2 + g r^4/24, and its
# 3D and 4D analogues, at p = 18, every level of s = 10, 1e8 samples; the 2D value against a tensor-product DVR.
VECTOR = dict(g=10.0, T=1.0, s=10, p=18, samples=100_000_000,
              ends={2: ((0.0, 0.0), (1.0, 0.4)), 3: ((0.0, 0.0, 0.0), (1.0, 0.4, -0.2)),
                    4: ((0.0, 0.0, 0.0, 0.0), (1.0, 0.4, -0.2, 0.3))})
RADIAL_E = {18: 102}                     # coefficients of the (u, z, w^2) table at p = 18
# Any polynomial V (component route): two particles on a line with a quartic pair interaction
# 0.1 (q1 - q2)^4 in an anisotropic trap with a field (d = 2, p = 10), an anisotropic 3D trap with
# cubic and quartic couplings (d = 3, p = 8) and two particles in two dimensions (d = 4, p = 8); one
# s = 10 run each (every level).
COMPONENT = dict(T=1.0, s=10, samples=4_000_000, cases=[
    dict(name="pair (q1-q2)^4 + trap, d=2", dim=2, p=10, a=(0.0, 0.0), b=(1.0, 0.4),
         terms=[(0.5, (2, 0)), (0.7, (0, 2)), (0.1, (4, 0)), (-0.4, (3, 1)), (0.6, (2, 2)), (-0.4, (1, 3)),
                (0.1, (0, 4)), (0.3, (1, 0)), (0.2, (1, 1))]),
    dict(name="anisotropic 3D trap, cubic + quartic couplings", dim=3, p=8, a=(0.0, 0.0, 0.0), b=(1.0, 0.4, -0.2),
         terms=[(0.5, (2, 0, 0)), (0.4, (0, 2, 0)), (0.3, (0, 0, 2)), (0.2, (0, 2, 1)), (0.05, (1, 1, 2)),
                (0.05, (0, 0, 4)), (0.1, (2, 2, 0)), (0.1, (0, 0, 1))]),
    # two particles in two dimensions: |r_1|^2/2 + |r_2|^2/2 + 0.1 |r_1 - r_2|^4, r_1 = (q1, q2), r_2 = (q3, q4)
    dict(name="two particles in 2D, quartic pair interaction, d=4", dim=4, p=8, samples=2_097_152,
         a=(0.0, 0.0, 0.0, 0.0), b=(1.0, 0.4, -0.2, 0.3),
         terms=[(0.1, (4, 0, 0, 0)), (-0.4, (3, 0, 1, 0)), (0.2, (2, 2, 0, 0)), (-0.4, (2, 1, 0, 1)), (0.6, (2, 0, 2, 0)),
                (0.2, (2, 0, 0, 2)), (0.5, (2, 0, 0, 0)), (-0.4, (1, 2, 1, 0)), (0.8, (1, 1, 1, 1)), (-0.4, (1, 0, 3, 0)),
                (-0.4, (1, 0, 1, 2)), (0.1, (0, 4, 0, 0)), (-0.4, (0, 3, 0, 1)), (0.2, (0, 2, 2, 0)), (0.6, (0, 2, 0, 2)),
                (0.5, (0, 2, 0, 0)), (-0.4, (0, 1, 2, 1)), (-0.4, (0, 1, 0, 3)), (0.1, (0, 0, 4, 0)), (0.2, (0, 0, 2, 2)),
                (0.5, (0, 0, 2, 0)), (0.1, (0, 0, 0, 4)), (0.5, (0, 0, 0, 2))]),
])
HBM_PEAK_GBS = 8000.0
# Modified Poeschl-Teller potential (the paper's Fig. 2): V = -lambda/cosh^2(alpha q), lambda = alpha = 1,
# A_N^(p)(-0.5, 0.5; 1) for p in {1, 2, 10} from one s = 10 run each (every N = 2^0..2^10).
MPT = dict(lam=1.0, alpha=1.0, a=-0.5, b=0.5, T=1.0, s=10, ps=(1, 2, 10), samples=100_000_000)
KERNEL_SOURCES = ["pimc_device.hpp", "pimc_kernels_q64.hip", "pimc_walker.hpp", "pimc_internal.hpp", "pimc_tables.hpp",
                  "pimc_math.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_amplitude_quartic64_p18_s10.json")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "counters_k_amplitude_quartic64_p18_s10.json")


def _progress(msg):
    """One line per finished step of the bench, on stderr (the JSON line is the only stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the estimation kernel's sources: a traffic measurement is valid only for this hash."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        path = os.path.join(ROOT, "paper_1105_0542_amd", "csrc", name)
        if os.path.exists(path):
            h.update(name.encode())
            h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(samples: int):
    """HBM bytes per launch from the committed FETCH_SIZE/WRITE_SIZE measurement (scaled by the
    plain-copy factors), or None when the kernel sources changed since it was taken."""
    import json as _json
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = _json.load(open(TRAFFIC_FILE))
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec["bytes_per_sample"] * samples


def measured_counter_flops():
    """FP64 VALU FLOPs per sample of the headline kernel from the committed rocprofv3 counter record
    (SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes), or None when the kernel sources changed since."""
    import json as _json
    if not os.path.exists(COUNTERS_FILE):
        return None
    rec = _json.load(open(COUNTERS_FILE))
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec


def copy_probe():
    """Plain device copy of known size (512 MiB): the reference for FETCH_SIZE/WRITE_SIZE scaling."""
    import torch
    x = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
    x.fill_(1.0)
    torch.cuda.synchronize()
    for _ in range(3):
        y = x.clone()
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": x.numel() * 8, "copies": 3, "check": float(y[0])}), flush=True)


def slices_per_sample(s: int, hierarchy: bool) -> int:
    return (2 ** (s + 1) - 2) if hierarchy else 2 ** s


def _oracle_worker(args):
    g, T, first, count = args
    import numpy as np
    from oracle import effective_action as ea
    from oracle import pimc as opimc
    idx = np.arange(first, first + count, dtype=np.uint64)
    S = opimc.path_actions(ea.quartic(1, g), 1, 0.0, 1.0, T, S_DEPTH, P_LEVEL, 1, 0, idx)
    return float(S[:, S_DEPTH].sum())


def _oracle_chunk(args):
    g, T, s, p, first, count, shift = args
    from oracle import effective_action as ea
    from oracle import pimc as opimc
    return opimc.chunk_sums(ea.quartic(1, g), 1, 0.0, 1.0, T, s, p, 1, 0, first, count, shift)


def oracle_precision_reference():
    """Oracle amplitude at level s of the precision workload on its first paths (shifted sums)."""
    import multiprocessing as mp
    import numpy as np
    from oracle import effective_action as ea
    from oracle import pimc as opimc
    g, T, s, p, n = PREC["g"], PREC["T"], PREC["s"], PREC["p"], PREC["oracle_paths"]
    shift = opimc.straight_line_actions(ea.quartic(1, g), 1, 0.0, 1.0, T, s, p)
    jobs = [(g, T, s, p, st, min(1000, n - st), shift) for st in range(0, n, 1000)]
    with mp.get_context("fork").Pool(min(len(os.sched_getaffinity(0)), 16)) as pool:
        parts = pool.map(_oracle_chunk, jobs)
    tot = np.sum(parts, axis=0)[s]
    K0 = opimc.free_kernel(0.0, 1.0, T)
    return K0 * math.exp(-shift[s]) * (1.0 + tot[1] / tot[0])


def oracle_spectrum_reference():
    """Low-lying levels of the spectrum workloads by the oracle's sinc-DVR diagonalization (CPU)."""
    from oracle import closed_forms as cf
    out = []
    for case in SPECTRUM:
        _, E, _ = cf.dvr_eigen(cf.quartic_V(case["A"], case["g"]), L=case["L"], h=0.02)
        out.append([float(v) for v in E[:SPEC_K]])
    return out


def _oracle_vector_worker(args):
    dim, first, count = args
    import numpy as np
    from oracle import vector as ov
    a, b = VECTOR["ends"][dim]
    idx = np.arange(first, first + count, dtype=np.uint64)
    ov.path_actions([0.0, 0.5, VECTOR["g"] / 24.0], dim, 1.0, a, b, VECTOR["T"], VECTOR["s"], VECTOR["p"], 1, 0, idx)
    return count


def _oracle_mpt_worker(args):
    p, first, count = args
    import numpy as np
    from oracle import mpt
    idx = np.arange(first, first + count, dtype=np.uint64)
    mpt.path_actions(MPT["lam"], MPT["alpha"], 1.0, MPT["a"], MPT["b"], MPT["T"], MPT["s"], p, 1, 0, idx)
    return count


def _oracle_component_worker(args):
    k, first, count = args
    import numpy as np
    from oracle import vector as ov
    case = COMPONENT["cases"][k]
    idx = np.arange(first, first + count, dtype=np.uint64)
    ov.poly_path_actions(case["terms"], case["dim"], 1.0, case["a"], case["b"], COMPONENT["T"], COMPONENT["s"],
                         case["p"], 1, 0, idx)
    return count


def _oracle_general_worker(args):
    p, first, count = args
    import numpy as np
    from oracle import effective_action as ea
    from oracle import general as og
    idx = np.arange(first, first + count, dtype=np.uint64)
    og.path_actions(p, 1.0, 10, 0.0, 1.0, 1, 0, idx, poly=[float(c) for c in ea.quartic(1, 10)])
    return count


def _timed_pool(worker, jobs):
    import multiprocessing as mp
    cores = min(len(os.sched_getaffinity(0)), 16)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        done = sum(pool.map(worker, jobs))
    return done, time.perf_counter() - t0, cores


def oracle_section_baselines(which):
    """The oracle as it stands, timed on the host cores on bounded samples of the workloads of the
    several-coordinate, Poeschl-Teller, general-potential and spectrum sections (each a few seconds)."""
    out = {}
    sl = slices_per_sample(10, True)
    if "vector" in which:
        out["vector"] = {}
        for dim in (2, 3, 4):
            n, dt, cores = _timed_pool(_oracle_vector_worker, [(dim, 256 * i, 256) for i in range(16)])
            out["vector"][str(dim)] = {"value": n * sl / dt, "unit": "slice-evals/s", "cores": cores, "kind": "oracle",
                                       "sample": f"first {n} paths of the d={dim} workload (p=18, s=10, every level), "
                                                 f"{dt:.1f} s wall"}
        out["vector"]["component"] = []
        slc = slices_per_sample(COMPONENT["s"], True)
        for k, case in enumerate(COMPONENT["cases"]):
            n, dt, cores = _timed_pool(_oracle_component_worker, [(k, 128 * i, 128) for i in range(16)])
            out["vector"]["component"].append({
                "value": n * slc / dt, "unit": "slice-evals/s", "cores": cores, "kind": "oracle",
                "sample": f"first {n} paths of the {case['name']} workload (p={case['p']}, s={COMPONENT['s']}, "
                          f"every level), {dt:.1f} s wall"})
    if "mpt" in which:
        n, dt, cores = _timed_pool(_oracle_mpt_worker, [(10, 1024 * i, 1024) for i in range(16)])
        out["mpt"] = {"value": n * sl / dt, "unit": "slice-evals/s", "cores": cores, "kind": "oracle",
                      "sample": f"first {n} paths at p=10 (s=10, every level), {dt:.1f} s wall"}
    if "general" in which:
        n, dt, cores = _timed_pool(_oracle_general_worker, [(8, 512 * i, 512) for i in range(16)])
        out["general"] = {"value": n * sl / dt, "unit": "slice-evals/s", "cores": cores, "kind": "oracle",
                          "sample": f"first {n} paths of the quartic in the derivative-symbol mode (p=8, s=10, "
                                    f"every level), {dt:.1f} s wall"}
    if "spectrum" in which:
        import numpy as np
        from oracle import effective_action as ea
        from oracle import spectrum as osp
        n = 2048
        case = SPECTRUM[0]
        t0 = time.perf_counter()
        M, _, _ = osp.evolution_matrix(ea.quartic(case["A"], case["g"]), 1.0, case["t"], SPEC_P, case["L"], n)
        t1 = time.perf_counter()
        np.linalg.eigh(M)
        t2 = time.perf_counter()
        out["spectrum"] = {"value": n * (n + 1) / 2 / (t1 - t0), "unit": "distinct matrix elements/s", "cores": 1,
                           "kind": "oracle", "eigh_s": t2 - t1,
                           "sample": f"{case['name']} at n={n} (the matrix of the oracle, then numpy's dense eigh), "
                                     f"{t1 - t0:.1f} s + {t2 - t1:.1f} s wall"}
    return out


def oracle_mpt_reference():
    """A(-0.5, 0.5; 1) of the Poeschl-Teller workload by the oracle's DVR diagonalization (CPU)."""
    from oracle import closed_forms as cf
    lam, alpha = MPT["lam"], MPT["alpha"]
    return float(cf.dvr_amplitude(lambda x: -lam / np.cosh(alpha * x) ** 2, MPT["a"], MPT["b"], MPT["T"],
                                  L=20.0, h=0.025))


def oracle_vector_reference():
    """A((0,0), (1,0.4); 1) of the 2D workload by the oracle's tensor-product DVR (CPU)."""
    from oracle import vector as ov
    g = VECTOR["g"]
    a, b = VECTOR["ends"][2]
    return float(ov.dvr_amplitude_2d(lambda X, Y: 0.5 * (X * X + Y * Y) + g / 24.0 * (X * X + Y * Y) ** 2,
                                     a, b, VECTOR["T"], L=6.0, h=0.2))


def _fit_continuum(levels, p):
    """Weighted least squares of eq.(fit), A_N = A + B/N^p + C/N^(p+1), over the given levels with
    N = 2^n >= 16 (at T = 5 the levels N = 4, 8 carry higher orders than the two terms of the model);
    returns (A, its standard error). The levels of one run share their paths, so
    their errors are correlated: A = sum_n h_n A_N is linear in the levels, and the error returned is
    sum_n |h_n| err_N, the bound that holds for any correlation (the independent-error formula
    understates it by a factor of about 2.5 here)."""
    rows, rhs, w = [], [], []
    for n, r in levels:
        N = float(1 << n)
        if N < 16 or r.err <= 0:
            continue
        rows.append([1.0, N ** -p, N ** -(p + 1)])
        rhs.append(r.amp)
        w.append(1.0 / r.err)
    X = np.array(rows) * np.array(w)[:, None]
    y = np.array(rhs) * np.array(w)
    coef, *_ = np.linalg.lstsq(X, y, rcond=None)
    h = np.linalg.pinv(X)[0]                  # A = sum_n h_n w_n A_N, and w_n err_N = 1
    return float(coef[0]), float(np.sum(np.abs(h)))


def mpt_section(P, ctx, dvr, base=None):
    """Convergence of A_N^(p) with N for the Poeschl-Teller potential at p = 1, 2, 10 (Fig. 2),
    eq.(fit) extrapolations, and the DVR continuum value when given."""
    M = MPT
    out = {"workload": f"V=-{M['lam']:g}/cosh^2({M['alpha']:g} q), A_N^(p)({M['a']:g}, {M['b']:g}; {M['T']:g}), "
                       f"one s={M['s']} run per p (N = 1..{1 << M['s']}), {M['samples']:.0e} samples each",
           "per_p": {}}
    for p in M["ps"]:
        res, st = ctx.amplitude_mpt(M["lam"], M["alpha"], 1.0, M["a"], M["b"], M["T"], 1 << M["s"], p, M["samples"],
                                    1, 0, P.FLAG_HIERARCHY)
        ms = ctx.last_kernel_ms()
        A, dA = _fit_continuum(list(enumerate(res)), p)
        rate = M["samples"] * slices_per_sample(M["s"], True) / (ms / 1e3)
        # FP64 operations per slice of the Poeschl-Teller evaluator: p groups of degree p in
        # u = tanh^2 (p^2 fma), p - 1 Horner steps in dlt^2, mid-point, deviation, the two squares and
        # the accumulation (6); the tanh itself (about 40 operations) is not counted
        flop = 2 * p * p + 2 * (p - 1) + 6
        row = {"A_N": [r.amp for r in res], "err_N": [r.err for r in res], "fit_A": A, "fit_err": dA,
               "kernel_ms": ms, "slice_evals_per_s": rate, "flop_per_slice": flop,
               "fp64_frac": rate * flop / 1e12 / FP64_PEAK_TFLOPS, "status": st}
        if dvr is not None:
            row["A_N_minus_dvr_over_err_at_N1024"] = (res[M["s"]].amp - dvr) / res[M["s"]].err
            row["fit_minus_dvr_over_err"] = (A - dvr) / dA if dA > 0 else None
        out["per_p"][str(p)] = row
    if dvr is not None:
        out["dvr_continuum"] = dvr
    if base is not None:
        out["cpu_baseline"] = base
    return out


# FP64 operations per slice of the general-mode evaluator at p = 8 for a polynomial potential, counted
# in the code generated for that level: the prefix-tree sums of the monomials (192 fma, 63 products),
# 36 fma for the derivatives of the polynomial (degree-8 rows), 15 + 1 level scalings, and mid-point,
# deviation, its square and the accumulation (4).
GENERAL_FLOP_PER_SLICE_P8 = 2 * 192 + 63 + 2 * 36 + 16 + 4
# p = 18: the out-of-line evaluator's 24,195 fma and 6,185 multiplications (24,196 monomials), the
# polynomial rows of the derivatives, the scaling of the 35 derivatives and the fixed slice work
GENERAL_FLOP_PER_SLICE_P18 = 2 * 24195 + 6185 + 2 * 36 + 35 + 4


def general_section(P, ctx, base=None):
    """Cost of the general-potential (derivative-symbol) mode against the specialized quartic
    kernel on the same problem, and a non-polynomial potential (Gaussian barrier in an oscillator);
    p = 8, every level of s = 10, 1e7 samples."""
    n, s, p = 10_000_000, 10, 8
    rows = {}
    coefs = P.quartic(1.0, 10.0)
    res_q, _ = ctx.amplitude(coefs, 1.0, 0.0, 1.0, 1.0, 1 << s, p, n, 1, 0, P.FLAG_HIERARCHY)
    ms_q = ctx.last_kernel_ms()
    res_g, _ = ctx.amplitude_general(1.0, 0.0, 1.0, 1.0, 1 << s, p, n, 1, 0, P.FLAG_HIERARCHY, poly=coefs)
    ms_g = ctx.last_kernel_ms()
    sl = n * slices_per_sample(s, True)
    rows["quartic_g10_specialized"] = {"slice_evals_per_s": sl / (ms_q / 1e3), "A_1024": res_q[s].amp,
                                       "err": res_q[s].err}
    tflops = sl * GENERAL_FLOP_PER_SLICE_P8 / (ms_g / 1e3) / 1e12
    rows["quartic_g10_general_mode"] = {"slice_evals_per_s": sl / (ms_g / 1e3), "A_1024": res_g[s].amp,
                                        "err": res_g[s].err,
                                        "rel_diff_vs_specialized": abs(res_g[s].amp - res_q[s].amp) / res_q[s].amp,
                                        "roofline": {"bound": "alu", "achieved": tflops, "peak": FP64_PEAK_TFLOPS,
                                                     "unit": "TFLOP/s", "frac": tflops / FP64_PEAK_TFLOPS,
                                                     "flop_per_slice": GENERAL_FLOP_PER_SLICE_P8}}
    res_b, _ = ctx.amplitude_general(1.0, -0.3, 0.4, 1.0, 1 << s, p, n, 1, 0, P.FLAG_HIERARCHY, poly=(0, 0, 0.5),
                                     gauss=((2.0, 1.0),))
    ms_b = ctx.last_kernel_ms()
    rows["gaussian_barrier"] = {"potential": "q^2/2 + 2 exp(-q^2), A(-0.3, 0.4; 1)",
                                "slice_evals_per_s": sl / (ms_b / 1e3), "A_1024": res_b[s].amp, "err": res_b[s].err}
    # the paper's highest level for a general potential: 24,196 monomials per slice
    n18 = 200_000
    res_h, _ = ctx.amplitude_general(1.0, -0.3, 0.4, 1.0, 1 << s, 18, n18, 1, 0, P.FLAG_HIERARCHY, poly=(0, 0, 0.5),
                                     gauss=((2.0, 1.0),))
    ms_h = ctx.last_kernel_ms()
    sl18 = n18 * slices_per_sample(s, True)
    tf18 = sl18 * GENERAL_FLOP_PER_SLICE_P18 / (ms_h / 1e3) / 1e12
    rows["gaussian_barrier_p18"] = {
        "potential": "q^2/2 + 2 exp(-q^2), A(-0.3, 0.4; 1)", "p": 18, "samples": n18,
        "slice_evals_per_s": sl18 / (ms_h / 1e3), "A_1024": res_h[s].amp, "err": res_h[s].err,
        "diff_vs_p8_in_sigma": abs(res_h[s].amp - res_b[s].amp) / math.hypot(res_h[s].err, res_b[s].err),
        "roofline": {"bound": "alu", "achieved": tf18, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": tf18 / FP64_PEAK_TFLOPS, "flop_per_slice": GENERAL_FLOP_PER_SLICE_P18}}
    out = {"workload": f"p={p}, s={s} (every level), {n:.0e} samples; p=18 on {n18:.0e} samples", **rows}
    if base is not None:
        out["cpu_baseline"] = base
    return out


def vector_section(P, ctx, dvr, base=None):
    """Several coordinates: A_N^(18) of the 2D, 3D and 4D anharmonic oscillators from one s = 10 run each
    (every level), the kernel rate against the FP64 vector peak, and the 2D value against the DVR."""
    V = VECTOR
    coefs = (0.0, 0.5, V["g"] / 24.0)
    out = {"workload": f"V=r^2/2+{V['g']:g} r^4/24 in d=2, 3 and 4, p={V['p']}, s={V['s']} (every level), "
                       f"T={V['T']:g}, {V['samples']:.0e} samples", "per_dim": {}}
    for dim in (2, 3, 4):
        a, b = V["ends"][dim]
        ctx.amplitude_radial(coefs, dim, 1.0, a, b, V["T"], 1 << V["s"], V["p"], 1 << 20, 1, 0, P.FLAG_HIERARCHY)
        res, st = ctx.amplitude_radial(coefs, dim, 1.0, a, b, V["T"], 1 << V["s"], V["p"], V["samples"], 1, 0,
                                       P.FLAG_HIERARCHY)
        ms = ctx.last_kernel_ms()
        rate = V["samples"] * slices_per_sample(V["s"], True) / (ms / 1e3)
        flop = 2 * (RADIAL_E[V["p"]] - 1) + 8 * dim + 2
        row = {"a": a, "b": b, "A_N": [r.amp for r in res], "err_N": [r.err for r in res], "status": st,
               "kernel_ms": ms, "slice_evals_per_s": rate, "flop_per_slice": flop,
               "fp64_frac": rate * flop / 1e12 / FP64_PEAK_TFLOPS}
        if dim == 2 and dvr is not None:
            row["dvr_continuum"] = dvr
            row["A_N_minus_dvr_over_err"] = [(r.amp - dvr) / r.err if r.err > 0 else None for r in res]
        if base is not None:
            row["cpu_baseline"] = base[str(dim)]
        out["per_dim"][str(dim)] = row
        _progress(f"vector d={dim}: {rate:.3e} slice-evals/s")
    out["component"] = component_rows(P, ctx, base.get("component") if base is not None else None)
    return out


def component_rows(P, ctx, base=None):
    """Any polynomial V through the component evaluator: the rate, and the FP64 fraction counting one
    FMA (2 flops) per monomial of eps W_p, the least any Horner scheme over the monomials does."""
    C = COMPONENT
    rows = []
    for case in C["cases"]:
        args = (case["terms"], case["dim"], 1.0, case["a"], case["b"], C["T"], 1 << C["s"], case["p"])
        ns = case.get("samples", C["samples"])
        # warm-up: the host recursion of (V, m, p) (cached) and the code object, at N = 2
        ctx.amplitude_poly(case["terms"], case["dim"], 1.0, case["a"], case["b"], C["T"], 2, case["p"], 4096, 1, 0,
                           P.FLAG_HIERARCHY)
        res, st = ctx.amplitude_poly(*args, ns, 1, 0, P.FLAG_HIERARCHY)
        ms = ctx.last_kernel_ms()
        rate = ns * slices_per_sample(C["s"], True) / (ms / 1e3)
        coef, _ = P.level_table_poly(case["terms"], case["dim"], 1.0, C["T"], case["p"], C["s"])
        flop = 2 * coef.size
        rows.append({"workload": f"{case['name']}, p={case['p']}, s={C['s']} (every level), T={C['T']:g}, "
                                 f"{ns:.0e} samples", "status": st,
                     "A_N": [r.amp for r in res], "err_N": [r.err for r in res], "kernel_ms": ms,
                     "slice_evals_per_s": rate, "monomials": int(coef.size), "flop_per_slice": flop,
                     "fp64_frac": rate * flop / 1e12 / FP64_PEAK_TFLOPS})
        if base is not None:
            rows[-1]["cpu_baseline"] = base[len(rows) - 1]
        _progress(f"component {case['name']}: {rate:.3e} slice-evals/s")
    return rows


def spectrum_section(P, ctx, dvr, base=None):
    """Matrix build (ALU: level-p Horner + exp per element) and Lanczos (HBM: one pass over the
    matrix per step) for the spectrum workloads; levels against the DVR reference when given."""
    rows = []
    for ci, case in enumerate(SPECTRUM):
        coefs = P.quartic(case["A"], case["g"])
        ctx.spectrum(coefs, 1.0, case["t"], SPEC_P, case["L"], 1024, 4)            # warm
        E, _, info, st = ctx.spectrum(coefs, 1.0, case["t"], SPEC_P, case["L"], SPEC_N, SPEC_K, max_iter=1024,
                                      tol=1e-10)
        tab, deg, _ = P.level_table(coefs, 1.0, case["t"], SPEC_P, 0)
        flop_el = 2 * (tab.size - 1) + 10          # Horner over the table, mid/dlt/squares, Gaussian term
        # the matrix is exactly symmetric: n(n+1)/2 distinct elements are built and streamed per step
        n2 = float(SPEC_N) * (SPEC_N + 1) / 2.0
        mat_tflops = n2 * flop_el / (info.matrix_ms / 1e3) / 1e12
        bytes_iter = n2 * 8.0
        row = {"workload": f"{case['name']}, t={case['t']:g}, L={case['L']:g}, n={SPEC_N}, p={SPEC_P}",
               "status": st, "E": [float(v) for v in E], "lanczos_steps": info.iterations,
               "max_residual": info.max_residual,
               "matrix_ms": info.matrix_ms, "matrix_roofline": {
                   "bound": "alu", "achieved": mat_tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                   "frac": mat_tflops / FP64_PEAK_TFLOPS, "flop_per_element": flop_el,
                   "note": "exp per element not counted"},
               "solve_ms": info.solve_ms,
               "lanczos_stream_GBs": bytes_iter * info.iterations / (info.solve_ms / 1e3) / 1e9,
               "lanczos_ms_per_step": info.solve_ms / max(info.iterations, 1),
               "lanczos_note": "solve time includes the reorthogonalization and host checks every 16 steps; "
                               "the matrix pass alone is bound by HBM (the upper 64x64 tiles, 1.08 GB per "
                               "step at n = 16384); rates count the n(n+1)/2 distinct elements"}
        if dvr is not None:
            ref = np.asarray(dvr[ci])
            row["max_abs_diff_vs_dvr"] = float(np.max(np.abs(np.asarray(E) - ref)))
        if base is not None and ci == 0:
            row["cpu_baseline"] = base
        rows.append(row)
    return rows


def _host_cpus():
    return {"host_cpus": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0))}


def cpu_baseline(paths_per_point: int):
    """The oracle as it stands, on the host cores: level actions of the first paths of each point.
    `cores` is the number of worker processes actually used (at most 16, the host's CPU share for one
    GPU);
    the host's own counts are reported beside it."""
    import multiprocessing as mp
    cores = min(len(os.sched_getaffinity(0)), 16)
    chunk = 256
    jobs = [(g, T, st, min(chunk, paths_per_point - st)) for (g, T) in POINTS for st in range(0, paths_per_point, chunk)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        pool.map(_oracle_worker, jobs)
    dt = time.perf_counter() - t0
    n_slices = len(POINTS) * paths_per_point * slices_per_sample(S_DEPTH, True)
    return {"value": n_slices / dt, "unit": "slice-evals/s", "cores": cores, "kind": "oracle", **_host_cpus(),
            "sample": f"first {paths_per_point} paths of each of the {len(POINTS)} points (p=18, s=10, every level), "
                      f"{dt:.1f} s wall"}


def c2_references():
    """CPU references of the convergence sweep, computed before the GPU is touched: the sinc-DVR
    continuum A(0, 1; T) of each (g, T), and for g = 0 (T = 1) the exact discretized amplitude
    A_N^(p) of every level (mpmath Gaussian integral) and the Mehler kernel."""
    from oracle import closed_forms as cf
    cont = {f"{g:g},{T:g}": float(cf.dvr_amplitude(cf.quartic_V(1.0, g), 0.0, 1.0, T))
            for g in C2["gs"] for T in C2["Ts"]}
    exact0 = {str(p): [cf.gaussian_discretized(0.0, 1.0, 1.0, 1 << n, p) for n in range(C2["s"] + 1)]
              for p in C2["ps"]}
    return {"continuum": cont, "g0_exact": exact0, "mehler": cf.mehler(0.0, 1.0, 1.0)}


def _slope_fit(levels, ref, p):
    """Convergence order from |A_N - A| against N on the levels whose deviation exceeds 3 sigma (and
    1e-11 relative, the accuracy of the reference): least squares of log|A_N - A| on log N over the
    longest run of such consecutive levels (N >= 2) that ends at the finest significant level. Returns
    (slope, N range, points)."""
    sig = [n for n, r in levels if n >= 1 and r.err > 0 and abs(r.amp - ref) > max(3 * r.err, 1e-11 * abs(ref))]
    if len(sig) < 2:
        return None, [], len(sig)
    run = [sig[-1]]
    for n in reversed(sig[:-1]):
        if n == run[-1] - 1:
            run.append(n)
        else:
            break
    run = sorted(run)
    if len(run) < 2:
        return None, [], 1
    x = np.array([math.log(2.0 ** n) for n in run])
    y = np.array([math.log(abs(levels[n][1].amp - ref)) for n in run])
    k = float(np.polyfit(x, y, 1)[0])
    return -k, [1 << run[0], 1 << run[-1]], len(run)


C2_PAIR_PATHS = 1 << 18     # paths whose per-path level actions give the paired differences' spread


def _pair_slope(P, ctx, g, T, p, stream, res):
    """Convergence order from the paired differences A_N - A_2N of one hierarchical run (both levels
    from the same samples, so most of the Monte Carlo noise cancels): the differences from the
    full run, their standard errors from the spread of w_N - w_2N (w = K_0 e^{-S}, the per-path
    weights) over the first C2_PAIR_PATHS paths of the same stream; least squares of log|A_N - A_2N|
    on log N over the longest run of consecutive levels that ends at the finest level whose
    difference exceeds 3 standard errors, within which every difference exceeds 3 standard errors,
    has the same sign and is smaller than the one before, then without the coarse levels whose
    local order departs by more than 1 from the median local order of the finer ones (the
    asymptotic regime); at least 3 levels, else no slope. Returns (slope, N range, points)."""
    s = C2["s"]
    S = ctx.path_actions(P.quartic(1.0, g), 1.0, 0.0, 1.0, T, 1 << s, p, 1, stream, P.FLAG_HIERARCHY, 0, C2_PAIR_PATHS)
    K0 = math.exp(-1.0 / (2.0 * T)) / math.sqrt(2.0 * math.pi * T)
    with np.errstate(over="ignore", invalid="ignore"):
        w = K0 * np.exp(-S)
    n_all = C2["samples"]
    sig = []
    np_err = np.seterr(over="ignore", invalid="ignore")
    for n in range(1, s):
        dw = w[:, n] - w[:, n + 1]
        if not np.all(np.isfinite(dw)):
            continue
        se = float(np.std(dw, ddof=1)) / math.sqrt(n_all)
        diff = res[n].amp - res[n + 1].amp
        if math.isfinite(diff) and math.isfinite(se) and se > 0 and abs(diff) > 3 * se:
            sig.append((n, diff))
    np.seterr(**np_err)
    if not sig:
        return None, [], 0
    run = [sig[-1]]
    for item in reversed(sig[:-1]):
        prev = run[-1]
        if item[0] == prev[0] - 1 and (item[1] > 0) == (prev[1] > 0) and abs(item[1]) > abs(prev[1]):
            run.append(item)
        else:
            break
    run = sorted(run)
    # the asymptotic regime: drop coarse levels while their local order (log2 of the ratio of
    # successive differences) is more than 1 away from the median local order of the finer ones
    while len(run) >= 3:
        loc = [math.log2(abs(run[i][1]) / abs(run[i + 1][1])) for i in range(len(run) - 1)]
        if abs(loc[0] - float(np.median(loc[1:]))) <= 1.0:
            break
        run = run[1:]
    if len(run) < 3:
        return None, [], len(run)
    x = np.array([n * math.log(2.0) for n, _ in run])
    y = np.array([math.log(abs(d)) for _, d in run])
    return -float(np.polyfit(x, y, 1)[0]), [1 << run[0][0], 1 << run[-1][0]], len(run)


def c2_section(P, ctx, refs):
    """Every point of the convergence sweep on the GPU: A_N^(p) for N = 1..1024 from one s = 10 run
    per (g, p, T) (1e8 samples), the 1/N^p order fitted against the DVR continuum and from the paired
    differences A_N - A_2N, the eq.(fit) extrapolation, and g = 0 against the exact discretized
    amplitude and the Mehler kernel."""
    C = C2
    s = C["s"]
    rows = {}
    tot_slices, tot_s = 0.0, 0.0
    for gi, g in enumerate(C["gs"]):
        for T in C["Ts"]:
            A_cont = refs["continuum"][f"{g:g},{T:g}"] if refs else None
            for p in C["ps"]:
                stream = 1000 + len(rows)
                res, st = ctx.amplitude(P.quartic(1.0, g), 1.0, 0.0, 1.0, T, 1 << s, p, C["samples"], 1, stream,
                                        P.FLAG_HIERARCHY)
                ms = ctx.last_kernel_ms()
                tot_slices += C["samples"] * slices_per_sample(s, True)
                tot_s += ms / 1e3
                row = {"A_N": [r.amp for r in res], "err_N": [r.err for r in res], "status": st,
                       "nonfinite": [int(r.n_nonfinite) for r in res], "kernel_ms": ms}
                ps_, pr_, pn_ = _pair_slope(P, ctx, g, T, p, stream, res)
                row.update({"pair_slope": ps_, "pair_N_range": pr_, "pair_points": pn_})
                if A_cont is not None:
                    slope, nrange, npts = _slope_fit(list(enumerate(res)), A_cont, p)
                    A, dA = _fit_continuum([(n, r) for n, r in enumerate(res) if math.isfinite(r.err)], p)
                    row.update({"continuum_dvr": A_cont, "slope": slope, "slope_N_range": nrange,
                                "slope_points": npts, "fit_A": A, "fit_err": dA,
                                "z_N1024": (res[s].amp - A_cont) / res[s].err if res[s].err > 0 else None})
                rows[f"g={g:g},p={p},T={T:g}"] = row
    g0 = {}
    if refs:
        for p in C["ps"]:
            res, st = ctx.amplitude(P.quartic(1.0, 0.0), 1.0, 0.0, 1.0, 1.0, 1 << s, p, C["samples"], 1, 2000 + p,
                                    P.FLAG_HIERARCHY)
            ex = refs["g0_exact"][str(p)]
            z = [(res[n].amp - ex[n]) / res[n].err for n in range(1, s + 1)]
            exact_slope, _, _ = _slope_fit([(n, P.LevelResult(ex[n], 1e-300, 0, 0, 0, 0, 0)) for n in range(s + 1)],
                                           refs["mehler"], p)
            g0[str(p)] = {"max_abs_z_vs_exact_discretized": float(np.max(np.abs(z))), "z": z,
                          "A_1024": res[s].amp, "exact_1024": ex[s], "mehler": refs["mehler"],
                          "exact_slope_vs_mehler": exact_slope, "status": st}
    return {"workload": f"V=q^2/2+g q^4/24, g in {list(C['gs'])}, p in {list(C['ps'])}, T in {list(C['Ts'])}, a=0, b=1, "
                        f"one s={s} run per point with every level, {C['samples']:.0e} samples each; g=0 at T=1",
            "points": rows, "g0": g0, "slice_evals_per_s": tot_slices / tot_s, "device_s": tot_s}


def _train_and_estimate(P, ctx, coefs, N, batch, steps, est_stream, run_to_target):
    """Train, measure relvar on est_samples, then (run_to_target) estimate again from the predicted
    n* = relvar / target^2 samples on a fresh stream and time that run."""
    F = FLOW
    f = P.Flow(ctx, coefs, 1.0, 0.0, 1.0, F["T"], N, F["p"], layers=F["layers"], batch=batch, lr=F["lr"],
               beta=F["beta"])
    untrained, _, _ = f.amplitude(F["est_samples"], 1, est_stream)
    losses, train_ms = f.train(1, 1 << 31, steps)
    f.amplitude(1 << 20, 1, est_stream)                      # warm
    trained, est_ms, _ = f.amplitude(F["est_samples"], 1, est_stream)
    final = None
    if run_to_target:
        n_star = int(math.ceil(trained.relvar / F["target"] ** 2))
        r, ms, _ = f.amplitude(n_star, 1, est_stream + 1)
        final = {"samples": n_star, "A": r.amp, "err": r.err, "rel_err": r.err / r.amp, "device_s": ms / 1e3}
    f.close()
    return untrained, trained, losses, train_ms, F["est_samples"] / (est_ms / 1e3), final


def proposal_section(P, ctx, steps):
    """Plain bisection sampler against the trained affine-coupling proposal on one problem: weight
    variance, effective sample size, estimation rate, training time, and the device time to reach
    a relative error of 1e-5 (samples needed n* = relvar / 1e-10, predicted from the measured rate,
    then run: the n*-sample estimate on a fresh stream, its achieved relative error and device
    time). Two training shapes over the same number of training paths: batches of 4096, and
    batches of 16384 (fewer, wider steps)."""
    F = FLOW
    coefs = P.quartic(1.0, F["g"])
    N = 1 << F["s"]
    est_stream = 1 << 30
    res, _ = ctx.amplitude(coefs, 1.0, 0.0, 1.0, F["T"], N, F["p"], F["plain_samples"], 1, est_stream, 0)
    plain = res[F["s"]]
    plain_rate = F["plain_samples"] / (ctx.last_kernel_ms() / 1e3)
    tgt2 = F["target"] ** 2
    t_plain = plain.relvar / tgt2 / plain_rate
    # run the plain sampler to its predicted n* (level s only, fresh stream)
    n_star = int(math.ceil(plain.relvar / tgt2))
    res2, _ = ctx.amplitude(coefs, 1.0, 0.0, 1.0, F["T"], N, F["p"], n_star, 1, est_stream + 1, 0)
    plain_final = {"samples": n_star, "A": res2[F["s"]].amp, "err": res2[F["s"]].err,
                   "rel_err": res2[F["s"]].err / res2[F["s"]].amp, "device_s": ctx.last_kernel_ms() / 1e3}
    out = {
        "workload": f"V=q^2/2+{F['g']:g} q^4/24, p={F['p']}, N={N}, T={F['T']:g}, a=0, b=1; {F['layers']} affine "
                    f"couplings (bf16 MFMA MLPs 64-128-128), Adam lr {F['lr']:g}, loss {1 - F['beta']:g} log E[w^2] + "
                    f"{F['beta']:g} KL, {steps * F['batch']:.3g} training paths",
        "plain": {"A": plain.amp, "err": plain.err, "relvar": plain.relvar, "ess_frac": plain.ess / plain.n,
                  "paths_per_s": plain_rate, "samples": plain.n, "time_to_rel_err_1e-5_s": t_plain,
                  "run_to_target": plain_final},
    }
    for key, batch in (("proposal", F["batch"]), ("proposal_wide_batch", F["wide_batch"])):
        nsteps = max(1, steps * F["batch"] // batch)
        untrained, trained, losses, train_ms, rate, final = _train_and_estimate(P, ctx, coefs, N, batch, nsteps,
                                                                                est_stream, run_to_target=True)
        t_est = trained.relvar / tgt2 / rate
        out[key] = {
            "batch": batch, "steps": nsteps, "train_ms": train_ms, "train_paths": nsteps * batch,
            "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
            "relvar_untrained": untrained.relvar,
            "A": trained.amp, "err": trained.err, "relvar": trained.relvar, "ess_frac": trained.ess / trained.n,
            "paths_per_s": rate, "samples": trained.n,
            "agreement_sigma": abs(trained.amp - plain.amp) / math.hypot(trained.err, plain.err),
            "relvar_ratio": plain.relvar / trained.relvar,
            "time_to_rel_err_1e-5_s": {"estimation": t_est, "with_training": t_est + train_ms / 1e3},
            "run_to_target": final,
        }
    return out


def batched_section(P, ctx, samples, tune_samples):
    """Batched grid: 2 systems x 3 T x 3 p x 128 x 128 endpoints, mixed N. The autotuner picks a
    launch shape per kernel class (and the grid and grab) on the same grid with tune_samples per
    task; the choice is cached and applied to the grid with `samples` per task, run as graph replays
    of at most C3_REPLAY_SAMPLES per task on disjoint streams and merged per task (equal counts: the
    mean of the replay estimates, their errors added in quadrature)."""
    from paper_1105_0542_amd import workloads
    tune_path = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"pimc_batch_tune_{os.getpid()}.txt")
    t0 = time.perf_counter()
    systems, rows_t = workloads.evolution_matrix_tasks(samples=tune_samples)
    bt = P.Batch(ctx, systems, rows_t, seed=1, flags=0)
    choice = bt.autotune(tune_path)
    tuned_classes = bt.classes()
    _, tuned_small_ms, _ = bt.run()
    for k in range(len(tuned_classes)):
        bt.set_shape(k, 0)
    bt.set_tuning(2, 1)
    _, default_small_ms, _ = bt.run()
    bt.close()
    t_tune = time.perf_counter() - t0
    _progress(f"batched: autotuned in {t_tune:.1f} s")
    n_tasks = len(rows_t)
    replays = max(1, -(-samples // C3_REPLAY_SAMPLES))
    per = -(-samples // replays)
    amp_sum = err2 = None
    n_tot = nonfinite = None
    ms_total = t_plan = 0.0
    st = 0
    for r in range(replays):
        t0 = time.perf_counter()
        systems, rows = workloads.evolution_matrix_tasks(samples=per, stream_base=r * n_tasks)
        bt = P.Batch(ctx, systems, rows, seed=1, flags=0)
        applied = bt.autotune(tune_path)                 # the cached choice: no timing
        t_plan += time.perf_counter() - t0
        out, ms, st_r = bt.run()
        bt.close()
        st = st or st_r
        ms_total += ms
        lev = np.array([int(row[5]).bit_length() - 1 for row in rows])
        res = out[np.arange(len(rows)), lev]
        if amp_sum is None:
            amp_sum, err2 = np.zeros(len(rows)), np.zeros(len(rows))
            n_tot, nonfinite = np.zeros(len(rows), dtype=np.int64), np.zeros(len(rows), dtype=np.int64)
        amp_sum += res["amp"]
        err2 += res["err"] ** 2
        n_tot += res["n"].astype(np.int64)
        nonfinite += res["n_nonfinite"].astype(np.int64)
        _progress(f"batched: replay {r + 1}/{replays} ({per} samples per task) {ms / 1e3:.1f} s")
    amp = amp_sum / replays
    err = np.sqrt(err2) / replays
    rel = err / np.abs(amp)
    slices = sum(row[7] * row[5] for row in rows) * replays
    # FP64 operations: per slice 2 (E_p - 1) for the Horner chains plus 6, as for the headline kernel
    flops = sum(row[7] * row[5] * (2 * (E_TABLE[row[6]] - 1) + 6) for row in rows) * replays
    classes = [{"p": c["p"], "N": "16" if c["n16"] else "32..512", "tasks": c["n_tasks"],
                "shape": {"subtree_levels": c["subtree_levels"], "block": c["block"],
                          "waves_per_eu": c["waves_per_eu"], "slice_batch": c["slice_batch"]},
                "candidates": c["n_shapes"], "tuned_ms": c["tuned_ms"], "default_ms": c["default_ms"],
                "gain": c["default_ms"] / c["tuned_ms"] if c["tuned_ms"] > 0 else None} for c in tuned_classes]
    line = {
        "workload": "128x128 endpoint grid on [-4,4]^2, (A,g) in {(1,1),(-1,4)}, T in {0.5,1,2}, p in {8,12,18}, "
                    f"N in 16..512 by a fixed hash, {per * replays} samples per task, level N only",
        "tasks": n_tasks, "samples_per_task": per * replays, "replays": replays, "samples_per_replay": per,
        "graph_ms": ms_total, "slice_evals_per_s": slices / (ms_total / 1e3),
        "fp64_frac": flops / (ms_total / 1e3) / 1e12 / FP64_PEAK_TFLOPS,
        "rel_err_median": float(np.median(rel)), "rel_err_p99": float(np.quantile(rel, 0.99)),
        "samples_counted": int(n_tot.sum()),
        "autotune": {"tuned_on_samples_per_task": tune_samples, "tune_s": t_tune, "grid_mult_x2": choice[0],
                     "grab": choice[1], "applied": list(applied), "classes": classes,
                     "graph_ms_tuned": tuned_small_ms, "graph_ms_default": default_small_ms},
        "plan_s": t_plan, "tasks_with_nonfinite_weights": int((nonfinite > 0).sum()),
        "nonfinite_weights": int(nonfinite.sum()), "status": st,
    }
    try:
        os.remove(tune_path)
    except OSError:
        pass
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--samples", type=int, default=N_SAMPLES)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision-samples", type=int, default=PREC["samples"])
    ap.add_argument("--batch-samples", type=int, default=C3_SAMPLES,
                    help="samples per task of the batched 128x128 grid (0 skips it)")
    ap.add_argument("--batch-tune-samples", type=int, default=C3_TUNE_SAMPLES,
                    help="samples per task of the grid the autotuner times")
    ap.add_argument("--c2-samples", type=int, default=C2["samples"],
                    help="samples per point of the convergence sweep (0 skips it)")
    ap.add_argument("--only-c2", action="store_true", help="run only the convergence sweep, with its CPU references")
    ap.add_argument("--copy-probe", action="store_true", help="only run the 512 MiB copy used to scale HBM counters")
    ap.add_argument("--only-headline", action="store_true",
                    help="run only the timed p=18 sweep (for profiler runs): no other section, no cpu baseline")
    ap.add_argument("--only-proposal", action="store_true",
                    help="run only the proposal section (for profiler runs): no other section, no cpu baseline")
    ap.add_argument("--only-general", action="store_true", help="run only the general-potential section")
    ap.add_argument("--only-mpt", action="store_true",
                    help="run only the Poeschl-Teller convergence section, with its DVR reference")
    ap.add_argument("--only-vector", action="store_true",
                    help="run only the several-coordinate section, with its DVR reference")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the batched-grid section (for profiler runs): no other section, no cpu baseline")
    ap.add_argument("--only-spectrum", action="store_true",
                    help="run only the spectrum section (for profiler runs), with its DVR reference")
    ap.add_argument("--flow-steps", type=int, default=FLOW["steps"],
                    help="training steps of the learned proposal (0 skips the proposal section)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU per process; splitting path ranges over "
                                   "several GPUs is not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    # The oracle runs first, in worker processes forked before this process touches the GPU.
    skip_cpu = (args.no_cpu_baseline or args.only_headline or args.only_proposal or args.only_spectrum or
                args.only_mpt or args.only_general or args.only_vector or args.only_batched or args.only_c2)
    C2["samples"] = args.c2_samples
    c2_refs = c2_references() if ((not skip_cpu or args.only_c2) and args.c2_samples > 0) else None
    if c2_refs is not None:
        _progress("convergence-sweep references done")
    cpu = None if skip_cpu else cpu_baseline(CPU_SAMPLE_PATHS)
    if cpu is not None:
        _progress(f"cpu baseline done ({cpu['value']:.3g} {cpu['unit']})")
    prec_ref = None if skip_cpu else oracle_precision_reference()
    spec_ref = None if (skip_cpu and not args.only_spectrum) else oracle_spectrum_reference()
    mpt_ref = None if (skip_cpu and not args.only_mpt) else oracle_mpt_reference()
    vec_ref = None if (skip_cpu and not args.only_vector) else oracle_vector_reference()
    wanted = []
    for name, only in (("vector", args.only_vector), ("mpt", args.only_mpt), ("general", args.only_general),
                       ("spectrum", args.only_spectrum)):
        if (not skip_cpu or only) and not args.no_cpu_baseline:
            wanted.append(name)
    bases = oracle_section_baselines(wanted) if wanted else {}
    if not skip_cpu:
        _progress("oracle references and section baselines done")

    import paper_1105_0542_amd as P

    ctx = P.Context(device=0)
    H = P.FLAG_HIERARCHY
    if args.only_proposal:
        print(json.dumps({"proposal": proposal_section(P, ctx, args.flow_steps)}), flush=True)
        ctx.close()
        return
    if args.only_batched:
        print(json.dumps({"batched": batched_section(P, ctx, args.batch_samples, args.batch_tune_samples)}), flush=True)
        ctx.close()
        return
    if args.only_c2:
        print(json.dumps({"c2": c2_section(P, ctx, c2_refs)}), flush=True)
        ctx.close()
        return
    if args.only_spectrum:
        print(json.dumps({"spectrum": spectrum_section(P, ctx, spec_ref, bases.get("spectrum"))}), flush=True)
        ctx.close()
        return
    if args.only_mpt:
        print(json.dumps({"mpt": mpt_section(P, ctx, mpt_ref, bases.get("mpt"))}), flush=True)
        ctx.close()
        return
    if args.only_general:
        print(json.dumps({"general": general_section(P, ctx, bases.get("general"))}), flush=True)
        ctx.close()
        return
    if args.only_vector:
        print(json.dumps({"vector": vector_section(P, ctx, vec_ref, bases.get("vector"))}), flush=True)
        ctx.close()
        return
    N = 1 << S_DEPTH

    def step():
        out = []
        kms = 0.0
        for i, (g, T) in enumerate(POINTS):
            res, st = ctx.amplitude(P.quartic(1.0, g), 1.0, 0.0, 1.0, T, N, P_LEVEL, args.samples, 1, i, H)
            kms += ctx.last_kernel_ms()
            out.append((g, T, res))
        return out, kms

    for _ in range(args.warmup):
        step()
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kernel_ms = 0.0
    last = None
    for _ in range(args.steps):
        last, kms = step()
        kernel_ms += kms
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    _progress(f"headline: {args.steps} timed steps in {wall:.2f} s")
    slices_step = len(POINTS) * args.samples * slices_per_sample(S_DEPTH, True)
    value = slices_step * args.steps / wall
    launches = args.steps * len(POINTS)
    kernel_avg_s = kernel_ms / launches / 1e3
    flop_per_launch = args.samples * slices_per_sample(S_DEPTH, True) * FLOP_PER_SLICE
    achieved = flop_per_launch / kernel_avg_s / 1e12

    if args.only_headline:
        print(json.dumps({"metric": "slice-evals/s (p=18, FP64)", "value": value, "unit": "slice-evals/s",
                          "kernel_avg_ms": kernel_avg_s * 1e3, "steps": args.steps, "warmup": args.warmup,
                          "samples_per_point": args.samples, "note": "headline sweep only"}), flush=True)
        ctx.close()
        return

    # level-s only (no hierarchy): one point, same kernel family, for the second figure
    res_s, _ = ctx.amplitude(P.quartic(1.0, 10.0), 1.0, 0.0, 1.0, 1.0, N, P_LEVEL, args.samples, 1, 100, 0)
    ms_s = ctx.last_kernel_ms()
    level_s_rate = args.samples * slices_per_sample(S_DEPTH, False) / (ms_s / 1e3)

    # precision workload: FP64 and FP32 slice polynomials on identical samples (level s only)
    prec = {}
    g, pp, ss, TT, ns = PREC["g"], PREC["p"], PREC["s"], PREC["T"], args.precision_samples
    for name, fl in (("fp64", 0), ("fp32", P.FLAG_FP32_POLY)):
        r, _ = ctx.amplitude(P.quartic(1.0, g), 1.0, 0.0, 1.0, TT, 1 << ss, pp, ns, 1, 0, fl)
        ms = ctx.last_kernel_ms()
        prec[name] = {"A_512": r[ss].amp, "err": r[ss].err, "slice_evals_per_s": ns * (1 << ss) / (ms / 1e3),
                      "kernel_ms": ms}
    small = {}
    for name, fl in (("fp64", 0), ("fp32", P.FLAG_FP32_POLY)):
        r, _ = ctx.amplitude(P.quartic(1.0, g), 1.0, 0.0, 1.0, TT, 1 << ss, pp, PREC["oracle_paths"], 1, 0, fl)
        small[name] = r[ss].amp
    prec_line = {
        "workload": f"V=q^2/2+{g:g} q^4/24, p={pp}, N={1 << ss}, T={TT:g}, a=0, b=1, {ns:.0e} samples, level s only",
        "fp64": prec["fp64"], "fp32": prec["fp32"],
        "rel_diff_fp32_vs_fp64_gpu": abs(prec["fp32"]["A_512"] - prec["fp64"]["A_512"]) / prec["fp64"]["A_512"],
        "rel_stat_err": prec["fp64"]["err"] / prec["fp64"]["A_512"],
        "fp32_frac_of_fp32_peak": prec["fp32"]["slice_evals_per_s"] * FLOP_PER_SLICE / 1e12 / 157.3,
        "note": "FP32 polynomials run as non-packed FP32 (packed FP32 instructions are disabled at compile time), "
                "whose issue rate equals FP64 on MI355X; the 157.3 TFLOP/s FP32 peak needs packed FP32",
    }
    if prec_ref is not None:
        prec_line[f"oracle_first_{PREC['oracle_paths']}"] = {
            "A_512": prec_ref,
            "rel_diff_fp64_gpu": abs(small["fp64"] - prec_ref) / prec_ref,
            "rel_diff_fp32_gpu": abs(small["fp32"] - prec_ref) / prec_ref}

    _progress("level-s-only and precision sections done")
    batch_line = (batched_section(P, ctx, args.batch_samples, args.batch_tune_samples)
                  if args.batch_samples > 0 else None)
    c2_line = c2_section(P, ctx, c2_refs) if args.c2_samples > 0 else None
    _progress("convergence sweep done")
    flow_line = proposal_section(P, ctx, args.flow_steps) if args.flow_steps > 0 else None
    _progress("proposal section done")
    spec_line = spectrum_section(P, ctx, spec_ref, bases.get("spectrum"))
    mpt_line = mpt_section(P, ctx, mpt_ref, bases.get("mpt"))
    _progress("spectrum and Poeschl-Teller sections done")
    gen_line = general_section(P, ctx, bases.get("general"))
    vec_line = vector_section(P, ctx, vec_ref, bases.get("vector"))
    _progress("general and vector sections done")

    counters = measured_counter_flops()
    roofline = {
        "bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
        "frac": achieved / FP64_PEAK_TFLOPS, "traffic": measured_traffic(args.samples),
        "kernel": "k_amplitude<Shape<4,256,2,16>, QuarticEval64<18>>", "kernel_avg_ms": kernel_avg_s * 1e3,
        "flop_per_slice": FLOP_PER_SLICE, "flop_per_launch": flop_per_launch,
    }
    if counters is not None:
        # hardware FP64 FLOPs (all of them: slices, Box-Muller, bridge, reductions) per launch at this size
        hw = counters["fp64_flops_per_sample"] * args.samples
        roofline["counter_frac"] = hw / kernel_avg_s / 1e12 / FP64_PEAK_TFLOPS
        roofline["counter_valu_insts_per_sample"] = counters["valu_insts_per_sample"]
    line = {
        "metric": "slice-evals/s (p=18, FP64)",
        "value": value,
        "unit": "slice-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (Philox4x32-10 samples, seed 1, stream = point index)",
        "config": {
            "workload": "p=18 column of the convergence sweep: V=q^2/2+g q^4/24, g in {1,10,48}, T in {1,2,5}, "
                        "a=0, b=1, N=2^1..2^10 from one s=10 bisection run per point, "
                        f"{args.samples:.0e} samples per point",
            "p": P_LEVEL, "s": S_DEPTH, "samples_per_point": args.samples, "points": len(POINTS),
            "slice_evals_per_sample": slices_per_sample(S_DEPTH, True),
        },
        "roofline": roofline,
        "results": {f"g={g:g},T={T:g}": {"A_1024": r[S_DEPTH].amp, "err": r[S_DEPTH].err,
                                          "relvar": r[S_DEPTH].relvar, "nonfinite": r[S_DEPTH].n_nonfinite}
                    for (g, T, r) in last},
    }
    # detailed sections first (long arrays), then a compact summary of every section as the last key
    # (after cpu_baseline), so that the end of the line -- what a log tail keeps -- carries the figures
    if c2_line is not None:
        line["c2"] = c2_line
    line["spectrum"] = spec_line
    line["mpt"] = mpt_line
    line["general"] = gen_line
    line["vector"] = vec_line
    if flow_line is not None:
        line["proposal"] = flow_line
    if batch_line is not None:
        line["batched"] = batch_line
    line["precision"] = prec_line
    line["level_s_only"] = {"slice_evals_per_s": level_s_rate,
                            "frac": level_s_rate * FLOP_PER_SLICE / 1e12 / FP64_PEAK_TFLOPS,
                            "note": "same point g=10 T=1 without the coarser levels: 1024 slices per sample"}
    if cpu is not None:
        line["cpu_baseline"] = cpu
    line["summary"] = summarize(line)
    print(json.dumps(line), flush=True)
    ctx.close()


def _r(x, d=4):
    return None if x is None else float(f"{x:.{d}g}")


def summarize(line):
    """Compact figures of every section (about 2 KB past the convergence tables) for the end of the
    line: the convergence slopes first, the headline last."""
    out = {"headline": {"value": _r(line["value"]), "frac": _r(line["roofline"]["frac"]),
                        "counter_frac": _r(line["roofline"].get("counter_frac")),
                        "kernel_avg_ms": _r(line["roofline"]["kernel_avg_ms"])},
           "level_s_only": {"value": _r(line["level_s_only"]["slice_evals_per_s"]),
                            "frac": _r(line["level_s_only"]["frac"])}}
    pr = line.get("precision")
    if pr:
        out["precision"] = {"fp64_rate": _r(pr["fp64"]["slice_evals_per_s"]), "fp32_rate": _r(pr["fp32"]["slice_evals_per_s"]),
                            "rel_diff_fp32_vs_fp64_gpu": _r(pr["rel_diff_fp32_vs_fp64_gpu"]),
                            "rel_stat_err": _r(pr["rel_stat_err"])}
        for k, v in pr.items():
            if k.startswith("oracle_first_"):
                out["precision"][k] = {kk: _r(vv) for kk, vv in v.items()}
    b = line.get("batched")
    if b:
        out["batched"] = {"samples_per_task": b["samples_per_task"], "replays": b.get("replays"),
                          "graph_s": _r(b["graph_ms"] / 1e3), "rel_err_median": _r(b.get("rel_err_median")),
                          "slice_evals_per_s": _r(b["slice_evals_per_s"]), "fp64_frac": _r(b["fp64_frac"]),
                          "graph_ms_tuned_vs_default_small": [_r(b["autotune"]["graph_ms_tuned"]),
                                                              _r(b["autotune"]["graph_ms_default"])],
                          "classes": [[c["p"], c["N"], [c["shape"][k] for k in ("subtree_levels", "block",
                                                                                  "waves_per_eu", "slice_batch")],
                                       _r(c["gain"], 3)] for c in b["autotune"]["classes"]]}
    f = line.get("proposal")
    if f:
        out["proposal"] = {"plain": {"relvar": _r(f["plain"]["relvar"]), "t_1e-5_s": _r(f["plain"]["time_to_rel_err_1e-5_s"]),
                                     "run_s": _r(f["plain"]["run_to_target"]["device_s"])}}
        for key in ("proposal",):                  # the configured batch (the wide one: detailed section)
            if key in f:
                g = f[key]
                out["proposal"][key] = {"batch": g["batch"], "train_s": _r(g["train_ms"] / 1e3), "relvar": _r(g["relvar"]),
                                        "ess_frac": _r(g["ess_frac"]),
                                        "t_1e-5_s": _r(g["time_to_rel_err_1e-5_s"]["estimation"]),
                                        "t_1e-5_with_training_s": _r(g["time_to_rel_err_1e-5_s"]["with_training"]),
                                        "run_s": _r(g["run_to_target"]["device_s"]) if g.get("run_to_target") else None,
                                        "agreement_sigma": _r(g["agreement_sigma"], 3)}
    c = line.get("c2")
    if c:
        slopes = {}
        pair = {}
        for key, r in c["points"].items():
            g, p, T = key.split(",")
            if r.get("slope") is not None:
                slopes.setdefault(f"{g},{T}", {})[p.split("=")[1]] = _r(r["slope"], 3)
            if r.get("pair_slope") is not None:
                pair.setdefault(f"{g},{T}", {})[p.split("=")[1]] = _r(r["pair_slope"], 3)
        out["c2"] = {"slice_evals_per_s": _r(c["slice_evals_per_s"]), "slopes": slopes, "pair_slopes": pair,
                     "g0_max_abs_z": {p: _r(v["max_abs_z_vs_exact_discretized"], 3) for p, v in c["g0"].items()},
                     "max_abs_z_N1024_vs_dvr": {}, "max_abs_z_fit_vs_dvr": {}}
        for key, r in c["points"].items():
            p_key = key.split(",")[1].split("=")[1]
            if r.get("z_N1024") is not None:
                zmax = out["c2"]["max_abs_z_N1024_vs_dvr"]
                zmax[p_key] = max(zmax.get(p_key, 0.0), _r(abs(r["z_N1024"]), 3))
            if r.get("fit_err") and r.get("continuum_dvr") is not None:
                zf = abs(r["fit_A"] - r["continuum_dvr"]) / r["fit_err"]
                zmax = out["c2"]["max_abs_z_fit_vs_dvr"]
                zmax[p_key] = max(zmax.get(p_key, 0.0), _r(zf, 3))
    out["mpt"] = {p: {"rate": _r(r["slice_evals_per_s"]), "frac": _r(r["fp64_frac"])} for p, r in line["mpt"]["per_p"].items()}
    gq = line["general"]["quartic_g10_general_mode"]
    out["general"] = {"rate": _r(gq["slice_evals_per_s"]), "frac": _r(gq["roofline"]["frac"])}
    g18 = line["general"].get("gaussian_barrier_p18")
    if g18:
        out["general"]["p18"] = {"rate": _r(g18["slice_evals_per_s"]), "frac": _r(g18["roofline"]["frac"]),
                                 "diff_vs_p8_sigma": _r(g18["diff_vs_p8_in_sigma"], 3)}
    out["vector"] = {d: {"rate": _r(r["slice_evals_per_s"]), "frac": _r(r["fp64_frac"])} for d, r in line["vector"]["per_dim"].items()}
    out["vector"]["component"] = [{"rate": _r(r["slice_evals_per_s"]), "frac": _r(r["fp64_frac"])}
                                  for r in line["vector"].get("component", [])]
    out["spectrum"] = [{"matrix_ms": _r(r["matrix_ms"]), "lanczos_ms_per_step": _r(r["lanczos_ms_per_step"]),
                        "max_abs_diff_vs_dvr": _r(r.get("max_abs_diff_vs_dvr"), 3)} for r in line["spectrum"]]
    order = ("c2", "spectrum", "general", "mpt", "vector", "batched", "proposal", "precision", "level_s_only",
             "headline")
    return {k: out[k] for k in order if k in out}


if __name__ == "__main__":
    main()
