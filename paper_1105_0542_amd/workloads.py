"""Synthetic workloads (inputs only; no part of the estimator's arithmetic).

The paper's experiments use model potentials, not datasets (Sec. 3.3, Sec. 4.2): the anharmonic
oscillator V = A q^2/2 + g q^4/24 and endpoints/times chosen per study. These generators produce
the inputs of the benchmarks and tests deterministically.
"""
from __future__ import annotations

from typing import List, Tuple

MASK64 = (1 << 64) - 1


def quartic_coefs(A: float, g: float) -> List[float]:
    """V = A q^2/2 + g q^4/24 as polynomial coefficients."""
    return [0.0, 0.0, A / 2.0, 0.0, g / 24.0]


def splitmix64(x: int) -> int:
    """SplitMix64 finalizer (Steele, Lea, Flood, OOPSLA 2014): a fixed integer hash."""
    x = (x + 0x9E3779B97F4A7C15) & MASK64
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & MASK64
    return x ^ (x >> 31)


def endpoint_grid(n: int = 128, lo: float = -4.0, hi: float = 4.0) -> List[float]:
    """Evenly spaced endpoints lo + (hi - lo) i/(n-1), i = 0..n-1 (a matrix of A(x_i, x_j; T))."""
    return [lo + (hi - lo) * i / (n - 1) for i in range(n)]


def evolution_matrix_tasks(n_grid: int = 128, samples: int = 10_000, seed: int = 1,
                           systems: Tuple[Tuple[float, float], ...] = ((1.0, 1.0), (-1.0, 4.0)),
                           times=(0.5, 1.0, 2.0), levels=(8, 12, 18), s_choices=(4, 5, 6, 7, 8, 9),
                           stream_base: int = 0):
    """Batched grid: every (system, T, p, a_i, b_j), N = 2^s with s from a fixed hash of the task
    index (s = s_choices[splitmix64(seed*2^32 + j) mod len]). Returns (system coefficient lists,
    task rows (system, m, a, b, T, N, p, samples, stream)); stream = stream_base + task index, so
    that runs with stream bases a task count apart draw disjoint samples."""
    xs = endpoint_grid(n_grid)
    sys_coefs = [quartic_coefs(A, g) for (A, g) in systems]
    rows = []
    j = 0
    for si in range(len(systems)):
        for T in times:
            for p in levels:
                for a in xs:
                    for b in xs:
                        s = s_choices[splitmix64(((seed & 0xFFFFFFFF) << 32) + j) % len(s_choices)]
                        rows.append((si, 1.0, a, b, T, 1 << s, p, samples, stream_base + j))
                        j += 1
    return sys_coefs, rows
