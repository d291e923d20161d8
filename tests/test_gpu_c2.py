"""The convergence sweep's checks on the GPU (Sec. 4: errors of A_N^(p) fall as 1/N^p; eq.(fit)):
the harmonic case g = 0 against the exact discretized amplitude at every N and p, and the fitted
convergence order of the anharmonic oscillator against a grid-diagonalization continuum."""
import math

import numpy as np
import pytest

import paper_1105_0542_amd as P
from oracle import closed_forms as cf
from oracle import effective_action as ea

pytestmark = pytest.mark.gpu

S = 10


@pytest.fixture(scope="module")
def ctx():
    c = P.Context()
    yield c
    c.close()


@pytest.mark.parametrize("p", [1, 2, 4, 8, 12, 18])
def test_harmonic_levels_match_the_exact_discretized_amplitude(ctx, p):
    """g = 0: every level N = 2^1..2^10 of one s = 10 run within 5 standard errors of the exact
    A_N^(p) (a Gaussian integral, mpmath; its approach to the Mehler kernel as 1/N^p is pinned by
    the oracle tests)."""
    n = 4_000_000
    print(f"g=0 p={p} s={S} n={n}", flush=True)
    res, st = ctx.amplitude(P.quartic(1.0, 0.0), 1.0, 0.0, 1.0, 1.0, 1 << S, p, n, 1, 2000 + p, P.FLAG_HIERARCHY)
    assert st == 0
    for lev in range(1, S + 1):
        exact = cf.gaussian_discretized(0.0, 1.0, 1.0, 1 << lev, p)
        assert abs(res[lev].amp - exact) <= 5 * res[lev].err, (lev, res[lev].amp, exact, res[lev].err)


def _order(res, ref, levels):
    x = np.log([2.0 ** n for n in levels])
    y = np.log([abs(res[n].amp - ref) for n in levels])
    return -np.polyfit(x, y, 1)[0]


@pytest.mark.parametrize("p,levels,n", [(1, (4, 5, 6, 7), 20_000_000), (2, (1, 2, 3), 200_000_000)])
def test_anharmonic_convergence_order(ctx, p, levels, n):
    """g = 10, T = 1: log|A_N - A| against log N over levels where the discretization error is many
    standard errors above the noise has slope -p (the 1/N^p law, Sec. 4); A from sinc-DVR. (At p = 2
    the significant levels are N = 2..8, still pre-asymptotic: local orders 1.7-1.8.)"""
    print(f"g=10 p={p} order, n={n}", flush=True)
    res, st = ctx.amplitude(P.quartic(1.0, 10.0), 1.0, 0.0, 1.0, 1.0, 1 << S, p, n, 1, 3000 + p, P.FLAG_HIERARCHY)
    ref = cf.dvr_amplitude(cf.quartic_V(1.0, 10.0), 0.0, 1.0, 1.0)
    for lev in levels:
        assert abs(res[lev].amp - ref) > 8 * res[lev].err, (lev, res[lev].amp, ref, res[lev].err)
    k = _order(res, ref, levels)
    assert abs(k - p) < 0.2 * p, k


def test_anharmonic_levels_match_the_discretized_amplitude(ctx):
    """g = 10, p = 4, T = 1: every level N = 2..1024 of one s = 10 run within 5 standard errors of
    A_N^(4) computed by repeated quadrature of the level-4 short-time amplitudes (the discretized
    integral of Sec. 4 evaluated deterministically)."""
    n = 20_000_000
    res, st = ctx.amplitude(P.quartic(1.0, 10.0), 1.0, 0.0, 1.0, 1.0, 1 << S, 4, n, 1, 3100, P.FLAG_HIERARCHY)
    assert st == 0
    V = ea.quartic(1, 10)
    for lev in range(1, S + 1):
        ref = cf.transfer_discretized(V, 4, 0.0, 1.0, 1.0, 1 << lev, L=6.0, h=0.025)
        assert abs(res[lev].amp - ref) <= 5 * res[lev].err, (lev, res[lev].amp, ref, res[lev].err)
