"""Pins of the oracle's paths, actions and Monte Carlo amplitude (O3/O4) against exact results."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import effective_action as ea
from oracle import pimc


def _z(res, exact):
    return (res["amp"] - exact) / res["err"]


def test_free_particle_is_exact():
    """V = 0: every weight is 1, so A_n = K_0 exactly with zero error at every level (Sec. 2.1)."""
    K0 = math.exp(-0.5) / math.sqrt(2 * math.pi)
    assert pimc.free_kernel(0.0, 1.0, 1.0) == pytest.approx(0.24197072451914337, rel=1e-15)
    assert abs(pimc.free_kernel(0.0, 1.0, 1.0) - K0) < 1e-16
    res = pimc.amplitude(ea.poly([]), 1, 0.0, 1.0, 1.0, 5, 4, 3000, 1, 0)
    for r in res:
        assert r["amp"] == pytest.approx(K0, rel=1e-15)
        assert r["err"] == 0.0


def test_free_particle_dvr_agrees():
    """The grid-diagonalization reference itself reproduces K_0 (pins that reference)."""
    assert cf.dvr_amplitude(lambda x: 0 * x, 0.0, 1.0, 1.0) == pytest.approx(0.24197072451914337, rel=1e-11)


def test_dvr_reproduces_mehler():
    assert cf.dvr_amplitude(cf.quartic_V(1, 0), 0.0, 1.0, 1.0) == pytest.approx(cf.mehler(0, 1, 1), rel=1e-11)
    assert cf.dvr_amplitude(cf.quartic_V(4, 0), -0.5, 1.0, 0.7) == pytest.approx(
        cf.mehler(-0.5, 1.0, 0.7, A=4), rel=1e-11)


def test_mehler_effective_potential_reproduces_the_kernel():
    """The exact oscillator effective potential W*(x, xbar; T) in the ideal-action form of Sec. 2.1:
    (2 pi T)^(-1/2) exp(-(b-a)^2/(2T) - T W*) is the Mehler kernel."""
    for a, b, T in ((0.0, 1.0, 1.0), (-0.7, 0.4, 0.3), (1.5, 2.0, 2.5)):
        x, xb = 0.5 * (a + b), 0.5 * (b - a)
        got = math.exp(-(b - a) ** 2 / (2 * T) - T * cf.mehler_W(x, xb, T)) / math.sqrt(2 * math.pi * T)
        assert got == pytest.approx(cf.mehler(a, b, T), rel=1e-14)


@pytest.mark.parametrize("p", [2, 4, 6])
def test_level_tables_approach_the_exact_oscillator_potential(p):
    """eps W_p agrees with eps W* to order eps^p (the error of the level-p action is O(eps^(p+1)),
    Sec. 2.1): halving eps divides the difference by 2^(p+1)."""
    x = np.array([-1.3, 0.2, 0.9])
    xb = np.array([0.05, -0.2, 0.1])
    diffs = []
    for eps in (0.1, 0.05):
        tab = pimc.level_tables(ea.quartic(1, 0), p, eps, 0)[0]
        exact = np.array([eps * cf.mehler_W(xi, xbi, eps) for xi, xbi in zip(x, xb)])
        diffs.append(np.abs(pimc.eps_W(tab, x, xb) - exact))
    assert np.all(np.abs(np.log2(diffs[0] / diffs[1]) - (p + 1)) < 0.15), diffs


@pytest.mark.parametrize("p,slope", [(1, 1.0), (2, 2.0), (4, 4.0)])
def test_gaussian_discretized_converges_to_mehler(p, slope):
    """Exact A_N^(p) of the oscillator approaches the Mehler value as 1/N^p (Sec. 2.1)."""
    ex = cf.mehler(0.0, 1.0, 1.0)
    errs = [cf.gaussian_discretized(0.0, 1.0, 1.0, N, p) - ex for N in (32, 64, 128)]
    got = math.log2(abs(errs[-2] / errs[-1]))
    assert abs(got - slope) < 0.05


def test_gaussian_discretized_equals_quadrature():
    """Two independent evaluations of the same discretized integral (closed Gaussian form vs grid quadrature)."""
    for N in (1, 2, 4):
        a = cf.gaussian_discretized(0.3, -0.7, 1.3, N, 3)
        b = cf.transfer_discretized(ea.quartic(1, 0), 3, 0.3, -0.7, 1.3, N, L=7.0, h=0.02)
        assert a == pytest.approx(b, rel=1e-11)


def test_harmonic_mc_matches_exact_discretized():
    """C1 harmonic variant: MC A_16^(4) within 4 sigma of the exact Gaussian value at every level."""
    res = pimc.amplitude(ea.quartic(1, 0), 1, 0.0, 1.0, 1.0, 4, 4, 100000, 1, 0)
    assert res[0]["amp"] == pytest.approx(cf.gaussian_discretized(0.0, 1.0, 1.0, 1, 4), rel=1e-13)
    for n in range(1, 5):
        assert abs(_z(res[n], cf.gaussian_discretized(0.0, 1.0, 1.0, 1 << n, 4))) < 4


def test_quartic_mc_matches_exact_discretized_and_continuum():
    """C1: g=1, p=4: MC within 4 sigma of the quadrature A_N^(4) and of the continuum amplitude."""
    V = ea.quartic(1, 1)
    res = pimc.amplitude(V, 1, 0.0, 1.0, 1.0, 4, 4, 100000, 1, 0)
    for n in range(1, 5):
        ex = cf.transfer_discretized(V, 4, 0.0, 1.0, 1.0, 1 << n)
        assert abs(_z(res[n], ex)) < 4
    cont = cf.dvr_amplitude(cf.quartic_V(1, 1), 0.0, 1.0, 1.0)
    assert abs(_z(res[4], cont)) < 4
    assert res[4]["relvar"] == pytest.approx(0.028, abs=0.01)


def test_level0_is_the_analytic_short_time_amplitude():
    V = ea.quartic(1, 1)
    res = pimc.amplitude(V, 1, 0.0, 1.0, 1.0, 2, 4, 10, 1, 0)
    assert res[0]["err"] == 0.0
    assert res[0]["amp"] == pytest.approx(cf.transfer_discretized(V, 4, 0.0, 1.0, 1.0, 1), rel=1e-15)


def test_linear_potential_mc_is_exact_in_expectation():
    """V = F q: W_p is exact for p >= 3, so every A_N equals the exact kernel (odd-potential support)."""
    Fv, a, b, T = 0.8, -0.3, 0.9, 1.5
    exact = pimc.free_kernel(a, b, T) * math.exp(-Fv * T * (a + b) / 2 + Fv * Fv * T ** 3 / 24)
    res = pimc.amplitude(ea.poly([0, Fv]), 1, a, b, T, 3, 3, 50000, 2, 0)
    assert res[0]["amp"] == pytest.approx(exact, rel=1e-14)
    for n in range(1, 4):
        assert abs(_z(res[n], exact)) < 4


def test_literal_width_reading_gives_the_same_expectation():
    """The paper's quoted width sqrt(T/2^n) with explicit kinetic term and proposal density estimates
    the same A_N^(p) as exact-bridge sampling (the kinetic cancellation and K_0 prefactor)."""
    V = ea.quartic(1, 1)
    s = 3
    ex = cf.transfer_discretized(V, 4, 0.0, 1.0, 1.0, 1 << s)
    amp, err = pimc.amplitude_literal_width(V, 0.0, 1.0, 1.0, s, 4, 200000, 3, 0)
    assert abs(amp - ex) < 4 * err


def test_hierarchy_levels_equal_separate_runs():
    """Level n of an s-run is bitwise the n-run on the same samples (Sec. 4.1 subsets)."""
    V = ea.quartic(1, 10)
    idx = np.arange(100, 300, dtype=np.uint64)
    S6 = pimc.path_actions(V, 1, 0.0, 1.0, 1.0, 6, 8, 1, 0, idx)
    for n in range(0, 7):
        Sn = pimc.path_actions(V, 1, 0.0, 1.0, 1.0, n, 8, 1, 0, idx)
        assert np.array_equal(S6[:, n], Sn[:, n])


def test_mass_rescaling_against_mehler_with_mass():
    """m != 1 reading: A_m(a,b;T) = sqrt(m) A_1(sqrt(m) a, sqrt(m) b; T) with V(y/sqrt(m))."""
    m, k, a, b, T = 2.0, 3.0, 0.2, 0.7, 1.1
    Vt, at, bt, pref = pimc.rescale_mass(ea.quartic(k, 0), m, a, b)
    A_eff = float(Vt[2]) * 2
    got = pref * cf.gaussian_discretized(at, bt, T, 512, 6, A=Fraction(A_eff))
    assert got == pytest.approx(cf.mehler(a, b, T, A=k, m=m), rel=1e-10)
    # free particle with mass: exact at every level
    res = pimc.amplitude(ea.poly([]), m, a, b, T, 2, 3, 10, 1, 0)
    assert res[2]["amp"] == pytest.approx(math.sqrt(m / (2 * math.pi * T)) * math.exp(-m * (b - a) ** 2 / (2 * T)), rel=1e-14)


def test_path_subsets_are_reproducible():
    """Counter-based sampling: any path range gives the same actions as inside a larger run."""
    V = ea.quartic(1, 1)
    big = pimc.path_actions(V, 1, 0.0, 1.0, 1.0, 4, 4, 1, 0, np.arange(0, 1000, dtype=np.uint64))
    part = pimc.path_actions(V, 1, 0.0, 1.0, 1.0, 4, 4, 1, 0, np.arange(500, 700, dtype=np.uint64))
    assert np.array_equal(big[500:700], part)


def test_chunk_sums_merge_to_the_amplitude():
    """Shifted per-chunk sums merged over disjoint ranges reproduce the plain estimate."""
    V = ea.quartic(1, 1)
    shift = pimc.straight_line_actions(V, 1, 0.0, 1.0, 1.0, 4, 4)
    parts = [pimc.chunk_sums(V, 1, 0.0, 1.0, 1.0, 4, 4, 1, 0, st, 2500, shift) for st in (0, 2500, 5000, 7500)]
    tot = np.sum(parts, axis=0)
    res = pimc.amplitude(V, 1, 0.0, 1.0, 1.0, 4, 4, 10000, 1, 0)
    K0 = pimc.free_kernel(0.0, 1.0, 1.0)
    for n in range(1, 5):
        n_, sd, sd2 = tot[n]
        amp = K0 * math.exp(-shift[n]) * (1 + sd / n_)
        var = (sd2 - sd * sd / n_) / (n_ - 1)
        err = K0 * math.exp(-shift[n]) * math.sqrt(var / n_)
        assert amp == pytest.approx(res[n]["amp"], rel=1e-13)
        assert err == pytest.approx(res[n]["err"], rel=1e-9)
