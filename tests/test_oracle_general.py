"""Pins of the general-potential oracle (O9): the derivative-symbol coefficients against the
polynomial and Poeschl-Teller recursions, and their dimensional structure."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import effective_action as ea
from oracle import general as og
from oracle import mpt
from oracle import pimc as opimc


class _EP:
    """Exact polynomial with + and * (for substituting into the symbolic coefficients)."""

    def __init__(self, p):
        self.p = tuple(p)

    def __add__(self, o):
        return _EP(ea.padd(self.p, o.p))

    def __mul__(self, o):
        return _EP(ea.pmul(self.p, o.p)) if isinstance(o, _EP) else _EP(ea.pscale(self.p, o))

    __rmul__ = __mul__


P_LEVEL = 6


def test_monomials_have_weight_2m_plus_2():
    for (m, k), terms in og.coefficients(P_LEVEL):
        assert terms
        for mono, _ in terms:
            assert sum(e * (j + 2) for j, e in enumerate(mono)) == 2 * m + 2, (m, k, mono)


@pytest.mark.parametrize("coefs", [(0, 0, Fraction(1, 2), 0, Fraction(10, 24)), (Fraction(1, 4), -1, 2, Fraction(1, 3), 0,
                                                                              Fraction(-1, 50))])
def test_polynomial_substitution_is_the_polynomial_recursion(coefs):
    V = ea.poly(coefs)
    derivs = [_EP(ea.pder(V, j)) for j in range(2 * P_LEVEL - 1)]
    sub = og.substitute(P_LEVEL, derivs)
    ref = ea.coefficients(V, P_LEVEL)
    for key, val in sub.items():
        assert val.p == ref[key], key


def test_poeschl_teller_substitution_is_the_tanh_recursion():
    lam, alpha = Fraction(3, 2), Fraction(4, 5)
    Vy = ea._trim([-lam, Fraction(0), lam])
    derivs = [_EP(mpt.yder(Vy, alpha, j)) for j in range(2 * P_LEVEL - 1)]
    sub = og.substitute(P_LEVEL, derivs)
    ref = dict(mpt.coefficients(lam, alpha, P_LEVEL))
    for key, val in sub.items():
        assert val.p == ref[key], key


def test_slice_action_matches_the_model_specific_tables():
    x = np.linspace(-2.5, 2.0, 9)
    xb = np.linspace(-0.3, 0.4, 9)
    eps = 0.2
    coefs = (0.0, 0.0, 0.5, 0.0, 10 / 24)
    d = og.derivative_functions(P_LEVEL, poly=coefs)
    got = og.eps_W(P_LEVEL, eps, d, x, xb)
    tab = opimc.level_tables(ea.poly(coefs), P_LEVEL, eps, 0)[0]
    assert np.allclose(got, opimc.eps_W(tab, x, xb), rtol=1e-12, atol=1e-14)
    d = og.derivative_functions(P_LEVEL, sech2=((-1.5, 0.8),))
    got = og.eps_W(P_LEVEL, eps, d, x, xb)
    tab = mpt.level_tables(1.5, Fraction(0.8), P_LEVEL, eps, 0)[0]
    assert np.allclose(got, mpt.eps_W(tab, 0.8, x, xb), rtol=1e-12, atol=1e-14)


# ----------------------------------------------------------------------------- Gaussian terms
def _hermite_coefficients(j):
    """Coefficients of the physicists' Hermite polynomial H_j by H_{n+1} = 2y H_n - 2n H_{n-1}."""
    h0, h1 = [Fraction(1)], [Fraction(0), Fraction(2)]
    if j == 0:
        return h0
    for n in range(1, j):
        h2 = [Fraction(0)] + [2 * c for c in h1]
        for i, c in enumerate(h0):
            h2[i] -= 2 * n * c
        h0, h1 = h1, h2
    return h1


def test_gaussian_term_derivatives_are_hermite_functions():
    """d^j/dx^j B exp(-b x^2) = B (-sqrt b)^j H_j(sqrt b x) exp(-b x^2) (Rodrigues' formula), here
    after the mass rescaling V(x / sqrt m): b -> b/m. B = 2, b = 9/4, m = 4 give sqrt(b/m) = 3/4,
    so H_j is evaluated exactly at rational points; every derivative order of p = 18 (j <= 34)."""
    p = 18
    B, b, m = Fraction(2), Fraction(9, 4), Fraction(4)
    sb = Fraction(3, 4)
    assert sb * sb == b / m
    d = og.derivative_functions(p, gauss=((float(B), float(b)),), m=float(m))
    assert len(d) == 2 * p - 1
    for x in (Fraction(-5, 2), Fraction(-1), Fraction(-1, 4), Fraction(0), Fraction(1, 2), Fraction(7, 4), Fraction(3)):
        g = np.exp(-float(b / m * x * x))
        y = sb * x
        for j in range(2 * p - 1):
            H = _hermite_coefficients(j)
            ref = float(B * (-sb) ** j * sum(c * y ** i for i, c in enumerate(H))) * g
            scale = float(B * sb ** j * sum(abs(c) * abs(y) ** i for i, c in enumerate(H))) * g
            got = float(d[j](float(x)))
            assert abs(got - ref) <= 1e-13 * scale, (x, j, got, ref)


def _barrier_amplitude(p, N):
    """A_N^(p)(0, 1; 1) for V = q^2/2 + 2 exp(-q^2) by quadrature of the product of the level-p
    short-time amplitudes built from ``og.eps_W`` (the discretized amplitude of Sec. 4)."""
    d = og.derivative_functions(p, poly=(0.0, 0.0, 0.5), gauss=((2.0, 1.0),))
    eps = 1.0 / N
    kern = lambda q, qp: cf.short_time_from_epsW(lambda x, xb: og.eps_W(p, eps, d, x, xb), eps, q, qp)
    return cf.transfer_product(kern, 0.0, 1.0, N, L=6.0, h=0.025)


def _barrier_continuum():
    return cf.dvr_amplitude(lambda x: 0.5 * x * x + 2.0 * np.exp(-x * x), 0.0, 1.0, 1.0, L=10.0, h=0.025)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_gaussian_barrier_converges_as_inverse_N_to_the_p(p):
    """The level-p discretized amplitude of a potential with a Gaussian term approaches the sinc-DVR
    continuum as 1/N^p (Sec. 3.1: general V through its derivatives; Sec. 4): a wrong sign, scale or
    index in the Gaussian derivatives breaks the order."""
    exact = _barrier_continuum()
    errs = [_barrier_amplitude(p, N) - exact for N in (16, 32, 64)]
    slope = np.log2(abs(errs[-2] / errs[-1]))
    assert abs(slope - p) < 0.25, (errs, slope)


def test_gaussian_barrier_high_level_reaches_the_continuum():
    """At p = 8 and N = 16 the discretized amplitude equals the continuum to ~1e-12."""
    exact = _barrier_continuum()
    assert abs(_barrier_amplitude(8, 16) - exact) < 1e-11 * exact


def test_error_scale_bounds_the_action():
    """eps_W_abs (the sum of the absolute monomial terms, the error scale of the GPU comparisons) is
    at least |eps_W| everywhere, and equals eps_W where there is a single non-negative term (p = 1:
    eps V(x) for V >= 0)."""
    x = np.linspace(-3.0, 3.0, 41)
    xb = np.linspace(-0.4, 0.5, 41)
    d = og.derivative_functions(P_LEVEL, poly=(0.0, 0.3, 0.5), sech2=((-1.5, 0.8),), gauss=((2.0, 1.0),))
    w = og.eps_W(P_LEVEL, 0.3, d, x, xb)
    wa = og.eps_W_abs(P_LEVEL, 0.3, d, x, xb)
    assert np.all(wa >= np.abs(w) * (1 - 1e-14))
    assert np.any(wa > 1.01 * np.abs(w))                 # terms of both signs somewhere
    d1 = og.derivative_functions(1, poly=(0.0, 0.0, 0.5), gauss=((2.0, 1.0),))
    assert np.allclose(og.eps_W_abs(1, 0.3, d1, x, xb), og.eps_W(1, 0.3, d1, x, xb), rtol=1e-15, atol=0)
