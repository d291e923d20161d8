"""Pins of the modified Poeschl-Teller oracle (O8): the ansatz, the polynomial recursion on the
Taylor polynomial of V, and the closed-form bound states."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import effective_action as ea
from oracle import mpt


def _tanh_series(order):
    """Exact Taylor coefficients of tanh z up to z^order from T' = 1 - T^2, T(0) = 0."""
    t = [Fraction(0)] * (order + 1)
    for n in range(order):
        # coefficient of z^n in 1 - T^2
        sq = sum(t[i] * t[n - i] for i in range(n + 1))
        rhs = (1 if n == 0 else 0) - sq
        t[n + 1] = Fraction(rhs) / (n + 1)
    return t


def _compose(poly_y, tser, alpha, order):
    """Taylor coefficients (to z^order) of P(tanh(alpha x)) for a polynomial P in y."""
    ty = [c * alpha ** i for i, c in enumerate(tser)]          # tanh(alpha x) series
    out = [Fraction(0)] * (order + 1)
    pw = [Fraction(1)] + [Fraction(0)] * order                   # y^0
    for j, c in enumerate(poly_y):
        if j > 0:
            new = [Fraction(0)] * (order + 1)
            for a_, av in enumerate(pw):
                if av == 0:
                    continue
                for b_, bv in enumerate(ty[:order + 1 - a_]):
                    if bv:
                        new[a_ + b_] += av * bv
            pw = new
        for i in range(order + 1):
            out[i] += c * pw[i]
    return out


def test_coefficients_have_the_ansatz_form():
    """Every c_{m,k} is even in y = tanh(alpha x), of degree <= 2m + 2, and of the form of
    eq.(1D-MPTansatz) (divisible by 1 - y^2 = 1/cosh^2)."""
    p = 7
    c = dict(mpt.coefficients(1, Fraction(3, 2), p))
    for (m, k), poly in c.items():
        assert len(poly) <= 2 * m + 3
        d = mpt.ansatz_d(1, Fraction(3, 2), p, m, k)
        assert len(d) == m + 1


@pytest.mark.parametrize("lam,alpha", [(1, 1), (Fraction(5, 2), Fraction(3, 4))])
def test_taylor_coefficients_match_the_polynomial_recursion(lam, alpha):
    """The recursion in y with d/dx = alpha (1 - y^2) d/dy agrees with the (pinned) polynomial
    recursion applied to the Taylor polynomial of V = -lambda/cosh^2(alpha x) on every Taylor
    coefficient the truncation leaves exact."""
    order, p = 26, 5
    tser = _tanh_series(order + 1)
    lam, alpha = Fraction(lam), Fraction(alpha)
    Vx = _compose((-lam, Fraction(0), lam), tser, alpha, order)    # -lambda (1 - tanh^2)
    cx = ea.coefficients(ea._trim(list(Vx)), p)
    cy = dict(mpt.coefficients(lam, alpha, p))
    for (m, k), py in cy.items():
        ser = _compose(py, tser, alpha, order)
        exact_to = order + 1 - 2 * m - 2                          # truncation of V at x^order
        px = cx[(m, k)]
        for i in range(exact_to):
            assert ser[i] == (px[i] if i < len(px) else 0), (m, k, i)


@pytest.mark.parametrize("lam,alpha", [(1.0, 1.0), (3.0, 1.0), (6.0, 1.5)])
def test_bound_states_from_the_evolution_matrix(lam, alpha):
    """The largest eigenvalues of the short-time matrix give the Poeschl-Teller bound states
    E_n = -(alpha^2/2)(s - n)^2 with s(s + 1) = 2 lambda/alpha^2."""
    ref = mpt.bound_states(lam, alpha)
    M, x, D = mpt.evolution_matrix(lam, alpha, 1.0, 0.05, 8, 16.0, 640)
    lam_ = np.sort(np.linalg.eigvalsh(M))[::-1][:len(ref)]
    E = -np.log(lam_) / 0.05
    assert np.max(np.abs(E - np.array(ref))) < 1e-9, (E, ref)


def test_slice_action_is_the_unfolded_double_sum():
    lam, alpha, p, eps = 2.0, 0.8, 6, 0.125
    tab = mpt.level_tables(lam, Fraction(alpha), p, eps, 0)[0]
    x = np.linspace(-3, 3, 7)
    xb = np.linspace(-0.4, 0.5, 7)
    got = mpt.eps_W(tab, alpha, x, xb)
    c = dict(mpt.coefficients(lam, Fraction(alpha), p))
    y = np.tanh(alpha * x)
    ref = np.zeros_like(x)
    for (m, k), poly in c.items():
        val = sum(float(cf) * y ** j for j, cf in enumerate(poly))
        ref += eps ** (m - k + 1) * val * xb ** (2 * k)
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-15)
