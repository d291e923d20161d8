"""Pins of the general-potential oracle (O9): the derivative-symbol coefficients against the
polynomial and Poeschl-Teller recursions, and their dimensional structure."""
from fractions import Fraction

import numpy as np
import pytest

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
