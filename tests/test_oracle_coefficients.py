"""Pins of the exact effective-action coefficients (oracle O1) against what the paper and
mathematics fix, independently of how eq.(1Drec) was transcribed."""
from fractions import Fraction
from math import comb

import numpy as np
import pytest
import sympy as sp

from oracle import closed_forms as cf
from oracle import effective_action as ea

F = Fraction


# ----------------------------------------------------------------------------- helpers
def W_trivariate(V, p):
    """W_p as {(i, j, e): coef} for the term x^i xbar^j eps^e, from eq.(ansatz) truncated at m<=p-1."""
    c = ea.coefficients(V, p)
    out = {}
    for (m, k), poly in c.items():
        for i, a in enumerate(poly):
            if a:
                key = (i, 2 * k, m - k)
                out[key] = out.get(key, 0) + a
    return out


def _mul(A, B):
    out = {}
    for (i1, j1, e1), a in A.items():
        for (i2, j2, e2), b in B.items():
            key = (i1 + i2, j1 + j2, e1 + e2)
            out[key] = out.get(key, 0) + a * b
    return out


def _add(A, B, s=1):
    out = dict(A)
    for k, v in B.items():
        out[k] = out.get(k, 0) + s * v
    return out


def _dx(A):
    return {(i - 1, j, e): v * i for (i, j, e), v in A.items() if i > 0}


def _dxb(A):
    return {(i, j - 1, e): v * j for (i, j, e), v in A.items() if j > 0}


def _times(A, i=0, j=0, e=0, s=1):
    return {(a + i, b + j, c + e): v * s for (a, b, c), v in A.items()}


def pde_residual(V, p):
    """LHS - RHS of eq.(eqW) for W = W_p, as a trivariate polynomial (exact)."""
    W = W_trivariate(V, p)
    R = dict(W)
    R = _add(R, {k: v * k[1] for k, v in W.items()})                 # xbar d/dxbar W
    R = _add(R, {k: v * k[2] for k, v in W.items()})                 # eps d/deps W
    R = _add(R, _times(_dx(_dx(W)), e=1, s=F(-1, 8)))                # -eps/8 W_xx
    R = _add(R, _times(_dxb(_dxb(W)), e=1, s=F(-1, 8)))              # -eps/8 W_xbxb
    Wx = _dx(W)
    Wb = _dxb(W)
    R = _add(R, _times(_mul(Wx, Wx), e=2, s=F(1, 8)))                # +eps^2/8 (W_x)^2
    R = _add(R, _times(_mul(Wb, Wb), e=2, s=F(1, 8)))                # +eps^2/8 (W_xbar)^2
    # RHS: (V(x+xbar) + V(x-xbar))/2, expanded by the binomial theorem
    for d, a in enumerate(V):
        for j in range(0, d + 1):
            if j % 2 == 0:
                key = (d - j, j, 0)
                R[key] = R.get(key, 0) - a * comb(d, j)
    return {k: v for k, v in R.items() if v != 0}


POTENTIALS = {
    "aho_1_1": ea.quartic(1, 1),
    "double_well": ea.quartic(-1, 4),
    "aho_1_48": ea.quartic(1, 48),
    "general_odd": ea.poly([F(1, 3), F(-1, 2), F(1), F(3, 10), F(1, 24)]),
    "sextic": ea.poly([0, 0, F(1, 2), 0, F(-1, 5), 0, F(1, 30)]),
}


# ----------------------------------------------------------------------------- eq.(eqW)
@pytest.mark.parametrize("name", sorted(POTENTIALS))
@pytest.mark.parametrize("p", [1, 2, 3, 5, 8])
def test_pde_satisfied_through_order_p_minus_1(name, p):
    """W_p solves eq.(eqW) for every term eps^e xbar^(2k) of order e+k <= p-1 (Sec. 2.1)."""
    V = POTENTIALS[name]
    res = pde_residual(V, p)
    low = {k: v for k, v in res.items() if k[2] + k[1] // 2 <= p - 1}
    assert not low, f"residual at low order: {sorted(low)[:5]}"
    if p >= 3 and len(V) > 3:
        # the truncation must leave something at order p (otherwise the check is vacuous)
        assert any(k[2] + k[1] // 2 == p for k in res)


def test_pde_check_catches_a_planted_mistake():
    """A single wrong sign in one coefficient must show up in the residual check."""
    V = ea.quartic(1, 1)
    c = ea.coefficients(V, 4)
    bad = dict(c)
    bad[(2, 1)] = ea.pscale(c[(2, 1)], -1)
    W = {}
    for (m, k), poly in bad.items():
        for i, a in enumerate(poly):
            if a:
                W[(i, 2 * k, m - k)] = W.get((i, 2 * k, m - k), 0) + a
    orig = ea._coefficients_cached
    try:
        ea._coefficients_cached = lambda Vt, p: tuple(sorted(bad.items()))
        res = pde_residual(V, 4)
    finally:
        ea._coefficients_cached = orig
    assert any(k[2] + k[1] // 2 <= 3 for k in res)


# ----------------------------------------------------------------------------- harmonic case
@pytest.mark.parametrize("A", [F(1), F(4), F(1, 4)])
def test_harmonic_coefficients_equal_mehler_series(A):
    """For V = A q^2/2 the exact W follows from the Mehler kernel; its eps-series is W_p."""
    p = 9
    eps, x, xb = sp.symbols("eps x xb", positive=True)
    w = sp.sqrt(sp.Rational(A.numerator, A.denominator))
    Wex = (x ** 2 * w * sp.tanh(w * eps / 2) / eps
           + xb ** 2 * (w * sp.coth(w * eps / 2) - 2 / eps) / eps
           + sp.log(sp.sinh(w * eps) / (w * eps)) / (2 * eps))
    ser = sp.expand(sp.series(Wex, eps, 0, p).removeO())
    c = ea.coefficients(ea.quartic(A, 0), p)
    for m in range(p):
        for k in range(m + 1):
            expect = sp.expand(ser.coeff(eps, m - k).coeff(xb, 2 * k))
            poly = c[(m, k)]
            got = sum(sp.Rational(v.numerator, v.denominator) * x ** i for i, v in enumerate(poly))
            assert sp.simplify(expect - got) == 0, (m, k, expect, got)


def test_linear_potential_is_exact():
    """V = F q: exact W = F x - F^2 eps^2 / 24 (linear-potential kernel), so only c_00 and c_20 survive."""
    Fv = F(7, 3)
    c = ea.coefficients(ea.poly([0, Fv]), 10)
    nonzero = {k: v for k, v in c.items() if v}
    assert nonzero == {(0, 0): (F(0), Fv), (2, 0): (-Fv * Fv / 24,)}


def test_diagonal_closed_form():
    """eq.(diagonal) for a sextic, where it is non-trivial up to m = 3."""
    V = POTENTIALS["sextic"]
    c = ea.coefficients(V, 6)
    assert c[(3, 3)] == (F(720) * V[6] / 5040,)
    assert c[(4, 4)] == () and c[(5, 5)] == ()


def test_even_potential_gives_even_coefficients():
    c = ea.coefficients(ea.quartic(1, 10), 12)
    for poly in c.values():
        assert all(v == 0 for v in poly[1::2])


def test_folding_equals_literal_double_sum():
    """sum_k xbar^(2k) Q_k(x) is the double sum of eq.(ansatz) regrouped."""
    V = ea.quartic(1, 10)
    p, eps = 7, 1.0 / 64
    rng = np.random.default_rng(3)
    x = rng.normal(0, 1.5, 200)
    xb = rng.normal(0, 0.1, 200)
    Q = ea.xbar_groups_float(V, p, eps)
    from oracle.pimc import eps_W
    a = eps_W(Q, x, xb)
    b = ea.eps_W_unfolded(V, p, eps, x, xb)
    assert np.allclose(a, b, rtol=1e-13, atol=1e-16)


# ----------------------------------------------------------------------------- 1/N^p convergence
@pytest.mark.parametrize("p", [1, 2, 3])
def test_discretized_amplitude_converges_as_inverse_N_to_the_p(p):
    """A_N^(p) - A ~ 1/N^p for the quartic (Sec. 2.1, Sec. 4), A from grid diagonalization."""
    V = ea.quartic(1, 10)
    exact = cf.dvr_amplitude(cf.quartic_V(1, 10), 0.0, 1.0, 1.0)
    Ns = [4, 8, 16]
    errs = [cf.transfer_discretized(V, p, 0.0, 1.0, 1.0, N, L=6.0, h=0.025) - exact for N in Ns]
    slopes = [np.log2(abs(errs[i] / errs[i + 1])) for i in range(len(Ns) - 1)]
    assert abs(slopes[-1] - p) < 0.35, slopes


def test_high_level_reaches_the_continuum():
    """At p = 10 and N = 8 the discretized amplitude equals the continuum to ~1e-10."""
    V = ea.quartic(1, 10)
    exact = cf.dvr_amplitude(cf.quartic_V(1, 10), 0.0, 1.0, 1.0)
    got = cf.transfer_discretized(V, 10, 0.0, 1.0, 1.0, 8, L=6.0, h=0.025)
    assert abs(got - exact) < 1e-10 * exact
