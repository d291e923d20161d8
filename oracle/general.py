"""O9 -- general-potential mode: the effective potential in the derivative symbols v_j = V^(j)(x).

Test infrastructure only (see ``oracle/__init__``).

Sec. 3.1/3.2: for a general potential the coefficients c_{m,k} of eq.(ansatz) are expressions in V
and its derivatives up to order 2p-2 (the paper's generated function for p = 18 is ~2 MB of C). Here
eq.(1Drec) and eq.(diagonal) are run exactly on polynomials in the symbols v_0, v_1, ..., v_{2p-2}
with the derivation d/dx v_j = v_{j+1} (c_{0,0} = v_0); the result does not depend on V. For a
given potential the slice action is eps W_p = sum_k xbar^(2k) sum_m eps^(m-k+1) c_{m,k}(v(x)) with
the derivative values at the mid-point x.

Potentials of this mode (shared with the device): V(x) = sum_n c_n x^n + sum_i A_i / cosh^2(a_i x)
+ sum_i B_i exp(-b_i x^2); the oracle takes the derivatives symbolically (sympy) and evaluates them
in FP64.

Pins (tests/test_oracle_general.py): substituting the exact derivatives of a polynomial V
reproduces ``effective_action.coefficients`` exactly; substituting those of -lambda/cosh^2(alpha x)
(as polynomials in tanh) reproduces ``mpt.coefficients`` exactly; every monomial of c_{m,k} has
weight sum (j + 2) = 2m + 2 (the dimension of eps^(m-k) xbar^(2k) c_{m,k} is that of V).
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache
from math import factorial
from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import pimc as opimc

Mono = Tuple[int, ...]          # exponents of v_0 .. v_J
SPoly = Dict[Mono, Fraction]


def _norm(a: SPoly) -> SPoly:
    return {k: v for k, v in a.items() if v != 0}


def sadd(a: SPoly, b: SPoly, s=1) -> SPoly:
    out = dict(a)
    for k, v in b.items():
        out[k] = out.get(k, Fraction(0)) + s * v
    return _norm(out)


def sscale(a: SPoly, s) -> SPoly:
    return _norm({k: v * s for k, v in a.items()})


def smul(a: SPoly, b: SPoly) -> SPoly:
    out: SPoly = {}
    for ka, va in a.items():
        for kb, vb in b.items():
            k = tuple(x + y for x, y in zip(ka, kb))
            out[k] = out.get(k, Fraction(0)) + va * vb
    return _norm(out)


def sder(a: SPoly, times: int = 1) -> SPoly:
    """d/dx with d v_j / dx = v_{j+1} (the exponent tuples must have room for j+1)."""
    for _ in range(times):
        out: SPoly = {}
        for k, v in a.items():
            for j, e in enumerate(k):
                if e:
                    nk = list(k)
                    nk[j] -= 1
                    nk[j + 1] += 1
                    t = tuple(nk)
                    out[t] = out.get(t, Fraction(0)) + v * e
        a = _norm(out)
    return a


@lru_cache(maxsize=16)
def coefficients(p: int) -> Tuple[Tuple[Tuple[int, int], Tuple[Tuple[Mono, Fraction], ...]], ...]:
    """c_{m,k}(v_0..v_{2p-2}), 0 <= k <= m <= p-1, exactly (Sec. 2.1: eq.(diagonal), then
    eq.(1Drec) for k = m-1..0; Fig. 1)."""
    J = 2 * p - 2
    nv = J + 2                                       # one spare slot for the last derivative
    unit = [0] * nv
    v0 = list(unit)
    v0[0] = 1
    c: Dict[Tuple[int, int], SPoly] = {(0, 0): {tuple(v0): Fraction(1)}}
    d1: Dict[Tuple[int, int], SPoly] = {}

    def dc(key):
        if key not in d1:
            d1[key] = sder(c[key])
        return d1[key]

    for m in range(1, p):
        vm = list(unit)
        vm[2 * m] = 1
        c[(m, m)] = {tuple(vm): Fraction(1, factorial(2 * m + 1))}
        for k in range(m - 1, -1, -1):
            rhs = sscale(c[(m, k + 1)], (2 * k + 2) * (2 * k + 1))
            rhs = sadd(rhs, sder(c[(m - 1, k)], 2))
            for l in range(0, m - 1):
                for r in range(max(0, k - m + l + 2), min(k, l) + 1):
                    rhs = sadd(rhs, smul(dc((l, r)), dc((m - l - 2, k - r))), -1)
            for l in range(1, m - 1):
                for r in range(max(0, k - m + l + 2), min(k, l) + 1):
                    f = 2 * r * (2 * k - 2 * r + 2)
                    if f:
                        rhs = sadd(rhs, smul(c[(l, r)], c[(m - l - 1, k - r + 1)]), -f)
            c[(m, k)] = sscale(rhs, Fraction(1, 8 * (m + k + 1)))
    # drop the spare slot (never used: the highest derivative appears only on the diagonal)
    out = []
    for key in sorted(c):
        terms = []
        for mono, v in sorted(c[key].items()):
            assert mono[-1] == 0
            terms.append((mono[:-1], v))
        out.append((key, tuple(terms)))
    return tuple(out)


def substitute(p: int, derivs: Sequence) -> Dict[Tuple[int, int], object]:
    """c_{m,k} with v_j replaced by derivs[j] (anything supporting + and *, e.g. exact polynomials
    given as callables' results); derivs[j] for j = 0..2p-2."""
    out = {}
    for key, terms in coefficients(p):
        acc = None
        for mono, coef in terms:
            t = coef
            for j, e in enumerate(mono):
                for _ in range(e):
                    t = t * derivs[j]
            acc = t if acc is None else acc + t
        out[key] = acc
    return out


# ------------------------------------------------------------------------------- potentials
def potential_expr(poly=(), sech2=(), gauss=(), m=1.0):
    """sympy expression of V(x / sqrt(m)) (the mass rescaling) for the potentials of this mode:
    sum c_n x^n + sum A/cosh^2(a x) + sum B exp(-b x^2); the rational values of the FP64 inputs."""
    import sympy as sp
    x = sp.Symbol("x", real=True)
    sm = sp.Rational(Fraction(math.sqrt(m))) if m != 1 else sp.Integer(1)
    y = x / sm
    V = sp.Integer(0)
    for n, cn in enumerate(poly):
        V += sp.Rational(Fraction(cn)) * y ** n
    for A, a in sech2:
        V += sp.Rational(Fraction(A)) / sp.cosh(sp.Rational(Fraction(a)) * y) ** 2
    for B, b in gauss:
        V += sp.Rational(Fraction(B)) * sp.exp(-sp.Rational(Fraction(b)) * y ** 2)
    return x, V


def derivative_functions(p, poly=(), sech2=(), gauss=(), m=1.0):
    """FP64 numpy callables for V^(j), j = 0..2p-2, of the rescaled potential (symbolic diff)."""
    import sympy as sp
    x, V = potential_expr(poly, sech2, gauss, m)
    out = []
    d = V
    for j in range(2 * p - 1):
        out.append(sp.lambdify(x, d, "numpy"))
        d = sp.diff(d, x)
    return out


def eps_W(p, eps, dfun, x, xbar):
    """eps W_p(x, xbar) = sum_{m,k} eps^(m-k+1) xbar^(2k) c_{m,k}(v(x)) (FP64)."""
    x = np.asarray(x, dtype=np.float64)
    xb2 = np.asarray(xbar, dtype=np.float64) ** 2
    v = [np.broadcast_to(np.asarray(f(x), dtype=np.float64), x.shape) for f in dfun]
    total = np.zeros(np.broadcast(x, xb2).shape)
    for (m, k), terms in coefficients(p):
        val = np.zeros_like(total)
        for mono, coef in terms:
            t = np.full_like(total, float(coef))
            for j, e in enumerate(mono):
                if e:
                    t = t * v[j] ** e
            val = val + t
        total = total + float(Fraction(eps) ** (m - k + 1)) * xb2 ** k * val
    return total


def eps_W_abs(p, eps, dfun, x, xbar):
    """sum_{m,k} eps^(m-k+1) xbar^(2k) sum |monomial terms of c_{m,k}(v(x))|: the scale of the FP64
    rounding error of eps_W (the same sum without cancellation between terms)."""
    x = np.asarray(x, dtype=np.float64)
    xb2 = np.asarray(xbar, dtype=np.float64) ** 2
    v = [np.broadcast_to(np.asarray(f(x), dtype=np.float64), x.shape) for f in dfun]
    total = np.zeros(np.broadcast(x, xb2).shape)
    for (m, k), terms in coefficients(p):
        val = np.zeros_like(total)
        for mono, coef in terms:
            t = np.full_like(total, abs(float(coef)))
            for j, e in enumerate(mono):
                if e:
                    t = t * np.abs(v[j]) ** e
            val = val + t
        total = total + float(Fraction(eps) ** (m - k + 1)) * xb2 ** k * val
    return total


def path_action_scales(p, T, s, a, b, seed, stream, paths, poly=(), sech2=(), gauss=(), m=1.0, levels=None):
    """Per path and level the sum over slices of eps_W_abs (the error scale of path_actions)."""
    dfun = derivative_functions(p, poly, sech2, gauss, m)
    sm = math.sqrt(m)
    q = opimc.bisection_paths(a * sm, b * sm, T, s, seed, stream, paths)
    out = np.zeros((q.shape[0], s + 1))
    for n in (range(s + 1) if levels is None else levels):
        step = 1 << (s - n)
        qa = q[:, 0:-1:step]
        qb = q[:, step::step]
        out[:, n] = eps_W_abs(p, T / (1 << n), dfun, 0.5 * (qa + qb), 0.5 * (qb - qa)).sum(axis=1)
    return out


def path_actions(p, T, s, a, b, seed, stream, paths, poly=(), sech2=(), gauss=(), m=1.0, levels=None):
    """Per-path level actions (rows: paths, columns: n = 0..s) after the mass rescaling; only the
    columns in `levels` (default: every level) are computed, the others are left 0."""
    dfun = derivative_functions(p, poly, sech2, gauss, m)
    sm = math.sqrt(m)
    q = opimc.bisection_paths(a * sm, b * sm, T, s, seed, stream, paths)
    out = np.zeros((q.shape[0], s + 1))
    for n in (range(s + 1) if levels is None else levels):
        step = 1 << (s - n)
        qa = q[:, 0:-1:step]
        qb = q[:, step::step]
        out[:, n] = eps_W(p, T / (1 << n), dfun, 0.5 * (qa + qb), 0.5 * (qb - qa)).sum(axis=1)
    return out
