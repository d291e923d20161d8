"""O8 -- the modified Poeschl-Teller potential V = -lambda / cosh^2(alpha x) (Sec. 3.3, eq.(1D-MPT)).

Test infrastructure only (see ``oracle/__init__``).

The paper's model-specific route for this potential writes the coefficients of the effective
potential in the form of eq.(1D-MPTansatz): c_{m,k}(x) = sum_l d_{m,k,l} tanh^{2l}(alpha x) /
cosh^{2m-2l+2}(alpha x). With y = tanh(alpha x) every such term is a polynomial in y (1/cosh^2 =
1 - y^2), V itself is -lambda (1 - y^2), and d/dx = alpha (1 - y^2) d/dy maps polynomials in y to
polynomials in y. So eq.(1Drec) and eq.(diagonal) can be run exactly in the ring of polynomials in y
with that derivative: the result is c_{m,k} as an exact polynomial in y (even, degree <= 2m + 2,
divisible by 1 - y^2 -- the ansatz), from which the d_{m,k,l} follow.

The slice action is eps W_p = sum_k xbar^(2k) Q_k(y), Q_k = sum_{m=k}^{p-1} eps^(m-k+1) c_{m,k},
y = tanh(alpha x) at the mid-point x; everything else (bisection paths, estimator) is the plain
path of ``oracle.pimc``.

Mass: V(x/sqrt(m)) is the same family with alpha -> alpha/sqrt(m) (the rescaling of the main
estimator).

Pins (tests/test_oracle_mpt.py): the ansatz structure; the low Taylor coefficients of c_{m,k}
against the polynomial recursion of ``effective_action`` applied to the Taylor polynomial of V;
the bound states E_n = -(alpha^2/2)(s - n)^2, s(s+1) = 2 lambda/alpha^2, from the evolution-operator
matrix built with these amplitudes.
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache
from math import factorial
from typing import Dict, List, Tuple

import numpy as np

from . import effective_action as ea
from . import pimc as opimc
from .philox import node_normals

Poly = ea.Poly


def yder(a: Poly, alpha: Fraction, times: int = 1) -> Poly:
    """d/dx of a polynomial in y = tanh(alpha x): alpha (1 - y^2) d/dy."""
    one_minus_y2 = (Fraction(1), Fraction(0), Fraction(-1))
    for _ in range(times):
        a = ea.pscale(ea.pmul(one_minus_y2, ea.pder(a)), alpha)
    return a


@lru_cache(maxsize=32)
def coefficients(lam, alpha, p: int) -> Tuple[Tuple[Tuple[int, int], Poly], ...]:
    """c_{m,k}(y), 0 <= k <= m <= p-1, exact: eq.(diagonal) then eq.(1Drec) for k = m-1..0
    (Sec. 2.1, Fig. 1), derivatives by ``yder``."""
    lam = Fraction(lam)
    alpha = Fraction(alpha)
    V = ea._trim([-lam, Fraction(0), lam])                       # -lambda (1 - y^2)
    c: Dict[Tuple[int, int], Poly] = {(0, 0): V}
    d1: Dict[Tuple[int, int], Poly] = {}

    def dc(key):
        if key not in d1:
            d1[key] = yder(c[key], alpha)
        return d1[key]

    for m in range(1, p):
        c[(m, m)] = ea.pscale(yder(V, alpha, 2 * m), Fraction(1, factorial(2 * m + 1)))
        for k in range(m - 1, -1, -1):
            rhs = ea.pscale(c[(m, k + 1)], (2 * k + 2) * (2 * k + 1))
            rhs = ea.padd(rhs, yder(c[(m - 1, k)], alpha, 2))
            for l in range(0, m - 1):
                for r in range(max(0, k - m + l + 2), min(k, l) + 1):
                    rhs = ea.padd(rhs, ea.pscale(ea.pmul(dc((l, r)), dc((m - l - 2, k - r))), -1))
            for l in range(1, m - 1):
                for r in range(max(0, k - m + l + 2), min(k, l) + 1):
                    f = 2 * r * (2 * k - 2 * r + 2)
                    if f:
                        rhs = ea.padd(rhs, ea.pscale(ea.pmul(c[(l, r)], c[(m - l - 1, k - r + 1)]), -f))
            c[(m, k)] = ea.pscale(rhs, Fraction(1, 8 * (m + k + 1)))
    return tuple(sorted(c.items()))


def ansatz_d(lam, alpha, p: int, m: int, k: int) -> List[Fraction]:
    """d_{m,k,l}, l = 0..m, of eq.(1D-MPTansatz): c_{m,k} = sum_l d_l y^(2l) (1 - y^2)^(m-l+1),
    found by peeling powers of (1 - y^2); raises if c_{m,k} is not of that form."""
    c = dict(coefficients(lam, alpha, p))[(m, k)]
    # in u = y^2: c(u) = sum_l d_l u^l (1-u)^(m-l+1)
    cu = [c[i] for i in range(0, len(c), 2)] if c else []
    if any(c[i] != 0 for i in range(1, len(c), 2)):
        raise ValueError("c_{m,k} is not even in y")
    # solve the triangular system in the basis u^l (1-u)^(m-l+1) (lowest power of basis l is l)
    n = m + 2
    basis = []
    for l in range(m + 1):
        b = [Fraction(0)] * n
        pol = [Fraction(1)]
        for _ in range(m - l + 1):
            pol = [a - (pol[i - 1] if i else 0) for i, a in enumerate(pol + [Fraction(0)])]
        for i, v in enumerate(pol):
            b[i + l] += v
        basis.append(b)
    target = cu + [Fraction(0)] * (n - len(cu))
    d = [Fraction(0)] * (m + 1)
    rest = list(target)
    for l in range(m + 1):
        d[l] = rest[l] / basis[l][l]
        rest = [r - d[l] * bv for r, bv in zip(rest, basis[l])]
    if any(r != 0 for r in rest):
        raise ValueError("c_{m,k} is not of the ansatz form")
    return d


def xbar_groups(lam, alpha, p: int, eps) -> List[Poly]:
    """Exact Q_k(y) with eps W_p = sum_k xbar^(2k) Q_k(y), y = tanh(alpha x)."""
    eps = Fraction(eps)
    c = dict(coefficients(lam, alpha, p))
    out = []
    for k in range(p):
        acc: Poly = ()
        for m in range(k, p):
            acc = ea.padd(acc, ea.pscale(c[(m, k)], eps ** (m - k + 1)))
        out.append(acc)
    while out and not out[-1]:
        out.pop()
    return out


def _alpha_m(alpha, m) -> Fraction:
    """alpha / sqrt(m) as the exact value of its FP64 rounding (the mass reading)."""
    if m == 1:
        return Fraction(alpha)
    return Fraction(float(alpha) / math.sqrt(float(m)))


def level_tables(lam, alpha, p: int, T: float, s: int) -> List[List[List[float]]]:
    Tf = Fraction(T)
    return [[[float(c) for c in q] for q in xbar_groups(lam, alpha, p, Tf / (1 << n))] for n in range(s + 1)]


def eps_W(tab, alpha: float, x, xbar):
    """eps W_p(x, xbar) = sum_k xbar^(2k) Q_k(tanh(alpha x)) (FP64)."""
    y = np.tanh(alpha * np.asarray(x, dtype=np.float64))
    xb2 = np.asarray(xbar, dtype=np.float64) ** 2
    total = np.zeros(np.broadcast(y, xb2).shape)
    pw = np.ones_like(total)
    for Q in tab:
        val = np.zeros_like(total)
        for coef in reversed(Q):
            val = val * y + coef
        total = total + pw * val
        pw = pw * xb2
    return total


def level_actions(q, s, tables, alpha):
    """Level-n action sum_k eps_n W_p of the level-s paths q (rows) for n = 0..s."""
    out = np.zeros((q.shape[0], s + 1))
    for n in range(s + 1):
        step = 1 << (s - n)
        qa = q[:, 0:-1:step]
        qb = q[:, step::step]
        out[:, n] = eps_W(tables[n], alpha, 0.5 * (qa + qb), 0.5 * (qb - qa)).sum(axis=1)
    return out


def path_actions(lam, alpha, m, a, b, T, s, p, seed, stream, paths):
    """Per-path level actions (rows: paths, columns: n = 0..s) after the mass rescaling."""
    am = float(_alpha_m(alpha, m))
    sm = math.sqrt(m)
    q = opimc.bisection_paths(a * sm, b * sm, T, s, seed, stream, paths)
    return level_actions(q, s, level_tables(lam, _alpha_m(alpha, m), p, T, s), am)


def straight_line_actions(lam, alpha, m, a, b, T, s, p):
    am = float(_alpha_m(alpha, m))
    sm = math.sqrt(m)
    tabs = level_tables(lam, _alpha_m(alpha, m), p, T, s)
    out = np.zeros(s + 1)
    for n in range(s + 1):
        k = np.arange((1 << n) + 1, dtype=np.float64)
        q = a * sm + (b * sm - a * sm) * k / (1 << n)
        out[n] = eps_W(tabs[n], am, 0.5 * (q[1:] + q[:-1]), 0.5 * (q[1:] - q[:-1])).sum()
    return out


def amplitude(lam, alpha, m, a, b, T, s, p, n_samples, seed, stream):
    """A_{2^n}^(p) and its error per level n = 0..s from paths 0..n_samples-1 (math.fsum), as the
    plain estimator: sqrt(m) K_0 e^{-S_ref} (1 + mean(expm1(-(S - S_ref))))."""
    S = path_actions(lam, alpha, m, a, b, T, s, p, seed, stream, np.arange(n_samples))
    ref = straight_line_actions(lam, alpha, m, a, b, T, s, p)
    sm = math.sqrt(m)
    K0 = opimc.free_kernel(a * sm, b * sm, T)
    out = []
    for n in range(s + 1):
        d = np.expm1(-(S[:, n] - ref[n]))
        mean = math.fsum(d) / n_samples
        var = (math.fsum(d * d) - n_samples * mean * mean) / (n_samples - 1)
        base = sm * K0 * math.exp(-ref[n])
        out.append(dict(amp=base * (1 + mean), err=base * math.sqrt(max(var, 0.0) / n_samples)))
    return out


def bound_states(lam, alpha):
    """E_n = -(alpha^2/2)(s - n)^2 for n < s, s(s+1) = 2 lambda / alpha^2 (hbar = m = 1)."""
    s = 0.5 * (-1.0 + math.sqrt(1.0 + 8.0 * lam / alpha ** 2))
    return [-(alpha ** 2) / 2.0 * (s - n) ** 2 for n in range(int(math.ceil(s)))]


def evolution_matrix(lam, alpha, m, t, p, L, n):
    """M_ij = D A_1^(p)(x_i, x_j; t) on the grid of ``oracle.spectrum``, MPT short-time amplitude,
    zero where the free-particle factor is below exp(-40) (see ``oracle.spectrum``)."""
    from .spectrum import GAUSS_CUT, grid
    x, D = grid(L, n)
    am = _alpha_m(alpha, m)
    tab = level_tables(lam, am, p, t, 0)[0]
    y = x * math.sqrt(m)
    a_ = y[:, None]
    b_ = y[None, :]
    S = eps_W(tab, float(am), 0.5 * (a_ + b_), 0.5 * (b_ - a_))
    g = (b_ - a_) ** 2 / (2.0 * t)
    with np.errstate(over="ignore"):
        M = D * math.sqrt(m) / math.sqrt(2.0 * math.pi * t) * np.exp(-g - S)
    M[g > GAUSS_CUT] = 0.0
    return M, x, D
