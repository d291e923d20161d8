"""O1 -- exact coefficients of the level-p effective potential for a polynomial potential V.

Test infrastructure only (see ``oracle/__init__``).

Source: Sec. 2.1 of the paper.
* The short-time amplitude is written with the mid-point x=(q+q')/2 and the half-deviation
  xbar=(q'-q)/2 as  A(q,q';eps) = (2 pi eps)^(-1/2) exp(-2 xbar^2/eps - eps W(x,xbar;eps))  (eq. above
  eq.(eqW)).
* W is expanded as  W = sum_{m>=0} sum_{k=0..m} c_{m,k}(x) eps^(m-k) xbar^(2k)   (eq.(ansatz)), and the
  level-p potential W_p keeps m = 0..p-1.
* The coefficients obey eq.(1Drec) with the r-range max{0, k-m+l+2}..min{k,l}, start from
  c_{0,0}=V, have the diagonal closed form eq.(diagonal) c_{m,m} = V^(2m)/(2m+1)!, and are computed
  for each m first on the diagonal and then for k = m-1, ..., 0 (Fig. 1).

Here V is a polynomial with rational coefficients, so every c_{m,k}(x) is a polynomial in x with
rational coefficients, computed exactly with ``fractions.Fraction`` (the "model-specific" mode of
Sec. 3.3, where derivatives of V are taken explicitly).

Pins (tests/test_oracle_coefficients.py): the PDE eq.(eqW) is satisfied exactly through order p-1
by W_p (an independent trivariate-polynomial check of the PDE, not of the recursion); the harmonic
case reproduces the Taylor series of the exact Mehler effective potential; the linear case
reproduces the exact W = F x - F^2 eps^2/24; the short-time amplitude built from W_p converges to a
grid-diagonalization amplitude with error O(eps^(p+1)).
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
from math import factorial
from typing import Dict, List, Sequence, Tuple

Poly = Tuple[Fraction, ...]          # coefficients in x, index = power; trailing zeros trimmed


# --------------------------------------------------------------------------- polynomial helpers
def _trim(c: List[Fraction]) -> Poly:
    while c and c[-1] == 0:
        c.pop()
    return tuple(c)


def poly(coefs: Sequence) -> Poly:
    """Exact polynomial from coefficients; strings/ints/Fractions convert exactly, floats exactly."""
    out = []
    for c in coefs:
        if isinstance(c, Fraction):
            out.append(c)
        elif isinstance(c, str):
            out.append(Fraction(c))
        else:
            out.append(Fraction(c))          # Fraction(float) is the exact binary value
    return _trim(out)


def padd(a: Poly, b: Poly) -> Poly:
    n = max(len(a), len(b))
    return _trim([(a[i] if i < len(a) else 0) + (b[i] if i < len(b) else 0) for i in range(n)])


def pscale(a: Poly, s) -> Poly:
    s = Fraction(s)
    return _trim([c * s for c in a])


def pmul(a: Poly, b: Poly) -> Poly:
    if not a or not b:
        return ()
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, ai in enumerate(a):
        if ai == 0:
            continue
        for j, bj in enumerate(b):
            out[i + j] += ai * bj
    return _trim(out)


def pder(a: Poly, times: int = 1) -> Poly:
    for _ in range(times):
        a = _trim([a[i] * i for i in range(1, len(a))])
    return a


def peval(a: Poly, x):
    """Exact (Fraction x) or float evaluation, highest power first."""
    acc = 0
    for c in reversed(a):
        acc = acc * x + c
    return acc


# --------------------------------------------------------------------------- eq.(1Drec) / eq.(diagonal)
def coefficients(V: Poly, p: int) -> Dict[Tuple[int, int], Poly]:
    """All c_{m,k}(x) for 0 <= k <= m <= p-1, exactly.

    Diagonal first by eq.(diagonal), then k = m-1 .. 0 by eq.(1Drec) (Sec. 2.1, Fig. 1).
    """
    return dict(_coefficients_cached(tuple(V), int(p)))


@lru_cache(maxsize=64)
def _coefficients_cached(V: Poly, p: int):
    if p < 1:
        raise ValueError("level p must be >= 1")
    c: Dict[Tuple[int, int], Poly] = {(0, 0): V}
    d1: Dict[Tuple[int, int], Poly] = {}          # first derivatives, cached

    def dc(key):
        if key not in d1:
            d1[key] = pder(c[key])
        return d1[key]

    for m in range(1, p):
        # eq.(diagonal): c_{m,m} = V^(2m) / (2m+1)!
        c[(m, m)] = pscale(pder(V, 2 * m), Fraction(1, factorial(2 * m + 1)))
        for k in range(m - 1, -1, -1):
            # eq.(1Drec), right-hand side
            rhs = pscale(c[(m, k + 1)], (2 * k + 2) * (2 * k + 1))
            rhs = padd(rhs, pder(c[(m - 1, k)], 2))
            for l in range(0, m - 1):                       # l = 0 .. m-2
                for r in range(max(0, k - m + l + 2), min(k, l) + 1):
                    rhs = padd(rhs, pscale(pmul(dc((l, r)), dc((m - l - 2, k - r))), -1))
            for l in range(1, m - 1):                       # l = 1 .. m-2
                for r in range(max(0, k - m + l + 2), min(k, l) + 1):
                    f = 2 * r * (2 * k - 2 * r + 2)
                    if f:
                        rhs = padd(rhs, pscale(pmul(c[(l, r)], c[(m - l - 1, k - r + 1)]), -f))
            c[(m, k)] = pscale(rhs, Fraction(1, 8 * (m + k + 1)))
    return tuple(sorted(c.items()))


# --------------------------------------------------------------------------- the slice action
def xbar_groups(V: Poly, p: int, eps) -> List[Poly]:
    """Exact Q_k(x) with  eps * W_p(x, xbar; eps) = sum_k xbar^(2k) Q_k(x).

    Q_k(x) = sum_{m=k}^{p-1} eps^(m-k+1) c_{m,k}(x): the level-p sum of eq.(ansatz) multiplied by eps
    and collected by powers of xbar (the combination entering eq.(SNp)). ``eps`` is converted
    exactly (Fraction(float) for floats).
    """
    eps = Fraction(eps)
    c = coefficients(V, p)
    out = []
    for k in range(p):
        acc: Poly = ()
        for m in range(k, p):
            acc = padd(acc, pscale(c[(m, k)], eps ** (m - k + 1)))
        out.append(acc)
    while out and not out[-1]:
        out.pop()
    return out


def xbar_groups_float(V: Poly, p: int, eps) -> List[List[float]]:
    """``xbar_groups`` with every coefficient rounded once to FP64."""
    return [[float(c) for c in q] for q in xbar_groups(V, p, eps)]


def eps_W_unfolded(V: Poly, p: int, eps: float, x, xbar):
    """eps*W_p evaluated literally as the double sum of eq.(ansatz) truncated at m <= p-1.

    FP64 numpy evaluation, c_{m,k} rounded to FP64. Slow; used to check ``xbar_groups``.
    """
    import numpy as np
    c = coefficients(V, p)
    x = np.asarray(x, dtype=np.float64)
    xbar = np.asarray(xbar, dtype=np.float64)
    total = np.zeros(np.broadcast(x, xbar).shape)
    for m in range(p):
        for k in range(m + 1):
            ck = [float(v) for v in c[(m, k)]]
            val = np.zeros_like(x)
            for coef in reversed(ck):
                val = val * x + coef
            total = total + val * eps ** (m - k) * xbar ** (2 * k)
    return eps * total


def quartic(A, g) -> Poly:
    """V = A q^2/2 + g q^4/24 (the 1D anharmonic oscillator of Sec. 3.3), exact."""
    return poly([0, 0, Fraction(A) / 2, 0, Fraction(g) / 24])
