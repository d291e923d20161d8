"""Exact references for the amplitude estimator.

Test infrastructure only (see ``oracle/__init__``).

* ``mehler``        -- imaginary-time harmonic-oscillator kernel (the exactly solvable case that
                       defines the ideal effective action of Sec. 2.1), for V = A q^2/2, mass m.
* ``mehler_W``      -- the exact effective potential W(x, xbar; T) of that kernel, from
                       A = (2 pi T)^(-1/2) exp(-S*), S* = T[(b-a)^2/(2T^2) + W] (Sec. 2.1).
* ``gaussian_discretized`` -- the discretized amplitude A_N^(p) of Sec. 4 for a quadratic potential:
                       eps W_p is quadratic in (x, xbar), so the N-1 dimensional integral is Gaussian;
                       evaluated with a tridiagonal determinant and solve in mpmath (30 digits).
* ``transfer_discretized`` -- A_N^(p) for any potential by repeated quadrature of the product of
                       short-time amplitudes (eq.(AMC) with the level-p short-time amplitude), on a
                       uniform grid (trapezoid rule, exponentially accurate for these integrands).
* ``transfer_product`` / ``short_time_from_epsW`` -- the same quadrature for a short-time kernel
                       given as a callable (any effective potential, e.g. the general mode's).
* ``dvr_amplitude`` -- continuum A(a,b;T) = <b|exp(-T H)|a> from a sinc-DVR diagonalization
                       (Colbert and Miller, J. Chem. Phys. 96, 1982 (1992)) of H = p^2/2 + V.
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import Callable, Sequence

import numpy as np

from . import effective_action as ea


def mehler(a: float, b: float, T: float, A: float = 1.0, m: float = 1.0) -> float:
    """<b| exp(-T H) |a> for H = p^2/(2m) + A q^2/2, A > 0 (omega = sqrt(A/m))."""
    w = math.sqrt(A / m)
    sh = math.sinh(w * T)
    ch = math.cosh(w * T)
    return math.sqrt(m * w / (2 * math.pi * sh)) * math.exp(-m * w * ((a * a + b * b) * ch - 2 * a * b) / (2 * sh))


def mehler_W(x: float, xbar: float, T: float) -> float:
    """Exact W(x, xbar; T) of the unit oscillator V = q^2/2 (m = 1)."""
    return (x * x * math.tanh(T / 2) / T + xbar * xbar * (1 / math.tanh(T / 2) - 2 / T) / T
            + math.log(math.sinh(T) / T) / (2 * T))


def _quadratic_parts(p: int, T, N: int, A):
    """(gamma, alpha, beta) with eps W_p = gamma + alpha x^2 + beta xbar^2 for V = A q^2/2, exact."""
    eps = Fraction(T) / N
    Q = ea.xbar_groups(ea.poly([0, 0, Fraction(A) / 2]), p, eps)
    Q = list(Q) + [()] * (2 - len(Q))
    q0 = list(Q[0]) + [Fraction(0)] * 3
    q1 = list(Q[1]) + [Fraction(0)] * 3
    if any(len(q) > 0 for q in Q[2:]) or q0[1] or q1[1] or any(q1[2:]) or any(q0[3:]):
        raise ValueError("not a quadratic effective action")
    return q0[0], q0[2], q1[0]


def gaussian_discretized(a: float, b: float, T: float, N: int, p: int, A=1, dps: int = 30) -> float:
    """Exact A_N^(p)(a,b;T) of Sec. 4 for V = A q^2/2 (mass 1), to ``dps`` digits.

    Per slice: (dq)^2/(2 eps) + eps W_p = u (q_k^2 + q_{k+1}^2) + v q_k q_{k+1} + gamma with
    u = 1/(2 eps) + (alpha + beta)/4 and v = -1/eps + (alpha - beta)/2. The interior integral
    int exp(-q^T M q/2 + J^T q) = (2 pi)^((N-1)/2) det(M)^(-1/2) exp(J^T M^-1 J / 2) with the
    tridiagonal M (4u on the diagonal, v off it) and J = -v (a e_1 + b e_{N-1}).
    """
    import mpmath as mp
    with mp.workdps(dps):
        gamma, alpha, beta = (mp.mpf(c.numerator) / c.denominator for c in _quadratic_parts(p, T, N, A))
        eps = mp.mpf(Fraction(T).numerator) / Fraction(T).denominator / N
        a_ = mp.mpf(a)
        b_ = mp.mpf(b)
        u = 1 / (2 * eps) + (alpha + beta) / 4
        v = -1 / eps + (alpha - beta) / 2
        c0 = u * (a_ ** 2 + b_ ** 2) + N * gamma
        pref = (2 * mp.pi * eps) ** (-mp.mpf(N) / 2)
        if N == 1:
            return float(pref * mp.exp(-(c0 + v * a_ * b_)))
        n = N - 1
        J = [mp.mpf(0)] * n
        J[0] += -v * a_
        J[-1] += -v * b_
        # Thomas algorithm: LDL^T of the symmetric tridiagonal M.
        d = [mp.mpf(0)] * n
        y = [mp.mpf(0)] * n
        d[0] = 4 * u
        y[0] = J[0]
        for i in range(1, n):
            l = v / d[i - 1]
            d[i] = 4 * u - l * v
            y[i] = J[i] - l * y[i - 1]
        xs = [mp.mpf(0)] * n
        xs[-1] = y[-1] / d[-1]
        for i in range(n - 2, -1, -1):
            xs[i] = (y[i] - v * xs[i + 1]) / d[i]
        logdet = mp.fsum(mp.log(di) for di in d)
        quad = mp.fsum(J[i] * xs[i] for i in range(n))
        val = pref * (2 * mp.pi) ** (mp.mpf(n) / 2) * mp.exp(-logdet / 2 + quad / 2 - c0)
        return float(val)


def short_time_amplitude(tab_eps: Sequence[Sequence[float]], eps: float, q, qp):
    """Level-p short-time amplitude (2 pi eps)^(-1/2) exp(-(q'-q)^2/(2 eps) - eps W_p) (Sec. 2.1).

    ``tab_eps`` holds the FP64 Q_k(x) with eps W_p = sum_k xbar^(2k) Q_k(x).
    """
    q = np.asarray(q, dtype=np.float64)
    qp = np.asarray(qp, dtype=np.float64)
    x = 0.5 * (q + qp)
    xb = 0.5 * (qp - q)
    ew = np.zeros(np.broadcast(x, xb).shape)
    pw = np.ones_like(ew)
    for Q in tab_eps:
        val = np.zeros_like(ew)
        for c in reversed(Q):
            val = val * x + c
        ew = ew + pw * val
        pw = pw * xb * xb
    return np.exp(-(qp - q) ** 2 / (2 * eps) - ew) / math.sqrt(2 * math.pi * eps)


def transfer_discretized(V: ea.Poly, p: int, a: float, b: float, T: float, N: int,
                         L: float = 8.0, h: float = 0.02) -> float:
    """A_N^(p)(a,b;T) by quadrature of eq.(AMC) with level-p short-time amplitudes (mass 1).

    Interior coordinates on the grid -L..L with spacing h (trapezoid rule). The integrand is an
    entire function with Gaussian decay, so the rule converges exponentially in 1/h; L only has to
    cover the support. For levels whose leading x-coefficient is negative the formal integral over
    the whole line diverges (radius of convergence, Sec. 4); the value on [-L, L] is the
    pre-asymptotic amplitude that sampling sees.
    """
    eps = T / N
    tab = ea.xbar_groups_float(V, p, Fraction(eps))
    return transfer_product(lambda q, qp: short_time_amplitude(tab, eps, q, qp), a, b, N, L, h)


def transfer_product(kernel: Callable, a: float, b: float, N: int, L: float = 8.0, h: float = 0.02) -> float:
    """int dq_1..dq_{N-1} prod_k kernel(q_k, q_{k+1}), q_0 = a, q_N = b, by the trapezoid rule on the
    grid -L..L with spacing h (the discretized amplitude of Sec. 4 for any short-time kernel)."""
    if N == 1:
        return float(kernel(a, b))
    x = np.arange(-L, L + 0.5 * h, h)
    left = kernel(a, x) * h                                     # row vector over q_1
    right = kernel(x, b)                                        # column over q_{N-1}
    if N == 2:
        return float(left @ right)
    K = kernel(x[:, None], x[None, :]) * h
    vec = left
    for _ in range(N - 2):
        vec = vec @ K
    return float(vec @ right)


def short_time_from_epsW(epsW: Callable, eps: float, q, qp, cutoff: float = 40.0):
    """(2 pi eps)^(-1/2) exp(-(q'-q)^2/(2 eps) - epsW(x, xbar)) with x the mid-point and xbar the
    half-deviation (Sec. 2.1), for an effective potential given as a callable.

    The short-time expansion has a finite radius in xbar (Sec. 4): where the free factor
    exp(-(q'-q)^2/(2 eps)) is below exp(-cutoff) the kernel is set to 0 (there the truncated
    exponent may grow without bound while the true amplitude is negligible).
    """
    q = np.asarray(q, dtype=np.float64)
    qp = np.asarray(qp, dtype=np.float64)
    free = (qp - q) ** 2 / (2 * eps)
    with np.errstate(over="ignore", invalid="ignore"):
        ew = epsW(0.5 * (q + qp), 0.5 * (qp - q))
        val = np.exp(-free - ew) / math.sqrt(2 * math.pi * eps)
    return np.where(free > cutoff, 0.0, val)


def dvr_eigen(V: Callable[[np.ndarray], np.ndarray], L: float = 10.0, h: float = 0.025):
    """Grid x_i = i h on [-L, L], eigenpairs of the sinc-DVR Hamiltonian p^2/2 + V (mass 1)."""
    M = int(round(L / h))
    x = h * np.arange(-M, M + 1)
    i = np.arange(x.size)
    diff = i[:, None] - i[None, :]
    with np.errstate(divide="ignore"):
        Tm = np.where(diff == 0, math.pi ** 2 / 3.0, 2.0 * (-1.0) ** np.abs(diff) / np.where(diff == 0, 1, diff) ** 2)
    Tm = Tm / (2 * h * h)
    H = Tm + np.diag(V(x))
    E, vecs = np.linalg.eigh(H)
    return x, E, vecs


def dvr_amplitude(V: Callable[[np.ndarray], np.ndarray], a: float, b: float, T: float,
                  L: float = 10.0, h: float = 0.025) -> float:
    """<b| exp(-T H) |a> = sum_n psi_n(a) psi_n(b) exp(-T E_n), with a and b on the DVR grid."""
    x, E, vecs = dvr_eigen(V, L, h)
    ia = int(np.argmin(np.abs(x - a)))
    ib = int(np.argmin(np.abs(x - b)))
    if abs(x[ia] - a) > 1e-9 or abs(x[ib] - b) > 1e-9:
        raise ValueError("endpoints must lie on the DVR grid")
    w = np.exp(-T * (E - E[0]))
    return float(math.exp(-T * E[0]) * np.sum(vecs[ia] * vecs[ib] * w) / h)


def quartic_V(A: float, g: float) -> Callable[[np.ndarray], np.ndarray]:
    return lambda x: 0.5 * A * x * x + g * x ** 4 / 24.0
