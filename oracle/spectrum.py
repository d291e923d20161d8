"""O7 -- energy spectrum from the space-discretized evolution operator, FP64.

Test infrastructure only (see ``oracle/__init__``).

The paper's application of short-time amplitudes (Sec. 4.2, Fig. 3; Sec. 2): on a grid x_i the
matrix of transition amplitudes A(x_i, x_j; t) times the spacing is the discretized evolution
operator exp(-t H); its eigenvalues are exp(-t E_n) and its eigenvectors sample the eigenfunctions.
For a short time t the level-p amplitude is used directly (N = 1, no Monte Carlo):

    A_1^(p)(a, b; t) = (2 pi t)^(-1/2) exp(-(b - a)^2 / (2t) - t W_p((a+b)/2, (b-a)/2; t))

with W_p from eq.(ansatz) and eq.(1Drec)/(diagonal) (mass m by the rescaling of the main
estimator: coordinates times sqrt(m), coefficient j of V times m^(-j/2), amplitude times sqrt(m)).

Grid reading (the paper states L and the spacing only): x_i = -L + (i + 1/2) D, i = 0..n-1,
D = 2L/n -- symmetric about 0, so parity is kept exactly.

Cutoff reading: the short-time expansion in the half-deviation xbar has a finite radius (Sec. 4;
for the Poeschl-Teller potential the poles of 1/cosh^2), so far from the diagonal the truncated
exponent can grow without bound where the true amplitude is negligible. Elements whose
free-particle factor exp(-(x_j - x_i)^2 / (2t)) is below exp(-40) (4e-18) are set to zero.

Pins (tests/test_oracle_spectrum.py): the harmonic oscillator gives E_n = (n + 1/2)/sqrt(m) and its
ground state pi^(-1/4) exp(-x^2/2) (closed forms); the anharmonic oscillator and the double well
agree with an independent sinc-DVR diagonalization of H (``closed_forms.dvr_eigen``).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from . import effective_action as ea
from . import pimc as opimc


GAUSS_CUT = 40.0


def grid(L: float, n: int):
    """(x, D): x_i = -L + (i + 1/2) D, D = 2L/n."""
    D = 2.0 * L / n
    return -L + (np.arange(n) + 0.5) * D, D


def evolution_matrix(V, m, t, p, L, n):
    """M_ij = D A_1^(p)(x_i, x_j; t) (dense, symmetric), and the grid."""
    Vp = ea.poly(V) if not isinstance(V, tuple) else V
    Vt, _, _, sm = opimc.rescale_mass(Vp, m, 0.0, 0.0)
    tab = opimc.level_tables(Vt, p, t, 0)[0]
    x, D = grid(L, n)
    y = x * sm
    a = y[:, None]
    b = y[None, :]
    mid = 0.5 * (a + b)
    half = 0.5 * (b - a)
    S = opimc.eps_W(tab, mid, half)
    g = (b - a) ** 2 / (2.0 * t)
    logA = -g - S
    with np.errstate(over="ignore"):
        M = D * sm / math.sqrt(2.0 * math.pi * t) * np.exp(logA)
    M[g > GAUSS_CUT] = 0.0
    return M, x, D


def spectrum(V, m, t, p, L, n, k):
    """Lowest k energies E = -ln(lambda)/t of the discretized evolution operator, and the
    eigenfunctions on the grid (columns, normalized sum psi^2 D = 1, largest |psi| positive)."""
    M, x, D = evolution_matrix(V, m, t, p, L, n)
    lam, vec = np.linalg.eigh(M)
    order = np.argsort(lam)[::-1][:k]
    lam = lam[order]
    psi = vec[:, order] / math.sqrt(D)
    for j in range(k):
        i = int(np.argmax(np.abs(psi[:, j])))
        if psi[i, j] < 0:
            psi[:, j] = -psi[:, j]
    return -np.log(lam) / t, psi, x, D


def quartic(A, g):
    return ea.quartic(Fraction(A), Fraction(g))
