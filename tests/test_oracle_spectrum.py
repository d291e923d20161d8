"""Pins of the evolution-operator spectrum oracle (O7): closed forms and an independent method."""
import math

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import spectrum as osp


def test_harmonic_oscillator_levels_are_n_plus_half():
    """V = q^2/2: E_n = n + 1/2 exactly in the continuum; at t = 0.1, p = 10 the short-time error
    is O(t^p) and the grid error (spacing 0.04 against kernel width 0.3) is exponentially small."""
    E, _, _, _ = osp.spectrum(osp.quartic(1, 0), 1.0, 0.1, 10, 8.0, 400, 10)
    assert np.max(np.abs(E - (np.arange(10) + 0.5))) < 1e-12


def test_mass_scales_the_oscillator_frequency():
    """m = 2 with V = q^2/2: omega = 1/sqrt(2), E_n = (n + 1/2)/sqrt(2)."""
    E, _, _, _ = osp.spectrum(osp.quartic(1, 0), 2.0, 0.1, 10, 8.0, 400, 6)
    assert np.max(np.abs(E - (np.arange(6) + 0.5) / math.sqrt(2.0))) < 1e-12


def test_ground_state_wavefunction():
    E, psi, x, D = osp.spectrum(osp.quartic(1, 0), 1.0, 0.1, 10, 8.0, 400, 2)
    ref = math.pi ** -0.25 * np.exp(-x * x / 2)
    assert np.max(np.abs(psi[:, 0] - ref)) < 1e-8
    # the first excited state is odd
    assert np.max(np.abs(psi[:, 1] + psi[::-1, 1])) < 1e-8


def test_low_level_p_is_less_accurate():
    """The short-time error shrinks with p (the speedup of Sec. 2.1): p = 2 is visibly off at
    t = 0.1 for the anharmonic oscillator, p = 10 agrees with DVR."""
    _, Ed, _ = cf.dvr_eigen(cf.quartic_V(1.0, 48.0), L=8.0, h=0.02)
    e2, _, _, _ = osp.spectrum(osp.quartic(1, 48), 1.0, 0.1, 2, 8.0, 400, 5)
    e10, _, _, _ = osp.spectrum(osp.quartic(1, 48), 1.0, 0.1, 10, 8.0, 400, 5)
    err2 = np.max(np.abs(e2 - Ed[:5]))
    err10 = np.max(np.abs(e10 - Ed[:5]))
    assert err10 < 1e-5 and err2 > 100 * err10


@pytest.mark.parametrize("A,g,t,L", [(1.0, 48.0, 0.02, 8.0), (-10.0, 12.0, 0.02, 10.0)])
def test_anharmonic_and_double_well_match_dvr(A, g, t, L):
    """The paper's two potentials of Fig. 3 (smaller grids): low-lying levels against a sinc-DVR
    diagonalization of p^2/2 + V; the double well's near-degenerate pairs included."""
    _, Ed, _ = cf.dvr_eigen(cf.quartic_V(A, g), L=L, h=0.02)
    E, _, _, _ = osp.spectrum(osp.quartic(A, g), 1.0, t, 10, L, 600, 8)
    assert np.max(np.abs(E - Ed[:8]) / np.maximum(1.0, np.abs(Ed[:8]))) < 1e-9
