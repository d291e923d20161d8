"""GPU parity of the general-potential mode (derivative symbols) against the model-specific modes,
the oracle (oracle/general.py, symbolic derivatives) and a DVR continuum reference.

Tolerances: per-path level actions 1e-12 of max(1, |S|) -- the monomial sums of the derivative
form and the folded tables of the model-specific forms are different FP64 evaluations of the same
polynomial (the largest difference measured over these cases is logged by each test). Against the
oracle, whose derivatives come from other formulas (symbolic differentiation), 1e-12 of the sum of
the absolute monomial terms, the scale of the rounding error where terms cancel (at the coarse
levels of paths far from the origin that sum is up to 80 times |S|). Amplitudes on identical
samples 1e-10 relative; the continuum check within 5 MC standard errors.
"""
import sys

import numpy as np
import pytest

import paper_1105_0542_amd as P
from oracle import closed_forms as cf
from oracle import general as og

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = P.Context()
    yield c
    c.close()


def _close(got, ref, tol=1e-12, scale=None):
    """|got - ref| <= tol * max(1, scale), scale = |ref| or the sum of the absolute monomial terms
    (oracle path_action_scales) where the terms cancel."""
    err = np.abs(got - ref)
    sc = np.maximum(1.0, np.abs(ref) if scale is None else scale)
    lim = tol * sc
    _log(f"  max |diff| / max(1, scale) = {(err / sc).max():.2e}")
    assert np.all(err <= lim), (err / lim).max()


@pytest.mark.parametrize("s,p,flags", [(5, 6, P.FLAG_HIERARCHY), (7, 8, 0), (2, 10, P.FLAG_HIERARCHY)])
def test_polynomial_through_derivatives_equals_polynomial_mode(ctx, s, p, flags):
    coefs = P.quartic(1.0, 10.0)
    k = 1000
    g = ctx.path_actions_general(1.0, 0.0, 1.0, 2.0, 1 << s, p, 4, 2, flags, 0, k, poly=coefs)
    r = ctx.path_actions(coefs, 1.0, 0.0, 1.0, 2.0, 1 << s, p, 4, 2, flags, 0, k)
    for n in (range(1, s + 1) if flags else [s]):
        _close(g[:, n], r[:, n])


@pytest.mark.parametrize("p", range(1, 19))
def test_every_generated_level_equals_polynomial_mode(ctx, p):
    """Every evaluator generated at build time (p = 1..10 inline, 11..18 out of line), with one-level
    (U = 1) and deeper walks, on a degree-8 polynomial with odd terms, against the polynomial tables."""
    coefs = [0.3, -0.2, 0.5, 0.1, 0.05, 0.0, 0.01, 0.0, 0.002]
    k = 512
    for s in (1, 3):
        g = ctx.path_actions_general(1.0, -0.2, 0.7, 1.0, 1 << s, p, 6, 1, P.FLAG_HIERARCHY, 0, k, poly=coefs)
        r = ctx.path_actions(coefs, 1.0, -0.2, 0.7, 1.0, 1 << s, p, 6, 1, P.FLAG_HIERARCHY, 0, k)
        for n in range(0, s + 1):
            _close(g[:, n], r[:, n])


def test_sech2_through_derivatives_equals_poeschl_teller_mode(ctx):
    k = 1000
    g = ctx.path_actions_general(1.3, -0.5, 0.5, 1.0, 64, 8, 9, 1, P.FLAG_HIERARCHY, 0, k, sech2=((-2.0, 1.2),))
    r = ctx.path_actions_mpt(2.0, 1.2, 1.3, -0.5, 0.5, 1.0, 64, 8, 9, 1, P.FLAG_HIERARCHY, 0, k)
    for n in range(1, 7):
        _close(g[:, n], r[:, n])


@pytest.mark.parametrize("p", [12, 14, 18])
def test_high_levels_sech2_equal_poeschl_teller_mode(ctx, p):
    """The out-of-line evaluators on -lambda/cosh^2(alpha q) against the model-specific tanh ansatz
    (an independent form of the same level-p action), at the levels where the series converges
    well (eps = T/N <= 1/32)."""
    k = 256
    s = 5
    _log(f"general p={p} sech2 vs Poeschl-Teller mode, N={1 << s}, {k} paths")
    g = ctx.path_actions_general(1.3, -0.5, 0.5, 1.0, 1 << s, p, 9, 1, 0, 0, k, sech2=((-2.0, 1.2),))
    r = ctx.path_actions_mpt(2.0, 1.2, 1.3, -0.5, 0.5, 1.0, 1 << s, p, 9, 1, 0, 0, k)
    d = np.abs(g[:, s] - r[:, s]) / np.maximum(1.0, np.abs(r[:, s]))
    _log(f"  max relative difference {d.max():.2e}")
    _close(g[:, s], r[:, s])


CASES = [  # m, a, b, T, s, p, poly, sech2, gauss
    (1.0, -0.3, 0.4, 1.0, 5, 6, (0, 0, 0.5), (), ((2.0, 1.0),)),                        # barrier in an oscillator
    (1.7, 0.2, -0.6, 0.5, 4, 8, (0.1, 0.2, 0.4, 0.0, 0.02), ((-1.0, 0.8),), ((0.5, 2.0), (-0.3, 0.5))),
    (1.0, 0.1, 0.3, 0.5, 3, 4, (0, 0, 0.5), ((-1.0, 0.8), (0.5, 1.5), (-0.2, 2.0), (0.3, 0.5)),   # every term slot
     ((0.5, 2.0), (-0.3, 0.5), (0.2, 1.0), (0.1, 3.0))),
    (1.0, -9.0, 11.0, 1.0, 5, 5, (0, 0, 0.5), ((-1.0, 3.0),), ((2.0, 4.0),)),   # saturated tanh, tiny Gaussian
]


CASES_HI = [  # m, a, b, T, s, p, poly, sech2, gauss: the out-of-line levels, level s only (eps = T/N)
    (1.0, -0.3, 0.4, 0.5, 4, 12, (0, 0, 0.5), ((-1.0, 0.8),), ((2.0, 1.0),)),
    (1.7, 0.2, -0.6, 0.5, 4, 14, (0.1, 0.2, 0.4, 0.0, 0.02), ((-1.0, 0.8),), ((0.5, 2.0), (-0.3, 0.5))),
    (1.0, -0.3, 0.4, 0.5, 4, 18, (0, 0, 0.5), ((-1.0, 0.8),), ((2.0, 1.0),)),
]


@pytest.mark.parametrize("case", CASES_HI)
def test_high_level_path_actions_match_oracle(ctx, case):
    m, a, b, T, s, p, poly, sech2, gauss = case
    _log(f"general actions (out of line) m={m} a={a} b={b} T={T} s={s} p={p} poly={poly} sech2={sech2} gauss={gauss}")
    k = 128
    got = ctx.path_actions_general(m, a, b, T, 1 << s, p, 3, 8, 0, 50, k, poly=poly, sech2=sech2, gauss=gauss)
    ref = og.path_actions(p, T, s, a, b, 3, 8, np.arange(50, 50 + k), poly=poly, sech2=sech2, gauss=gauss, m=m,
                          levels=[s])
    d = np.abs(got[:, s] - ref[:, s]) / np.maximum(1.0, np.abs(ref[:, s]))
    _log(f"  max relative difference {d.max():.2e}")
    _close(got[:, s], ref[:, s])


@pytest.mark.parametrize("case", CASES)
def test_path_actions_match_oracle(ctx, case):
    m, a, b, T, s, p, poly, sech2, gauss = case
    _log(f"general actions m={m} a={a} b={b} T={T} s={s} p={p} poly={poly} sech2={sech2} gauss={gauss}")
    k = 600
    got = ctx.path_actions_general(m, a, b, T, 1 << s, p, 3, 8, P.FLAG_HIERARCHY, 50, k, poly=poly, sech2=sech2,
                                   gauss=gauss)
    ref = og.path_actions(p, T, s, a, b, 3, 8, np.arange(50, 50 + k), poly=poly, sech2=sech2, gauss=gauss, m=m)
    scale = og.path_action_scales(p, T, s, a, b, 3, 8, np.arange(50, 50 + k), poly=poly, sech2=sech2, gauss=gauss,
                                  m=m)
    for n in range(1, s + 1):
        _close(got[:, n], ref[:, n], scale=scale[:, n])


def test_amplitude_matches_oracle_on_identical_samples(ctx):
    m, a, b, T, s, p, poly, sech2, gauss = CASES[0]
    n = 20000
    res, _ = ctx.amplitude_general(m, a, b, T, 1 << s, p, n, 6, 0, P.FLAG_HIERARCHY, poly=poly, sech2=sech2,
                                   gauss=gauss)
    S = og.path_actions(p, T, s, a, b, 6, 0, np.arange(n), poly=poly, sech2=sech2, gauss=gauss, m=m)
    import math
    for lev in range(1, s + 1):
        M = 1 << lev
        q = a + (b - a) * np.arange(M + 1) / M
        d = og.derivative_functions(p, poly, sech2, gauss, m)
        ref_line = og.eps_W(p, T / M, d, 0.5 * (q[1:] + q[:-1]), 0.5 * (q[1:] - q[:-1])).sum()
        w = np.expm1(-(S[:, lev] - ref_line))
        K0 = math.exp(-(b - a) ** 2 / (2 * T)) / math.sqrt(2 * math.pi * T)
        amp = K0 * math.exp(-ref_line) * (1 + math.fsum(w) / n)
        assert res[lev].amp == pytest.approx(amp, rel=1e-10), lev


def test_gaussian_barrier_converges_to_the_continuum(ctx):
    """V = q^2/2 + 2 exp(-q^2): A(-0.3, 0.4; 1) at p = 8 against a DVR diagonalization of H."""
    V = lambda x: 0.5 * x * x + 2.0 * np.exp(-x * x)
    ref = cf.dvr_amplitude(V, -0.3, 0.4, 1.0, L=8.0, h=0.025 / 2.5)
    res, _ = ctx.amplitude_general(1.0, -0.3, 0.4, 1.0, 256, 8, 2_000_000, 12, 0, P.FLAG_HIERARCHY,
                                   poly=(0, 0, 0.5), gauss=((2.0, 1.0),))
    _log(f"DVR {ref:.8f}; p=8 N=16..256: " + " ".join(f"{r.amp:.7f}+-{r.err:.1e}" for r in res[4:]))
    for lev in range(4, 9):
        assert abs(res[lev].amp - ref) <= 5 * res[lev].err, (lev, res[lev].amp, ref)


def test_invalid_arguments(ctx):
    with pytest.raises(P.PimcError):
        ctx.amplitude_general(1.0, 0, 1, 1, 16, 19, 100, 1, poly=(0, 0, 0.5))       # p > 18
    with pytest.raises(P.PimcError):
        ctx.amplitude_general(1.0, 0, 1, 1, 16, 4, 100, 1, gauss=((1.0, -1.0),))     # beta <= 0
    with pytest.raises(P.PimcError) as e:
        ctx.amplitude_general(1.0, 0, 1, 1, 16, 4, 100, 1, 0, P.FLAG_FP32_POLY, poly=(0, 0, 0.5))
    assert e.value.status == -2
