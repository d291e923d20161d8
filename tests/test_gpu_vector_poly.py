"""GPU parity of the several-coordinate mode for any polynomial potential (eq.(MBrec)/(DIA) in the
components of x and xbar, Sec. 2.2) against the oracle's component route (oracle/vector.py), the
rotation-invariant route, the one-dimensional route and the Mehler kernels of coupled oscillators.

Tolerances: per-path level actions within 1e-12 of the sum over slices of the absolute monomial
terms (both sides FP64; the library's coefficients come from an FP64 recursion that agrees with the
exact one to ~1e-15 relative, the kernel evaluates by Horner over the prefix tree of the monomials,
the oracle sums the monomials one by one, so the rounding differences scale with the terms, not with
their sum); amplitudes on identical samples 1e-10 relative, errors 1e-7; exact kernels within 5
Monte Carlo standard errors.
"""
import math
import sys

import numpy as np
import pytest

import paper_1105_0542_amd as P
from oracle import closed_forms as cf
from oracle import effective_action as ea
from oracle import pimc as opimc
from oracle import vector as ov

pytestmark = pytest.mark.gpu

# 0.1 (q1 - q2)^4 plus an anisotropic quadratic part and a linear field: two particles on a line
COUPLED_2D = [(0.5, (2, 0)), (0.7, (0, 2)), (0.1, (4, 0)), (-0.4, (3, 1)), (0.6, (2, 2)), (-0.4, (1, 3)),
              (0.1, (0, 4)), (0.3, (1, 0)), (0.2, (1, 1))]
# an anisotropic trap with cubic and quartic couplings in three coordinates
COUPLED_3D = [(0.5, (2, 0, 0)), (0.4, (0, 2, 0)), (0.3, (0, 0, 2)), (0.2, (0, 2, 1)), (0.05, (1, 1, 2)),
              (0.05, (0, 0, 4)), (0.1, (2, 2, 0)), (0.1, (0, 0, 1))]
# two particles in two dimensions, r_1 = (q_1, q_2), r_2 = (q_3, q_4): |r_1|^2/2 + |r_2|^2/2 + 0.1 |r_1 - r_2|^4
TWO_PARTICLES_2D = [
    (0.1, (4, 0, 0, 0)), (-0.4, (3, 0, 1, 0)), (0.2, (2, 2, 0, 0)), (-0.4, (2, 1, 0, 1)), (0.6, (2, 0, 2, 0)),
    (0.2, (2, 0, 0, 2)), (0.5, (2, 0, 0, 0)), (-0.4, (1, 2, 1, 0)), (0.8, (1, 1, 1, 1)), (-0.4, (1, 0, 3, 0)),
    (-0.4, (1, 0, 1, 2)), (0.1, (0, 4, 0, 0)), (-0.4, (0, 3, 0, 1)), (0.2, (0, 2, 2, 0)), (0.6, (0, 2, 0, 2)),
    (0.5, (0, 2, 0, 0)), (-0.4, (0, 1, 2, 1)), (-0.4, (0, 1, 0, 3)), (0.1, (0, 0, 4, 0)), (0.2, (0, 0, 2, 2)),
    (0.5, (0, 0, 2, 0)), (0.1, (0, 0, 0, 4)), (0.5, (0, 0, 0, 2))]


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = P.Context()
    yield c
    c.close()


CASES = [  # terms, dim, m, a, b, T, s, p, flags, k
    (COUPLED_2D, 2, 1.0, (0.0, 0.0), (0.5, 0.3), 1.0, 5, 6, P.FLAG_HIERARCHY, 1200),
    (COUPLED_3D, 3, 2.0, (0.1, -0.2, 0.3), (0.4, 0.1, -0.5), 2.0, 6, 4, 0, 1200),
    (COUPLED_2D, 2, 1.0, (0.2, 0.1), (-0.3, 0.6), 0.5, 2, 5, P.FLAG_HIERARCHY, 1200),    # U = 2
    (COUPLED_3D, 3, 1.0, (0.0, 0.2, 0.0), (0.5, 0.0, -0.1), 0.7, 1, 6, P.FLAG_HIERARCHY, 1200),  # U = 1
    (COUPLED_3D, 3, 1.5, (0.3, 0.2, -0.1), (0.5, -0.4, 0.2), 1.0, 3, 5, P.FLAG_HIERARCHY, 1200),   # U = 3
    (COUPLED_2D, 2, 1.0, (0.1, -0.1), (0.6, 0.2), 1.0, 4, 7, P.FLAG_HIERARCHY, 1200),           # U = 4
    (COUPLED_2D, 2, 1.0, (0.0, 0.0), (1.0, 0.0), 1.0, 10, 10, P.FLAG_HIERARCHY, 200),     # full size
    (COUPLED_3D, 3, 1.0, (0.0, 0.0, 0.0), (0.5, 0.5, 0.0), 1.0, 8, 8, P.FLAG_HIERARCHY, 200),
    (TWO_PARTICLES_2D, 4, 1.0, (0.0, 0.1, 0.2, 0.0), (0.3, 0.0, 0.1, -0.2), 1.0, 6, 6, P.FLAG_HIERARCHY, 400),  # d = 4
    (TWO_PARTICLES_2D, 4, 2.0, (0.1, 0.0, 0.0, 0.2), (0.0, 0.3, 0.1, 0.0), 0.5, 3, 5, 0, 400),      # d = 4, U = 3
    (TWO_PARTICLES_2D, 4, 1.0, (0.2, 0.0, -0.1, 0.1), (0.1, 0.2, 0.0, -0.3), 1.0, 7, 4, P.FLAG_HIERARCHY, 100),
    # d = 4, U = 7 (one subtree, no walk levels)
    (COUPLED_3D, 3, 1.0, (0.1, 0.0, 0.2), (0.0, -0.3, 0.4), 1.5, 9, 5, P.FLAG_HIERARCHY, 100),  # U = 7, 2 walk levels
]


def _check_levels(got, ref, scale, s, flags):
    levels = range(1, s + 1) if flags & P.FLAG_HIERARCHY else [s]
    for n in levels:
        err = np.abs(got[:, n] - ref[:, n])
        assert np.all(err <= 1e-12 * scale[:, n]), (n, float(np.max(err / scale[:, n])))


@pytest.mark.parametrize("case", CASES)
def test_path_actions_match_oracle(ctx, case):
    terms, dim, m, a, b, T, s, p, flags, k = case
    _log(f"poly actions dim={dim} m={m} a={a} b={b} T={T} s={s} p={p} flags={flags} k={k}")
    got = ctx.path_actions_poly(terms, dim, m, a, b, T, 1 << s, p, 7, 3, flags, 100, k)
    ref, scale = ov.poly_path_actions(terms, dim, m, a, b, T, s, p, 7, 3, np.arange(100, 100 + k),
                                      with_scale=True)
    _check_levels(got, ref, scale, s, flags)


@pytest.mark.parametrize("case", CASES[:6])
def test_amplitude_matches_oracle_on_identical_samples(ctx, case):
    terms, dim, m, a, b, T, s, p, _, _ = case
    n = 20000
    _log(f"poly amplitude dim={dim} s={s} p={p}")
    res, st = ctx.amplitude_poly(terms, dim, m, a, b, T, 1 << s, p, n, 5, 1, P.FLAG_HIERARCHY)
    assert st == 0
    ref = ov.poly_amplitude(terms, dim, m, a, b, T, s, p, n, 5, 1)
    for lev in range(s + 1):
        assert res[lev].amp == pytest.approx(ref[lev]["amp"], rel=1e-10), lev
        if lev:
            assert res[lev].err == pytest.approx(ref[lev]["err"], rel=1e-7), lev


def _radial_terms(a, d):
    return [(float(c), k[:d]) for k, c in ov.radial_to_components(a, d).items()]


@pytest.mark.parametrize("dim,p,s", [(2, 12, 6), (3, 8, 5), (4, 8, 6)])
def test_rotation_invariant_V_equals_the_radial_route(ctx, dim, p, s):
    """V = r^2/2 + r^4/4 written out in components: per-path actions equal the oracle's invariant route
    (and the library's radial mode) on the same paths."""
    a = (0.0, 0.5, 0.25)
    terms = _radial_terms(a, dim)
    qa, qb = (0.1, -0.2, 0.3, 0.0)[:dim], (0.4, 0.1, -0.2, 0.1)[:dim]
    _log(f"poly isotropic dim={dim} p={p} s={s}")
    got = ctx.path_actions_poly(terms, dim, 1.5, qa, qb, 1.0, 1 << s, p, 11, 2, P.FLAG_HIERARCHY, 0, 400)
    ref = ov.path_actions(a, dim, 1.5, qa, qb, 1.0, s, p, 11, 2, np.arange(400))
    _, scale = ov.poly_path_actions(terms, dim, 1.5, qa, qb, 1.0, s, p, 11, 2, np.arange(400), with_scale=True)
    _check_levels(got, ref, scale, s, P.FLAG_HIERARCHY)
    rad = ctx.path_actions_radial(a, dim, 1.5, qa, qb, 1.0, 1 << s, p, 11, 2, P.FLAG_HIERARCHY, 0, 400)
    _check_levels(got, rad, scale, s, P.FLAG_HIERARCHY)


def test_one_coordinate_equals_the_one_dimensional_route(ctx):
    """d = 1, V = sum c_n q^n (odd terms included): the one-dimensional oracle's path actions."""
    coefs = [0.2, -0.3, 0.5, 0.1, 0.25]
    terms = [(c, (n,)) for n, c in enumerate(coefs)]
    s, p = 7, 8
    got = ctx.path_actions_poly(terms, 1, 2.0, (0.3,), (-0.4,), 1.0, 1 << s, p, 9, 1, P.FLAG_HIERARCHY, 0, 600)
    ref = opimc.path_actions(ea.poly(coefs), 2.0, 0.3, -0.4, 1.0, s, p, 9, 1, np.arange(600))
    _, scale = ov.poly_path_actions(terms, 1, 2.0, (0.3,), (-0.4,), 1.0, s, p, 9, 1, np.arange(600), with_scale=True)
    _check_levels(got, ref, scale, s, P.FLAG_HIERARCHY)


def test_free_particle_and_split_runs(ctx):
    """No potential terms: every action is 0 and the amplitude is the free kernel. A run split at an
    arbitrary path index gives the same actions bitwise (canonical chunks)."""
    res, st = ctx.amplitude_poly([], 2, 1.0, (0.0, 0.0), (0.3, 0.4), 1.0, 64, 6, 5000, 1, 0, P.FLAG_HIERARCHY)
    K0 = ov.free_kernel((0.0, 0.0), (0.3, 0.4), 1.0)
    assert st == 0
    for r in res:
        assert r.amp == pytest.approx(K0, rel=1e-14) and r.err == 0.0
    whole = ctx.path_actions_poly(COUPLED_2D, 2, 1.0, (0.0, 0.1), (0.3, 0.0), 1.0, 256, 6, 4, 0, P.FLAG_HIERARCHY,
                                  1000, 5000)
    a = ctx.path_actions_poly(COUPLED_2D, 2, 1.0, (0.0, 0.1), (0.3, 0.0), 1.0, 256, 6, 4, 0, P.FLAG_HIERARCHY,
                              1000, 1777)
    b = ctx.path_actions_poly(COUPLED_2D, 2, 1.0, (0.0, 0.1), (0.3, 0.0), 1.0, 256, 6, 4, 0, P.FLAG_HIERARCHY,
                              2777, 3223)
    assert np.array_equal(whole, np.concatenate([a, b]))


def test_path_indices_beyond_32_bits(ctx):
    """Path indices above 2^32 (the high word enters the generator counter): the oracle's paths."""
    first = (1 << 33) + 7
    got = ctx.path_actions_poly(COUPLED_2D, 2, 1.0, (0.1, 0.0), (0.4, -0.2), 1.0, 16, 5, 3, 9, P.FLAG_HIERARCHY,
                                first, 300)
    ref, scale = ov.poly_path_actions(COUPLED_2D, 2, 1.0, (0.1, 0.0), (0.4, -0.2), 1.0, 4, 5, 3, 9,
                                      np.arange(first, first + 300, dtype=np.uint64), with_scale=True)
    _check_levels(got, ref, scale, 4, P.FLAG_HIERARCHY)


def test_two_particles_in_two_dimensions(ctx):
    """Four coordinates: amplitudes on identical samples against the oracle, and the exact separation
    R = (r_1 + r_2)/sqrt 2, rho = (r_1 - r_2)/sqrt 2 (|R|^2/2 + |rho|^2/2 + 0.4 |rho|^4, same free
    measure): at the continuum the amplitude is the Mehler product in R times the two-dimensional
    anharmonic oscillator in rho, which the radial mode gives (here both at p = 10, N = 64)."""
    a, b, T = (0.0, 0.1, 0.2, 0.0), (0.3, 0.0, 0.1, -0.2), 1.0
    n = 4000
    res, st = ctx.amplitude_poly(TWO_PARTICLES_2D, 4, 1.0, a, b, T, 16, 5, n, 5, 1, P.FLAG_HIERARCHY)
    ref = ov.poly_amplitude(TWO_PARTICLES_2D, 4, 1.0, a, b, T, 4, 5, n, 5, 1)
    assert st == 0
    for lev in range(5):
        assert res[lev].amp == pytest.approx(ref[lev]["amp"], rel=1e-10), lev
        if lev:
            assert res[lev].err == pytest.approx(ref[lev]["err"], rel=1e-7), lev
    r2 = math.sqrt(2.0)
    Ra, Rb = [(a[i] + a[i + 2]) / r2 for i in (0, 1)], [(b[i] + b[i + 2]) / r2 for i in (0, 1)]
    ra, rb = [(a[i] - a[i + 2]) / r2 for i in (0, 1)], [(b[i] - b[i + 2]) / r2 for i in (0, 1)]
    full, _ = ctx.amplitude_poly(TWO_PARTICLES_2D, 4, 1.0, a, b, T, 64, 10, 2_000_000, 3, 0, P.FLAG_HIERARCHY)
    rel, _ = ctx.amplitude_radial((0.0, 0.5, 0.4), 2, 1.0, ra, rb, T, 64, 10, 2_000_000, 4, 0, P.FLAG_HIERARCHY)
    com = cf.mehler(Ra[0], Rb[0], T) * cf.mehler(Ra[1], Rb[1], T)
    ref6 = com * rel[6].amp
    err6 = math.hypot(full[6].err, com * rel[6].err)
    _log(f"two particles in 2D: {full[6].amp:.8e} +- {full[6].err:.1e}; separated {ref6:.8e}")
    assert abs(full[6].amp - ref6) <= 5 * err6, (full[6].amp, ref6, err6)


def test_largest_size_nests(ctx):
    """Three coordinates at N = 2^20 (the deepest walk): levels 0..8 of the per-path actions equal an
    s = 8 run of the same paths bitwise, and the finest level is finite and converged."""
    args = (COUPLED_3D, 3, 1.0, (0.0, 0.1, 0.0), (0.3, 0.0, 0.2), 1.0)
    big = ctx.path_actions_poly(*args, 1 << 20, 4, 3, 1, P.FLAG_HIERARCHY, 0, 64)
    small = ctx.path_actions_poly(*args, 1 << 8, 4, 3, 1, P.FLAG_HIERARCHY, 0, 64)
    assert np.array_equal(big[:, :9], small)
    assert np.all(np.isfinite(big[:, 20]))
    assert np.abs(big[:, 20] - big[:, 19]).mean() < 1e-3 * np.abs(big[:, 5] - big[:, 4]).mean()


def test_largest_four_coordinate_walk_nests(ctx):
    """Two particles in two dimensions at N = 2^20 (7-level subtrees, 13 walk levels: 61 LDS slots
    per lane, 128,992 bytes per workgroup): levels 0..8 of the per-path actions equal an s = 8 run of
    the same paths bitwise, and the finest level is finite."""
    args = (TWO_PARTICLES_2D, 4, 1.0, (0.0, 0.1, 0.0, -0.2), (0.3, 0.0, 0.2, 0.1), 1.0)
    big = ctx.path_actions_poly(*args, 1 << 20, 4, 3, 1, P.FLAG_HIERARCHY, 0, 64)
    small = ctx.path_actions_poly(*args, 1 << 8, 4, 3, 1, P.FLAG_HIERARCHY, 0, 64)
    assert np.array_equal(big[:, :9], small)
    assert np.all(np.isfinite(big[:, 20]))


def test_coupled_oscillators_are_a_mehler_product(ctx):
    """V = q1^2/2 + q2^2/2 + g (q1 - q2)^2 separates in r = (q1 - q2)/sqrt 2 (omega^2 = 1 + 4g) and
    s = (q1 + q2)/sqrt 2 (omega = 1); the exact kernel is the product of the two Mehler kernels at the
    rotated endpoints (the free measure is rotation invariant)."""
    g, m, T = 0.3, 1.5, 1.0
    terms = [(0.5 + g, (2, 0)), (0.5 + g, (0, 2)), (-2 * g, (1, 1))]
    a, b = (0.1, -0.3), (0.4, 0.2)
    res, _ = ctx.amplitude_poly(terms, 2, m, a, b, T, 64, 10, 1_000_000, 4, 2, P.FLAG_HIERARCHY)
    r2 = math.sqrt(2.0)
    ref = (cf.mehler((a[0] - a[1]) / r2, (b[0] - b[1]) / r2, T, 1.0 + 4 * g, m)
           * cf.mehler((a[0] + a[1]) / r2, (b[0] + b[1]) / r2, T, 1.0, m))
    _log(f"coupled oscillators: exact {ref:.10f}; " + " ".join(f"{r.amp:.10f}+-{r.err:.1e}" for r in res[2:]))
    for lev in (2, 4, 6):
        assert abs(res[lev].amp - ref) <= 5 * res[lev].err + 1e-12 * ref, (lev, res[lev].amp, ref, res[lev].err)


def test_invalid_arguments(ctx):
    with pytest.raises(P.PimcError) as e:
        ctx.amplitude_poly(COUPLED_2D, 2, 1.0, (0, 0), (1, 0), 1.0, 16, 4, 100, 1, 0, P.FLAG_FP32_POLY)
    assert e.value.status == -2
    with pytest.raises(P.PimcError):
        ctx.amplitude_poly(COUPLED_2D, 2, 1.0, (0, 0), (1, 0), 1.0, 16, 19, 100, 1)       # p > 18
    with pytest.raises(P.PimcError):
        ctx.amplitude_poly([(0.1, (5, 0))], 2, 1.0, (0, 0), (1, 0), 1.0, 16, 4, 100, 1)   # degree 5
    with pytest.raises(ValueError):
        ctx.amplitude_poly(COUPLED_2D, 2, 1.0, (0, 0, 0), (1, 0), 1.0, 16, 4, 100, 1)
