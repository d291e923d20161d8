"""GPU parity of the several-coordinate mode (rotation-invariant potentials in d = 1..3 dimensions,
eq.(MBrec)/(DIA) in the invariants) against the oracle (oracle/vector.py), the one-dimensional
kernels, closed forms and a two-dimensional DVR continuum.

Tolerances: per-path level actions 1e-12 of max(1, |S|) (both sides FP64; the library's tables come
from an FP64 recursion that agrees with the exact one to ~1e-16, and the kernels evaluate by Horner
in (u, z, w^2) where the oracle sums explicit powers); amplitudes on identical samples 1e-10
relative, errors 1e-7; continuum checks within 5 Monte Carlo standard errors.
"""
import math
import sys

import numpy as np
import pytest

import paper_1105_0542_amd as P
from oracle import closed_forms as cf
from oracle import vector as ov

pytestmark = pytest.mark.gpu

AHO6 = (0.0, 0.5, 6.0 / 24.0)            # (A/2) r^2 + (g/24) r^4, A = 1, g = 6


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = P.Context()
    yield c
    c.close()


CASES = [  # coefs, dim, m, a, b, T, s, p, flags, k
    (AHO6, 2, 1.0, (0.0, 0.0), (0.5, 0.3), 1.0, 5, 10, P.FLAG_HIERARCHY, 1500),        # compile-time shape
    ((0.3, 0.5, 1 / 24), 3, 2.0, (0.1, -0.2, 0.3), (0.4, 0.1, -0.5), 2.0, 6, 8, 0, 1500),
    ((0.0, 0.5), 2, 1.0, (0.2, 0.1), (-0.3, 0.6), 0.5, 2, 4, P.FLAG_HIERARCHY, 1500),  # shape array, U = 2
    (AHO6, 2, 1.0, (0.1, 0.0), (0.3, -0.4), 1.0, 3, 9, P.FLAG_HIERARCHY, 1500),  # shape array, U = 3
    ((0.25, 1.0, 0.125), 1, 1.0, (0.3,), (-0.4,), 1.0, 7, 12, P.FLAG_HIERARCHY, 1500),  # one coordinate
    (AHO6, 3, 1.0, (0.0, 0.2, 0.0), (0.5, 0.0, -0.1), 0.7, 1, 18, P.FLAG_HIERARCHY, 1500),  # U = 1, p = 18
    ((0.0, 0.5, 48 / 24), 2, 1.0, (0.0, 0.0), (1.0, 0.0), 1.0, 10, 18, P.FLAG_HIERARCHY, 300),  # full size
    ((0.0, 0.5, 0.4), 4, 1.5, (0.0, 0.1, 0.2, -0.1), (0.3, 0.0, -0.2, 0.1), 1.0, 6, 12, P.FLAG_HIERARCHY, 600),  # d = 4
    ((0.1, 0.5, 0.4), 4, 1.0, (0.1, 0.0, 0.0, 0.2), (0.0, 0.3, 0.1, 0.0), 0.5, 2, 6, P.FLAG_HIERARCHY, 600),  # d = 4, U = 2
]


@pytest.mark.parametrize("case", CASES)
def test_path_actions_match_oracle(ctx, case):
    coefs, dim, m, a, b, T, s, p, flags, k = case
    _log(f"radial actions coefs={coefs} dim={dim} m={m} a={a} b={b} T={T} s={s} p={p} flags={flags}")
    got = ctx.path_actions_radial(coefs, dim, m, a, b, T, 1 << s, p, 7, 3, flags, 100, k)
    ref = ov.path_actions([float(c) for c in coefs], dim, m, a, b, T, s, p, 7, 3, np.arange(100, 100 + k))
    levels = range(0, s + 1) if flags & P.FLAG_HIERARCHY else [s]
    for n in levels:
        if n == 0 and not (flags & P.FLAG_HIERARCHY):
            continue
        err = np.abs(got[:, n] - ref[:, n])
        assert np.all(err <= 1e-12 * np.maximum(1.0, np.abs(ref[:, n]))), (n, err.max())


@pytest.mark.parametrize("case", CASES[:4])
def test_amplitude_matches_oracle_on_identical_samples(ctx, case):
    coefs, dim, m, a, b, T, s, p, flags, _ = case
    n = 20000
    _log(f"radial amplitude dim={dim} s={s} p={p}")
    res, st = ctx.amplitude_radial(coefs, dim, m, a, b, T, 1 << s, p, n, 5, 1, P.FLAG_HIERARCHY)
    assert st == 0
    ref = ov.amplitude([float(c) for c in coefs], dim, m, a, b, T, s, p, n, 5, 1)
    for lev in range(s + 1):
        assert res[lev].amp == pytest.approx(ref[lev]["amp"], rel=1e-10), lev
        if lev:
            assert res[lev].err == pytest.approx(ref[lev]["err"], rel=1e-7), lev


def test_one_coordinate_equals_the_one_dimensional_kernel(ctx):
    """V = a0 + a1 q^2 + a2 q^4 through the radial mode in d = 1 and through the one-dimensional
    quartic kernel: same paths (coordinate 0 draws the one-dimensional normals), same actions."""
    a0, a1, a2 = 0.25, 0.5, 10 / 24
    for s, p in ((6, 12), (10, 18)):
        r = ctx.path_actions_radial((a0, a1, a2), 1, 1.3, (0.2,), (0.9,), 1.5, 1 << s, p, 9, 4,
                                    P.FLAG_HIERARCHY, 0, 2048)
        o = ctx.path_actions([a0, 0, a1, 0, a2], 1.3, 0.2, 0.9, 1.5, 1 << s, p, 9, 4, P.FLAG_HIERARCHY, 0, 2048)
        assert np.max(np.abs(r - o) / np.maximum(1.0, np.abs(o))) < 1e-12, (s, p)


def test_hierarchy_levels_equal_separate_runs(ctx):
    """Level n of an s-run is bitwise the n-run on the same paths (the bisection nests), across the
    compile-time (s >= 4) and the shape-array (s < 4) evaluators, and so are the amplitudes and
    errors (the canonical chunks do not depend on s)."""
    big = ctx.path_actions_radial(AHO6, 2, 1.0, (0.0, 0.0), (0.5, 0.3), 1.0, 64, 10, 2, 0, P.FLAG_HIERARCHY, 0, 3000)
    full, _ = ctx.amplitude_radial(AHO6, 2, 1.0, (0.0, 0.0), (0.5, 0.3), 1.0, 64, 10, 30000, 2, 0, P.FLAG_HIERARCHY)
    for s in (1, 2, 3, 5):
        small = ctx.path_actions_radial(AHO6, 2, 1.0, (0.0, 0.0), (0.5, 0.3), 1.0, 1 << s, 10, 2, 0,
                                        P.FLAG_HIERARCHY, 0, 3000)
        assert np.array_equal(big[:, :s + 1], small), s
        part, _ = ctx.amplitude_radial(AHO6, 2, 1.0, (0.0, 0.0), (0.5, 0.3), 1.0, 1 << s, 10, 30000, 2, 0, 0)
        assert part[s].amp == full[s].amp, s
        assert part[s].err == full[s].err, s


def test_single_slice_is_the_short_time_amplitude(ctx):
    res, st = ctx.amplitude_radial(AHO6, 2, 1.7, (0.1, 0.2), (0.4, -0.3), 0.3, 1, 12, 100, 1)
    ref = ov.short_time_amplitude([float(c) for c in AHO6], 2, 1.7, (0.1, 0.2), (0.4, -0.3), 0.3, 12)
    assert st == 0 and res[0].amp == pytest.approx(ref, rel=1e-13) and res[0].err == 0.0


def test_largest_size_nests(ctx):
    """Three coordinates at N = 2^20 (the deepest walk, 65 LDS slots per lane): levels 0..8 of the
    per-path actions equal an s = 8 run of the same paths bitwise, and the finest level is finite."""
    big = ctx.path_actions_radial(AHO6, 3, 1.0, (0.0, 0.1, 0.0), (0.3, 0.0, 0.2), 1.0, 1 << 20, 6, 3, 1,
                                  P.FLAG_HIERARCHY, 0, 256)
    small = ctx.path_actions_radial(AHO6, 3, 1.0, (0.0, 0.1, 0.0), (0.3, 0.0, 0.2), 1.0, 1 << 8, 6, 3, 1,
                                    P.FLAG_HIERARCHY, 0, 256)
    assert np.array_equal(big[:, :9], small)
    assert np.all(np.isfinite(big[:, 20]))
    # the fine levels converge: N = 2^19 and 2^20 differ by far less than N = 2^4 and 2^5
    d_fine = np.abs(big[:, 20] - big[:, 19]).mean()
    d_coarse = np.abs(big[:, 5] - big[:, 4]).mean()
    assert d_fine < 1e-3 * d_coarse


def test_largest_four_coordinate_walk_nests(ctx):
    """Four coordinates at N = 2^19, the deepest walk whose LDS (16 level sums and the pending right
    endpoints of levels 2..16, 76 slots per lane, 159,616 bytes per workgroup) fits in 160 KB: levels
    0..8 of the per-path actions equal an s = 8 run of the same paths bitwise."""
    a, b = (0.0, 0.1, 0.0, -0.2), (0.3, 0.0, 0.2, 0.1)
    big = ctx.path_actions_radial(AHO6, 4, 1.0, a, b, 1.0, 1 << 19, 6, 5, 2, P.FLAG_HIERARCHY, 0, 128)
    small = ctx.path_actions_radial(AHO6, 4, 1.0, a, b, 1.0, 1 << 8, 6, 5, 2, P.FLAG_HIERARCHY, 0, 128)
    assert np.array_equal(big[:, :9], small)
    assert np.all(np.isfinite(big[:, 19]))


def test_convergence_to_the_2d_continuum(ctx):
    """The 2D anharmonic oscillator (A = 1, g = 6), A((0,0), (0.4,0.2); 1) from one s = 10 run per p:
    p = 10 agrees with a tensor-product sinc-DVR at every N >= 16 within the MC error, while p = 1 at
    N = 16 is visibly off (its discretization error is O(1/N))."""
    V = lambda X, Y: 0.5 * (X ** 2 + Y ** 2) + 0.25 * (X ** 2 + Y ** 2) ** 2
    ref = ov.dvr_amplitude_2d(V, (0.0, 0.0), (0.4, 0.2), 1.0, L=6.0, h=0.2)
    n = 2_000_000
    r10, _ = ctx.amplitude_radial(AHO6, 2, 1.0, (0.0, 0.0), (0.4, 0.2), 1.0, 1024, 10, n, 11, 0, P.FLAG_HIERARCHY)
    r1, _ = ctx.amplitude_radial(AHO6, 2, 1.0, (0.0, 0.0), (0.4, 0.2), 1.0, 1024, 1, n, 11, 0, P.FLAG_HIERARCHY)
    _log(f"DVR {ref:.8f}; p=10: " + " ".join(f"{r.amp:.6f}" for r in r10[4:]) +
         "; p=1: " + " ".join(f"{r.amp:.6f}" for r in r1[4:]))
    for lev in range(4, 11):
        assert abs(r10[lev].amp - ref) <= 5 * r10[lev].err, (lev, r10[lev].amp, ref, r10[lev].err)
    assert abs(r1[4].amp - ref) > 10 * r1[4].err
    assert abs(r1[10].amp - ref) < abs(r1[4].amp - ref)


def test_isotropic_oscillator_is_the_mehler_product(ctx):
    """Three coordinates, V = r^2/2, mass 2: the exact kernel is the product of three Mehler kernels."""
    a, b, T, m = (0.1, -0.3, 0.2), (0.4, 0.2, -0.1), 1.2, 2.0
    res, _ = ctx.amplitude_radial((0.0, 0.5), 3, m, a, b, T, 256, 12, 1_000_000, 4, 2, P.FLAG_HIERARCHY)
    ref = math.prod(cf.mehler(x, y, T, 1.0, m) for x, y in zip(a, b))
    for lev in (3, 6, 8):
        assert abs(res[lev].amp - ref) <= 5 * res[lev].err, (lev, res[lev].amp, ref, res[lev].err)


def test_four_dimensional_oscillator_is_the_mehler_product(ctx):
    """Four coordinates (two particles in two dimensions, no interaction), V = r^2/2, mass 1.5: the
    exact kernel is the product of four Mehler kernels."""
    a, b, T, m = (0.1, -0.3, 0.2, 0.0), (0.4, 0.2, -0.1, 0.3), 1.0, 1.5
    res, _ = ctx.amplitude_radial((0.0, 0.5), 4, m, a, b, T, 256, 12, 1_000_000, 4, 2, P.FLAG_HIERARCHY)
    ref = math.prod(cf.mehler(x, y, T, 1.0, m) for x, y in zip(a, b))
    for lev in (3, 6, 8):
        assert abs(res[lev].amp - ref) <= 5 * res[lev].err, (lev, res[lev].amp, ref, res[lev].err)


def test_invalid_arguments(ctx):
    with pytest.raises(P.PimcError) as e:
        ctx.amplitude_radial(AHO6, 2, 1.0, (0, 0), (1, 0), 1.0, 16, 4, 100, 1, 0, P.FLAG_FP32_POLY)
    assert e.value.status == -2
    with pytest.raises(P.PimcError) as e:             # four coordinates: the walk's LDS at N = 2^20
        ctx.amplitude_radial(AHO6, 4, 1.0, (0, 0, 0, 0), (1, 0, 0, 0), 1.0, 1 << 20, 4, 100, 1)
    assert e.value.status == -2
    with pytest.raises(P.PimcError):
        ctx.amplitude_radial(AHO6, 2, 1.0, (0, 0), (1, 0), 1.0, 16, 19, 100, 1)           # p > 18
    with pytest.raises(P.PimcError):
        ctx.amplitude_radial(AHO6, 2, 1.0, (0, float("inf")), (1, 0), 1.0, 16, 4, 100, 1)
    with pytest.raises(ValueError):
        ctx.amplitude_radial(AHO6, 2, 1.0, (0, 0, 0), (1, 0), 1.0, 16, 4, 100, 1)
