"""Pins of the many-coordinate effective action (oracle O10) against what the paper and the
mathematics fix, independently of how eq.(MBrec) and the invariant operators were transcribed."""
import math
from fractions import Fraction as F
from math import comb

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import effective_action as ea
from oracle import pimc as opimc
from oracle import vector as ov


# ----------------------------------------------------------------------------- polynomial helpers
# Polynomials in (x_1..x_d, xbar_1..xbar_d, eps) as {exponent tuple: Fraction}, written here again so
# that the PDE check shares nothing with the oracle's recursion.
def _p_add(A, B, s=1):
    out = dict(A)
    for k, v in B.items():
        out[k] = out.get(k, 0) + s * v
    return {k: v for k, v in out.items() if v != 0}


def _p_mul(A, B):
    out = {}
    for ka, a in A.items():
        for kb, b in B.items():
            k = tuple(x + y for x, y in zip(ka, kb))
            out[k] = out.get(k, 0) + a * b
    return {k: v for k, v in out.items() if v != 0}


def _p_d(A, var):
    out = {}
    for k, v in A.items():
        if k[var]:
            nk = list(k)
            nk[var] -= 1
            out[tuple(nk)] = out.get(tuple(nk), 0) + v * k[var]
    return out


def _p_times(A, var=None, s=1):
    out = {}
    for k, v in A.items():
        nk = list(k)
        if var is not None:
            nk[var] += 1
        out[tuple(nk)] = v * s
    return out


def W_full(Wmk, d, p):
    """W_p with eps as the last variable: sum_{m<p} eps^(m-k) W_{m,k}."""
    out = {}
    for (m, k), poly in Wmk.items():
        if m >= p:
            continue
        for mono, c in poly.items():
            key = tuple(mono) + (m - k,)
            out[key] = out.get(key, 0) + c
    return out


def shifted_potential_average(V, d):
    """(V(x + xbar) + V(x - xbar))/2 for a polynomial V in the components x (binomial expansion)."""
    out = {}
    for mono, c in V.items():
        # product over coordinates of (x_i +- xbar_i)^(e_i); the +- terms average to the even ones
        terms = {tuple([0] * (2 * d + 1)): F(1)}
        for i in range(d):
            e = mono[i]
            fac = {}
            for j in range(e + 1):
                k = [0] * (2 * d + 1)
                k[i] = e - j
                k[d + i] = j
                fac[tuple(k)] = F(comb(e, j))
            terms = _p_mul(terms, fac)
        for k, v in terms.items():
            if sum(k[d:2 * d]) % 2 == 0:
                out[k] = out.get(k, 0) + c * v
    return out


def pde_residual(Wmk, V, d, p):
    """LHS - RHS of eq.(eqWMB) for W = W_p (vectors x, xbar of d components, exact)."""
    W = W_full(Wmk, d, p)
    ne = 2 * d                                     # index of eps
    R = dict(W)
    R = _p_add(R, {k: v * sum(k[d:2 * d]) for k, v in W.items()})          # xbar . gradbar W
    R = _p_add(R, {k: v * k[ne] for k, v in W.items()})                    # eps d/deps W
    for i in range(d):
        R = _p_add(R, _p_times(_p_d(_p_d(W, i), i), ne, F(-1, 8)))          # -eps/8 grad^2 W
        R = _p_add(R, _p_times(_p_d(_p_d(W, d + i), d + i), ne, F(-1, 8)))  # -eps/8 gradbar^2 W
        gi = _p_d(W, i)
        R = _p_add(R, _p_times(_p_times(_p_mul(gi, gi), ne), ne, F(1, 8)))  # +eps^2/8 (grad W)^2
        gb = _p_d(W, d + i)
        R = _p_add(R, _p_times(_p_times(_p_mul(gb, gb), ne), ne, F(1, 8)))  # +eps^2/8 (gradbar W)^2
    Vx = {tuple(k) + (0,): v for k, v in V.items()}
    R = _p_add(R, shifted_potential_average(Vx, d), -1)
    return R


def low_order(R, d, p):
    """Terms eps^e (xbar-degree 2k) with e + k <= p - 1."""
    return {k: v for k, v in R.items() if k[2 * d] + sum(k[d:2 * d]) // 2 <= p - 1}


def comp(d, terms):
    """Polynomial in the components from {((x exponents), (xbar exponents)): coef}."""
    return {tuple(x) + tuple(xb): F(c) for (x, xb), c in terms.items()}


GENERAL_2D = comp(2, {((2, 0), (0, 0)): F(1, 2), ((0, 2), (0, 0)): F(3, 2), ((1, 2), (0, 0)): F(1, 3),
                      ((4, 0), (0, 0)): F(1, 5), ((1, 1), (0, 0)): F(-1, 4)})
POTENTIALS = {
    "aho2d": (2, ov.radial_to_components(ov.aho2d(1, 6), 2)),
    "aho3d": (3, ov.radial_to_components(ov.aho2d(2, 1), 3)),
    "radial_sextic_2d": (2, ov.radial_to_components((F(1, 3), F(1, 2), F(-1, 4), F(1, 12)), 2)),
    "general_2d": (2, GENERAL_2D),
}


# ----------------------------------------------------------------------------- eq.(eqWMB)
@pytest.mark.parametrize("name", sorted(POTENTIALS))
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_pde_satisfied_through_order_p_minus_1(name, p):
    """W_p of the component route solves eq.(eqWMB) at every eps^e xbar^(2k) with e + k <= p-1."""
    d, V = POTENTIALS[name]
    W = ov.component_coefficients(V, d, p)
    R = pde_residual(W, V, d, p)
    assert not low_order(R, d, p), sorted(low_order(R, d, p))[:5]
    if p >= 2:
        assert any(k[2 * d] + sum(k[d:2 * d]) // 2 == p for k in R)     # not vacuous


def test_pde_check_catches_a_planted_mistake():
    d, V = POTENTIALS["aho2d"]
    W = ov.component_coefficients(V, d, 4)
    bad = dict(W)
    bad[(3, 1)] = {k: -v for k, v in W[(3, 1)].items()}
    assert low_order(pde_residual(bad, V, d, 4), d, 4)
    bad = dict(W)
    key = next(iter(W[(2, 0)]))
    bad[(2, 0)] = dict(W[(2, 0)])
    bad[(2, 0)][key] = W[(2, 0)][key] * 2
    assert low_order(pde_residual(bad, V, d, 4), d, 4)


# ----------------------------------------------------------------------------- reductions
@pytest.mark.parametrize("V1", [ea.quartic(1, 6), ea.poly([F(1, 3), F(-1, 2), F(1), F(3, 10), F(1, 24)])])
def test_one_coordinate_equals_the_one_dimensional_recursion(V1):
    p = 6
    V = {(n, 0): c for n, c in enumerate(V1) if c}
    W = ov.component_coefficients(V, 1, p)
    c = ea.coefficients(V1, p)
    for (m, k), poly in W.items():
        assert poly == {(i, 2 * k): v for i, v in enumerate(c[(m, k)]) if v}, (m, k)


def test_separable_potential_gives_the_sum_of_one_dimensional_actions():
    """V = V1(x_1) + V2(x_2): the short-time amplitude factorizes, so W_{m,k} is the sum of the
    one-dimensional contractions c1_{m,k}(x_1) xbar_1^(2k) + c2_{m,k}(x_2) xbar_2^(2k)."""
    p = 5
    V1 = ea.quartic(1, 6)
    V2 = ea.poly([F(1, 3), F(-1, 2), F(1), F(3, 10), F(1, 24)])
    V = {}
    for n, c in enumerate(V1):
        if c:
            V[(n, 0, 0, 0)] = V.get((n, 0, 0, 0), 0) + c
    for n, c in enumerate(V2):
        if c:
            V[(0, n, 0, 0)] = V.get((0, n, 0, 0), 0) + c
    W = ov.component_coefficients(V, 2, p)
    c1 = ea.coefficients(V1, p)
    c2 = ea.coefficients(V2, p)
    for (m, k), poly in W.items():
        ref = {}
        for i, v in enumerate(c1[(m, k)]):
            if v:
                ref[(i, 0, 2 * k, 0)] = ref.get((i, 0, 2 * k, 0), 0) + v
        for i, v in enumerate(c2[(m, k)]):
            if v:
                ref[(0, i, 0, 2 * k)] = ref.get((0, i, 0, 2 * k), 0) + v
        ref = {kk: v for kk, v in ref.items() if v != 0}
        assert poly == ref, (m, k)


@pytest.mark.parametrize("d,p", [(2, 3), (2, 5), (3, 3), (3, 4), (4, 3)])
@pytest.mark.parametrize("a", [ov.aho2d(1, 6), (F(1, 3), F(1, 2), F(-1, 4), F(1, 12))])
def test_invariant_route_equals_the_component_route(d, p, a):
    Wc = ov.component_coefficients(ov.radial_to_components(a, d), d, p)
    Wi = ov.invariant_coefficients(a, d, p)
    assert set(Wc) == set(Wi)
    for key in Wc:
        assert ov.invariants_to_components(Wi[key], d) == Wc[key], key


@pytest.mark.parametrize("p", [4, 10, 14])
def test_one_coordinate_invariant_tables_give_the_one_dimensional_action(p):
    """In d = 1 the invariant polynomials are representatives of the one-dimensional W_p: the
    folded slice action agrees with the one-dimensional oracle's to rounding."""
    a = (F(1, 4), F(1, 2), F(5, 24))                     # V = 1/4 + x^2/2 + 5 x^4/24
    V1 = ea.poly([a[0], 0, a[1], 0, a[2]])
    eps = 0.3
    tab_v = ov.level_tables(a, 1, p, eps, 0)[0]
    tab_1 = ea.xbar_groups_float(V1, p, F(eps))
    rng = np.random.default_rng(3)
    x = rng.uniform(-1.5, 1.5, 200)
    xb = rng.uniform(-0.6, 0.6, 200)
    got = ov.eps_W(tab_v, x[:, None], xb[:, None])
    ref = opimc.eps_W(tab_1, x, xb)
    scale = np.abs(ref) + 1.0
    assert np.max(np.abs(got - ref) / scale) < 1e-13


def test_w_power_is_even_and_tables_have_the_contraction_form():
    for d in (1, 2, 3):
        for (m, k), poly in ov.invariant_coefficients(ov.aho2d(1, 48), d, 9).items():
            for (i, j, l), c in poly.items():
                assert j % 2 == 0 and j // 2 + l == k, (d, m, k, i, j, l)


# ----------------------------------------------------------------------------- paths
def test_coordinate_zero_is_the_one_dimensional_path():
    idx = np.arange(5, 40, dtype=np.uint64)
    qv = ov.bisection_paths((0.1, -0.3, 0.2), (0.5, 0.4, -0.1), 1.3, 5, 11, 2, idx)
    q1 = opimc.bisection_paths(0.1, 0.5, 1.3, 5, 11, 2, idx)
    assert np.array_equal(qv[:, :, 0], q1)
    # the other coordinates are bridges of their own: different draws, same endpoints
    assert not np.allclose(qv[:, 1:-1, 1], qv[:, 1:-1, 0])
    assert np.all(qv[:, 0, 1] == -0.3) and np.all(qv[:, -1, 2] == -0.1)


def test_bridge_covariance():
    """Each coordinate at the middle of [0, T] is N((a+b)/2, T/4); coordinates are uncorrelated."""
    idx = np.arange(20000, dtype=np.uint64)
    q = ov.bisection_paths((0.0, 1.0), (2.0, -1.0), 2.0, 3, 5, 0, idx)
    mid = q[:, 4, :]
    assert abs(mid[:, 0].mean() - 1.0) < 0.02 and abs(mid[:, 1].mean()) < 0.02
    assert abs(mid[:, 0].var() - 0.5) < 0.02 and abs(mid[:, 1].var() - 0.5) < 0.02
    assert abs(np.corrcoef(mid[:, 0], mid[:, 1])[0, 1]) < 0.03


# ----------------------------------------------------------------------------- continuum
def test_short_time_amplitude_converges_to_the_2d_continuum():
    """2D anharmonic oscillator (A = 1, g = 6), A_1^(p)((0,0), (0.4,0.2); 0.25) against a
    tensor-product sinc-DVR: the error falls with p and is below 1e-9 at p = 8."""
    V = lambda X, Y: 0.5 * (X ** 2 + Y ** 2) + 0.25 * (X ** 2 + Y ** 2) ** 2
    ex = ov.dvr_amplitude_2d(V, (0.0, 0.0), (0.4, 0.2), 0.25, L=6.0, h=0.2)
    errs = [abs(ov.short_time_amplitude(ov.aho2d(1, 6), 2, 1.0, (0.0, 0.0), (0.4, 0.2), 0.25, p) / ex - 1)
            for p in (1, 2, 4, 6, 8)]
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1)), errs
    assert errs[-1] < 1e-9 and errs[0] > 1e-3


def test_harmonic_short_time_amplitude_is_the_mehler_product():
    """Isotropic oscillator: the 2D kernel is the product of two Mehler kernels; A_1^(p) converges."""
    errs = []
    for p in (2, 4, 8, 12):
        a = ov.short_time_amplitude(ov.aho2d(1, 0), 2, 1.0, (0.3, -0.2), (0.5, 0.4), 0.5, p)
        errs.append(abs(a / (cf.mehler(0.3, 0.5, 0.5) * cf.mehler(-0.2, 0.4, 0.5)) - 1))
    assert all(errs[i + 1] < 0.05 * errs[i] for i in range(len(errs) - 1)), errs
    assert errs[-1] < 1e-10


def test_mass_rescaling():
    """H = p^2/(2m) + V: the amplitude equals m^(d/2) times that of V(y/sqrt(m)) at sqrt(m) q; for
    the oscillator this is the Mehler product with omega = sqrt(A/m)."""
    m = 2.5
    a = ov.short_time_amplitude(ov.aho2d(1, 0), 2, m, (0.3, -0.2), (0.5, 0.4), 0.4, 12)
    ref = cf.mehler(0.3, 0.5, 0.4, 1.0, m) * cf.mehler(-0.2, 0.4, 0.4, 1.0, m)
    assert abs(a / ref - 1) < 1e-10


# ----------------------------------------------------------------------------- any polynomial V
def _terms_of(C, d):
    """[(coef, exponents of q)] of a component polynomial with no xbar part."""
    return [(float(c), k[:d]) for k, c in C.items()]


@pytest.mark.parametrize("d,p", [(2, 6), (3, 4), (4, 4)])
def test_component_slice_action_of_a_radial_V_is_the_invariant_one(d, p):
    """For V = sum a_n (q.q)^n written out in components, the component-route slice action (fold over
    m, k of the exact W_{m,k} and term-by-term evaluation) equals the invariant-route tables evaluated
    by Horner in (u, w^2, z)."""
    a = (F(1, 3), F(1, 2), F(-1, 4), F(1, 12))
    V = ov.terms_to_components(_terms_of(ov.radial_to_components(a, d), d), d)
    rng = np.random.default_rng(3)
    x = rng.uniform(-1.5, 1.5, (40, d))
    xb = rng.uniform(-0.4, 0.4, (40, d))
    for eps in (F(1), F(1, 8)):
        tab = ov.component_tables(V, d, p, float(eps), 0)[0]
        got = ov.component_eps_W(tab, x, xb)
        ref = ov.eps_W(ov.level_tables(a, d, p, float(eps), 0)[0], x, xb)
        scale = ov.component_eps_W_abs(tab, x, xb)
        assert np.all(np.abs(got - ref) <= 1e-13 * scale), np.max(np.abs(got - ref) / scale)
        assert np.all(scale >= np.abs(got) * (1 - 1e-14))


def test_component_slice_action_of_a_rotated_separable_V():
    """Two particles on a line with a pair interaction, V = a (q1 - q2)^4 + c (q1 - q2)^2 + b (q1 + q2)^2,
    separate in r = (q1 - q2)/sqrt 2, s = (q1 + q2)/sqrt 2 into 4a r^4 + 2c r^2 and 2b s^2. The
    effective action is covariant under the rotation, so the component route (every cross term
    q1^i q2^j of W) equals the sum of the one-dimensional actions at the rotated x and xbar."""
    a, b, c = F(1, 10), F(1, 4), F(1, 8)
    V = {}
    for i in range(5):                                    # (q1 - q2)^4
        V[(i, 4 - i, 0, 0)] = V.get((i, 4 - i, 0, 0), 0) + a * comb(4, i) * (-1) ** (4 - i)
    for i in range(3):                                    # (q1 - q2)^2 and (q1 + q2)^2
        V[(i, 2 - i, 0, 0)] = V.get((i, 2 - i, 0, 0), 0) + (c * (-1) ** (2 - i) + b) * comb(2, i)
    V = {k: v for k, v in V.items() if v}
    p, eps = 6, 0.3
    tab = ov.component_tables(V, 2, p, eps, 0)[0]
    rng = np.random.default_rng(5)
    x = rng.uniform(-1.5, 1.5, (40, 2))
    xb = rng.uniform(-0.4, 0.4, (40, 2))
    got = ov.component_eps_W(tab, x, xb)
    r2 = math.sqrt(2.0)
    tr = opimc.level_tables(ea.poly([0, 0, 2 * c, 0, 4 * a]), p, eps, 0)[0]
    ts = opimc.level_tables(ea.poly([0, 0, 2 * b]), p, eps, 0)[0]
    ref = (opimc.eps_W(tr, (x[:, 0] - x[:, 1]) / r2, (xb[:, 0] - xb[:, 1]) / r2)
           + opimc.eps_W(ts, (x[:, 0] + x[:, 1]) / r2, (xb[:, 0] + xb[:, 1]) / r2))
    scale = ov.component_eps_W_abs(tab, x, xb)
    assert np.all(np.abs(got - ref) <= 1e-13 * scale + 1e-15), np.max(np.abs(got - ref))
    # the cross terms matter: dropping them changes the action
    keep = np.array([not (e[0] and e[1]) and not (e[2] and e[3]) for e in tab[0]])
    part = ov.component_eps_W((tab[0][keep], tab[1][keep]), x, xb)
    assert np.max(np.abs(part - ref)) > 1e-3


def test_component_paths_and_mass_equal_the_radial_route():
    """Path actions of the component route for a rotation-invariant V (mass 4, d = 2) equal those of
    the invariant route level by level (same paths, same tables up to rounding); the level-0 amplitude
    is the short-time amplitude."""
    a = (0.0, 0.5, 0.25)
    d, m, qa, qb, T, s, p = 2, 4.0, (0.1, -0.2), (0.3, 0.4), 1.0, 4, 6
    terms = _terms_of(ov.radial_to_components(a, d), d)
    S, scale = ov.poly_path_actions(terms, d, m, qa, qb, T, s, p, 7, 3, np.arange(20, 84), with_scale=True)
    ref = ov.path_actions(a, d, m, qa, qb, T, s, p, 7, 3, np.arange(20, 84))
    assert np.all(np.abs(S - ref) <= 1e-13 * scale)
    amp = ov.poly_amplitude(terms, d, m, qa, qb, T, 2, p, 256, 7, 3)
    assert amp[0]["amp"] == pytest.approx(ov.short_time_amplitude(a, d, m, qa, qb, T, p), rel=1e-13)
    ref_amp = ov.amplitude(a, d, m, qa, qb, T, 2, p, 256, 7, 3)
    for n in (1, 2):
        assert amp[n]["amp"] == pytest.approx(ref_amp[n]["amp"], rel=1e-12)


def test_one_coordinate_component_route_is_the_one_dimensional_path_action():
    """d = 1: the component route on V = sum c_n q^n gives the one-dimensional path actions (same
    paths: coordinate 0 draws the one-dimensional normals)."""
    coefs = [0.2, -0.3, 0.5, 0.1, 0.25]
    terms = [(c, (n,)) for n, c in enumerate(coefs)]
    S, scale = ov.poly_path_actions(terms, 1, 2.0, (0.3,), (-0.4,), 1.0, 4, 5, 9, 1, np.arange(40), with_scale=True)
    ref = opimc.path_actions(ea.poly(coefs), 2.0, 0.3, -0.4, 1.0, 4, 5, 9, 1, np.arange(40))
    assert np.all(np.abs(S - ref) <= 1e-13 * scale)


# two particles in two dimensions, r_1 = (q_1, q_2), r_2 = (q_3, q_4): V = |r_1|^2/2 + |r_2|^2/2
# + 0.1 |r_1 - r_2|^4, expanded in the four coordinates
TWO_PARTICLES_2D = [
    (0.1, (4, 0, 0, 0)), (-0.4, (3, 0, 1, 0)), (0.2, (2, 2, 0, 0)), (-0.4, (2, 1, 0, 1)), (0.6, (2, 0, 2, 0)),
    (0.2, (2, 0, 0, 2)), (0.5, (2, 0, 0, 0)), (-0.4, (1, 2, 1, 0)), (0.8, (1, 1, 1, 1)), (-0.4, (1, 0, 3, 0)),
    (-0.4, (1, 0, 1, 2)), (0.1, (0, 4, 0, 0)), (-0.4, (0, 3, 0, 1)), (0.2, (0, 2, 2, 0)), (0.6, (0, 2, 0, 2)),
    (0.5, (0, 2, 0, 0)), (-0.4, (0, 1, 2, 1)), (-0.4, (0, 1, 0, 3)), (0.1, (0, 0, 4, 0)), (0.2, (0, 0, 2, 2)),
    (0.5, (0, 0, 2, 0)), (0.1, (0, 0, 0, 4)), (0.5, (0, 0, 0, 2))]


def test_two_particles_in_two_dimensions_separate_into_centre_of_mass_and_relative_motion():
    """With R = (r_1 + r_2)/sqrt 2 and rho = (r_1 - r_2)/sqrt 2 the potential is |R|^2/2 + |rho|^2/2 +
    0.4 |rho|^4 and the free measure is unchanged, so the four-coordinate slice action (component
    route, every cross term of the pair interaction) equals the two-dimensional isotropic oscillator's
    at (R, Rbar) plus the two-dimensional anharmonic oscillator's at (rho, rhobar), both from the
    invariant route."""
    p, eps = 5, 0.3
    tab = ov.component_tables(ov.terms_to_components(TWO_PARTICLES_2D, 4), 4, p, eps, 0)[0]
    rng = np.random.default_rng(11)
    x = rng.uniform(-1.2, 1.2, (30, 4))
    xb = rng.uniform(-0.3, 0.3, (30, 4))
    got = ov.component_eps_W(tab, x, xb)
    r2 = math.sqrt(2.0)

    def split(v):
        return (v[:, :2] + v[:, 2:]) / r2, (v[:, :2] - v[:, 2:]) / r2
    (R, rho), (Rb, rhob) = split(x), split(xb)
    ref = (ov.eps_W(ov.level_tables((0.0, 0.5), 2, p, eps, 0)[0], R, Rb)
           + ov.eps_W(ov.level_tables((0.0, 0.5, 0.4), 2, p, eps, 0)[0], rho, rhob))
    scale = ov.component_eps_W_abs(tab, x, xb)
    assert np.all(np.abs(got - ref) <= 1e-13 * scale + 1e-15), np.max(np.abs(got - ref))
