"""Host-side checks of the C ABI library: it loads, exports what include/pimc.h declares, validates
arguments, and its FP64 effective-action tables agree with the oracle's exact ones. No device use."""
import ctypes
import math
import os
import re
from fractions import Fraction

import numpy as np
import pytest

import paper_1105_0542_amd as P
from oracle import effective_action as ea
from oracle import pimc as opimc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(pimc_\w+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(P.lib_path())
    decl = _declared_functions()
    assert len(decl) >= 10
    missing = [n for n in decl if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("args,ok", [
    ((P.quartic(1, 1), 1.0, 0.0, 1.0, 1.0, 16, 4, 100000), True),
    ((P.quartic(1, 1), 1.0, 0.0, 1.0, 1.0, 15, 4, 100000), False),          # N not a power of two
    ((P.quartic(1, 1), 1.0, 0.0, 1.0, 1.0, 0, 4, 100000), False),
    ((P.quartic(1, 1), 1.0, 0.0, 1.0, 1.0, 1 << 21, 4, 100000), False),    # N > 2^20
    ((P.quartic(1, 1), 1.0, 0.0, 1.0, 1.0, 16, 0, 100000), False),         # p < 1
    ((P.quartic(1, 1), 1.0, 0.0, 1.0, 1.0, 16, 19, 100000), False),        # p > 18
    ((P.quartic(1, 1), 1.0, 0.0, 1.0, 0.0, 16, 4, 100000), False),         # T <= 0
    ((P.quartic(1, 1), 0.0, 0.0, 1.0, 1.0, 16, 4, 100000), False),         # m <= 0
    ((P.quartic(1, 1), 1.0, 0.0, 1.0, 1.0, 16, 4, 1), False),              # n < 2
    ((P.quartic(1, 1), 1.0, float("nan"), 1.0, 1.0, 16, 4, 10), False),
    ((P.quartic(1, 1), 1.0, 0.0, 1.0, float("inf"), 16, 4, 10), False),
    (([0, 0, 0.5, 0, float("nan")], 1.0, 0.0, 1.0, 1.0, 16, 4, 10), False),
    ((list(range(1, 10)), 1.0, 0.0, 1.0, 1.0, 1, 18, 10), True),           # degree 8, N = 1
])
def test_argument_validation(args, ok):
    st = P.check_problem(*args)
    assert (st == 0) == ok
    if not ok:
        assert st == -1


def test_degree_above_limit_is_rejected():
    lib = P.load_library()
    V = P.binding.Potential()
    V.degree = 9
    assert lib.pimc_check_problem(ctypes.byref(V), 1.0, 0.0, 1.0, 1.0, 16, 4, 10) == -1
    assert b"degree" in lib.pimc_last_error(None)


def _oracle_table(coefs, m, T, p, level):
    Vex = ea.poly([Fraction(c) for c in coefs])
    Vt, _, _, _ = opimc.rescale_mass(Vex, m, 0.0, 0.0)
    even = all(c == 0 for c in Vt[1::2])
    Q = ea.xbar_groups(Vt, p, Fraction(T) / (1 << level))
    out = []
    degs = []
    for k, q in enumerate(Q):
        if even:
            cs = [q[i] if i < len(q) else 0 for i in range(0, max(len(q), 1), 2)]
        else:
            cs = list(q) if q else [0]
        degs.append(len(cs) - 1)
        out += [float(c / 4 ** k) for c in reversed(cs)]
    return np.array(out), degs, even


@pytest.mark.parametrize("coefs,m,T,p,level", [
    (P.quartic(1, 1), 1.0, 1.0, 4, 4),
    (P.quartic(1, 10), 1.0, 1.0, 18, 9),
    (P.quartic(1, 48), 1.0, 5.0, 18, 3),
    (P.quartic(-1, 4), 1.0, 2.0, 12, 6),
    (P.quartic(1, 10), 2.5, 2.0, 12, 5),
    ([0.25, -0.5, 1.0, 0.3, 1 / 24], 1.0, 1.0, 10, 3),
    ([0.0, 0.0, 0.5, 0.0, -0.2, 0.0, 1 / 30.0], 1.0, 0.5, 14, 4),
    ([0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9], 1.0, 1.0, 18, 8),
    (P.quartic(1, 48), 1.0, 0.02, 21, 0),         # the short-time tables of the spectrum (p = 21)
    (P.quartic(-10, 12), 1.0, 0.1, 21, 0),
])
def test_level_table_matches_exact_oracle(coefs, m, T, p, level):
    """The library's FP64 recursion and folding (eq.(1Drec), eq.(diagonal)) agree with the exact
    rational table to 1e-13 relative per entry, with the same layout."""
    tab, deg, even = P.level_table(coefs, m, T, p, level)
    ref, rdeg, reven = _oracle_table(coefs, m, T, p, level)
    assert even == reven
    assert deg == rdeg
    scale = np.maximum(np.abs(ref), 1e-300)
    big = np.abs(ref) > 1e-280
    assert np.max(np.abs(tab - ref)[big] / scale[big]) < 1e-13


def test_level_table_capacity_error():
    lib = P.load_library()
    V = P.potential_from_coefs(P.quartic(1, 1))
    need = ctypes.c_size_t(0)
    buf = (ctypes.c_double * 2)()
    st = lib.pimc_level_table(ctypes.byref(V), 1.0, 1.0, 18, 3, buf, 2, ctypes.byref(need), None, None, None)
    assert st == -1 and need.value == 48


def test_strerror_codes():
    lib = P.load_library()
    for code in (0, -1, -2, -3, -4, 1, 2):
        assert lib.pimc_strerror(code)


def test_create_without_device_reports_device_error():
    """On a host without a GPU, context creation fails with PIMC_EDEVICE and a message (no fallback)."""
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    with pytest.raises(P.PimcError) as ei:
        P.Context(use_torch_stream=False)
    assert ei.value.status == -4


def test_flow_entry_points_validate_without_a_device():
    """The proposal's entry points reject a missing context or handle before touching a device."""
    lib = P.load_library()
    V = P.potential_from_coefs(P.quartic(1, 10))
    cfg = P.binding.FlowConfig(8, 4096, 1e-3, 0.0, 0, 0.0)
    h = ctypes.c_void_p()
    assert lib.pimc_flow_create(None, ctypes.byref(V), 1.0, 0.0, 1.0, 2.0, 128, 12, ctypes.byref(cfg),
                                ctypes.byref(h)) == -1
    assert not h.value
    assert lib.pimc_flow_create(None, ctypes.byref(V), 1.0, 0.0, 1.0, 2.0, 100, 12, ctypes.byref(cfg),
                                ctypes.byref(h)) == -1          # N not a power of two
    assert lib.pimc_flow_destroy(None) == 0
    assert lib.pimc_flow_train(None, 1, 0, 1, None, None) == -1
    assert lib.pimc_flow_amplitude(None, 100, 1, 0, None, None) == -1
    loss = ctypes.c_double(0)
    assert lib.pimc_flow_grad(None, 1, 0, ctypes.byref(loss), None, None) == -1


def test_spectrum_entry_points_validate_without_a_device():
    lib = P.load_library()
    V = P.potential_from_coefs(P.quartic(1, 48))
    E = (ctypes.c_double * 4)()
    assert lib.pimc_spectrum(None, ctypes.byref(V), 1.0, 0.02, 21, 8.0, 1024, 4, 100, 1e-10, E, None, None) == -1
    assert lib.pimc_evolution_matrix(None, ctypes.byref(V), 1.0, 0.02, 8, 8.0, 64, None, 64) == -1
    assert lib.pimc_strerror(2)


@pytest.mark.parametrize("lam,alpha,m,T,p,level", [
    (1.0, 1.0, 1.0, 1.0, 10, 4), (3.0, 0.75, 1.0, 2.0, 12, 6), (2.0, 1.5, 2.0, 0.5, 8, 2), (1.0, 1.0, 1.0, 0.05, 21, 0),
])
def test_mpt_level_table_matches_exact_oracle(lam, alpha, m, T, p, level):
    """The Poeschl-Teller tables of the library (FP64 recursion in tanh(alpha x)) agree with the
    exact rational recursion of the oracle, folded the same way (P_k in u = tanh^2, 4^-k). Since
    0 <= u < 1, each P_k block is compared against the sum of its |coefficients| (the bound of its
    value): the FP64 fold cancels large alternating terms where eps is beyond the convergence
    radius (coarse levels at p >= 14), never in these cases."""
    from fractions import Fraction
    from oracle import mpt
    tab, deg = P.level_table_mpt(lam, alpha, m, T, p, level)
    am = mpt._alpha_m(alpha, m)
    Q = mpt.xbar_groups(lam, am, p, Fraction(T) / (1 << level))
    rdeg = []
    off = 0
    for k, q in enumerate(Q):
        assert all(q[i] == 0 for i in range(1, len(q), 2))
        blk = np.array([float(q[i] / 4 ** k) for i in range(0, len(q), 2)][::-1])
        rdeg.append(blk.size - 1)
        got = tab[off:off + blk.size]
        off += blk.size
        assert np.max(np.abs(got - blk)) <= 1e-14 * np.sum(np.abs(blk)), k
    assert deg == rdeg and off == tab.size


@pytest.mark.parametrize("coefs,dim,m,T,p,level", [
    ((0.0, 0.5, 10 / 24), 2, 1.0, 1.0, 18, 3), ((0.0, 0.5, 10 / 24), 2, 1.0, 2.0, 10, 0),
    ((0.3, 0.5, 1 / 24), 3, 2.0, 1.0, 12, 5), ((0.25, 1.0, 0.125), 1, 1.0, 0.5, 8, 2), ((1.0,), 2, 1.0, 1.0, 4, 1),
    ((0.0, 0.5, 0.4), 4, 1.5, 1.0, 10, 3),
])
def test_radial_level_table_matches_exact_oracle(coefs, dim, m, T, p, level):
    """Several coordinates: the library's FP64 invariant recursion folded per level agrees with the
    oracle's exact tables (component-pinned), group by group; every exact coefficient lies inside
    the compile-time shape."""
    from oracle import vector as ov
    tab, shape = P.level_table_radial(coefs, dim, m, T, p, level)
    a = ov.rescale_mass([Fraction(c) for c in coefs], m)
    Q = ov.level_groups(a, dim, p, Fraction(T) / (1 << level))
    seen = set()
    off = 0
    for k, j, ln in shape:
        ref = [float(c) for c in reversed(Q[k][j])] if k < len(Q) else []
        assert len(ref) <= ln, (k, j)
        ref = np.array([0.0] * (ln - len(ref)) + ref)
        got = tab[off:off + ln]
        off += ln
        assert np.all(np.abs(got - ref) <= 1e-14 * (np.abs(ref) + np.max(np.abs(tab)))), (k, j)
        seen.add((k, j))
    assert off == tab.size
    for k, row in enumerate(Q):
        for j, q in enumerate(row):
            if any(c != 0 for c in q):
                assert (k, j) in seen, (k, j)


COUPLED_2D = [(0.5, (2, 0)), (0.7, (0, 2)), (0.1, (4, 0)), (-0.4, (3, 1)), (0.6, (2, 2)), (-0.4, (1, 3)),
              (0.1, (0, 4)), (0.3, (1, 0)), (0.2, (1, 1))]        # 0.1 (q1 - q2)^4 + quadratic and linear


@pytest.mark.parametrize("terms,dim,m,T,p,level", [
    (COUPLED_2D, 2, 1.0, 1.0, 6, 2), (COUPLED_2D, 2, 4.0, 2.0, 5, 0),
    ([(0.5, (2, 0, 0)), (0.2, (0, 2, 1)), (0.05, (1, 1, 2)), (0.3, (0, 0, 2)), (0.1, (0, 0, 1))], 3, 2.0, 1.0, 4, 3),
    ([(0.2, (0,)), (-0.3, (1,)), (0.5, (2,)), (0.25, (4,))], 1, 1.0, 0.5, 7, 1),
    ([(0.5, (2, 0, 0, 0)), (0.5, (0, 0, 0, 2)), (0.1, (2, 0, 2, 0)), (-0.2, (1, 1, 1, 1)), (0.05, (0, 4, 0, 0)),
      (0.3, (0, 0, 1, 0))], 4, 2.0, 1.0, 5, 2),
])
def test_poly_level_table_matches_exact_oracle(terms, dim, m, T, p, level):
    """Any polynomial V: the library's FP64 component recursion folded per level agrees monomial by
    monomial with the oracle's exact eps W_p (the component route), and lists every monomial once."""
    from oracle import vector as ov
    coef, exps = P.level_table_poly(terms, dim, m, T, p, level)
    V = ov.terms_to_components(terms, dim, m)
    ref = ov.component_level_terms(V, dim, p, Fraction(T) / (1 << level))
    keys = [tuple(int(x) for x in e) for e in exps]
    assert len(set(keys)) == len(keys)
    got = dict(zip(keys, coef))
    top = max(abs(float(v)) for v in ref.values())
    for k, v in ref.items():
        assert abs(got.get(k, 0.0) - float(v)) <= 1e-14 * (abs(float(v)) + top), k
    for k, c in got.items():
        if k not in ref:
            assert abs(c) <= 1e-14 * top, k


def test_poly_entry_points_validate_without_a_device():
    lib = P.load_library()
    a = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    b = (ctypes.c_double * 3)(1.0, 0.0, 0.0)
    out = (ctypes.c_double * 16)()

    def st(V, N=16, p=4):
        return lib.pimc_path_actions_poly(None, ctypes.byref(V), 1.0, a, b, 1.0, N, p, 1, 0, 0, 0, 1, out)

    assert st(P.poly_potential([(0.5, (2, 0))], 0)) == -1                  # dim
    assert st(P.poly_potential([(0.5, (2, 0))], 5)) == -1
    assert st(P.poly_potential([(0.5, (2, 1, 1))], 2)) == -1               # exponent beyond dim
    assert st(P.poly_potential([(0.5, (3, 2))], 2)) == -1                  # total degree 5
    assert st(P.poly_potential([(0.5, (-1, 2))], 2)) == -1                 # negative exponent
    assert st(P.poly_potential([(float("nan"), (2, 0))], 2)) == -1
    assert st(P.poly_potential([(0.5, (2, 0))], 2), N=15) == -1
    assert st(P.poly_potential([(0.5, (2, 0))], 2), p=0) == -1
    V = P.poly_potential([(0.5, (2, 0))], 2)
    V.n_terms = 71
    assert st(V) == -1
    with pytest.raises(ValueError):
        P.poly_potential([(0.1, (1, 0))] * 71, 2)
    need = ctypes.c_size_t(0)
    V = P.poly_potential([(0.5, (2, 0))], 2)
    assert lib.pimc_level_table_poly(ctypes.byref(V), 1.0, 1.0, 4, 0, None, 0, None, 0, ctypes.byref(need)) == -1
    assert need.value == 3                       # x_1^2, xbar_1^2 and the constant of W_{1,0}
    assert lib.pimc_level_table_poly(ctypes.byref(V), 1.0, 1.0, 4, 0, None, 0, None, 0, None) == -1


def test_radial_entry_points_validate_without_a_device():
    lib = P.load_library()
    a = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    b = (ctypes.c_double * 3)(1.0, 0.0, 0.0)
    out = (ctypes.c_double * 16)()
    for dim, coefs in ((0, (0, 0.5)), (5, (0, 0.5)), (2, (0, 0.5, 0.1))):
        V = P.binding.RadialPotential()
        V.dim = dim
        V.degree = len(coefs) - 1
        for n, c in enumerate(coefs):
            V.coef[n] = c
        st = lib.pimc_path_actions_radial(None, ctypes.byref(V), 1.0, a, b, 1.0, 16, 4, 1, 0, 0, 0, 1, out)
        assert st == -1
    V = P.radial_potential((0, 0.5, float("nan")), 2)
    assert lib.pimc_path_actions_radial(None, ctypes.byref(V), 1.0, a, b, 1.0, 16, 4, 1, 0, 0, 0, 1, out) == -1
    V = P.radial_potential((0, 0.5), 2)
    assert lib.pimc_path_actions_radial(None, ctypes.byref(V), 1.0, a, b, 1.0, 15, 4, 1, 0, 0, 0, 1, out) == -1
    V.degree = 3
    need = ctypes.c_size_t(0)
    assert lib.pimc_level_table_radial(ctypes.byref(V), 1.0, 1.0, 4, 0, None, 0, ctypes.byref(need), None, 0,
                                       None) == -1
    with pytest.raises(ValueError):
        P.radial_potential((0, 0.5, 0.1, 0.01), 2)
