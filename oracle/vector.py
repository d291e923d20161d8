"""O10 -- effective action of several coordinates (Sec. 2.2: many-body systems, eq.(MBrec), eq.(DIA)).

Test infrastructure only (see ``oracle/__init__``).

With d = D*M coordinates (D dimensions, M particles, no quantum statistics) the short-time amplitude
is (2 pi eps)^(-d/2) exp(-(2/eps) xbar.xbar - eps W(x, xbar; eps)) with the mid-point vector x and
the half-deviation vector xbar. W = sum_m sum_{k<=m} eps^(m-k) W_{m,k}(x, xbar), where W_{m,k} is the
full contraction of the coefficient tensor with 2k copies of xbar (homogeneous of degree 2k in xbar),
and the level-p potential keeps m <= p-1. eq.(DIA) gives W_{m,m} = (xbar.grad)^(2m) V / (2m+1)!;
eq.(MBrec) gives W_{m,k} for k = m-1, ..., 0 (Fig. 1 order) from the gradient and Laplacian in x and
in xbar, with the r-range max{0, k-m+l+2}..min{k, l} of the one-dimensional recursion.

Two exact routes (rational arithmetic):

* ``component_coefficients`` -- the definition: W_{m,k} as polynomials in the 2d components
  x_1..x_d, xbar_1..xbar_d, every derivative taken component by component. Any polynomial V.
* ``invariant_coefficients`` -- for a rotation-invariant V = sum_n a_n (x.x)^n: W_{m,k} as
  polynomials in the invariants u = x.x, w = x.xbar, z = xbar.xbar, with the chain-rule forms of
  the operators in d dimensions (f_u etc. are partial derivatives in the invariants):
      grad^2 f        = 2d f_u + 4u f_uu + 4w f_uw + z f_ww
      gradbar^2 f     = 2d f_z + 4z f_zz + 4w f_wz + u f_ww
      grad f.grad g   = 4u f_u g_u + 2w (f_u g_w + f_w g_u) + z f_w g_w
      gradbar f.gradbar g = u f_w g_w + 2w (f_w g_z + f_z g_w) + 4z f_z g_z
      xbar.grad f     = 2w f_u + z f_w
  (the "tables over rotational invariants"). In d = 1 the invariants are dependent (w^2 = uz);
  the polynomial is then one of several representatives of the same function.

Slice action at level n (eps = T/2^n), from the invariant route: every term of W_{m,k} is
u^i w^(2j) z^(k-j) (even in w: W is even in xbar), so
    eps W_p = sum_j (w^2)^j sum_{l} z^l Q_{j+l,j}(u),   Q_{k,j}(u) = sum_{m>=k} eps^(m-k+1) [W_{m,k}]_{j}(u)
with [W_{m,k}]_j the coefficient polynomial of w^(2j) z^(k-j).

Paths: the d coordinates are independent bisection bridges (the free measure factorizes); coordinate
c of heap node h uses the normal of generator call (h >> 1) + c * 2^20 (``philox.node_normals`` with
a pair offset), so coordinate 0 is the one-dimensional path of the same seed, stream and index.
Mass m: coordinates times sqrt(m), a_n times m^(-n), amplitude times m^(d/2) (as in one dimension).

Pins (tests/test_oracle_vector.py): eq.(eqWMB) holds exactly through order p-1 for the component
route (a polynomial check of the PDE with eps as a variable, not of the recursion); in d = 1 the
component route equals the one-dimensional coefficients xbar^(2k) c_{m,k}; a separable V = V1(x_1) +
V2(x_2) gives the sum of the one-dimensional effective potentials; the invariant route expanded in
components equals the component route (d = 2, 3); the d = 1 invariant route evaluates to the
one-dimensional slice action; the short-time amplitude of the 2D anharmonic oscillator converges in
p to a two-dimensional sinc-DVR continuum amplitude.
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache
from math import factorial
from typing import Dict, List, Sequence, Tuple

import numpy as np

from .philox import node_normals

CPoly = Dict[Tuple[int, ...], Fraction]     # exponents of x_1..x_d, xbar_1..xbar_d
IPoly = Dict[Tuple[int, int, int], Fraction]  # exponents of u, w, z
COORD_PAIR_STRIDE = 1 << 20


# ------------------------------------------------------------------------- polynomial helpers
def _add(a, b, s=1):
    out = dict(a)
    for k, v in b.items():
        out[k] = out.get(k, 0) + s * v
    return {k: v for k, v in out.items() if v != 0}


def _scale(a, s):
    return {k: v * s for k, v in a.items() if v * s != 0}


def _mul(a, b):
    out = {}
    for ka, va in a.items():
        for kb, vb in b.items():
            k = tuple(x + y for x, y in zip(ka, kb))
            out[k] = out.get(k, 0) + va * vb
    return {k: v for k, v in out.items() if v != 0}


def _der(a, var: int):
    out = {}
    for k, v in a.items():
        e = k[var]
        if e:
            nk = list(k)
            nk[var] -= 1
            t = tuple(nk)
            out[t] = out.get(t, 0) + v * e
    return {k: v for k, v in out.items() if v != 0}


def _shift(a, var: int, times: int = 1):
    """a times variable ``var`` to the power ``times``."""
    out = {}
    for k, v in a.items():
        nk = list(k)
        nk[var] += times
        out[tuple(nk)] = v
    return out


# ------------------------------------------------------------------------- component route
def radial_to_components(a: Sequence, d: int) -> CPoly:
    """V = sum_n a_n (x.x)^n as a polynomial in the components (xbar exponents zero)."""
    nv = 2 * d
    r2: CPoly = {}
    for i in range(d):
        e = [0] * nv
        e[i] = 2
        r2[tuple(e)] = Fraction(1)
    out: CPoly = {}
    pw: CPoly = {tuple([0] * nv): Fraction(1)}
    for n, an in enumerate(a):
        if n:
            pw = _mul(pw, r2)
        out = _add(out, _scale(pw, Fraction(an)))
    return out


def _lap(f: CPoly, d: int, off: int) -> CPoly:
    out: CPoly = {}
    for i in range(d):
        out = _add(out, _der(_der(f, off + i), off + i))
    return out


def _gdot(f: CPoly, g: CPoly, d: int, off: int) -> CPoly:
    out: CPoly = {}
    for i in range(d):
        out = _add(out, _mul(_der(f, off + i), _der(g, off + i)))
    return out


def _xbar_grad(f: CPoly, d: int) -> CPoly:
    out: CPoly = {}
    for i in range(d):
        out = _add(out, _shift(_der(f, i), d + i))
    return out


def component_coefficients(V: CPoly, d: int, p: int) -> Dict[Tuple[int, int], CPoly]:
    """W_{m,k} for 0 <= k <= m <= p-1 (eq.(DIA) on the diagonal, eq.(MBrec) for k = m-1..0)."""
    W: Dict[Tuple[int, int], CPoly] = {(0, 0): dict(V)}
    for m in range(1, p):
        t = dict(V)
        for _ in range(2 * m):
            t = _xbar_grad(t, d)
        W[(m, m)] = _scale(t, Fraction(1, factorial(2 * m + 1)))
        for k in range(m - 1, -1, -1):
            rhs = _add(_lap(W[(m - 1, k)], d, 0), _lap(W[(m, k + 1)], d, d))
            for l in range(0, m - 1):
                for r in range(max(0, k - m + l + 2), min(k, l) + 1):
                    rhs = _add(rhs, _gdot(W[(l, r)], W[(m - l - 2, k - r)], d, 0), -1)
            for l in range(1, m - 1):
                for r in range(max(0, k - m + l + 2), min(k, l) + 1):
                    rhs = _add(rhs, _gdot(W[(l, r)], W[(m - l - 1, k - r + 1)], d, d), -1)
            W[(m, k)] = _scale(rhs, Fraction(1, 8 * (m + k + 1)))
    return W


# ------------------------------------------------------------------------- invariant route
def _du(f):
    return _der(f, 0)


def _dw(f):
    return _der(f, 1)


def _dz(f):
    return _der(f, 2)


def inv_lap(f: IPoly, d: int) -> IPoly:
    fu, fw = _du(f), _dw(f)
    out = _scale(fu, 2 * d)
    out = _add(out, _shift(_scale(_du(fu), 4), 0))
    out = _add(out, _shift(_scale(_dw(fu), 4), 1))
    out = _add(out, _shift(_dw(fw), 2))
    return out


def inv_lapbar(f: IPoly, d: int) -> IPoly:
    fz, fw = _dz(f), _dw(f)
    out = _scale(fz, 2 * d)
    out = _add(out, _shift(_scale(_dz(fz), 4), 2))
    out = _add(out, _shift(_scale(_dz(fw), 4), 1))
    out = _add(out, _shift(_dw(fw), 0))
    return out


def inv_gdot(f: IPoly, g: IPoly) -> IPoly:
    fu, fw, gu, gw = _du(f), _dw(f), _du(g), _dw(g)
    out = _shift(_scale(_mul(fu, gu), 4), 0)
    out = _add(out, _shift(_scale(_add(_mul(fu, gw), _mul(fw, gu)), 2), 1))
    out = _add(out, _shift(_mul(fw, gw), 2))
    return out


def inv_gbdot(f: IPoly, g: IPoly) -> IPoly:
    fz, fw, gz, gw = _dz(f), _dw(f), _dz(g), _dw(g)
    out = _shift(_mul(fw, gw), 0)
    out = _add(out, _shift(_scale(_add(_mul(fw, gz), _mul(fz, gw)), 2), 1))
    out = _add(out, _shift(_scale(_mul(fz, gz), 4), 2))
    return out


def inv_xbar_grad(f: IPoly) -> IPoly:
    return _add(_shift(_scale(_du(f), 2), 1), _shift(_dw(f), 2))


@lru_cache(maxsize=32)
def _invariant_cached(a: Tuple[Fraction, ...], d: int, p: int):
    V: IPoly = {(n, 0, 0): an for n, an in enumerate(a) if an != 0}
    W: Dict[Tuple[int, int], IPoly] = {(0, 0): V}
    for m in range(1, p):
        t = dict(V)
        for _ in range(2 * m):
            t = inv_xbar_grad(t)
        W[(m, m)] = _scale(t, Fraction(1, factorial(2 * m + 1)))
        for k in range(m - 1, -1, -1):
            rhs = _add(inv_lap(W[(m - 1, k)], d), inv_lapbar(W[(m, k + 1)], d))
            for l in range(0, m - 1):
                for r in range(max(0, k - m + l + 2), min(k, l) + 1):
                    rhs = _add(rhs, inv_gdot(W[(l, r)], W[(m - l - 2, k - r)]), -1)
            for l in range(1, m - 1):
                for r in range(max(0, k - m + l + 2), min(k, l) + 1):
                    rhs = _add(rhs, inv_gbdot(W[(l, r)], W[(m - l - 1, k - r + 1)]), -1)
            W[(m, k)] = _scale(rhs, Fraction(1, 8 * (m + k + 1)))
    return tuple(sorted((key, tuple(sorted(poly.items()))) for key, poly in W.items()))


def invariant_coefficients(a: Sequence, d: int, p: int) -> Dict[Tuple[int, int], IPoly]:
    """W_{m,k}(u, w, z) for V = sum_n a_n u^n in d dimensions, exactly."""
    a = tuple(Fraction(x) for x in a)
    return {key: dict(poly) for key, poly in _invariant_cached(a, int(d), int(p))}


def invariants_to_components(f: IPoly, d: int) -> CPoly:
    """Expand u = x.x, w = x.xbar, z = xbar.xbar into components."""
    nv = 2 * d
    one = tuple([0] * nv)

    def mono(i, j):
        e = [0] * nv
        e[i] += 1
        e[j] += 1
        return tuple(e)

    u = {mono(i, i): Fraction(1) for i in range(d)}
    w = {mono(i, d + i): Fraction(1) for i in range(d)}
    z = {mono(d + i, d + i): Fraction(1) for i in range(d)}
    powers = {}

    def pw(base, name, e):
        key = (name, e)
        if key not in powers:
            r = {one: Fraction(1)}
            for _ in range(e):
                r = _mul(r, base)
            powers[key] = r
        return powers[key]

    out: CPoly = {}
    for (i, j, l), c in f.items():
        t = _mul(_mul(pw(u, "u", i), pw(w, "w", j)), pw(z, "z", l))
        out = _add(out, _scale(t, c))
    return out


# ------------------------------------------------------------------------- slice action
def rescale_mass(a: Sequence, m) -> Tuple[Fraction, ...]:
    """a_n m^(-n): V(y / sqrt(m)) for V = sum a_n (x.x)^n (exact for the FP64 value of m)."""
    mi = 1 / Fraction(m)
    return tuple(Fraction(x) * mi ** n for n, x in enumerate(a))


def level_groups(a: Sequence, d: int, p: int, eps) -> List[List[List[Fraction]]]:
    """Exact Q_{k,j}(u) coefficient lists, Q[k][j][i], for eps W_p (see the module header)."""
    eps = Fraction(eps)
    W = invariant_coefficients(a, d, p)
    Q = [[dict() for _ in range(k + 1)] for k in range(p)]
    for (m, k), poly in W.items():
        f = eps ** (m - k + 1)
        for (i, jw, lz), c in poly.items():
            if jw % 2 or jw // 2 + lz != k:
                raise ValueError("W_{m,k} is not of the form u^i w^(2j) z^(k-j)")
            j = jw // 2
            Q[k][j][i] = Q[k][j].get(i, 0) + c * f
    out = []
    for k in range(p):
        row = []
        for j in range(k + 1):
            q = Q[k][j]
            deg = max((i for i, c in q.items() if c != 0), default=-1)
            row.append([q.get(i, Fraction(0)) for i in range(deg + 1)])
        out.append(row)
    return out


def level_tables(a: Sequence, d: int, p: int, T: float, s: int):
    """Per level n = 0..s: FP64-rounded Q[k][j][i] at eps_n = T/2^n."""
    Tf = Fraction(T)
    return [[[[float(c) for c in q] for q in row] for row in level_groups(a, d, p, Tf / (1 << n))]
            for n in range(s + 1)]


def eps_W(tab, x: np.ndarray, xbar: np.ndarray) -> np.ndarray:
    """eps W_p = sum_{k,j} w^(2j) z^(k-j) Q_{k,j}(u) with u = x.x, w = x.xbar, z = xbar.xbar (last axis
    = coordinates), each Q by Horner in u (FP64)."""
    u = np.sum(x * x, axis=-1)
    w2 = np.sum(x * xbar, axis=-1) ** 2
    z = np.sum(xbar * xbar, axis=-1)
    total = np.zeros_like(u)
    for k, row in enumerate(tab):
        for j, q in enumerate(row):
            val = np.zeros_like(u)
            for c in reversed(q):
                val = val * u + c
            total = total + w2 ** j * z ** (k - j) * val
    return total


# ------------------------------------------------------------------------- paths and estimator
def bisection_paths(a: Sequence[float], b: Sequence[float], T: float, s: int, seed: int, stream: int,
                    paths) -> np.ndarray:
    """Level-s trajectories q[path, 0..N, coordinate] (Sec. 4.1 per coordinate; see the header)."""
    paths = np.asarray(paths, dtype=np.uint64)
    d = len(a)
    N = 1 << s
    q = np.zeros((paths.size, N + 1, d), dtype=np.float64)
    q[:, 0, :] = np.asarray(a, dtype=np.float64)
    q[:, N, :] = np.asarray(b, dtype=np.float64)
    for n in range(1, s + 1):
        sigma = math.sqrt(T / 2.0 ** (n + 1))
        step = 1 << (s - n)
        for i in range(1 << (n - 1)):
            h = (1 << (n - 1)) + i
            j = (2 * i + 1) * step
            for c in range(d):
                z = node_normals(seed, stream, paths, np.uint64(h), c * COORD_PAIR_STRIDE)
                q[:, j, c] = sigma * z + 0.5 * (q[:, j - step, c] + q[:, j + step, c])
    return q


def level_actions(q: np.ndarray, s: int, tables) -> np.ndarray:
    """sum over slices of eps_n W_p for every level n = 0..s (rows: paths)."""
    out = np.zeros((q.shape[0], s + 1))
    for n in range(s + 1):
        sub = q[:, :: 1 << (s - n), :]
        x = 0.5 * (sub[:, 1:, :] + sub[:, :-1, :])
        xbar = 0.5 * (sub[:, 1:, :] - sub[:, :-1, :])
        out[:, n] = eps_W(tables[n], x, xbar).sum(axis=1)
    return out


def _scaled(a, m, qa, qb):
    sm = math.sqrt(float(m))
    at = [x * sm for x in qa]
    bt = [x * sm for x in qb]
    return rescale_mass(a, m), at, bt, sm ** len(qa)


def path_actions(a, d, m, qa, qb, T, s, p, seed, stream, paths) -> np.ndarray:
    at_coefs, at, bt, _ = _scaled(a, m, qa, qb)
    tabs = level_tables(at_coefs, d, p, T, s)
    q = bisection_paths(at, bt, T, s, seed, stream, paths)
    return level_actions(q, s, tabs)


def free_kernel(qa, qb, T) -> float:
    d = len(qa)
    r2 = sum((y - x) ** 2 for x, y in zip(qa, qb))
    return math.exp(-r2 / (2.0 * T)) / (2.0 * math.pi * T) ** (d / 2.0)


def short_time_amplitude(a, d, m, qa, qb, t, p) -> float:
    """A_1^(p)(qa, qb; t) = m^(d/2) (2 pi t)^(-d/2) exp(-|b-a|^2/(2t) - t W_p(x, xbar; t)) (scaled)."""
    coefs, at, bt, pref = _scaled(a, m, qa, qb)
    tab = level_tables(coefs, d, p, t, 0)[0]
    x = 0.5 * (np.asarray(at) + np.asarray(bt))
    xb = 0.5 * (np.asarray(bt) - np.asarray(at))
    return pref * free_kernel(at, bt, t) * math.exp(-float(eps_W(tab, x[None, :], xb[None, :])[0]))


def amplitude(a, d, m, qa, qb, T, s, p, n_samples, seed, stream, batch=2048) -> List[Dict]:
    """A_{2^n} and its MC error per level n = 0..s: K_0 mean exp(-S_n), err K_0 sqrt(var/n) (fsum)."""
    coefs, at, bt, pref = _scaled(a, m, qa, qb)
    tabs = level_tables(coefs, d, p, T, s)
    K0 = pref * free_kernel(at, bt, T)
    ws = [[] for _ in range(s + 1)]
    for start in range(0, n_samples, batch):
        idx = np.arange(start, min(start + batch, n_samples), dtype=np.uint64)
        S = level_actions(bisection_paths(at, bt, T, s, seed, stream, idx), s, tabs)
        for n in range(s + 1):
            ws[n].append(np.exp(-S[:, n]))
    out = []
    for n in range(s + 1):
        w = np.concatenate(ws[n])
        if n == 0:
            out.append(dict(amp=short_time_amplitude(a, d, m, qa, qb, T, p), err=0.0))
            continue
        mean = math.fsum(w) / w.size
        var = math.fsum((w - mean) ** 2) / (w.size - 1)
        out.append(dict(amp=K0 * mean, err=K0 * math.sqrt(var / w.size)))
    return out


# ------------------------------------------------------------------------- any polynomial V (components)
def terms_to_components(terms, d: int, m=1.0) -> CPoly:
    """V(q) = sum coef q_1^e_1 .. q_d^e_d from ``terms`` = [(coef, (e_1, .., e_d))], after the mass
    rescaling V(y / sqrt m): each coefficient times m^(-total degree / 2), rounded to FP64 as the
    library does (an irrational factor for odd degree)."""
    out: CPoly = {}
    for c, e in terms:
        e = tuple(int(x) for x in e) + (0,) * (d - len(e))
        deg = sum(e)
        k = e[:d] + (0,) * d
        out[k] = out.get(k, 0) + Fraction(float(c) * float(m) ** (-0.5 * deg))
    return {k: v for k, v in out.items() if v != 0}


@lru_cache(maxsize=16)
def _component_cached(V: Tuple, d: int, p: int):
    W = component_coefficients(dict(V), d, p)
    return tuple(sorted((key, tuple(sorted(poly.items()))) for key, poly in W.items()))


def component_level_terms(V: CPoly, d: int, p: int, eps) -> CPoly:
    """eps W_p = sum_{k <= m < p} eps^(m-k+1) W_{m,k} as one exact polynomial in the components."""
    eps = Fraction(eps)
    out: CPoly = {}
    for (m, k), poly in _component_cached(tuple(sorted(V.items())), int(d), int(p)):
        out = _add(out, _scale(dict(poly), eps ** (m - k + 1)))
    return out


def component_tables(V: CPoly, d: int, p: int, T: float, s: int):
    """Per level n = 0..s: (exponent array [terms, 2d], FP64 coefficients) of eps_n W_p, eps_n = T/2^n."""
    out = []
    for n in range(s + 1):
        f = component_level_terms(V, d, p, Fraction(T) / (1 << n))
        keys = sorted(f)
        out.append((np.array(keys, dtype=np.int64).reshape(len(keys), 2 * d),
                    np.array([float(f[k]) for k in keys], dtype=np.float64)))
    return out


def _component_terms(tab, x: np.ndarray, xbar: np.ndarray):
    """Each term c_t prod_i x_i^e_ti xbar_i^e_t(d+i) (last axis = coordinates), in table order (FP64;
    the powers of each variable are tabulated once)."""
    exps, coef = tab
    y = np.concatenate([x, xbar], axis=-1)
    top = int(exps.max()) if exps.size else 0
    pw = [[np.ones(y.shape[:-1])] for _ in range(y.shape[-1])]
    for v in range(y.shape[-1]):
        for _ in range(top):
            pw[v].append(pw[v][-1] * y[..., v])
    for e, c in zip(exps, coef):
        t = np.full(y.shape[:-1], c)
        for v, ev in enumerate(e):
            if ev:
                t = t * pw[v][ev]
        yield t


def component_eps_W(tab, x: np.ndarray, xbar: np.ndarray) -> np.ndarray:
    """sum_t c_t prod_i x_i^e_ti xbar_i^e_t(d+i), term by term (FP64)."""
    total = np.zeros(np.broadcast_shapes(x.shape, xbar.shape)[:-1])
    for t in _component_terms(tab, x, xbar):
        total = total + t
    return total


def component_eps_W_abs(tab, x: np.ndarray, xbar: np.ndarray) -> np.ndarray:
    """sum_t |c_t prod_i x_i^e_ti xbar_i^e_t(d+i)|: the scale of the rounding error of any order of
    summation of the terms."""
    total = np.zeros(np.broadcast_shapes(x.shape, xbar.shape)[:-1])
    for t in _component_terms(tab, x, xbar):
        total = total + np.abs(t)
    return total


def _component_level_sums(q: np.ndarray, s: int, tables):
    """Per path and level: (sum over slices of eps_n W_p, sum over slices of the absolute terms)."""
    S = np.zeros((q.shape[0], s + 1))
    A = np.zeros((q.shape[0], s + 1))
    for n in range(s + 1):
        sub = q[:, :: 1 << (s - n), :]
        x = 0.5 * (sub[:, 1:, :] + sub[:, :-1, :])
        xbar = 0.5 * (sub[:, 1:, :] - sub[:, :-1, :])
        tot = np.zeros(x.shape[:-1])
        ab = np.zeros(x.shape[:-1])
        for t in _component_terms(tables[n], x, xbar):
            tot = tot + t
            ab = ab + np.abs(t)
        S[:, n] = tot.sum(axis=1)
        A[:, n] = ab.sum(axis=1)
    return S, A


def poly_path_actions(terms, d, m, qa, qb, T, s, p, seed, stream, paths, with_scale=False):
    """Level actions [path, n] of the level-s paths for any polynomial V (component route); with
    ``with_scale`` also the sums of the absolute monomial terms (the rounding-error scale)."""
    sm = math.sqrt(float(m))
    V = terms_to_components(terms, d, m)
    tabs = component_tables(V, d, p, T, s)
    q = bisection_paths([x * sm for x in qa], [x * sm for x in qb], T, s, seed, stream, paths)
    S, A = _component_level_sums(q, s, tabs)
    return (S, A) if with_scale else S


def poly_amplitude(terms, d, m, qa, qb, T, s, p, n_samples, seed, stream, batch=2048) -> List[Dict]:
    """A_{2^n} and its MC error per level n = 0..s for any polynomial V (as ``amplitude``)."""
    sm = math.sqrt(float(m))
    at, bt = [x * sm for x in qa], [x * sm for x in qb]
    V = terms_to_components(terms, d, m)
    tabs = component_tables(V, d, p, T, s)
    K0 = sm ** d * free_kernel(at, bt, T)
    ws = [[] for _ in range(s + 1)]
    for start in range(0, n_samples, batch):
        idx = np.arange(start, min(start + batch, n_samples), dtype=np.uint64)
        S, _ = _component_level_sums(bisection_paths(at, bt, T, s, seed, stream, idx), s, tabs)
        for n in range(s + 1):
            ws[n].append(np.exp(-S[:, n]))
    out = []
    for n in range(s + 1):
        w = np.concatenate(ws[n])
        if n == 0:
            out.append(dict(amp=K0 * float(w[0]), err=0.0))
            continue
        mean = math.fsum(w) / w.size
        var = math.fsum((w - mean) ** 2) / (w.size - 1)
        out.append(dict(amp=K0 * mean, err=K0 * math.sqrt(var / w.size)))
    return out


# ------------------------------------------------------------------------- continuum reference
def dvr_amplitude_2d(V, qa, qb, T, L=6.0, h=0.2) -> float:
    """<b| exp(-T H) |a> for H = -(1/2) grad^2 + V(x, y) from a tensor-product sinc-DVR (Colbert and
    Miller, J. Chem. Phys. 96, 1982 (1992)) on the grid i h, |i h| <= L; a and b on the grid."""
    M = int(round(L / h))
    g = h * np.arange(-M, M + 1)
    n = g.size
    i = np.arange(n)
    diff = i[:, None] - i[None, :]
    with np.errstate(divide="ignore"):
        K1 = np.where(diff == 0, math.pi ** 2 / 3.0, 2.0 * (-1.0) ** np.abs(diff) / np.where(diff == 0, 1, diff) ** 2)
    K1 = K1 / (2 * h * h)
    X, Y = np.meshgrid(g, g, indexing="ij")
    H = np.kron(K1, np.eye(n)) + np.kron(np.eye(n), K1) + np.diag(V(X, Y).ravel())
    E, vecs = np.linalg.eigh(H)

    def idx(q):
        ix = int(np.argmin(np.abs(g - q[0])))
        iy = int(np.argmin(np.abs(g - q[1])))
        if abs(g[ix] - q[0]) > 1e-9 or abs(g[iy] - q[1]) > 1e-9:
            raise ValueError("endpoints must lie on the DVR grid")
        return ix * n + iy

    ia, ib = idx(qa), idx(qb)
    w = np.exp(-T * (E - E[0]))
    return float(math.exp(-T * E[0]) * np.sum(vecs[ia] * vecs[ib] * w) / (h * h))


def aho2d(A, g):
    """Coefficients a_n of V = (A/2) r^2 + (g/24) r^4 in u = r^2 (the paper's 2D anharmonic oscillator)."""
    return (Fraction(0), Fraction(A) / 2, Fraction(g) / 24)
