"""O3/O4/O5 -- bisection paths, discretized level-p action and the Monte Carlo amplitude.

Test infrastructure only (see ``oracle/__init__``).

Sources (Sec. 4 of the paper):
* discretized amplitude A_N^(p) = int dq_1..dq_{N-1} (2 pi eps)^(-N/2) exp(-S_N^(p)) and the action
  eq.(SNp): S = sum_k [(q_{k+1}-q_k)^2/(2 eps) + eps W_p(x_k, xbar_k; eps)], q_0=a, q_N=b,
  x_k=(q_{k+1}+q_k)/2, xbar_k=(q_{k+1}-q_k)/2, eps=T/N;
* bisection (Sec. 4.1): N = 2^s; at level n = 1..s the points q[(1+2i) 2^(s-n)] for i=0..2^(n-1)-1 are
  a Gaussian offset eta_i plus the mean of q[i 2^(s-n+1)] and q[(i+1) 2^(s-n+1)]; the level-n
  trajectory is the subset q[i 2^(s-n)], so one level-s path gives every A_{2^n}, n = 0..s;
* output: amplitude and MC error (standard deviation of the mean) for every level; level 0 is the
  analytic N=1 amplitude with error 0.

Readings (the paper is silent or loose here):
* Offset width: the paper quotes sigma_n = sqrt(T/2^n). The conditional (Brownian-bridge) law of a
  midpoint of an interval of length T/2^(n-1) under the free measure exp(-sum (dq)^2/(2 eps)) has
  variance T/2^(n+1); with that width the kinetic term and all Gaussian normalizations integrate out
  exactly to the free kernel K_0(a,b;T) = (2 pi T)^(-1/2) exp(-(b-a)^2/(2T)), and
  A_N^(p) = K_0 * E[exp(-sum_k eps W_p)].  ``amplitude_literal_width`` implements the paper's quoted
  width with explicit kinetic term and proposal density instead; both estimate the same A_N^(p).
* Error: err = sqrt(s^2/n) with the unbiased sample variance s^2.
* Mass m != 1 (hbar = 1 always): A_m(a,b;T) = sqrt(m) A_1(sqrt(m) a, sqrt(m) b; T) with the
  potential V(y/sqrt(m)), i.e. polynomial coefficient j scaled by m^(-j/2).

Every function works on explicit path indices, so any subset of a run is reproducible.
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import Dict, List, Sequence

import numpy as np

from . import effective_action as ea
from .philox import node_normals


def free_kernel(a: float, b: float, T: float) -> float:
    """K_0(a,b;T) = (2 pi T)^(-1/2) exp(-(b-a)^2/(2T)): the W = 0 case of the ideal-action form (Sec. 2.1)."""
    return math.exp(-(b - a) ** 2 / (2.0 * T)) / math.sqrt(2.0 * math.pi * T)


def rescale_mass(V: ea.Poly, m, a: float, b: float):
    """(V~, a~, b~, prefactor) of the mass reading: coefficient j times m^(-j/2), endpoints times sqrt(m)."""
    m = Fraction(m)
    sm = math.sqrt(float(m))
    if m == 1:
        return V, a, b, 1.0
    # m^(-j/2) is irrational in general: take the FP64 value of sqrt(m) exactly as a rational.
    inv_sqrt = Fraction(1.0 / sm)
    Vt = ea._trim([c * inv_sqrt ** j for j, c in enumerate(V)])
    return Vt, a * sm, b * sm, sm


def bisection_paths(a: float, b: float, T: float, s: int, seed: int, stream: int, paths) -> np.ndarray:
    """Level-s trajectories q[0..N] (one row per path index), built level by level as in Sec. 4.1."""
    paths = np.asarray(paths, dtype=np.uint64)
    N = 1 << s
    q = np.zeros((paths.size, N + 1), dtype=np.float64)
    q[:, 0] = a
    q[:, N] = b
    for n in range(1, s + 1):
        sigma = math.sqrt(T / 2.0 ** (n + 1))
        step = 1 << (s - n)
        for i in range(1 << (n - 1)):
            h = (1 << (n - 1)) + i
            z = node_normals(seed, stream, paths, np.uint64(h))
            j = (2 * i + 1) * step
            q[:, j] = sigma * z + 0.5 * (q[:, j - step] + q[:, j + step])
    return q


def level_tables(V: ea.Poly, p: int, T: float, s: int) -> List[List[List[float]]]:
    """Per level n = 0..s: the FP64-rounded Q_k(x) with eps_n W_p = sum_k xbar^(2k) Q_k(x), eps_n = T/2^n."""
    Tf = Fraction(T)
    return [ea.xbar_groups_float(V, p, Tf / (1 << n)) for n in range(s + 1)]


def eps_W(tab: Sequence[Sequence[float]], x: np.ndarray, xbar: np.ndarray) -> np.ndarray:
    """eps W_p(x, xbar) = sum_k xbar^(2k) Q_k(x), each Q_k by Horner in x (FP64)."""
    xb2 = xbar * xbar
    total = np.zeros_like(x)
    pw = np.ones_like(x)
    for k, Q in enumerate(tab):
        val = np.zeros_like(x)
        for coef in reversed(Q):
            val = val * x + coef
        total = total + pw * val
        pw = pw * xb2
    return total


def level_actions(q: np.ndarray, s: int, tables) -> np.ndarray:
    """Potential part sum_k eps_n W_p(x_k, xbar_k; eps_n) of eq.(SNp) for every level n = 0..s.

    Returns shape (paths, s+1). The kinetic part is integrated out by the bridge sampling (see the
    module header), so it is not included.
    """
    out = np.zeros((q.shape[0], s + 1))
    for n in range(s + 1):
        sub = q[:, :: 1 << (s - n)]                 # the level-n trajectory q[i 2^(s-n)]
        x = 0.5 * (sub[:, 1:] + sub[:, :-1])
        xbar = 0.5 * (sub[:, 1:] - sub[:, :-1])
        out[:, n] = eps_W(tables[n], x, xbar).sum(axis=1)
    return out


def level_action_scales(q: np.ndarray, s: int, tables) -> np.ndarray:
    """sum_k |eps_n W_p(x_k, xbar_k)| per path and level: the natural scale of a level action, used to
    state a rounding tolerance that does not blow up when the action itself is near zero."""
    out = np.zeros((q.shape[0], s + 1))
    for n in range(s + 1):
        sub = q[:, :: 1 << (s - n)]
        x = 0.5 * (sub[:, 1:] + sub[:, :-1])
        xbar = 0.5 * (sub[:, 1:] - sub[:, :-1])
        out[:, n] = np.abs(eps_W(tables[n], x, xbar)).sum(axis=1)
    return out


def path_actions_and_scales(V, m, a, b, T, s, p, seed, stream, paths):
    """(level actions, level scales) for explicit path indices, after the mass rescaling."""
    Vt, at, bt, _ = rescale_mass(ea.poly(V) if not isinstance(V, tuple) else V, m, a, b)
    tabs = level_tables(Vt, p, T, s)
    q = bisection_paths(at, bt, T, s, seed, stream, paths)
    return level_actions(q, s, tabs), level_action_scales(q, s, tabs)


def path_actions(V, m, a, b, T, s, p, seed, stream, paths) -> np.ndarray:
    """Level actions (paths, s+1) after the mass rescaling, for explicit path indices."""
    Vt, at, bt, _ = rescale_mass(ea.poly(V) if not isinstance(V, tuple) else V, m, a, b)
    tabs = level_tables(Vt, p, T, s)
    q = bisection_paths(at, bt, T, s, seed, stream, paths)
    return level_actions(q, s, tabs)


def level0_amplitude(V, m, a, b, T, p) -> float:
    """N=1 amplitude: (2 pi T)^(-1/2) exp(-(b-a)^2/(2T) - T W_p((a+b)/2,(b-a)/2;T)), error 0 (Sec. 4.2)."""
    Vt, at, bt, pref = rescale_mass(ea.poly(V) if not isinstance(V, tuple) else V, m, a, b)
    tab = ea.xbar_groups_float(Vt, p, Fraction(T))
    x = np.array([0.5 * (at + bt)])
    xbar = np.array([0.5 * (bt - at)])
    return pref * free_kernel(at, bt, T) * math.exp(-float(eps_W(tab, x, xbar)[0]))


def _fsum_stats(w: np.ndarray):
    n = w.size
    mean = math.fsum(w) / n
    var = math.fsum((w - mean) ** 2) / (n - 1)
    return mean, var


def amplitude(V, m, a, b, T, s, p, n_samples, seed, stream, first_path=0, batch=4096) -> List[Dict]:
    """A_{2^n} and its MC error for every level n = 0..s from ``n_samples`` paths.

    Plain definition: A_n = K_0 * mean_i exp(-S_n(i)) (after the mass rescaling), err_n = K_0 *
    sqrt(var/n). Sums with math.fsum.  Returns one dict per level with amp, err, n, n_nonfinite,
    relvar and ess.
    """
    Vp = ea.poly(V) if not isinstance(V, tuple) else V
    Vt, at, bt, pref = rescale_mass(Vp, m, a, b)
    tabs = level_tables(Vt, p, T, s)
    K0 = free_kernel(at, bt, T) * pref
    ws = [[] for _ in range(s + 1)]
    for start in range(first_path, first_path + n_samples, batch):
        idx = np.arange(start, min(start + batch, first_path + n_samples), dtype=np.uint64)
        q = bisection_paths(at, bt, T, s, seed, stream, idx)
        S = level_actions(q, s, tabs)
        for n in range(s + 1):
            ws[n].append(np.exp(-S[:, n]))
    out = []
    for n in range(s + 1):
        w = np.concatenate(ws[n])
        nonfinite = int(np.count_nonzero(~np.isfinite(w)))
        if n == 0:
            amp0 = level0_amplitude(Vp, m, a, b, T, p)
            out.append(dict(amp=amp0, err=0.0, n=w.size, n_nonfinite=0, relvar=0.0, ess=float(w.size)))
            continue
        mean, var = _fsum_stats(w)
        sw = math.fsum(w)
        sw2 = math.fsum(w * w)
        out.append(dict(amp=K0 * mean, err=K0 * math.sqrt(var / w.size), n=w.size,
                        n_nonfinite=nonfinite, relvar=var / (mean * mean) if mean != 0 else math.inf,
                        ess=(sw * sw / sw2) if sw2 > 0 else 0.0))
    return out


def chunk_sums(V, m, a, b, T, s, p, seed, stream, first_path, count, shift) -> np.ndarray:
    """(n, sum d, sum d^2) per level over paths [first_path, first_path+count) with
    d = exp(-(S_n - shift_n)) - 1, summed with math.fsum. ``shift`` is a per-level array.

    This is the plain definition of the shifted per-chunk sums that the amplitude estimator merges;
    the shift changes only the rounding, not the estimate.
    """
    S = path_actions(V, m, a, b, T, s, p, seed, stream, np.arange(first_path, first_path + count, dtype=np.uint64))
    out = np.zeros((s + 1, 3))
    for n in range(s + 1):
        d = np.expm1(-(S[:, n] - shift[n]))
        out[n] = (count, math.fsum(d), math.fsum(d * d))
    return out


def straight_line_actions(V, m, a, b, T, s, p) -> np.ndarray:
    """Potential part of eq.(SNp) on the straight line q_k = a + (b-a) k/2^n for every level n."""
    Vp = ea.poly(V) if not isinstance(V, tuple) else V
    Vt, at, bt, _ = rescale_mass(Vp, m, a, b)
    tabs = level_tables(Vt, p, T, s)
    out = np.zeros(s + 1)
    for n in range(s + 1):
        k = np.arange((1 << n) + 1, dtype=np.float64)
        q = at + (bt - at) * k / (1 << n)
        x = 0.5 * (q[1:] + q[:-1])
        xbar = 0.5 * (q[1:] - q[:-1])
        out[n] = eps_W(tabs[n], x, xbar).sum()
    return out


def amplitude_literal_width(V, a, b, T, s, p, n_samples, seed, stream, first_path=0, batch=4096):
    """A_N^(p) at level s with the paper's quoted offset width sigma_n = sqrt(T/2^n) (Sec. 4.1).

    With a proposal that is not the exact bridge, the weight keeps the full integrand of the
    discretized amplitude divided by the proposal density:
      w = (2 pi eps)^(-N/2) exp(-S_N^(p)) / prod_h phi_{sigma_n}(eta_h).
    Same expectation as ``amplitude`` (a check of the kinetic-term cancellation); larger variance.
    Returns (amp, err).
    """
    Vp = ea.poly(V) if not isinstance(V, tuple) else V
    tabs = level_tables(Vp, p, T, s)
    N = 1 << s
    eps = T / N
    ws = []
    for start in range(first_path, first_path + n_samples, batch):
        idx = np.arange(start, min(start + batch, first_path + n_samples), dtype=np.uint64)
        q = np.zeros((idx.size, N + 1))
        q[:, 0] = a
        q[:, N] = b
        logprop = np.zeros(idx.size)
        for n in range(1, s + 1):
            sig = math.sqrt(T / 2.0 ** n)
            step = 1 << (s - n)
            for i in range(1 << (n - 1)):
                z = node_normals(seed, stream, idx, np.uint64((1 << (n - 1)) + i))
                j = (2 * i + 1) * step
                q[:, j] = sig * z + 0.5 * (q[:, j - step] + q[:, j + step])
                logprop += -0.5 * z * z - math.log(sig * math.sqrt(2 * math.pi))
        dq = q[:, 1:] - q[:, :-1]
        kin = (dq * dq).sum(axis=1) / (2 * eps)
        pot = eps_W(tabs[s], 0.5 * (q[:, 1:] + q[:, :-1]), 0.5 * dq).sum(axis=1)
        logw = -0.5 * N * math.log(2 * math.pi * eps) - kin - pot - logprop
        ws.append(np.exp(logw))
    w = np.concatenate(ws)
    mean, var = _fsum_stats(w)
    return mean, math.sqrt(var / w.size)
