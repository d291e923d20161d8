"""O6 -- affine-coupling proposal over the bisection normals (the learned proposal), FP64.

Test infrastructure only (see ``oracle/__init__``).

The paper samples the bisection offsets from their exact Gaussian law (Sec. 4.1). A proposal q
for the standard normals z of the bisection (heap nodes h = 1..D, D = N-1) reweights exactly:
A_N^(p) = K_0 E_phi[exp(-sum eps W_p)] = K_0 E_q[w], with log w = -(S(z) - S_ref) + log phi(z) -
log q(z). q is the push-forward of u ~ N(0, I_D) through L affine couplings, so log q(z) =
log phi(u) - log det, and log w = -(S(z) - S_ref) - |z|^2/2 + |u|^2/2 + log det.

Specification (shared by the GPU kernels):
* layer c uses mask type c mod 4 over the heap nodes: 0: A = {1} + left subtree of node 1,
  B = right subtree; 1: A = {1} + right subtree, B = left subtree; 2: A = odd h, B = even h;
  3: A = even h, B = odd h. A and B are listed in increasing h; |A|, |B| <= 64.
* MLP: xa = x[A] padded with zeros to 64; pre = W1 xa + b1 (W1: 128 x 64); h = silu(pre);
  o = W2 h + b2 (W2: 128 x 128); s_hat = o[0:|B|], t = o[64:64+|B|]; s = 2 tanh(s_hat/2);
  y[B] = x[B] exp(s) + t, y[A] = x[A]; log det += sum s.
* GPU precision (mirrored by ``quantize=True``): xa, W1, h, W2 rounded to bfloat16 (round to
  nearest even) before the products, products accumulated in FP32 (here FP64), biases FP32, s and
  t from FP32 values, the affine update, log det, action and weights in FP64.
* Training objective: L = log mean_i exp(2 l_i) (the log second moment of the weights; its
  minimizer minimizes the variance since E_q[w] is fixed), optionally mixed with the reverse KL
  -mean_i l_i: dL = sum_i alpha_i dl_i with alpha = (1-beta) 2 softmax(2 l) - beta/B.

Parameters are one flat float vector per layer: W1 (128*64, row-major [hidden][in]), b1 (128),
W2 (128*128, row-major [out][hidden]), b2 (128).

Pins (tests/test_oracle_flow.py): analytic gradient vs central finite differences of the FP64
loss; zero last layer = identity (weights equal the plain estimator's); inverse(forward(u)) = u;
on V = 0 a random flow gives mean w = 1 within MC error; the log-det equals log|det J| of a
finite-difference Jacobian.
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np

from . import pimc as opimc
from .philox import node_normals

H = 128
KIN = 64
NPARAM = H * KIN + H + H * H + H        # 24832 per layer


# ----------------------------------------------------------------------------- masks
def _subtree_side(h: int) -> int:
    """0 for the left subtree of node 1, 1 for the right one, -1 for node 1."""
    if h == 1:
        return -1
    return (h >> (h.bit_length() - 2)) & 1


def masks(D: int, layer: int) -> Tuple[List[int], List[int]]:
    """(A, B) heap-node lists of a layer (nodes 1..D, increasing)."""
    t = layer % 4
    nodes = range(1, D + 1)
    if t == 0:
        A = [h for h in nodes if _subtree_side(h) <= 0]
    elif t == 1:
        A = [h for h in nodes if _subtree_side(h) != 0]
    elif t == 2:
        A = [h for h in nodes if h % 2 == 1]
    else:
        A = [h for h in nodes if h % 2 == 0]
    B = [h for h in nodes if h not in set(A)]
    return A, B


# ----------------------------------------------------------------------------- bf16
def bf16(x):
    """Round FP64 values to bfloat16 (via FP32, round to nearest even at both steps as the GPU's
    conversion from FP32 does) and return them as FP64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    nan = np.isnan(f)
    out = (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, out)


def split(theta_layer: np.ndarray):
    o = 0
    W1 = theta_layer[o:o + H * KIN].reshape(H, KIN); o += H * KIN
    b1 = theta_layer[o:o + H]; o += H
    W2 = theta_layer[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta_layer[o:o + H]
    return W1, b1, W2, b2


def silu(v):
    return v / (1.0 + np.exp(-v))


# ----------------------------------------------------------------------------- forward
def coupling_forward(theta_layer, x, layer, D, quantize=True):
    """One coupling on x (paths x D, FP64). Returns y, s (per path x |B|), cache for backward."""
    A, B = masks(D, layer)
    ia = np.array(A, dtype=np.int64) - 1
    ib = np.array(B, dtype=np.int64) - 1
    W1, b1, W2, b2 = split(np.asarray(theta_layer, dtype=np.float64))
    xa = np.zeros((x.shape[0], KIN))
    xa[:, :len(A)] = x[:, ia]
    q = bf16 if quantize else (lambda v: v)
    xa_q, W1_q, W2_q = q(xa), q(W1), q(W2)
    pre = xa_q @ W1_q.T + b1
    h = silu(pre)
    h_q = q(h)
    o = h_q @ W2_q.T + b2
    nb = len(B)
    s_hat = o[:, :nb]
    t = o[:, 64:64 + nb]
    s = 2.0 * np.tanh(s_hat / 2.0)
    y = x.copy()
    y[:, ib] = x[:, ib] * np.exp(s) + t
    cache = dict(ia=ia, ib=ib, xa_q=xa_q, W1_q=W1_q, W2_q=W2_q, pre=pre, h_q=h_q, s_hat=s_hat, s=s, t=t, x=x)
    return y, s, cache


def flow_forward(theta, u, D, quantize=True):
    """z = f(u) through all layers; returns z, log det (per path), caches."""
    x = np.asarray(u, dtype=np.float64)
    logdet = np.zeros(x.shape[0])
    caches = []
    for c in range(len(theta)):
        x, s, cache = coupling_forward(theta[c], x, c, D, quantize)
        logdet = logdet + s.sum(axis=1)
        caches.append(cache)
    return x, logdet, caches


def flow_inverse(theta, z, D, quantize=True):
    """u = f^-1(z): layers in reverse, x[B] = (y[B] - t) exp(-s) with s, t from y[A] = x[A]."""
    y = np.asarray(z, dtype=np.float64)
    for c in range(len(theta) - 1, -1, -1):
        _, s, cache = coupling_forward(theta[c], y, c, D, quantize)   # s, t depend on y[A] = x[A] only
        x = y.copy()
        x[:, cache["ib"]] = (y[:, cache["ib"]] - cache["t"]) * np.exp(-s)
        y = x
    return y


# ----------------------------------------------------------------------------- action and weights
def action_and_grad(z, V, m, a, b, T, s, p):
    """Level-s action S(z) of the bisection path built from normals z (paths x D), and dS/dz.

    The path is linear in z (Sec. 4.1 bisection with sigma_n^2 = T/2^(n+1)); the gradient is the
    adjoint of that linear map applied to dS/dq, with dS/dq from the slice polynomials.
    """
    from . import effective_action as ea
    Vp = ea.poly(V) if not isinstance(V, tuple) else V
    Vt, at, bt, _ = opimc.rescale_mass(Vp, m, a, b)
    tab = opimc.level_tables(Vt, p, T, s)[s]
    N = 1 << s
    P = z.shape[0]
    q = np.zeros((P, N + 1))
    q[:, 0] = at
    q[:, N] = bt
    order = []
    for n in range(1, s + 1):
        sig = math.sqrt(T / 2.0 ** (n + 1))
        step = 1 << (s - n)
        for i in range(1 << (n - 1)):
            h = (1 << (n - 1)) + i
            j = (2 * i + 1) * step
            q[:, j] = sig * z[:, h - 1] + 0.5 * (q[:, j - step] + q[:, j + step])
            order.append((h, j, step, sig))
    x = 0.5 * (q[:, 1:] + q[:, :-1])
    xb = 0.5 * (q[:, 1:] - q[:, :-1])
    S = opimc.eps_W(tab, x, xb).sum(axis=1)
    # d(eps W)/dx and d(eps W)/dxbar of each slice, from the same FP64 polynomials
    dx = np.zeros_like(x)
    dxb = np.zeros_like(x)
    xb2 = xb * xb
    pw = np.ones_like(x)
    for k, Q in enumerate(tab):
        val = np.zeros_like(x)
        der = np.zeros_like(x)
        for coef in reversed(Q):
            der = der * x + val
            val = val * x + coef
        dx = dx + pw * der
        if k > 0:
            dxb = dxb + 2 * k * xb ** (2 * k - 1) * val
        pw = pw * xb2
    gq = np.zeros_like(q)
    gq[:, :-1] += 0.5 * dx - 0.5 * dxb          # slice k: x = (q_k+q_{k+1})/2, xbar = (q_{k+1}-q_k)/2
    gq[:, 1:] += 0.5 * dx + 0.5 * dxb
    gz = np.zeros_like(z)
    for (h, j, step, sig) in reversed(order):
        gz[:, h - 1] = sig * gq[:, j]
        gq[:, j - step] += 0.5 * gq[:, j]
        gq[:, j + step] += 0.5 * gq[:, j]
    return S, gz


def log_weights(theta, u, V, m, a, b, T, s, p, shift, quantize=True):
    """log w per path and (z, logdet, caches)."""
    D = (1 << s) - 1
    z, logdet, caches = flow_forward(theta, u, D, quantize)
    S, _ = action_and_grad(z, V, m, a, b, T, s, p)
    l = -(S - shift) - 0.5 * (z * z).sum(axis=1) + 0.5 * (u * u).sum(axis=1) + logdet
    return l, z, logdet, caches


def loss_weights(l, beta=0.0):
    """(loss, alpha): L = (1-beta) log mean exp(2l) + beta * (-mean l), alpha_i = dL/dl_i."""
    B = l.size
    mx = np.max(2 * l)
    e = np.exp(2 * l - mx)
    se = math.fsum(e)
    L2 = mx + math.log(se / B)
    alpha = (1 - beta) * 2 * e / se - beta / B
    return (1 - beta) * L2 + beta * (-math.fsum(l) / B), alpha


# ----------------------------------------------------------------------------- backward
def flow_loss_and_grad(theta, u, V, m, a, b, T, s, p, shift, beta=0.0, quantize=True):
    """Loss and dL/dtheta (list of flat per-layer arrays, FP64), analytic reverse mode.

    With quantize=True the products use the same bfloat16 operands as the GPU backward: g_o and
    g_pre are rounded to bfloat16 where they enter a product, W1, W2, xa and h as in the forward.
    """
    D = (1 << s) - 1
    l, z, logdet, caches = log_weights(theta, u, V, m, a, b, T, s, p, shift, quantize)
    loss, alpha = loss_weights(l, beta)
    _, gS = action_and_grad(z, V, m, a, b, T, s, p)
    g = alpha[:, None] * (-gS - z)                 # d(alpha . l)/dz
    q = bf16 if quantize else (lambda v: v)
    grads = [None] * len(theta)
    for c in range(len(theta) - 1, -1, -1):
        C = caches[c]
        ia, ib = C["ia"], C["ib"]
        nb = len(ib)
        x = C["x"]
        es = np.exp(C["s"])
        gyB = g[:, ib]
        gx = g.copy()
        gx[:, ib] = gyB * es
        gs = gyB * x[:, ib] * es + alpha[:, None]
        gsh = gs * (1.0 - np.tanh(C["s_hat"] / 2.0) ** 2)
        go = np.zeros((x.shape[0], H))
        go[:, :nb] = gsh
        go[:, 64:64 + nb] = gyB
        go_q = q(go)
        gh = go_q @ C["W2_q"]                         # [paths, hidden]
        pre = C["pre"]
        sig = 1.0 / (1.0 + np.exp(-pre))
        gpre = gh * (sig * (1.0 + pre * (1.0 - sig)))
        gpre_q = q(gpre)
        gxa = gpre_q @ C["W1_q"]                      # [paths, 64]
        gx[:, ia] += gxa[:, :len(ia)]
        gW2 = go_q.T @ C["h_q"]
        gb2 = go.sum(axis=0)
        gW1 = gpre_q.T @ C["xa_q"]
        gb1 = gpre.sum(axis=0)
        grads[c] = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2])
        g = gx
    return loss, grads, l


def base_normals(seed, stream, paths, D):
    """u (paths x D): the bisection normals z_h of the plain sampler, h = 1..D."""
    paths = np.asarray(paths, dtype=np.uint64)
    return np.stack([node_normals(seed, stream, paths, np.uint64(h)) for h in range(1, D + 1)], axis=1)


def init_params(L, seed, scale=1.0):
    """Random W1 ~ U(-1/8, 1/8) (1/sqrt(64)), b1 = 0, W2 = b2 = 0 times `scale` (0: identity)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(L):
        th = np.zeros(NPARAM)
        th[:H * KIN] = rng.uniform(-0.125, 0.125, H * KIN)
        th[H * KIN + H:H * KIN + H + H * H] = scale * rng.uniform(-0.05, 0.05, H * H)
        out.append(th)
    return out
