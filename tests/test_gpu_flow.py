"""GPU parity of the learned proposal (affine couplings over the bisection normals) against the
oracle (oracle/flow.py, quantize=True: the same bfloat16 operands as the matrix cores).

Tolerances, from the arithmetic:
* Products of bfloat16 operands are exact in FP32; the only differences from the oracle (FP64
  accumulation of the same products) are the FP32 accumulation (relative ~K * 2^-24 of the sum of
  |terms|, K <= 128) and, where that moves a hidden activation across a bfloat16 rounding boundary,
  one bfloat16 ulp (2^-8 relative) of that activation. The first gives |delta| ~1e-5 on z and log w
  after 8 layers; the second happens for a few per cent of paths and moves them by up to ~1e-3.
  So: at least 95 % of paths within 1e-4 (a wrong index, mask, transpose or sign moves every path
  by O(1)), every path within 5e-2.
* Gradients (sums over paths of the same quantities, FP32 backward): against the oracle's FP64
  reverse mode on the same operands, each block of a layer (W1, b1, W2, b2) and the whole layer in
  relative L2. The bounds are twice the worst measured over the cases below at N = 8, 16 and 128,
  batches 200 and 4096 (measured worst: W1 2.7e-3, b1 2.0e-3, W2 2.0e-3, b2 7.4e-4, layer 2.0e-3,
  1 - cosine 1.9e-6); the bf16 boundary crossings above set their size (a few 1e-3), and a wrong
  bias row, transpose or path weight gives O(1).
* Identity map (W2 = b2 = 0): s = t = 0 exactly, so log w is the plain estimator's -(S - S_ref)
  up to the FP64 action (relative 1e-12 of the action scale).
"""
import math
import sys

import numpy as np
import pytest

import paper_1105_0542_amd as P
from oracle import effective_action as ea
from oracle import flow as oflow
from oracle import pimc as opimc

pytestmark = pytest.mark.gpu

QUARTIC = P.quartic(1.0, 10.0)
# one layer's parameters (include/pimc.h): W1 [128][64], b1 [128], W2 [128][128], b2 [128]
OFF_B1 = 128 * 64
OFF_W2 = OFF_B1 + 128
OFF_B2 = OFF_W2 + 128 * 128
NP = P.binding.FLOW_NPARAM
assert OFF_B2 + 128 == NP
ODD = [0.0, 0.3, 0.5, 0.1, 0.05]


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _exact_poly(coefs):
    from fractions import Fraction
    return ea.poly([Fraction(c) for c in coefs])


@pytest.fixture(scope="module")
def ctx():
    c = P.Context()
    yield c
    c.close()


def _random_params(L, seed, w2=0.05):
    rng = np.random.default_rng(seed)
    th = np.zeros((L, P.FLOW_NPARAM), dtype=np.float32)
    H, K = 128, 64
    for c in range(L):
        th[c, :H * K] = rng.uniform(-0.125, 0.125, H * K)
        th[c, H * K:H * K + H] = rng.uniform(-0.1, 0.1, H)
        th[c, H * K + H:H * K + H + H * H] = rng.uniform(-w2, w2, H * H)
        th[c, -H:] = rng.uniform(-0.05, 0.05, H)
    return th


def _oracle_theta(th):
    return [np.asarray(t, dtype=np.float64) for t in th]


def _near(got, ref, bulk=1e-4, worst=5e-2, frac=0.95):
    d = np.abs(np.asarray(got) - np.asarray(ref))
    if d.ndim > 1:
        d = d.max(axis=1)
    assert np.all(np.isfinite(d))
    assert np.mean(d <= bulk) >= frac, (np.mean(d <= bulk), np.sort(d)[-5:])
    assert d.max() <= worst, d.max()


CASES = [  # coefs, m, a, b, T, s, p, layers, paths
    (QUARTIC, 1.0, 0.0, 1.0, 2.0, 3, 8, 4, 300),
    (QUARTIC, 1.0, 0.0, 1.0, 2.0, 7, 12, 8, 4096 + 37),
    (ODD, 1.5, -0.5, 0.7, 1.0, 4, 6, 5, 130),
    (QUARTIC, 1.0, 0.2, -0.3, 0.5, 1, 4, 4, 70),       # N = 2: only mask type 3 transforms node 1
]


@pytest.mark.parametrize("case", CASES)
def test_forward_matches_oracle(ctx, case):
    coefs, m, a, b, T, s, p, L, k = case
    _log(f"flow forward coefs={coefs} m={m} a={a} b={b} T={T} s={s} p={p} L={L} paths={k}")
    f = P.Flow(ctx, coefs, m, a, b, T, 1 << s, p, layers=L, batch=64)
    th = _random_params(L, 11 + s)
    f.set_params(th)
    assert np.array_equal(f.get_params(), th)
    seed, stream, first = 7, 3, 1000
    ell, logdet, z = f.log_weights(seed, stream, first, k, want_z=True)
    D = (1 << s) - 1
    u = oflow.base_normals(seed, stream, np.arange(first, first + k), D)
    shift = opimc.straight_line_actions(_exact_poly(coefs), m, a, b, T, s, p)[s]
    l_ref, z_ref, ld_ref, _ = oflow.log_weights(_oracle_theta(th), u, _exact_poly(coefs), m, a, b, T, s, p, shift)
    _near(z, z_ref)
    _near(logdet, ld_ref)
    _near(ell, l_ref)
    assert np.max(np.abs(z - u)) > 1e-2                 # the map is not the identity
    f.close()


@pytest.mark.parametrize("case", CASES[:3])
def test_identity_map_is_the_plain_estimator(ctx, case):
    coefs, m, a, b, T, s, p, L, k = case
    _log(f"flow identity coefs={coefs} s={s} p={p} paths={k}")
    f = P.Flow(ctx, coefs, m, a, b, T, 1 << s, p, layers=L, batch=64, init_scale=0.0)
    ell, logdet, z = f.log_weights(5, 1, 0, k, want_z=True)
    u = ctx.normals(5, 1, 0, k, (1 << s) - 1)           # the plain sampler's normals, same bits
    assert np.array_equal(z, u) and np.all(logdet == 0.0)
    S = ctx.path_actions(coefs, m, a, b, T, 1 << s, p, 5, 1, 0, 0, k)[:, s]
    shift = opimc.straight_line_actions(_exact_poly(coefs), m, a, b, T, s, p)[s]
    assert np.allclose(ell, -(S - shift), rtol=0, atol=1e-12 * max(1.0, np.abs(S).max()))
    # and the estimate on the same paths is the plain one
    n = 50000
    r_plain, _ = ctx.amplitude(coefs, m, a, b, T, 1 << s, p, n, 5, 1)
    r_flow, _, _ = f.amplitude(n, 5, 1)
    assert r_flow.amp == pytest.approx(r_plain[s].amp, rel=1e-11)
    assert r_flow.err == pytest.approx(r_plain[s].err, rel=1e-8)
    f.close()


GRAD_BOUNDS = {"W1": 5.5e-3, "b1": 4e-3, "W2": 4e-3, "b2": 1.5e-3}


@pytest.mark.parametrize("beta", [0.0, 0.5])
@pytest.mark.parametrize("case", [CASES[0], CASES[2], CASES[1]])
def test_gradient_matches_oracle(ctx, case, beta):
    coefs, m, a, b, T, s, p, L, _ = case
    B = 200 if s < 7 else 4096
    _log(f"flow gradient coefs={coefs} s={s} p={p} L={L} batch={B} beta={beta}")
    f = P.Flow(ctx, coefs, m, a, b, T, 1 << s, p, layers=L, batch=B, beta=beta)
    th = _random_params(L, 21 + s)
    f.set_params(th)
    seed, stream = 9, 2**31 + 4
    loss, ell, g = f.grad(seed, stream)
    u = oflow.base_normals(seed, stream, np.arange(B), (1 << s) - 1)
    shift = opimc.straight_line_actions(_exact_poly(coefs), m, a, b, T, s, p)[s]
    loss_ref, g_ref, l_ref = oflow.flow_loss_and_grad(_oracle_theta(th), u, _exact_poly(coefs), m, a, b, T, s, p,
                                                      shift, beta, quantize=True)
    _near(ell, l_ref)
    assert loss == pytest.approx(loss_ref, rel=1e-3, abs=1e-4)
    blocks = {"W1": slice(0, OFF_B1), "b1": slice(OFF_B1, OFF_W2), "W2": slice(OFF_W2, OFF_B2), "b2": slice(OFF_B2, NP)}
    for c in range(L):
        gr = g_ref[c]
        gg = g[c].astype(np.float64)
        rel = np.linalg.norm(gg - gr) / np.linalg.norm(gr)
        cos = gg @ gr / (np.linalg.norm(gg) * np.linalg.norm(gr))
        per = {}
        for name, sl in blocks.items():
            d = np.linalg.norm(gr[sl])
            per[name] = np.linalg.norm(gg[sl] - gr[sl]) / d if d > 0 else np.linalg.norm(gg[sl])
        _log(f"  layer {c}: rel L2 {rel:.2e} cos {cos:.8f} " + " ".join(f"{k} {v:.2e}" for k, v in per.items()))
        assert rel <= 4e-3 and cos >= 1.0 - 4e-6, (c, rel, cos)
        for name, bound in GRAD_BOUNDS.items():
            assert per[name] <= bound, (c, name, per[name])
    f.close()


def test_training_graph_matches_eager_steps(ctx):
    """lr = 0: the captured step computes the same loss as the eager gradient call on the same
    stream, bit for bit, and leaves the parameters unchanged."""
    coefs, m, a, b, T, s, p = QUARTIC, 1.0, 0.0, 1.0, 2.0, 5, 10
    f = P.Flow(ctx, coefs, m, a, b, T, 1 << s, p, layers=4, batch=512, lr=0.0, init_scale=1.0, init_seed=3)
    th0 = f.get_params()
    losses, _ = f.train(17, 1000, 5)
    assert np.array_equal(f.get_params(), th0)
    for j in range(5):
        loss, _, _ = f.grad(17, 1000 + j)
        assert loss == losses[j], (j, loss, losses[j])
    # the step counter continues across calls: the next call starts at stream 1005
    more, _ = f.train(17, 1000, 2)
    assert more[0] == f.grad(17, 1005)[0]
    f.close()


def test_adam_step_matches_reference(ctx):
    coefs, m, a, b, T, s, p = QUARTIC, 1.0, 0.0, 1.0, 2.0, 4, 8
    lr = 1e-3
    f = P.Flow(ctx, coefs, m, a, b, T, 1 << s, p, layers=4, batch=256, lr=lr)
    th = _random_params(4, 5)
    f.set_params(th)
    _, _, g = f.grad(3, 77)
    f.train(3, 77, 1)
    got = f.get_params()
    g = g.astype(np.float32)
    mh = (np.float32(0.1) * g) / np.float32(1 - 0.9)
    vh = (np.float32(0.001) * g * g) / np.float32(1 - 0.999)
    ref = th - np.float32(lr) * mh / (np.sqrt(vh) + np.float32(1e-8))
    assert np.allclose(got, ref, rtol=1e-5, atol=1e-9)
    assert not np.array_equal(got, th)
    f.close()


def test_amplitude_sums_are_the_log_weights(ctx):
    """The canonical chunk sums of a proposal run equal sums of expm1(log w) of the same paths."""
    coefs, m, a, b, T, s, p = QUARTIC, 1.0, 0.0, 1.0, 2.0, 6, 10
    f = P.Flow(ctx, coefs, m, a, b, T, 1 << s, p, layers=4, batch=64)
    f.set_params(_random_params(4, 8, w2=0.02))
    n = 40000 + 123
    r, _, st = f.amplitude(n, 4, 9)
    assert st == 0 and r.n == n
    ell, _, _ = f.log_weights(4, 9, 0, n)
    total = ctx.last_partials(s, 0, 0)[2]
    parts, cp, total, shift = ctx.last_partials(s, 0, total)
    assert parts[:, 0].sum() == n
    for c in (0, total // 2, total - 1):
        d = np.expm1(ell[c * cp:(c + 1) * cp])
        assert parts[c, 0] == d.size
        assert parts[c, 1] == pytest.approx(math.fsum(d), rel=1e-12, abs=1e-12 * np.abs(d).sum())
        assert parts[c, 2] == pytest.approx(math.fsum(d * d), rel=1e-12)
    w = np.exp(ell)
    K0 = math.exp(-(b - a) ** 2 / (2 * T)) / math.sqrt(2 * math.pi * T)
    assert r.amp == pytest.approx(K0 * math.exp(-shift) * w.mean(), rel=1e-11)
    f.close()


def test_training_lowers_the_variance_and_stays_unbiased(ctx):
    """A short training run on the anharmonic oscillator lowers the weight variance; the estimate
    stays consistent with the plain estimator's (the reweighting is exact for any parameters).
    The loss mixes in the reverse KL (beta = 0.9): the second moment alone, estimated from samples
    of q itself, can be driven down by moving q away from the paths that matter."""
    coefs, m, a, b, T, s, p = QUARTIC, 1.0, 0.0, 1.0, 2.0, 7, 12
    f = P.Flow(ctx, coefs, m, a, b, T, 1 << s, p, layers=8, batch=4096, lr=1e-3, beta=0.9)
    n = 1 << 18
    r0, _, _ = f.amplitude(n, 1, 1 << 30)
    losses, ms = f.train(1, 1 << 31, 300)
    _log(f"loss {losses[0]:.4f} -> {losses[-1]:.4f} in {ms:.1f} ms")
    r1, _, _ = f.amplitude(n, 1, 1 << 30)
    _log(f"relvar plain {r0.relvar:.4f} flow {r1.relvar:.4f}; amp {r0.amp:.8e}+-{r0.err:.2e} vs "
         f"{r1.amp:.8e}+-{r1.err:.2e}")
    assert np.all(np.isfinite(losses))
    assert r1.relvar < 0.7 * r0.relvar
    assert abs(r1.amp - r0.amp) <= 5 * math.hypot(r0.err, r1.err)
    f.close()


def test_unsupported_and_invalid(ctx):
    with pytest.raises(P.PimcError) as e:
        P.Flow(ctx, QUARTIC, 1.0, 0.0, 1.0, 1.0, 256, 8)
    assert e.value.status == -2
    with pytest.raises(P.PimcError) as e:
        P.Flow(ctx, QUARTIC, 1.0, 0.0, 1.0, 1.0, 1, 8)
    assert e.value.status == -2
    with pytest.raises(P.PimcError) as e:
        P.Flow(ctx, QUARTIC, 1.0, 0.0, 1.0, 1.0, 16, 8, layers=0)
    assert e.value.status == -1
    f = P.Flow(ctx, QUARTIC, 1.0, 0.0, 1.0, 1.0, 16, 8, layers=2, batch=64)
    with pytest.raises(P.PimcError):
        f.set_params(np.zeros(10, dtype=np.float32))
    bad = f.get_params()
    bad[0, 0] = np.nan
    with pytest.raises(P.PimcError):
        f.set_params(bad)
    f.close()


def test_save_and_load_round_trip(ctx, tmp_path):
    coefs, m, a, b, T, s, p = QUARTIC, 1.0, 0.0, 1.0, 2.0, 5, 10
    f = P.Flow(ctx, coefs, m, a, b, T, 1 << s, p, layers=3, batch=64)
    f.set_params(_random_params(3, 4))
    path = str(tmp_path / "proposal.bin")
    f.save(path)
    g = P.Flow(ctx, coefs, m, a, b, T, 1 << s, p, layers=3, batch=64)
    g.load(path)
    assert np.array_equal(g.get_params(), f.get_params())
    assert np.array_equal(g.log_weights(1, 2, 0, 500)[0], f.log_weights(1, 2, 0, 500)[0])
    h = P.Flow(ctx, coefs, m, a, b, T, 1 << s, p, layers=4, batch=64)
    with pytest.raises(P.PimcError):
        h.load(path)                                   # another layer count
    with pytest.raises(P.PimcError):
        h.load(str(tmp_path / "missing.bin"))
    for x in (f, g, h):
        x.close()
