"""Pins of the FP64 affine-coupling proposal (oracle O6)."""
import math

import numpy as np
import pytest

from oracle import effective_action as ea
from oracle import flow
from oracle import pimc as opimc

V = ea.quartic(1, 10)
S_DEPTH = 3
D = (1 << S_DEPTH) - 1


def _setup(seed=0, scale=1.0, L=4, paths=64):
    theta = flow.init_params(L, seed, scale=scale)
    for th in theta:                          # non-zero biases so every parameter block matters
        rng = np.random.default_rng(seed + 7)
        th[flow.H * flow.KIN:flow.H * flow.KIN + flow.H] = rng.uniform(-0.1, 0.1, flow.H)
        th[-flow.H:] = rng.uniform(-0.05, 0.05, flow.H)
    u = flow.base_normals(1, 5, np.arange(paths), D)
    shift = opimc.straight_line_actions(V, 1, 0.0, 1.0, 2.0, S_DEPTH, 8)[S_DEPTH]
    return theta, u, shift


def test_masks_partition_every_node():
    for Dx in (7, 127):
        covered = set()
        for c in range(4):
            A, B = flow.masks(Dx, c)
            assert sorted(A + B) == list(range(1, Dx + 1))
            assert len(A) <= 64 and len(B) <= 64
            covered |= set(B)
        assert covered == set(range(1, Dx + 1))          # every node is transformed by some layer


def test_action_gradient_matches_finite_differences():
    z = np.random.default_rng(3).normal(size=(5, D))
    S, g = flow.action_and_grad(z, V, 1, 0.0, 1.0, 2.0, S_DEPTH, 8)
    h = 1e-6
    for k in range(D):
        zp, zm = z.copy(), z.copy()
        zp[:, k] += h
        zm[:, k] -= h
        fd = (flow.action_and_grad(zp, V, 1, 0.0, 1.0, 2.0, S_DEPTH, 8)[0] -
              flow.action_and_grad(zm, V, 1, 0.0, 1.0, 2.0, S_DEPTH, 8)[0]) / (2 * h)
        assert np.allclose(g[:, k], fd, rtol=1e-6, atol=1e-9)
    # and the action itself is the oracle's level action on the same path
    S2 = opimc.level_actions(opimc.bisection_paths(0.0, 1.0, 2.0, S_DEPTH, 1, 5, np.arange(5)), S_DEPTH,
                             opimc.level_tables(V, 8, 2.0, S_DEPTH))[:, S_DEPTH]
    u = flow.base_normals(1, 5, np.arange(5), D)
    assert np.allclose(flow.action_and_grad(u, V, 1, 0.0, 1.0, 2.0, S_DEPTH, 8)[0], S2, rtol=1e-14)


@pytest.mark.parametrize("beta", [0.0, 0.5])
def test_flow_gradient_matches_finite_differences(beta):
    theta, u, shift = _setup()
    loss, grads, _ = flow.flow_loss_and_grad(theta, u, V, 1, 0.0, 1.0, 2.0, S_DEPTH, 8, shift, beta, quantize=False)
    rng = np.random.default_rng(11)
    h = 1e-6
    blocks = [(0, flow.H * flow.KIN), (flow.H * flow.KIN, flow.H), (flow.H * flow.KIN + flow.H, flow.H * flow.H),
              (flow.NPARAM - flow.H, flow.H)]
    for c in (0, 2, 3):
        for (off, size) in blocks:
            for idx in rng.integers(off, off + size, 3):
                tp = [t.copy() for t in theta]
                tm = [t.copy() for t in theta]
                tp[c][idx] += h
                tm[c][idx] -= h
                lp = flow.flow_loss_and_grad(tp, u, V, 1, 0.0, 1.0, 2.0, S_DEPTH, 8, shift, beta, quantize=False)[0]
                lm = flow.flow_loss_and_grad(tm, u, V, 1, 0.0, 1.0, 2.0, S_DEPTH, 8, shift, beta, quantize=False)[0]
                fd = (lp - lm) / (2 * h)
                assert abs(grads[c][idx] - fd) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (c, off, idx, grads[c][idx], fd)


def test_zero_last_layer_is_the_plain_sampler():
    theta, u, shift = _setup(scale=0.0)
    for th in theta:
        th[-flow.H:] = 0.0                    # b2 = 0 with W2 = 0: s = t = 0
    l, z, logdet, _ = flow.log_weights(theta, u, V, 1, 0.0, 1.0, 2.0, S_DEPTH, 8, shift)
    assert np.array_equal(z, u) and np.all(logdet == 0)
    S = opimc.path_actions(V, 1, 0.0, 1.0, 2.0, S_DEPTH, 8, 1, 5, np.arange(u.shape[0]))[:, S_DEPTH]
    assert np.allclose(l, -(S - shift), rtol=1e-13, atol=1e-15)


def test_inverse_recovers_the_base_sample():
    theta, u, _ = _setup(scale=1.0)
    z, _, _ = flow.flow_forward(theta, u, D)
    assert np.allclose(flow.flow_inverse(theta, z, D), u, rtol=1e-11, atol=1e-12)
    assert np.max(np.abs(z - u)) > 1e-3                # the map is not the identity


def test_log_det_equals_jacobian_determinant():
    theta, u, _ = _setup(scale=1.0, paths=1)
    z, logdet, _ = flow.flow_forward(theta, u, D, quantize=False)
    J = np.zeros((D, D))
    h = 1e-6
    for k in range(D):
        up, um = u.copy(), u.copy()
        up[0, k] += h
        um[0, k] -= h
        J[:, k] = (flow.flow_forward(theta, up, D, quantize=False)[0][0] -
                   flow.flow_forward(theta, um, D, quantize=False)[0][0]) / (2 * h)
    assert logdet[0] == pytest.approx(np.linalg.slogdet(J)[1], abs=1e-7)


def test_random_flow_is_unbiased_on_free_particle():
    """V = 0: E_q[phi(z)/q(z)] = 1 for any flow (exact reweighting)."""
    theta = flow.init_params(4, 5, scale=1.0)
    u = flow.base_normals(3, 1, np.arange(40000), D)
    l, _, _, _ = flow.log_weights(theta, u, ea.poly([]), 1, 0.0, 1.0, 2.0, S_DEPTH, 8, 0.0)
    w = np.exp(l)
    assert abs(w.mean() - 1.0) < 4 * w.std() / math.sqrt(w.size)
    assert w.std() > 0.01                                  # the proposal differs from the target


def test_bf16_rounding_is_round_to_nearest_even():
    assert list(flow.bf16(np.array([1.0, -2.5, 0.0, 3.0]))) == [1.0, -2.5, 0.0, 3.0]
    # exact ties: 1 + 2^-8 is halfway between 1 and 1 + 2^-7 -> even (1.0); 1 + 3*2^-8 -> 1 + 2^-6
    assert flow.bf16(np.array([1.0 + 2 ** -8]))[0] == 1.0
    assert flow.bf16(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6
    assert flow.bf16(np.array([1.0 + 2 ** -8 + 2 ** -12]))[0] == 1.0 + 2 ** -7
