"""GPU parity: the HIP path (through the C ABI) against the oracle on identical Philox samples.

Tolerances (FP64):
* per-path level action: |S_gpu - S_orc| <= 1e-12 * max(|S_orc|, sum_k |eps W_k|) -- both sides
  use FP64 transcendental functions (log, sin/cos) that agree to a few ulp and evaluate the slice
  polynomial in different but equivalent forms, so differences are O(1e-15) of the scale;
* amplitude on identical samples: relative 1e-10; its Monte Carlo error: relative 1e-8.
"""
import math
import os
import sys

import numpy as np
import pytest

import paper_1105_0542_amd as P
from oracle import closed_forms as cf
from oracle import effective_action as ea
from oracle import pimc as opimc

pytestmark = pytest.mark.gpu

ACTION_TOL = 1e-12
AMP_TOL = 1e-10
ERR_TOL = 1e-8


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = P.Context()
    yield c
    c.close()


def _exact_poly(coefs):
    from fractions import Fraction
    return ea.poly([Fraction(c) for c in coefs])


def check_actions(ctx, coefs, m, a, b, T, s, p, seed, stream, flags, first, k):
    _log(f"actions coefs={coefs} m={m} a={a} b={b} T={T} s={s} p={p} seed={seed} stream={stream} "
         f"flags={flags} paths={first}+{k}")
    got = ctx.path_actions(coefs, m, a, b, T, 1 << s, p, seed, stream, flags, first, k)
    idx = np.arange(first, first + k, dtype=np.uint64)
    S, scale = opimc.path_actions_and_scales(_exact_poly(coefs), m, a, b, T, s, p, seed, stream, idx)
    levels = range(s + 1) if flags & P.FLAG_HIERARCHY else [s]
    for n in levels:
        err = np.abs(got[:, n] - S[:, n])
        lim = ACTION_TOL * np.maximum(np.abs(S[:, n]), scale[:, n]) + 1e-300
        bad = np.nonzero(err > lim)[0]
        assert bad.size == 0, (n, bad[:5], got[bad[:3], n], S[bad[:3], n])
    if not flags & P.FLAG_HIERARCHY:
        assert np.all(got[:, :s] == 0.0)
    return got


# ------------------------------------------------------------------------- normals (Philox + Box-Muller)
@pytest.mark.parametrize("seed,stream,first,k,nodes", [
    (1, 0, 0, 4096, 1023), (0xDEADBEEFCAFE, 7, (1 << 40) + 3, 512, 127), (5, 2**31 + 9, 123456789, 2000, 15),
])
def test_normals_match_oracle(ctx, seed, stream, first, k, nodes):
    """Device normals vs the oracle's (numpy log/sqrt/cos/sin in FP64) on the same counters: the
    uniforms are identical bits, the elementary functions agree to a few ulp."""
    _log(f"normals seed={seed} stream={stream} first={first} k={k} nodes={nodes}")
    got = ctx.normals(seed, stream, first, k, nodes)
    from oracle.philox import node_normals
    idx = np.arange(first, first + k, dtype=np.uint64)
    ref = np.stack([node_normals(seed, stream, idx, np.uint64(h)) for h in range(1, nodes + 1)], axis=1)
    # the oracle forms the angle 2*pi*u rounded (up to ~4e-16 absolute), so near zero crossings the
    # comparison is absolute; elsewhere relative
    err = np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)
    assert err.max() < 1e-14, err.max()


# ------------------------------------------------------------------------- C1 (N=16, p=4, 1e5)
def test_c1_path_actions_all_paths(ctx):
    check_actions(ctx, P.quartic(1, 1), 1.0, 0.0, 1.0, 1.0, 4, 4, 1, 0, P.FLAG_HIERARCHY, 0, 100000)


def test_c1_amplitude_identical_samples(ctx):
    n = 100000
    _log("amplitude C1")
    res, st = ctx.amplitude(P.quartic(1, 1), 1.0, 0.0, 1.0, 1.0, 16, 4, n, 1, 0, P.FLAG_HIERARCHY)
    assert st == 0
    ref = opimc.amplitude(ea.quartic(1, 1), 1, 0.0, 1.0, 1.0, 4, 4, n, 1, 0)
    for lv in range(5):
        assert res[lv].n == n
        assert res[lv].amp == pytest.approx(ref[lv]["amp"], rel=AMP_TOL)
        if lv == 0:
            assert res[lv].err == 0.0
        else:
            assert res[lv].err == pytest.approx(ref[lv]["err"], rel=ERR_TOL)
            assert res[lv].relvar == pytest.approx(ref[lv]["relvar"], rel=1e-7)
            assert res[lv].ess == pytest.approx(ref[lv]["ess"], rel=1e-9)
    # continuum (grid diagonalization): the p=4, N=16 discretization error is far below sigma
    cont = cf.dvr_amplitude(cf.quartic_V(1, 1), 0.0, 1.0, 1.0)
    assert abs(res[4].amp - cont) < 4 * res[4].err


def test_c1_free_particle_exact(ctx):
    K0 = math.exp(-0.5) / math.sqrt(2 * math.pi)
    res, st = ctx.amplitude([0.0], 1.0, 0.0, 1.0, 1.0, 16, 4, 100000, 1, 0, P.FLAG_HIERARCHY)
    assert st == 0
    for r in res:
        assert r.amp == pytest.approx(K0, rel=1e-15)
        assert r.err == 0.0


def test_c1_harmonic_matches_exact_discretized(ctx):
    res, st = ctx.amplitude(P.quartic(1, 0), 1.0, 0.0, 1.0, 1.0, 16, 4, 100000, 1, 0, P.FLAG_HIERARCHY)
    ref = opimc.amplitude(ea.quartic(1, 0), 1, 0.0, 1.0, 1.0, 4, 4, 100000, 1, 0)
    for lv in range(1, 5):
        ex = cf.gaussian_discretized(0.0, 1.0, 1.0, 1 << lv, 4)
        assert abs(res[lv].amp - ex) < 4 * res[lv].err
        assert res[lv].amp == pytest.approx(ref[lv]["amp"], rel=AMP_TOL)


# ------------------------------------------------------------------------- shapes and kernels
@pytest.mark.parametrize("s", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("p", [1, 2, 3, 8, 12, 18])
def test_actions_across_levels_and_depths(ctx, s, p):
    """Generic kernels (s < 4) and the specialized quartic kernels (s >= 4), every level."""
    check_actions(ctx, P.quartic(1, 10), 1.0, 0.0, 1.0, 1.0, s, p, 7, 3, P.FLAG_HIERARCHY, 12345, 700)


def test_actions_level_s_only(ctx):
    check_actions(ctx, P.quartic(1, 10), 1.0, 0.0, 1.0, 1.0, 6, 12, 2, 0, 0, 0, 1000)


@pytest.mark.parametrize("coefs,p,s", [
    ([0.25, -0.5, 1.0, 0.3, 1 / 24], 10, 5),                     # odd terms: generic odd kernel
    ([0.0, 0.0, 0.5, 0.0, -0.2, 0.0, 1 / 30.0], 12, 5),          # even sextic: generic even kernel
    ([0.0, 0.8], 6, 4),                                          # linear
    ([0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9], 6, 3),       # degree 8
])
def test_actions_general_potentials(ctx, coefs, p, s):
    check_actions(ctx, coefs, 1.0, -0.3, 0.4, 0.5, s, p, 11, 5, P.FLAG_HIERARCHY, 0, 600)


def test_actions_mass_and_endpoints(ctx):
    check_actions(ctx, P.quartic(-1, 4), 2.5, -1.5, 2.0, 2.0, 6, 8, 5, 9, P.FLAG_HIERARCHY, 999, 500)


def test_actions_p18_n1024(ctx):
    check_actions(ctx, P.quartic(1, 10), 1.0, 0.0, 1.0, 1.0, 10, 18, 1, 0, P.FLAG_HIERARCHY, 0, 1500)


def test_actions_large_path_indices(ctx):
    """Path words above 2^32 reach the third Philox counter word."""
    check_actions(ctx, P.quartic(1, 10), 1.0, 0.0, 1.0, 2.0, 5, 12, 3, 1, P.FLAG_HIERARCHY, (1 << 33) + 17, 300)


def test_largest_n_nests_bitwise(ctx):
    """N = 2^20 (the largest): levels 0..10 of every path equal the N = 2^10 run bit for bit (the
    deepest walk, 15 stack levels above the register subtrees), and every level is finite."""
    _log("largest N nesting")
    big = ctx.path_actions(P.quartic(1, 10), 1.0, 0.0, 1.0, 1.0, 1 << 20, 18, 5, 1, P.FLAG_HIERARCHY, 0, 256)
    small = ctx.path_actions(P.quartic(1, 10), 1.0, 0.0, 1.0, 1.0, 1 << 10, 18, 5, 1, P.FLAG_HIERARCHY, 0, 256)
    assert np.array_equal(big[:, :11], small)
    assert np.all(np.isfinite(big))


def test_hierarchy_level_equals_separate_run(ctx):
    """Level n of an s-run is bitwise the n-run on the same samples."""
    big = ctx.path_actions(P.quartic(1, 10), 1.0, 0.0, 1.0, 1.0, 1 << 8, 18, 1, 0, P.FLAG_HIERARCHY, 0, 2000)
    for n in (4, 6):
        small = ctx.path_actions(P.quartic(1, 10), 1.0, 0.0, 1.0, 1.0, 1 << n, 18, 1, 0, P.FLAG_HIERARCHY, 0, 2000)
        assert np.array_equal(big[:, n], small[:, n])


# ------------------------------------------------------------------------- amplitude parity
@pytest.mark.parametrize("n", [2, 255, 4097, 70001])
def test_amplitude_ragged_sample_counts(ctx, n):
    _log(f"amplitude ragged n={n}")
    res, st = ctx.amplitude(P.quartic(1, 10), 1.0, 0.0, 1.0, 2.0, 32, 10, n, 4, 2, P.FLAG_HIERARCHY)
    assert st == 0
    ref = opimc.amplitude(ea.quartic(1, 10), 1, 0.0, 1.0, 2.0, 5, 10, n, 4, 2)
    for lv in range(6):
        assert res[lv].n == n
        assert res[lv].amp == pytest.approx(ref[lv]["amp"], rel=AMP_TOL)
        if lv:
            assert res[lv].err == pytest.approx(ref[lv]["err"], rel=ERR_TOL)


def test_beyond_convergence_radius_is_flagged(ctx):
    """p = 12 (negative leading x-coefficient of the quartic W_p) at eps = 1: a path reaching
    |x| ~ 2.8 has action ~ -460 (finite radius of convergence, Sec. 4), its weight's square
    overflows FP64. Both sides keep it in the sums; the library reports err = +inf and warns."""
    n = 4097
    res, st = ctx.amplitude(P.quartic(1, 10), 1.0, 0.0, 1.0, 2.0, 32, 12, n, 4, 2, P.FLAG_HIERARCHY)
    ref = opimc.amplitude(ea.quartic(1, 10), 1, 0.0, 1.0, 2.0, 5, 12, n, 4, 2)
    assert st == P.binding.PIMC_WNONFINITE
    assert res[1].amp == pytest.approx(ref[1]["amp"], rel=AMP_TOL)
    assert math.isinf(ref[1]["err"]) and math.isinf(res[1].err)
    assert res[1].ess == 1.0
    for lv in range(2, 6):
        assert res[lv].amp == pytest.approx(ref[lv]["amp"], rel=AMP_TOL)
        assert res[lv].err == pytest.approx(ref[lv]["err"], rel=ERR_TOL)


def test_amplitude_without_hierarchy(ctx):
    res, st = ctx.amplitude(P.quartic(1, 10), 1.0, 0.0, 1.0, 1.0, 64, 8, 5000, 1, 0, 0)
    ref = opimc.amplitude(ea.quartic(1, 10), 1, 0.0, 1.0, 1.0, 6, 8, 5000, 1, 0)
    assert res[6].amp == pytest.approx(ref[6]["amp"], rel=AMP_TOL)
    assert res[0].amp == pytest.approx(ref[0]["amp"], rel=1e-14)
    for lv in range(1, 6):
        assert res[lv].n == 0


def test_amplitude_is_deterministic(ctx):
    a, _ = ctx.amplitude(P.quartic(1, 48), 1.0, 0.0, 1.0, 5.0, 256, 18, 300000, 9, 1, P.FLAG_HIERARCHY)
    b, _ = ctx.amplitude(P.quartic(1, 48), 1.0, 0.0, 1.0, 5.0, 256, 18, 300000, 9, 1, P.FLAG_HIERARCHY)
    same = lambda u, v: (u == v) or (math.isnan(u) and math.isnan(v))
    for x, y in zip(a, b):
        assert same(x.amp, y.amp) and same(x.err, y.err) and x.n_nonfinite == y.n_nonfinite


def test_full_size_c2_point_sampled_chunks(ctx):
    """The benchmark configuration (p=18, N=1024, 1e8 samples, every level): sampled canonical chunks
    against the oracle's per-chunk sums on the same paths, and the merged result against the chunks."""
    n = 100_000_000
    _log("full-size C2 point p=18 N=1024 n=1e8")
    res, st = ctx.amplitude(P.quartic(1, 10), 1.0, 0.0, 1.0, 1.0, 1024, 18, n, 1, 0, P.FLAG_HIERARCHY)
    assert st == 0
    part, cp, total, shift = ctx.last_partials(10, 0, 1)
    assert total == (n + cp - 1) // cp
    rng = np.random.default_rng(0)
    picks = [0, int(rng.integers(1, total - 1)), total - 1]
    assert cp == P.binding.PIMC_CHUNK_PATHS
    sh_all = [ctx.last_partials(l, 0, 0)[3] for l in range(11)]
    for c in picks:
        first = c * cp
        cnt = min(cp, n - first)
        ref = opimc.chunk_sums(ea.quartic(1, 10), 1, 0.0, 1.0, 1.0, 10, 18, 1, 0, first, cnt, sh_all)
        for lv in (10, 7, 3):
            got = ctx.last_partials(lv, c, 1)[0][0]
            assert got[0] == cnt
            assert got[1] == pytest.approx(ref[lv][1], rel=1e-9, abs=1e-12 * cnt)
            assert got[2] == pytest.approx(ref[lv][2], rel=1e-9, abs=1e-12 * cnt)
            assert got[3] == 0
    cont = cf.dvr_amplitude(cf.quartic_V(1, 10), 0.0, 1.0, 1.0)
    assert abs(res[10].amp - cont) < 5 * res[10].err
    assert res[10].n == n
