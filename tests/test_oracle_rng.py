"""Pins of the oracle's counter-based normals (O2) and of the bisection construction (O3)."""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

from oracle import philox
from oracle import pimc

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = [int(t, 16) for t in line.split()]
                rows.append((v[:4], v[4:6], v[6:]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_philox_known_answers(ctr, key, out):
    got = philox.philox4x32_10(*[[c] for c in ctr], key[0], key[1])
    assert [int(g[0]) for g in got] == out


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_bit_for_bit():
    """An independent implementation (rocRAND's open-source engine, called from a host program)."""
    rng = np.random.default_rng(11)
    ctrs = rng.integers(0, 2 ** 32, size=(200, 6), dtype=np.uint64)
    ctrs[:, 1] &= (1 << 29) - 1          # the host helper reaches counter word 1 < 2^30 only
    with tempfile.TemporaryDirectory() as td:
        exe = os.path.join(td, "rdump")
        subprocess.run(["hipcc", "-O1", "-o", exe, os.path.join(HERE, "rocrand_philox_dump.cpp")],
                       check=True, capture_output=True, timeout=600)
        inp = "\n".join(" ".join("%x" % int(v) for v in row) for row in ctrs) + "\n"
        res = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True, timeout=60)
    ref = [[int(t, 16) for t in line.split()] for line in res.stdout.strip().splitlines()]
    got = philox.philox4x32_10(ctrs[:, 0], ctrs[:, 1], ctrs[:, 2], ctrs[:, 3], 0, 0)
    # keys differ per row: evaluate row by row
    for i, row in enumerate(ctrs):
        g = philox.philox4x32_10([row[0]], [row[1]], [row[2]], [row[3]], int(row[4]), int(row[5]))
        assert [int(x[0]) for x in g] == ref[i], i
    assert got is not None


def test_uniform_conversion_is_open_and_exact():
    lo = np.array([0, 0xFFFFFFFF, 0x12345678, 0], dtype=np.uint64)
    hi = np.array([0, 0xFFFFFFFF, 0x9ABCDEF0, 0x80000000], dtype=np.uint64)
    u = philox.odd53(lo, hi)
    assert u[0] == 2.0 ** -53
    assert u[1] == 1.0 - 2.0 ** -53
    assert u[3] == 0.5 + 2.0 ** -53
    assert np.all((u > 0) & (u < 1))
    # odd multiples of 2^-53: exactly representable
    k = u * 2.0 ** 53
    assert np.all(k == np.round(k)) and np.all(k % 2 == 1)


def test_normals_moments_and_ks():
    n = 1 << 20
    paths = np.arange(n // 8, dtype=np.uint64)
    z = np.concatenate([philox.node_normals(1, 0, paths, np.uint64(h)) for h in range(1, 9)])
    se = 1 / math.sqrt(z.size)
    assert abs(z.mean()) < 5 * se
    assert abs(z.var() - 1) < 5 * math.sqrt(2) * se
    assert abs(stats.skew(z)) < 5 * math.sqrt(6) * se
    assert abs(stats.kurtosis(z)) < 5 * math.sqrt(24) * se
    assert stats.kstest(z, "norm").pvalue > 1e-4


def test_sibling_normals_are_independent():
    """cos/sin outputs of one call (nodes 2j, 2j+1) are uncorrelated standard normals."""
    paths = np.arange(200000, dtype=np.uint64)
    a = philox.node_normals(5, 3, paths, np.uint64(6))
    b = philox.node_normals(5, 3, paths, np.uint64(7))
    r = np.corrcoef(a, b)[0, 1]
    assert abs(r) < 5 / math.sqrt(paths.size)
    r2 = np.corrcoef(a * a, b * b)[0, 1]
    assert abs(r2) < 5 / math.sqrt(paths.size)


def test_streams_and_seeds_differ():
    paths = np.arange(1000, dtype=np.uint64)
    a = philox.node_normals(1, 0, paths, np.uint64(3))
    b = philox.node_normals(1, 1, paths, np.uint64(3))
    c = philox.node_normals(2, 0, paths, np.uint64(3))
    assert not np.any(a == b) and not np.any(a == c)


def test_bridge_covariance():
    """Bisection with sigma_n^2 = T/2^(n+1) samples the Brownian bridge: Cov = min(t,t') - t t'/T."""
    T, s = 2.0, 3
    N = 1 << s
    q = pimc.bisection_paths(0.0, 0.0, T, s, 7, 0, np.arange(200000, dtype=np.uint64))
    t = np.arange(N + 1) * T / N
    C = np.cov(q[:, 1:N].T)
    Cex = np.minimum.outer(t[1:N], t[1:N]) - np.outer(t[1:N], t[1:N]) / T
    assert np.max(np.abs(C - Cex)) < 0.02
    assert np.max(np.abs(q[:, 1:N].mean(axis=0))) < 0.01


def test_bridge_mean_follows_endpoints():
    a, b, T = -1.5, 2.0, 1.0
    q = pimc.bisection_paths(a, b, T, 4, 1, 0, np.arange(100000, dtype=np.uint64))
    t = np.arange(17) / 16
    assert np.max(np.abs(q.mean(axis=0) - (a + (b - a) * t))) < 0.01
    assert q[0, 0] == a and q[0, -1] == b
