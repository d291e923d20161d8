"""FP32 slice polynomials (FP64 mid-point/deviation, per-path sums and weights): per-path actions
against the oracle at FP32 tolerance, and the amplitude against the FP64 path on identical samples.

Tolerance derivation: each slice value is a Horner chain of <= 11 FP32 FMAs (relative rounding
~11 * 2^-24 ~ 7e-7 of the slice's magnitude scale) plus the FP32 rounding of mid-point and
deviation (2^-24 relative, amplified by the polynomial's log-derivative, <= ~20 for |x| <~ 5);
summed over slices in FP64 the action error stays below 2e-5 of sum_k |eps W_k|.
"""
import math

import numpy as np
import pytest

import paper_1105_0542_amd as P
from oracle import effective_action as ea
from oracle import pimc as opimc

pytestmark = pytest.mark.gpu
F32 = P.FLAG_FP32_POLY
H = P.FLAG_HIERARCHY


@pytest.fixture(scope="module")
def ctx():
    c = P.Context()
    yield c
    c.close()


@pytest.mark.parametrize("p,s,g,T", [(18, 9, 10.0, 1.0), (12, 7, 10.0, 2.0), (4, 4, 1.0, 1.0), (8, 6, 48.0, 5.0)])
def test_fp32_actions_vs_oracle(ctx, p, s, g, T):
    print(f"fp32 actions p={p} s={s} g={g} T={T}", flush=True)
    k = 2000
    got = ctx.path_actions(P.quartic(1, g), 1.0, 0.0, 1.0, T, 1 << s, p, 1, 0, F32 | H, 0, k)
    S, scale = opimc.path_actions_and_scales(ea.quartic(1, g), 1, 0.0, 1.0, T, s, p, 1, 0,
                                             np.arange(k, dtype=np.uint64))
    for n in range(s + 1):
        err = np.abs(got[:, n] - S[:, n])
        assert np.all(err <= 2e-5 * np.maximum(np.abs(S[:, n]), scale[:, n]) + 1e-30), n


def test_fp32_amplitude_vs_fp64_identical_samples(ctx):
    """Precision workload shape (g=10, p=18, N=512, T=1): |A_fp32 - A_fp64| well below the
    statistical error, on the same 2e6 samples."""
    n = 2_000_000
    a64, st64 = ctx.amplitude(P.quartic(1, 10), 1.0, 0.0, 1.0, 1.0, 512, 18, n, 1, 0, 0)
    a32, st32 = ctx.amplitude(P.quartic(1, 10), 1.0, 0.0, 1.0, 1.0, 512, 18, n, 1, 0, F32)
    assert st64 == 0 and st32 == 0
    rel = abs(a32[9].amp - a64[9].amp) / a64[9].amp
    print(f"fp32 vs fp64 relative difference {rel:.3e}, statistical {a64[9].err / a64[9].amp:.3e}", flush=True)
    assert abs(a32[9].amp - a64[9].amp) < 0.1 * a64[9].err
    assert rel < 1e-6
    assert a32[9].err == pytest.approx(a64[9].err, rel=1e-4)


def test_fp32_needs_the_specialized_kernel(ctx):
    with pytest.raises(P.PimcError) as ei:
        ctx.amplitude([0.1, 0.2, 0.3, 0.4, 0.05], 1.0, 0.0, 1.0, 1.0, 64, 8, 1000, 1, 0, F32)
    assert ei.value.status == -2
    with pytest.raises(P.PimcError):
        ctx.amplitude(P.quartic(1, 1), 1.0, 0.0, 1.0, 1.0, 8, 8, 1000, 1, 0, F32)
