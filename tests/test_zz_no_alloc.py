"""The estimation entry point that allocates nothing (pimc_amplitude_noalloc): through the C ABI,
the same results as pimc_amplitude bit for bit, on two calls in a row (the second smaller, so the
shared workspace holds the first call's contents), and a clear error beyond the workspace."""
import numpy as np
import pytest

import paper_1105_0542_amd as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = P.Context()
    yield c
    c.close()


def _same(a, b):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        assert (x.amp == y.amp or (np.isnan(x.amp) and np.isnan(y.amp))), (x, y)
        assert (x.err == y.err or (np.isnan(x.err) and np.isnan(y.err))), (x, y)
        assert x.n == y.n and x.n_nonfinite == y.n_nonfinite, (x, y)


def test_no_alloc_equals_the_allocating_entry_point(ctx):
    cases = [  # (coefs, m, a, b, T, N, p, n, seed, stream, flags): a large run, then a smaller one
        (P.quartic(1.0, 10.0), 1.0, 0.0, 1.0, 1.0, 1024, 18, 3_000_001, 1, 7, P.FLAG_HIERARCHY),
        (P.quartic(1.0, 1.0), 1.3, -0.2, 0.9, 2.0, 16, 4, 70_001, 5, 2, 0),
    ]
    for coefs, m, a, b, T, N, p, n, seed, stream, flags in cases:
        print(f"no-alloc N={N} p={p} n={n} flags={flags}", flush=True)
        got, st1 = ctx.amplitude_noalloc(coefs, m, a, b, T, N, p, n, seed, stream, flags)
        ref, st2 = ctx.amplitude(coefs, m, a, b, T, N, p, n, seed, stream, flags)
        assert st1 == st2
        _same(got, ref)
    # the chunk sums of the last call are readable (from the workspace) and merge to its result
    again, _ = ctx.amplitude_noalloc(P.quartic(1.0, 1.0), 1.0, 0.0, 1.0, 1.0, 32, 8, 9000, 3, 1, 0)
    parts, cp, total, shift = ctx.last_partials(5, 0, 3)
    assert cp == P.binding.PIMC_CHUNK_PATHS and total == 3 and parts[:, 0].sum() == 9000


def test_no_alloc_rejects_more_than_the_workspace(ctx):
    # every level of N = 1024 needs 11 x 32 bytes per chunk of 4096 paths: 2e8 samples exceed 16 MiB
    with pytest.raises(P.PimcError) as e:
        ctx.amplitude_noalloc(P.quartic(1.0, 1.0), 1.0, 0.0, 1.0, 1.0, 1024, 8, 200_000_000, 1, 0, P.FLAG_HIERARCHY)
    assert e.value.status == P.binding.PIMC_EINVAL
    assert "workspace" in str(e.value)
    # the context stays usable
    ok, st = ctx.amplitude_noalloc(P.quartic(1.0, 1.0), 1.0, 0.0, 1.0, 1.0, 64, 8, 5000, 1, 0, 0)
    assert st == 0 and ok[6].n == 5000
