"""Batched grids (mixed N, p, T in one graph launch): bitwise equal to single calls, independent of
the launch shape, stable across graph replays, and on identical samples equal to the oracle."""
import math
import os
import tempfile

import numpy as np
import pytest

import paper_1105_0542_amd as P
from paper_1105_0542_amd import workloads
from oracle import effective_action as ea
from oracle import pimc as opimc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = P.Context()
    yield c
    c.close()


def small_grid(samples=3000):
    systems, rows = workloads.evolution_matrix_tasks(n_grid=4, samples=samples, levels=(8, 12, 18),
                                                     times=(0.5, 2.0))
    return systems, rows


def same(u, v):
    return u == v or (math.isnan(u) and math.isnan(v))


def single(ctx, systems, row, seed, flags):
    si, m, a, b, T, N, p, n, stream = row
    res, st = ctx.amplitude(systems[si], m, a, b, T, N, p, n, seed, stream, flags)
    return res


@pytest.mark.parametrize("flags", [0, P.FLAG_HIERARCHY])
def test_batch_equals_single_calls_bitwise(ctx, flags):
    systems, rows = small_grid()
    print(f"batch of {len(rows)} tasks, flags={flags}", flush=True)
    bt = P.Batch(ctx, systems, rows, seed=7, flags=flags)
    out, ms, st = bt.run()
    for t in range(0, len(rows), 5):
        ref = single(ctx, systems, rows[t], 7, flags)
        s = int(rows[t][5]).bit_length() - 1
        levels = range(s + 1) if flags else [0, s]
        for n in levels:
            assert same(out[t, n]["amp"], ref[n].amp), (t, n)
            assert same(out[t, n]["err"], ref[n].err), (t, n)
            assert out[t, n]["n"] == ref[n].n
    bt.close()


def test_batch_launch_shape_does_not_change_bits(ctx):
    """Every compiled launch shape of every class (subtree depth, workgroup size, waves per SIMD,
    slice batch) and every grid and grab give the same bits: the canonical chunks fix the order of
    every sum."""
    systems, rows = small_grid()
    bt = P.Batch(ctx, systems, rows, seed=3, flags=P.FLAG_HIERARCHY)
    base, _, _ = bt.run()
    classes = bt.classes()
    assert {c["p"] for c in classes} == {8, 12, 18}
    for k, c in enumerate(classes):
        assert c["n_shapes"] == (5 if c["n16"] else 8)
        for shape in range(1, c["n_shapes"]):
            bt.set_shape(k, shape)
            info = bt.classes()[k]
            print(f"class {k} (p={c['p']}, n16={c['n16']}): shape {shape} U={info['subtree_levels']} "
                  f"block={info['block']} waves/EU={info['waves_per_eu']} batch={info['slice_batch']}", flush=True)
            out, _, _ = bt.run()
            assert np.array_equal(out["amp"], base["amp"], equal_nan=True), (k, shape)
            assert np.array_equal(out["err"], base["err"], equal_nan=True), (k, shape)
        bt.set_shape(k, 0)
    for g, grab in [(1, 1), (2, 4), (4, 16), (8, 64), (3, 7)]:
        bt.set_tuning(g, grab)
        out, _, _ = bt.run()
        assert np.array_equal(out["amp"], base["amp"], equal_nan=True), (g, grab)
        assert np.array_equal(out["err"], base["err"], equal_nan=True), (g, grab)
    bt.close()


def test_batch_results_into_device_memory(ctx):
    """The results of a replay written into a caller-owned device buffer (a torch tensor) equal the
    host-memory results bit for bit."""
    import torch
    systems, rows = small_grid(samples=1000)
    bt = P.Batch(ctx, systems, rows, seed=2, flags=P.FLAG_HIERARCHY)
    host, _, _ = bt.run()
    out = torch.full((len(rows), bt.s_max + 1, 7), float("nan"), dtype=torch.float64, device="cuda")
    ms, st = bt.run_to_device(out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for j, name in enumerate(("amp", "err", "log_amp", "relvar", "ess")):
        assert np.array_equal(got[..., j], host[name], equal_nan=True), name
    for j, name in ((5, "n"), (6, "n_nonfinite")):
        assert np.array_equal(np.ascontiguousarray(got[..., j]).view(np.uint64), host[name]), name
    with pytest.raises(ValueError):
        bt.run_to_device(torch.empty(3, dtype=torch.float64, device="cuda"))
    bt.close()


def test_graph_replays_match_eager(ctx):
    """Replays interleaved with eager work on the same context all reproduce the first result."""
    systems, rows = small_grid(samples=1000)
    bt = P.Batch(ctx, systems, rows, seed=5, flags=P.FLAG_HIERARCHY)
    first, _, _ = bt.run()
    eager = single(ctx, systems, rows[0], 5, P.FLAG_HIERARCHY)
    s0 = int(rows[0][5]).bit_length() - 1
    assert same(first[0, s0]["amp"], eager[s0].amp)
    for rep in range(4):
        ctx.amplitude(P.quartic(1, 1), 1.0, 0.0, 1.0, 1.0, 64, 4, 20000, 1, rep, 0)     # eager work between replays
        out, _, _ = bt.run()
        assert np.array_equal(out["amp"], first["amp"], equal_nan=True), rep
        assert np.array_equal(out["err"], first["err"], equal_nan=True), rep
    bt.close()


def test_batch_tasks_match_oracle(ctx):
    systems, rows = small_grid(samples=2000)
    bt = P.Batch(ctx, systems, rows, seed=11, flags=0)
    out, _, _ = bt.run()
    for t in (0, 17, 40, len(rows) - 1):
        si, m, a, b, T, N, p, n, stream = rows[t]
        s = int(N).bit_length() - 1
        A, g = ((1.0, 1.0), (-1.0, 4.0))[si]
        ref = opimc.amplitude(ea.quartic(A, g), 1, a, b, T, s, p, n, 11, stream)
        assert out[t, s]["amp"] == pytest.approx(ref[s]["amp"], rel=1e-10), t
        assert out[t, s]["err"] == pytest.approx(ref[s]["err"], rel=1e-8), t
    bt.close()


def test_autotune_cache_roundtrip(ctx):
    systems, rows = small_grid(samples=500)
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "tune.txt")
        bt = P.Batch(ctx, systems, rows, seed=1)
        choice = bt.autotune(path)
        res1, _, _ = bt.run()
        bt.close()
        assert os.path.exists(path) and open(path).read().strip()
        bt2 = P.Batch(ctx, systems, rows, seed=1)
        assert bt2.autotune(path) == choice
        res2, _, _ = bt2.run()
        assert np.array_equal(res1["amp"], res2["amp"], equal_nan=True)
        bt2.close()


def test_batch_rejects_unsupported(ctx):
    with pytest.raises(P.PimcError) as ei:
        P.Batch(ctx, [[0.0, 0.1, 0.5, 0.0, 0.04]], [(0, 1.0, 0.0, 1.0, 1.0, 64, 8, 100, 0)], seed=1)
    assert ei.value.status == -2
    with pytest.raises(P.PimcError) as ei:
        P.Batch(ctx, [P.quartic(1, 1)], [(0, 1.0, 0.0, 1.0, 1.0, 8, 8, 100, 0)], seed=1)
    assert ei.value.status == -2
    with pytest.raises(P.PimcError) as ei:
        P.Batch(ctx, [P.quartic(1, 1)], [(1, 1.0, 0.0, 1.0, 1.0, 64, 8, 100, 0)], seed=1)
    assert ei.value.status == -1
