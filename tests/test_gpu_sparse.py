"""Sparse scenes (at most 3 points per frame, as interest points usually
are) with long candidate lists: the packed schedule of the recursion (every
cell of a step on its own lane) against the FP64 oracle, per model and in
plans, windowed and on given lists."""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
import paper_1505_00581_amd as stm
from tolerances import energy_tol
from paper_1505_00581_amd import synth

pytestmark = pytest.mark.gpu



def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = stm.Context(0)
    yield c
    c.close()


def _np(x):
    return x.cpu().numpy() if hasattr(x, "cpu") else np.asarray(x)


def _sparse(seed, n_frames=160, per=(0, 3)):
    rng = np.random.Generator(np.random.PCG64(seed))
    m = synth.make_model(rng, 24, 160.0, 120.0, 10, frame_hi=36)
    counts = rng.integers(per[0], per[1] + 1, size=n_frames)
    xy, t, d = synth.clutter(rng, counts, 160.0, 120.0, m.dim)
    parts = ([xy], [t], [d])
    pxy, pt, pd, _ = synth.plant_copy(rng, m, n_frames, 160.0, 120.0)
    parts[0].append(pxy)
    parts[1].append(pt)
    parts[2].append(pd)
    s = synth.assemble_scene(*parts, n_frames)
    assert s.n <= 3 * n_frames
    return m, s


def check(m, s, p, res, ora, rows=None):
    e32 = _np(res["energy32"]).astype(np.float64)
    e64, A = _np(res["energy64"]), _np(res["assign"])
    if rows is not None:
        e32, e64, A = e32[rows], e64[rows], A[rows]
    E = ora["energy"]
    fin = np.isfinite(E)
    assert (np.isfinite(e32) == fin).all()
    tol = energy_tol(E[fin])
    assert (np.abs(e32[fin] - E[fin]) <= tol).all()
    eg, _ = oracle.energies(m, s, p, A[fin])
    assert (np.abs(eg - E[fin]) <= tol).all()
    np.testing.assert_allclose(e64[fin], eg, rtol=1e-9, atol=1e-9)
    return int(fin.sum())


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_windowed_long_lists_against_oracle(ctx, seed):
    m, s = _sparse(seed)
    p = synth.Params(window=20, k_max=64, T=10)
    res = ctx.match(m, s, p)
    rows = np.arange(0, int(_np(res["energy32"]).shape[0]), 9).astype(np.int32)
    n = check(m, s, p, res, oracle.match(m, s, p, taus=rows), rows=rows)
    say(f"  sparse seed {seed}: {n} of {len(rows)} sampled offsets feasible")
    assert n > 0


def test_plan_on_sparse_scenes_equals_per_model(ctx):
    ms, ss = zip(*[_sparse(10 + q) for q in range(3)])
    p = synth.Params(window=20, k_max=64, T=10)
    pairs = np.array([(i, j) for i in range(3) for j in range(3)], np.int32)
    plan = stm.Plan(ctx, list(ms), list(ss), pairs, p)
    out = plan.run()
    n = 0
    for q, (i, j) in enumerate(pairs):
        e32, e64, _, A = [_np(x) for x in plan.pair_rows(out, q)]
        ref = ctx.match(ms[i], ss[j], p)
        np.testing.assert_array_equal(e32, ref["energy32"])
        np.testing.assert_array_equal(A, ref["assign"])
        np.testing.assert_array_equal(e64, ref["energy64"])
        n += int(np.isfinite(e32).sum())
    assert n > 0
    plan.close()


def test_dense_caps_on_sparse_scenes_against_oracle(ctx):
    """Every cap from 33 to 64 with the same lists as the oracle's."""
    m, s = _sparse(5, per=(1, 3))
    for K in (33, 48, 64):
        p = synth.Params(window=25, k_max=K, T=0)
        res = ctx.match(m, s, p)
        rows = np.arange(0, int(_np(res["energy32"]).shape[0]), 17).astype(np.int32)
        check(m, s, p, res, oracle.match(m, s, p, taus=rows), rows=rows)
