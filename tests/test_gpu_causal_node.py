"""Causality by scene node order (STM_CAUSAL_NODE; Eq. 7 read as z_{i-1} <
z_i, equal frames allowed, closeness as Eq. 8) on MI355X against the FP64
oracle under the same reading.

Every recursion variant takes it through its schedule (each row a group of
its own): the per-offset kernel on 16-, 32- and 64-slot lists, the packed
schedule of sparse scenes, the persistent plan, and the degenerate re-run.
Covered: tiny cases, a small workload at every offset for several T, work
counts, one point per frame equal bit for bit to the frame-order reading, the
optimum at every offset of the realistic scene at or below the frame-order
optimum (node order admits a superset) with sampled offsets against the
oracle, plan = per-model calls, and the entry points that refuse the flag.
"""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
import paper_1505_00581_amd as stm
from parity_check import check, to_np
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


def _node(p, **kw):
    return dataclasses.replace(p, causal_node=True, **kw)


def _cut(s, n_frames):
    keep = s.t < n_frames
    return synth.Points(np.ascontiguousarray(s.xy[keep]), np.ascontiguousarray(s.t[keep]),
                        np.ascontiguousarray(s.desc[keep]), n_frames)


def test_tiny_cases_against_oracle(ctx):
    feas = 0
    for seed in range(60):
        w = synth.tiny(5100 + seed, T=[4, 2, 0, 1, 3][seed % 5], window=2, k_max=5, max_per_frame=3)
        m, s = w.models[0], w.scenes[0]
        p = _node(w.params)
        st = check(m, s, p, ctx.match(m, s, p), oracle.match(m, s, p))
        feas += st["feasible"]
    assert feas > 80


@pytest.mark.parametrize("T", [10, 3, 2, 1, 0])
def test_small_workload_all_offsets_and_counts(ctx, T):
    w = synth.config1(7)
    m, s = w.models[0], w.scenes[0]
    p = _node(w.params, T=T)
    ora = oracle.match(m, s, p)
    st = check(m, s, p, ctx.match(m, s, p), ora)
    assert ctx.count_work(m, s, p) == ora["counts"]
    say(f"  T={T}: {st}")
    if T in (10, 0):
        assert st["feasible"] > 0


@pytest.mark.parametrize("k_max", [12, 24, 64])
def test_list_capacities(ctx, k_max):
    w = synth.config2(61, n_models=1)
    m, s = w.models[0], _cut(w.scenes[0], 260)
    p = _node(w.params, k_max=k_max, T=6)
    res = ctx.match(m, s, p)
    n = res["energy32"].shape[0]
    taus = np.unique(np.linspace(0, n - 1, 5).astype(np.int32))
    st = check(m, s, p, res, oracle.match(m, s, p, taus=taus), rows=taus)
    say(f"  K={k_max}: {st}")
    assert st["feasible"] > 0


def test_sparse_scene_packed_schedule(ctx):
    rng = np.random.Generator(np.random.PCG64(64))
    m = synth.make_model(rng, 24, 160, 120, 10)
    nf = int(m.t[-1]) + 60
    s, _ = synth.make_scene(rng, [m], nf, rng.integers(0, 4, nf), 160, 120, 1)
    p = synth.Params(window=12, k_max=64, T=10, causal_node=True)
    res = ctx.match(m, s, p)
    n = res["energy32"].shape[0]
    taus = np.unique(np.linspace(0, n - 1, 8).astype(np.int32))
    st = check(m, s, p, res, oracle.match(m, s, p, taus=taus), rows=taus)
    say(f"  sparse: {st}")
    assert st["feasible"] > 0


def test_degenerate_points(ctx):
    feas = 0
    for seed in range(20):
        w = synth.tiny(5300 + seed, T=5, window=2, k_max=5, int_coords=True, max_per_frame=3)
        m, s = w.models[0], w.scenes[0]
        s = synth.Points(np.round(s.xy / 8) * 8, s.t, s.desc, s.n_frames)
        p = _node(w.params)
        feas += check(m, s, p, ctx.match(m, s, p), oracle.match(m, s, p))["feasible"]
    assert feas > 20


def test_one_point_per_frame_equals_frame_order(ctx):
    rng = np.random.Generator(np.random.PCG64(65))
    m = synth.make_model(rng, 20, 160, 120, 10)
    nf = int(m.t[-1]) + 80
    sxy, st, sd = synth.clutter(rng, rng.integers(0, 2, nf), 160.0, 120.0)
    s = synth.assemble_scene([sxy], [st], [sd], nf)
    assert (np.diff(s.t) > 0).all()
    p = synth.Params(window=3, k_max=64, T=10)
    a, b = ctx.match(m, s, p), ctx.match(m, s, _node(p))
    for k in ("energy32", "energy64", "assign"):
        np.testing.assert_array_equal(a[k], b[k])


def test_plan_equals_per_model(ctx):
    w = synth.config2(62, n_models=3)
    s = _cut(w.scenes[0], 300)
    p = _node(w.params, T=8)
    ms = [m for m in w.models if int(m.t[-1] - m.t[0]) < 250]
    assert ms
    plan = stm.Plan(ctx, ms, [s], np.array([[i, 0] for i in range(len(ms))], np.int32), p)
    out = plan.run()
    for q, m in enumerate(ms):
        res = ctx.match(m, s, p)
        rows = plan.pair_rows(out, q)
        np.testing.assert_array_equal(to_np(rows[0]), res["energy32"])
        np.testing.assert_array_equal(to_np(rows[1]), res["energy64"])
        np.testing.assert_array_equal(to_np(rows[3]).reshape(res["assign"].shape), res["assign"])
    plan.close()


def test_realistic_scene_bounded_and_sampled(ctx):
    import torch
    w = synth.config2(0, n_models=1)
    m, s, p = w.models[0], w.scenes[0], w.params
    dm, ds = stm.DevicePoints.from_host(m), stm.DevicePoints.from_host(s)
    rn = ctx.match(dm, ds, _node(p))
    rf = ctx.match(dm, ds, p)
    torch.cuda.synchronize()
    en, ef = to_np(rn["energy32"]).astype(np.float64), to_np(rf["energy32"]).astype(np.float64)
    fin = np.isfinite(ef)
    assert np.isfinite(en[fin]).all()
    assert (en[fin] <= ef[fin] + energy_tol(ef[fin])).all()
    n = en.shape[0]
    taus = np.unique(np.linspace(0, n - 1, 10).astype(np.int32))
    res = {k: to_np(v)[taus] for k, v in rn.items() if k in ("energy32", "energy64", "energy_u64", "assign")}
    st = check(m, s, _node(p), res, oracle.match(m, s, _node(p), taus=taus))
    say(f"  realistic scene: {st}, optimum below the frame-order one at {(en[fin] < ef[fin] - 1e-4).mean():.3f}")


def test_refusals(ctx):
    w = synth.config1(0)
    m, s, p = w.models[0], w.scenes[0], _node(w.params)
    for q in (dataclasses.replace(p, w_dummy=0.3), dataclasses.replace(p, closeness_span=True)):
        with pytest.raises(stm.StmError) as ei:
            ctx.match(m, s, q)
        assert ei.value.code == stm.STM_EUNSUPPORTED
    cand, cnt = ctx.candidates(m, s, w.params)
    with pytest.raises(stm.StmError) as ei:
        ctx.match_lists(m, s, p, cand, cnt)
    assert ei.value.code == stm.STM_EUNSUPPORTED
    pr = stm.Pruner(ctx, m.dim)
    with pytest.raises(stm.StmError) as ei:
        pr.match(m, s, p, topk=8)
    assert ei.value.code == stm.STM_EUNSUPPORTED
    pr.close()
    with pytest.raises(stm.StmError) as ei:
        stm.Trellis(ctx, [m], s, p)
    assert ei.value.code == stm.STM_EUNSUPPORTED
