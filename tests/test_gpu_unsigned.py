"""The unsigned reading of the triangle angles (STM_ANGLE_UNSIGNED; the angles
of Eq. 6 as magnitudes in [0, pi]) on MI355X against the FP64 oracle under
the same reading.

Covered: tiny cases and a small workload at every offset, lists shorter than
64 (the variant uses the 64-slot layout for every K), the span reading on
top, coincident points (the degenerate re-run), a mirrored planted copy found
at energy 0, the persistent plan and given lists equal to per-model calls bit
for bit, sampled offsets of the realistic scene bounded by the oriented
optimum, and the entry points that refuse the flag.
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


def _uns(p, **kw):
    return dataclasses.replace(p, angle_unsigned=True, **kw)


def _cut(s, n_frames):
    keep = s.t < n_frames
    return synth.Points(np.ascontiguousarray(s.xy[keep]), np.ascontiguousarray(s.t[keep]),
                        np.ascontiguousarray(s.desc[keep]), n_frames)


def test_tiny_cases_against_oracle(ctx):
    feas = 0
    for seed in range(40):
        w = synth.tiny(3100 + seed, T=[4, 5, 3, 0][seed % 4], window=2, k_max=5)
        m, s = w.models[0], w.scenes[0]
        p = _uns(w.params)
        st = check(m, s, p, ctx.match(m, s, p), oracle.match(m, s, p))
        feas += st["feasible"]
    assert feas > 50


@pytest.mark.parametrize("span", [False, True])
def test_small_workload_all_offsets(ctx, span):
    w = synth.config1(5)
    m, s = w.models[0], w.scenes[0]
    p = _uns(w.params, closeness_span=span)
    st = check(m, s, p, ctx.match(m, s, p), oracle.match(m, s, p))
    say(f"  config-1 workload, span={span}: {st}")
    assert st["feasible"] > 0


@pytest.mark.parametrize("k_max", [12, 40, 64])
def test_list_lengths(ctx, k_max):
    w = synth.config2(51, n_models=1)
    m, s = w.models[0], _cut(w.scenes[0], 260)
    p = _uns(w.params, k_max=k_max)
    res = ctx.match(m, s, p)
    n = res["energy32"].shape[0]
    taus = np.unique(np.linspace(0, n - 1, 5).astype(np.int32))
    st = check(m, s, p, res, oracle.match(m, s, p, taus=taus), rows=taus)
    say(f"  K={k_max}: {st}")
    assert st["feasible"] > 0


def test_degenerate_points(ctx):
    feas = 0
    for seed in range(20):
        w = synth.tiny(3300 + seed, T=5, window=2, k_max=5, int_coords=True, max_per_frame=3)
        m, s = w.models[0], w.scenes[0]
        s = synth.Points(np.round(s.xy / 8) * 8, s.t, s.desc, s.n_frames)
        p = _uns(w.params)
        feas += check(m, s, p, ctx.match(m, s, p), oracle.match(m, s, p))["feasible"]
    assert feas > 20


def test_mirrored_planted_copy(ctx):
    rng = np.random.default_rng(17)
    m = 12
    mxy = (np.round(rng.uniform(20, 140, (m, 2)) * 4) / 4).astype(np.float32)
    mt = np.cumsum(np.r_[0, rng.integers(1, 3, m - 1)]).astype(np.int32)
    desc = synth.dirichlet_desc(rng, m, synth.DIM)
    model = synth.Points(mxy, mt, desc)
    tau0, F = 20, 80
    counts = rng.integers(2, 6, F)
    cxy, ct, cd = synth.clutter(rng, counts, 160.0, 160.0)
    sxy = np.concatenate([np.stack([160 - mxy[:, 0], mxy[:, 1]], 1), cxy]).astype(np.float32)
    st = np.concatenate([mt + tau0, ct]).astype(np.int32)
    sd = np.concatenate([desc, cd]).astype(np.float32)
    order = np.argsort(st, kind="stable")
    scene = synth.Points(sxy[order], st[order], sd[order], F)
    planted = np.argsort(order)[:m].astype(np.int32)
    p = synth.Params(T=10, window=2, k_max=64)
    ru = ctx.match(model, scene, _uns(p), tau_begin=tau0, tau_end=tau0 + 1)
    ro = ctx.match(model, scene, p, tau_begin=tau0, tau_end=tau0 + 1)
    assert abs(float(ru["energy32"][0])) <= float(energy_tol(0.0))  # exact energy 0
    np.testing.assert_array_equal(ru["assign"][0], planted)
    assert float(ro["energy32"][0]) > 1e-2


def test_plan_and_lists_equal_per_model(ctx):
    w = synth.config2(52, n_models=3)
    s = _cut(w.scenes[0], 300)
    p = _uns(w.params, T=8)
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
        cand, cnt = ctx.candidates(m, s, p)
        lst = ctx.match_lists(m, s, p, cand, cnt)
        for k in ("energy32", "energy64", "assign"):
            np.testing.assert_array_equal(lst[k], res[k])
    plan.close()


def test_realistic_scene_sampled_and_bounded(ctx):
    import torch
    w = synth.config2(0, n_models=1)
    m, s, p = w.models[0], w.scenes[0], w.params
    dm, ds = stm.DevicePoints.from_host(m), stm.DevicePoints.from_host(s)
    ru = ctx.match(dm, ds, _uns(p))
    ro = ctx.match(dm, ds, p)
    torch.cuda.synchronize()
    eu, eo = to_np(ru["energy32"]).astype(np.float64), to_np(ro["energy32"]).astype(np.float64)
    fin = np.isfinite(eo)
    assert (np.isfinite(eu) == fin).all()
    # per triangle the unsigned D^g is at most the oriented one: so is the optimum
    assert (eu[fin] <= eo[fin] + energy_tol(eo[fin])).all()
    n = eu.shape[0]
    taus = np.unique(np.linspace(0, n - 1, 12).astype(np.int32))
    res = {k: to_np(v)[taus] for k, v in ru.items() if k in ("energy32", "energy64", "energy_u64", "assign")}
    st = check(m, s, _uns(p), res, oracle.match(m, s, _uns(p), taus=taus))
    say(f"  realistic scene: {st}, optimum below the oriented one at {(eu[fin] < eo[fin] - 1e-4).mean():.3f}")


def test_refusals(ctx):
    w = synth.config1(0)
    m, s, p = w.models[0], w.scenes[0], _uns(w.params)
    with pytest.raises(stm.StmError) as ei:
        ctx.match(m, s, dataclasses.replace(p, w_dummy=0.3))
    assert ei.value.code == stm.STM_EUNSUPPORTED
    pr = stm.Pruner(ctx, m.dim)
    pr.set_params(synth.pruner_init(m.dim, 0))
    with pytest.raises(stm.StmError) as ei:
        pr.match(m, s, p, topk=8)
    assert ei.value.code == stm.STM_EUNSUPPORTED
    plan = stm.Plan(ctx, [m], [s], np.array([[0, 0]], np.int32), p)
    with pytest.raises(stm.StmError) as ei:
        plan.run_pruned(pr, 8)
    assert ei.value.code == stm.STM_EUNSUPPORTED
    plan.close()
    pr.close()
    with pytest.raises(stm.StmError) as ei:
        stm.Trellis(ctx, [m], s, p)
    assert ei.value.code == stm.STM_EUNSUPPORTED
