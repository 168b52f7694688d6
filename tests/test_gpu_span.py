"""The span reading of temporal closeness (STM_CLOSENESS_SPAN; Section 3.4,
Eq. 14) on MI355X against the FP64 oracle under the same reading.

Every recursion variant that takes it is covered: the per-offset kernel on
16-, 32- and 64-slot lists, the packed schedule of sparse scenes, the
persistent plan, given lists, and the degenerate re-run; lambda3 = 0 makes
the excluded terms NaN instead of +inf inside the minimum.  At full size
the optimum is checked at every offset against the pairwise optima that
bound it: E*(pairwise, T - 1) <= E*(span, T) <= E*(pairwise, ceil(T / 2)).
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


def _span(p, **kw):
    return dataclasses.replace(p, closeness_span=True, **kw)


def _cut(s, n_frames):
    keep = s.t < n_frames
    return synth.Points(np.ascontiguousarray(s.xy[keep]), np.ascontiguousarray(s.t[keep]),
                        np.ascontiguousarray(s.desc[keep]), n_frames)


@pytest.mark.parametrize("T", [10, 6, 4, 3, 2, 0])
def test_plain_workload_all_offsets(ctx, T):
    w = synth.config1(3)
    m, s = w.models[0], w.scenes[0]
    p = _span(w.params, T=T)
    say(f"[span plain T={T}]")
    res = ctx.match(m, s, p)
    st = check(m, s, p, res, oracle.match(m, s, p))
    say(f"  {st}")
    if T == 2:  # a triangle spans at least 2 frames
        assert st["feasible"] == 0
    elif T in (0, 6, 10):  # (T = 3, 4 are tighter than this model's own triangle spans)
        assert st["feasible"] > 0


def test_tiny_cases_against_oracle(ctx):
    feas = 0
    for seed in range(40):
        w = synth.tiny(2100 + seed, T=[4, 5, 3, 6][seed % 4], window=2, k_max=5)
        m, s = w.models[0], w.scenes[0]
        p = _span(w.params)
        st = check(m, s, p, ctx.match(m, s, p), oracle.match(m, s, p))
        feas += st["feasible"]
    assert feas > 50


@pytest.mark.parametrize("k_max", [12, 24, 64])
def test_list_capacities_and_lambda3_zero(ctx, k_max):
    w = synth.config2(41, n_models=1)
    m, s = w.models[0], _cut(w.scenes[0], 260)
    for p in (_span(w.params, k_max=k_max, T=6), _span(w.params, k_max=k_max, T=6, lambda3=0.0)):
        res = ctx.match(m, s, p)
        n = res["energy32"].shape[0]
        taus = np.unique(np.linspace(0, n - 1, 5).astype(np.int32))
        st = check(m, s, p, res, oracle.match(m, s, p, taus=taus), rows=taus)
        say(f"  K={k_max} lambda3={p.lambda3}: {st}")


def test_plan_and_lists_equal_per_model(ctx):
    w = synth.config2(42, n_models=3)
    s = _cut(w.scenes[0], 300)
    p = _span(w.params, T=8)
    ms = [m for m in w.models if int(m.t[-1] - m.t[0]) < 250]
    assert ms
    plan = stm.Plan(ctx, ms, [s], np.array([[i, 0] for i in range(len(ms))], np.int32), p)
    out = plan.run()
    for q, m in enumerate(ms):
        res = ctx.match(m, s, p)
        rows = plan.pair_rows(out, q)
        np.testing.assert_array_equal(to_np(rows[0]), res["energy32"])
        np.testing.assert_array_equal(to_np(rows[3]).reshape(res["assign"].shape), res["assign"])
        cand, cnt = ctx.candidates(m, s, p)
        lst = ctx.match_lists(m, s, p, cand, cnt)
        for k in ("energy32", "energy64", "assign"):
            np.testing.assert_array_equal(lst[k], res[k])
    plan.close()


def test_sparse_scene_packed_schedule(ctx):
    # about one point per frame and wide windows: the packed schedule
    rng = np.random.Generator(np.random.PCG64(44))
    m = synth.make_model(rng, 24, 160, 120, 10)
    nf = int(m.t[-1]) + 60
    s, _ = synth.make_scene(rng, [m], nf, rng.integers(0, 4, nf), 160, 120, 1)
    p = synth.Params(window=12, k_max=64, T=10, closeness_span=True)
    res = ctx.match(m, s, p)
    n = res["energy32"].shape[0]
    taus = np.unique(np.linspace(0, n - 1, 8).astype(np.int32))
    st = check(m, s, p, res, oracle.match(m, s, p, taus=taus), rows=taus)
    say(f"  sparse: {st}")
    assert st["feasible"] > 0


def test_degenerate_points_under_span(ctx):
    # integer coordinates make coincident points, which the degenerate
    # variant re-runs
    feas = 0
    for seed in range(20):
        w = synth.tiny(2300 + seed, T=5, window=2, k_max=5, int_coords=True, max_per_frame=3)
        m, s = w.models[0], w.scenes[0]
        s = synth.Points(np.round(s.xy / 8) * 8, s.t, s.desc, s.n_frames)
        p = _span(w.params)
        feas += check(m, s, p, ctx.match(m, s, p), oracle.match(m, s, p))["feasible"]
    assert feas > 20


def test_realistic_sizes_bounded_by_pairwise_optima(ctx):
    import torch
    w = synth.config2(0, n_models=2)
    s, p = w.scenes[0], w.params
    ds = stm.DevicePoints.from_host(s)
    T = 10
    for m in w.models:
        dm = stm.DevicePoints.from_host(m)
        e = {}
        for key, q in (("lo", dataclasses.replace(p, T=T - 1)), ("span", _span(p, T=T)),
                       ("hi", dataclasses.replace(p, T=(T + 1) // 2))):
            r = ctx.match(dm, ds, q)
            torch.cuda.synchronize()
            e[key] = to_np(r["energy32"]).astype(np.float64)
            if key == "span":
                res, A = r, to_np(r["assign"])
        fin = np.isfinite(e["span"])
        tol = energy_tol(np.where(fin, e["span"], 1.0))
        assert (e["lo"] <= e["span"] + tol).all()
        assert (e["span"] <= e["hi"] + tol).all()
        # every returned assignment keeps causality and the span limit
        tz = s.t[A[fin]].astype(np.int64)
        assert (np.diff(tz, axis=1) > 0).all() and ((tz[:, 2:] - tz[:, :-2]) < T).all()
        taus = np.unique(np.linspace(0, e["span"].size - 1, 4).astype(np.int32))
        st = check(m, s, _span(p, T=T), res, oracle.match(m, s, _span(p, T=T), taus=taus), rows=taus)
        say(f"  M={m.n}: {st}, strictly between: {(e['lo'][fin] < e['span'][fin]).mean():.3f}")


def test_work_counts_under_span(ctx):
    w = synth.config1(2)
    m, s = w.models[0], w.scenes[0]
    for T in (4, 6, 10):
        p = _span(w.params, T=T)
        assert ctx.count_work(m, s, p) == oracle.match(m, s, p)["counts"]
