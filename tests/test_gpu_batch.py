"""The batched persistent launch (stm_plan_*) on MI355X.

* Every pair's rows equal, bit for bit, the per-pair stm_match results (the
  same forward pass, terms and tie rules run on the same inputs);
* sampled items agree with the FP64 oracle (density caps, uneven models);
* graph replays are identical, a new output buffer re-captures, host-pointer
  plans work, degenerate matchings inside a batch are redone exactly;
* the autotuner picks a valid shape, writes its cache and reads it back;
* every launch shape (waves, workgroups per CU, batch, dense or packed
  schedule) gives the same results, and a shape whose scratch cannot be
  allocated is refused with the plan left as it was.
"""
import json
import os
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


def _small_batch(seed=0, n_models=5, n_scenes=2):
    w = synth.config3(seed, n_models=n_models, n_scenes=n_scenes)
    # shorter scenes keep the per-pair reference and the oracle quick
    scenes = []
    for s in w.scenes:
        keep = s.t < 260
        scenes.append(synth.Points(np.ascontiguousarray(s.xy[keep]), np.ascontiguousarray(s.t[keep]),
                                   np.ascontiguousarray(s.desc[keep]), 260))
    models = [m for m in w.models if int(m.t[-1]) < 200]
    return models, scenes, w.params


def _all_pairs(nm, ns):
    return np.array([(i, j) for i in range(nm) for j in range(ns)], np.int32)


@pytest.mark.parametrize("device", [True, False])
def test_batch_equals_per_pair_matching(ctx, device):
    import torch
    models, scenes, p = _small_batch(1)
    pairs = _all_pairs(len(models), len(scenes))
    if device:
        dm = [stm.DevicePoints.from_host(m) for m in models]
        ds = [stm.DevicePoints.from_host(s) for s in scenes]
        plan = stm.Plan(ctx, dm, ds, pairs, p)
    else:
        plan = stm.Plan(ctx, models, scenes, pairs, p)
    out = plan.run()
    if device:
        torch.cuda.synchronize()
    n = 0
    for q, (i, j) in enumerate(pairs):
        e32, e64, eu, A = [_np(x) for x in plan.pair_rows(out, q)]
        ref = ctx.match(models[i], scenes[j], p)
        np.testing.assert_array_equal(e32, ref["energy32"])
        np.testing.assert_array_equal(A, ref["assign"])
        np.testing.assert_array_equal(e64, ref["energy64"])
        np.testing.assert_array_equal(eu, ref["energy_u64"])
        n += e32.size
    say(f"  {len(pairs)} pairs, {n} matchings identical to per-pair launches")
    plan.close()


def test_batch_against_oracle_and_replay(ctx):
    import torch
    models, scenes, p = _small_batch(2)
    pairs = _all_pairs(len(models), len(scenes))
    dm = [stm.DevicePoints.from_host(m) for m in models]
    ds = [stm.DevicePoints.from_host(s) for s in scenes]
    plan = stm.Plan(ctx, dm, ds, pairs, p)
    out = plan.run()
    out2 = plan.run(out)           # replay into the same buffers
    torch.cuda.synchronize()
    first = {k: _np(v).copy() for k, v in out.items()}
    out3 = plan.run()              # new buffers: captured again
    torch.cuda.synchronize()
    for k in ("energy32", "energy64", "assign"):
        np.testing.assert_array_equal(first[k], _np(out3[k]))
    checked = 0
    for q, (i, j) in enumerate(pairs):
        e32, e64, eu, A = [_np(x) for x in plan.pair_rows(out3, q)]
        if e32.size == 0:
            continue
        taus = np.unique(np.linspace(0, e32.size - 1, 3).astype(np.int32))
        ora = oracle.match(models[i], scenes[j], p, taus=taus)
        E = ora["energy"]
        fin = np.isfinite(E)
        assert (np.isfinite(e32[taus]) == fin).all()
        tol = energy_tol(E[fin])
        assert (np.abs(e32[taus][fin] - E[fin]) <= tol).all()
        eg, _ = oracle.energies(models[i], scenes[j], p, A[taus][fin])
        assert (np.abs(eg - E[fin]) <= tol).all()
        np.testing.assert_allclose(e64[taus][fin], eg, rtol=1e-9)
        checked += int(fin.sum())
    say(f"  {checked} sampled batch matchings agree with the oracle")
    assert checked > 5
    plan.close()


def test_degenerate_matchings_inside_a_batch(ctx):
    models, scenes = [], []
    for seed in range(6):
        w = synth.tiny(1000 + seed, int_coords=True, max_per_frame=3, n_frames=12)
        w.scenes[0].xy[:] = np.round(w.scenes[0].xy / 8.0) * 8.0
        w.models[0].xy[:] = np.round(w.models[0].xy / 8.0) * 8.0
        models.append(w.models[0])
        scenes.append(w.scenes[0])
    p = synth.tiny(1000).params
    pairs = np.array([(i, i) for i in range(6)] + [(0, 3), (4, 1)], np.int32)
    plan = stm.Plan(ctx, models, scenes, pairs, p)
    out = plan.run()
    for q, (i, j) in enumerate(pairs):
        e32, _, _, A = plan.pair_rows(out, q)
        ref = ctx.match(models[i], scenes[j], p)
        np.testing.assert_array_equal(e32, ref["energy32"])
        np.testing.assert_array_equal(A, ref["assign"])
        ora = oracle.match(models[i], scenes[j], p)
        fin = np.isfinite(ora["energy"])
        assert (np.isfinite(e32) == fin).all()
        assert (np.abs(e32[fin] - ora["energy"][fin]) <= energy_tol(ora["energy"][fin])).all()
    plan.close()


def test_autotune_and_cache(ctx, tmp_path):
    models, scenes, p = _small_batch(3, n_models=4, n_scenes=1)
    pairs = _all_pairs(len(models), len(scenes))
    plan = stm.Plan(ctx, models, scenes, pairs, p)
    ref = plan.run()
    ref = {k: v.copy() for k, v in ref.items()}
    cache = str(tmp_path / "tune.json")
    ch = plan.autotune(cache, n_sample=64)
    assert ch["waves"] in (4, 8, 16) and 1 <= ch["wgs_per_cu"] <= 3 and not ch["cached"]
    assert 1 <= ch["batch"] <= min(8, ch["waves"]) and ch["packed"] in (0, 1)
    data = json.load(open(cache))
    assert len(data) == 1 and list(data.values())[0]["waves"] == ch["waves"]
    ch2 = plan.autotune(cache)
    assert ch2["cached"] and all(ch2[k] == ch[k] for k in ("waves", "wgs_per_cu", "batch", "packed"))
    out = plan.run()
    for k in ("energy32", "energy64", "assign"):
        np.testing.assert_array_equal(out[k], ref[k])
    # results do not depend on the launch shape
    for w_, g in [(4, 3), (16, 2), (8, 1)]:
        plan.set_tuning(w_, g)
        out = plan.run()
        for k in ("energy32", "energy64", "assign"):
            np.testing.assert_array_equal(out[k], ref[k])
    plan.close()


def test_shapes_and_refused_scratch(ctx):
    """Batches of 1..8 items per workgroup and both schedule variants give the
    same rows; with plan allocations refused (the library's failure injection)
    a shape that needs more value-table scratch fails with STM_ENOMEM and the
    plan keeps its shape, scratch and results."""
    import torch
    models, scenes, p = _small_batch(6, n_models=4, n_scenes=1)
    pairs = _all_pairs(len(models), len(scenes))
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    stride = (max(m.n for m in models) - 2) * p.k_max * p.k_max
    one = n_cu * 3 * stride * 4   # bytes of the value tables at 3 workgroups per CU, batch 1
    say(f"n_cu {n_cu}, scratch of one item per workgroup at 3 per CU: {one} bytes")
    os.environ["STM_FAILPOINT_PLAN_ALLOC"] = str(one)
    try:
        plan = stm.Plan(ctx, models, scenes, pairs, p)   # the scratch of larger batches is refused
    finally:
        del os.environ["STM_FAILPOINT_PLAN_ALLOC"]
    assert plan.shape()["batch"] == 1
    ref = {k: v.copy() for k, v in plan.run().items()}
    for w_, g, b, sc in [(8, 3, 1, 0), (8, 1, 2, 1), (4, 3, 1, 1), (16, 1, 1, 0)]:
        plan.set_shape(w_, g, b, sc)
        eff = plan.shape()
        assert eff["batch"] == b and eff["packed"] == sc and eff["wgs_per_cu"] == g
        out = plan.run()
        for k in ("energy32", "energy64", "assign"):
            np.testing.assert_array_equal(out[k], ref[k])
    plan.set_shape(8, 3, 1, 0)
    before = plan.shape()
    os.environ["STM_FAILPOINT_PLAN_ALLOC"] = "0"
    try:
        with pytest.raises(stm.StmError) as ei:
            plan.set_shape(8, 3, 4, 0)   # four times the scratch it has
        assert ei.value.code == stm.STM_ENOMEM
        assert plan.shape() == before
        plan.set_tuning(8, 2)            # keeps the batch request; fits the scratch it has
        assert plan.shape()["wgs_per_cu"] == 2
    finally:
        del os.environ["STM_FAILPOINT_PLAN_ALLOC"]
    out = plan.run()
    for k in ("energy32", "energy64", "assign"):
        np.testing.assert_array_equal(out[k], ref[k])
    # allocations allowed again: larger batches, dense and packed, same rows
    for w_, g, b, sc in [(8, 3, 8, 0), (8, 2, 4, 1), (16, 2, 8, 0)]:
        plan.set_shape(w_, g, b, sc)
        assert plan.shape()["batch"] == b
        out = plan.run()
        for k in ("energy32", "energy64", "assign"):
            np.testing.assert_array_equal(out[k], ref[k])
    plan.close()


def test_invalid_pairs_rejected(ctx):
    models, scenes, p = _small_batch(4, n_models=2, n_scenes=1)
    with pytest.raises(stm.StmError):
        stm.Plan(ctx, models, scenes, np.array([[0, 1]], np.int32), p)
    bad = synth.Points(scenes[0].xy, scenes[0].t[::-1].copy(), scenes[0].desc, scenes[0].n_frames)
    with pytest.raises(stm.StmError):
        stm.Plan(ctx, models, [bad], np.array([[0, 0]], np.int32), p)


def test_profiled_plan_runs(ctx):
    """Timed plan runs launch the kernels directly with two events around the
    recursion; the results do not change and each run adds one timed launch."""
    models, scenes, p = _small_batch(5, n_models=3, n_scenes=1)
    pairs = _all_pairs(len(models), len(scenes))
    plan = stm.Plan(ctx, models, scenes, pairs, p)
    ref = {k: v.copy() for k, v in plan.run().items()}
    ctx.profile_enable(True)
    for _ in range(3):
        out = plan.run()
        for k in ("energy32", "energy64", "assign"):
            np.testing.assert_array_equal(out[k], ref[k])
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    assert prof["dp_launches"] == 3 and prof["dp_ms"] > 0
    assert prof["dp_matchings"] == 3 * plan.n_rows
    out = plan.run()   # graph replay again
    np.testing.assert_array_equal(out["energy32"], ref["energy32"])
    plan.close()
