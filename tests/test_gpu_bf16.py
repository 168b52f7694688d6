"""Split-precision unary table (STM_UNARY_BF16) on MI355X.

* The BF16/MFMA table equals, to FP32 rounding, the FP64 distance of the
  BF16-rounded descriptors (rounded here independently, round-to-nearest-
  even on the float32 bit patterns); this also pins the MFMA lane layout.
* Against the exact FP32 descriptors the table differs only by the BF16
  rounding of the inputs.
* Matching with the BF16 table: the FP32 recursion's optimum stays within the
  error the BF16 table introduces; the returned assignments are re-scored in
  FP64 from the FP32 descriptors and can never beat the oracle's optimum.
"""
import sys

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
import paper_1505_00581_amd as stm
from parity_check import to_np
from paper_1505_00581_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def bf16_round(x):
    b = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


@pytest.fixture(scope="module")
def ctx():
    c = stm.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("which", ["c1", "c2_slice", "ragged"])
def test_bf16_table_equals_rounded_definition(ctx, which):
    if which == "c1":
        w = synth.config1(0)
        m, s = w.models[0], w.scenes[0]
    elif which == "c2_slice":
        w = synth.config2(0, n_models=1)
        m = w.models[0]
        s = w.scenes[0]
    else:  # dims and counts that are not multiples of the tile sizes
        rng = np.random.Generator(np.random.PCG64(5))
        m = synth.Points(rng.uniform(0, 9, (37, 2)).astype(np.float32), np.arange(37, dtype=np.int32),
                         synth.dirichlet_desc(rng, 37, 75))
        s = synth.Points(rng.uniform(0, 9, (301, 2)).astype(np.float32),
                         np.sort(rng.integers(0, 50, 301)).astype(np.int32),
                         synth.dirichlet_desc(rng, 301, 75), 50)
    p = synth.Params(unary_bf16=True)
    U = ctx.unary(m, s, p)
    fr = bf16_round(m.desc).astype(np.float64)
    gr = bf16_round(s.desc).astype(np.float64)
    ref = cdist(fr, gr)
    err = np.abs(U - ref)
    say(f"  {which}: max |U_bf16 - U_ref(rounded inputs)| = {err.max():.3e}")
    assert err.max() < 2e-5
    exact = cdist(m.desc.astype(np.float64), s.desc.astype(np.float64))
    rel = np.abs(U - exact) / np.maximum(exact, 1e-3)
    say(f"  {which}: max relative deviation from exact FP32 inputs = {rel.max():.3e}")
    assert rel.max() < 3e-2


def test_bf16_matching_against_oracle(ctx):
    w = synth.config2(0, n_models=2)
    s = w.scenes[0]
    p32 = w.params
    pbf = synth.Params(**{**p32.__dict__, "unary_bf16": True})
    errs, gaps, agree, n = [], [], 0, 0
    for mi, m in enumerate(w.models):
        b, e = ctx.offsets(m, s)
        taus = np.unique(np.concatenate([np.linspace(0, e - 1, 6).astype(int),
                                         [t for (mm, _, t) in w.planted if mm == mi][:2]])).astype(np.int32)
        r = ctx.match(m, s, pbf)
        ora = oracle.match(m, s, p32, taus=taus)
        E = ora["energy"]
        fin = np.isfinite(E)
        e32 = r["energy32"][taus].astype(np.float64)
        assert (np.isfinite(e32) == fin).all()
        errs += list(np.abs(e32[fin] - E[fin]) / np.abs(E[fin]))
        eg, _ = oracle.energies(m, s, p32, r["assign"][taus][fin])
        np.testing.assert_allclose(r["energy64"][taus][fin], eg, rtol=1e-9)
        gap = (eg - E[fin]) / np.abs(E[fin])
        assert (gap >= -1e-9).all()  # nothing beats the exact optimum
        gaps += list(gap)
        agree += int((r["assign"][taus][fin] == ora["assign"][fin]).all(1).sum())
        n += int(fin.sum())
    errs, gaps = np.array(errs), np.array(gaps)
    say(f"  BF16 unary vs FP64 oracle over {n} matchings: energy rel err max {errs.max():.3e} "
        f"mean {errs.mean():.3e}; re-scored gap max {gaps.max():.3e} mean {gaps.mean():.3e}; "
        f"assignment agreement {agree / n:.3f}")
    assert errs.max() < 5e-3 and errs.mean() < 1e-3
    assert gaps.mean() < 1e-3


def test_bf16_plan_equals_per_model_calls(ctx):
    """Split precision in a persistent plan (the unary tables of all models in
    one BF16 MFMA pass per scene, graph-replayed) gives the rows of one
    stm_match call per model bit for bit."""
    import torch
    w = synth.config2(3, n_models=3)
    s = w.scenes[0]
    keep = s.t < 400
    s = synth.Points(np.ascontiguousarray(s.xy[keep]), np.ascontiguousarray(s.t[keep]),
                     np.ascontiguousarray(s.desc[keep]), 400)
    pbf = synth.Params(**{**w.params.__dict__, "unary_bf16": True})
    ms = [m for m in w.models if int(m.t[-1] - m.t[0]) < 350]
    assert ms
    dms = [stm.DevicePoints.from_host(m) for m in ms]
    ds = stm.DevicePoints.from_host(s)
    plan = stm.Plan(ctx, dms, [ds], np.array([(i, 0) for i in range(len(ms))], np.int32), pbf)
    out = plan.run()
    out = plan.run(out)
    torch.cuda.synchronize()
    for q, dm in enumerate(dms):
        res = ctx.match(dm, ds, pbf)
        torch.cuda.synchronize()
        rows = plan.pair_rows(out, q)
        for got, key in zip(rows, ("energy32", "energy64", "energy_u64", "assign")):
            np.testing.assert_array_equal(to_np(got).reshape(to_np(res[key]).shape), to_np(res[key]))
    say(f"  BF16 plan over {len(ms)} models = per-model calls bit for bit")
    plan.close()
