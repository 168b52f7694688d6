"""Edge cases of the exact path on MI355X: empty offset ranges, scenes
shorter than the model, a one-point scene, zero-width windows, and a plan
whose pairs include one without offsets."""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
import paper_1505_00581_amd as stm
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


def _short_scene(s, n_frames):
    keep = s.t < n_frames
    return synth.Points(np.ascontiguousarray(s.xy[keep]), np.ascontiguousarray(s.t[keep]),
                        np.ascontiguousarray(s.desc[keep]), n_frames)


def test_empty_offset_range(ctx):
    w = synth.config1(0)
    m, s, p = w.models[0], w.scenes[0], w.params
    r = ctx.match(m, s, p, 5, 5)
    assert _np(r["energy32"]).shape == (0,) and _np(r["assign"]).shape == (0, m.n)


def test_scene_shorter_than_the_model(ctx):
    w = synth.config1(1)
    m, s, p = w.models[0], w.scenes[0], w.params
    short = _short_scene(s, int(m.t[-1] - m.t[0]))  # span frames: no full fit
    assert ctx.offsets(m, short) == (0, 0)
    r = ctx.match(m, short, p)
    assert _np(r["energy32"]).shape == (0,)
    with pytest.raises(stm.StmError, match="offset range"):
        ctx.match(m, short, p, 0, 1)


def test_one_point_scene(ctx):
    w = synth.config1(2)
    m, p = w.models[0], w.params
    s = synth.Points(np.array([[10.0, 20.0]], np.float32), np.array([40], np.int32),
                     w.scenes[0].desc[:1].copy(), 100)
    r = ctx.match(m, s, p)
    assert not np.isfinite(_np(r["energy32"])).any() and (_np(r["assign"]) == -1).all()
    pd = dataclasses.replace(p, w_dummy=0.3)
    r = ctx.match(m, s, pd)
    o = oracle.match(m, s, pd)
    e32 = _np(r["energy32"]).astype(np.float64)
    assert np.allclose(e32, o["energy"], rtol=1e-5, atol=1e-4)
    np.testing.assert_allclose(_np(r["energy64"]), oracle.energies(m, s, pd, _np(r["assign"]))[0], rtol=1e-9)
    assert ((_np(r["assign"]) == 0) | (_np(r["assign"]) == -2)).all()


def test_zero_width_window(ctx):
    w = synth.config1(3)
    m, s = w.models[0], w.scenes[0]
    p = dataclasses.replace(w.params, window=0)
    r = ctx.match(m, s, p)
    o = oracle.match(m, s, p)
    e32 = _np(r["energy32"]).astype(np.float64)
    fin = np.isfinite(o["energy"])
    assert (np.isfinite(e32) == fin).all()
    assert np.allclose(e32[fin], o["energy"][fin], rtol=1e-5, atol=1e-4)
    say(f"  W=0: {int(fin.sum())} of {fin.size} offsets feasible")


def test_plan_with_a_pair_without_offsets(ctx):
    w = synth.config1(4)
    m, s, p = w.models[0], w.scenes[0], w.params
    short = _short_scene(s, int(m.t[-1] - m.t[0]))
    plan = stm.Plan(ctx, [m], [s, short], np.array([[0, 0], [0, 1]], np.int32), p)
    assert plan.row_offsets.tolist()[1] == plan.row_offsets.tolist()[2]
    out = plan.run()
    e32, _, _, A = [_np(x) for x in plan.pair_rows(out, 0)]
    ref = ctx.match(m, s, p)
    np.testing.assert_array_equal(e32, ref["energy32"])
    np.testing.assert_array_equal(A, ref["assign"])
    assert _np(plan.pair_rows(out, 1)[0]).shape == (0,)
    plan.close()
