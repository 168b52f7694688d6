"""Pins of the oracle's trellis over a scene block (the paper's own problem,
Section 2.2: every model point may take any node of the block, under
causality and closeness).

* the recursion on whole-block lists = brute force over every assignment of
  tiny blocks (the definition), under the pairwise and the span reading of
  closeness, with infeasible cases;
* a sub-block is the same problem on fewer nodes: brute force with the
  block's nodes only;
* the trellis searches a superset of every per-offset window, so its optimum
  is at most the smallest windowed optimum (equal when the windows hold the
  trellis optimum);
* an exact similarity copy of the model inside random clutter has energy 0
  and is found.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from oracle import energy as E
from paper_1505_00581_amd import synth


def _tiny_block(seed, n_frames=6, per_frame=(0, 2), m=4):
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.integers(1, 3, size=m - 1)
    t = np.concatenate([[0], np.cumsum(gaps)]).astype(np.int32)
    model = synth.Points(rng.uniform(0, 40, (m, 2)).astype(np.float32), t, synth.dirichlet_desc(rng, m, 8))
    counts = rng.integers(per_frame[0], per_frame[1] + 1, size=n_frames)
    sxy, st, sd = synth.clutter(rng, counts, 40.0, 40.0, 8)
    return model, synth.assemble_scene([sxy], [st], [sd], n_frames)


@pytest.mark.parametrize("span", [False, True])
def test_trellis_equals_brute_force_on_tiny_blocks(span):
    feasible = infeasible = 0
    for seed in range(60):
        m, s = _tiny_block(3000 + seed, m=[3, 4][seed % 2])
        if s.n == 0 or s.n > 9:
            continue
        T = [3, 4, 0, 2, 5][seed % 5]
        p = synth.Params(T=T, closeness_span=span, lambda1=[0.6, 0.0][seed % 3 == 0])
        r = oracle.match_trellis(m, s, p)
        eb, zs = E.brute_force(m, s, p, 0, lists=[list(range(s.n))] * m.n)
        if math.isinf(eb):
            infeasible += 1
            assert math.isinf(r["energy"][0]) and (r["assign"][0] == -1).all()
        else:
            feasible += 1
            assert abs(r["energy"][0] - eb) <= 1e-12 * max(1.0, eb)
            assert [int(v) for v in r["assign"][0]] in [[int(v) for v in z] for z in zs]
    assert feasible > 15 and infeasible > 3


def test_sub_block_is_brute_force_on_its_nodes():
    checked = 0
    for seed in range(20):
        m, s = _tiny_block(3200 + seed, n_frames=9, m=3)
        if s.n < 6:
            continue
        b, e = 1, s.n - 1
        p = synth.Params(T=4)
        r = oracle.match_trellis(m, s, p, b, e)
        eb, zs = E.brute_force(m, s, p, 0, lists=[list(range(b, e))] * m.n)
        assert (math.isinf(eb) and math.isinf(r["energy"][0])) or abs(r["energy"][0] - eb) <= 1e-12 * max(1, eb)
        if math.isfinite(eb):
            assert [int(v) for v in r["assign"][0]] in [[int(v) for v in z] for z in zs]
            assert ((r["assign"][0] >= b) & (r["assign"][0] < e)).all()
        checked += 1
    assert checked >= 8


def test_trellis_bounded_by_windowed_optima():
    w = synth.config1(4)
    m, s = w.models[0], w.scenes[0]
    for T in (10, 4):
        p = dataclasses.replace(w.params, T=T)
        keep = s.t < 45
        s2 = synth.Points(s.xy[keep].copy(), s.t[keep].copy(), s.desc[keep].copy(), 45)
        win = oracle.match(m, s2, p)
        tr = oracle.match_trellis(m, s2, p)
        best = win["energy"].min()
        assert tr["energy"][0] <= best + 1e-12 * max(1.0, abs(best))
        # the trellis optimum is an admissible assignment of the same energy
        e, _ = oracle.energies(m, s2, p, tr["assign"])
        assert abs(e[0] - tr["energy"][0]) <= 1e-12 * max(1.0, abs(e[0]))


def test_exact_copy_in_clutter_is_found_with_zero_energy():
    rng = np.random.Generator(np.random.PCG64(77))
    m = synth.make_model(rng, 12, 160, 120, 10, frame_hi=18)
    nf = 60
    cxy, ct, cd = synth.clutter(rng, rng.integers(0, 2, nf), 160, 120)
    tau0, a = 23, 0.7
    R = np.array([[math.cos(a), -math.sin(a)], [math.sin(a), math.cos(a)]])
    copy = ((m.xy.astype(np.float64) - 80) @ R.T * 0.9 + 70).astype(np.float32)
    s = synth.assemble_scene([cxy, copy], [ct, (tau0 + m.t - m.t[0]).astype(np.int32)], [cd, m.desc.copy()], nf)
    p = synth.Params(T=10)
    r = oracle.match_trellis(m, s, p)
    assert r["energy"][0] < 1e-6
    z = r["assign"][0]
    assert (s.t[z] == tau0 + m.t - m.t[0]).all()
    np.testing.assert_allclose(s.xy[z], copy, atol=1e-6)


def test_stored_whole_video_rows_are_the_oracles():
    """The full-size trellis fixture (tests/golden/trellis_whole_video.json)
    holds the oracle's own results: its T = 10 rows recomputed now agree bit
    for bit (the row without a closeness limit takes the oracle minutes and is
    left to the script that wrote it), and every stored assignment's literal
    energy equals its stored optimum."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "trellis_whole_video.json")) as f:
        gold = json.load(f)
    w = synth.paper_blocks(0, n_models=50)
    s = w.scenes[0]
    for r in gold["rows"]:
        p = dataclasses.replace(w.params, T=r["T"])
        m = w.models[r["model"]]
        z = np.array([r["assign"]], np.int32)
        e, eu = oracle.energies(m, s, p, z)
        assert abs(e[0] - r["energy"]) <= 1e-12 * max(1.0, abs(r["energy"]))
        assert abs(eu[0] - r["energy_u"]) <= 1e-12 * max(1.0, abs(r["energy_u"]))
        if r["T"] == 10:
            o = oracle.match_trellis(m, s, p)
            assert o["energy"][0] == r["energy"]
            np.testing.assert_array_equal(o["assign"][0], z[0])
