"""Pins of the oracle's node-order reading of causality (flag STM_CAUSAL_NODE;
an alternative reading of Eq. 7): consecutive model points take increasing
scene node ids, z_{i-1} < z_i, which in a scene sorted by frame lets them
share a frame; closeness stays Eq. 8's.

* hand-counted admissible assignments on a scene with two points per frame,
  where the readings differ;
* one point per frame: node order is frame order, so both readings give the
  same optima and assignments;
* the node order admits every assignment the frame order does (a scene sorted
  by frame), so its optimum is at most the frame-order optimum;
* the C recursion under node order = brute force (Python energy);
* work counts under node order by enumeration.
"""
import dataclasses
import itertools
import math

import numpy as np

import oracle
from oracle import energy as E
from paper_1505_00581_amd import synth


def _scene(frames):
    rng = np.random.default_rng(9)
    n = len(frames)
    xy = rng.uniform(0, 50, (n, 2)).astype(np.float32)
    return synth.Points(xy, np.asarray(frames, np.int32), synth.dirichlet_desc(rng, n, 8), int(max(frames)) + 1)


def _model(m: int):
    rng = np.random.default_rng(13)
    return synth.Points(rng.uniform(0, 50, (m, 2)).astype(np.float32), np.arange(m, dtype=np.int32),
                        synth.dirichlet_desc(rng, m, 8))


def _count(m, s, p):
    zs = np.array(list(itertools.product(range(s.n), repeat=m.n)), np.int32)
    e_c, _ = oracle.energies(m, s, p, zs)
    e_py = np.array([E.energy(m, s, list(z), p) for z in zs])
    assert (np.isfinite(e_c) == np.isfinite(e_py)).all()
    return int(np.isfinite(e_c).sum())


# Scene nodes 0..4 in frames 0, 0, 1, 1, 2; M = 3.
#   Frame order: strictly increasing frames, only (f0, f1, f2): 2 x 2 x 1 = 4
#   (T = 0 or T = 2 alike).
#   Node order, T = 0: every increasing node triple, C(5, 3) = 10.
#   Node order, T = 2 (consecutive frames at most 1 apart): of the 10 triples only
#   (0, 1, 4) has a step of two frames -> 9.
#   Node order, T = 1 (equal frames only): (0, 1, x) needs x in frame 0 -> none;
#   (2, 3, x) needs a later node in frame 1 -> none -> 0.
def test_admissible_assignments_hand_counted():
    m, s = _model(3), _scene([0, 0, 1, 1, 2])
    base = synth.Params(window=5, k_max=16)
    assert _count(m, s, dataclasses.replace(base, T=0)) == 4
    assert _count(m, s, dataclasses.replace(base, T=2)) == 4
    assert _count(m, s, dataclasses.replace(base, T=0, causal_node=True)) == 10
    assert _count(m, s, dataclasses.replace(base, T=2, causal_node=True)) == 9
    assert _count(m, s, dataclasses.replace(base, T=1, causal_node=True)) == 0


def test_one_point_per_frame_is_frame_order():
    for seed in range(10):
        w = synth.tiny(4500 + seed, T=[4, 0][seed % 2], window=2, k_max=5, max_per_frame=1)
        m, s = w.models[0], w.scenes[0]
        assert (np.diff(s.t) > 0).all()
        a = oracle.match(m, s, w.params)
        b = oracle.match(m, s, dataclasses.replace(w.params, causal_node=True))
        np.testing.assert_array_equal(a["energy"], b["energy"])
        np.testing.assert_array_equal(a["assign"], b["assign"])


def test_node_optimum_at_most_frame_optimum_and_recursion_equals_brute_force():
    total = below = infeasible = 0
    for seed in range(100):
        T = [4, 3, 0, 2, 1][seed % 5]
        w = synth.tiny(4600 + seed, T=T, window=[1, 2][seed % 2], k_max=5, max_per_frame=3)
        m, s = w.models[0], w.scenes[0]
        pn = dataclasses.replace(w.params, causal_node=True)
        rn = oracle.match(m, s, pn)
        rf = oracle.match(m, s, w.params)
        eb, zs = E.brute_force_all(m, s, pn)
        for j in range(eb.shape[0]):
            a, b = rn["energy"][j], eb[j]
            total += 1
            if math.isinf(b):
                infeasible += 1
                assert math.isinf(a) and (rn["assign"][j] == -1).all() and math.isinf(rf["energy"][j])
                continue
            assert abs(a - b) <= 1e-12 * max(1.0, abs(b)), (seed, j, a, b)
            assert [int(v) for v in rn["assign"][j]] in [[int(v) for v in z] for z in zs[j]]
            assert a <= rf["energy"][j] + 1e-12 * max(1.0, abs(a))
            below += a < rf["energy"][j] - 1e-9
    assert total > 250 and below > 20 and infeasible > 5, (total, below, infeasible)


def test_work_counts_under_node_order_by_enumeration():
    for seed in range(8):
        w = synth.tiny(4800 + seed, T=[4, 2][seed % 2], window=2, k_max=5, max_per_frame=3)
        m, s = w.models[0], w.scenes[0]
        p = dataclasses.replace(w.params, causal_node=True)
        r = oracle.match(m, s, p)
        T = p.T
        pair = lambda a, b: a < b and (T <= 0 or int(s.t[b]) - int(s.t[a]) < T)  # noqa: E731
        dc = fc = dr = fr = 0
        for tau in r["taus"]:
            c = E.candidate_lists(m, s, p, int(tau))
            for i in range(1, m.n):
                for b in c[i - 1]:
                    for a in c[i]:
                        dc += 1
                        fc += pair(b, a)
            for i in range(2, m.n):
                for cc in c[i - 2]:
                    for b in c[i - 1]:
                        for a in c[i]:
                            dr += 1
                            fr += pair(cc, b) and pair(b, a)
        assert r["counts"] == dict(dense_cells=dc, feasible_cells=fc, dense_relax=dr, feasible_relax=fr)
