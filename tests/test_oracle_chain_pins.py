"""Pins of the oracle's multiple-points variant 2 (Section 4, Table 4):
independent single-point chains, distance averaged over the chains.

* the chain split by hand on a small frame/confidence pattern (ties by point
  order, chains of fewer than 3 points dropped);
* a model with one point per frame is a single chain: the variant equals the
  exact matching;
* exact copies of every chain planted at one offset give mean energy 0 and
  the identity assignment there.
"""
import numpy as np

import oracle
from oracle import chains as C
from paper_1505_00581_amd import synth


def test_chain_split_by_hand():
    t = np.array([0, 0, 0, 1, 2, 2, 4, 5, 5, 5], np.int32)
    sal = np.array([0.2, 0.9, 0.5, 0.1, 0.3, 0.3, 0.7, 0.1, 0.8, 0.4], np.float32)
    # frame 0 ranks points 1, 2, 0; frame 2 ties 4 and 5 (point order); frame 5 ranks 8, 9, 7.
    # The third chain (0, 7) has two points and is dropped.
    assert C.build_chains(t, sal, 3) == [[1, 3, 4, 6, 8], [2, 5, 9]]
    assert C.build_chains(t, sal, 1) == [[1, 3, 4, 6, 8]]
    assert C.build_chains(t, None, 3) == [[0, 3, 4, 6, 7], [1, 5, 8]]


def test_one_point_per_frame_is_the_exact_matching():
    w = synth.config1(2)
    m, s, p = w.models[0], w.scenes[0], w.params
    sal = np.random.default_rng(0).uniform(size=m.n)
    got = C.match_chains(m, s, p, sal, 3)
    ref = oracle.match(m, s, p)
    assert got["chains"] == [list(range(m.n))]
    np.testing.assert_array_equal(got["energy"], ref["energy"])
    np.testing.assert_array_equal(got["assign"], ref["assign"])


def test_exact_copies_of_every_chain_give_zero():
    rng = np.random.Generator(np.random.PCG64(4))
    ft = np.array([0, 1, 3, 4, 6, 7, 9, 10], np.int32)
    t = np.repeat(ft, 2)
    m = t.shape[0]
    xy = np.round(rng.uniform(0, 40, (m, 2))).astype(np.float32)
    model = synth.Points(xy, t, synth.dirichlet_desc(rng, m, 16))
    sal = rng.uniform(size=m)
    n_frames, tau0 = int(t[-1]) + 10, 4
    cxy, ct, cd = synth.clutter(rng, np.full(n_frames, 3), 64.0, 64.0, 16)
    copy = (np.stack([-xy[:, 1], xy[:, 0]], 1) * 2.0 + np.array([100.0, 7.0])).astype(np.float32)
    s = synth.assemble_scene([np.round(cxy), copy], [ct, (tau0 + t).astype(np.int32)],
                             [cd, model.desc.copy()], n_frames)
    ids = [int(np.nonzero((s.t == tau0 + t[i]) & (s.xy == copy[i]).all(1))[0][0]) for i in range(m)]
    p = synth.Params(window=1, k_max=64, T=10)
    r = C.match_chains(model, s, p, sal, 3, taus=[tau0, tau0 + 2])
    assert len(r["chains"]) == 2
    assert r["energy"][0] == 0.0
    assert [int(v) for v in r["assign"][0]] == ids
    assert r["energy"][1] > 0.0


def test_points_of_dropped_chains_are_marked():
    w = synth.multipoint(3, n_models=1, frames=(10, 14), per_frame=3, n_frames=50,
                         clutter_per_frame=3, window=1, k_max=8)
    m, s, p = w.models[0], w.scenes[0], w.params
    r = C.match_chains(m, s, p, w.saliency[0], 2, taus=[0, 5])
    used = sorted(q for c in r["chains"] for q in c)
    unused = sorted(set(range(m.n)) - set(used))
    assert unused  # frames with 3 points leave their least salient point out
    assert (r["assign"][:, unused] == C.UNCHAINED).all()
    assert (r["assign"][:, used] != C.UNCHAINED).all()
