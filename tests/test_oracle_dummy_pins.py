"""Pins of the oracle's dummy assignments (Eq. 2: a model point may stay
unmatched, z_i = epsilon, at the unary cost W^d).

The paper fixes only U(epsilon) = W^d.  The reading taken for the rest: a
Delta term of D^t counts when both of its points are scene points, D^g when
all three are, and causality and closeness bind consecutive points that are
both scene points.  Pinned here by:
  * hand-derived energies of assignments with a dummy in the middle and at the
    end of the chain (small integers, exact in FP64);
  * brute force (the definition) against the C backward recursion on tiny
    random inputs, windowed and given lists;
  * W^d = 0: the all-dummy assignment has energy 0 and every term is >= 0;
  * lambda2 = 0 with disjoint windows: per point, the smaller of W^d and the
    nearest descriptor (scipy's cdist), empty windows forced to the dummy;
  * a very large W^d reproduces the matching without dummies wherever that
    one is feasible; the optimum is non-decreasing in W^d and never above the
    matching without dummies;
  * an exact planted copy keeps energy 0 and the identity assignment.
"""
import math

import numpy as np
from scipy.spatial.distance import cdist

import oracle
from oracle import energy as E
from paper_1505_00581_amd import synth

EPS = E.DUMMY


def _as_ints(z):
    return [int(v) for v in z]


def _hand_case():
    """Model t = 0..3 and one scene node per point.  Scene frames 0, 1, 3, 5;
    the scene triangle of nodes 0, 1, 2 is the model's triangle of points
    0, 1, 2 turned by 90 degrees and doubled (so its angles are equal in
    FP64: cross and dot products scale by 4 exactly).  Descriptor differences
    f_i - g_i: (3, 4), (0, 0), (0, 0), (6, 8), so U = 5, 0, 0, 10."""
    mxy = np.array([[0, 0], [4, 0], [4, 3], [9, 1]], np.float32)
    sxy = np.stack([-mxy[:, 1], mxy[:, 0]], 1) * 2.0 + np.array([10.0, 20.0])
    sxy[3] = [50.0, 50.0]
    mt = np.array([0, 1, 2, 3], np.int32)
    st = np.array([0, 1, 3, 5], np.int32)
    md = np.array([[3, 4], [1, 1], [2, 2], [6, 8]], np.float32)
    sd = np.array([[0, 0], [1, 1], [2, 2], [0, 0]], np.float32)
    model = synth.Points(mxy, mt, md)
    scene = synth.Points(sxy.astype(np.float32), st, sd, 6)
    return model, scene


def test_hand_energy_dummy_in_the_middle():
    model, scene = _hand_case()
    p = synth.Params(lambda1=0.5, lambda2=0.25, lambda3=5.0, T=10, w_dummy=2.0)
    # z = (n0, eps, n2, n3): triangle (2,1,0) holds the dummy at its middle,
    # so no term survives; triangle (3,2,1) keeps Delta(3,2) = |1 - 2| = 1.
    # E = 0.5 (5 + 2 + 0 + 10) + 0.25 * 1 = 8.75
    z = [0, EPS, 2, 3]
    assert E.energy(model, scene, z, p) == 8.75
    e, eu = oracle.energies(model, scene, p, np.array([z]))
    assert e[0] == 8.75 and eu[0] == 8.5


def test_hand_energy_dummy_at_the_end():
    model, scene = _hand_case()
    p = synth.Params(lambda1=0.5, lambda2=0.25, lambda3=5.0, T=10, w_dummy=2.0)
    # z = (n0, n1, n2, eps): triangle (2,1,0): Delta(2,1) = |1 - 2| = 1,
    # Delta(1,0) = 0, D^g = 0 (similar triangles); triangle (3,2,1): only
    # Delta(2,1) = 1 survives.  E = 0.5 (5 + 0 + 0 + 2) + 0.25 * 2 = 4.0
    z = [0, 1, 2, EPS]
    assert E.energy(model, scene, z, p) == 4.0
    e, _ = oracle.energies(model, scene, p, np.array([z]))
    assert e[0] == 4.0


def test_dummy_lifts_constraints_and_is_refused_when_disabled():
    model, scene = _hand_case()
    p = synth.Params(lambda1=0.5, lambda2=0.25, lambda3=5.0, T=2, w_dummy=2.0)
    # n1 (frame 1) -> n0 (frame 0) breaks causality; a dummy between them lifts it
    assert math.isinf(E.energy(model, scene, [1, 0, 2, 3], p))
    assert math.isinf(E.energy(model, scene, [1, EPS, 2, 3], p))  # (n2, n3) still too far
    assert math.isfinite(E.energy(model, scene, [1, EPS, 2, EPS], p))
    # T = 2: n1 (frame 1) -> n2 (frame 3) is too far apart; with n2 replaced by
    # the dummy, no constraint links n1 and n3 (frames 1 and 5)
    assert math.isinf(E.energy(model, scene, [0, 1, 2, 3], p))
    assert math.isfinite(E.energy(model, scene, [0, 1, EPS, 3], p))
    p_off = synth.Params(lambda1=0.5, lambda2=0.25, lambda3=5.0, T=10)
    assert math.isinf(E.energy(model, scene, [0, EPS, 2, 3], p_off))
    e, _ = oracle.energies(model, scene, p_off, np.array([[0, EPS, 2, 3]]))
    assert math.isinf(e[0])


def _tiny_dummy(seed):
    w = synth.tiny(seed, m=3 + seed % 3, k_max=3, T=[4, 2, 0][seed % 3])
    w.params.w_dummy = [0.05, 0.2, 0.5, 2.0][seed % 4]
    w.params.lambda1 = [0.6, 1.3][seed % 2]
    return w


def test_dummy_recursion_equals_brute_force_random_tiny():
    n_dummy = 0
    total = 0
    for seed in range(90):
        w = _tiny_dummy(seed)
        m, s, p = w.models[0], w.scenes[0], w.params
        r = oracle.match(m, s, p)
        eb, zs = E.brute_force_all(m, s, p)
        for j in range(eb.shape[0]):
            total += 1
            assert math.isfinite(eb[j])  # the all-dummy assignment is always allowed
            assert abs(r["energy"][j] - eb[j]) <= 1e-12 * max(1.0, abs(eb[j])), (seed, j)
            assert _as_ints(r["assign"][j]) in [_as_ints(z) for z in zs[j]], (seed, j)
            n_dummy += int((r["assign"][j] == EPS).any())
    assert total > 150 and n_dummy > 40, (total, n_dummy)


def test_dummy_recursion_on_given_lists_equals_brute_force():
    rng = np.random.default_rng(11)
    for seed in range(30):
        w = _tiny_dummy(500 + seed)
        m, s, p = w.models[0], w.scenes[0], w.params
        rows, cnts, bf = [], [], []
        for tau in E.offsets(m.t, s.n_frames):
            sub = [sorted(int(x) for x in c if rng.random() < 0.7)
                   for c in E.candidate_lists(m, s, p, tau)]
            row = np.full((m.n, p.k_max), -1, np.int32)
            cnt = np.zeros(m.n, np.int32)
            for i, c in enumerate(sub):
                row[i, :len(c)] = c
                cnt[i] = len(c)
            rows.append(row)
            cnts.append(cnt)
            bf.append(E.brute_force(m, s, p, tau, lists=sub))
        if not rows:
            continue
        got = oracle.match_lists(m, s, p, np.array(rows), np.array(cnts))
        for j, (e, zs) in enumerate(bf):
            assert abs(got["energy"][j] - e) <= 1e-12 * max(1.0, abs(e))
            assert _as_ints(got["assign"][j]) in [_as_ints(z) for z in zs]


def test_zero_dummy_cost_gives_zero_energy():
    for seed in range(10):
        w = synth.tiny(40 + seed, k_max=4)
        w.params.w_dummy = 0.0
        r = oracle.match(w.models[0], w.scenes[0], w.params)
        assert (r["energy"] == 0.0).all()
    w = synth.config1(0)
    w.params.w_dummy = 0.0
    r = oracle.match(w.models[0], w.scenes[0], w.params, taus=np.arange(0, 60, 7))
    assert (r["energy"] == 0.0).all()


def test_lambda2_zero_is_per_point_min_of_dummy_and_nearest_descriptor():
    rng = np.random.Generator(np.random.PCG64(5))
    m, W, wd = 7, 1, 0.33
    t = (np.arange(m) * (2 * W + 2)).astype(np.int32)  # disjoint windows
    model = synth.Points(rng.uniform(0, 50, (m, 2)).astype(np.float32), t,
                         synth.dirichlet_desc(rng, m, 12))
    nf = int(t[-1]) + 5
    sxy, st, sd = synth.clutter(rng, rng.integers(0, 4, nf), 50.0, 50.0, 12)
    scene = synth.assemble_scene([sxy], [st], [sd], nf)
    p = synth.Params(lambda1=0.6, lambda2=0.0, window=W, k_max=64, T=0, w_dummy=wd)
    r = oracle.match(model, scene, p)
    D = cdist(model.desc.astype(np.float64), scene.desc.astype(np.float64))
    n_empty = n_dummy = 0
    for j, tau in enumerate(r["taus"]):
        want, zs = 0.0, []
        for i in range(m):
            win = np.nonzero(np.abs(scene.t - (tau + t[i])) <= W)[0]
            n_empty += win.size == 0
            if win.size and D[i, win].min() < wd:
                k = win[np.argmin(D[i, win])]
                want += 0.6 * D[i, k]
                zs.append(int(k))
            else:
                want += 0.6 * wd
                zs.append(EPS)
        n_dummy += zs.count(EPS)
        assert abs(r["energy"][j] - want) < 1e-12 * max(1, want)
        assert _as_ints(r["assign"][j]) == zs
    assert n_empty > 0 and n_dummy > n_empty


def test_large_dummy_cost_reproduces_the_exact_matching_and_monotone():
    for seed in range(12):
        w = synth.tiny(700 + seed, k_max=4)
        m, s, p = w.models[0], w.scenes[0], w.params
        ex = oracle.match(m, s, p)
        prev = None
        for wd in (0.0, 0.1, 0.4, 1.5, 1e9):
            p.w_dummy = wd
            r = oracle.match(m, s, p)
            assert (r["energy"] <= ex["energy"]).all()
            if prev is not None:
                assert (r["energy"] >= prev).all()
            prev = r["energy"]
        fin = np.isfinite(ex["energy"])
        np.testing.assert_array_equal(r["energy"][fin], ex["energy"][fin])
        np.testing.assert_array_equal(r["assign"][fin], ex["assign"][fin])
        assert (r["energy"][~fin] >= 1e9 * p.lambda1).all()
        p.w_dummy = None


def test_exact_copy_keeps_zero_energy_with_dummies():
    rng = np.random.Generator(np.random.PCG64(21))
    mm = 8
    t = np.concatenate([[0], np.cumsum(rng.integers(1, 3, mm - 1))]).astype(np.int32)
    xy = np.round(rng.uniform(0, 40, (mm, 2))).astype(np.float32)
    model = synth.Points(xy, t, synth.dirichlet_desc(rng, mm, 16))
    n_frames, tau0 = int(t[-1]) + 10, 4
    cxy, ct, cd = synth.clutter(rng, np.full(n_frames, 3), 64.0, 64.0, 16)
    copy = (np.stack([-xy[:, 1], xy[:, 0]], 1) * 2.0 + np.array([100.0, 7.0])).astype(np.float32)
    s = synth.assemble_scene([np.round(cxy), copy], [ct, (tau0 + t).astype(np.int32)],
                             [cd, model.desc.copy()], n_frames)
    ids = [int(np.nonzero((s.t == tau0 + t[i]) & (s.xy == copy[i]).all(1))[0][0]) for i in range(mm)]
    p = synth.Params(window=1, k_max=64, T=10, w_dummy=0.05)
    r = oracle.match(model, s, p, taus=[tau0])
    assert r["energy"][0] == 0.0
    assert _as_ints(r["assign"][0]) == ids
