"""Pins of the CPU oracle to facts other than itself (runs without a GPU).

* brute force = the definition of the exact optimum (Section 2.2) on tiny
  random inputs, against the C literal backward recursion (Eq. 10-13);
* hand-derived closed forms of D^g and D^t (Eq. 4-6), tests/golden/;
* zero-energy planted copies (every term is >= 0, Eq. 1-6);
* special cases that reduce to a library routine (lambda2 = 0 -> per-point
  nearest descriptor by scipy's cdist), integer-valued D^t (lambda1 =
  lambda3 = 0), invariances (similarity transforms, time shifts, mirror);
* monotonicity in K, T and W; hand-derived candidate lists.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
from oracle import energy as E
from paper_1505_00581_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _close(a, b, rel=1e-12):
    if math.isinf(a) or math.isinf(b):
        return math.isinf(a) and math.isinf(b)
    return abs(a - b) <= rel * max(1.0, abs(b))


def _as_ints(z):
    return [int(v) for v in z]


# --------------------------------------------------------------------------
# Recursion == brute force (the definition) on tiny inputs.
# --------------------------------------------------------------------------

def _check_against_brute(w):
    m, s, p = w.models[0], w.scenes[0], w.params
    r = oracle.match(m, s, p)
    eb, zs = E.brute_force_all(m, s, p)
    assert r["energy"].shape == eb.shape
    n_inf = 0
    for j in range(eb.shape[0]):
        assert _close(r["energy"][j], eb[j]), (w.name, j, r["energy"][j], eb[j])
        if math.isinf(eb[j]):
            n_inf += 1
            assert (r["assign"][j] == -1).all()
        else:
            assert _as_ints(r["assign"][j]) in [_as_ints(z) for z in zs[j]]
    return eb.shape[0], n_inf


def test_recursion_equals_brute_force_random_tiny():
    total = infeasible = 0
    for seed in range(240):
        T = [4, 2, 0, 3][seed % 4]
        w = synth.tiny(seed, T=T)
        w.params.lambda1 = [0.6, 1.3, 0.1][seed % 3]
        w.params.lambda3 = [5.0, 0.7][seed % 2]
        n, ni = _check_against_brute(w)
        total += n
        infeasible += ni
    assert total > 500 and infeasible > 20, (total, infeasible)


def test_recursion_equals_brute_force_integer_coords_degenerate():
    # integer coordinates make coincident points (zero-length sides) likely
    for seed in range(60):
        w = synth.tiny(1000 + seed, int_coords=True, max_per_frame=3)
        w.scenes[0].xy[:] = np.round(w.scenes[0].xy / 8.0) * 8.0
        _check_against_brute(w)


def test_brute_force_sees_degenerate_triangles():
    # a triangle with coincident scene points: both scene angles are 0
    m = synth.Points(np.array([[0, 1], [0, 0], [1, 0]], np.float32), np.array([0, 1, 2], np.int32),
                     np.zeros((3, 4), np.float32))
    s = synth.Points(np.array([[3, 3], [3, 3], [5, 1]], np.float32), np.array([0, 1, 2], np.int32),
                     np.zeros((3, 4), np.float32), 3)
    p = synth.Params(lambda1=0.6, lambda2=0.2, lambda3=5.0, T=10, window=0, k_max=4)
    # model angle at j = +pi/2, at i = -pi/4; degenerate scene angles are 0
    want = 0.2 * 5.0 * math.sqrt((math.pi / 2) ** 2 + (math.pi / 4) ** 2)
    e, _ = oracle.energies(m, s, p, np.array([[0, 1, 2]]))
    assert abs(e[0] - want) < 1e-12
    assert abs(E.energy(m, s, [0, 1, 2], p) - want) < 1e-12


# --------------------------------------------------------------------------
# Closed forms (tests/golden/triangles.json).
# --------------------------------------------------------------------------

def _tri_case(c):
    m = synth.Points(np.array(c["model_xy"], np.float64).astype(np.float32),
                     np.array(c["model_t"], np.int32), np.full((3, 4), 0.25, np.float32))
    s = synth.Points(np.array(c["scene_xy"], np.float64).astype(np.float32),
                     np.array(c["scene_t"], np.int32), np.full((3, 4), 0.25, np.float32),
                     int(max(c["scene_t"])) + 1)
    return m, s


@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLD, "triangles.json")))["cases"],
                         ids=lambda c: c["name"])
def test_triangle_closed_forms(case):
    m, s = _tri_case(case)
    dg = eval(case["dg_expr"], {"math": math})
    p = synth.Params(lambda1=0.6, lambda2=0.2, lambda3=5.0, T=10)
    want_d = case["dt"] + p.lambda3 * dg
    # float32 storage of the coordinates moves angles by < 1e-7 rad
    got_py = E.triangle_cost(m, s, 2, 2, 1, 0, p.lambda3)
    assert abs(got_py - want_d) < 2e-6
    e, eu = oracle.energies(m, s, p, np.array([[0, 1, 2]]))
    assert eu[0] == 0.0  # identical descriptors
    assert abs(e[0] - p.lambda2 * want_d) < 1e-6


def test_unsigned_reading_would_differ_on_mirror():
    # the mirrored case discriminates oriented from unsigned angles
    c = json.load(open(os.path.join(GOLD, "triangles.json")))["cases"]
    m, s = _tri_case(c[1])
    unsigned = math.sqrt((math.pi / 6) ** 2 + (math.pi / 12) ** 2)
    got = E.triangle_cost(m, s, 2, 2, 1, 0, 1.0)
    assert abs(got - unsigned) > 1.0


# --------------------------------------------------------------------------
# Zero-energy planted copies.
# --------------------------------------------------------------------------

def _planted_scene(model, tau0, xy_copy, desc_copy, seed, n_frames, per_frame=3, width=64):
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = np.full(n_frames, per_frame)
    cxy, ct, cd = synth.clutter(rng, counts, float(width), float(width), model.dim)
    cxy = np.round(cxy)  # integers keep every difference exact
    ts = tau0 + model.t - model.t[0]
    s = synth.assemble_scene([cxy, xy_copy], [ct, ts.astype(np.int32)], [cd, desc_copy], n_frames)
    # node id of each planted point
    ids = []
    for i in range(model.n):
        hit = np.nonzero((s.t == ts[i]) & (s.xy == xy_copy[i]).all(1))[0]
        ids.append(int(hit[0]))
    return s, ids


def _int_model(seed, m=8):
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.concatenate([[0], np.cumsum(rng.integers(1, 3, m - 1))]).astype(np.int32)
    xy = np.round(rng.uniform(0, 40, (m, 2))).astype(np.float32)
    return synth.Points(xy, t, synth.dirichlet_desc(rng, m, 16))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_exact_similarity_copy_has_zero_energy(seed):
    model = _int_model(seed)
    # rotation by 90 degrees, scale 2, integer translation: exact in float
    xy = model.xy.astype(np.float64)
    copy = np.stack([-xy[:, 1], xy[:, 0]], 1) * 2.0 + np.array([100.0, 7.0])
    n_frames = int(model.t[-1]) + 12
    tau0 = 5
    s, ids = _planted_scene(model, tau0, copy.astype(np.float32), model.desc.copy(), seed + 50,
                            n_frames)
    p = synth.Params(window=1, k_max=64, T=10)
    r = oracle.match(model, s, p, taus=[tau0])
    assert r["energy"][0] == 0.0
    assert _as_ints(r["assign"][0]) == ids
    # D^t only sees relative times, so offsets within the window of tau0 still
    # contain the whole copy (energy 0); offsets farther away cannot
    allr = oracle.match(model, s, p)
    near = np.abs(allr["taus"] - tau0) <= p.window
    assert (allr["energy"][near] == 0.0).all()
    assert (allr["energy"][~near] > 0).all()


def test_generic_similarity_copy_near_zero_and_mirror_is_not():
    model = _int_model(7, m=10)
    xy = model.xy.astype(np.float64)
    a = 0.7
    R = np.array([[math.cos(a), -math.sin(a)], [math.sin(a), math.cos(a)]])
    copy = (xy @ R.T) * 1.3 + np.array([50.5, 60.25])
    n_frames = int(model.t[-1]) + 6
    s, ids = _planted_scene(model, 2, copy.astype(np.float32), model.desc.copy(), 99, n_frames)
    p = synth.Params(window=1, k_max=64, T=10)
    r = oracle.match(model, s, p, taus=[2])
    assert r["energy"][0] < 1e-4
    assert _as_ints(r["assign"][0]) == ids
    # mirrored copy: oriented angles flip sign, so the energy of the copy is large
    mir = copy.copy()
    mir[:, 0] = -mir[:, 0] + 400.0
    s2, ids2 = _planted_scene(model, 2, mir.astype(np.float32), model.desc.copy(), 99, n_frames)
    e_mir, _ = oracle.energies(model, s2, p, np.array([ids2]))
    assert e_mir[0] > 0.5


# --------------------------------------------------------------------------
# Special cases that reduce to textbook routines.
# --------------------------------------------------------------------------

def test_lambda2_zero_is_per_point_nearest_descriptor():
    rng = np.random.Generator(np.random.PCG64(3))
    m = 6
    W = 1
    # model frames spaced 2W+1 apart: windows are disjoint, so order is automatic
    t = (np.arange(m) * (2 * W + 2)).astype(np.int32)
    model = synth.Points(rng.uniform(0, 50, (m, 2)).astype(np.float32), t,
                         synth.dirichlet_desc(rng, m, 12))
    nf = int(t[-1]) + 5
    sxy, st, sd = synth.clutter(rng, rng.integers(1, 5, nf), 50.0, 50.0, 12)
    scene = synth.assemble_scene([sxy], [st], [sd], nf)
    p = synth.Params(lambda1=0.6, lambda2=0.0, window=W, k_max=64, T=0)
    r = oracle.match(model, scene, p)
    D = cdist(model.desc.astype(np.float64), scene.desc.astype(np.float64))  # Euclidean
    for j, tau in enumerate(r["taus"]):
        want, zs = 0.0, []
        for i in range(m):
            f = tau + t[i]
            win = np.nonzero(np.abs(scene.t - f) <= W)[0]
            if win.size == 0:
                want = math.inf
                break
            k = win[np.argmin(D[i, win])]
            want += 0.6 * D[i, k]
            zs.append(int(k))
        if math.isinf(want):
            assert math.isinf(r["energy"][j])
        else:
            assert abs(r["energy"][j] - want) < 1e-12 * max(1, want)
            assert _as_ints(r["assign"][j]) == zs


def test_time_only_energy_is_integer_multiple_of_lambda2():
    for seed in range(20):
        w = synth.tiny(300 + seed, T=0)
        w.params.lambda1, w.params.lambda3 = 0.0, 0.0
        r = oracle.match(w.models[0], w.scenes[0], w.params)
        for e in r["energy"]:
            if math.isfinite(e):
                q = e / w.params.lambda2
                assert abs(q - round(q)) < 1e-9


def test_pure_time_shifted_copy_has_zero_time_energy():
    model = _int_model(11)
    s, ids = _planted_scene(model, 3, model.xy.copy(), model.desc.copy(), 5,
                            int(model.t[-1]) + 8)
    p = synth.Params(lambda1=0.0, lambda3=0.0, window=1, k_max=64, T=10)
    r = oracle.match(model, s, p, taus=[3])
    assert r["energy"][0] == 0.0


# --------------------------------------------------------------------------
# Invariances.
# --------------------------------------------------------------------------

def _cfg1_small(seed):
    w = synth.config1(seed)
    return w.models[0], w.scenes[0], w.params


def test_exact_similarity_transform_of_scene_leaves_energies_unchanged():
    w = synth.tiny(17, int_coords=True)
    m, s, p = w.models[0], w.scenes[0], w.params
    r0 = oracle.match(m, s, p)
    xy = s.xy.astype(np.float64)
    s2 = synth.Points(np.ascontiguousarray((np.stack([-xy[:, 1], xy[:, 0]], 1) * 4.0 + 12.0)
                                           .astype(np.float32)), s.t, s.desc, s.n_frames)
    r1 = oracle.match(m, s2, p)
    np.testing.assert_array_equal(r0["energy"], r1["energy"])
    np.testing.assert_array_equal(r0["assign"], r1["assign"])


def test_time_shift_of_scene_shifts_offsets():
    m, s, p = _cfg1_small(2)
    taus = np.arange(0, 20, dtype=np.int32)
    r0 = oracle.match(m, s, p, taus=taus)
    sh = 7
    s2 = synth.Points(s.xy, (s.t + sh).astype(np.int32), s.desc, s.n_frames + sh)
    r1 = oracle.match(m, s2, p, taus=taus + sh)
    np.testing.assert_array_equal(r0["energy"], r1["energy"])
    np.testing.assert_array_equal(r0["assign"], r1["assign"])


def test_permutation_within_frames_when_cap_not_binding():
    w = synth.tiny(23, max_per_frame=3)
    m, s, p = w.models[0], w.scenes[0], w.params
    p.k_max = 64
    r0 = oracle.match(m, s, p)
    rng = np.random.Generator(np.random.PCG64(0))
    perm = np.arange(s.n)
    for f in np.unique(s.t):
        idx = np.nonzero(s.t == f)[0]
        perm[idx] = rng.permutation(idx)
    s2 = synth.Points(s.xy[perm], s.t[perm], s.desc[perm], s.n_frames)
    r1 = oracle.match(m, s2, p)
    np.testing.assert_allclose(r0["energy"], r1["energy"], rtol=1e-12)


# --------------------------------------------------------------------------
# Monotonicity.
# --------------------------------------------------------------------------

def test_monotone_in_k_t_and_w():
    m, s, p = _cfg1_small(4)
    taus = np.arange(0, 71, 5, dtype=np.int32)
    base = oracle.match(m, s, p, taus=taus)["energy"]
    import dataclasses
    bigger_k = oracle.match(m, s, dataclasses.replace(p, k_max=24), taus=taus)["energy"]
    bigger_t = oracle.match(m, s, dataclasses.replace(p, T=0), taus=taus)["energy"]
    bigger_w = oracle.match(m, s, dataclasses.replace(p, window=3, k_max=64), taus=taus)["energy"]
    smaller_k = oracle.match(m, s, dataclasses.replace(p, k_max=6), taus=taus)["energy"]
    assert (bigger_k <= base + 1e-12).all()
    assert (bigger_t <= base + 1e-12).all()
    assert (bigger_w <= oracle.match(m, s, dataclasses.replace(p, k_max=64), taus=taus)["energy"]
            + 1e-12).all()
    assert (smaller_k >= base - 1e-12).all()


# --------------------------------------------------------------------------
# Candidate lists (tests/golden/candidates.json) and work counts.
# --------------------------------------------------------------------------

def test_candidate_lists_hand_derived():
    g = json.load(open(os.path.join(GOLD, "candidates.json")))
    counts = np.array(g["scene_frame_counts"])
    st = np.repeat(np.arange(counts.size), counts).astype(np.int32)
    scene = synth.Points(np.zeros((st.size, 2), np.float32), st,
                         np.zeros((st.size, 2), np.float32), counts.size)
    model = synth.Points(np.zeros((2, 2), np.float32), np.array(g["model_t"], np.int32),
                         np.zeros((2, 2), np.float32))
    for c in g["cases"]:
        p = synth.Params(window=c["W"], k_max=c["K"])
        got_py = E.candidates(model.t, scene.t, c["tau"], c["point"], c["W"], c["K"])
        got_c = oracle.candidate_list(model, scene, p, c["tau"], c["point"])
        assert list(got_py) == c["expected"], c
        assert list(got_c) == c["expected"], c


def _ranges(rs):
    return [n for lo, hi in rs for n in range(lo, hi + 1)]


def test_density_capped_lists_hand_derived():
    """The density cap (rho over frames f-1..f+1, rounding, the clamp to [8, 64]
    and k_max, scene edges) against hand-derived lists, through the C oracle,
    its Python twin and the Python cap alone."""
    g = json.load(open(os.path.join(GOLD, "candidates.json")))["density"]
    counts = np.array(g["scene_frame_counts"])
    st = np.repeat(np.arange(counts.size), counts).astype(np.int32)
    scene = synth.Points(np.zeros((st.size, 2), np.float32), st,
                         np.zeros((st.size, 2), np.float32), counts.size)
    model = synth.Points(np.zeros((2, 2), np.float32), np.array(g["model_t"], np.int32),
                         np.zeros((2, 2), np.float32))
    W = g["W"]
    for c in g["cases"]:
        want = _ranges(c["expected_ranges"])
        assert len(want) == c["K"], c
        assert int(np.count_nonzero(np.abs(st - c["frame"]) <= 1)) == c["rho"], c
        assert E.density_k(st, c["frame"], c["k_max"]) == c["K"], c
        p = synth.Params(window=W, k_max=c["k_max"], k_density=True)
        got_py = E.candidates(model.t, scene.t, c["tau"], c["point"], W, c["k_max"], True)
        got_c = oracle.candidate_list(model, scene, p, c["tau"], c["point"])
        assert list(got_py) == want, c
        assert list(got_c) == want, c
    c = g["no_density_case"]
    p = synth.Params(window=W, k_max=c["k_max"], k_density=False)
    want = _ranges(c["expected_ranges"])
    assert list(oracle.candidate_list(model, scene, p, c["tau"], c["point"])) == want
    assert list(E.candidates(model.t, scene.t, c["tau"], c["point"], W, c["k_max"], False)) == want


def test_work_counts_by_enumeration():
    for seed in range(10):
        w = synth.tiny(500 + seed)
        m, s, p = w.models[0], w.scenes[0], w.params
        r = oracle.match(m, s, p)
        dc = fc = dr = fr = 0
        for tau in r["taus"]:
            c = E.candidate_lists(m, s, p, int(tau))
            for i in range(1, m.n):
                for b in c[i - 1]:
                    for a in c[i]:
                        dc += 1
                        fc += E.admissible(int(s.t[b]), int(s.t[a]), p.T)
            for i in range(2, m.n):
                for cc in c[i - 2]:
                    for b in c[i - 1]:
                        for a in c[i]:
                            dr += 1
                            fr += (E.admissible(int(s.t[cc]), int(s.t[b]), p.T)
                                   and E.admissible(int(s.t[b]), int(s.t[a]), p.T))
        assert r["counts"] == dict(dense_cells=dc, feasible_cells=fc, dense_relax=dr,
                                   feasible_relax=fr)


def test_c_and_python_energy_agree_on_config1_assignments():
    m, s, p = _cfg1_small(0)
    r = oracle.match(m, s, p)
    for j in range(0, len(r["taus"]), 7):
        if math.isfinite(r["energy"][j]):
            e_py = E.energy(m, s, _as_ints(r["assign"][j]), p)
            assert abs(e_py - r["energy"][j]) <= 1e-12 * max(1.0, e_py)


def _lists_array(lists, M, K):
    row = np.full((M, K), -1, np.int32)
    cnt = np.zeros(M, np.int32)
    for i, c in enumerate(lists):
        row[i, :len(c)] = c
        cnt[i] = len(c)
    return row, cnt


def test_recursion_on_given_lists_equals_brute_force():
    """The explicit-list entry point (used to check pruned matchings) against
    enumeration over random subsets of the windowed lists."""
    rng = np.random.default_rng(7)
    feasible = 0
    for seed in range(40):
        w = synth.tiny(200 + seed)
        m, s, p = w.models[0], w.scenes[0], w.params
        rows, cnts, bf = [], [], []
        for tau in E.offsets(m.t, s.n_frames):
            sub = [sorted(int(x) for x in c if rng.random() < 0.75)
                   for c in E.candidate_lists(m, s, p, tau)]
            r, c = _lists_array(sub, m.n, p.k_max)
            rows.append(r)
            cnts.append(c)
            bf.append(E.brute_force(m, s, p, tau, lists=sub))
        if not rows:
            continue
        got = oracle.match_lists(m, s, p, np.array(rows), np.array(cnts))
        for j, (e, zs) in enumerate(bf):
            if not np.isfinite(e):
                assert not np.isfinite(got["energy"][j])
                assert (got["assign"][j] == -1).all()
                continue
            feasible += 1
            assert abs(got["energy"][j] - e) <= 1e-9 * max(1.0, abs(e))
            assert [int(x) for x in got["assign"][j]] in [list(z) for z in zs]
    assert feasible >= 40


def test_recursion_on_windowed_lists_equals_match():
    w = synth.config1(3)
    m, s, p = w.models[0], w.scenes[0], w.params
    taus = np.arange(0, len(E.offsets(m.t, s.n_frames)), 7, dtype=np.int32)
    rows, cnts = [], []
    for tau in taus:
        r, c = _lists_array([oracle.candidate_list(m, s, p, int(tau), i) for i in range(m.n)], m.n,
                            p.k_max)
        rows.append(r)
        cnts.append(c)
    a = oracle.match(m, s, p, taus=taus)
    b = oracle.match_lists(m, s, p, np.array(rows), np.array(cnts))
    np.testing.assert_array_equal(a["energy"], b["energy"])
    np.testing.assert_array_equal(a["assign"], b["assign"])
