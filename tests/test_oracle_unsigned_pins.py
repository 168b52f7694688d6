"""Pins of the oracle's unsigned reading of the triangle angles (flag
STM_ANGLE_UNSIGNED; an alternative reading of Eq. 6): each angle of a triangle
is the magnitude of the oriented one, in [0, pi], so a triangle and its mirror
image have the same angles.

* hand-derived triangles: a right isosceles triangle against its mirror image
  (oriented D^g = pi sqrt(5) / 2, unsigned 0), and against a triangle of other
  angles and that triangle's mirror image (both readings by hand), through both
  the Python and the C energy;
* a mirrored planted copy: energy 0 at its offset, with the planted nodes,
  under the unsigned reading, and above 0 under the oriented one;
* an inequality fixed by the definitions: | |a| - |b| | <= |wrap(a - b)| for
  angles in (-pi, pi], so every triangle's unsigned D^g is at most its
  oriented one and the unsigned optimum is at most the oriented optimum;
* the C recursion under the unsigned reading = brute force (Python energy).
"""
import dataclasses
import math

import numpy as np

import oracle
from oracle import energy as E
from paper_1505_00581_amd import synth


def _pts(xy, t, desc=None):
    xy = np.asarray(xy, np.float32)
    n = xy.shape[0]
    d = np.full((n, 4), 0.25, np.float32) if desc is None else np.asarray(desc, np.float32)
    return synth.Points(xy, np.asarray(t, np.int32), d, int(np.max(t)) + 1)


# Model triangle k=(0,0), j=(1,0), i=(1,1) (points 0, 1, 2 of the chain):
#   angle at j from ray j->i (0,1) to ray j->k (-1,0): cross = 1, dot = 0 -> +pi/2;
#   angle at i from ray i->j (0,-1) to ray i->k (-1,-1): cross = -1, dot = 1 -> -pi/4.
# Its mirror image x -> -x has the angles -pi/2 and +pi/4.  Oriented:
#   wrap(pi/2 + pi/2) = pi, wrap(-pi/4 - pi/4) = -pi/2, D^g = sqrt(pi^2 + pi^2/4) = pi sqrt(5)/2;
# unsigned: both differences 0.
# The triangle k=(0,0), j=(2,0), i=(3,sqrt 3) (isosceles, apex j) has at j the
# angle from ray j->i (1, sqrt 3) to ray j->k (-2, 0): cross = 2 sqrt 3, dot = -2
# -> 2pi/3; at i from ray i->j (-1, -sqrt 3) to ray i->k (-3, -sqrt 3): cross =
# -2 sqrt 3, dot = 6 -> -pi/6.  Its mirror image k=(0,0), j=(-2,0), i=(-3,sqrt 3)
# has -2pi/3 and +pi/6.  Against the model, unsigned: pi/2 - 2pi/3 = -pi/6 and
# pi/4 - pi/6 = pi/12, D^g = pi sqrt(5)/12 for both; oriented, the triangle:
# wrap(pi/2 - 2pi/3) = -pi/6, wrap(-pi/4 + pi/6) = -pi/12, pi sqrt(5)/12; its
# mirror: wrap(pi/2 + 2pi/3) = -5pi/6, wrap(-pi/4 - pi/6) = -5pi/12, 5 pi sqrt(5)/12.
MODEL = _pts([[0, 0], [1, 0], [1, 1]], [0, 1, 2])


def _triangle_cost(scene_xy, unsigned):
    s = _pts(scene_xy, [0, 1, 2])
    p = synth.Params(lambda1=0.0, lambda2=1.0, lambda3=1.0, T=0, window=0, k_max=1, angle_unsigned=unsigned)
    py = E.triangle_cost(MODEL, s, 2, 2, 1, 0, 1.0, unsigned)
    c, _ = oracle.energies(MODEL, s, p, np.array([[0, 1, 2]], np.int32))
    assert abs(c[0] - py) <= 1e-12
    return py


def test_mirror_triangle_by_hand():
    mirror = [[0, 0], [-1, 0], [-1, 1]]
    assert abs(_triangle_cost(mirror, False) - math.pi * math.sqrt(5) / 2) <= 1e-12
    assert _triangle_cost(mirror, True) <= 1e-15


def test_other_triangles_by_hand():
    r3 = math.sqrt(3)
    tri, mirror = [[0, 0], [2, 0], [3, r3]], [[0, 0], [-2, 0], [-3, r3]]
    small, large = math.pi * math.sqrt(5) / 12, 5 * math.pi * math.sqrt(5) / 12
    tol = 1e-6  # float32 coordinates
    assert abs(_triangle_cost(tri, True) - small) <= tol
    assert abs(_triangle_cost(tri, False) - small) <= tol
    assert abs(_triangle_cost(mirror, True) - small) <= tol
    assert abs(_triangle_cost(mirror, False) - large) <= tol


def test_mirrored_planted_copy_has_zero_energy_only_unsigned():
    rng = np.random.default_rng(5)
    m = 6
    mxy = (np.round(rng.uniform(10, 60, (m, 2)) * 4) / 4).astype(np.float32)  # exact mirror images
    mt = np.array([0, 2, 3, 5, 6, 8], np.int32)
    desc = synth.dirichlet_desc(rng, m, 8)
    model = synth.Points(mxy, mt, desc)
    tau0, F = 4, 20
    # scene: the model mirrored (x -> 80 - x) at frames mt + tau0, plus clutter
    cxy = rng.uniform(0, 80, (30, 2)).astype(np.float32)
    ct = rng.integers(0, F, 30).astype(np.int32)
    cd = synth.dirichlet_desc(rng, 30, 8)
    sxy = np.concatenate([np.stack([80 - mxy[:, 0], mxy[:, 1]], 1), cxy]).astype(np.float32)
    st = np.concatenate([mt + tau0, ct]).astype(np.int32)
    sd = np.concatenate([desc, cd]).astype(np.float32)
    order = np.argsort(st, kind="stable")
    scene = synth.Points(sxy[order], st[order], sd[order], F)
    planted = np.argsort(order)[:m]  # new ids of the mirrored model points
    p = synth.Params(T=0, window=1, k_max=16)
    pu = dataclasses.replace(p, angle_unsigned=True)
    ru = oracle.match(model, scene, pu, taus=[tau0])
    ro = oracle.match(model, scene, p, taus=[tau0])
    assert ru["energy"][0] <= 1e-9
    np.testing.assert_array_equal(ru["assign"][0], planted)
    eo, _ = oracle.energies(model, scene, p, planted[None, :].astype(np.int32))
    assert eo[0] > 0.5 and ro["energy"][0] > 1e-3


def test_unsigned_difference_at_most_wrapped_difference():
    rng = np.random.default_rng(3)
    a = rng.uniform(-math.pi, math.pi, 20000)
    b = rng.uniform(-math.pi, math.pi, 20000)
    lhs = np.abs(np.abs(a) - np.abs(b))
    rhs = np.array([abs(E.wrap(x - y)) for x, y in zip(a, b)])
    assert (lhs <= rhs + 1e-12).all()


def test_unsigned_optimum_at_most_oriented_and_recursion_equals_brute_force():
    total = below = 0
    for seed in range(80):
        T = [4, 3, 0, 6][seed % 4]
        w = synth.tiny(2300 + seed, T=T, window=[1, 2][seed % 2], k_max=5)
        m, s = w.models[0], w.scenes[0]
        pu = dataclasses.replace(w.params, angle_unsigned=True)
        ru = oracle.match(m, s, pu)
        ro = oracle.match(m, s, w.params)
        eb, zs = E.brute_force_all(m, s, pu)
        for j in range(eb.shape[0]):
            a, b = ru["energy"][j], eb[j]
            if math.isinf(b):
                assert math.isinf(a) and math.isinf(ro["energy"][j])
                continue
            assert abs(a - b) <= 1e-12 * max(1.0, abs(b)), (seed, j, a, b)
            assert [int(v) for v in ru["assign"][j]] in [[int(v) for v in z] for z in zs[j]]
            assert a <= ro["energy"][j] + 1e-12 * max(1.0, abs(a))
            below += a < ro["energy"][j] - 1e-9
            total += 1
    assert total > 200 and below > 20
