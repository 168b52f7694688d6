"""Pins of the pruner oracle (oracle/pruner.py) to facts other than itself:
central finite differences of the loss for every gradient, closed forms of
the softmax cross-entropy and of Adam's first step, and hand-derived
features."""
import math

import numpy as np

from oracle import pruner as PR
from paper_1505_00581_amd import synth


def _toy(seed=0, G=3, K=5, dim=4):
    rng = np.random.Generator(np.random.PCG64(seed))
    P = PR.init_params(dim, seed)
    # shrink the hidden layers for a fast finite-difference sweep
    P["W1"], P["b1"] = P["W1"][:6], rng.normal(0, 0.1, 6)
    P["W2"], P["b2"] = P["W2"][:5, :6], rng.normal(0, 0.1, 5)
    P["w3"], P["b3"] = P["w3"][:5], np.array([0.3])
    P = {k: np.ascontiguousarray(v, np.float64).copy() for k, v in P.items()}
    X = rng.normal(0, 1, (G * K, PR.n_inputs(dim)))
    valid = rng.random((G, K)) > 0.2
    valid[:, 0] = True
    labels = np.array([int(rng.choice(np.nonzero(v)[0])) for v in valid])
    return P, X, labels, valid


def test_gradients_match_central_differences():
    P, X, labels, valid = _toy()
    G, K = valid.shape
    s, cache = PR.forward(P, X)
    loss, ds = PR.group_loss(s.reshape(G, K), None, labels, valid)
    g = PR.backward(P, cache, ds.reshape(-1))
    h = 1e-6
    for k in P:
        flat = P[k].reshape(-1)
        for idx in range(flat.size):
            old = flat[idx]
            flat[idx] = old + h
            lp = PR.loss_of(P, X, (G, K), labels, valid)
            flat[idx] = old - h
            lm = PR.loss_of(P, X, (G, K), labels, valid)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (k, idx, fd, an)


def test_softmax_cross_entropy_closed_forms():
    G, K = 2, 6
    valid = np.ones((G, K), bool)
    valid[1, 4:] = False
    scores = np.zeros((G, K))
    loss, ds = PR.group_loss(scores, None, np.array([0, 3]), valid)
    # uniform scores: -log(1/K_valid), averaged over groups
    assert abs(loss - (math.log(6) + math.log(4)) / 2) < 1e-12
    assert np.allclose(ds.sum(1), 0.0)
    assert (ds[1, 4:] == 0).all()
    assert abs(ds[0, 0] - (1 / 6 - 1) / 2) < 1e-12


def test_adam_first_step_is_minus_lr_sign():
    P = dict(a=np.array([1.0, -2.0, 3.0]))
    g = dict(a=np.array([0.5, -4.0, 1e-3]))
    st = {}
    PR.adam_step(P, g, st, lr=0.01, step=1)
    want = np.array([1.0, -2.0, 3.0]) - 0.01 * g["a"] / (np.abs(g["a"]) + 1e-8)
    assert np.allclose(P["a"], want, rtol=0, atol=1e-12)


def test_features_hand_derived():
    # model: 3 points; scene: 4 nodes over frames 0..3
    m = synth.Points(np.array([[0, 0], [10, 0], [10, 20]], np.float32), np.array([0, 1, 3], np.int32),
                     np.zeros((3, 2), np.float32))
    s = synth.Points(np.array([[100, 50], [110, 50], [112, 49], [111, 70]], np.float32),
                     np.array([0, 1, 1, 3], np.int32), np.zeros((4, 2), np.float32), 4)
    U_1 = np.array([0.0, 0.5, 0.25, 0.0])
    # point i = 1 at tau = 0 (target frame 1); neighbours a = 0 (q_a = node 0),
    # b = 2 (q_b = node 3); candidate node 2 at frame 1
    phi = PR.features(m, s, 0, 1, [1, 2], 0, 3, U_1)[1]
    assert phi[0] == 0.0                                   # frame offset 1 - 1
    assert np.allclose(phi[1:3], [((112 - 100) - 10) / 64, ((49 - 50) - 0) / 64])
    assert np.allclose(phi[3:5], [((112 - 111) - 0) / 64, ((49 - 70) - (-20)) / 64])
    assert abs(phi[5] - math.log((math.hypot(12, -1) + 1) / (10 + 1))) < 1e-12
    # U relative to the group's best candidate: node 2 (0.25) is the best
    assert phi[6] == 0.0 and phi[7] == 0.5
    assert PR.features(m, s, 0, 1, [1, 2], 0, 3, U_1)[0][6] == 0.25
    # descriptors enter scaled by their dimension
    x = PR.inputs(m, s, 1, [1, 2], np.zeros((2, 8)))
    assert np.allclose(x[:, :2], 2 * m.desc[1]) and np.allclose(x[1, 2:4], 2 * s.desc[2])
    # chain end: point 0 uses neighbour 1 for both sides
    phi0 = PR.features(m, s, 0, 0, [0], 1, 1, np.zeros(4))[0]
    assert np.allclose(phi0[1:3], phi0[3:5])
    assert phi0[7] == 0.0
