"""FP64 CPU oracle of the learned candidate pruner.

TEST INFRASTRUCTURE ONLY (like the rest of `oracle/`): the tests use it to
pin the GPU pruner's features, forward pass, loss, gradients and Adam step.

The pruner is not part of the paper.  It scores each candidate scene node n
of a model point i at an offset tau and keeps the best k, so that the exact
recursion (Section 2.2) runs on shorter candidate lists; the exact recursion
stays the fallback and the reference for the energy gap.

Input of one (tau, i, n): x = [D f_i (D), D g_n (D), phi (8)], D = descriptor
dim (the descriptors are L1-normalised, so the factor D brings their entries
to order 1).
phi (fixed before any training):
  0  (t'_n - (tau + t_i - t_0)) / 4                       frame offset
  1,2 ((p'_n - p'_{q_a}) - (p_i - p_a)) / 64               x, y consistency with neighbour a
  3,4 ((p'_n - p'_{q_b}) - (p_i - p_b)) / 64               x, y consistency with neighbour b
  5  log((|p'_n - p'_{q_a}| + 1) / (|p_i - p_a| + 1))       scale ratio against neighbour a
  6  U(i, n) - min over the group's candidates n' of U(i, n')  appearance (Eq. 2)
  7  i / (M - 1)                                            position in the chain
Neighbours: a = i - 1 and b = i + 1; at the chain ends the one neighbour is
used for both.  q_j is the candidate of neighbour j at tau with the smallest
U (lowest index on ties); if neighbour j has no candidate, its terms are 0.
Network: h1 = relu(W1 x + b1) (128), h2 = relu(W2 h1 + b2) (128),
s = w3 . h2 + b3.  Loss of a group (the candidates of one (tau, i)): softmax
cross-entropy of the scores against the index of the exact optimum's
candidate; the batch loss is the mean over groups.
"""
from __future__ import annotations

import math

import numpy as np

HIDDEN = 128
NPHI = 8


def n_inputs(dim: int) -> int:
    return 2 * dim + NPHI


def init_params(dim: int, seed: int) -> dict:
    """He-uniform initial weights (the GPU pruner draws the same from the seed
    only through the tests, which pass weights explicitly)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_in = n_inputs(dim)

    def he(o, i):
        lim = math.sqrt(6.0 / i)
        return rng.uniform(-lim, lim, (o, i))

    return dict(W1=he(HIDDEN, n_in), b1=np.zeros(HIDDEN), W2=he(HIDDEN, HIDDEN), b2=np.zeros(HIDDEN),
                w3=he(1, HIDDEN)[0], b3=np.zeros(1))


def neighbour_argmin(U_rows, cand_j):
    """Index into cand_j of the smallest U (lowest index on ties), or -1."""
    if len(cand_j) == 0:
        return -1
    return int(np.argmin(U_rows[cand_j]))


def features(model, scene, tau: int, i: int, cand_i, q_a: int, q_b: int, U_i) -> np.ndarray:
    """phi [K, 8] of the candidates cand_i (node ids) of point i at tau, given
    the chosen neighbour candidates q_a, q_b (node ids, -1 for none) and the
    unary row U_i (indexed by node id)."""
    M = model.n
    a = i - 1 if i >= 1 else i + 1
    b = i + 1 if i <= M - 2 else i - 1
    mt = model.t.astype(np.int64)
    f0 = tau + int(mt[i] - mt[0])
    p = model.xy.astype(np.float64)
    q = scene.xy.astype(np.float64)
    out = np.zeros((len(cand_i), NPHI))
    u_min = min(U_i[int(n)] for n in cand_i) if len(cand_i) else 0.0
    for r, n in enumerate(cand_i):
        n = int(n)
        out[r, 0] = (int(scene.t[n]) - f0) / 4.0
        if q_a >= 0:
            d = (q[n] - q[q_a]) - (p[i] - p[a])
            out[r, 1], out[r, 2] = d[0] / 64.0, d[1] / 64.0
            out[r, 5] = math.log((math.hypot(*(q[n] - q[q_a])) + 1.0) / (math.hypot(*(p[i] - p[a])) + 1.0))
        if q_b >= 0:
            d = (q[n] - q[q_b]) - (p[i] - p[b])
            out[r, 3], out[r, 4] = d[0] / 64.0, d[1] / 64.0
        out[r, 6] = U_i[n] - u_min
        out[r, 7] = i / (M - 1)
    return out


def inputs(model, scene, i: int, cand_i, phi) -> np.ndarray:
    """x [K, 2D + 8] of one group."""
    D = model.desc.shape[1]
    f = D * np.repeat(model.desc[i:i + 1].astype(np.float64), len(cand_i), 0)
    g = D * scene.desc[np.asarray(cand_i, np.int64)].astype(np.float64)
    return np.concatenate([f, g, phi], 1)


def forward(P: dict, X: np.ndarray):
    """Scores [N] and the activations needed by backward."""
    z1 = X @ P["W1"].T + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(z2, 0.0)
    s = h2 @ P["w3"] + P["b3"][0]
    return s, (X, h1, h2)


def group_loss(scores, groups, labels, valid):
    """Mean over groups of -log softmax(score)[label] and d loss / d score.
    scores: [G, K]; valid: [G, K] bool; labels: [G] index into the group."""
    G, K = scores.shape
    s = np.where(valid, scores, -np.inf)
    m = s.max(1, keepdims=True)
    e = np.where(valid, np.exp(s - m), 0.0)
    z = e.sum(1, keepdims=True)
    p = e / z
    loss = float(np.mean(-(s[np.arange(G), labels] - m[:, 0] - np.log(z[:, 0]))))
    ds = p.copy()
    ds[np.arange(G), labels] -= 1.0
    return loss, ds / G


def backward(P: dict, cache, ds: np.ndarray) -> dict:
    """Gradients of the loss with respect to every parameter; ds [N]."""
    X, h1, h2 = cache
    g = {}
    g["w3"] = ds @ h2
    g["b3"] = np.array([ds.sum()])
    dz2 = np.outer(ds, P["w3"]) * (h2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ P["W2"]) * (h1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(0)
    return g


def loss_of(P, X, groups_shape, labels, valid):
    s, _ = forward(P, X)
    return group_loss(s.reshape(groups_shape), None, labels, valid)[0]


ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def adam_step(P: dict, grads: dict, state: dict, lr: float, step: int) -> None:
    """One Adam update (Kingma and Ba), step counted from 1, in place."""
    for k in P:
        m = state.setdefault("m_" + k, np.zeros_like(P[k]))
        v = state.setdefault("v_" + k, np.zeros_like(P[k]))
        m[...] = ADAM_B1 * m + (1 - ADAM_B1) * grads[k]
        v[...] = ADAM_B2 * v + (1 - ADAM_B2) * grads[k] ** 2
        mh = m / (1 - ADAM_B1 ** step)
        vh = v / (1 - ADAM_B2 ** step)
        P[k] = P[k] - lr * mh / (np.sqrt(vh) + ADAM_EPS)
