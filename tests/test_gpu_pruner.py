"""The learned candidate pruner on MI355X, against the FP64 pruner oracle
(oracle/pruner.py) and the FP64 recursion oracle (oracle.match_lists).

* features: candidate lists bit-exact, neighbour choices valid (the smallest
  FP64 unary within FP32 rounding), phi within FP32 rounding of the oracle's;
* FP32 training pass: scores, loss and every gradient element against the
  FP64 oracle (1e-3 relative plus the FP32 rounding bound of its sums), Adam
  steps, label checks, a loss that falls under training;
* BF16 inference: scores close to the FP32 forward, the top-k rule exact on
  the returned scores, the zero network keeps the first slots;
* matching on given lists and on pruned lists: identical to stm_match when
  nothing is pruned, equal to the oracle's recursion on the same lists
  otherwise, exact fallback rows identical to stm_match.
"""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
import paper_1505_00581_amd as stm
from tolerances import energy_tol
from oracle import energy as E
from oracle import pruner as PR
from paper_1505_00581_amd import synth

pytestmark = pytest.mark.gpu

H = 128
HID = H


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def unpack(theta, dim):
    ni = 2 * dim + 8
    sizes = [("W1", (H, ni)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))]
    out, o = {}, 0
    for k, shp in sizes:
        n = int(np.prod(shp))
        out[k] = np.asarray(theta[o:o + n], np.float64).reshape(shp)
        o += n
    assert o == theta.size
    return out


def cut(scene, n_frames):
    keep = scene.t < n_frames
    return synth.Points(np.ascontiguousarray(scene.xy[keep]), np.ascontiguousarray(scene.t[keep]),
                        np.ascontiguousarray(scene.desc[keep]), n_frames)


@pytest.fixture(scope="module")
def ctx():
    c = stm.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def small():
    w = synth.config1(5)
    return w.models[0], w.scenes[0], w.params


@pytest.fixture(scope="module")
def mid():
    w = synth.config2(21, n_models=1)
    return w.models[0], cut(w.scenes[0], 320), w.params


def random_groups(model, scene, n, seed):
    rng = np.random.default_rng(seed)
    n_off = len(E.offsets(model.t, scene.n_frames))
    taus = rng.integers(0, n_off, n)
    i = rng.integers(0, model.n, n)
    i[:2] = [0, model.n - 1]
    return np.stack([taus, i], 1).astype(np.int32)


def unary_row(model, scene, i, nodes):
    u = np.zeros(scene.n)
    for n in nodes:
        u[n] = E.unary(model.desc[i], scene.desc[n])
    return u


def oracle_rows(model, scene, params, groups, node, q):
    """Oracle inputs X [G*64, 2D+8] and valid [G, 64] of the groups, with the
    neighbour choices q checked and then shared."""
    G, D = len(groups), model.dim
    X = np.zeros((G * 64, 2 * D + 8))
    valid = np.zeros((G, 64), bool)
    for g, (tau, i) in enumerate(groups):
        tau, i = int(tau), int(i)
        cand = oracle.candidate_list(model, scene, params, tau, i)
        k = len(cand)
        np.testing.assert_array_equal(node[g, :k], cand)
        assert (node[g, k:] == -1).all()
        valid[g, :k] = True
        a = i - 1 if i >= 1 else i + 1
        b = i + 1 if i <= model.n - 2 else i - 1
        for j, qj in ((a, q[g, 0]), (b, q[g, 1])):
            cj = oracle.candidate_list(model, scene, params, tau, j)
            if len(cj) == 0:
                assert qj == -1
                continue
            uj = unary_row(model, scene, j, cj)
            assert qj in cj
            # FP32 unary on the device decides; it must be the FP64 minimum up to rounding
            assert uj[qj] <= uj[cj].min() * (1 + 1e-5) + 1e-6
        phi = PR.features(model, scene, tau, i, cand, int(q[g, 0]), int(q[g, 1]),
                          unary_row(model, scene, i, cand))
        X[g * 64:g * 64 + k] = PR.inputs(model, scene, i, cand, phi)
    return X, valid


@pytest.mark.parametrize("which", ["small", "mid"])
def test_features_against_oracle(ctx, request, which):
    model, scene, p = request.getfixturevalue(which)
    pr = stm.Pruner(ctx, model.dim)
    groups = random_groups(model, scene, 24, seed=3)
    node, phi, q = pr.features(model, scene, p, groups)
    X, valid = oracle_rows(model, scene, p, groups, node, q)
    D = model.dim
    got = phi.reshape(-1, 8)[valid.reshape(-1)]
    want = X[valid.reshape(-1), 2 * D:]
    err = np.abs(got - want)
    assert (err <= 2e-5 + 2e-5 * np.abs(want)).all(), err.max(0)
    assert (phi.reshape(-1, 8)[~valid.reshape(-1)] == 0).all()
    say(f"  {which}: {int(valid.sum())} feature rows, max err {err.max():.2e}")
    pr.close()


def _labelled(model, scene, node, seed):
    rng = np.random.default_rng(seed)
    labels, slots = [], []
    for g in range(node.shape[0]):
        k = int((node[g] >= 0).sum())
        a = int(rng.integers(0, k))
        labels.append(node[g, a])
        slots.append(a)
    return np.array(labels, np.int32), np.array(slots)


@pytest.mark.parametrize("which", ["small", "mid"])
def test_gradient_against_oracle(ctx, request, which):
    model, scene, p = request.getfixturevalue(which)
    D = model.dim
    pr = stm.Pruner(ctx, D)
    theta = synth.pruner_init(D, 11)
    rng = np.random.default_rng(5)
    n1 = H * (2 * D + 8)
    theta[n1:n1 + H] = rng.normal(0, 0.05, H)                       # b1
    theta[-1 - 2 * H:-1 - H] = rng.normal(0, 0.05, H)               # b2
    pr.set_params(theta)
    groups = random_groups(model, scene, 16, seed=9)
    node, _, q = pr.features(model, scene, p, groups)
    labels, slots = _labelled(model, scene, node, 2)
    loss, grad, scores = pr.gradient(model, scene, p, groups, labels)
    X, valid = oracle_rows(model, scene, p, groups, node, q)
    P = unpack(theta.astype(np.float64), D)
    s, cache = PR.forward(P, X)
    want_loss, ds = PR.group_loss(s.reshape(-1, 64), None, slots, valid)
    g = PR.backward(P, cache, ds.reshape(-1))
    assert abs(loss - want_loss) <= 1e-4 * max(1.0, abs(want_loss)), (loss, want_loss)
    sv = s.reshape(-1, 64)[valid]
    assert (np.abs(scores[valid] - sv) <= 1e-4 * (1 + np.abs(sv))).all()
    assert np.isneginf(scores[~valid]).all()
    G = unpack(grad, D)
    mag, extra = _gradient_magnitudes(P, cache, ds.reshape(-1))
    # FP32 rounding of a sum of n terms is at most about n u times the sum of
    # their magnitudes; the longest chain behind an element is the reduction
    # over the batch's rows plus the sums of the forward and backward layers
    u = 2.0 ** -24
    n_chain = X.shape[0] + 2 * (2 * D + 8) + 2 * H
    say(f"  {which}: {X.shape[0]} rows, chain length {n_chain}, "
        f"{int(sum((e > 0).sum() for e in extra.values()))} elements touched by pre-activations within rounding of 0")
    for k in P:
        err = np.abs(G[k] - g[k])
        tol = 1e-3 * np.abs(g[k]) + n_chain * u * mag[k] + extra[k]
        ratio = err / np.maximum(tol, 1e-300)
        worst = np.unravel_index(int(np.argmax(ratio)), ratio.shape)
        say(f"  {which} d{k}: max |G-g| {err.max():.2e}, worst element {tuple(int(x) for x in worst)} "
            f"at {ratio[worst]:.3f} of its tolerance (|g| {abs(g[k][worst]):.3e}, magnitude {mag[k][worst]:.3e})")
        assert (err <= tol).all(), (k, worst, float(G[k][worst]), float(g[k][worst]), float(tol[worst]))
    pr.close()


def _gradient_magnitudes(P, cache, ds):
    """Per gradient element, the sum of the magnitudes of the terms behind it
    (the backward pass of oracle/pruner.py with every operand replaced by its
    absolute value), and the additional magnitude of the terms of units whose
    pre-activation lies within FP32 rounding of 0, where the two sides may
    take the ReLU differently."""
    X, h1, h2 = cache
    u = 2.0 ** -24
    aX = np.abs(X)
    z1 = X @ P["W1"].T + P["b1"]
    z2 = h1 @ P["W2"].T + P["b2"]
    n1 = X.shape[1]
    amb1 = np.abs(z1) <= n1 * u * (aX @ np.abs(P["W1"]).T + np.abs(P["b1"]))
    amb2 = np.abs(z2) <= (n1 + HID) * u * (np.abs(h1) @ np.abs(P["W2"]).T + np.abs(P["b2"]))

    def magnitudes(m1, m2):
        g = {}
        a = np.abs(ds)
        g["w3"] = a @ np.abs(h2)
        g["b3"] = np.array([a.sum()])
        dz2 = np.outer(a, np.abs(P["w3"])) * m2
        g["W2"] = dz2.T @ np.abs(h1)
        g["b2"] = dz2.sum(0)
        dz1 = (dz2 @ np.abs(P["W2"])) * m1
        g["W1"] = dz1.T @ aX
        g["b1"] = dz1.sum(0)
        return g

    strict = magnitudes(h1 > 0, h2 > 0)
    loose = magnitudes((h1 > 0) | amb1, (h2 > 0) | amb2)
    return strict, {k: loose[k] - strict[k] for k in strict}


def test_label_outside_list_rejected(ctx, small):
    model, scene, p = small
    pr = stm.Pruner(ctx, model.dim)
    pr.set_params(synth.pruner_init(model.dim, 0))
    groups = random_groups(model, scene, 4, seed=1)
    node, _, _ = pr.features(model, scene, p, groups)
    labels = node[:, 0].copy()
    outside = np.setdiff1d(np.arange(scene.n), node[1])
    labels[1] = outside[0]
    with pytest.raises(stm.StmError):
        pr.gradient(model, scene, p, groups, labels)
    with pytest.raises(stm.StmError):
        pr.train_step(model, scene, p, groups, labels, 1e-3)
    # nothing was updated
    np.testing.assert_array_equal(pr.get_params(), synth.pruner_init(model.dim, 0))
    pr.close()


def test_adam_steps_against_oracle(ctx, small):
    model, scene, p = small
    D = model.dim
    pr = stm.Pruner(ctx, D)
    theta = synth.pruner_init(D, 4)
    pr.set_params(theta)
    groups = random_groups(model, scene, 12, seed=4)
    node, _, _ = pr.features(model, scene, p, groups)
    labels, _ = _labelled(model, scene, node, 4)
    P = {"theta": theta.astype(np.float64)}
    state = {}
    for step in (1, 2, 3):
        _, grad, _ = pr.gradient(model, scene, p, groups, labels)
        pr.train_step(model, scene, p, groups, labels, 1e-3)
        PR.adam_step(P, {"theta": grad.astype(np.float64)}, state, lr=1e-3, step=step)
        got = pr.get_params()
        assert np.abs(got - P["theta"]).max() <= 1e-6 + 1e-6 * np.abs(P["theta"]).max()
        P["theta"] = got.astype(np.float64)   # follow the device's FP32 parameters
    pr.close()


def test_training_lowers_the_loss(ctx, mid):
    model, scene, p = mid
    r = ctx.match(model, scene, p)
    feas = np.nonzero(np.isfinite(r["energy32"]))[0]
    rng = np.random.default_rng(0)
    taus = rng.choice(feas, 256)
    i = rng.integers(0, model.n, 256)
    groups = np.stack([taus, i], 1).astype(np.int32)
    labels = r["assign"][taus, i].astype(np.int32)
    pr = stm.Pruner(ctx, model.dim)
    pr.set_params(synth.pruner_init(model.dim, 1))
    losses = [pr.train_step(model, scene, p, groups, labels, 2e-3) for _ in range(60)]
    say(f"  loss {losses[0]:.3f} -> {losses[-1]:.3f}")
    assert losses[-1] < 0.7 * losses[0]
    pr.close()


@pytest.mark.parametrize("which,rule", [("small", 0), ("mid", 0), ("small", 1), ("mid", 1), ("mid", 2)])
def test_infer_bf16_and_topk(ctx, request, which, rule):
    model, scene, p = request.getfixturevalue(which)
    pr = stm.Pruner(ctx, model.dim)
    pr.set_rule(rule)
    pr.set_params(synth.pruner_init(model.dim, 6))
    groups = random_groups(model, scene, 32, seed=6)
    node, _, _ = pr.features(model, scene, p, groups)
    labels, _ = _labelled(model, scene, node, 6)
    _, _, s32 = pr.gradient(model, scene, p, groups, labels)
    for topk in (1, 5, 16, 64):
        sb, cand, count = pr.infer(model, scene, p, groups, topk)
        valid = node >= 0
        assert np.isneginf(sb[~valid]).all()
        scale = np.abs(s32[valid]).mean() + 1.0
        err = np.abs(sb[valid] - s32[valid]).max()
        assert err <= 0.03 * scale, (err, scale)
        for g in range(len(groups)):
            k = int(valid[g].sum())
            tau, i = groups[g]
            df = np.abs(scene.t[node[g, :k]] - (tau + model.t[i] - model.t[0]))
            order = sorted(range(k), key=lambda a: ((df[a] if rule else 0), (-sb[g, a] if rule != 2 else 0), a))
            order = order[:topk]
            want = np.sort(node[g, order])
            assert count[g] == min(topk, k)
            np.testing.assert_array_equal(cand[g, :count[g]], want)
    say(f"  {which}: bf16 score err {err:.3e} (scale {scale:.3f})")
    # the zero network scores every candidate 0: the score rule keeps the
    # first slots, the frames-first and time-nearest rules the windowed rule's
    # first k
    pr.set_params(np.zeros(pr.n_params, np.float32))
    sb, cand, count = pr.infer(model, scene, p, groups, 4)
    for g in range(len(groups)):
        k = int((node[g] >= 0).sum())
        if rule == 0:
            np.testing.assert_array_equal(cand[g, :count[g]], node[g, :min(4, k)])
        else:
            want = oracle.candidate_list(model, scene, dataclasses.replace(p, k_max=4), int(groups[g][0]),
                                           int(groups[g][1]))
            np.testing.assert_array_equal(cand[g, :count[g]], want)
    pr.close()


@pytest.mark.parametrize("which,topk", [("small", 6), ("mid", 16)])
def test_zero_network_frames_first_is_the_windowed_rule(ctx, request, which, topk):
    """With every score equal, the frames-first selection keeps exactly the
    windowed rule's first k, so the pruned matching is stm_match at k_max = k
    wherever that is feasible (elsewhere the exact fallback answers)."""
    model, scene, p = request.getfixturevalue(which)
    pr = stm.Pruner(ctx, model.dim)
    pr.set_rule(stm.Pruner.FRAMES_FIRST)
    pr.set_params(np.zeros(pr.n_params, np.float32))
    got = pr.match(model, scene, p, topk=topk)
    small = ctx.match(model, scene, dataclasses.replace(p, k_max=topk))
    ok = np.isfinite(small["energy32"])
    assert (got["fell_back"][ok] == 0).all() and (got["fell_back"][~ok] == 1).all()
    for k in ("energy32", "energy64", "assign"):
        np.testing.assert_array_equal(got[k][ok], small[k][ok])
    pr.close()


@pytest.mark.parametrize("which,topk,device", [("small", 6, False), ("mid", 16, True), ("small", 1, False)])
def test_time_nearest_rule_is_match_at_k(ctx, request, which, topk, device):
    """The time-nearest rule (the pruner's default) ignores the network: with
    random weights the pruned matching is stm_match at k_max = k where that is
    feasible, and the exact matching (fell_back = 1) elsewhere."""
    import torch
    model, scene, p = request.getfixturevalue(which)
    pr = stm.Pruner(ctx, model.dim)
    assert pr.rule == stm.Pruner.TIME_NEAREST
    pr.set_params(synth.pruner_init(model.dim, 21))
    if device:
        got = pr.match(stm.DevicePoints.from_host(model), stm.DevicePoints.from_host(scene), p, topk=topk)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() if hasattr(v, "cpu") else v for k, v in got.items()}
    else:
        got = pr.match(model, scene, p, topk=topk)
    small = ctx.match(model, scene, dataclasses.replace(p, k_max=topk))
    ex = ctx.match(model, scene, p)
    ok = np.isfinite(small["energy32"])
    assert (got["fell_back"][ok] == 0).all() and (got["fell_back"][~ok] == 1).all()
    for k in ("energy32", "energy64", "energy_u64", "assign"):
        np.testing.assert_array_equal(got[k][ok], small[k][ok])
        np.testing.assert_array_equal(got[k][~ok], ex[k][~ok])
    say(f"  {which} top-{topk}: {int(ok.sum())} offsets on the time-nearest lists, {int((~ok).sum())} fell back")
    pr.close()


def test_match_lists_reproduces_match(ctx, small):
    model, scene, p = small
    cand, cnt = ctx.candidates(model, scene, p)
    a = ctx.match(model, scene, p)
    b = ctx.match_lists(model, scene, p, cand, cnt)
    for k in ("energy32", "energy64", "energy_u64", "assign"):
        np.testing.assert_array_equal(a[k], b[k])


@pytest.mark.parametrize("which", ["small", "mid"])
def test_match_lists_against_oracle(ctx, request, which):
    model, scene, p = request.getfixturevalue(which)
    cand, cnt = ctx.candidates(model, scene, p)
    rng = np.random.default_rng(8)
    n, M, K = cand.shape
    sub = np.full((n, M, 16), -1, np.int32)
    scnt = np.zeros((n, M), np.int32)
    for t in range(n):
        for i in range(M):
            keep = [int(x) for x in cand[t, i, :cnt[t, i]] if rng.random() < 0.6][:16]
            sub[t, i, :len(keep)] = keep
            scnt[t, i] = len(keep)
    got = ctx.match_lists(model, scene, p, sub, scnt)
    taus = np.unique(np.linspace(0, n - 1, 24).astype(int))
    ora = oracle.match_lists(model, scene, p, sub[taus], scnt[taus])
    e = ora["energy"]
    fin = np.isfinite(e)
    assert (np.isfinite(got["energy32"][taus]) == fin).all()
    assert (np.abs(got["energy32"][taus][fin] - e[fin]) <= energy_tol(e[fin])).all()
    eg, _ = oracle.energies(model, scene, p, got["assign"][taus][fin])
    assert (np.abs(eg - e[fin]) <= energy_tol(e[fin])).all()
    np.testing.assert_allclose(got["energy64"][taus][fin], eg, rtol=1e-9)
    assert (got["assign"][taus][~fin] == -1).all()
    say(f"  {which}: {int(fin.sum())} feasible / {len(taus)} sampled offsets on sub-lists")


def test_invalid_lists_rejected(ctx, small):
    model, scene, p = small
    cand, cnt = ctx.candidates(model, scene, p)
    bad = cand.copy()
    bad[0, 0, :2] = bad[0, 0, 1::-1]       # not ascending
    with pytest.raises(stm.StmError):
        ctx.match_lists(model, scene, p, bad, cnt)
    c2 = cnt.copy()
    c2[1, 1] = cand.shape[2] + 1
    with pytest.raises(stm.StmError):
        ctx.match_lists(model, scene, p, cand, c2)


def test_pruned_keeping_everything_equals_exact(ctx, small):
    model, scene, p = small
    pr = stm.Pruner(ctx, model.dim)
    pr.set_params(synth.pruner_init(model.dim, 2))
    a = ctx.match(model, scene, p)
    b = pr.match(model, scene, p, topk=64)
    for k in ("energy32", "energy64", "energy_u64", "assign"):
        np.testing.assert_array_equal(a[k], b[k])
    assert (b["fell_back"] == np.where(np.isfinite(a["energy32"]), 0, 1)).all()
    pr.close()


@pytest.mark.parametrize("which,topk,rule", [("small", 6, 1), ("mid", 16, 1), ("small", 6, 0), ("small", 1, 0),
                                             ("mid", 16, 2)])
def test_pruned_against_oracle_and_fallback(ctx, request, which, topk, rule):
    """Pruned matchings against the oracle on the same lists; with the score
    rule and one candidate per point most offsets are infeasible and must be
    answered by the exact fallback."""
    import torch
    model, scene, p = request.getfixturevalue(which)
    pr = stm.Pruner(ctx, model.dim)
    pr.set_rule(rule)
    pr.set_params(synth.pruner_init(model.dim, 3))
    ex = ctx.match(model, scene, p)
    got = pr.match(model, scene, p, topk=topk)
    n, M = got["assign"].shape
    # device-resident inputs and outputs give the same rows
    dm, ds = stm.DevicePoints.from_host(model), stm.DevicePoints.from_host(scene)
    dev = pr.match(dm, ds, p, topk=topk)
    torch.cuda.synchronize()
    for k in ("energy32", "energy64", "assign", "fell_back"):
        np.testing.assert_array_equal(got[k], dev[k].cpu().numpy())
    fell = got["fell_back"].astype(bool)
    # fallback rows are the exact rows
    for k in ("energy32", "energy64", "assign"):
        np.testing.assert_array_equal(got[k][fell], ex[k][fell])
    # pruned optimum: never below the exact one, and the oracle's on the same lists
    fin = np.isfinite(ex["energy32"])
    assert (got["energy32"][fin] >= ex["energy32"][fin] - energy_tol(ex["energy32"][fin])).all()
    groups = np.array([(t, i) for t in range(n) for i in range(M)], np.int32)
    _, cand, count = pr.infer(model, scene, p, groups, topk)
    cand, count = cand.reshape(n, M, topk), count.reshape(n, M)
    taus = np.nonzero(~fell)[0]
    taus = taus[np.unique(np.linspace(0, len(taus) - 1, 20).astype(int))] if len(taus) else taus
    if len(taus):
        ora = oracle.match_lists(model, scene, p, cand[taus], count[taus])
        e = ora["energy"]
        assert np.isfinite(e).all()
        assert (np.abs(got["energy32"][taus] - e) <= energy_tol(e)).all()
        for t in taus:   # the assignment uses the pruned lists
            for i in range(M):
                assert got["assign"][t, i] in cand[t, i, :count[t, i]]
    gap = (got["energy32"][fin] - ex["energy32"][fin]) / np.maximum(ex["energy32"][fin], 1e-6)
    say(f"  {which} top-{topk} rule {rule}: fallback {fell.mean():.3f}, mean gap {gap.mean():.4f}, "
        f"{len(taus)} offsets checked against the oracle")
    if topk == 1 and rule == 0:
        assert fell.any()
    pr.close()


def test_save_load_roundtrip(ctx, small, tmp_path):
    model, scene, p = small
    a = stm.Pruner(ctx, model.dim)
    th = synth.pruner_init(model.dim, 8)
    a.set_params(th)
    path = tmp_path / "pruner.bin"
    a.save(path)
    b = stm.Pruner(ctx, model.dim)
    b.load(path)
    np.testing.assert_array_equal(b.get_params(), th)
    c = stm.Pruner(ctx, 16)
    with pytest.raises(stm.StmError):
        c.load(path)
    for x in (a, b, c):
        x.close()


@pytest.mark.parametrize("topk,rule,device", [(16, 1, True), (1, 0, False), (48, 1, False), (16, 2, True),
                                               (1, 2, False)])
def test_plan_pruned_equals_per_pair_pruned(ctx, topk, rule, device):
    """The batched pruned run (lists, recursion, device-side fallback, all in
    one graph) gives every pair the rows of stm_match_pruned bit for bit; with
    one candidate per point under the score rule the fallback answers most
    offsets."""
    import torch
    w = synth.config2(41, n_models=3)
    scene = cut(w.scenes[0], 320)
    models, p = w.models, w.params
    pr = stm.Pruner(ctx, models[0].dim)
    pr.set_rule(rule)
    pr.set_params(synth.pruner_init(models[0].dim, 12))
    pairs = np.array([(i, 0) for i in range(len(models))], np.int32)
    if device:
        dm = [stm.DevicePoints.from_host(m) for m in models]
        plan = stm.Plan(ctx, dm, [stm.DevicePoints.from_host(scene)], pairs, p)
    else:
        plan = stm.Plan(ctx, models, [scene], pairs, p)
    out = plan.run_pruned(pr, topk)
    out2 = plan.run_pruned(pr, topk, out=out)     # graph replay
    if device:
        torch.cuda.synchronize()
    fell_total = 0
    for q, (i, _) in enumerate(pairs):
        e32, e64, _, A = [x.cpu().numpy() if hasattr(x, "cpu") else x for x in plan.pair_rows(out2, q)]
        r0, r1 = plan.row_offsets[q], plan.row_offsets[q + 1]
        fb = out2["fell_back"][r0:r1]
        fb = fb.cpu().numpy() if hasattr(fb, "cpu") else fb
        ref = pr.match(models[i], scene, p, topk=topk)
        np.testing.assert_array_equal(e32, ref["energy32"])
        np.testing.assert_array_equal(e64, ref["energy64"])
        np.testing.assert_array_equal(A, ref["assign"])
        np.testing.assert_array_equal(fb, ref["fell_back"])
        fell_total += int(fb.sum())
    say(f"  plan top-{topk} rule {rule}: {plan.n_rows} rows identical, {fell_total} answered by the fallback")
    if topk == 1 and rule == 0:
        assert fell_total > 0
    plan.close()
    pr.close()
