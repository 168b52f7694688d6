"""Training and evaluation of the learned candidate pruner.

Labels are the exact optimum's choices a*_i, produced on the GPU by the exact
recursion (stm_match); training runs on the GPU through the pruner's own FP32
forward and backward kernels and Adam (stm_pruner_train_step).  Evaluation
compares the pruned matching with the exact one and with two pruning rules
that need no training: the top-k candidates by unary cost U (Eq. 2) and the
top-k nearest in time (the windowed rule with k_max = k).

Run `python -m paper_1505_00581_amd.pruner_train --help` for the command line.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import sys
import time

import numpy as np

from . import _binding as B
from . import synth


def _host(x):
    return x.cpu().numpy() if hasattr(x, "cpu") else np.asarray(x)


@dataclasses.dataclass
class Item:
    model: object      # DevicePoints
    scene: object      # DevicePoints
    groups: np.ndarray  # [G, 2] (tau, i)
    labels: np.ndarray  # [G] node ids


def label_pair(ctx, model, scene, params, n_groups: int, rng) -> tuple:
    """n_groups (tau, i) groups drawn uniformly over the feasible offsets and
    the model points, with the exact optimum's node as label."""
    r = ctx.match(model, scene, params)
    e32, assign = _host(r["energy32"]), _host(r["assign"])
    feas = np.nonzero(np.isfinite(e32))[0]
    if len(feas) == 0 or n_groups <= 0:
        return np.zeros((0, 2), np.int32), np.zeros(0, np.int32)
    M = assign.shape[1]
    t = rng.choice(feas, n_groups)
    i = rng.integers(0, M, n_groups)
    groups = np.stack([t + r["tau_begin"], i], 1).astype(np.int32)
    return groups, assign[t, i].astype(np.int32)


def training_set(ctx, seeds, groups_per_model: int, n_models: int = 10, seed: int = 0, log=None) -> list:
    """Items from realistic single-scene workloads (one scene of 1500 frames and
    n_models models per seed), inputs resident on the device."""
    rng = np.random.default_rng(seed)
    items = []
    for s in seeds:
        w = synth.config2(int(s), n_models=n_models)
        ds = B.DevicePoints.from_host(w.scenes[0])
        for m in w.models:
            dm = B.DevicePoints.from_host(m)
            g, lab = label_pair(ctx, dm, ds, w.params, groups_per_model, rng)
            if len(g):
                items.append(Item(dm, ds, g, lab))
        if log:
            log(f"labels: seed {s}, {sum(len(it.groups) for it in items)} groups so far")
    return items


def train(pruner, items, params, epochs: int = 4, batch: int = 1024, lr: float = 2e-3,
          lr_final: float = 2e-4, seed: int = 0, log=None) -> list:
    """Adam over mini-batches of one (model, scene) pair each; the learning
    rate decays geometrically from lr to lr_final.  Returns the mean loss of
    every epoch."""
    rng = np.random.default_rng(seed)
    batches = []
    for k, it in enumerate(items):
        for b0 in range(0, len(it.groups), batch):
            batches.append((k, b0))
    n_steps = max(1, epochs * len(batches))
    decay = (lr_final / lr) ** (1.0 / n_steps)
    step, cur, history = 0, lr, []
    for ep in range(epochs):
        order = rng.permutation(len(batches))
        tot, n = 0.0, 0
        for j in order:
            k, b0 = batches[j]
            it = items[k]
            g, lab = it.groups[b0:b0 + batch], it.labels[b0:b0 + batch]
            loss = pruner.train_step(it.model, it.scene, params, g, lab, cur)
            tot += loss * len(g)
            n += len(g)
            step += 1
            cur *= decay
        history.append(tot / max(n, 1))
        if log:
            log(f"epoch {ep + 1}/{epochs}: mean loss {history[-1]:.4f}")
    return history


def u_ranked_lists(ctx, model, scene, params, topk: int):
    """The topk candidates of each (tau, i) with the smallest U (lower slot
    first on ties), ascending: [n, M, topk] and counts [n, M]."""
    cand, cnt = ctx.candidates(model, scene, params)
    cand, cnt = _host(cand), _host(cnt)
    U = _host(ctx.unary(model, scene, params))
    n, M, K = cand.shape
    slot = np.arange(K)
    valid = slot[None, None, :] < cnt[:, :, None]
    u = np.where(valid, U[np.arange(M)[None, :, None], np.maximum(cand, 0)], np.inf)
    order = np.argsort(u, axis=2, kind="stable")[:, :, :topk]
    keep = np.take_along_axis(cand, order, 2)
    kv = np.take_along_axis(valid, order, 2)
    keep = np.where(kv, keep, np.iinfo(np.int32).max)
    keep = np.sort(keep, axis=2)
    keep = np.where(keep == np.iinfo(np.int32).max, -1, keep).astype(np.int32)
    return keep, np.minimum(cnt, topk).astype(np.int32)


def _gap_stats(e, ex, fin):
    g = (e[fin] - ex[fin]) / np.maximum(ex[fin], 1e-12)
    return dict(mean_gap=float(g.mean()) if g.size else 0.0, max_gap=float(g.max()) if g.size else 0.0,
                total_gap=float((e[fin] - ex[fin]).sum() / max(ex[fin].sum(), 1e-12)))


def evaluate(ctx, pruner, model, scene, params, topks=(16,), baselines: bool = True, rule: int = 1) -> dict:
    """Energy gap, recall of the exact optimum's choices and fallback rate of
    the pruned matching at each k in topks under selection rule `rule` (the
    learned frames-first rule unless told otherwise; the pruner's own rule is
    restored afterwards), and of the baselines, with the same exact fallback."""
    saved = pruner.rule
    pruner.set_rule(rule)
    try:
        return _evaluate(ctx, pruner, model, scene, params, topks, baselines)
    finally:
        pruner.set_rule(saved)


def _evaluate(ctx, pruner, model, scene, params, topks, baselines) -> dict:
    ex = ctx.match(model, scene, params)
    e_ex, a_ex = _host(ex["energy32"]).astype(np.float64), _host(ex["assign"])
    fin = np.isfinite(e_ex)
    n, M = a_ex.shape
    out = {"offsets": int(n), "feasible": int(fin.sum()), "k": {}}
    groups = np.array([(t, i) for t in range(n) for i in range(M)], np.int32)
    groups[:, 0] += ex["tau_begin"]
    for k in topks:
        r = {}
        pr = pruner.match(model, scene, params, topk=k)
        e_pr, fell = _host(pr["energy32"]).astype(np.float64), _host(pr["fell_back"]).astype(bool)
        _, cand, count = pruner.infer(model, scene, params, groups, k)
        cand, count = cand.reshape(n, M, k), count.reshape(n, M)
        r["mlp"] = dict(_gap_stats(e_pr, e_ex, fin), fallback=float(fell.mean()),
                        recall=_recall(cand, count, a_ex, fin))
        if baselines:
            uc, ucnt = u_ranked_lists(ctx, model, scene, params, k)
            ru = ctx.match_lists(model, scene, params, uc, ucnt)
            e_u = _host(ru["energy32"]).astype(np.float64)
            fb_u = ~np.isfinite(e_u)
            e_u = np.where(fb_u, e_ex, e_u)
            r["u_ranked"] = dict(_gap_stats(e_u, e_ex, fin), fallback=float(fb_u.mean()),
                                 recall=_recall(uc, ucnt, a_ex, fin))
            pt = dataclasses.replace(params, k_max=k)
            rt = ctx.match(model, scene, pt)
            e_t = _host(rt["energy32"]).astype(np.float64)
            fb_t = ~np.isfinite(e_t)
            e_t = np.where(fb_t, e_ex, e_t)
            tc, tcnt = ctx.candidates(model, scene, pt)
            r["time_nearest"] = dict(_gap_stats(e_t, e_ex, fin), fallback=float(fb_t.mean()),
                                     recall=_recall(_host(tc), _host(tcnt), a_ex, fin))
        out["k"][int(k)] = r
    return out


def summarise(results: list) -> dict:
    """Means over evaluated (model, scene) pairs, per k and method."""
    out = {}
    for k in results[0]["k"]:
        out[k] = {}
        for meth in results[0]["k"][k]:
            rows = [r["k"][k][meth] for r in results]
            out[k][meth] = {f: round(float(np.mean([x[f] for x in rows])), 5) for f in rows[0]}
            out[k][meth]["max_gap"] = round(float(max(x["max_gap"] for x in rows)), 5)
    return out


def _recall(cand, count, a_ex, fin):
    """Fraction of (feasible offset, point) whose exact choice is kept."""
    n, M, k = cand.shape
    slot = np.arange(k)
    hit = ((cand == a_ex[:, :, None]) & (slot[None, None, :] < count[:, :, None])).any(2)
    return float(hit[fin].mean()) if fin.any() else 0.0


def main(argv=None):
    ap = argparse.ArgumentParser(description="train the candidate pruner on exact-recursion labels")
    ap.add_argument("--train-seeds", default="100-129")
    ap.add_argument("--test-seeds", default="900-904")
    ap.add_argument("--groups", type=int, default=200000, help="training groups in total")
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--topk", default="16,32,48", help="comma-separated list sizes to evaluate")
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--out", default=None, help="write the trained parameters here")
    ap.add_argument("--report", default=None, help="write the evaluation as JSON here")
    a = ap.parse_args(argv)

    def seeds(s):
        lo, hi = (int(x) for x in s.split("-"))
        return list(range(lo, hi + 1))

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    train_seeds = seeds(a.train_seeds)
    ctx = B.Context(0)
    params = synth.config2(train_seeds[0], n_models=1).params
    t0 = time.time()
    per_model = max(1, a.groups // (10 * len(train_seeds)))
    items = training_set(ctx, train_seeds, per_model, log=log)
    t1 = time.time()
    pruner = B.Pruner(ctx, synth.DIM)
    pruner.set_params(synth.pruner_init(synth.DIM, a.init_seed))
    hist = train(pruner, items, params, epochs=a.epochs, batch=a.batch, lr=a.lr, log=log)
    t2 = time.time()
    if a.out:
        pruner.save(a.out)
    report = dict(groups=int(sum(len(it.groups) for it in items)), label_s=t1 - t0, train_s=t2 - t1,
                  loss=hist, test=[])
    topks = tuple(int(x) for x in a.topk.split(","))
    for s in seeds(a.test_seeds):
        w = synth.config2(s)
        ds = B.DevicePoints.from_host(w.scenes[0])
        for m in w.models:
            r = evaluate(ctx, pruner, B.DevicePoints.from_host(m), ds, w.params, topks=topks)
            r["seed"] = s
            report["test"].append(r)
        log(f"test seed {s}: {json.dumps(summarise(report['test']))}")
    report["summary"] = summarise(report["test"])
    print(json.dumps(report["summary"]))
    if a.report:
        with open(a.report, "w") as f:
            json.dump(report, f, indent=1)


if __name__ == "__main__":
    main()
