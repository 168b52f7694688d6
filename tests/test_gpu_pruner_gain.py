"""What the trained pruner gains over pruning without it (MI355X).

The network is trained on the GPU by its own kernels on labels from the exact
recursion (realistic single-scene workloads, seeds 100-129), then evaluated on a
held-out seed against the exact matching, beside two rules that need no
training: the k candidates with the smallest unary cost U, and the k nearest
in time (the windowed rule capped at k).  Measured gaps, recalls and fallback
rates are printed; the assertions are what the learned selection must
deliver on these inputs: far less energy lost than U-ranking, and less than
keeping the first k nearest in time at k = 16, where the learned score picks
which nodes of the nearest frames survive.
"""
import sys

import numpy as np
import pytest

import paper_1505_00581_amd as stm
from paper_1505_00581_amd import pruner_train as PT
from paper_1505_00581_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def trained():
    ctx = stm.Context(0)
    items = PT.training_set(ctx, range(100, 130), 667)
    p = synth.config2(100, n_models=1).params
    pr = stm.Pruner(ctx, synth.DIM)
    pr.set_params(synth.pruner_init(synth.DIM, 0))
    hist = PT.train(pr, items, p, epochs=4)
    say(f"  trained on {sum(len(it.groups) for it in items)} groups, loss {hist[0]:.4f} -> {hist[-1]:.4f}")
    del items
    yield ctx, pr, hist
    pr.close()
    ctx.close()


def test_training_lowers_the_loss_on_exact_labels(trained):
    _, _, hist = trained
    assert hist[-1] < hist[0]


def test_gain_over_rules_without_training(trained):
    ctx, pr, _ = trained
    w = synth.config2(900, n_models=3)
    ds = stm.DevicePoints.from_host(w.scenes[0])
    res = [PT.evaluate(ctx, pr, stm.DevicePoints.from_host(m), ds, w.params, topks=(16, 48))
           for m in w.models]
    s = PT.summarise(res)
    for k in (16, 48):
        for meth in ("mlp", "time_nearest", "u_ranked"):
            say(f"  k={k} {meth}: {s[k][meth]}")
    for k in (16, 48):
        assert s[k]["mlp"]["mean_gap"] < 0.5 * s[k]["u_ranked"]["mean_gap"]
        assert s[k]["mlp"]["recall"] > s[k]["u_ranked"]["recall"]
        assert s[k]["mlp"]["fallback"] == 0.0
    assert s[16]["mlp"]["mean_gap"] < s[16]["time_nearest"]["mean_gap"]
    # the pruned optimum never undercuts the exact one (lists are subsets)
    assert all(r["k"][k]["mlp"]["mean_gap"] >= 0 for r in res for k in (16, 48))
