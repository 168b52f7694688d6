"""The multiple-points variant 2 (stm_match_chains) on MI355X against the
oracle's restatement (oracle.chains): mean chain energies within the exact
path's tolerance (1e-5 relative, 1e-4 absolute floor), each chain's
assignment identical or of equal oracle energy, FP64 means to 1e-9."""
import sys

import numpy as np
import pytest

import oracle
import paper_1505_00581_amd as stm
from tolerances import energy_tol
from oracle import chains as C
from paper_1505_00581_amd import synth

pytestmark = pytest.mark.gpu



def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = stm.Context(0)
    yield c
    c.close()


def _np(x):
    return x.cpu().numpy() if hasattr(x, "cpu") else np.asarray(x)


def check(m, s, p, res, ora, rows=None):
    e32 = _np(res["energy32"]).astype(np.float64)
    e64, A = _np(res["energy64"]), _np(res["assign"])
    if rows is not None:
        e32, e64, A = e32[rows], e64[rows], A[rows]
    E = ora["energy"]
    fin = np.isfinite(E)
    assert (np.isfinite(e32) == fin).all()
    tol = energy_tol(E[fin])
    assert (np.abs(e32[fin] - E[fin]) <= tol).all(), np.abs(e32[fin] - E[fin]).max()
    assert (A[:, [q for q in range(m.n) if q not in sum(ora["chains"], [])]] == C.UNCHAINED).all()
    # the FP64 mean is the mean of the oracle's literal energies of the GPU's chain assignments
    lit = np.zeros(A.shape[0])
    for idx in ora["chains"]:
        e, _ = oracle.energies(C.sub_model(m, idx), s, p, A[:, idx])
        lit += e
    lit /= len(ora["chains"])
    assert np.allclose(e64[fin], lit[fin], rtol=1e-9, atol=1e-9)
    same = (A == ora["assign"]).all(1)
    assert (np.abs(lit[fin & ~same] - E[fin & ~same]) <= energy_tol(E[fin & ~same])).all()
    return dict(n=len(E), feasible=int(fin.sum()), agree=float(same.mean()), chains=len(ora["chains"]))


@pytest.mark.parametrize("seed,n_chains", [(0, 3), (1, 2), (2, 3)])
def test_small_multipoint_all_offsets(ctx, seed, n_chains):
    w = synth.multipoint(seed, n_models=1, frames=(12, 20), per_frame=3, n_frames=70, clutter_per_frame=4,
                         window=2, k_max=16, width=160.0, height=120.0, planted_per_model=2)
    m, s, p, sal = w.models[0], w.scenes[0], w.params, w.saliency[0]
    res = ctx.match_chains(m, s, p, sal, n_chains)
    ora = C.match_chains(m, s, p, sal, n_chains)
    assert res["chains_used"] == len(ora["chains"])
    st = check(m, s, p, res, ora)
    say(f"[chains seed={seed} N={n_chains}] {st}")
    assert st["feasible"] > 0


@pytest.mark.parametrize("reading", ["angle_unsigned", "causal_node"])
def test_alternative_readings(ctx, reading):
    import dataclasses
    w = synth.multipoint(3, n_models=1, frames=(12, 20), per_frame=3, n_frames=70, clutter_per_frame=4,
                         window=2, k_max=16, width=160.0, height=120.0, planted_per_model=2)
    m, s, sal = w.models[0], w.scenes[0], w.saliency[0]
    p = dataclasses.replace(w.params, **{reading: True})
    res = ctx.match_chains(m, s, p, sal, 3)
    ora = C.match_chains(m, s, p, sal, 3)
    st = check(m, s, p, res, ora)
    say(f"[chains {reading}] {st}")
    assert st["feasible"] > 0


def test_one_point_per_frame_equals_stm_match(ctx):
    w = synth.config1(5)
    m, s, p = w.models[0], w.scenes[0], w.params
    res = ctx.match_chains(m, s, p, np.random.default_rng(1).uniform(size=m.n), 3)
    ref = ctx.match(m, s, p)
    assert res["chains_used"] == 1
    for k in ("energy32", "energy64", "energy_u64", "assign"):
        np.testing.assert_array_equal(res[k], ref[k])


def test_device_pointers_equal_host_pointers(ctx):
    import torch
    w = synth.multipoint(4, n_models=1, frames=(12, 20), n_frames=70, clutter_per_frame=4, window=2, k_max=16,
                         width=160.0, height=120.0, planted_per_model=2)
    m, s, p, sal = w.models[0], w.scenes[0], w.params, w.saliency[0]
    host = ctx.match_chains(m, s, p, sal, 3)
    dev = ctx.match_chains(stm.DevicePoints.from_host(m), stm.DevicePoints.from_host(s), p,
                           torch.as_tensor(sal, device="cuda"), 3)
    torch.cuda.synchronize()
    for k in ("energy32", "energy64", "energy_u64", "assign"):
        np.testing.assert_array_equal(_np(dev[k]), host[k])


def test_realistic_scene_sampled_offsets(ctx):
    """Three points per model frame against the realistic 1500-frame scene
    (K = 64): every chain runs the 64-slot recursion."""
    w = synth.multipoint(0, n_models=1)
    m, s, p, sal = w.models[0], w.scenes[0], w.params, w.saliency[0]
    res = ctx.match_chains(m, s, p, sal, 3)
    n = int(_np(res["energy32"]).shape[0])
    rows = np.sort(np.random.default_rng(2).choice(n, 24, replace=False)).astype(np.int32)
    say(f"[chains realistic] M={m.n} S={s.n} offsets={n} chains={res['chains_used']}")
    st = check(m, s, p, res, C.match_chains(m, s, p, sal, 3, taus=rows), rows=rows)
    say(f"  {st}")
    assert st["chains"] == 3 and st["feasible"] > 0


def test_invalid_chain_inputs(ctx):
    w = synth.multipoint(5, n_models=1, frames=(12, 20), n_frames=70, clutter_per_frame=4, window=2, k_max=16)
    m, s, p = w.models[0], w.scenes[0], w.params
    bad = synth.Points(m.xy.copy(), m.t[::-1].copy(), m.desc.copy())
    with pytest.raises(stm.StmError, match="non-decreasing"):
        ctx.match_chains(bad, s, p, None, 3, 0, 1)
    one = synth.Points(m.xy[:2].copy(), m.t[:2].copy(), m.desc[:2].copy())
    with pytest.raises(stm.StmError):
        ctx.match_chains(one, s, p, None, 3, 0, 1)
    t2 = np.zeros(m.n, np.int32)  # every point in one frame: chains of one point each
    with pytest.raises(stm.StmError, match="no chain"):
        ctx.match_chains(synth.Points(m.xy.copy(), t2, m.desc.copy()), s, p, None, 3, 0, 1)
