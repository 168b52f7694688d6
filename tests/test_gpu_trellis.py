"""The trellis over a scene block (stm_trellis_*; the paper's own problem,
Section 2.2, with the band of Section 3.4's loop bounds) on MI355X against
the FP64 oracle's literal recursion on whole-block lists
(oracle.match_trellis, pinned by brute force).

Energies within tolerances.energy_tol, assignments identical or of the
optimal FP64 energy, the FP64 re-score equal to the oracle's energy of the
GPU assignment to 1e-9.  Covered: tiny blocks (pairwise and span closeness,
infeasible cases, coincident points), the paper's video of 754 points in 723
frames at T = 10 (all 50 models in one object, sampled models against the
oracle, properties for all), no closeness limit on a 180-node block (wide
tiles) and on the whole video (properties), a 60-node block equal bit for
bit to the windowed kernel on the same lists, host = device pointers, the
one-launch run of bands that fit LDS equal bit for bit to one launch per
step, and the refused arguments.
"""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
import paper_1505_00581_amd as stm
from parity_check import check, to_np
from tolerances import energy_tol
from paper_1505_00581_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = stm.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def video():
    return synth.paper_blocks(0, n_models=50)


def _rows(tr, out, q):
    return dict(energy32=to_np(out["energy32"])[q:q + 1], energy64=to_np(out["energy64"])[q:q + 1],
                energy_u64=to_np(out["energy_u64"])[q:q + 1], assign=to_np(tr.model_rows(out, q))[None, :])


def _check_models(ctx, models, s, p, qs, b=0, e=None):
    tr = stm.Trellis(ctx, models, s, p, b, e)
    out = tr.run()
    stats = []
    for q in qs:
        ora = oracle.match_trellis(models[q], s, p, b, e)
        stats.append(check(models[q], s, p, _rows(tr, out, q), ora))
    info = tr.info()
    tr.close()
    return out, stats, info


def _tiny(seed, n_frames=7, m=4, per_frame=(0, 2), int_grid=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.integers(1, 3, size=m - 1)
    t = np.concatenate([[0], np.cumsum(gaps)]).astype(np.int32)
    model = synth.Points(rng.uniform(0, 40, (m, 2)).astype(np.float32), t, synth.dirichlet_desc(rng, m, 8))
    counts = rng.integers(per_frame[0], per_frame[1] + 1, size=n_frames)
    sxy, st, sd = synth.clutter(rng, counts, 40.0, 40.0, 8)
    if int_grid:
        sxy = (np.round(sxy / int_grid) * int_grid).astype(np.float32)
    return model, synth.assemble_scene([sxy], [st], [sd], n_frames)


@pytest.mark.parametrize("span", [False, True])
def test_tiny_blocks_against_oracle(ctx, span):
    feas = inf = 0
    for seed in range(40):
        m, s = _tiny(4000 + seed, m=[3, 4, 5][seed % 3])
        if s.n < 2:
            continue
        p = synth.Params(T=[3, 4, 0, 2, 6][seed % 5], closeness_span=span)
        _, st, _ = _check_models(ctx, [m], s, p, [0])
        feas += st[0]["feasible"]
        inf += 1 - st[0]["feasible"]
    say(f"  tiny: {feas} feasible, {inf} infeasible")
    assert feas > 15 and inf > 3


def test_tiny_blocks_with_coincident_points(ctx):
    degen = 0
    for seed in range(30):
        m, s = _tiny(4200 + seed, n_frames=8, per_frame=(1, 3), int_grid=10)
        p = synth.Params(T=5)
        _, st, info = _check_models(ctx, [m], s, p, [0])
        degen += info["degenerate"]
    assert degen > 5


def test_paper_video_t10_all_models(ctx, video):
    import torch
    s, p = video.scenes[0], video.params
    ds = stm.DevicePoints.from_host(s)
    dms = [stm.DevicePoints.from_host(m) for m in video.models]
    tr = stm.Trellis(ctx, dms, ds, p)
    out = tr.run()
    torch.cuda.synchronize()
    info = tr.info()
    say(f"  video T=10: {info}")
    e32 = to_np(out["energy32"]).astype(np.float64)
    e64 = to_np(out["energy64"])
    assert np.isfinite(e32).all()
    assert (np.abs(e32 - e64) <= energy_tol(e64)).all()  # every model: FP32 optimum = FP64 re-score
    for q, m in enumerate(video.models):
        z = to_np(tr.model_rows(out, q))
        tz = s.t[z].astype(np.int64)
        assert (np.diff(tz) > 0).all() and (np.diff(tz) < p.T).all()
    for q in (0, 1, 17, 33, 49):
        st = check(video.models[q], s, p, _rows(tr, out, q), oracle.match_trellis(video.models[q], s, p))
        say(f"  model {q}: {st}")
    tr.close()


def test_paper_video_span_reading(ctx, video):
    s = video.scenes[0]
    p = dataclasses.replace(video.params, closeness_span=True)
    _, stats, _ = _check_models(ctx, video.models[:6], s, p, [0, 3, 5])
    assert all(st["feasible"] == 1 for st in stats)


def test_no_closeness_limit_wide_tiles(ctx, video):
    # T <= 0: the upper-triangular trellis, rows of more than 128 successors
    s = video.scenes[0]
    p = dataclasses.replace(video.params, T=0)
    out, stats, info = _check_models(ctx, video.models[:4], s, p, [0, 2], 100, 280)
    say(f"  T=inf, 180 nodes: {info}, {stats}")
    assert info["tiles"] > 0


def test_no_closeness_limit_whole_video_properties(ctx, video):
    import torch
    s = video.scenes[0]
    ds = stm.DevicePoints.from_host(s)
    dms = [stm.DevicePoints.from_host(m) for m in video.models[:8]]
    res = {}
    for T in (10, 0):
        tr = stm.Trellis(ctx, dms, ds, dataclasses.replace(video.params, T=T))
        out = tr.run()
        torch.cuda.synchronize()
        res[T] = (to_np(out["energy32"]).astype(np.float64), to_np(out["energy64"]),
                  [to_np(tr.model_rows(out, q)) for q in range(len(dms))])
        tr.close()
    e_inf, e64_inf, z_inf = res[0]
    e_10 = res[10][0]
    assert (e_inf <= e_10 + energy_tol(e_10)).all()  # dropping closeness can only lower the optimum
    assert (np.abs(e_inf - e64_inf) <= energy_tol(e64_inf)).all()
    p_inf = dataclasses.replace(video.params, T=0)
    for q, m in enumerate(video.models[:8]):
        eg, _ = oracle.energies(m, s, p_inf, z_inf[q][None, :])
        assert abs(eg[0] - e64_inf[q]) <= 1e-9 * max(1.0, abs(eg[0]))
    say(f"  T=inf vs T=10 optimum: {np.round(e_inf, 3)} vs {np.round(e_10, 3)}")


def test_small_block_equals_windowed_kernel_on_same_lists(ctx, video):
    s, p = video.scenes[0], video.params
    b, e = 200, 260
    ms = video.models[:3]
    tr = stm.Trellis(ctx, ms, s, p, b, e)
    out = tr.run()
    for q, m in enumerate(ms):
        lists = np.broadcast_to(np.arange(b, e, dtype=np.int32), (1, m.n, e - b)).copy()
        cnt = np.full((1, m.n), e - b, np.int32)
        ref = ctx.match_lists(m, s, p, lists, cnt, 0, 1)
        assert to_np(out["energy32"])[q] == ref["energy32"][0]
        np.testing.assert_array_equal(to_np(tr.model_rows(out, q)), ref["assign"][0])
        assert to_np(out["energy64"])[q] == ref["energy64"][0]
    tr.close()


def test_host_and_device_pointers_agree(ctx, video):
    import torch
    s, p = video.scenes[0], video.params
    ms = video.models[:3]
    host = stm.Trellis(ctx, ms, s, p, 0, 400).run()
    tr = stm.Trellis(ctx, [stm.DevicePoints.from_host(m) for m in ms], stm.DevicePoints.from_host(s), p, 0, 400)
    dev = tr.run()
    torch.cuda.synchronize()
    for k in ("energy32", "energy64", "energy_u64", "assign"):
        np.testing.assert_array_equal(to_np(dev[k]), host[k])
    tr.close()


def test_refused_arguments(ctx, video):
    s, p = video.scenes[0], video.params
    m = video.models[0]
    for b, e in ((10, 10), (-1, 5), (0, s.n + 1)):
        with pytest.raises(stm.StmError) as ei:
            stm.Trellis(ctx, [m], s, p, b, e)
        assert ei.value.code == stm.STM_EINVAL
    for q in (dataclasses.replace(p, unary_bf16=True), dataclasses.replace(p, w_dummy=0.5),
              dataclasses.replace(p, k_density=True)):
        with pytest.raises(stm.StmError) as ei:
            stm.Trellis(ctx, [m], s, q)
        assert ei.value.code == stm.STM_EUNSUPPORTED


def _same_runs(a, b):
    for k in ("energy32", "energy64", "energy_u64", "assign"):
        np.testing.assert_array_equal(to_np(a[k]), to_np(b[k]), err_msg=k)


def test_fused_run_equals_stepwise_launches(ctx, video):
    """Bands that fit one workgroup's LDS run every step in one launch; the
    same trellis with one launch per step (STM_TRELLIS_STEPWISE) gives the
    same bits: the whole video at T = 10 (50 models, both closeness readings),
    tiny blocks with coincident points (the degenerate variant), and a block
    too large for LDS takes the per-step launches either way."""
    s = video.scenes[0]
    for p in (video.params, dataclasses.replace(video.params, closeness_span=True)):
        a = stm.Trellis(ctx, video.models, s, p)
        b = stm.Trellis(ctx, video.models, s, p, stepwise=True)
        assert a.info()["fused"] and not b.info()["fused"]
        _same_runs(a.run(), b.run())
        a.close()
        b.close()
    degen = 0
    for seed in range(30):
        m, sc = _tiny(4200 + seed, n_frames=8, per_frame=(1, 3), int_grid=10)
        p = synth.Params(T=5)
        a = stm.Trellis(ctx, [m], sc, p)
        b = stm.Trellis(ctx, [m], sc, p, stepwise=True)
        ia = a.info()
        assert ia["fused"] == (ia["cells_per_step"] > 0)
        degen += ia["degenerate"]
        _same_runs(a.run(), b.run())
        a.close()
        b.close()
    assert degen > 5
    big = stm.Trellis(ctx, video.models[:2], s, dataclasses.replace(video.params, T=0))
    assert not big.info()["fused"]
    big.close()
    say(f"  fused = stepwise on the video (both readings) and 30 tiny blocks ({degen} degenerate)")


def test_step_launch_variants_agree(ctx, video):
    """Tiles and step-launch variants change no bit.  A step launch of many
    workgroups stages fewer predecessors at a time at a higher occupancy than a
    small one, and a trellis whose step launches would have fewer than 1024
    workgroups is cut into smaller tiles (down to 256 cells).  A model's rows
    from a 50-model run (1024-cell tiles, the many-workgroup variant) equal
    those of a run of that model alone (smaller tiles) bit for bit, on the
    whole video (still many workgroups) and on a 200-node block (the
    small-launch variant)."""
    import torch
    s = video.scenes[0]
    ds = stm.DevicePoints.from_host(s)
    dms = [stm.DevicePoints.from_host(m) for m in video.models]
    p = dataclasses.replace(video.params, T=0)
    for n1, small in ((s.n, False), (200, True)):
        tr = stm.Trellis(ctx, dms, ds, p, 0, n1)
        assert tr.info()["tiles"] * len(dms) >= 1024
        out = tr.run()
        torch.cuda.synchronize()
        for q in (0, 7, 49):
            one = stm.Trellis(ctx, [dms[q]], ds, p, 0, n1)
            n_one = one.info()["tiles"]
            assert n_one > tr.info()["tiles"]
            assert (n_one < 1024) == small
            r = one.run()
            torch.cuda.synchronize()
            assert to_np(r["energy32"])[0] == to_np(out["energy32"])[q]
            assert to_np(r["energy64"])[0] == to_np(out["energy64"])[q]
            np.testing.assert_array_equal(to_np(one.model_rows(r, 0)), to_np(tr.model_rows(out, q)))
            one.close()
        say(f"  nodes 0..{n1}: {tr.info()['tiles']} tiles for 50 models, {n_one} for one")
        tr.close()


def test_graph_replays_equal_direct_launches(ctx, video):
    # runs into the same outputs replay one captured graph; a profiled run
    # launches the kernels directly: every replay, with eager work and
    # synchronisations between them, equals the direct run bit for bit
    import torch
    s, p = video.scenes[0], video.params
    dms = [stm.DevicePoints.from_host(m) for m in video.models[:5]]
    ds = stm.DevicePoints.from_host(s)
    for T in (10, 0):
        tr = stm.Trellis(ctx, dms, ds, dataclasses.replace(p, T=T), 0, 500)
        ctx.profile_enable(True)
        ref = tr.run()
        torch.cuda.synchronize()
        ctx.profile_enable(False)
        ref = {k: v.clone() for k, v in ref.items()}
        out = tr.run()
        for rep in range(3):
            torch.cuda.synchronize()
            for k in ref:
                assert torch.equal(out[k], ref[k]), (T, rep, k)
            x = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
            out["energy32"].fill_(-1.0)
            out["assign"].fill_(-7)
            torch.cuda.synchronize()
            assert float(x) == float(x)
            tr.run(out)
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(out[k], ref[k]), (T, k)
        tr.close()


def test_whole_video_against_stored_oracle_optima(ctx, video):
    """The whole 754-node video at full size, in the runs' own launch
    configurations (at T = 10 one launch for every step; with no closeness
    limit a lone model's step launches of 1,160 small tiles), against the FP64
    oracle's optima that tests/golden/make_trellis_whole_video.py stored (the
    oracle takes minutes on the no-limit trellis): energies within the
    tolerance, assignments identical or of oracle energy equal to the optimum,
    the FP64 re-score equal to the oracle's energy of the returned assignment."""
    import json
    import os
    import torch
    with open(os.path.join(os.path.dirname(__file__), "golden", "trellis_whole_video.json")) as f:
        gold = json.load(f)
    s = video.scenes[0]
    ds = stm.DevicePoints.from_host(s)
    for T in sorted({r["T"] for r in gold["rows"]}):
        rows = [r for r in gold["rows"] if r["T"] == T]
        qs = [r["model"] for r in rows]
        p = dataclasses.replace(video.params, T=T)
        tr = stm.Trellis(ctx, [stm.DevicePoints.from_host(video.models[q]) for q in qs], ds, p)
        info = tr.info()
        out = tr.run()
        torch.cuda.synchronize()
        for j, (q, g) in enumerate(zip(qs, rows)):
            m = video.models[q]
            res = _rows(tr, out, j)
            ora = dict(energy=np.array([g["energy"]]), energy_u=np.array([g["energy_u"]]),
                       assign=np.array([g["assign"]], np.int32))
            st = check(m, s, p, res, ora)
            assert st["feasible"] == 1
            say(f"  T={T} model {q}: {st}, fused={info['fused']}, tiles={info['tiles']}")
        tr.close()
