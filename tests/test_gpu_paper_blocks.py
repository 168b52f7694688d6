"""The paper's own streaming workload on MI355X (Table 2's 60-node blocks):
M=30 models against overlapping blocks of 60 consecutive scene points, every
block one candidate list for every model point.  The recursion on those lists
(stm_match_lists) against the FP64 oracle's recursion on the same lists."""
import sys

import numpy as np
import pytest

import oracle
import paper_1505_00581_amd as stm
from tolerances import energy_tol
from oracle import energy as E
from paper_1505_00581_amd import synth

pytestmark = pytest.mark.gpu



def test_blocks_against_oracle():
    ctx = stm.Context(0)
    w = synth.paper_blocks(0, n_models=2)
    s, p = w.scenes[0], w.params
    checked = 0
    for m in w.models:
        n_blocks = min(40, len(E.offsets(m.t, s.n_frames)))
        cand, cnt = synth.block_lists(m, s, n_blocks)
        got = ctx.match_lists(m, s, p, cand, cnt, 0, n_blocks)
        sample = np.array([0, 7, 19, 33, n_blocks - 1])
        ora = oracle.match_lists(m, s, p, cand[sample], cnt[sample])
        e = ora["energy"]
        fin = np.isfinite(e)
        assert (np.isfinite(got["energy32"][sample]) == fin).all()
        assert (np.abs(got["energy32"][sample][fin] - e[fin]) <= energy_tol(e[fin])).all()
        eg, _ = oracle.energies(m, s, p, got["assign"][sample][fin])
        assert (np.abs(eg - e[fin]) <= energy_tol(e[fin])).all()
        np.testing.assert_allclose(got["energy64"][sample][fin], eg, rtol=1e-9)
        checked += int(fin.sum())
    print(f"  {checked} block matchings agree with the oracle", file=sys.stderr)
    assert checked >= 6
    ctx.close()


def _plan_block_lists(m, s, n_rows, block=60):
    """Block lists for every row of a plan pair: row b lists scene points b ..
    b + block - 1 while they exist, no candidates after (infeasible rows)."""
    n_blocks = min(n_rows, s.n - block + 1)
    cand = np.zeros((n_rows, m.n, block), np.int32)
    cnt = np.zeros((n_rows, m.n), np.int32)
    c, n = synth.block_lists(m, s, n_blocks, block)
    cand[:n_blocks], cnt[:n_blocks] = c, n
    return cand, cnt


def test_plan_on_lists_equals_per_model_lists():
    import torch
    ctx = stm.Context(0)
    w = synth.paper_blocks(1, n_models=5)
    s, p = w.scenes[0], w.params
    ds = stm.DevicePoints.from_host(s)
    dms = [stm.DevicePoints.from_host(m) for m in w.models]
    plan = stm.Plan(ctx, dms, [ds], np.array([(i, 0) for i in range(len(dms))], np.int32), p)
    cands, counts = [], []
    for q, m in enumerate(w.models):
        n_rows = int(plan.row_offsets[q + 1] - plan.row_offsets[q])
        c, n = _plan_block_lists(m, s, n_rows)
        cands.append(torch.as_tensor(c, device="cuda"))
        counts.append(torch.as_tensor(n, device="cuda"))
    out = plan.run_lists(cands, counts, 60)
    out2 = plan.run_lists(cands, counts, 60, out={k: torch.empty_like(v) for k, v in out.items()})
    torch.cuda.synchronize()
    n = 0
    for q, m in enumerate(w.models):
        e32, e64, eu, A = [x.cpu().numpy() for x in plan.pair_rows(out, q)]
        ref = ctx.match_lists(m, s, p, cands[q].cpu().numpy(), counts[q].cpu().numpy(), 0, e32.shape[0])
        np.testing.assert_array_equal(e32, ref["energy32"])
        np.testing.assert_array_equal(A, ref["assign"])
        np.testing.assert_array_equal(e64, ref["energy64"])
        np.testing.assert_array_equal(plan.pair_rows(out2, q)[0].cpu().numpy(), e32)
        n += int(np.isfinite(e32).sum())
    print(f"  {n} feasible block matchings identical to per-model list runs", file=sys.stderr)
    assert n > 100
    bad = [c.clone() for c in counts]
    bad[0][0, 0] = 61
    with pytest.raises(stm.StmError, match="candidate lists"):
        plan.run_lists(cands, bad, 60)
    plan.close()
    ctx.close()
