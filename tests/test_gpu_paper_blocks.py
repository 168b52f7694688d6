"""The paper's own streaming workload on MI355X (Table 2's 60-node blocks):
M=30 models against overlapping blocks of 60 consecutive scene points, every
block one candidate list for every model point.  The recursion on those lists
(stm_match_lists) against the FP64 oracle's recursion on the same lists."""
import sys

import numpy as np
import pytest

import oracle
import paper_1505_00581_amd as stm
from oracle import energy as E
from paper_1505_00581_amd import synth

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-5, 1e-4


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
        assert (np.abs(got["energy32"][sample][fin] - e[fin]) <= np.maximum(RTOL * e[fin], ATOL)).all()
        eg, _ = oracle.energies(m, s, p, got["assign"][sample][fin])
        assert (np.abs(eg - e[fin]) <= np.maximum(RTOL * e[fin], ATOL)).all()
        np.testing.assert_allclose(got["energy64"][sample][fin], eg, rtol=1e-9)
        checked += int(fin.sum())
    print(f"  {checked} block matchings agree with the oracle", file=sys.stderr)
    assert checked >= 6
    ctx.close()
