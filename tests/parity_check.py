"""Element-wise comparison of GPU matching results with the FP64 oracle's,
shared by the GPU parity tests.

Energies within tolerances.energy_tol; infeasible offsets identical (+inf,
assignment -1); assignments identical, or (several optima, or a margin below
the tolerance) the oracle's FP64 energy of the GPU assignment equal to the
optimum within the same tolerance; the GPU's FP64 re-score equal to the
oracle's literal energy of the same assignment to 1e-9.
"""
import numpy as np

import oracle
from tolerances import energy_tol


def to_np(x):
    if hasattr(x, "cpu"):
        return x.cpu().numpy()
    return np.asarray(x)


def check(m, s, p, res, ora, rows=None):
    """Compares rows `rows` (default all) of GPU results `res` with oracle
    results `ora`; returns a small summary."""
    e32 = to_np(res["energy32"]).astype(np.float64)
    e64 = to_np(res["energy64"])
    eu64 = to_np(res["energy_u64"])
    A = to_np(res["assign"])
    if rows is not None:
        e32, e64, eu64, A = e32[rows], e64[rows], eu64[rows], A[rows]
    E, Z = ora["energy"], ora["assign"]
    inf_g, inf_o = ~np.isfinite(e32), ~np.isfinite(E)
    assert (inf_g == inf_o).all(), np.nonzero(inf_g != inf_o)[0][:10]
    assert (A[inf_g] == -1).all()
    assert (~np.isfinite(e64[inf_g])).all()
    fin = ~inf_o
    if not fin.any():
        return dict(n=len(E), feasible=0, agree=1.0, max_rel=0.0)
    tol = energy_tol(E[fin])
    err = np.abs(e32[fin] - E[fin])
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, f"energy mismatch at {bad[:5]}: gpu {e32[fin][bad[:5]]} oracle {E[fin][bad[:5]]}"
    Af, Zf = A[fin], Z[fin]
    same = (Af == Zf).all(1)
    eg, eu = oracle.energies(m, s, p, Af)
    if not same.all():
        d = np.abs(eg[~same] - E[fin][~same])
        assert (d <= tol[~same]).all(), f"different assignment with energy gap {d.max()}"
    assert np.allclose(e64[fin], eg, rtol=1e-9, atol=1e-9), np.abs(e64[fin] - eg).max()
    assert np.allclose(eu64[fin], eu, rtol=1e-9, atol=1e-9)
    return dict(n=len(E), feasible=int(fin.sum()), agree=float(same.mean()),
                max_rel=float((err / np.maximum(np.abs(E[fin]), 1e-30)).max()))
