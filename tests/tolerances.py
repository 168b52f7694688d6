"""Energy tolerances of the GPU parity tests (FP32 recursion against the FP64
oracle).

* |E| > 0.1: 1e-5 relative, the stated target for energies.
* |E| <= 0.1: 1e-4 absolute.  Such energies come from exact or near-exact
  copies of the model, where the exact energy is 0 or close to it: each FP32
  scene direction carries up to 3.5e-7 rad from the atan2 polynomial and the
  rounding of its inputs, so every triangle can add a few 1e-7 of D^g
  (lambda2 lambda3 = 1 at the paper's weights) and a chain of ~150 triangles
  up to ~1e-4, while no relative bound is meaningful near 0.
"""
import numpy as np

RTOL = 1e-5
NEAR_ZERO = 0.1
ATOL_NEAR_ZERO = 1e-4


def energy_tol(e):
    """Per-element tolerance of an FP32 energy against the oracle's E."""
    a = np.abs(np.asarray(e, np.float64))
    return np.where(a > NEAR_ZERO, RTOL * a, ATOL_NEAR_ZERO)


def max_rel_err(got, want):
    """Largest |got - want| / |want| over energies above NEAR_ZERO (0 if none)."""
    got, want = np.asarray(got, np.float64), np.asarray(want, np.float64)
    m = np.abs(want) > NEAR_ZERO
    return float((np.abs(got[m] - want[m]) / np.abs(want[m])).max()) if m.any() else 0.0
