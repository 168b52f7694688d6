"""Multiple points per model frame, variant 2 of Section 4 (Table 4): several
single-point models (second-order chains), each solved independently by the
exact matching; the matching distance is the average over the chains.

TEST INFRASTRUCTURE ONLY (like the rest of `oracle`).

READING (the paper defers the details to another publication): chain c takes
the c-th most salient point of every model frame that has more than c points
(salient = the detector's confidence, as the paper uses it to keep one point
per frame, Section 2.1; equal confidences by point order), for c = 0 ..
n_chains - 1; chains of fewer than 3 points are dropped.  A model offset tau
places the model's first frame at scene frame tau; chain c is matched at its
own offset tau + (first frame of c - first frame of the model).  The distance
at tau is the mean of the chains' optimal energies (+inf if one is infeasible).
"""
from __future__ import annotations

import numpy as np

from . import energy as E
from . import match as _match

UNCHAINED = -3  # assignment value of a point that belongs to no chain


def build_chains(t, saliency, n_chains: int) -> list:
    """Point indices of each kept chain, in frame order."""
    t = np.asarray(t)
    n = t.shape[0]
    sal = np.zeros(n) if saliency is None else np.asarray(saliency, np.float64)
    chains = [[] for _ in range(n_chains)]
    start = 0
    while start < n:
        end = start
        while end < n and t[end] == t[start]:
            end += 1
        ranked = sorted(range(start, end), key=lambda q: (-sal[q], q))
        for c, q in enumerate(ranked[:n_chains]):
            chains[c].append(q)
        start = end
    return [c for c in chains if len(c) >= 3]


class _Chain:
    """The points idx of a model as a model of their own."""

    def __init__(self, model, idx):
        idx = np.asarray(idx)
        self.xy = np.ascontiguousarray(model.xy[idx])
        self.t = np.ascontiguousarray(model.t[idx])
        self.desc = np.ascontiguousarray(model.desc[idx])
        self.n = int(idx.shape[0])
        self.dim = int(self.desc.shape[1])


def sub_model(model, idx):
    return _Chain(model, idx)


def match_chains(model, scene, params, saliency, n_chains: int, taus=None):
    """Mean chain energy at each model offset (default: every offset of the
    whole model) and the assignment of every model point.  Returns dict(energy,
    energy_u, assign [n, M] (UNCHAINED for points of no chain), chains, taus)."""
    chains = build_chains(model.t, saliency, n_chains)
    if not chains:
        raise ValueError("no chain of 3 or more points")
    if taus is None:
        taus = np.arange(len(E.offsets(model.t, scene.n_frames)), dtype=np.int32)
    taus = np.asarray(taus, np.int32)
    n = taus.shape[0]
    e = np.zeros(n)
    eu = np.zeros(n)
    A = np.full((n, model.n), UNCHAINED, np.int32)
    for idx in chains:
        delta = int(model.t[idx[0]]) - int(model.t[0])
        r = _match(sub_model(model, idx), scene, params, taus=taus + delta)
        e += r["energy"]
        eu += r["energy_u"]
        A[:, idx] = r["assign"]
    return dict(energy=e / len(chains), energy_u=eu / len(chains), assign=A, chains=chains, taus=taus)
