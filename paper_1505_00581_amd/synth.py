"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random point sets; it holds none of the matching
method's arithmetic, so both the CPU oracle tests and the HIP path use it.

Stand-ins (the KTH videos, their STIP points and HoG/HoF features are not
available): image planes of 160x120 (KTH, Section 4) or 320x240 px, 162-D
non-negative L1-normalised descriptors drawn from Dirichlet(0.5), models with
one point per frame and strictly increasing frames (Section 2.1), scenes with
many points per frame sorted by frame.  Planted copies of each model give the
scene true matches: a scaled and translated copy with Gaussian xy jitter,
frame jitter and descriptor noise.

All generators use numpy's PCG64 with an explicit seed.  Coordinates and
descriptors are float32, frames int32.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

DIM = 162


@dataclasses.dataclass
class Points:
    """A point set: xy [n,2] float32 px, t [n] int32 frames, desc [n,dim] float32."""

    xy: np.ndarray
    t: np.ndarray
    desc: np.ndarray
    n_frames: int = 0  # scenes only: number of frames; frames lie in [0, n_frames)

    @property
    def n(self) -> int:
        return int(self.t.shape[0])

    @property
    def dim(self) -> int:
        return int(self.desc.shape[1])


@dataclasses.dataclass
class Params:
    """Energy weights and search window (defaults: Section 4 of the paper)."""

    lambda1: float = 0.6
    lambda2: float = 0.2
    lambda3: float = 5.0
    T: int = 10          # temporal closeness in frames; <= 0 means no limit
    window: int = 2      # candidate window half-width W in frames
    k_max: int = 16      # candidate cap K
    k_density: bool = False  # per-point K from local density (batched workload)
    unary_bf16: bool = False  # unary table from BF16 descriptors on MFMA
    w_dummy: float | None = None  # W^d: unary cost of a dummy assignment (Eq. 2); None = no dummies
    closeness_span: bool = False  # closeness as the triangle span t'(z_i) - t'(z_{i-2}) < T (Eq. 14)
    angle_unsigned: bool = False  # triangle angles as magnitudes in [0, pi] (Eq. 6, alternative reading)
    causal_node: bool = False  # causality as node order z_{i-1} < z_i (Eq. 7, alternative reading)


@dataclasses.dataclass
class Workload:
    models: list
    scenes: list
    params: Params
    planted: list  # (model index, scene index, tau) of every planted copy
    name: str = ""
    saliency: list = dataclasses.field(default_factory=list)  # per model: detector confidence per point


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def dirichlet_desc(rng: np.random.Generator, n: int, dim: int = DIM) -> np.ndarray:
    return rng.dirichlet(np.full(dim, 0.5), size=n).astype(np.float32)


def model_frames(rng: np.random.Generator, m: int, hi: int, T: int) -> np.ndarray:
    """m distinct frames from {0..hi}, sorted, redrawn until every gap is < T."""
    for _ in range(10000):
        f = np.sort(rng.choice(hi + 1, size=m, replace=False))
        if T <= 0 or m < 2 or int(np.max(np.diff(f))) < T:
            return (f - f[0]).astype(np.int32)
    raise RuntimeError("could not draw model frames")


def make_model(rng, m: int, width: float, height: float, T: int,
               frame_hi: int | None = None, dim: int = DIM) -> Points:
    hi = frame_hi if frame_hi is not None else int(math.ceil(1.5 * m))
    t = model_frames(rng, m, hi, T)
    xy = np.stack([rng.uniform(0, width, m), rng.uniform(0, height, m)], 1)
    return Points(xy.astype(np.float32), t, dirichlet_desc(rng, m, dim))


def plant_copy(rng, model: Points, n_frames: int, width: float, height: float,
               xy_sigma: float = 3.0, t_sigma: float = 1.0, desc_sigma: float = 0.02,
               tau: int | None = None):
    """A scaled, translated, jittered copy of `model` placed at offset tau."""
    span = int(model.t[-1] - model.t[0])
    if tau is None:
        tau = int(rng.integers(0, n_frames - span))
    s = rng.uniform(0.9, 1.1)
    c = model.xy.astype(np.float64).mean(0)
    target = np.array([rng.uniform(0, width), rng.uniform(0, height)])
    xy = (model.xy - c) * s + target + rng.normal(0, xy_sigma, model.xy.shape)
    tt = tau + (model.t - model.t[0]) + np.rint(rng.normal(0, t_sigma, model.n))
    tt = np.clip(tt, 0, n_frames - 1).astype(np.int32)
    g = np.maximum(model.desc + rng.normal(0, desc_sigma, model.desc.shape), 0.0)
    sums = g.sum(1, keepdims=True)
    g = np.where(sums > 0, g / np.where(sums > 0, sums, 1.0), model.desc)
    return xy.astype(np.float32), tt, g.astype(np.float32), tau


def assemble_scene(xy_parts, t_parts, d_parts, n_frames: int) -> Points:
    """Concatenate parts and sort by (frame, x); node ids are the sorted order."""
    xy = np.concatenate(xy_parts).astype(np.float32)
    t = np.concatenate(t_parts).astype(np.int32)
    d = np.concatenate(d_parts).astype(np.float32)
    order = np.lexsort((xy[:, 0], t))
    return Points(np.ascontiguousarray(xy[order]), np.ascontiguousarray(t[order]),
                  np.ascontiguousarray(d[order]), n_frames)


def clutter(rng, counts: np.ndarray, width: float, height: float, dim: int = DIM):
    """Uniform clutter: counts[f] points in frame f."""
    n = int(counts.sum())
    t = np.repeat(np.arange(counts.shape[0], dtype=np.int32), counts)
    xy = np.stack([rng.uniform(0, width, n), rng.uniform(0, height, n)], 1)
    return xy.astype(np.float32), t, dirichlet_desc(rng, n, dim)


def make_scene(rng, models, n_frames: int, counts: np.ndarray, width: float,
               height: float, planted_per_model: int, n_scenes_for_plant=None):
    xy, t, d = clutter(rng, counts, width, height, models[0].dim if models else DIM)
    parts = ([xy], [t], [d])
    planted = []
    for mi, m in enumerate(models):
        for _ in range(planted_per_model):
            pxy, pt, pd, tau = plant_copy(rng, m, n_frames, width, height)
            parts[0].append(pxy)
            parts[1].append(pt)
            parts[2].append(pd)
            planted.append((mi, 0, tau))
    return assemble_scene(*parts, n_frames), planted


# ---------------------------------------------------------------------------
# The five workloads.  Sizes follow the configurations the benchmarks quote.
# ---------------------------------------------------------------------------

def config1(seed: int = 0) -> Workload:
    """One model of M=20 points (160x120 px, frames in 0..30) against a scene of
    100 frames with 4 clutter points per frame plus 2 planted copies.
    W=2, K=16."""
    rng = _rng(seed)
    p = Params(window=2, k_max=16)
    model = make_model(rng, 20, 160.0, 120.0, p.T, frame_hi=30)
    scene, planted = make_scene(rng, [model], 100, np.full(100, 4), 160.0, 120.0, 2)
    return Workload([model], [scene], p, planted, "c1_exact_m20_s100x4_k16")


def config2(seed: int = 0, n_models: int = 10) -> Workload:
    """10 models with M in {50..100} against one 1500-frame scene (320x240 px,
    20 clutter points per frame, 5 planted copies per model).  W=3, K=64."""
    rng = _rng(seed)
    p = Params(window=3, k_max=64)
    ms = [make_model(rng, int(rng.integers(50, 101)), 320.0, 240.0, p.T)
          for _ in range(n_models)]
    scene, planted = make_scene(rng, ms, 1500, np.full(1500, 20), 320.0, 240.0, 5)
    return Workload(ms, [scene], p, planted, "c2_realistic_10models_s1500x20_k64")


def config3(seed: int = 0, n_models: int = 64, n_scenes: int = 8) -> Workload:
    """64 models with M in [30,150] against 8 scenes of 500..3000 frames with
    10..30 points per frame; 2 planted copies of each model in random scenes.
    W=3, per-point K in [8,64] from the local point density."""
    rng = _rng(seed)
    p = Params(window=3, k_max=64, k_density=True)
    ms = [make_model(rng, int(rng.integers(30, 151)), 320.0, 240.0, p.T)
          for _ in range(n_models)]
    frames = [int(rng.integers(500, 3001)) for _ in range(n_scenes)]
    parts = []
    for f in frames:
        counts = rng.integers(10, 31, size=f)
        parts.append(list(clutter(rng, counts, 320.0, 240.0)))
    planted = []
    for mi, m in enumerate(ms):
        for _ in range(2):
            si = int(rng.integers(0, n_scenes))
            span = int(m.t[-1] - m.t[0])
            if frames[si] - span < 1:
                continue
            pxy, pt, pd, tau = plant_copy(rng, m, frames[si], 320.0, 240.0)
            parts[si][0] = np.concatenate([parts[si][0], pxy])
            parts[si][1] = np.concatenate([parts[si][1], pt])
            parts[si][2] = np.concatenate([parts[si][2], pd])
            planted.append((mi, si, tau))
    scenes = [assemble_scene([a], [b], [c], f) for (a, b, c), f in zip(parts, frames)]
    return Workload(ms, scenes, p, planted, "c3_batched_64models_8scenes_kdensity")


def tiny(seed: int, m: int | None = None, max_per_frame: int = 3, n_frames: int | None = None,
         window: int = 1, k_max: int = 5, T: int = 4, int_coords: bool = False) -> Workload:
    """Tiny random cases for brute-force checks: M in 3..6 points, a short scene
    with 0..max_per_frame points per frame, small windows so every candidate
    list has at most k_max entries.  Some offsets are infeasible on purpose
    (empty frames, tight T)."""
    rng = _rng(seed)
    m = m if m is not None else int(rng.integers(3, 7))
    gaps = rng.integers(1, 3, size=m - 1)
    t = np.concatenate([[0], np.cumsum(gaps)]).astype(np.int32)
    xy = rng.uniform(0, 40, (m, 2))
    if int_coords:
        xy = np.round(xy)
    model = Points(xy.astype(np.float32), t, dirichlet_desc(rng, m, 8))
    nf = n_frames if n_frames is not None else int(t[-1]) + int(rng.integers(2, 5))
    counts = rng.integers(0, max_per_frame + 1, size=nf)
    sxy, st, sd = clutter(rng, counts, 40.0, 40.0, 8)
    if int_coords:
        sxy = np.round(sxy).astype(np.float32)
    scene = assemble_scene([sxy], [st], [sd], nf)
    p = Params(window=window, k_max=k_max, T=T)
    return Workload([model], [scene], p, [], f"tiny_{seed}")


def paper_blocks(seed: int = 0, n_models: int = 50, block: int = 60) -> Workload:
    """The paper's own timing workload (Table 2, streaming mode): models of
    M=30 points (160x120 px, frames in 0..45) against one video of 723 frames
    with 754 points (about one per frame, as KTH's interest points are), matched
    against overlapping blocks of `block` consecutive scene points (about 55
    frames).  Five models have one planted copy each; the rest is clutter.
    W and K do not apply: each block is one candidate list for every point."""
    rng = _rng(seed)
    p = Params(window=0, k_max=block)
    models = [make_model(rng, 30, 160.0, 120.0, p.T, frame_hi=45) for _ in range(n_models)]
    n_frames, n_points, n_planted = 723, 754, min(5, n_models)
    counts = rng.multinomial(n_points - 30 * n_planted, np.full(n_frames, 1.0 / n_frames))
    xy, t, d = clutter(rng, counts, 160.0, 120.0)
    parts = ([xy], [t], [d])
    planted = []
    for mi in range(n_planted):
        pxy, pt, pd, tau = plant_copy(rng, models[mi], n_frames, 160.0, 120.0)
        parts[0].append(pxy)
        parts[1].append(pt)
        parts[2].append(pd)
        planted.append((mi, 0, tau))
    scene = assemble_scene(*parts, n_frames)
    return Workload(models, [scene], p, planted, f"paper_blocks_m30_s{n_points}_b{block}")


def multipoint(seed: int = 0, n_models: int = 2, frames: tuple = (50, 100), per_frame: int = 3,
               n_frames: int = 1500, clutter_per_frame: int = 20, window: int = 3, k_max: int = 64,
               width: float = 320.0, height: float = 240.0, planted_per_model: int = 5) -> Workload:
    """Models with 1..per_frame interest points in each model frame (the
    multiple-points models of Table 4) against one scene with planted copies.
    Model frames: distinct, drawn from {0..1.5 F_m} with gaps < T; points per
    frame U{1..per_frame}, raised so that no chain level skips more than 3
    frames; each point gets a detector confidence U(0, 1) (Workload.saliency).
    Points are stored by frame, then by draw order."""
    rng = _rng(seed)
    p = Params(window=window, k_max=k_max)
    models, sal = [], []
    for _ in range(n_models):
        nf = int(rng.integers(frames[0], frames[1] + 1))
        ft = model_frames(rng, nf, int(math.ceil(1.5 * nf)), p.T)
        per = rng.integers(1, per_frame + 1, size=nf)
        # keep every chain level dense: a frame more than 3 frames after the
        # last one holding a (c+1)-th point gets one
        for c in range(1, per_frame):
            last = None
            for k in range(nf):
                if per[k] > c:
                    last = ft[k]
                elif last is not None and ft[k] - last > 3:
                    per[k] = c + 1
                    last = ft[k]
        t = np.repeat(ft, per).astype(np.int32)
        m = int(t.shape[0])
        xy = np.stack([rng.uniform(0, width, m), rng.uniform(0, height, m)], 1).astype(np.float32)
        models.append(Points(xy, t, dirichlet_desc(rng, m)))
        sal.append(rng.uniform(0.0, 1.0, m).astype(np.float32))
    scene, planted = make_scene(rng, models, n_frames, np.full(n_frames, clutter_per_frame), width, height,
                                planted_per_model)
    return Workload(models, [scene], p, planted, f"multipoint_{n_models}models_{per_frame}perframe",
                    saliency=sal)


def block_lists(model: Points, scene: Points, n_blocks: int, block: int = 60):
    """Candidate lists of the block workload: offset b lists scene points
    b .. b + block - 1 for every model point.  Returns cand [n, M, block] and
    count [n, M] (int32)."""
    M = model.n
    base = np.arange(block, dtype=np.int32)
    cand = np.broadcast_to((np.arange(n_blocks, dtype=np.int32)[:, None] + base[None, :])[:, None, :],
                           (n_blocks, M, block)).copy()
    count = np.full((n_blocks, M), block, np.int32)
    return cand, count


def pruner_init(dim: int = DIM, seed: int = 0, hidden: int = 128) -> np.ndarray:
    """Initial weights of the learned candidate pruner, packed float32
    [W1 (hidden x (2 dim + 8)), b1, W2 (hidden x hidden), b2, w3, b3]:
    He-uniform weights (bound sqrt(6 / fan_in)), zero biases."""
    rng = _rng(seed)
    n_in = 2 * dim + 8
    parts = [rng.uniform(-1, 1, (hidden, n_in)) * math.sqrt(6.0 / n_in), np.zeros(hidden),
             rng.uniform(-1, 1, (hidden, hidden)) * math.sqrt(6.0 / hidden), np.zeros(hidden),
             rng.uniform(-1, 1, hidden) * math.sqrt(6.0 / hidden), np.zeros(1)]
    return np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)
