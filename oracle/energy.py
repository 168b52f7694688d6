"""Plain FP64 definitions of the matching energy and a brute-force minimiser.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module;
only the tests, the smoke check and the benchmark's CPU-baseline leg use it.

Every function restates one passage of Lombardi, Wolf, Celiktutan and Sankur,
"Activity recognition from videos with parallel hypergraph matching on GPUs"
(arXiv 1505.00581).  Readings where the paper is silent are marked READING and
listed, with reasons, in the design notes of the repository.

Conventions (all FP64; float32 inputs are upcast exactly):
  * model: M points, xy [M,2], frames t [M] strictly increasing, desc [M,D];
  * scene: S points sorted by frame, xy [S,2], frames t' [S], desc [S,D];
  * an assignment z maps model point i (0-based here) to a scene node id, or
    to the dummy value epsilon (DUMMY = -2) when dummy assignments are enabled
    (params.w_dummy = W^d, the dummy's unary cost of Eq. 2; None = disabled).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

INF = math.inf
DUMMY = -2  # the dummy value epsilon of Eq. 2 in assignments


def w_dummy(params):
    """W^d of Eq. 2, or None when dummy assignments are disabled."""
    return getattr(params, "w_dummy", None)


def offsets(model_t: np.ndarray, n_frames: int) -> range:
    """Scene time offsets tau at which the whole model fits in the scene.

    READING: the paper matches a model against a scene block (Section 2); the
    per-offset search places model frame t_i at scene frame tau + t_i - t_1, for
    every tau with the last model frame still inside the scene."""
    span = int(model_t[-1]) - int(model_t[0])
    return range(0, max(0, n_frames - span))


def density_k(scene_t: np.ndarray, f: int, k_max: int) -> int:
    """Per-point candidate cap from the local point density (batched workload):
    rho = points in frames f-1..f+1; K = 8 + 56 (rho - 30) / 60 rounded half up,
    clamped to [8, 64], and never above k_max."""
    rho = int(np.count_nonzero(np.abs(scene_t.astype(np.int64) - f) <= 1))
    k = (56 * rho - 1170) // 60  # floor(8 + 56 (rho-30)/60 + 1/2)
    return int(min(max(k, 8), 64, k_max))


def candidates(model_t, scene_t, tau: int, i: int, window: int, k_max: int,
               k_density: bool = False) -> np.ndarray:
    """Candidate scene nodes of model point i at offset tau.

    Nodes whose frame lies within `window` frames of tau + (t_i - t_1); the
    first K of them ordered by (|frame difference|, node id) are kept and
    returned in ascending node order.  READING: a bounded per-point search
    window stands in for the paper's trellis pruning by causality and
    closeness (Sections 3.2 and 3.4); the integer-only rule keeps candidate
    sets identical across precisions."""
    f = tau + int(model_t[i]) - int(model_t[0])
    st = scene_t.astype(np.int64)
    nodes = [n for n in range(st.shape[0]) if abs(int(st[n]) - f) <= window]
    nodes.sort(key=lambda n: (abs(int(st[n]) - f), n))
    k = density_k(scene_t, f, k_max) if k_density else k_max
    return np.array(sorted(nodes[:k]), dtype=np.int64)


def unary(f_model: np.ndarray, g_scene: np.ndarray) -> float:
    """U(z_i) = ||f_i - f'_{z_i}||, the Euclidean descriptor distance (Eq. 2).
    Squares are summed in index order, then the square root is taken."""
    d = f_model.astype(np.float64) - g_scene.astype(np.float64)
    s = 0.0
    for v in d:
        s += float(v) * float(v)
    return math.sqrt(s)


def ang(a, b, c) -> float:
    """Oriented angle subtended at vertex b by the triangle (a, b, c), from ray
    b->a to ray b->c, in (-pi, pi]: atan2(cross, dot) of the two sides.

    READING: image-plane angles (the temporal part is handled by D^t, Eq. 3);
    oriented, since the paper asks for differences on the circular domain
    (Eq. 6).  A zero-length side gives angle 0."""
    ux, uy = float(a[0]) - float(b[0]), float(a[1]) - float(b[1])
    vx, vy = float(c[0]) - float(b[0]), float(c[1]) - float(b[1])
    if (ux == 0.0 and uy == 0.0) or (vx == 0.0 and vy == 0.0):
        return 0.0
    return math.atan2(ux * vy - uy * vx, ux * vx + uy * vy)


def wrap(x: float) -> float:
    """Angle difference on the circle: x - 2 pi round(x / 2 pi)."""
    return x - 2.0 * math.pi * round(x / (2.0 * math.pi))


def closeness_span(params) -> bool:
    """True for the span reading of temporal closeness (flag STM_CLOSENESS_SPAN)."""
    return bool(getattr(params, "closeness_span", False))


def span_ok(tp_first: int, tp_last: int, T: int) -> bool:
    """Span reading of temporal closeness, from the loop bounds of Section 3.4
    (Eq. 14, second line): the scene frames of the three points of a triangle
    (z_{i-2}, z_{i-1}, z_i) lie less than T apart, t'(z_i) - t'(z_{i-2}) < T.
    T <= 0 means no limit.  Under this reading consecutive points keep
    causality (Eq. 7) only; their closeness follows from the triangles."""
    return T <= 0 or int(tp_last) - int(tp_first) < T


def causal_node(params) -> bool:
    """True for causality by scene node order (flag STM_CAUSAL_NODE): z_{i-1} <
    z_i as node ids, which in a scene sorted by frame allows equal frames."""
    return bool(getattr(params, "causal_node", False))


def admissible_node(z_prev: int, z_cur: int, tp_prev: int, tp_cur: int, T: int) -> bool:
    """Causality by node order and temporal closeness (Eq. 8) for consecutive
    model points: z_{i-1} < z_i, scene frames less than T apart."""
    return z_prev < z_cur and (T <= 0 or tp_cur - tp_prev < T)


def admissible(tp_prev: int, tp_cur: int, T: int) -> bool:
    """Causality (Eq. 7) for consecutive model points i-1 < i: the scene frames
    must be strictly increasing.  Temporal closeness (Eq. 8): consecutive scene
    frames less than T apart; T <= 0 means no closeness limit."""
    if not tp_prev < tp_cur:
        return False
    return T <= 0 or tp_cur - tp_prev < T


def delta(t_p: int, t_q: int, tp_p: int, tp_q: int) -> float:
    """Delta(p, q) = |(t(p) - t(q)) - (t'(z_p) - t'(z_q))| (Eq. 5)."""
    return float(abs((int(t_p) - int(t_q)) - (int(tp_p) - int(tp_q))))


def angle_unsigned(params) -> bool:
    """True for the unsigned reading of the triangle angles (flag
    STM_ANGLE_UNSIGNED): each angle is the magnitude of the oriented one, in
    [0, pi], so a triangle and its mirror image have the same angles."""
    return bool(getattr(params, "angle_unsigned", False))


def triangle_cost(model, scene, i: int, zi: int, zj: int, zk: int, lambda3: float,
                  unsigned: bool = False) -> float:
    """D(z_i, z_{i-1}, z_{i-2}) = D^t + lambda3 D^g for the hyperedge
    (i, j, k) = (i, i-1, i-2) of the chain (Eq. 3, Eq. 9).

    D^t = Delta(i, j) + Delta(j, k) (Eq. 4).
    D^g = L2 norm of the wrapped differences of the angle at j and the angle
    at i between model and scene triangles (Eq. 6); with `unsigned`, of the
    differences of their magnitudes.

    READING for dummies (the paper defines only U for them, Eq. 2): a Delta
    term counts only when both of its points are scene points, D^g only when
    all three are."""
    j, k = i - 1, i - 2
    mt, st = model.t, scene.t
    dt = 0.0
    if zi != DUMMY and zj != DUMMY:
        dt += delta(mt[i], mt[j], st[zi], st[zj])
    if zj != DUMMY and zk != DUMMY:
        dt += delta(mt[j], mt[k], st[zj], st[zk])
    if DUMMY in (zi, zj, zk):
        return dt
    p, q = model.xy.astype(np.float64), scene.xy.astype(np.float64)
    a_mid = (ang(p[i], p[j], p[k]), ang(q[zi], q[zj], q[zk]))
    a_end = (ang(p[j], p[i], p[k]), ang(q[zj], q[zi], q[zk]))
    if unsigned:
        a_mid = (abs(a_mid[0]), abs(a_mid[1]))
        a_end = (abs(a_end[0]), abs(a_end[1]))
    d_mid = wrap(a_mid[0] - a_mid[1])
    d_end = wrap(a_end[0] - a_end[1])
    return dt + lambda3 * math.sqrt(d_mid * d_mid + d_end * d_end)


def unary_of(model, scene, i: int, zi: int, params) -> float:
    """U(z_i) of Eq. 2: the descriptor distance, or W^d for the dummy."""
    return float(w_dummy(params)) if zi == DUMMY else unary(model.desc[i], scene.desc[zi])


def energy(model, scene, z, params) -> float:
    """E(z) = lambda1 sum_i U(z_i) + lambda2 sum_{i>=3} D(z_i, z_{i-1}, z_{i-2})
    (Eq. 1 restricted to the chain hypergraph, Eq. 9), or +inf when a pair of
    consecutive points breaks causality or closeness (Eq. 7, Eq. 8).  READING:
    the constraints bind consecutive points that are both scene points; a
    dummy on either side lifts them.  With params.closeness_span, closeness is
    the span of each triangle instead (span_ok, Section 3.4); with
    params.angle_unsigned, D^g compares the magnitudes of the angles; with
    params.causal_node, causality is node order (admissible_node)."""
    M = len(z)
    if DUMMY in list(z) and w_dummy(params) is None:
        return INF
    if closeness_span(params):
        if DUMMY in list(z):
            raise ValueError("the span reading of closeness is not defined with dummies")
        st = scene.t
        for i in range(1, M):
            if not int(st[z[i - 1]]) < int(st[z[i]]):  # causality (Eq. 7)
                return INF
        for i in range(2, M):
            if not span_ok(st[z[i - 2]], st[z[i]], params.T):
                return INF
    else:
        for i in range(1, M):
            if z[i - 1] == DUMMY or z[i] == DUMMY:
                continue
            tp, tc = int(scene.t[z[i - 1]]), int(scene.t[z[i]])
            ok = (admissible_node(int(z[i - 1]), int(z[i]), tp, tc, params.T) if causal_node(params)
                  else admissible(tp, tc, params.T))
            if not ok:
                return INF
    eu = sum(unary_of(model, scene, i, z[i], params) for i in range(M))
    ed = sum(triangle_cost(model, scene, i, z[i], z[i - 1], z[i - 2], params.lambda3, angle_unsigned(params))
             for i in range(2, M))
    return params.lambda1 * eu + params.lambda2 * ed


def energy_u(model, scene, z, params) -> float:
    """The appearance part lambda1 sum_i U(z_i) alone (the distance used by the
    paper's nearest-prototype classifier, Section 4)."""
    return params.lambda1 * sum(unary_of(model, scene, i, z[i], params) for i in range(len(z)))


def candidate_lists(model, scene, params, tau: int):
    return [candidates(model.t, scene.t, tau, i, params.window, params.k_max, params.k_density)
            for i in range(model.n)]


def brute_force(model, scene, params, tau: int, lists=None):
    """Minimum of E over every assignment drawn from the candidate lists, by
    enumeration: the definition of the exact matching (Section 2.2).  `lists`
    replaces the windowed lists of offset tau when given.

    With dummy assignments enabled every point may also take DUMMY.

    Returns (E*, list of all optimal assignments); E* = +inf and [] when no
    assignment is admissible.  Only for tiny inputs."""
    cands = candidate_lists(model, scene, params, tau) if lists is None else lists
    if w_dummy(params) is not None:
        cands = [list(c) + [DUMMY] for c in cands]
    if any(len(c) == 0 for c in cands):
        return INF, []
    best, arg = INF, []
    for z in itertools.product(*[list(c) for c in cands]):
        e = energy(model, scene, list(z), params)
        if e < best:
            best, arg = e, [list(z)]
        elif e == best and e < INF:
            arg.append(list(z))
    return best, arg


def brute_force_all(model, scene, params):
    """brute_force at every offset: (energies [n_tau], optimal sets)."""
    es, zs = [], []
    for tau in offsets(model.t, scene.n_frames):
        e, z = brute_force(model, scene, params, tau)
        es.append(e)
        zs.append(z)
    return np.array(es, dtype=np.float64), zs
