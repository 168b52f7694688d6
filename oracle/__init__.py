"""CPU FP64 oracle of the exact space-time hypergraph matching.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP path and must never be used as a fallback for it.

Two independent restatements of the paper (arXiv 1505.00581):
  * `oracle.energy`  — Python: the energy terms (Eq. 1-8) and brute-force
    minimisation over every assignment (tiny inputs only);
  * `stm_oracle.c`   — C, built here with gcc: the same terms plus the
    literal backward recursion of Section 2.2 (Eq. 10-13), parallel over
    offsets with OpenMP; wrapped by `match`, `energies`, `candidate_list`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

from . import energy  # noqa: F401  (re-exported)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stm_oracle.c")
_LIB = os.path.join(_HERE, "libstm_oracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile stm_oracle.c with gcc (-O2 -fopenmp) into libstm_oracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = ctypes.CDLL(build())
            P = ctypes.c_void_p
            i32, f64 = ctypes.c_int32, ctypes.c_double
            lib.oracle_match.restype = ctypes.c_int
            lib.oracle_match.argtypes = [i32, P, P, P, i32, i32, P, P, P, i32, f64, f64, f64,
                                         i32, i32, i32, i32, i32, i32, f64, P, i32, P, P, P, P, i32]
            lib.oracle_match_lists.restype = ctypes.c_int
            lib.oracle_match_lists.argtypes = [i32, P, P, P, i32, i32, P, P, P, i32, f64, f64, f64,
                                               i32, i32, i32, i32, f64, P, P, i32, P, P, P, i32]
            lib.oracle_energies.restype = None
            lib.oracle_energies.argtypes = [i32, P, P, P, i32, i32, P, P, P, i32, f64, f64, f64,
                                            i32, i32, i32, f64, P, i32, P, P]
            lib.oracle_candidate_list.restype = i32
            lib.oracle_candidate_list.argtypes = [i32, P, i32, P, i32, i32, i32, i32, i32, P]
            lib.oracle_num_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def offsets(model, scene) -> range:
    return energy.offsets(model.t, scene.n_frames)


def _dummy(params):
    """(enabled, W^d) of the dummy assignment (Eq. 2); params.w_dummy None = off."""
    w = getattr(params, "w_dummy", None)
    return (0, 0.0) if w is None else (1, float(w))


def _readings(params) -> int:
    """Bits of the alternative readings: 1 the span reading of temporal
    closeness (params.closeness_span), 2 unsigned triangle angles
    (params.angle_unsigned), 4 causality by scene node order
    (params.causal_node)."""
    span = int(bool(getattr(params, "closeness_span", False)))
    if span and getattr(params, "w_dummy", None) is not None:
        raise ValueError("the span reading of closeness is not defined with dummies")
    node = bool(getattr(params, "causal_node", False))
    if node and span:
        raise ValueError("node-order causality is taken with the pairwise reading of closeness only")
    return span | (2 if getattr(params, "angle_unsigned", False) else 0) | (4 if node else 0)


def match(model, scene, params, taus=None, n_threads: int = 0):
    """Exact optimum at each offset in `taus` (default: every offset).

    Returns dict(energy [n] f64, energy_u [n] f64, assign [n,M] int32 (-1 rows
    if infeasible, -2 for a dummy), counts dict(dense_cells, feasible_cells,
    dense_relax, feasible_relax) over scene candidates, taus)."""
    lib = _load()
    if taus is None:
        taus = np.arange(len(offsets(model, scene)), dtype=np.int32)
    taus = _i32(taus)
    n, M = taus.shape[0], model.n
    e = np.empty(n, np.float64)
    eu = np.empty(n, np.float64)
    z = np.empty((n, M), np.int32)
    c = np.zeros(4, np.int64)
    keep = [_f32(model.xy), _i32(model.t), _f32(model.desc), _f32(scene.xy), _i32(scene.t),
            _f32(scene.desc)]
    rc = lib.oracle_match(M, _ptr(keep[0]), _ptr(keep[1]), _ptr(keep[2]), scene.n, scene.n_frames,
                          _ptr(keep[3]), _ptr(keep[4]), _ptr(keep[5]), model.dim,
                          params.lambda1, params.lambda2, params.lambda3, params.T, _readings(params),
                          params.window, params.k_max, int(params.k_density), *_dummy(params),
                          _ptr(taus), n,
                          _ptr(e), _ptr(eu), _ptr(z), _ptr(c), n_threads)
    if rc != 0:
        raise RuntimeError(f"oracle_match failed ({rc}): recursion and literal energy disagree")
    return dict(energy=e, energy_u=eu, assign=z, taus=taus,
                counts=dict(dense_cells=int(c[0]), feasible_cells=int(c[1]),
                            dense_relax=int(c[2]), feasible_relax=int(c[3])))


def match_lists(model, scene, params, lists, counts, n_threads: int = 0):
    """The exact recursion on given candidate lists: lists [n, M, K] int32
    (ascending node ids), counts [n, M].  Returns dict(energy, energy_u,
    assign) like match."""
    lib = _load()
    lists = _i32(lists)
    counts = _i32(counts)
    n, M, K = lists.shape
    assert counts.shape == (n, M) and M == model.n and (counts <= K).all() and (counts >= 0).all()
    e = np.empty(n, np.float64)
    eu = np.empty(n, np.float64)
    z = np.empty((n, M), np.int32)
    keep = [_f32(model.xy), _i32(model.t), _f32(model.desc), _f32(scene.xy), _i32(scene.t),
            _f32(scene.desc)]
    rc = lib.oracle_match_lists(M, _ptr(keep[0]), _ptr(keep[1]), _ptr(keep[2]), scene.n,
                                scene.n_frames, _ptr(keep[3]), _ptr(keep[4]), _ptr(keep[5]),
                                model.dim, params.lambda1, params.lambda2, params.lambda3, params.T,
                                _readings(params), K, *_dummy(params), _ptr(lists), _ptr(counts), n, _ptr(e), _ptr(eu),
                                _ptr(z),
                                n_threads)
    if rc != 0:
        raise RuntimeError(f"oracle_match_lists failed ({rc}): recursion and literal energy disagree")
    return dict(energy=e, energy_u=eu, assign=z)


def match_trellis(model, scene, params, node_begin: int = 0, node_end=None, n_threads: int = 0):
    """The paper's own problem (Section 2.2): one trellis in which every model
    point may take any scene node of the block [node_begin, node_end), under
    causality and closeness (Eq. 7, 8; the loop bounds of Section 3.4 are a
    consequence of these, not extra constraints).  The literal recursion on
    the lists that hold the whole block for every point.  Returns dict(energy,
    energy_u, assign) with one row."""
    e = scene.n if node_end is None else int(node_end)
    b = int(node_begin)
    assert 0 <= b < e <= scene.n
    M = model.n
    lists = np.broadcast_to(np.arange(b, e, dtype=np.int32), (1, M, e - b)).copy()
    counts = np.full((1, M), e - b, np.int32)
    return match_lists(model, scene, params, lists, counts, n_threads)


def energies(model, scene, params, assign):
    """Literal FP64 energy (Eq. 1) of each assignment row; returns (E, E_U)."""
    lib = _load()
    z = _i32(np.atleast_2d(assign))
    n = z.shape[0]
    e = np.empty(n, np.float64)
    eu = np.empty(n, np.float64)
    keep = [_f32(model.xy), _i32(model.t), _f32(model.desc), _f32(scene.xy), _i32(scene.t),
            _f32(scene.desc)]
    lib.oracle_energies(model.n, _ptr(keep[0]), _ptr(keep[1]), _ptr(keep[2]), scene.n,
                        scene.n_frames, _ptr(keep[3]), _ptr(keep[4]), _ptr(keep[5]), model.dim,
                        params.lambda1, params.lambda2, params.lambda3, params.T, _readings(params),
                        *_dummy(params), _ptr(z), n,
                        _ptr(e), _ptr(eu))
    return e, eu


def candidate_list(model, scene, params, tau: int, i: int) -> np.ndarray:
    lib = _load()
    out = np.empty(max(params.k_max, 1), np.int32)
    mt, st = _i32(model.t), _i32(scene.t)
    n = lib.oracle_candidate_list(model.n, _ptr(mt), scene.n, _ptr(st), params.window,
                                  params.k_max, int(params.k_density), tau, i, _ptr(out))
    return out[:n].copy()


def num_threads() -> int:
    return int(_load().oracle_num_threads())
