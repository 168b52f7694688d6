"""The scene directions of the HIP recursion use a polynomial atan2
(paper_1505_00581_amd/csrc/dp_math.h, neg_atan2).  This CPU test reads its
coefficients from the source, evaluates it with float32 roundings (one
rounding per fused multiply-add) and checks the error bound the source
states against numpy's FP64 arctan2, over the whole plane and near the axes
and diagonals."""
import math
import os
import re

import numpy as np

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_1505_00581_amd", "csrc", "dp_math.h")
BOUND = 3.5e-7


def _coeffs():
    src = open(SRC).read()
    found = dict(re.findall(r"kAtanC(\d) = ([-0-9.e]+)f;", src))
    return np.array([float(found[str(k)]) for k in range(len(found))], np.float32)


def neg_atan2_f32(y, x):
    c = _coeffs()
    f32 = np.float32
    ax, ay = np.abs(x).astype(f32), np.abs(y).astype(f32)
    t = (np.minimum(ax, ay) * (f32(1) / np.maximum(ax, ay)).astype(f32)).astype(f32)
    s = (t * t).astype(f32)
    p = np.full_like(s, c[-1])
    for k in range(len(c) - 2, -1, -1):
        p = (p.astype(np.float64) * s + np.float64(c[k])).astype(f32)
    a = (t * p).astype(f32)
    a = np.where(ay > ax, (f32(math.pi / 2) - a).astype(f32), a)
    a = np.where(x < 0, (f32(math.pi) - a).astype(f32), a)
    return np.where(y < 0, a, -a)


def _err(y, x):
    got = neg_atan2_f32(y, x).astype(np.float64)
    ref = -np.arctan2(y.astype(np.float64), x.astype(np.float64))
    d = np.abs(got - ref)
    return np.minimum(d, 2 * np.pi - d)


def test_polynomial_bound_uniform_plane():
    rng = np.random.default_rng(0)
    y = rng.uniform(-320, 320, 1_000_000).astype(np.float32)
    x = rng.uniform(-320, 320, 1_000_000).astype(np.float32)
    assert _err(y, x).max() <= BOUND


def test_polynomial_axes_and_diagonals():
    v = np.float32([1e-30, 1e-6, 0.5, 1.0, 3.0, 250.0])
    ys, xs = [], []
    for a in v:
        for b in (np.float32(0), a, -a, a * np.float32(1.0000001), a * np.float32(0.9999999)):
            for sx in (1, -1):
                for sy in (1, -1):
                    ys.append(sy * a)
                    xs.append(sx * b)
                    ys.append(sy * b)
                    xs.append(sx * a)
    y, x = np.array(ys, np.float32), np.array(xs, np.float32)
    keep = (x != 0) | (y != 0)
    assert _err(y[keep], x[keep]).max() <= BOUND


def test_generator_reproduces_coefficients():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "gen_atan_poly", os.path.join(os.path.dirname(SRC), "gen_atan_poly.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    c, e = mod.remez(mod.DEG)
    assert e < 5e-8
    np.testing.assert_array_equal(np.float32(c), _coeffs())
