"""Fits the polynomial used by the kernels' atan2: atan(t) ~ t * P(t^2) on
[0, 1], P of degree 7, minimising the maximum absolute error by the Remez
exchange algorithm, and prints the float32 coefficients as C literals.

    python paper_1505_00581_amd/csrc/gen_atan_poly.py
"""
import math

import numpy as np

DEG = 7


def remez(deg: int, iters: int = 60):
    n = deg + 2
    ref = np.sort(0.5 - 0.5 * np.cos(np.linspace(0, np.pi, n)))
    ref[0] = 1e-6
    grid = np.linspace(1e-6, 1, 200001)
    err = None
    c = None
    for _ in range(iters):
        A = np.zeros((n, n))
        b = np.zeros(n)
        for r, t in enumerate(ref):
            A[r, :deg + 1] = t * (t * t) ** np.arange(deg + 1)
            A[r, deg + 1] = (-1) ** r
            b[r] = math.atan(t)
        sol = np.linalg.solve(A, b)
        c = sol[:deg + 1]
        err = grid * np.polyval(c[::-1], grid * grid) - np.arctan(grid)
        sgn = np.sign(err)
        ext, start = [], 0
        for i in range(1, len(grid)):
            if sgn[i] != sgn[start]:
                ext.append(start + int(np.argmax(np.abs(err[start:i]))))
                start = i
        ext.append(start + int(np.argmax(np.abs(err[start:]))))
        if len(ext) < n:
            break
        ext = np.array(ext)
        best = max((np.min(np.abs(err[ext[s:s + n]])), s) for s in range(len(ext) - n + 1))
        ref = grid[ext[best[1]:best[1] + n]]
    return c, float(np.max(np.abs(err)))


if __name__ == "__main__":
    c, e = remez(DEG)
    print(f"// minimax |error| {e:.3g} before float32 rounding")
    for k, v in enumerate(np.float32(c)):
        print(f"constexpr float kAtanC{k} = {float(v)!r}f;")
