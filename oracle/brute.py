"""Pure-Python per-cell loops for tiny grids -- TEST ORACLE.

A second, independent spelling of Eq. (1) of the paper (Sect. 1.1) with Python
floats (IEEE binary64, round to nearest, no fused operations) and numpy
float32 scalars for the single-precision sweep.  Used to cross-check the C
oracle on every shape up to 8^3; far too slow for anything larger.
"""

from __future__ import annotations

import numpy as np

C6 = 1.0 / 6.0
C6F = np.float32(1.0) / np.float32(6.0)


def sweep_f64(box):
    nz2, ny2, nx2 = box.shape
    a = [[[float(box[k, j, i]) for i in range(nx2)] for j in range(ny2)]
         for k in range(nz2)]
    out = np.array(box, dtype=np.float64, copy=True)
    for k in range(1, nz2 - 1):
        for j in range(1, ny2 - 1):
            for i in range(1, nx2 - 1):
                s = a[k][j][i - 1]
                s = s + a[k][j][i + 1]
                s = s + a[k][j - 1][i]
                s = s + a[k][j + 1][i]
                s = s + a[k - 1][j][i]
                s = s + a[k + 1][j][i]
                out[k, j, i] = s * C6
    return out


def sweeps_f64(box, n):
    out = np.array(box, dtype=np.float64, copy=True)
    for _ in range(n):
        out = sweep_f64(out)
    return out


def sweep_f32(box, rhs=None):
    nz2, ny2, nx2 = box.shape
    out = np.array(box, dtype=np.float32, copy=True)
    for k in range(1, nz2 - 1):
        for j in range(1, ny2 - 1):
            for i in range(1, nx2 - 1):
                s = np.float32(box[k, j, i - 1])
                s = np.float32(s + box[k, j, i + 1])
                s = np.float32(s + box[k, j - 1, i])
                s = np.float32(s + box[k, j + 1, i])
                s = np.float32(s + box[k - 1, j, i])
                s = np.float32(s + box[k + 1, j, i])
                if rhs is not None:
                    s = np.float32(s + rhs[k, j, i])
                out[k, j, i] = np.float32(s * C6F)
    return out


def residual(box):
    nz2, ny2, nx2 = box.shape
    r = np.zeros_like(box, dtype=np.float64)
    for k in range(1, nz2 - 1):
        for j in range(1, ny2 - 1):
            for i in range(1, nx2 - 1):
                s = float(box[k, j, i - 1])
                s = s + float(box[k, j, i + 1])
                s = s + float(box[k, j - 1, i])
                s = s + float(box[k, j + 1, i])
                s = s + float(box[k - 1, j, i])
                s = s + float(box[k + 1, j, i])
                r[k, j, i] = s - 6.0 * float(box[k, j, i])
    return r


# 27-point Jacobi update (the definition and fold order of
# jacobi_oracle.c's sweep27_f64), spelled per cell from offset lists.
_W27 = (7.0 / 64.0, 3.0 / 128.0, 1.0 / 128.0)
_CROSS = ((-1, 0), (1, 0), (0, -1), (0, 1))
_DIAG = ((-1, -1), (1, -1), (-1, 1), (1, 1))


def sweep27_f64(box):
    nz2, ny2, nx2 = box.shape
    a = [[[float(box[k, j, i]) for i in range(nx2)] for j in range(ny2)]
         for k in range(nz2)]
    out = np.array(box, dtype=np.float64, copy=True)

    def fold(p, j, i, offs):
        s = a[p][j + offs[0][1]][i + offs[0][0]]
        for di, dj in offs[1:]:
            s = s + a[p][j + dj][i + di]
        return s

    for k in range(1, nz2 - 1):
        for j in range(1, ny2 - 1):
            for i in range(1, nx2 - 1):
                b = [fold(p, j, i, _CROSS) for p in (k - 1, k, k + 1)]
                c = [fold(p, j, i, _DIAG) for p in (k - 1, k, k + 1)]
                f = (b[1] + a[k - 1][j][i]) + a[k + 1][j][i]
                e = (c[1] + b[0]) + b[2]
                kk = c[0] + c[2]
                out[k, j, i] = (_W27[0] * f + _W27[1] * e) + _W27[2] * kk
    return out


def sweeps27_f64(box, n):
    out = np.array(box, dtype=np.float64, copy=True)
    for _ in range(n):
        out = sweep27_f64(out)
    return out
