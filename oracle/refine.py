"""FP32 sweeps with FP64 residual and FP64 defect correction -- TEST ORACLE.

Mixed-precision iterative refinement of the discrete Laplace problem solved by
the Jacobi method of the paper (Sect. 1.1, Eq. (1)); the refinement itself is
not in the paper.  One outer step, in this order:

1. r = fold(u nbrs) - fl(6u)                    (FP64, interior cells)
2. s = exponent of max|r| as returned by frexp, so |r| * 2^-s < 1
   (if max|r| == 0 the field is an exact fixed point and nothing is done)
3. rhs = fl32(r * 2^-s)                          (exact scaling, RNE to FP32)
4. e = 0 everywhere (zero Dirichlet boundary), then m_in FP32 sweeps
       e <- (fold(e nbrs) + rhs) * fl32(1/6)
   -- the Jacobi iteration for 6e - sum6(e) = rhs
5. u <- u + fl64(e) * 2^s                        (FP64, interior cells)

Since 6(u+E) - sum6(u+E) = 0 with E = e * 2^s exactly when 6E - sum6(E) = r,
step 4 approximates the correction that solves the FP64 equation.
"""

from __future__ import annotations

import numpy as np


def refine_outer_f32(box: np.ndarray, m_in: int, nthreads: int = 0):
    """One outer refinement step; returns (new_box, s, max_abs_r)."""
    from . import residual_f64, sweeps_f32
    u = np.array(box, dtype=np.float64, copy=True)
    r = residual_f64(u, nthreads)
    mx = float(np.max(np.abs(r[1:-1, 1:-1, 1:-1])))
    if mx == 0.0:
        return u, 0, 0.0
    _, s = np.frexp(mx)
    s = int(s)
    rhs = np.ldexp(r, -s).astype(np.float32)
    e = np.zeros(u.shape, dtype=np.float32)
    e = sweeps_f32(e, m_in, rhs, nthreads)
    inner = u[1:-1, 1:-1, 1:-1]
    inner += np.ldexp(e[1:-1, 1:-1, 1:-1].astype(np.float64), s)
    return u, s, mx


def refine_f32(box: np.ndarray, m_in: int, n_outer: int, nthreads: int = 0):
    """``n_outer`` outer steps of ``refine_outer_f32``; returns the new box."""
    u = np.array(box, dtype=np.float64, copy=True)
    for _ in range(n_outer):
        u, _s, mx = refine_outer_f32(u, m_in, nthreads)
        if mx == 0.0:
            break
    return u
