"""Plain run-to-tolerance driver -- TEST ORACLE.

Not in the paper (it performs a fixed number of sweeps).  Stopping rule used by
the solver: starting from ``box``, apply ``check_every`` sweeps at a time and
stop at the first check where ||r||_2 <= rel_tol * r0; r0 defaults to the
residual norm of ``box`` itself (the zero-interior start).
"""

from __future__ import annotations

import numpy as np


def solve_to_tol(box: np.ndarray, rel_tol: float, check_every: int,
                 max_sweeps: int, r0: float | None = None, nthreads: int = 0):
    """Return (box, sweeps_done, final_norm, r0)."""
    from . import residual_norm, sweeps_f64
    u = np.array(box, dtype=np.float64, copy=True)
    if r0 is None:
        r0 = residual_norm(u)
    done = 0
    rn = residual_norm(u)
    while rn > rel_tol * r0 and done < max_sweeps:
        m = min(check_every, max_sweeps - done)
        u = sweeps_f64(u, m, nthreads)
        done += m
        rn = residual_norm(u)
    return u, done, rn, r0
