"""Multigrid V-cycle with weighted-Jacobi smoothing -- TEST ORACLE.

Only ``tests/`` may use this module; the GPU library never imports it.

The paper calls the Jacobi update the central component of many multigrid
solvers (Sect. 1.1), and in its conclusions it names a pipelined stencil
code used as a multigrid smoother.  This module spells out that use for the
correction equation of the mixed-precision refinement (``refine.py``): the
m_in plain FP32 sweeps of its step 4 are replaced by one V-cycle.  The
V-cycle is textbook geometric multigrid.  Nothing below is taken from the
paper except the Jacobi update it smooths with.

Grids are vertex-centred: an n^3 interior with n = 2^k - 1 and a zero
Dirichlet boundary layer (the correction vanishes on the boundary); coarse
point I sits on fine point 2I, so the coarse interior is (n-1)/2.  All
arithmetic is float32 with round-to-nearest and no fused operations, in the
order written:

* weighted Jacobi sweep for 6e - sum6(e) = rhs (weight w = fl32(6/7), which
  equalises the damping of the highest and of the smoothest
  high-frequency modes of the 7-point operator):
      v = ((fold6(e) + rhs) * fl32(1/6)),   e' = e + w (v - e);
  fold6 is the left fold i-1, i+1, j-1, j+1, k-1, k+1 of Eq. (1);
* residual: r = (fold6(e) + rhs) - fl32(6 e);
* restriction (full weighting times the factor 4 of the coarse operator's
  doubled spacing): rhs_c[I] = sum over the 27 offsets d in the order
  dz, dy, dx = -1, 0, 1 of c(d) r[2I + d], with c(d) = 2^-(1 + |dx| + |dy| +
  |dz|) (exact power-of-two weights);
* prolongation and correction: e[i] += sum over the contributing coarse
  points (z, y, x ascending) of c e_c, trilinear weights 1 or 1/2 per axis;
* V-cycle: NU1 sweeps, residual, restriction, V-cycle on the coarse grid
  from zero, prolongation, NU2 sweeps; on a grid with n <= 3, NU_COARSE
  sweeps.
"""

from __future__ import annotations

import numpy as np

W = np.float32(6.0 / 7.0)
C6F = np.float32(1.0 / 6.0)
SIX = np.float32(6.0)
NU1 = 2
NU2 = 2
NU_COARSE = 32


def _fold6(e):
    """fold(e nbrs) on the interior of a float32 box, in Eq. (1) order."""
    s = e[1:-1, 1:-1, :-2] + e[1:-1, 1:-1, 2:]
    s = s + e[1:-1, :-2, 1:-1]
    s = s + e[1:-1, 2:, 1:-1]
    s = s + e[:-2, 1:-1, 1:-1]
    s = s + e[2:, 1:-1, 1:-1]
    return s


def wsweeps(e, rhs, nsweeps, w=W):
    """nsweeps weighted Jacobi sweeps (A/B) of 6e - sum6(e) = rhs; the
    boundary layer of e is kept.  Returns a new float32 box."""
    e = np.array(e, dtype=np.float32, copy=True)
    w = np.float32(w)
    for _ in range(nsweeps):
        c = e[1:-1, 1:-1, 1:-1]
        v = (_fold6(e) + rhs[1:-1, 1:-1, 1:-1]) * C6F
        new = c + w * (v - c)
        e = e.copy()
        e[1:-1, 1:-1, 1:-1] = new
    return e


def residual(e, rhs):
    """r = (fold6(e) + rhs) - 6e on the interior (boundary 0), float32."""
    r = np.zeros_like(e)
    r[1:-1, 1:-1, 1:-1] = (_fold6(e) + rhs[1:-1, 1:-1, 1:-1]) - SIX * e[1:-1, 1:-1, 1:-1]
    return r


def restrict(r):
    """Coarse right-hand side 4 x full weighting of the fine residual box."""
    n = r.shape[0] - 2
    nc = (n - 1) // 2
    out = np.zeros((nc + 2,) * 3, dtype=np.float32)
    idx = 2 * np.arange(1, nc + 1)
    acc = np.zeros((nc,) * 3, dtype=np.float32)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                c = np.float32(2.0 ** -(1 + abs(dx) + abs(dy) + abs(dz)))
                acc = acc + c * r[np.ix_(idx + dz, idx + dy, idx + dx)]
    out[1:-1, 1:-1, 1:-1] = acc
    return out


def _axis_terms(n):
    """Per fine index 1..n: list of (coarse index, weight)."""
    terms = []
    for i in range(1, n + 1):
        if i % 2 == 0:
            terms.append(((i // 2, 1.0),))
        else:
            terms.append((((i - 1) // 2, 0.5), ((i + 1) // 2, 0.5)))
    return terms


def prolong_add(e, ec):
    """e += trilinear prolongation of the coarse correction ec (float32)."""
    n = e.shape[0] - 2
    out = np.array(e, dtype=np.float32, copy=True)
    terms = _axis_terms(n)
    # group fine indices by parity; the terms of each parity class share a
    # shape, so each class is one vectorised fold
    for pz in (0, 1):
        for py in (0, 1):
            for px in (0, 1):
                iz = np.arange(1, n + 1)[(np.arange(1, n + 1) % 2) == pz]
                iy = np.arange(1, n + 1)[(np.arange(1, n + 1) % 2) == py]
                ix = np.arange(1, n + 1)[(np.arange(1, n + 1) % 2) == px]
                if not (len(iz) and len(iy) and len(ix)):
                    continue
                tz = [terms[i - 1] for i in iz]
                ty = [terms[i - 1] for i in iy]
                tx = [terms[i - 1] for i in ix]
                val = np.zeros((len(iz), len(iy), len(ix)), dtype=np.float32)
                for a in range(len(tz[0])):
                    cz = np.array([t[a][0] for t in tz])
                    wz = tz[0][a][1]
                    for b in range(len(ty[0])):
                        cy = np.array([t[b][0] for t in ty])
                        wy = ty[0][b][1]
                        for c in range(len(tx[0])):
                            cx = np.array([t[c][0] for t in tx])
                            wx = tx[0][c][1]
                            wgt = np.float32(wz * wy * wx)
                            val = val + wgt * ec[np.ix_(cz, cy, cx)]
                sel = np.ix_(iz, iy, ix)
                out[sel] = out[sel] + val
    return out


def vcycle(e, rhs):
    """One V-cycle for 6e - sum6(e) = rhs from e (float32 boxes)."""
    n = e.shape[0] - 2
    if n <= 3:
        return wsweeps(e, rhs, NU_COARSE)
    e = wsweeps(e, rhs, NU1)
    rc = restrict(residual(e, rhs))
    ec = vcycle(np.zeros_like(rc), rc)
    e = prolong_add(e, ec)
    return wsweeps(e, rhs, NU2)


def levels_ok(n: int) -> bool:
    """n = 2^k - 1 with k >= 1."""
    return n >= 1 and (n + 1) & n == 0


def mg_outer(box, nthreads: int = 0):
    """One outer step of the refinement with a V-cycle as the inner solve:
    FP64 residual, rhs = fl32(r 2^-s), e = V-cycle from zero, u += fl64(e) 2^s
    (the steps of ``refine.refine_outer_f32`` with step 4 replaced).
    Returns (new_box, s, max_abs_r)."""
    from . import residual_f64
    u = np.array(box, dtype=np.float64, copy=True)
    r = residual_f64(u, nthreads)
    mx = float(np.max(np.abs(r[1:-1, 1:-1, 1:-1])))
    if mx == 0.0:
        return u, 0, 0.0
    _, s = np.frexp(mx)
    s = int(s)
    rhs = np.ldexp(r, -s).astype(np.float32)
    e = vcycle(np.zeros(u.shape, dtype=np.float32), rhs)
    inner = u[1:-1, 1:-1, 1:-1]
    inner += np.ldexp(e[1:-1, 1:-1, 1:-1].astype(np.float64), s)
    return u, s, mx


def mg_refine(box, n_outer: int, nthreads: int = 0):
    """n_outer outer steps of ``mg_outer``; returns the new box."""
    u = np.array(box, dtype=np.float64, copy=True)
    for _ in range(n_outer):
        u, _s, mx = mg_outer(u, nthreads)
        if mx == 0.0:
            break
    return u
