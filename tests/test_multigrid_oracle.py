"""Pins of the multigrid oracle (oracle/multigrid.py) -- no GPU.

Each piece is checked against a fact that does not come from the oracle
itself: the smoothing factor 1 - w + w*lambda of a sine mode, exact
reproduction of constants by the restriction and of affine fields by the
prolongation, the textbook V-cycle contraction, the closed-form product
bump, and the closed-form harmonic solution for sine-mode faces within the
residual bound."""

import numpy as np
import pytest

import synth
from oracle import multigrid as mg
from tests import closed_form as cf


def test_weighted_sweep_decays_sine_mode_by_smoothing_factor():
    n = 15
    for p, q, r in ((1, 1, 1), (15, 15, 15), (8, 3, 12)):
        u = cf.sine_mode(n, n, n, p, q, r).astype(np.float32)
        lam = cf.sine_mode_eigenvalue(n, n, n, p, q, r)
        g = 1.0 - (6.0 / 7.0) + (6.0 / 7.0) * lam
        out = mg.wsweeps(u, np.zeros_like(u), 1)
        assert np.max(np.abs(out - g * u.astype(np.float64))) < 4e-7, (p, q, r)
    # the highest mode (lambda close to -1) is damped to about |1 - 2w| = 5/7,
    # where a plain Jacobi sweep (w = 1) hardly damps it: the smoother's point
    u = cf.sine_mode(n, n, n, n, n, n).astype(np.float32)
    lam = cf.sine_mode_eigenvalue(n, n, n, n, n, n)
    ratio = np.linalg.norm(mg.wsweeps(u, np.zeros_like(u), 1)) / np.linalg.norm(u)
    assert abs(ratio - abs(1 - 6 / 7 + 6 / 7 * lam)) < 1e-6 and ratio < 0.72
    plain = np.linalg.norm(mg.wsweeps(u, np.zeros_like(u), 1, w=1.0)) / np.linalg.norm(u)
    assert plain > 0.95


def test_restriction_reproduces_four_times_constants_and_affine_fields():
    n = 15
    i, j, k = cf.index_grids(n, n, n)
    for f in (lambda i, j, k: 3.0 + 0 * i + 0 * j + 0 * k,
              lambda i, j, k: 2 * i - 3 * j + k + 1):
        r = np.zeros((n + 2,) * 3, dtype=np.float32)
        r[1:-1, 1:-1, 1:-1] = np.broadcast_to(f(i, j, k), r.shape)[1:-1, 1:-1, 1:-1]
        rc = mg.restrict(r)
        nc = (n - 1) // 2
        ic, jc, kc = cf.index_grids(nc, nc, nc)
        want = 4 * np.broadcast_to(f(2 * ic, 2 * jc, 2 * kc), rc.shape)
        assert np.array_equal(rc[1:-1, 1:-1, 1:-1], want[1:-1, 1:-1, 1:-1].astype(np.float32))


def test_prolongation_reproduces_affine_fields():
    n = 15
    nc = (n - 1) // 2
    f = lambda i, j, k: 5 - 2 * i + 3 * j + 4 * k  # noqa: E731
    ic, jc, kc = cf.index_grids(nc, nc, nc)
    ec = np.broadcast_to(f(2 * ic, 2 * jc, 2 * kc), (nc + 2,) * 3).astype(np.float32)
    e = mg.prolong_add(np.zeros((n + 2,) * 3, dtype=np.float32), ec)
    i, j, k = cf.index_grids(n, n, n)
    want = np.broadcast_to(f(i, j, k), e.shape).astype(np.float32)
    assert np.array_equal(e[1:-1, 1:-1, 1:-1], want[1:-1, 1:-1, 1:-1])


@pytest.mark.parametrize("n", [15, 31, 63])
def test_vcycle_contracts_the_residual(n):
    rng = np.random.default_rng(n)
    rhs = np.zeros((n + 2,) * 3, dtype=np.float32)
    rhs[1:-1, 1:-1, 1:-1] = rng.standard_normal((n, n, n))
    e = np.zeros_like(rhs)
    prev = np.linalg.norm(mg.residual(e, rhs))
    factors = []
    for _ in range(4):
        e = mg.vcycle(e, rhs)
        cur = np.linalg.norm(mg.residual(e, rhs).astype(np.float64))
        factors.append(cur / prev)
        prev = cur
    assert max(factors) < 0.25, factors


def test_vcycles_converge_to_the_product_bump():
    n = 31
    e_star, rhs = cf.product_bump(n, n, n)
    rhs32 = rhs.astype(np.float32)
    e = np.zeros((n + 2,) * 3, dtype=np.float32)
    for _ in range(12):
        e = mg.vcycle(e, rhs32)
    rel = np.linalg.norm(e - e_star) / np.linalg.norm(e_star)
    assert rel < 1e-5, rel


def test_mg_refinement_meets_closed_form_solution():
    n = 31
    box = synth.sine_face_box(n, n, n, seed=7)
    modes = synth.sine_face_modes(7)
    ustar = cf.harmonic_from_sine_faces(n, n, n, modes)
    import oracle
    r0 = oracle.residual_norm(box)
    u = box
    for it in range(30):
        u, _s, _mx = mg.mg_outer(u)
        rn = oracle.residual_norm(u)
        if rn <= 1e-10 * r0:
            break
    assert it < 20, it
    err = np.linalg.norm((u - ustar)[1:-1, 1:-1, 1:-1])
    assert err <= cf.laplace_error_bound(n, n, n, rn) * 1.01 + 1e-12
    assert mg.levels_ok(n) and not mg.levels_ok(32)
