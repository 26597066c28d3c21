"""Pins of the CPU oracle to facts that do not come from the oracle itself.

Every check here is chosen so that a plausible slip in the oracle -- a dropped
neighbour, a wrong sign or index, a transposed axis, a missing A/B swap, a
wrong constant -- fails at least one of them:

* integer harmonic polynomials are exact fixed points of Eq. (1) (the fold sum
  is exactly 6v and fl(6v * fl(1/6)) == v, checked exhaustively below);
* sine modes decay by the closed-form factor (cos a + cos b + cos c)/3 per
  sweep (within rounding);
* with faces carrying sine modes the discrete Laplace problem has a closed
  form solution (sinh profiles); the run-to-tolerance driver must land within
  the residual error bound of it;
* max principle and exact monotonicity from a zero start;
* reflection symmetry in i is bitwise (it only swaps the first two addends);
* u = i^2 has residual exactly 2 at every interior cell;
* a second, pure-Python spelling agrees bit for bit on every small shape;
* the FP32 right-hand-side sweep has the exact fixed point f(i)g(j)h(k).
"""

import itertools
import math

import numpy as np
import pytest

import oracle
import synth
from tests import closed_form as cf


def bits(a):
    return a.view(np.uint64) if a.dtype == np.float64 else a.view(np.uint32)


def test_fl_one_sixth_undoes_exact_multiples():
    c6 = 1.0 / 6.0
    assert c6.hex() == "0x1.5555555555555p-3"
    v = np.arange(-200000, 200001, dtype=np.float64)
    assert np.array_equal((6.0 * v) * c6, v)
    c6f = np.float32(1.0) / np.float32(6.0)
    assert int(c6f.view(np.uint32)) == 0x3E2AAAAB
    vf = np.arange(-200000, 200001, dtype=np.float32)
    assert np.array_equal((np.float32(6.0) * vf) * c6f, vf)


@pytest.mark.parametrize("name", sorted(cf.HARMONIC))
@pytest.mark.parametrize("dims", [(7, 5, 3), (3, 9, 4), (1, 1, 1), (6, 1, 8)])
def test_harmonic_polynomials_are_exact_fixed_points(name, dims):
    nx, ny, nz = dims
    u = cf.harmonic_box(name, nx, ny, nz)
    out = oracle.sweeps_f64(u, 5)
    assert np.array_equal(bits(out), bits(u))
    r = oracle.residual_f64(u)
    assert np.all(r == 0.0)


@pytest.mark.parametrize("dims,mode", [((11, 7, 5), (1, 1, 1)),
                                        ((11, 7, 5), (3, 2, 4)),
                                        ((6, 13, 9), (2, 5, 1))])
def test_sine_mode_decays_by_closed_form_factor(dims, mode):
    nx, ny, nz = dims
    u0 = cf.sine_mode(nx, ny, nz, *mode)
    lam = cf.sine_mode_eigenvalue(nx, ny, nz, *mode)
    m = float(np.max(np.abs(u0)))
    for n in (1, 2, 7):
        un = oracle.sweeps_f64(u0, n)
        err = float(np.max(np.abs(un - lam ** n * u0)))
        assert err <= 8 * n * np.finfo(np.float64).eps * m, (n, err)
    # residual of an eigenmode: (6 lam - 6) u, norm via a library routine
    r = oracle.residual_f64(u0)
    assert np.allclose(r, 6.0 * (lam - 1.0) * u0, atol=32 * np.finfo(float).eps)
    assert math.isclose(oracle.residual_norm(u0),
                        abs(6.0 * (lam - 1.0)) * float(np.linalg.norm(u0)),
                        rel_tol=1e-12)


def test_missing_swap_or_in_place_update_would_be_caught():
    # The decay factor over two sweeps is lam^2 only with separate grids;
    # an in-place (Gauss-Seidel-like) update gives a different field.
    nx, ny, nz = 9, 8, 7
    u0 = cf.sine_mode(nx, ny, nz, 1, 1, 1)
    lam = cf.sine_mode_eigenvalue(nx, ny, nz, 1, 1, 1)
    gs = u0.copy()
    for k in range(1, nz + 1):
        for j in range(1, ny + 1):
            for i in range(1, nx + 1):
                gs[k, j, i] = (gs[k, j, i - 1] + gs[k, j, i + 1] + gs[k, j - 1, i]
                               + gs[k, j + 1, i] + gs[k - 1, j, i]
                               + gs[k + 1, j, i]) / 6.0
    assert np.max(np.abs(gs - lam * u0)) > 1e-3
    assert np.max(np.abs(oracle.sweeps_f64(u0, 1) - lam * u0)) < 1e-14


def test_residual_of_quadratic_is_exactly_two():
    nx, ny, nz = 6, 5, 4
    i, j, k = cf.index_grids(nx, ny, nz)
    u = np.array(np.broadcast_to(i * i + 0 * j + 0 * k,
                                             (nz + 2, ny + 2, nx + 2)))
    r = oracle.residual_f64(u)
    assert np.all(r[1:-1, 1:-1, 1:-1] == 2.0)
    assert np.all(r[0] == 0) and np.all(r[:, :, 0] == 0)
    assert math.isclose(oracle.residual_norm(u), 2.0 * math.sqrt(nx * ny * nz),
                        rel_tol=1e-15)


def test_residual_norm_matches_library_norm():
    box = synth.uniform_box(17, 9, 12, seed=5)
    box = oracle.sweeps_f64(box, 3)
    r = oracle.residual_f64(box)
    assert math.isclose(oracle.residual_norm(box),
                        float(np.linalg.norm(r[1:-1, 1:-1, 1:-1])), rel_tol=1e-13)


@pytest.mark.parametrize("seed", [11, 12])
def test_converged_field_matches_closed_form_sine_faces(seed):
    nx, ny, nz = 10, 9, 8
    modes = synth.sine_face_modes(seed, modes_per_face=3, pmax=3)
    box = synth.sine_face_box(nx, ny, nz, seed, modes_per_face=3, pmax=3)
    ustar = cf.harmonic_from_sine_faces(nx, ny, nz, modes)
    # the closed form is a discrete solution: its residual vanishes
    ustar_box = box.copy()
    ustar_box[1:-1, 1:-1, 1:-1] = ustar[1:-1, 1:-1, 1:-1]
    assert oracle.residual_norm(ustar_box) < 1e-12 * np.abs(box).max() * 100
    u, done, rn, r0 = oracle.solve_to_tol(box, 1e-10, check_every=50,
                                          max_sweeps=20000)
    assert rn <= 1e-10 * r0 and done > 0
    err = float(np.linalg.norm((u - ustar_box)[1:-1, 1:-1, 1:-1]))
    bound = cf.laplace_error_bound(nx, ny, nz, rn)
    assert err <= bound * 1.01 + 1e-12, (err, bound)


def test_max_principle_and_exact_monotonicity():
    box = synth.uniform_box(9, 7, 8, seed=3)
    m = float(box.max())
    prev = box
    for n in range(1, 25):
        cur = oracle.sweeps_f64(prev, 1)
        assert np.all(cur >= prev)
        assert float(cur.max()) <= m * (1 + 4 * n * 2.0 ** -53)
        prev = cur


def test_composition_is_bitwise():
    box = synth.uniform_box(8, 6, 7, seed=4)
    a = oracle.sweeps_f64(oracle.sweeps_f64(box, 3), 4)
    b = oracle.sweeps_f64(box, 7)
    assert np.array_equal(bits(a), bits(b))
    c = oracle.sweeps_f64(box, 0)
    assert np.array_equal(bits(c), bits(box))


def test_reflection_in_i_is_bitwise():
    box = synth.uniform_box(9, 6, 5, seed=6)
    out = oracle.sweeps_f64(box, 6)
    outr = oracle.sweeps_f64(np.ascontiguousarray(box[:, :, ::-1]), 6)
    assert np.array_equal(bits(np.ascontiguousarray(out[:, :, ::-1])), bits(outr))


def test_thread_count_does_not_change_bits():
    box = synth.uniform_box(13, 11, 17, seed=8)
    a = oracle.sweeps_f64(box, 5, nthreads=1)
    b = oracle.sweeps_f64(box, 5, nthreads=oracle.max_threads())
    assert np.array_equal(bits(a), bits(b))


SMALL = [1, 2, 3, 5, 8]


@pytest.mark.parametrize("dims", list(itertools.product(SMALL, SMALL, SMALL)))
def test_c_oracle_equals_pure_python_loops(dims):
    nx, ny, nz = dims
    box = synth.uniform_box(nx, ny, nz, seed=nx * 100 + ny * 10 + nz)
    box[1:-1, 1:-1, 1:-1] = np.random.default_rng(1).random((nz, ny, nx))
    a = oracle.sweeps_f64(box, 2)
    b = oracle.brute.sweeps_f64(box, 2)
    assert np.array_equal(bits(a), bits(b))


def test_single_cell_problem():
    box = synth.uniform_box(1, 1, 1, seed=9)
    box[1, 1, 1] = 0.25
    out = oracle.sweeps_f64(box, 1)
    s = box[1, 1, 0]
    for v in (box[1, 1, 2], box[1, 0, 1], box[1, 2, 1], box[0, 1, 1], box[2, 1, 1]):
        s = s + v
    assert out[1, 1, 1] == s * (1.0 / 6.0)
    # boundary untouched
    mask = np.ones(box.shape, bool)
    mask[1, 1, 1] = False
    assert np.array_equal(out[mask], box[mask])


# ---------------------------------------------------------------- FP32 ------

def test_f32_integer_fixed_point_with_rhs():
    nx, ny, nz = 7, 6, 5
    e, rhs = cf.product_bump(nx, ny, nz)
    e32 = e.astype(np.float32)
    rhs32 = rhs.astype(np.float32)
    assert np.array_equal(e32.astype(np.float64), e)  # exact in FP32
    out = oracle.sweeps_f32(e32, 4, rhs32)
    assert np.array_equal(bits(out), bits(e32))


@pytest.mark.parametrize("name", ["affine", "ijk", "mixed"])
def test_f32_harmonic_fixed_point(name):
    u = cf.harmonic_box(name, 6, 5, 7).astype(np.float32)
    out = oracle.sweeps_f32(u, 3)
    assert np.array_equal(bits(out), bits(u))


@pytest.mark.parametrize("dims", [(1, 1, 1), (3, 2, 5), (8, 3, 2), (5, 5, 5)])
def test_f32_c_oracle_equals_python_loops(dims):
    nx, ny, nz = dims
    rng = np.random.default_rng(7)
    box = rng.random((nz + 2, ny + 2, nx + 2)).astype(np.float32)
    rhs = rng.standard_normal((nz + 2, ny + 2, nx + 2)).astype(np.float32)
    a = oracle.sweeps_f32(box, 2, rhs)
    b = oracle.brute.sweep_f32(oracle.brute.sweep_f32(box, rhs), rhs)
    assert np.array_equal(bits(a), bits(b))


def test_f32_sine_mode_decay():
    nx, ny, nz = 11, 7, 5
    u0 = cf.sine_mode(nx, ny, nz, 2, 1, 3)
    lam = cf.sine_mode_eigenvalue(nx, ny, nz, 2, 1, 3)
    out = oracle.sweeps_f32(u0.astype(np.float32), 3)
    assert np.max(np.abs(out - lam ** 3 * u0)) < 3e-6


# ---------------------------------------------------- FP32 refinement -------

def test_refine_leaves_exact_solution_alone():
    u = cf.harmonic_box("mixed", 6, 5, 4)
    out, s, mx = oracle.refine_outer_f32(u, 10)
    assert mx == 0.0 and np.array_equal(bits(out), bits(u))


def test_refine_converges_to_affine_solution():
    nx, ny, nz = 9, 8, 7
    sol = cf.harmonic_box("affine", nx, ny, nz) / 17.0
    box = sol.copy()
    box[1:-1, 1:-1, 1:-1] = 0.0
    r0 = oracle.residual_norm(box)
    u = oracle.refine_f32(box, m_in=60, n_outer=40)
    assert oracle.residual_norm(u) <= 1e-8 * r0
    assert np.max(np.abs(u - sol)) <= 1e-8 * np.abs(sol).max()


def test_refine_step_reduces_residual_like_fp32_precision():
    # With many inner sweeps the correction is solved to FP32 accuracy, so the
    # FP64 residual drops by roughly FP32 precision in one outer step.
    nx, ny, nz = 6, 6, 6
    box = synth.uniform_box(nx, ny, nz, seed=21)
    before = oracle.residual_norm(box)
    u, s, mx = oracle.refine_outer_f32(box, 600)
    after = oracle.residual_norm(u)
    assert after <= 1e-5 * before, (before, after)
    assert 0.5 <= mx * 2.0 ** -s < 1.0


def test_refine_meets_closed_form_solution():
    nx, ny, nz = 10, 9, 8
    seed = 31
    modes = synth.sine_face_modes(seed, modes_per_face=3, pmax=3)
    box = synth.sine_face_box(nx, ny, nz, seed, modes_per_face=3, pmax=3)
    ustar = cf.harmonic_from_sine_faces(nx, ny, nz, modes)
    r0 = oracle.residual_norm(box)
    u = oracle.refine_f32(box, m_in=100, n_outer=60)
    rn = oracle.residual_norm(u)
    assert rn <= 1e-8 * r0
    err = float(np.linalg.norm((u - ustar)[1:-1, 1:-1, 1:-1]))
    assert err <= cf.laplace_error_bound(nx, ny, nz, rn) * 1.01 + 1e-12
