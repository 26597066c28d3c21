"""Pins of the 27-point Jacobi oracle (oracle.sweeps27_f64) -- no GPU.

The update is the Jacobi step of the 27-point Laplacian with face, edge and
corner weights 14, 3 and 1 over 128 (one of the other stencils the k-streaming
pipeline carries; not in the paper).  Pinned against: per-cell Python loops
(bitwise), exact rational arithmetic for one cell, fields the operator leaves
exactly unchanged, the closed-form decay of sine modes and the maximum
principle."""

import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute


def _random_box(nx, ny, nz, seed):
    # the whole boundary layer, edges and corners included, is data
    return np.random.default_rng(seed).random((nz + 2, ny + 2, nx + 2))


@pytest.mark.parametrize("dims", list(itertools.product((1, 2, 3, 5), repeat=3)))
def test_c_oracle_equals_python_loops(dims):
    box = _random_box(*dims, seed=sum(dims))
    got = oracle.sweeps27_f64(box, 3)
    want = brute.sweeps27_f64(box, 3)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


def test_single_cell_matches_exact_weights():
    """One interior cell: the result is within 2 ulp of (14 sum(faces) +
    3 sum(edges) + sum(corners)) / 128 in exact arithmetic, and moving one
    neighbour moves the result by exactly its weight."""
    rng = np.random.default_rng(7)
    for trial in range(50):
        box = np.round(rng.random((3, 3, 3)) * 2 ** 20) / 2 ** 20
        got = oracle.sweeps27_f64(box, 1)[1, 1, 1]
        exact = Fraction(0)
        for dk, dj, di in itertools.product((-1, 0, 1), repeat=3):
            n = abs(dk) + abs(dj) + abs(di)
            if n == 0:
                continue
            w = {1: Fraction(14, 128), 2: Fraction(3, 128), 3: Fraction(1, 128)}[n]
            exact += w * Fraction(float(box[1 + dk, 1 + dj, 1 + di]))
        assert abs(Fraction(got) - exact) <= 2 * Fraction(np.spacing(got))
    for (dk, dj, di), w in (((1, 0, 0), 14), ((0, -1, 1), 3), ((-1, 1, 1), 1)):
        box = np.zeros((3, 3, 3))
        box[1 + dk, 1 + dj, 1 + di] = 128.0
        assert oracle.sweeps27_f64(box, 1)[1, 1, 1] == w


@pytest.mark.parametrize("name", ["affine", "i2-j2", "ij", "j2-k2"])
def test_fixed_points_are_exact(name):
    """Affine fields and the quadratic harmonics are reproduced bit for bit:
    with integer values every sum and every product by the dyadic weights is
    exact, and the operator is exact on quadratics."""
    nx, ny, nz = 9, 7, 6
    k, j, i = np.meshgrid(np.arange(nz + 2), np.arange(ny + 2), np.arange(nx + 2),
                          indexing="ij")
    f = {"affine": 3 + 2 * i - 5 * j + 7 * k, "i2-j2": i * i - j * j, "ij": i * j,
         "j2-k2": j * j - k * k}[name].astype(np.float64)
    got = oracle.sweeps27_f64(f, 5)
    assert np.array_equal(got, f)


def test_sine_mode_decays_by_closed_form_factor():
    """u = sin(pi p i/(n+1)) sin(pi q j/(n+1)) sin(pi r k/(n+1)) with a zero
    boundary is an eigenvector: one sweep multiplies it by
    (28 (cx+cy+cz) + 12 (cx cy + cy cz + cz cx) + 8 cx cy cz) / 128."""
    nx, ny, nz = 11, 9, 7
    for p, q, r in ((1, 1, 1), (2, 3, 1), (5, 2, 6)):
        ax = [np.sin(np.pi * p * np.arange(nx + 2) / (nx + 1)),
              np.sin(np.pi * q * np.arange(ny + 2) / (ny + 1)),
              np.sin(np.pi * r * np.arange(nz + 2) / (nz + 1))]
        u = ax[2][:, None, None] * ax[1][None, :, None] * ax[0][None, None, :]
        u[0], u[-1], u[:, 0], u[:, -1], u[:, :, 0], u[:, :, -1] = 0, 0, 0, 0, 0, 0
        cx, cy, cz = (np.cos(np.pi * p / (nx + 1)), np.cos(np.pi * q / (ny + 1)),
                      np.cos(np.pi * r / (nz + 1)))
        lam = (28 * (cx + cy + cz) + 12 * (cx * cy + cy * cz + cz * cx) + 8 * cx * cy * cz) / 128
        got = oracle.sweeps27_f64(u, 4)
        assert np.max(np.abs(got - lam ** 4 * u)) < 1e-14


def test_maximum_principle():
    box = _random_box(12, 10, 9, seed=3)
    box[1:-1, 1:-1, 1:-1] = 0.0
    lo, hi = box.min(), box.max()
    out = oracle.sweeps27_f64(box, 20)
    assert out.min() >= lo and out.max() <= hi
