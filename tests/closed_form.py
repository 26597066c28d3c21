"""Closed-form facts about the discrete Laplace problem used as oracle pins.

Written independently of ``oracle/`` and of the GPU library; nothing here runs
a Jacobi sweep.
"""

from __future__ import annotations

import math

import numpy as np


def index_grids(nx, ny, nz):
    k = np.arange(nz + 2, dtype=np.float64)[:, None, None]
    j = np.arange(ny + 2, dtype=np.float64)[None, :, None]
    i = np.arange(nx + 2, dtype=np.float64)[None, None, :]
    return i, j, k


# Integer polynomials whose discrete 7-point Laplacian vanishes identically.
HARMONIC = {
    "affine": lambda i, j, k: 3 + 2 * i - 5 * j + 7 * k,
    "ij": lambda i, j, k: i * j + 0 * k,
    "jk": lambda i, j, k: j * k + 0 * i,
    "ik": lambda i, j, k: i * k + 0 * j,
    "ijk": lambda i, j, k: i * j * k,
    "i2-j2": lambda i, j, k: i * i - j * j + 0 * k,
    "2i2-j2-k2": lambda i, j, k: 2 * i * i - j * j - k * k,
    "mixed": lambda i, j, k: 4 * i * j - 3 * j * k + i * i - k * k + 11,
}


def harmonic_box(name, nx, ny, nz):
    i, j, k = index_grids(nx, ny, nz)
    return np.ascontiguousarray(
        np.broadcast_to(HARMONIC[name](i, j, k), (nz + 2, ny + 2, nx + 2)),
        dtype=np.float64)


def sine_mode(nx, ny, nz, p, q, r):
    """Interior eigenvector of the zero-boundary Jacobi iteration."""
    i, j, k = index_grids(nx, ny, nz)
    u = (np.sin(math.pi * p * i / (nx + 1)) * np.sin(math.pi * q * j / (ny + 1))
         * np.sin(math.pi * r * k / (nz + 1)))
    u = np.array(np.broadcast_to(u, (nz + 2, ny + 2, nx + 2)))
    u[0, :, :] = 0
    u[-1, :, :] = 0
    u[:, 0, :] = 0
    u[:, -1, :] = 0
    u[:, :, 0] = 0
    u[:, :, -1] = 0
    return u


def sine_mode_eigenvalue(nx, ny, nz, p, q, r):
    """One Jacobi sweep multiplies the sine mode (p, q, r) by this factor."""
    return (math.cos(math.pi * p / (nx + 1)) + math.cos(math.pi * q / (ny + 1))
            + math.cos(math.pi * r / (nz + 1))) / 3.0


def slowest_factor(nx, ny, nz):
    return sine_mode_eigenvalue(nx, ny, nz, 1, 1, 1)


def _face_term(n_norm, pos, th_a, th_b, ga, gb, far):
    """sinh-profile of one face mode along its normal axis.

    cosh(beta) = 3 - cos(th_a) - cos(th_b) makes sin(th_a a) sin(th_b b) f(x)
    discretely harmonic when f(x+1) + f(x-1) = 2 cosh(beta) f(x).
    """
    beta = math.acosh(3.0 - math.cos(th_a) - math.cos(th_b))
    d = (n_norm + 1 - pos) if not far else pos
    return np.sinh(beta * d) / math.sinh(beta * (n_norm + 1))


def harmonic_from_sine_faces(nx, ny, nz, modes):
    """Exact solution of the discrete Laplace problem for sine-mode faces.

    ``modes`` is the list of six per-face lists of (p, q, amplitude) in face
    order i=0, i=nx+1, j=0, j=ny+1, k=0, k=nz+1, in-plane axes in (i, j, k)
    order (first axis carries p).  Superposition of one separable solution per
    face mode.
    """
    i, j, k = index_grids(nx, ny, nz)
    u = np.zeros((nz + 2, ny + 2, nx + 2), dtype=np.float64)
    specs = [
        # (normal axis grid, n_normal, axis-a grid, n_a, axis-b grid, n_b, far)
        (i, nx, j, ny, k, nz, False),
        (i, nx, j, ny, k, nz, True),
        (j, ny, i, nx, k, nz, False),
        (j, ny, i, nx, k, nz, True),
        (k, nz, i, nx, j, ny, False),
        (k, nz, i, nx, j, ny, True),
    ]
    for face, (gn, nn, ga, na, gb, nb, far) in zip(modes, specs):
        for p, q, amp in face:
            th_a = math.pi * p / (na + 1)
            th_b = math.pi * q / (nb + 1)
            prof = _face_term(nn, gn, th_a, th_b, ga, gb, far)
            u = u + amp * np.sin(th_a * ga) * np.sin(th_b * gb) * prof
    return np.ascontiguousarray(u)


def laplace_error_bound(nx, ny, nz, rnorm):
    """||u - u*||_2 <= ||r||_2 / (6 (1 - mu1)) for the zero-boundary operator."""
    mu1 = slowest_factor(nx, ny, nz)
    return rnorm / (6.0 * (1.0 - mu1))


def product_bump(nx, ny, nz):
    """e* = f(i) g(j) h(k) with f(i) = i (nx+1-i): zero on the boundary layer.

    Its exact right-hand side for 6e - sum6(e) is 2 (gh + fh + fg), since the
    second difference of f is -2.
    """
    i, j, k = index_grids(nx, ny, nz)
    f = i * (nx + 1 - i)
    g = j * (ny + 1 - j)
    h = k * (nz + 1 - k)
    e = np.array(np.broadcast_to(f * g * h, (nz + 2, ny + 2, nx + 2)))
    rhs = np.ascontiguousarray(np.broadcast_to(2 * (g * h + f * h + f * g),
                                               (nz + 2, ny + 2, nx + 2)))
    return e, rhs
