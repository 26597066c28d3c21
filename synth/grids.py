"""Seeded box generators (see the package docstring for the layout)."""

from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def interior(box: np.ndarray) -> np.ndarray:
    """View of the interior cells of a (nz+2, ny+2, nx+2) box."""
    return box[1:-1, 1:-1, 1:-1]


def zero_edges(box: np.ndarray) -> np.ndarray:
    """Set the 12 edge lines and 8 corners of the box to zero (in place).

    A cell is on an edge when at least two of its indices are on the outer
    layer; those cells are never read by the 7-point stencil.
    """
    nz2, ny2, nx2 = box.shape
    k = np.arange(nz2)[:, None, None]
    j = np.arange(ny2)[None, :, None]
    i = np.arange(nx2)[None, None, :]
    on = ((k == 0) | (k == nz2 - 1)).astype(np.int8) \
        + ((j == 0) | (j == ny2 - 1)).astype(np.int8) \
        + ((i == 0) | (i == nx2 - 1)).astype(np.int8)
    box[on >= 2] = 0
    return box


def uniform_box(nx: int, ny: int, nz: int, seed: int,
                dtype=np.float64) -> np.ndarray:
    """Boundary values U[0,1), interior zero, edges zero.

    Draw order: one ``rng.random((nz+2, ny+2, nx+2))`` for the whole box, then
    the interior and the edges are overwritten with zeros.
    """
    rng = _rng(seed)
    box = rng.random((nz + 2, ny + 2, nx + 2))
    box[1:-1, 1:-1, 1:-1] = 0.0
    zero_edges(box)
    return box.astype(dtype, copy=False)


def full_random_box(nx: int, ny: int, nz: int, seed: int,
                    dtype=np.float64) -> np.ndarray:
    """Every cell U[0,1): interior, faces, and the edges and corners of the
    boundary layer (which a 27-point update reads).

    Draw order: one ``rng.random((nz+2, ny+2, nx+2))`` for the whole box.
    """
    return _rng(seed).random((nz + 2, ny + 2, nx + 2)).astype(dtype, copy=False)


# Faces in this fixed order: i=0, i=nx+1, j=0, j=ny+1, k=0, k=nz+1.
FACES = ("i0", "i1", "j0", "j1", "k0", "k1")


def sine_face_modes(seed: int, modes_per_face: int = 8, pmax: int = 4):
    """Random low-frequency sine modes for the six faces.

    Per face (in ``FACES`` order), per mode: p ~ U{1..pmax}, q ~ U{1..pmax}
    (drawn as ``rng.integers(1, pmax+1, 2)``), then the amplitude
    a ~ N(0, 1).  Returns a list of six lists of (p, q, a).
    """
    rng = _rng(seed)
    out = []
    for _ in FACES:
        face = []
        for _m in range(modes_per_face):
            p, q = (int(v) for v in rng.integers(1, pmax + 1, 2))
            a = float(rng.standard_normal())
            face.append((p, q, a))
        out.append(face)
    return out


def _face_values(modes, na: int, nb: int) -> np.ndarray:
    """g(a, b) = sum a_m sin(pi p a/(na+1)) sin(pi q b/(nb+1)), a in 0..na+1.

    Returned with shape (nb+2, na+2) (b is the slower in-plane axis).
    """
    ia = np.arange(na + 2, dtype=np.float64)
    ib = np.arange(nb + 2, dtype=np.float64)
    g = np.zeros((nb + 2, na + 2), dtype=np.float64)
    for p, q, amp in modes:
        g += amp * np.outer(np.sin(np.pi * q * ib / (nb + 1)),
                            np.sin(np.pi * p * ia / (na + 1)))
    return g


def sine_face_box(nx: int, ny: int, nz: int, seed: int,
                  modes_per_face: int = 8, pmax: int = 4,
                  dtype=np.float64) -> np.ndarray:
    """Boundary = sum of random low-frequency sine modes per face.

    For each face the two in-plane axes are taken in (i, j, k) order: the
    i-faces use (j, k), the j-faces (i, k), the k-faces (i, j); the first of
    the two carries p, the second q.  Interior and edges are zero.
    """
    modes = sine_face_modes(seed, modes_per_face, pmax)
    box = np.zeros((nz + 2, ny + 2, nx + 2), dtype=np.float64)
    gi0 = _face_values(modes[0], ny, nz)   # shape (nz+2, ny+2)
    gi1 = _face_values(modes[1], ny, nz)
    gj0 = _face_values(modes[2], nx, nz)   # shape (nz+2, nx+2)
    gj1 = _face_values(modes[3], nx, nz)
    gk0 = _face_values(modes[4], nx, ny)   # shape (ny+2, nx+2)
    gk1 = _face_values(modes[5], nx, ny)
    box[:, :, 0] = gi0
    box[:, :, -1] = gi1
    box[:, 0, :] = gj0
    box[:, -1, :] = gj1
    box[0, :, :] = gk0
    box[-1, :, :] = gk1
    box[1:-1, 1:-1, 1:-1] = 0.0
    zero_edges(box)
    return box.astype(dtype, copy=False)


def batch_dims(count: int, seed: int, lo: int = 32, step: int = 16,
               nsteps: int = 11):
    """Interior dims of a batch, drawn as the first step of ``batch_problems``.

    Only the dims are returned; the boxes are skipped.  Because boxes are drawn
    from the same stream between dims, this replays the full draw order.
    """
    return [(nx, ny, nz) for nx, ny, nz, _ in
            batch_problems(count, seed, lo, step, nsteps, with_boxes=False)]


def batch_problems(count: int, seed: int, lo: int = 32, step: int = 16,
                   nsteps: int = 11, with_boxes: bool = True):
    """Yield (nx, ny, nz, box) for a batch of independent problems.

    Per problem, in order: dims = lo + step * rng.integers(0, nsteps, 3) taken
    as (nx, ny, nz); then a U[0,1) box drawn as in ``uniform_box`` (one
    ``rng.random`` call for the whole box; interior and edges zeroed).
    With ``with_boxes=False`` the random box values are still drawn (to keep
    the stream aligned) but not returned.
    """
    rng = _rng(seed)
    for _ in range(count):
        d = lo + step * rng.integers(0, nsteps, 3)
        nx, ny, nz = (int(v) for v in d)
        box = rng.random((nz + 2, ny + 2, nx + 2))
        if with_boxes:
            box[1:-1, 1:-1, 1:-1] = 0.0
            zero_edges(box)
            yield nx, ny, nz, box
        else:
            yield nx, ny, nz, None


def sine_faces(n: int, seed: int, modes_per_face: int = 8, pmax: int = 4):
    """The six face arrays of ``sine_face_box(n, n, n, seed)`` (cubic grids).

    Returns an array of shape (6, n+2, n+2): face f in ``FACES`` order, indexed
    [b, a] with (a, b) the face's in-plane axes in (i, j, k) order.  Values
    on the box edges are left as computed (the stencil never reads them).
    """
    modes = sine_face_modes(seed, modes_per_face, pmax)
    return np.stack([_face_values(m, n, n) for m in modes]), modes


def unit_face_mode_box(n: int, face: int, p: int, q: int) -> np.ndarray:
    """Cubic box whose face ``face`` (``FACES`` order) carries the single mode
    sin(pi p a/(n+1)) sin(pi q b/(n+1)); other faces, interior and edges 0."""
    g = _face_values([(p, q, 1.0)], n, n)
    box = np.zeros((n + 2, n + 2, n + 2), dtype=np.float64)
    if face == 0:
        box[:, :, 0] = g
    elif face == 1:
        box[:, :, -1] = g
    elif face == 2:
        box[:, 0, :] = g
    elif face == 3:
        box[:, -1, :] = g
    elif face == 4:
        box[0, :, :] = g
    else:
        box[-1, :, :] = g
    box[1:-1, 1:-1, 1:-1] = 0.0
    zero_edges(box)
    return box
