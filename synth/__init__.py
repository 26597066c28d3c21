"""Seeded synthetic inputs for the 3D 7-point Jacobi problem.

This module only draws random numbers and lays them out; it holds none of the
solver's arithmetic.  Both the CPU oracle (through the tests) and the GPU path
(through the tests and the benchmark) take their inputs from here, so that the
two sides see the same bytes.

Layout of every grid ("box"): a C-ordered array of shape (nz+2, ny+2, nx+2),
i.e. the i index is contiguous, then j, then k.  The outer layer of the box is
the Dirichlet boundary of the boundary value problem (Sect. 1.1 of the paper
treats Jacobi as a solver for a boundary value problem); the interior
(1..nx, 1..ny, 1..nz) is the unknown field, initialised to zero.  The 12 edge
lines and 8 corners of the box are never read by the 7-point stencil; the
generators set them to zero.

Random source: numpy ``Generator(PCG64(seed))``; the order in which values are
drawn is part of the definition of each input.
"""

from .grids import (  # noqa: F401
    uniform_box,
    full_random_box,
    sine_face_box,
    sine_face_modes,
    sine_faces,
    unit_face_mode_box,
    batch_dims,
    batch_problems,
    zero_edges,
    interior,
)
