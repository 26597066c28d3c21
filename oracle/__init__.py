"""CPU oracle for the 3D 7-point Jacobi method -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline leg
of ``bench.py`` may import this package.  It shares no code with the GPU
library (``paper_1006_3148_amd``) and never imports it.

Contents
--------
* ``sweeps_f64``      -- Eq. (1) of the paper, successive A/B sweeps (Sect. 1.1),
                         plain C loops (``jacobi_oracle.c``).
* ``sweeps_f32``      -- the same sweep in single precision with a right-hand
                         side, used by the mixed-precision refinement.
* ``residual_f64``    -- per-cell residual fold(neighbours) - 6u of the
                         discrete Laplace equation (not in the paper; it is the
                         stopping test of the solver).
* ``residual_norm``   -- its 2-norm, long-double accumulation.
* ``refine_f32``      -- FP32 inner sweeps with FP64 residual and FP64
                         defect-correction update (``refine.py``).
* ``solve_to_tol``    -- plain run-to-tolerance driver.
* ``brute``           -- pure-Python per-cell loops for tiny grids.
* ``conv``            -- FP64 reference of the learned-guess network layers.

Each function states the passage it follows.  See ``jacobi_oracle.c`` for the
arithmetic readings (fold order, multiply by fl(1/6), no FMA).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jacobi_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-shared", "-fPIC", "-Wall"]

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle into ``oracle/liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    i64 = ctypes.c_int64
    lib.oracle_sweeps_f64.argtypes = [dp, dp, i64, i64, i64, i64, ctypes.c_int]
    lib.oracle_sweeps_f64.restype = ctypes.c_int
    lib.oracle_sweeps27_f64.argtypes = [dp, dp, i64, i64, i64, i64, ctypes.c_int]
    lib.oracle_sweeps27_f64.restype = ctypes.c_int
    lib.oracle_sweeps_f32.argtypes = [fp, fp, fp, i64, i64, i64, i64, ctypes.c_int]
    lib.oracle_sweeps_f32.restype = ctypes.c_int
    lib.oracle_residual_f64.argtypes = [dp, dp, i64, i64, i64, ctypes.c_int]
    lib.oracle_residual_f64.restype = ctypes.c_int
    lib.oracle_residual_norm_f64.argtypes = [dp, i64, i64, i64]
    lib.oracle_residual_norm_f64.restype = ctypes.c_double
    lib.oracle_max_threads.argtypes = []
    lib.oracle_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def max_threads() -> int:
    """Threads an OpenMP region of the oracle uses by default."""
    return int(_load().oracle_max_threads())


def _dims(box: np.ndarray):
    nz2, ny2, nx2 = box.shape
    return nx2 - 2, ny2 - 2, nz2 - 2


def _check_box(box: np.ndarray, dtype) -> None:
    if box.dtype != dtype or box.ndim != 3 or not box.flags.c_contiguous:
        raise ValueError("box must be a C-contiguous 3-D %s array" % np.dtype(dtype))
    if min(box.shape) < 3:
        raise ValueError("every interior dimension must be >= 1")


def sweeps_f64(box: np.ndarray, nsweeps: int, nthreads: int = 0) -> np.ndarray:
    """Return ``box`` after ``nsweeps`` Jacobi sweeps (Eq. (1), Sect. 1.1).

    The input is not modified.  ``nthreads=0`` uses all OpenMP threads.
    """
    _check_box(box, np.float64)
    a = np.array(box, dtype=np.float64, copy=True, order="C")
    b = np.empty_like(a)
    nx, ny, nz = _dims(a)
    nt = nthreads if nthreads > 0 else max_threads()
    dp = ctypes.POINTER(ctypes.c_double)
    rc = _load().oracle_sweeps_f64(a.ctypes.data_as(dp), b.ctypes.data_as(dp),
                                   nx, ny, nz, int(nsweeps), nt)
    if rc != 0:
        raise ValueError("oracle_sweeps_f64 rejected its arguments")
    return a


def sweeps27_f64(box: np.ndarray, nsweeps: int, nthreads: int = 0) -> np.ndarray:
    """Return ``box`` after ``nsweeps`` sweeps of the 27-point Jacobi update
    (faces, edges, corners weighted 14, 3, 1 over 128; the fold order is in
    jacobi_oracle.c).  Not in the paper: one of the other stencils the
    k-streaming pipeline carries.  The whole boundary layer, edges and corners
    included, is read and kept."""
    _check_box(box, np.float64)
    a = np.array(box, dtype=np.float64, copy=True, order="C")
    b = np.empty_like(a)
    nx, ny, nz = _dims(a)
    nt = nthreads if nthreads > 0 else max_threads()
    dp = ctypes.POINTER(ctypes.c_double)
    rc = _load().oracle_sweeps27_f64(a.ctypes.data_as(dp), b.ctypes.data_as(dp),
                                     nx, ny, nz, int(nsweeps), nt)
    if rc != 0:
        raise ValueError("oracle_sweeps27_f64 rejected its arguments")
    return a


def sweeps_f32(box: np.ndarray, nsweeps: int, rhs: np.ndarray | None = None,
               nthreads: int = 0) -> np.ndarray:
    """Single-precision sweeps e <- (fold(e nbrs) + rhs) * fl32(1/6).

    ``rhs`` is a float32 box of the same shape (interior entries are used) or
    None for rhs = 0.  Returns a new array.
    """
    _check_box(box, np.float32)
    a = np.array(box, dtype=np.float32, copy=True, order="C")
    b = np.empty_like(a)
    nx, ny, nz = _dims(a)
    fp = ctypes.POINTER(ctypes.c_float)
    rptr = None
    if rhs is not None:
        _check_box(rhs, np.float32)
        if rhs.shape != box.shape:
            raise ValueError("rhs must have the shape of the box")
        rptr = rhs.ctypes.data_as(fp)
    nt = nthreads if nthreads > 0 else max_threads()
    rc = _load().oracle_sweeps_f32(a.ctypes.data_as(fp), b.ctypes.data_as(fp),
                                   rptr, nx, ny, nz, int(nsweeps), nt)
    if rc != 0:
        raise ValueError("oracle_sweeps_f32 rejected its arguments")
    return a


def residual_f64(box: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """Per-cell residual r = fold(u nbrs) - fl(6u) on the interior (boundary 0)."""
    _check_box(box, np.float64)
    u = np.ascontiguousarray(box, dtype=np.float64)
    r = np.empty_like(u)
    nx, ny, nz = _dims(u)
    nt = nthreads if nthreads > 0 else max_threads()
    dp = ctypes.POINTER(ctypes.c_double)
    rc = _load().oracle_residual_f64(u.ctypes.data_as(dp), r.ctypes.data_as(dp),
                                     nx, ny, nz, nt)
    if rc != 0:
        raise ValueError("oracle_residual_f64 rejected its arguments")
    return r


def residual_norm(box: np.ndarray) -> float:
    """||fold(u nbrs) - 6u||_2 over the interior, long-double accumulation."""
    _check_box(box, np.float64)
    u = np.ascontiguousarray(box, dtype=np.float64)
    nx, ny, nz = _dims(u)
    dp = ctypes.POINTER(ctypes.c_double)
    return float(_load().oracle_residual_norm_f64(u.ctypes.data_as(dp), nx, ny, nz))


from .refine import refine_f32, refine_outer_f32  # noqa: E402,F401
from .solve import solve_to_tol  # noqa: E402,F401
from . import brute  # noqa: E402,F401
