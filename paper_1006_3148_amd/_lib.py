"""ctypes declarations of the C-ABI in include/jacobi.h."""

from __future__ import annotations

import ctypes
import os

# torch first: its bundled HIP runtime carries the same soname as the one
# libjacobi.so links (libamdhip64.so.7), so loading torch first makes both use
# a single runtime instance in the process.
import torch  # noqa: F401

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libjacobi.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libjacobi.so is not built (expected at %s); run "
        "`python -c 'import __graft_entry__ as g; g.build()'` first" % LIB_PATH)

lib = ctypes.CDLL(LIB_PATH)

JACOBI_OK = 0
STATUS = {
    -1: "JACOBI_EINVAL",
    -2: "JACOBI_EUNSUPPORTED",
    -3: "JACOBI_EWORKSPACE",
    -4: "JACOBI_EHIP",
    -5: "JACOBI_ETIMEOUT",
    -6: "JACOBI_ESTATE",
}
F64, F32_REFINED, F32_MULTIGRID = 0, 1, 2
LAYOUT_AB, LAYOUT_COMPRESSED = 0, 1


class JacobiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code
        self.name = STATUS.get(code, "?")


def check(rc: int) -> None:
    if rc != JACOBI_OK:
        raise JacobiError(rc, lib.jacobi_last_error().decode())


class JacobiDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
        ("dtype", ctypes.c_int32), ("layout", ctypes.c_int32),
        ("t", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
        ("rows_per_wave", ctypes.c_int32), ("seg_len", ctypes.c_int32),
        ("inner_sweeps", ctypes.c_int32), ("use_graph", ctypes.c_int32),
        ("teams", ctypes.c_int32), ("looseness", ctypes.c_int32),
        ("grid0", ctypes.c_void_p), ("grid1", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p), ("stencil", ctypes.c_int32),
    ]


class JacobiBatchDesc(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("dims", ctypes.POINTER(ctypes.c_int64)),
        ("grid0", ctypes.POINTER(ctypes.c_void_p)),
        ("grid1", ctypes.POINTER(ctypes.c_void_p)),
        ("t", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
        ("rows_per_wave", ctypes.c_int32), ("inner_sweeps", ctypes.c_int32),
        ("use_graph", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p),
    ]


_h = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_descp = ctypes.POINTER(JacobiDesc)
_bdescp = ctypes.POINTER(JacobiBatchDesc)

_SIGS = {
    "jacobi_grid_bytes": ([_descp, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "jacobi_workspace_size": ([_descp, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "jacobi_create": ([_descp, ctypes.POINTER(_h)], ctypes.c_int),
    "jacobi_sweep": ([_h, ctypes.c_int64], ctypes.c_int),
    "jacobi_residual": ([_h, _dp, _dp], ctypes.c_int),
    "jacobi_solve": ([_h, ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                      ctypes.c_int64, _i64p, _dp], ctypes.c_int),
    "jacobi_sync": ([_h], ctypes.c_int),
    "jacobi_current": ([_h, ctypes.POINTER(ctypes.c_void_p), _i64p], ctypes.c_int),
    "jacobi_info": ([_h, _i64p, _i32p, _i32p, _i32p], ctypes.c_int),
    "jacobi_destroy": ([_h], ctypes.c_int),
    "jacobi_last_error": ([], ctypes.c_char_p),
    "jacobi_tile_supported": ([ctypes.c_int32] * 4, ctypes.c_int),
    "jacobi_batch_workspace_size": ([_bdescp, ctypes.POINTER(ctypes.c_size_t)],
                                    ctypes.c_int),
    "jacobi_batch_create": ([_bdescp, ctypes.POINTER(_h)], ctypes.c_int),
    "jacobi_batch_sweep": ([_h, ctypes.c_int64], ctypes.c_int),
    "jacobi_batch_residual": ([_h, _dp, _dp], ctypes.c_int),
    "jacobi_batch_solve": ([_h, ctypes.c_double, _dp, ctypes.c_int64, ctypes.c_int64,
                            _i64p, _dp], ctypes.c_int),
    "jacobi_batch_current": ([_h, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p),
                              _i64p], ctypes.c_int),
    "jacobi_batch_info": ([_h, _i64p, _i32p, _i32p, _i32p, _dp], ctypes.c_int),
    "jacobi_batch_tune_log": ([_h, ctypes.c_int32, _i32p, _i32p, _i32p, _dp, _i32p],
                              ctypes.c_int),
    "jacobi_batch_sync": ([_h], ctypes.c_int),
    "jacobi_batch_destroy": ([_h], ctypes.c_int),
    "jacobi_tune_log": ([_h, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
                         ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "jacobi_residual_noalloc": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                 ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                 ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "jacobi_probe_copy": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                           ctypes.c_void_p], ctypes.c_int),
    "jacobi_probe_update": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p],
                            ctypes.c_int),
}

for _name, (_args, _res) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_SIGS)
