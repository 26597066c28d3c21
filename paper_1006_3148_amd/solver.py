"""Python handle over the C-ABI solver (argument marshalling only)."""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import JacobiDesc, check, lib


def _stream_ptr(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def tile_supported(t: int, tile_rows: int, rows_per_wave: int,
                   dtype: str = "f64") -> bool:
    d = _lib.F64 if dtype == "f64" else _lib.F32_REFINED
    return bool(lib.jacobi_tile_supported(d, t, tile_rows, rows_per_wave))


def probe_copy(src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
    """STREAM-copy probe dst[:] = src[:] (float64, even length)."""
    check(lib.jacobi_probe_copy(src.data_ptr(), dst.data_ptr(), src.numel(),
                                _stream_ptr(stream)))


def probe_update(a: torch.Tensor, stream=None) -> None:
    """Array-update probe a[:] += 1 (float64, even length)."""
    check(lib.jacobi_probe_update(a.data_ptr(), a.numel(), _stream_ptr(stream)))


class Jacobi:
    """One Laplace problem on the GPU.

    ``box`` is the initial (nz+2, ny+2, nx+2) float64 box (numpy or torch):
    Dirichlet boundary layer plus initial interior.  Grids and workspace are
    torch allocations owned by this object.
    """

    def __init__(self, box, t: int = 4, layout: str = "ab", dtype: str = "f64",
                 inner_sweeps: int = 0, tile_rows: int = 0,
                 rows_per_wave: int = 0, seg_len: int = 0, stream=None,
                 device: str = "cuda", use_graph: bool = False, teams: int = 0,
                 looseness: int = -1, stencil: int = 7):
        if isinstance(box, np.ndarray):
            box_t = torch.from_numpy(np.ascontiguousarray(box, dtype=np.float64))
        else:
            box_t = box.to(torch.float64)
        if box_t.dim() != 3 or min(box_t.shape) < 3:
            raise ValueError("box must be (nz+2, ny+2, nx+2) with every dim >= 3")
        nz2, ny2, nx2 = box_t.shape
        self.nx, self.ny, self.nz = nx2 - 2, ny2 - 2, nz2 - 2
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        d = JacobiDesc()
        d.nx, d.ny, d.nz = self.nx, self.ny, self.nz
        d.dtype = {"f64": _lib.F64, "f32_refined": _lib.F32_REFINED,
                   "f32_multigrid": _lib.F32_MULTIGRID}[dtype]
        d.layout = _lib.LAYOUT_AB if layout == "ab" else _lib.LAYOUT_COMPRESSED
        d.t = t
        d.tile_rows = tile_rows
        d.rows_per_wave = rows_per_wave
        d.seg_len = seg_len
        d.inner_sweeps = inner_sweeps
        d.use_graph = 1 if use_graph else 0
        d.teams = teams
        d.looseness = looseness
        d.stencil = stencil
        self.layout = layout
        gb = ctypes.c_size_t()
        check(lib.jacobi_grid_bytes(ctypes.byref(d), ctypes.byref(gb)))
        wb = ctypes.c_size_t()
        check(lib.jacobi_workspace_size(ctypes.byref(d), ctypes.byref(wb)))
        n = gb.value // 8
        with torch.cuda.stream(self.stream):
            self.grid0 = torch.empty(n, dtype=torch.float64, device=device)
            self.grid1 = (torch.empty(n, dtype=torch.float64, device=device)
                          if layout == "ab" else None)
            self.ws = torch.empty(max(wb.value, 256), dtype=torch.uint8, device=device)
        if layout == "ab":
            self.grid0.view(nz2, ny2, nx2).copy_(box_t, non_blocking=False)
        d.grid0 = self.grid0.data_ptr()
        d.grid1 = self.grid1.data_ptr() if self.grid1 is not None else None
        d.workspace = self.ws.data_ptr()
        d.workspace_bytes = self.ws.numel()
        d.stream = _stream_ptr(self.stream)
        self._desc = d
        h = ctypes.c_void_p()
        check(lib.jacobi_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        if layout != "ab":
            self.current().copy_(box_t.to(self.grid0.device))
        torch.cuda.synchronize()

    # -- calls -------------------------------------------------------------
    def sweep(self, n: int) -> None:
        check(lib.jacobi_sweep(self._h, int(n)))

    def residual(self):
        l2 = ctypes.c_double()
        mx = ctypes.c_double()
        check(lib.jacobi_residual(self._h, ctypes.byref(l2), ctypes.byref(mx)))
        return l2.value, mx.value

    def solve(self, rel_tol: float, max_sweeps: int, check_every: int,
              r0: float = 0.0):
        done = ctypes.c_int64()
        fin = ctypes.c_double()
        check(lib.jacobi_solve(self._h, rel_tol, r0, int(max_sweeps),
                               int(check_every), ctypes.byref(done),
                               ctypes.byref(fin)))
        return done.value, fin.value

    def sync(self) -> None:
        check(lib.jacobi_sync(self._h))

    def info(self):
        s = ctypes.c_int64()
        t = ctypes.c_int32()
        rows = ctypes.c_int32()
        seg = ctypes.c_int32()
        check(lib.jacobi_info(self._h, ctypes.byref(s), ctypes.byref(t),
                              ctypes.byref(rows), ctypes.byref(seg)))
        return {"sweeps": s.value, "t": t.value, "tile_rows": rows.value,
                "seg_len": seg.value}

    def tune_log(self):
        """Autotuner measurements of a t=0 handle and the tuning time (ms)."""
        cap = 32
        t = (ctypes.c_int32 * cap)()
        rows = (ctypes.c_int32 * cap)()
        rpw = (ctypes.c_int32 * cap)()
        g = (ctypes.c_double * cap)()
        n = ctypes.c_int32()
        ms = ctypes.c_double()
        check(lib.jacobi_tune_log(self._h, cap, t, rows, rpw, g, ctypes.byref(n),
                                  ctypes.byref(ms)))
        return ([{"t": t[q], "tile_rows": rows[q], "rows_per_wave": rpw[q],
                  "glups": g[q]} for q in range(min(n.value, cap))], ms.value)

    def current(self) -> torch.Tensor:
        """Strided torch view of the current iterate (nz+2, ny+2, nx+2)."""
        origin = ctypes.c_void_p()
        strides = (ctypes.c_int64 * 3)()
        check(lib.jacobi_current(self._h, ctypes.byref(origin), strides))
        base = self.grid0 if self.grid1 is None else None
        if base is None:
            p0 = self.grid0.data_ptr()
            base = self.grid0 if origin.value == p0 else self.grid1
        off = (origin.value - base.data_ptr()) // 8
        return torch.as_strided(base, (self.nz + 2, self.ny + 2, self.nx + 2),
                                (strides[2], strides[1], strides[0]), off)

    def box(self) -> np.ndarray:
        """Copy of the current iterate as a contiguous numpy float64 box."""
        self.sync()
        return self.current().contiguous().cpu().numpy()

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib.jacobi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
