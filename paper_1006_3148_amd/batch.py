"""Python handle over the batched C-ABI (argument marshalling only)."""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import JacobiBatchDesc, check, lib


def _align(n: int, a: int) -> int:
    return (n + a - 1) // a * a


class JacobiBatch:
    """Many independent problems swept together.

    ``boxes``: list of (nz+2, ny+2, nx+2) float64 boxes (numpy).  All grids live
    in two flat torch allocations carved at 256-byte offsets.
    """

    def __init__(self, boxes, t: int = 0, dtype: str = "f64",
                 inner_sweeps: int = 0, use_graph: bool = True,
                 tile_rows: int = 0, rows_per_wave: int = 0, stream=None,
                 device: str = "cuda"):
        self.count = len(boxes)
        self.shapes = [tuple(b.shape) for b in boxes]
        dims = []
        offs = []
        off = 0
        for (nz2, ny2, nx2) in self.shapes:
            dims += [nx2 - 2, ny2 - 2, nz2 - 2]
            offs.append(off)
            off = _align(off + nx2 * ny2 * nz2, 32)  # 256 B in doubles
        self.offs = offs
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        with torch.cuda.stream(self.stream):
            self.g0 = torch.empty(max(off, 1), dtype=torch.float64, device=device)
            self.g1 = torch.empty(max(off, 1), dtype=torch.float64, device=device)
        for b, o in zip(boxes, offs):
            n = b.size
            self.g0[o:o + n].copy_(torch.from_numpy(
                np.ascontiguousarray(b, dtype=np.float64)).reshape(-1))
        self._dims = (ctypes.c_int64 * len(dims))(*dims)
        base0, base1 = self.g0.data_ptr(), self.g1.data_ptr()
        self._p0 = (ctypes.c_void_p * self.count)(*[base0 + 8 * o for o in offs])
        self._p1 = (ctypes.c_void_p * self.count)(*[base1 + 8 * o for o in offs])
        d = JacobiBatchDesc()
        d.count = self.count
        d.dtype = _lib.F64 if dtype == "f64" else _lib.F32_REFINED
        d.dims = self._dims
        d.grid0 = self._p0
        d.grid1 = self._p1
        d.t = t
        d.tile_rows = tile_rows
        d.rows_per_wave = rows_per_wave
        d.inner_sweeps = inner_sweeps
        d.use_graph = 1 if use_graph else 0
        wb = ctypes.c_size_t()
        check(lib.jacobi_batch_workspace_size(ctypes.byref(d), ctypes.byref(wb)))
        with torch.cuda.stream(self.stream):
            self.ws = torch.empty(max(wb.value, 256), dtype=torch.uint8, device=device)
        d.workspace = self.ws.data_ptr()
        d.workspace_bytes = self.ws.numel()
        d.stream = int(self.stream.cuda_stream)
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        check(lib.jacobi_batch_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self._desc = d

    def sweep(self, n: int) -> None:
        check(lib.jacobi_batch_sweep(self._h, int(n)))

    def residual(self):
        l2 = (ctypes.c_double * self.count)()
        mx = (ctypes.c_double * self.count)()
        check(lib.jacobi_batch_residual(self._h, l2, mx))
        return np.array(l2[:]), np.array(mx[:])

    def solve(self, rel_tol: float, max_sweeps: int, check_every: int, r0=None):
        """Per-problem first sweep count at which ||r|| <= rel_tol * r0."""
        ref = None
        if r0 is not None:
            ref = (ctypes.c_double * self.count)(*[float(x) for x in r0])
        done = (ctypes.c_int64 * self.count)()
        fin = (ctypes.c_double * self.count)()
        check(lib.jacobi_batch_solve(self._h, rel_tol, ref, int(max_sweeps),
                                     int(check_every), done, fin))
        return np.array(done[:]), np.array(fin[:])

    def sync(self) -> None:
        check(lib.jacobi_batch_sync(self._h))

    def info(self):
        s = ctypes.c_int64()
        t = ctypes.c_int32()
        rows = ctypes.c_int32()
        rpw = ctypes.c_int32()
        ms = ctypes.c_double()
        check(lib.jacobi_batch_info(self._h, ctypes.byref(s), ctypes.byref(t),
                                    ctypes.byref(rows), ctypes.byref(rpw),
                                    ctypes.byref(ms)))
        return {"sweeps": s.value, "t": t.value, "tile_rows": rows.value,
                "rows_per_wave": rpw.value, "tune_ms": ms.value}

    def tune_log(self):
        cap = 64
        t = (ctypes.c_int32 * cap)()
        rows = (ctypes.c_int32 * cap)()
        rpw = (ctypes.c_int32 * cap)()
        g = (ctypes.c_double * cap)()
        n = ctypes.c_int32()
        check(lib.jacobi_batch_tune_log(self._h, cap, t, rows, rpw, g,
                                        ctypes.byref(n)))
        return [{"t": t[i], "tile_rows": rows[i], "rows_per_wave": rpw[i],
                 "glups": g[i]} for i in range(min(n.value, cap))]

    def current(self, i: int) -> torch.Tensor:
        origin = ctypes.c_void_p()
        st = (ctypes.c_int64 * 3)()
        check(lib.jacobi_batch_current(self._h, i, ctypes.byref(origin), st))
        base = self.g0 if origin.value < self.g1.data_ptr() or \
            origin.value >= self.g1.data_ptr() + 8 * self.g1.numel() else self.g1
        off = (origin.value - base.data_ptr()) // 8
        nz2, ny2, nx2 = self.shapes[i]
        return torch.as_strided(base, (nz2, ny2, nx2), (st[2], st[1], st[0]), off)

    def box(self, i: int) -> np.ndarray:
        self.sync()
        return self.current(i).contiguous().cpu().numpy()

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib.jacobi_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
