"""Small driver that runs trips of one configuration, for profiling.

    python -m paper_1006_3148_amd.tripbench --n 512 --t 5 --layout ab --sweeps 20

Builds a seeded U[0,1)-boundary box (seed 2, interior 0; n x n x n, or
n x n x nz with --nz), creates a handle
with the given configuration, runs one warm-up call and then ``--reps``
calls of ``--sweeps`` sweeps, and prints one JSON line with the HIP-event
time per call and the GLUP/s.  ``--t`` may be a comma-separated list: each
t gets its own handle, in turn (one profiler run covers all of them).
Every sweep runs in libjacobi's kernels.
"""

from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--nz", type=int, default=0, help="k extent (0 = n): an n x n x nz box")
    ap.add_argument("--t", default="5")
    ap.add_argument("--layout", default="ab")
    ap.add_argument("--dtype", default="f64")
    ap.add_argument("--sweeps", type=int, default=0, help="per call (0 = 4t)")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--rows-per-wave", type=int, default=0)
    ap.add_argument("--teams", type=int, default=0)
    ap.add_argument("--looseness", type=int, default=-1)
    ap.add_argument("--seg-len", type=int, default=0, help="k planes per segment (0 = auto)")
    ap.add_argument("--stencil", type=int, default=7, help="7 or 27 (27-point update)")
    a = ap.parse_args(argv)
    import torch
    import synth
    from paper_1006_3148_amd import Jacobi
    torch.cuda.set_device(0)
    nz = a.nz if a.nz > 0 else a.n
    box = torch.from_numpy(synth.uniform_box(a.n, a.n, nz, seed=2)).cuda()
    for t in [int(v) for v in a.t.split(",")]:
        sweeps = a.sweeps if a.sweeps > 0 else 4 * t
        j = Jacobi(box, t=t, layout=a.layout, dtype=a.dtype, tile_rows=a.tile_rows,
                   rows_per_wave=a.rows_per_wave, teams=a.teams, looseness=a.looseness,
                   seg_len=a.seg_len, stencil=a.stencil)
        j.sweep(sweeps)
        j.sync()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(j.stream)
        for _ in range(a.reps):
            j.sweep(sweeps)
        ev[1].record(j.stream)
        j.sync()
        ms = ev[0].elapsed_time(ev[1]) / a.reps
        info = j.info()
        j.close()
        print(json.dumps({"n": a.n, "nz": nz, "t": t, "layout": a.layout, "dtype": a.dtype,
                          "stencil": a.stencil, "rows_per_wave": a.rows_per_wave,
                          "sweeps_per_call": sweeps, "tile_rows": info["tile_rows"],
                          "seg_len": info["seg_len"], "ms_per_call": round(ms, 4),
                          "glups": round(a.n * a.n * nz * sweeps / (ms * 1e-3) / 1e9, 1)}),
              flush=True)


if __name__ == "__main__":
    main()
