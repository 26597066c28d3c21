"""Benchmark of the temporally blocked FP64 3D 7-point Jacobi hot path.

One "step" = 200 FP64 Jacobi sweeps of a 512^3 interior (514^3 box, Dirichlet
boundary U[0,1) from seed 2, interior 0) through the trip kernel, followed by
one residual-norm check -- the workload the headline metric is quoted on.

Prints ONE JSON line (rank 0) with GLUP/s (interior cells x sweeps / s / 1e9),
the roofline of the dominant kernel (the trip kernel, HBM-bound: algorithmic
16 B per interior cell per trip) measured with HIP events on the solver's
stream, and the CPU oracle timed on a bounded sample on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--t T]
                       [--layout ab|compressed] [--no-extra] [--no-cpu]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# FP64 vector issue peak for separate adds and multiplies (no fused
# multiply-add): 256 CUs x 4 SIMDs x 16 FP64 lanes x 2.4 GHz, half of the
# published 78.6 TFLOP/s, which counts an FMA as two operations.
FP64_ADDMUL_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# FP64 adds and multiplies of one 27-point update (per interior cell and
# sweep): plane sums 1 + 2 + 2, the three folds 2 + 2 + 1, weights 3 + 2, and
# the two partial folds carried to the next plane 1 + 1 (the kernel's and the
# oracle's fold order; 53 if the 26 neighbours were summed term by term).
S27_OPS_PER_LUP = 16


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=512, help="interior edge length")
    ap.add_argument("--sweeps", type=int, default=200, help="sweeps per step")
    ap.add_argument("--t", type=int, default=0, help="sweeps per trip (0=best)")
    ap.add_argument("--layout", default="", help="ab | compressed ('' = best)")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--tts-only", type=int, default=0, metavar="N",
                    help="only measure time to 1e-8 at N^3 and print it as JSON")
    ap.add_argument("--tts-budget", type=float, default=0.0, metavar="S",
                    help="with --tts-only: seconds per form before extrapolating")
    ap.add_argument("--mg-tts", type=int, default=0, metavar="N",
                    help="only measure the multigrid-corrected time to 1e-8 at N^3 "
                         "(N = 2^k - 1)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=40.0)
    ap.add_argument("--quick", action="store_true",
                    help="skip the batched / 1024^3 / time-to-tolerance extras")
    ap.add_argument("--probe", action="store_true",
                    help="only run the copy probe (1 GiB in, 1 GiB out) 5 times; "
                         "used to scale HBM byte counters")
    return ap.parse_args()


# Default configuration of the headline line; chosen from the measured sweep
# over t and layouts (the "extra" block reproduces that sweep on every run).
DEFAULT_T = 5
DEFAULT_LAYOUT = "ab"


def time_steps(j, steps, sweeps, t, torch, residual=True):
    """Time `steps` steps; per-trip HIP events give the trip-kernel duration."""
    stream = j.stream
    trips_per_step = []
    left = sweeps
    while left > 0:
        trips_per_step.append(min(t, left))
        left -= trips_per_step[-1]
    full = [L for L in trips_per_step if L == t]
    ev = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        for L in trips_per_step:
            if L == t:
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                j.sweep(L)
                b.record(stream)
                ev.append((a, b))
            else:
                j.sweep(L)
        if residual:
            j.residual()
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = start.elapsed_time(end)
    trip_ms = [a.elapsed_time(b) for a, b in ev]
    j.sync()
    return wall, gpu_ms, trip_ms, len(full)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n, seconds):
    """The plain C oracle on the host cores: all OpenMP threads (the reported
    value) and one thread, each on a bounded number of sweeps of the same
    512^3 box (about seconds/2 of CPU time each)."""
    import oracle
    import synth
    box = synth.uniform_box(n, n, n, seed=2)
    out = {}
    for nt in (oracle.max_threads(), 1):
        t0 = time.perf_counter()
        oracle.sweeps_f64(box, 1, nthreads=nt)
        one = time.perf_counter() - t0
        s = max(1, int(0.5 * seconds / max(one, 1e-3)))
        t0 = time.perf_counter()
        oracle.sweeps_f64(box, s, nthreads=nt)
        dt = time.perf_counter() - t0
        out[nt] = (s, dt, n ** 3 * s / dt / 1e9)
    nt = oracle.max_threads()
    s, dt, g = out[nt]
    s1, dt1, g1 = out[1]
    return {"value": round(g, 4), "unit": "GLUP/s", "cores": nt, "kind": "oracle",
            "single_thread": round(g1, 4), "cpu_model": _cpu_model(),
            "nproc": os.cpu_count(),
            "sample": "%d^3 interior, plain C oracle (OpenMP over k planes): %d FP64 "
                      "sweeps on %d threads in %.1f s; %d sweeps on 1 thread in %.1f s"
                      % (n, s, nt, dt, s1, dt1)}


def glups(n, sweeps, seconds):
    return n ** 3 * sweeps / seconds / 1e9


def run_config(n, sweeps, t, layout, steps, warmup, torch, synth_box):
    from paper_1006_3148_amd import Jacobi
    j = Jacobi(synth_box, t=t, layout=layout)
    for _ in range(warmup):
        j.sweep(sweeps)
    j.sync()
    wall, gpu_ms, trip_ms, _ = time_steps(j, steps, sweeps, t, torch)
    info = j.info()
    j.close()
    return wall, gpu_ms, trip_ms, info


def probe_bw(torch, nbytes=2 << 30, reps=10):
    from paper_1006_3148_amd import probe_copy, probe_update
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    probe_copy(a, b)
    probe_update(a)
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        probe_copy(a, b)
    e.record()
    torch.cuda.synchronize()
    copy = 2 * nbytes * reps / (s.elapsed_time(e) * 1e-3) / 1e9
    s.record()
    for _ in range(reps):
        probe_update(a)
    e.record()
    torch.cuda.synchronize()
    upd = 2 * nbytes * reps / (s.elapsed_time(e) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return copy, upd


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; "
                          "--gpus %d is not supported" % args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch
    import synth

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.probe:
        from paper_1006_3148_amd import probe_copy
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            probe_copy(a, b)
        torch.cuda.synchronize()
        print(json.dumps({"probe": "copy", "bytes_read": a.numel() * 8,
                          "bytes_written": b.numel() * 8, "launches": 5}))
        return
    if args.mg_tts:
        print(json.dumps({"multigrid_time_to_1e-8": bench_multigrid_tts(torch, args.mg_tts)}),
              flush=True)
        return
    if args.tts_only:
        res = bench_time_to_tol(torch, args.tts_only, args.t or DEFAULT_T,
                                budget=args.tts_budget, layout=args.layout or "ab")
        print(json.dumps({"time_to_1e-8": res}), flush=True)
        return
    n, sweeps = args.n, args.sweeps
    t = args.t or DEFAULT_T
    layout = args.layout or DEFAULT_LAYOUT
    box = synth.uniform_box(n, n, n, seed=2)

    wall, gpu_ms, trip_ms, info = run_config(n, sweeps, t, layout, args.steps,
                                             args.warmup, torch, box)
    value = glups(n, sweeps * args.steps, wall)
    trip_avg_ms = float(np.mean(trip_ms))
    alg_bytes = 16.0 * n ** 3  # one read + one write per interior cell per trip
    achieved = alg_bytes / (trip_avg_ms * 1e-3) / 1e9

    traffic = None
    tpath = os.path.join(ROOT, "profiles", "trip_kernel_traffic.json")
    if os.path.exists(tpath):
        with open(tpath) as f:
            tr = json.load(f)
        if tr.get("kernel_config") == {"t": t, "layout": layout, "n": n,
                                       "tile_rows": info["tile_rows"]} and \
                tr.get("source_hash") == _kernel_hash():
            traffic = tr.get("bytes_per_launch")

    out = {
        "metric": "GLUP/s FP64 7-pt Jacobi 512^3 (200 sweeps/step), "
                  "temporally blocked",
        "value": round(value, 3),
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: boundary U[0,1) seed 2, interior 0",
        "config": {"workload": "%d^3 interior FP64 Jacobi, %d sweeps + 1 "
                               "residual per step" % (n, sweeps),
                   "t": t, "layout": layout, "tile_rows": info["tile_rows"],
                   "seg_len": info["seg_len"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": "trip_kernel<double,T=%d>" % t,
                     "launch_ms": round(trip_avg_ms, 4),
                     "alg_bytes_per_launch": alg_bytes},
        "gpu_event_ms_per_step": round(gpu_ms / args.steps, 4),
    }

    if not args.no_extra:
        extra = {}
        copy_bw, upd_bw = probe_bw(torch)
        extra["copy_probe_GBs"] = round(copy_bw, 1)
        extra["update_probe_GBs"] = round(upd_bw, 1)
        extra["roofline_glups_t1_spec"] = HBM_PEAK_GBS / 16.0
        extra["roofline_glups_t1_copy"] = round(copy_bw / 16.0, 1)
        tab = {}
        for lay in ("ab", "compressed"):
            for tt in range(1, 9):
                w, _, tm, _ = run_config(n, sweeps, tt, lay, 1, 1, torch, box)
                tab["%s_t%d" % (lay, tt)] = round(glups(n, sweeps, w), 1)
        extra["glups_by_layout_t_512"] = tab
        extra["stencil27_512"] = bench_stencil27(torch, n, sweeps, box)
        if not args.quick:
            extra["n64_100_sweeps"] = bench_small_64(torch)
            box1k = torch.from_numpy(synth.sine_face_box(1024, 1024, 1024, seed=3)).cuda()
            extra["n1024"] = bench_1024(torch, t, box1k)
            extra["stencil27_1024"] = bench_stencil27(torch, 1024, 48, box1k,
                                                      shapes=((3, 24, 3), (2, 36, 3)))
            del box1k
            torch.cuda.empty_cache()
            extra["teams_512"] = bench_teams(torch)
            extra["multigrid_time_to_1e-8_511"] = bench_multigrid_tts(torch, 511)
            extra["batched_256"] = bench_batched(torch)
            extra["time_to_1e-8_256"] = bench_time_to_tol(torch, 256, t)
            extra["time_to_1e-8_512_1024"] = ("profiles/time_to_tol_512.json, "
                                              "profiles/time_to_tol_1024.json (bench.py --tts-only N)")
        out["extra"] = extra

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(n, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def bench_1024(torch, t, box, sweeps=50):
    """1024^3 interior, sine-mode faces (`box`, on the GPU): the compressed
    single grid (8.6 GB plus shift planes) and the A/B layout (17.2 GB),
    GLUP/s of `sweeps` sweeps after a warm-up trip."""
    from paper_1006_3148_amd import Jacobi
    out = {"sweeps": sweeps, "t": t}
    for layout in ("compressed", "ab"):
        j = Jacobi(box, t=t, layout=layout)
        j.sweep(2 * t)
        j.sync()
        torch.cuda.synchronize()
        a = time.perf_counter()
        j.sweep(sweeps)
        j.sync()
        dt = time.perf_counter() - a
        info = j.info()
        j.close()
        del j
        torch.cuda.empty_cache()
        g = 1024 ** 3 * sweeps / dt / 1e9
        out[layout] = {"seg_len": info["seg_len"], "glups": round(g, 1),
                       "roofline_frac_spec": round(g / (HBM_PEAK_GBS * t / 16.0), 4)}
    return out


def bench_stencil27(torch, n, sweeps, box, shapes=((2, 36, 3), (3, 24, 3), (4, 24, 3))):
    """27-point A/B FP64 sweeps of the n^3 box for each tile shape (t, tile
    rows, rows per wave): GLUP/s over `sweeps` sweeps after a warm-up trip,
    and the roofline of the trip kernel from per-trip HIP events on the
    solver's stream.  The kernel is bound by FP64 vector issue (16 adds and
    multiplies per cell and sweep, see S27_OPS_PER_LUP), not by HBM (16 B per
    cell and trip)."""
    from paper_1006_3148_amd import Jacobi
    out = {"n": n, "sweeps": sweeps, "ops_per_lup": S27_OPS_PER_LUP}
    for t, rows, rpw in shapes:
        j = Jacobi(box, t=t, layout="ab", tile_rows=rows, rows_per_wave=rpw, stencil=27)
        j.sweep(t)
        j.sync()
        wall, _, trip_ms, _ = time_steps(j, 1, sweeps, t, torch, residual=False)
        j.close()
        del j
        ms = sum(trip_ms) / len(trip_ms)
        tops = S27_OPS_PER_LUP * n ** 3 * t / (ms * 1e-3) / 1e12
        gbs = 16.0 * n ** 3 / (ms * 1e-3) / 1e9
        out["t%d_%dx%d" % (t, rows // rpw, rpw)] = {
            "glups": round(glups(n, sweeps, wall), 1),
            "roofline": {"bound": "alu", "achieved": round(tops, 3),
                         "peak": round(FP64_ADDMUL_PEAK_TOPS, 2), "unit": "TFLOP/s",
                         "frac": round(tops / FP64_ADDMUL_PEAK_TOPS, 4),
                         "launch_ms": round(ms, 4), "hbm_alg_GBs": round(gbs, 1)}}
    torch.cuda.empty_cache()
    return out


def bench_teams(torch, n=512, sweeps=200):
    """Trips in one persistent launch (teams, per-tile counters, looseness
    d_u) against one launch per trip, and 16 sweeps per launch as two
    chained teams of t=8."""
    import synth
    from paper_1006_3148_amd import Jacobi
    box = torch.from_numpy(synth.uniform_box(n, n, n, seed=2)).cuda()
    out = {"n": n, "sweeps": sweeps}
    for name, kw in (("kernel_boundaries_t5", dict(t=5)),
                     ("teams40_t5_relaxed", dict(t=5, teams=40, looseness=-1)),
                     ("teams40_t5_lockstep", dict(t=5, teams=40, looseness=0)),
                     ("teams40_t5_du2", dict(t=5, teams=40, looseness=2)),
                     ("kernel_boundaries_t8", dict(t=8)),
                     ("t16_as_2_teams_of_8", dict(t=8, teams=2, looseness=-1))):
        j = Jacobi(box, **kw)
        j.sweep(sweeps)
        j.sync()
        torch.cuda.synchronize()
        a = time.perf_counter()
        j.sweep(sweeps)
        j.sync()
        dt = time.perf_counter() - a
        j.close()
        out[name] = round(n ** 3 * sweeps / dt / 1e9, 1)
    del box
    torch.cuda.empty_cache()
    return out


def bench_batched(torch, count=256, seed=4, sweeps=500):
    """256 uneven problems (edges 32..192 step 16), 500 sweeps, autotuned
    tile shape and t, hipGraph replay; FP64 and FP32-refined."""
    import synth
    from paper_1006_3148_amd import JacobiBatch
    probs = list(synth.batch_problems(count, seed))
    boxes = [p[3] for p in probs]
    cells = float(sum(p[0] * p[1] * p[2] for p in probs))
    res = {"problems": count, "cells": cells, "sweeps": sweeps}
    for dtype in ("f64", "f32_refined"):
        b = JacobiBatch(boxes, t=0, dtype=dtype, inner_sweeps=50)
        torch.cuda.synchronize()
        a = time.perf_counter()
        b.sweep(sweeps)          # autotune + capture + replay
        b.sync()
        first = time.perf_counter() - a
        a = time.perf_counter()
        b.sweep(sweeps)          # graph replay of the same schedule
        b.sync()
        steady = time.perf_counter() - a
        info = b.info()
        res[dtype] = {"first_call_s": round(first, 4), "steady_s": round(steady, 4),
                      "glups": round(cells * sweeps / steady / 1e9, 1),
                      "t": info["t"], "tile_rows": info["tile_rows"],
                      "tune_ms": round(info["tune_ms"], 2),
                      "tune_log": [(e["t"], e["tile_rows"], round(e["glups"], 1))
                                   for e in b.tune_log()]}
        b.close()
    del boxes
    torch.cuda.empty_cache()
    return res


def bench_small_64(torch, sweeps=100, reps=5):
    """64^3 interior (fits in L2/MALL), 100 single sweeps: launch-latency bound.
    Eager one launch per sweep (t=1), the same replayed as a captured hipGraph
    (single-problem and batch paths), and the blocked default for reference."""
    import synth
    from paper_1006_3148_amd import Jacobi, JacobiBatch
    box = synth.uniform_box(64, 64, 64, seed=1)
    cells = 64 ** 3
    res = {"n": 64, "sweeps": sweeps}

    def timed(obj):
        obj.sweep(sweeps)            # warm-up (and capture, for graphs)
        obj.sync()
        best = 1e30
        for _ in range(reps):
            torch.cuda.synchronize()
            a = time.perf_counter()
            obj.sweep(sweeps)
            obj.sync()
            best = min(best, time.perf_counter() - a)
        return best

    j = Jacobi(box, t=1)
    dt = timed(j)
    j.close()
    res["eager_t1"] = {"seconds": round(dt, 6), "glups": round(cells * sweeps / dt / 1e9, 1),
                       "us_per_sweep": round(dt / sweeps * 1e6, 2)}
    j = Jacobi(box, t=1, use_graph=True)
    dt = timed(j)
    j.close()
    res["graph_t1"] = {"seconds": round(dt, 6), "glups": round(cells * sweeps / dt / 1e9, 1),
                       "us_per_sweep": round(dt / sweeps * 1e6, 2)}
    b = JacobiBatch([box], t=1, use_graph=True)
    dt = timed(b)
    b.close()
    res["batch_graph_t1"] = {"seconds": round(dt, 6),
                             "glups": round(cells * sweeps / dt / 1e9, 1),
                             "us_per_sweep": round(dt / sweeps * 1e6, 2)}
    j = Jacobi(box, t=0)
    dt = timed(j)
    info = j.info()
    j.close()
    res["eager_blocked"] = {"t": info["t"], "seconds": round(dt, 6),
                            "glups": round(cells * sweeps / dt / 1e9, 1)}
    return res


def _closed_form(torch, n, modes):
    """Exact solution of the discrete Laplace problem for sine-mode faces on
    the GPU (float64): one separable term per face mode,
    sin(th_a a) sin(th_b b) sinh(beta d) / sinh(beta (n+1)) with
    cosh(beta) = 3 - cos(th_a) - cos(th_b) and d the distance from the
    opposite face; faces i0, i1, j0, j1, k0, k1, in-plane axes in (i, j, k)
    order (the first carries p)."""
    import math
    idx = torch.arange(n + 2, dtype=torch.float64, device="cuda")
    u = torch.zeros((n + 2,) * 3, dtype=torch.float64, device="cuda")
    # axis index in the (k, j, i) tensor: i -> 2, j -> 1, k -> 0
    specs = [(2, 1, 0, False), (2, 1, 0, True), (1, 2, 0, False), (1, 2, 0, True),
             (0, 2, 1, False), (0, 2, 1, True)]
    for face, (ax_n, ax_a, ax_b, far) in zip(modes, specs):
        for p, q, amp in face:
            ta, tb = math.pi * p / (n + 1), math.pi * q / (n + 1)
            beta = math.acosh(3.0 - math.cos(ta) - math.cos(tb))
            d = idx if far else (n + 1) - idx
            prof = torch.sinh(beta * d) / math.sinh(beta * (n + 1))
            shape = [1, 1, 1]
            va, vb = torch.sin(ta * idx), torch.sin(tb * idx)
            sa, sb, sn = list(shape), list(shape), list(shape)
            sa[ax_a] = n + 2
            sb[ax_b] = n + 2
            sn[ax_n] = n + 2
            u += amp * va.view(sa) * vb.view(sb) * prof.view(sn)
    return u


def _field_errors(torch, u, ref):
    """max |u - ref| and ||u - ref||_2 / ||ref||_2 over the interior."""
    d = (u[1:-1, 1:-1, 1:-1] - ref[1:-1, 1:-1, 1:-1])
    r = ref[1:-1, 1:-1, 1:-1]
    return {"max_abs": float(d.abs().max()),
            "rel_l2": float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(r))}


def bench_time_to_tol(torch, n, t, rel_tol=1e-8, check=1024, budget=0.0, layout="ab"):
    """Sweeps and seconds to ||r|| <= 1e-8 ||r0|| from the zero start with
    sine-mode faces (seed 3): FP64 blocked (t), FP32-refined (FP32 sweeps of
    the correction equation, FP64 residual and update) and plain FP64 single
    sweeps (t=1, A/B grids whatever `layout` the blocked forms use).

    Each solve runs in calls of 16 checks with r0 fixed, printing progress.
    With budget > 0 (seconds) a form stops when its budget is spent; the rest
    of the way to the tolerance is then extrapolated at the decay rate of the
    residual over the last 16 checks and at the form's measured GLUP/s (and
    labelled so).  The FP32-refined run stops at the FP64 run's sweep count,
    so that the two fields are compared at equal sweeps; the single-sweep
    form is timed on the first 8 checks only and extrapolated to the FP64
    count (its iterates are bitwise those of the blocked form).  The FP32 and
    FP64 fields are compared with each other and with the closed-form
    solution, next to the residual bound ||r||/(6 (1 - mu1)) on ||u - u*||."""
    import math
    import synth
    from paper_1006_3148_amd import Jacobi
    modes = synth.sine_face_modes(3)
    box = torch.from_numpy(synth.sine_face_box(n, n, n, seed=3)).cuda()
    mu1 = math.cos(math.pi / (n + 1))
    res = {"n": n, "rel_tol": rel_tol, "check_every": check, "layout": layout, "t": t,
           "budget_s": budget, "slowest_mode_factor": mu1}
    fields = {}
    r0 = None
    target_sweeps = None
    for name, kw in (("f64_blocked", dict(t=t)),
                     ("f32_refined", dict(t=t, dtype="f32_refined", inner_sweeps=check)),
                     ("f64_single_sweep", dict(t=1))):
        # plain Jacobi (the single-sweep baseline) keeps separate A/B grids
        j = Jacobi(box, layout="ab" if name == "f64_single_sweep" else layout, **kw)
        if r0 is None:
            r0, _ = j.residual()
            res["r0"] = r0
        torch.cuda.synchronize()
        a = time.perf_counter()
        total, hist = 0, []
        fin = r0
        stop = target_sweeps if name != "f64_blocked" else None
        if name == "f64_single_sweep":
            stop = 8 * check
        while fin > rel_tol * r0:
            chunk = 16 * check
            if stop is not None:
                chunk = min(chunk, stop - total)
                if chunk <= 0:
                    break
            done, fin = j.solve(rel_tol, chunk, check, r0)
            total += done
            hist.append((total, fin))
            el = time.perf_counter() - a
            print("time-to-tol n=%d %s: %d sweeps, ||r||/||r0|| = %.3e, %.1f s"
                  % (n, name, total, fin / r0, el), file=sys.stderr, flush=True)
            if budget > 0 and el > budget and name == "f64_blocked":
                break
        dt = time.perf_counter() - a
        rate = n ** 3 * total / dt / 1e9
        rec = {"sweeps": total, "seconds": round(dt, 3), "final_l2": fin,
               "final_rel": fin / r0, "glups": round(rate, 1), "converged": fin <= rel_tol * r0}
        if name == "f64_blocked":
            target_sweeps = total
            if not rec["converged"]:
                # The residual decays ever more slowly towards the slowest
                # mode's factor mu1 per sweep, so the rest of the way is
                # estimated at mu1 (at 512^3 this predicted the measured
                # remainder from ||r||/||r0|| ~ 1.5e-6 within 2 %); the local
                # decay of the last 16 checks gives a lower bound.
                more = math.log(rel_tol * r0 / fin) / math.log(mu1)
                more = int(math.ceil(more / check)) * check
                rec["extrapolated"] = {
                    "sweeps": total + more,
                    "seconds": round(dt + n ** 3 * more / (rate * 1e9), 1),
                    "how": "remaining sweeps at the slowest mode's decay mu1 per sweep, "
                           "at the measured GLUP/s"}
                if len(hist) >= 17:
                    (s0, f0), (s1, f1) = hist[-17], hist[-1]
                    rho = (f1 / f0) ** (1.0 / (s1 - s0))
                    low = int(math.ceil(math.log(rel_tol * r0 / f1) / math.log(rho) / check)) * check
                    rec["extrapolated"]["local_decay_per_sweep"] = rho
                    rec["extrapolated"]["sweeps_lower_bound"] = total + low
            fields["f64"] = j.current().clone()
        elif name == "f32_refined":
            fields["f32"] = j.current().clone()
            base = res["f64_blocked"]
            if not base["converged"]:
                ex = base["extrapolated"]
                rec["extrapolated"] = {
                    "sweeps": ex["sweeps"],
                    "seconds": round(dt + n ** 3 * (ex["sweeps"] - total) / (rate * 1e9), 1),
                    "how": "the FP64 run's extrapolated sweep count at this form's GLUP/s"}
        else:
            want = res["f64_blocked"].get("extrapolated", res["f64_blocked"])["sweeps"]
            rec = {"sweeps_timed": total, "seconds_timed": round(dt, 3),
                   "glups": round(rate, 1), "sweeps": want,
                   "seconds_extrapolated": round(n ** 3 * want / (rate * 1e9), 1),
                   "how": "timed on %d sweeps; the blocked form's sweep count at this rate "
                          "(same iterates bit for bit)" % total}
        j.close()
        res[name] = rec
    # errors: FP32-refined vs FP64 at equal sweeps, both vs the closed form
    ustar = _closed_form(torch, n, modes)
    bound = lambda l2: l2 / (6.0 * (1.0 - mu1))  # noqa: E731
    res["errors"] = {
        "f32_refined_vs_f64": _field_errors(torch, fields["f32"], fields["f64"]),
        "f64_vs_closed_form": _field_errors(torch, fields["f64"], ustar),
        "f32_refined_vs_closed_form": _field_errors(torch, fields["f32"], ustar),
        "residual_bound_l2_f64": bound(res["f64_blocked"]["final_l2"]),
        "residual_bound_l2_f32_refined": bound(res["f32_refined"]["final_l2"]),
        "closed_form_l2": float(torch.linalg.vector_norm(ustar[1:-1, 1:-1, 1:-1])),
        "note": "at equal sweep counts; the bound ||r||/(6(1-mu1)) holds for ||u - u*||_2",
    }
    d64 = torch.linalg.vector_norm((fields["f64"] - ustar)[1:-1, 1:-1, 1:-1])
    res["errors"]["f64_abs_l2_vs_closed_form"] = float(d64)
    del fields, ustar, box
    torch.cuda.empty_cache()
    return res


def bench_multigrid_tts(torch, n, rel_tol=1e-8):
    """Time to ||r|| <= 1e-8 ||r0|| with the multigrid-corrected refinement
    (one FP32 V(2,2)-cycle of weighted-Jacobi smoothing per FP64 outer step)
    on an n^3 interior, n = 2^k - 1, sine-mode faces (seed 3), zero start;
    checking after every outer step.  Reports the steps, the seconds, the
    error against the closed-form solution and the residual bound."""
    import math
    import synth
    from paper_1006_3148_amd import Jacobi
    box = torch.from_numpy(synth.sine_face_box(n, n, n, seed=3)).cuda()
    mu1 = math.cos(math.pi / (n + 1))
    j = Jacobi(box, dtype="f32_multigrid")
    r0, _ = j.residual()
    j.sweep(1)             # warm-up step (first launches of every kernel)
    j.close()
    j = Jacobi(box, dtype="f32_multigrid")
    torch.cuda.synchronize()
    a = time.perf_counter()
    steps, fin = j.solve(rel_tol, 200, 1, r0)
    dt = time.perf_counter() - a
    u = j.current().clone()
    j.close()
    ustar = _closed_form(torch, n, synth.sine_face_modes(3))
    err = _field_errors(torch, u, ustar)
    err["abs_l2"] = float(torch.linalg.vector_norm((u - ustar)[1:-1, 1:-1, 1:-1]))
    err["residual_bound_l2"] = fin / (6.0 * (1.0 - mu1))
    del u, ustar, box
    torch.cuda.empty_cache()
    return {"n": n, "rel_tol": rel_tol, "outer_steps": steps, "seconds": round(dt, 4),
            "final_rel": fin / r0, "r0": r0, "vs_closed_form": err,
            "method": "FP64 residual + FP32 V(2,2)-cycle, weighted Jacobi w=6/7 "
                      "(trip kernel, t=2 trips), full weighting, trilinear prolongation"}


def _kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for name in ("trip_kernel.h", "trip_device.h", "trip_configs.h", "internal.h",
                 "kernels_trip.hip", "trip_f64_m0.hip", "trip_f64_m1.hip"):
        with open(os.path.join(ROOT, "paper_1006_3148_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
