"""In-chip performance model of the trip kernel (the GPU counterpart of the
model of Sect. 2.3 of the paper).

The paper bounds temporally blocked Jacobi by two terms.  Eq. (4) is the
memory stream: t updates per 16 bytes of main-memory traffic.  The second is
the in-cache transfer rate of the update pipeline, which must satisfy
(t+1) B_j <= M_uc,max for t stages sharing one cache.  On MI355X the same
two sides are:

* HBM: one read and one write stream per trip, 16 N^3 bytes, plus ghost
  reads that miss L2 (tile halos, k-segment ghost planes);
* in-chip: VALU issue.  Every wave of a tile runs T stages on R rows per
  step.  Its instruction count per step is a*T*R + b*T + c: a per
  cell-stage (5 FP64 adds, 1 multiply, 4 DPP lane moves), b per stage, c per
  step.  Ghost zones make the computed cells exceed the owned ones by
  64*H / ((64-2T)(H-2T)), and that is the GPU's price for keeping every
  stage on one CU.  LDS carries 3T instructions (4T x 512 bytes) per wave
  per step, well below its bandwidth; in the shapes that issue a step's
  edge-row reads together right after the barrier (the kernel's register
  rule: T*R <= 24, 15, 10 for 8, 12, 16 waves) the compiler pairs some of the
  2T reads into one instruction, so T to 2T reads remain.

Prediction for a trip: t_valu = (VALU wave-instructions x 4 cycles) /
(1024 SIMDs x f x e) and t_hbm = bytes / BW, combined as
(t_valu^p + t_hbm^p)^(1/p).  The two throughputs overlap imperfectly, so
the combination is smooth rather than a plain max.  a, b, c come from
SQ_INSTS_VALU.  phi (the fraction of halo reads that miss L2), p and the
VALU efficiency e (one value for the shapes with batched edge-row reads, one
for the others, since the batching removes per-stage LDS stalls) are fitted
once to the measured t = 1..8 sweep at 512^3
(profiles/trip_sweep_512.json), with BW the bandwidth the stencil streams at
(fitted between 70 % and 100 % of the copy probe's 5.52 TB/s).

    python -m paper_1006_3148_amd.perfmodel [profiles/trip_sweep_512.json]

prints predicted vs measured VALU instructions, LDS instructions, HBM bytes,
kernel time and GLUP/s per t, and the t the model picks.  Host arithmetic
only: no GPU.
"""

from __future__ import annotations

import json
import math
import os
import sys

import numpy as np

CUS = 256
SIMDS = 4 * CUS
CLOCK_HZ = 2.4e9
LDS_BYTES_PER_CLK = 128
PF = 2  # steps per unrolled chunk of the trip kernel
E_MAX = 0.75  # highest measured VALU issue share of a SIMD (SQ counters, 512^3: 0.73 for
#                the 7-point t=5 kernel, 0.75 for the 27-point t=3 kernel)

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_DATA = os.path.join(os.path.dirname(HERE), "profiles", "trip_sweep_512.json")


def geometry(n: int, T: int, R: int, W: int, seg_len: int) -> dict:
    """Tiles, waves, executed steps and loaded planes of one trip over an n^3
    interior (the tiling of the trip kernel: 64 x R*W tiles overlapping by T
    cells, k segments of seg_len planes with T ghost planes each side)."""
    ox, h = 64 - 2 * T, R * W
    oy = h - 2 * T
    tx = math.ceil((n + 2) / ox)
    ty = math.ceil((n + 2) / oy)
    segs = math.ceil((n + 2) / seg_len)
    steps = planes = 0
    for s in range(segs):
        k0 = s * seg_len
        k1 = min(k0 + seg_len, n + 2)
        a = max(k0 - T, 0)
        b = min(k1 - 1 + T, n + 1)
        steps += PF * math.ceil((k1 - a + 2 * T - 1) / PF)
        planes += b - a + 1
    return {"tiles": tx * ty * segs, "waves": tx * ty * segs * W,
            "wave_steps": tx * ty * steps * W, "planes_loaded": planes,
            "tile_cells": 64 * h, "owned_cells": ox * oy,
            "redundancy": 64.0 * h / (ox * oy)}


def batched_reads(T: int, R: int, W: int) -> bool:
    """True for the shapes whose edge-row LDS reads of a step are issued
    together (the trip kernel's register rule for the 7-point update)."""
    return T * R <= (24 if W <= 8 else 15 if W <= 12 else 10)


def fit_valu(rows, n):
    """Least-squares a, b, c of VALU per wave per step = a T R + b T + c."""
    A, y = [], []
    for r in rows:
        g = geometry(n, r["t"], r["rows_per_wave"], r["waves"], r["seg_len"])
        A.append([r["t"] * r["rows_per_wave"], r["t"], 1.0])
        y.append(r["SQ_INSTS_VALU"] / g["wave_steps"])
    coef, *_ = np.linalg.lstsq(np.array(A), np.array(y), rcond=None)
    return [float(c) for c in coef]


def hbm_bytes(n, T, R, W, seg_len, phi):
    """Predicted HBM traffic of one trip: every owned cell written once; every
    loaded plane read once per tile column, of which the owned part and a
    fraction phi of the halo reach HBM."""
    g = geometry(n, T, R, W, seg_len)
    plane_owned = (n + 2) ** 2
    halo = g["tile_cells"] / g["owned_cells"] - 1.0
    reads = 8.0 * plane_owned * g["planes_loaded"] * (1.0 + phi * halo)
    writes = 8.0 * (n + 2) ** 3
    return reads + writes


def predict(n, T, R, W, seg_len, params):
    a, b, c = params["valu"]
    g = geometry(n, T, R, W, seg_len)
    valu = g["wave_steps"] * (a * T * R + b * T + c)
    batched = batched_reads(T, R, W)
    lds = g["wave_steps"] * 3 * T
    lds_min = g["wave_steps"] * (2 * T if batched else 3 * T)
    hb = hbm_bytes(n, T, R, W, seg_len, params["phi"])
    e = params["e_batched"] if batched else params["e"]
    t_valu = valu * 4 / (SIMDS * CLOCK_HZ * e)
    t_lds = g["wave_steps"] * 4 * T * 512 / (CUS * LDS_BYTES_PER_CLK * CLOCK_HZ)
    t_hbm = hb / params["bw"]
    p = params["p"]
    t = (t_valu ** p + t_hbm ** p) ** (1.0 / p)
    t = max(t, t_lds)
    return {"valu": valu, "lds": lds, "lds_min": lds_min, "batched": batched,
            "hbm_bytes": hb, "t_valu_us": t_valu * 1e6,
            "t_hbm_us": t_hbm * 1e6, "t_lds_us": t_lds * 1e6, "time_us": t * 1e6,
            "glups": n ** 3 * T / t / 1e9, "redundancy": g["redundancy"]}


def calibrate(doc, bw=5.52e12):
    """Fits a, b, c (VALU counts), phi (HBM counters), and e, p (kernel
    times) to a measured t sweep."""
    rows = doc["rows"]
    n = doc.get("n", 512)
    sf, sw = doc["probe_scale"]["FETCH_SIZE"], doc["probe_scale"]["WRITE_SIZE"]
    params = {"valu": fit_valu(rows, n), "bw": bw}
    # phi: least squares on the measured byte counts
    best = None
    for phi in np.linspace(0.0, 1.0, 101):
        err = sum((hbm_bytes(n, r["t"], r["rows_per_wave"], r["waves"], r["seg_len"], phi)
                   - 1024.0 * (sf * r["FETCH_SIZE_KiB"] + sw * r["WRITE_SIZE_KiB"])) ** 2
                  for r in rows)
        if best is None or err < best[0]:
            best = (err, phi)
    params["phi"] = float(best[1])
    # e, e_batched, p, BW: minimise the worst relative time error over a grid
    # (vectorised: the VALU and HBM terms of each row at e = BW-scale = 1)
    base = dict(params, e=1.0, e_batched=1.0, bw=1.0, p=1.0)
    tv, th, tl, bat, meas = [], [], [], [], []
    for r in rows:
        pr = predict(n, r["t"], r["rows_per_wave"], r["waves"], r["seg_len"], base)
        tv.append(pr["t_valu_us"]); th.append(pr["t_hbm_us"]); tl.append(pr["t_lds_us"])
        bat.append(pr["batched"]); meas.append(r["mean_us"])
    tv, th, tl, meas = map(np.array, (tv, th, tl, meas))
    bat = np.array(bat)
    # VALU efficiency cannot exceed the share of time a SIMD issues VALU
    # instructions (E_MAX, measured)
    E = np.linspace(0.5, E_MAX, 24)
    best = None
    for bw_fit in np.linspace(0.70 * bw, bw, 16):
        thb = th / bw_fit
        for p in np.linspace(1.0, 6.0, 26):
            for e in E:
                # rows without batched reads depend on e only
                t_o = np.maximum((((tv / e) ** p + thb ** p) ** (1.0 / p)), tl)
                err_o = np.max(np.abs(t_o[~bat] - meas[~bat]) / meas[~bat], initial=0.0)
                for eb in E:
                    t_b = np.maximum((((tv / eb) ** p + thb ** p) ** (1.0 / p)), tl)
                    err = max(err_o, np.max(np.abs(t_b[bat] - meas[bat]) / meas[bat],
                                            initial=0.0))
                    if best is None or err < best[0]:
                        best = (float(err), float(p), float(e), float(eb), float(bw_fit))
    params.update(p=best[1], e=best[2], e_batched=best[3], bw=best[4], max_time_err=best[0])
    return params


def report(path=DEFAULT_DATA):
    with open(path) as f:
        doc = json.load(f)
    n = doc.get("n", 512)
    params = calibrate(doc)
    sf, sw = doc["probe_scale"]["FETCH_SIZE"], doc["probe_scale"]["WRITE_SIZE"]
    out = []
    for r in doc["rows"]:
        pr = predict(n, r["t"], r["rows_per_wave"], r["waves"], r["seg_len"], params)
        meas_bytes = 1024.0 * (sf * r["FETCH_SIZE_KiB"] + sw * r["WRITE_SIZE_KiB"])
        out.append({"t": r["t"], "tile": "%dx%d" % (r["rows_per_wave"], r["waves"]),
                    "redundancy": round(pr["redundancy"], 3),
                    "valu_pred": pr["valu"], "valu_meas": r["SQ_INSTS_VALU"],
                    "lds_pred": pr["lds"], "lds_pred_min": pr["lds_min"],
                    "lds_meas": r["SQ_INSTS_LDS"], "batched": pr["batched"],
                    "hbm_pred": pr["hbm_bytes"], "hbm_meas": meas_bytes,
                    "t_valu_us": round(pr["t_valu_us"], 1), "t_hbm_us": round(pr["t_hbm_us"], 1),
                    "t_lds_us": round(pr["t_lds_us"], 1),
                    "time_pred_us": round(pr["time_us"], 1), "time_meas_us": r["mean_us"],
                    "glups_pred": round(pr["glups"], 1),
                    "glups_meas": round(n ** 3 * r["t"] / (r["mean_us"] * 1e-6) / 1e9, 1)})
    return params, out


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    params, rows = report(argv[0] if argv else DEFAULT_DATA)
    a, b, c = params["valu"]
    print("VALU per wave per step = %.2f T R %+.2f T %+.2f;  phi = %.2f, e = %.2f "
          "(batched edge-row reads: %.2f), p = %.2f, BW = %.2f TB/s; worst time error %.1f %%" % (
              a, b, c, params["phi"], params["e"], params["e_batched"], params["p"],
              params["bw"] / 1e12, 100 * params["max_time_err"]))
    print("| t | tile | redundancy | VALU pred/meas | LDS pred/meas | HBM GB pred/meas | "
          "t_valu us | t_hbm us | t_lds us | time pred/meas us | GLUP/s pred/meas |")
    print("|---|---|---|---|---|---|---|---|---|---|---|")
    for r in rows:
        print("| %d | %s | %.2f | %.3g / %.3g | %.3g / %.3g | %.2f / %.2f | %.0f | %.0f | %.0f | "
              "%.0f / %.0f | %.0f / %.0f |" % (
                  r["t"], r["tile"], r["redundancy"], r["valu_pred"], r["valu_meas"],
                  r["lds_pred"], r["lds_meas"], r["hbm_pred"] / 1e9, r["hbm_meas"] / 1e9,
                  r["t_valu_us"], r["t_hbm_us"], r["t_lds_us"], r["time_pred_us"],
                  r["time_meas_us"], r["glups_pred"], r["glups_meas"]))
    best = max(rows, key=lambda r: r["glups_pred"])
    print("model's best t: %d (measured best: %d)" % (
        best["t"], max(rows, key=lambda r: r["glups_meas"])["t"]))


if __name__ == "__main__":
    main()
