"""Learned initial guess: training data from the solver, training, evaluation.

Pipeline (every numerical step runs in libjacobi's kernels; torch only holds
device memory and does the data plumbing noted below):

1. Basis solutions.  The discrete Laplace problem is linear in its boundary
   data, and every synthetic boundary is a sum of sine modes
   sin(pi p a/(n+1)) sin(pi q b/(n+1)) on the six faces (p, q in 1..pmax).
   The solver (batched, autotuned, FP64, temporally blocked) solves the
   6*pmax^2 unit-mode problems to ||r|| <= tol * ||r0||.
2. Training targets.  The converged field of a sample is the same linear
   combination of the basis solutions as its boundary is of the unit modes
   (the combination is a torch axpy: data plumbing, not the solver).
3. Training.  The U-Net (jacobi_guess.h) is trained with its own MFMA
   forward/backward kernels and Adam on the GPU, MSE to the targets.
4. Evaluation.  Held-out problems are solved to 1e-8 * ||r0(zero start)||
   from (a) the zero start, (b) the network's guess, (c) a non-learned blend
   of the face values; the sweep counts and times are compared.
"""

from __future__ import annotations

import math
import time

import numpy as np
import torch

import synth

from .batch import JacobiBatch
from .guess import GuessNet, init_params


def basis_index(face: int, p: int, q: int, pmax: int) -> int:
    return (face * pmax + (p - 1)) * pmax + (q - 1)


def solve_basis(n: int, pmax: int = 4, rel_tol: float = 1e-8,
                check_every: int = 512, max_sweeps: int = 400000, t: int = 0):
    """FP32 interiors [6*pmax^2, n, n, n] of the unit-mode solutions."""
    boxes = [synth.unit_face_mode_box(n, f, p, q)
             for f in range(6) for p in range(1, pmax + 1) for q in range(1, pmax + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = JacobiBatch(boxes, t=t)
    sweeps, fin = b.solve(rel_tol, max_sweeps, check_every)
    b.sync()
    dt = time.perf_counter() - t0
    info = b.info()
    U = torch.empty((len(boxes), n, n, n), dtype=torch.float32, device="cuda")
    for i in range(len(boxes)):
        U[i].copy_(b.current(i)[1:-1, 1:-1, 1:-1])
    b.close()
    del boxes
    torch.cuda.empty_cache()
    cells = len(U) * n ** 3
    return U, {"problems": len(U), "sweeps_max": int(sweeps.max()),
               "sweeps_mean": float(sweeps.mean()), "converged": bool((sweeps >= 0).all()),
               "seconds": dt, "glups": cells * float(info["sweeps"]) / dt / 1e9,
               "t": info["t"], "tile_rows": info["tile_rows"]}


def target_from_modes(U: torch.Tensor, modes, pmax: int, out: torch.Tensor):
    """out = sum over faces and modes of a * U[basis(face, p, q)]."""
    out.zero_()
    for f, face in enumerate(modes):
        for p, q, a in face:
            out.add_(U[basis_index(f, p, q, pmax)], alpha=float(a))
    return out


def face_box(n: int, seed: int, box: torch.Tensor):
    """Write the faces of sine_face_box(n, n, n, seed) into a device box."""
    faces, modes = synth.sine_faces(n, seed)
    ft = torch.from_numpy(faces).to(box.device)
    box[:, :, 0] = ft[0]
    box[:, :, -1] = ft[1]
    box[:, 0, :] = ft[2]
    box[:, -1, :] = ft[3]
    box[0, :, :] = ft[4]
    box[-1, :, :] = ft[5]
    return modes


def train(net: GuessNet, U: torch.Tensor, n: int, pmax: int, seeds, epochs: int,
          lr: float, accum: int = 1, val_seeds=(), log=None):
    box = torch.zeros((n + 2,) * 3, dtype=torch.float64, device="cuda")
    tgt = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
    steps = epochs * math.ceil(len(seeds) / accum)
    rng = np.random.default_rng(0)
    history = []
    step = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = rng.permutation(len(seeds))
        tot, cnt = 0.0, 0
        net.zero_grads()
        for pos, idx in enumerate(order):
            modes = face_box(n, seeds[idx], box)
            target_from_modes(U, modes, pmax, tgt)
            net.forward(box)
            want = (pos + 1) % 16 == 0
            loss = net.backward(tgt, want_loss=want)
            if want:
                tot += loss
                cnt += 1
            if (pos + 1) % accum == 0 or pos == len(order) - 1:
                frac = step / max(steps - 1, 1)
                cur = lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * frac)))
                net.adam(cur)
                net.zero_grads()
                step += 1
        history.append(tot / max(cnt, 1))
        if log:
            log("epoch %d train loss %.4e (%.1f s)" % (ep, history[-1],
                                                        time.perf_counter() - t0))
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    val = []
    for s in val_seeds:
        modes = face_box(n, s, box)
        target_from_modes(U, modes, pmax, tgt)
        net.forward(box)
        out = net.out.view(n, n, n)
        val.append(float(((out - tgt) ** 2).mean() / (tgt ** 2).mean()))
    return {"epochs": epochs, "samples": len(seeds), "train_loss": history,
            "val_rel_mse": float(np.mean(val)) if val else None, "seconds": seconds,
            "steps": step}


def evaluate(net: GuessNet, n: int, seeds, rel_tol: float = 1e-8,
             check_every: int = 256, max_sweeps: int = 400000, t: int = 0,
             single: int = 4):
    """Sweeps (batched solve) and single-problem wall times to rel_tol * r0."""
    from .solver import Jacobi
    boxes = [synth.sine_face_box(n, n, n, s) for s in seeds]
    res = {}
    # zero start
    bz = JacobiBatch(boxes, t=t)
    r0, _ = bz.residual()
    t0 = time.perf_counter()
    sz, _ = bz.solve(rel_tol, max_sweeps, check_every, r0=r0)
    res["zero_batch_seconds"] = time.perf_counter() - t0
    tz = bz.info()["t"]
    bz.close()
    # learned start: network output written into each box's interior
    guesses = []
    t0 = time.perf_counter()
    for b in boxes:
        bt = torch.from_numpy(b).cuda()
        net.forward(bt)
        net.write_guess(bt)
        guesses.append(bt.cpu().numpy())
    torch.cuda.synchronize()
    res["inference_seconds_total"] = time.perf_counter() - t0
    bl = JacobiBatch(guesses, t=tz)
    t0 = time.perf_counter()
    sl, _ = bl.solve(rel_tol, max_sweeps, check_every, r0=r0)
    res["learned_batch_seconds"] = time.perf_counter() - t0
    bl.close()
    # blended faces
    blends = []
    for b in boxes:
        bt = torch.from_numpy(b).cuda()
        net.write_blend(bt)
        blends.append(bt.cpu().numpy())
    bb = JacobiBatch(blends, t=tz)
    sb, _ = bb.solve(rel_tol, max_sweeps, check_every, r0=r0)
    bb.close()
    res.update({
        "problems": len(seeds), "check_every": check_every, "rel_tol": rel_tol,
        "sweeps_zero_mean": float(np.mean(sz)), "sweeps_learned_mean": float(np.mean(sl)),
        "sweeps_blend_mean": float(np.mean(sb)),
        "sweeps_zero": sz.tolist(), "sweeps_learned": sl.tolist(), "sweeps_blend": sb.tolist(),
        "all_converged": bool((sz >= 0).all() and (sl >= 0).all() and (sb >= 0).all()),
    })
    d = (sz - sl).astype(np.float64)
    res["sweeps_saved_mean"] = float(d.mean())
    res["sweeps_saved_ci95"] = float(1.96 * d.std(ddof=1) / math.sqrt(len(d))) if len(d) > 1 else None
    res["sweeps_saved_frac"] = float(d.mean() / np.mean(sz))
    # paired against the non-learned blend the network corrects
    e = (sb - sl).astype(np.float64)
    res["sweeps_saved_vs_blend_mean"] = float(e.mean())
    res["sweeps_saved_vs_blend_ci95"] = (float(1.96 * e.std(ddof=1) / math.sqrt(len(e)))
                                         if len(e) > 1 else None)
    res["problems_better_than_blend"] = int((e > 0).sum())
    # single-problem wall time: zero start vs (inference + solve)
    tz_s, tl_s = [], []
    for q in range(min(single, len(seeds))):
        j = Jacobi(boxes[q], t=tz)
        torch.cuda.synchronize()
        a = time.perf_counter()
        j.solve(rel_tol, max_sweeps, check_every, r0=float(r0[q]))
        tz_s.append(time.perf_counter() - a)
        j.close()
        bt = torch.from_numpy(boxes[q]).cuda()
        torch.cuda.synchronize()
        a = time.perf_counter()
        net.forward(bt)
        net.write_guess(bt)
        torch.cuda.synchronize()
        inf = time.perf_counter() - a
        j = Jacobi(bt, t=tz)
        a = time.perf_counter()
        j.solve(rel_tol, max_sweeps, check_every, r0=float(r0[q]))
        tl_s.append(inf + time.perf_counter() - a)
        j.close()
    res["single_zero_seconds"] = tz_s
    res["single_learned_seconds"] = tl_s
    return res


def time_layers(n: int, reps: int = 10):
    """One stride-1 convolution at n^3 through the single-layer entry points
    (forward, data gradient, weight gradient): ms per call (HIP events) and
    TFLOP/s at 2 x 27 x 16 x 16 flops per voxel, against the 2.5 PFLOP/s
    dense BF16 MFMA peak."""
    from . import guess
    g = torch.Generator(device="cuda").manual_seed(0)
    xb = torch.randn((n, n, n, 16), device="cuda", generator=g).relu().to(torch.bfloat16)
    wb = (0.1 * torch.randn((27, 16, 16), device="cuda", generator=g)).to(torch.bfloat16)
    x, w = xb.view(torch.int16), wb.view(torch.int16)
    b = torch.zeros(16, device="cuda")
    dy = torch.randn((n, n, n, 16), device="cuda", generator=g)
    flop = 2.0 * 27 * 16 * 16 * n ** 3
    out = {}
    for name, fn in (("forward", lambda: guess.conv3_forward(x, w, b)),
                     ("data_grad", lambda: guess.conv3_backward_data(dy, w)),
                     ("weight_grad", lambda: guess.conv3_backward_weight(x, dy))):
        fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(reps):
            fn()
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / reps
        out[name] = {"ms": round(ms, 4), "tflops": round(flop / (ms * 1e-3) / 1e12, 1),
                     "frac_bf16_peak": round(flop / (ms * 1e-3) / 2.5e15, 4)}
    return out


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--pmax", type=int, default=4)
    ap.add_argument("--train", type=int, default=3840)
    ap.add_argument("--val", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=2)
    ap.add_argument("--accum", type=int, default=4)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--eval", type=int, default=64)
    ap.add_argument("--check-every", type=int, default=256)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--low-weight", type=float, default=0.0,
                    help="weight of the low-mode term of the loss (0: plain MSE)")
    ap.add_argument("--time-only", action="store_true")
    a = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)  # noqa: E731
    torch.cuda.set_device(0)
    theta = init_params(a.levels, a.seed)
    net = GuessNet(a.n, a.levels, theta)
    box = torch.from_numpy(synth.sine_face_box(a.n, a.n, a.n, 1)).cuda()
    tgt = torch.zeros((a.n,) * 3, dtype=torch.float32, device="cuda")
    for _ in range(2):
        net.forward(box)
        net.backward(tgt, want_loss=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        net.forward(box)
    torch.cuda.synchronize()
    fwd = (time.perf_counter() - t0) / 5
    t0 = time.perf_counter()
    for _ in range(5):
        net.forward(box)
        net.backward(tgt, want_loss=False)
    torch.cuda.synchronize()
    step = (time.perf_counter() - t0) / 5
    report = {"n": a.n, "levels": a.levels, "forward_ms": fwd * 1e3,
              "train_step_ms": step * 1e3, "layers": time_layers(a.n)}
    log(json.dumps(report))
    if a.time_only:
        return report
    U, basis = solve_basis(a.n, a.pmax, check_every=512)
    log("basis: " + json.dumps(basis))
    net.set_low_mode_weight(a.low_weight)
    report["low_weight"] = a.low_weight
    seeds = list(range(1000, 1000 + a.train))
    val = list(range(1000 + a.train, 1000 + a.train + a.val))
    tr = train(net, U, a.n, a.pmax, seeds, a.epochs, a.lr, a.accum, val, log)
    log("train: " + json.dumps({k: v for k, v in tr.items()}))
    del U
    torch.cuda.empty_cache()
    ev = evaluate(net, a.n, list(range(900000, 900000 + a.eval)),
                  check_every=a.check_every)
    report.update({"basis": basis, "train": tr, "eval": ev})
    log("RESULT " + json.dumps(report))
    return report


if __name__ == "__main__":
    main()
