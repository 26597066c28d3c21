"""GPU parity of the learned-guess network kernels against the FP64 oracle on
the same BF16-rounded operands, and a training sanity check."""

import numpy as np
import pytest

import synth
from oracle import conv as cv
from tests import closed_form as cf

pytestmark = pytest.mark.gpu


def _theta(levels, seed):
    rng = np.random.default_rng(seed)
    th = cv.init_params(levels, seed)
    th = th + 0.02 * rng.standard_normal(th.size)   # non-zero biases
    return th.astype(np.float32).astype(np.float64)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("n,levels", [(16, 3), (32, 4), (24, 2)])
def test_forward_and_gradient_match_oracle(n, levels):
    import torch
    from paper_1006_3148_amd import GuessNet
    print("case guess n=%d levels=%d" % (n, levels), flush=True)
    theta = _theta(levels, 3)
    box = synth.sine_face_box(n, n, n, seed=5)
    rng = np.random.default_rng(9)
    target = rng.standard_normal((n, n, n)).astype(np.float32)
    net = GuessNet(n, levels, theta)
    bt = torch.from_numpy(box).cuda()
    out = net.forward(bt).cpu().numpy().astype(np.float64)
    ref, _ = cv.forward(theta, box, levels, round_bf16=True)
    assert _rel(out, ref) < 1e-2, _rel(out, ref)
    net.zero_grads()
    loss = net.backward(torch.from_numpy(target).cuda())
    g = net.grads.cpu().numpy().astype(np.float64)
    lref, gref, _ = cv.loss_and_grad(theta, box, target.astype(np.float64), levels,
                                     round_bf16=True)
    assert abs(loss - lref) <= 1e-3 * abs(lref)
    assert _rel(g, gref) < 3e-2, _rel(g, gref)
    # every layer's gradient points the same way
    o = 0
    for name, shp in cv.param_shapes(levels):
        k = int(np.prod(shp))
        a, b = g[o:o + k], gref[o:o + k]
        o += k
        if np.linalg.norm(b) > 1e-12:
            cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
            assert cos > 0.995, (name, cos)
    net.close()


@pytest.mark.parametrize("weight", [0.0, 40.0])
def test_low_mode_loss_matches_oracle(weight):
    """Loss with the low-mode term (and plain MSE again after it is switched
    back off), on a target with a large smooth component."""
    import torch
    from paper_1006_3148_amd import GuessNet
    n, levels = 16, 3
    print("case guess low-mode weight=%g" % weight, flush=True)
    theta = _theta(levels, 4)
    box = synth.sine_face_box(n, n, n, seed=6)
    rng = np.random.default_rng(10)
    target = (0.3 * rng.standard_normal((n, n, n))
              + 2.0 * cv.low_mode((n, n, n), (1, 1, 1))
              - 1.0 * cv.low_mode((n, n, n), (2, 1, 2))).astype(np.float32)
    net = GuessNet(n, levels, theta)
    bt = torch.from_numpy(box).cuda()
    tt = torch.from_numpy(target).cuda()
    for w in (weight, 0.0):
        net.set_low_mode_weight(w)
        net.forward(bt)
        net.zero_grads()
        loss = net.backward(tt)
        g = net.grads.cpu().numpy().astype(np.float64)
        lref, gref, _ = cv.loss_and_grad(theta, box, target.astype(np.float64), levels,
                                         round_bf16=True, low_weight=w)
        assert abs(loss - lref) <= 2e-3 * abs(lref), (w, loss, lref)
        assert _rel(g, gref) < 3e-2, (w, _rel(g, gref))
    net.close()


def test_adam_step_matches_oracle():
    import torch
    from paper_1006_3148_amd import GuessNet
    levels, n = 2, 8
    theta = _theta(levels, 4)
    net = GuessNet(n, levels, theta)
    rng = np.random.default_rng(11)
    m = np.zeros(theta.size)
    v = np.zeros(theta.size)
    th = theta.copy()
    for step in range(1, 4):
        g = rng.standard_normal(theta.size).astype(np.float32)
        net.grads.copy_(torch.from_numpy(g))
        net.adam(1e-3)
        th, m, v = cv.adam_step(th, g.astype(np.float64), m, v, step, 1e-3)
    got = net.params.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - th)) < 1e-6


def test_training_reduces_loss_on_closed_form_targets():
    import torch
    from paper_1006_3148_amd import GuessNet
    n, levels = 16, 3
    print("case guess training n=16", flush=True)
    boxes, targets = [], []
    for s in range(4):
        modes = synth.sine_face_modes(100 + s, modes_per_face=8, pmax=4)
        box = synth.sine_face_box(n, n, n, 100 + s)
        u = cf.harmonic_from_sine_faces(n, n, n, modes)
        boxes.append(torch.from_numpy(box).cuda())
        targets.append(torch.from_numpy(u[1:-1, 1:-1, 1:-1].astype(np.float32)).cuda())
    net = GuessNet(n, levels, cv.init_params(levels, 1))
    first = None
    for it in range(60):
        net.zero_grads()
        tot = 0.0
        for b, t in zip(boxes, targets):
            net.forward(b)
            tot += net.backward(t)
        if first is None:
            first = tot
        net.adam(3e-3)
    assert tot < 0.3 * first, (first, tot)
