"""Pins of the FP64 network oracle (oracle/conv.py) to library routines and to
finite differences -- no GPU."""

import numpy as np
import pytest
import torch

from oracle import conv as cv


def _torch_w(w):
    # (27, Cout, Cin) -> (Cout, Cin, 3, 3, 3), tap t = (dz+1)*9 + (dy+1)*3 + (dx+1)
    return torch.from_numpy(w.reshape(3, 3, 3, w.shape[1], w.shape[2]).transpose(3, 4, 0, 1, 2).copy())


@pytest.mark.parametrize("stride,shape", [(1, (6, 5, 7)), (2, (8, 6, 4))])
def test_conv3_matches_torch_conv3d(stride, shape):
    rng = np.random.default_rng(1)
    x = rng.standard_normal(shape + (16,))
    w = rng.standard_normal((27, 16, 16))
    b = rng.standard_normal(16)
    y = cv.conv3(x, w, b, stride)
    xt = torch.from_numpy(x.transpose(3, 0, 1, 2)[None].copy())
    yt = torch.nn.functional.conv3d(xt, _torch_w(w), torch.from_numpy(b), stride=stride, padding=1)
    assert np.allclose(y, yt[0].numpy().transpose(1, 2, 3, 0), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("stride", [1, 2])
def test_conv3_backward_matches_autograd(stride):
    rng = np.random.default_rng(2)
    x = rng.standard_normal((6, 4, 8, 16))
    w = rng.standard_normal((27, 16, 16))
    b = rng.standard_normal(16)
    dy = rng.standard_normal((6 // stride, 4 // stride, 8 // stride, 16))
    dx, dw, db = cv.conv3_backward(x, w, dy, stride)
    xt = torch.from_numpy(x.transpose(3, 0, 1, 2)[None].copy()).requires_grad_()
    wt = _torch_w(w).requires_grad_()
    bt = torch.from_numpy(b).requires_grad_()
    yt = torch.nn.functional.conv3d(xt, wt, bt, stride=stride, padding=1)
    yt.backward(torch.from_numpy(dy.transpose(3, 0, 1, 2)[None].copy()))
    assert np.allclose(dx, xt.grad[0].numpy().transpose(1, 2, 3, 0), rtol=1e-11, atol=1e-11)
    gw = wt.grad.numpy().transpose(2, 3, 4, 0, 1).reshape(27, 16, 16)
    assert np.allclose(dw, gw, rtol=1e-11, atol=1e-11)
    assert np.allclose(db, bt.grad.numpy(), rtol=1e-12)


def test_up2_adjoint():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 3, 4, 16))
    y = rng.standard_normal((4, 6, 8, 16))
    assert np.isclose(np.sum(cv.up2(x) * y), np.sum(x * cv.up2_backward(y)))


def test_lift_channels():
    rng = np.random.default_rng(4)
    box = rng.random((6, 5, 7))
    x = cv.lift(box)
    assert x.shape == (4, 3, 5, 16)
    k, j, i = 2, 1, 3  # interior (k+1, j+1, i+1)
    assert x[k, j, i, 0] == box[k + 1, j + 1, 0]
    assert x[k, j, i, 1] == box[k + 1, j + 1, -1]
    assert x[k, j, i, 2] == box[k + 1, 0, i + 1]
    assert x[k, j, i, 3] == box[k + 1, -1, i + 1]
    assert x[k, j, i, 4] == box[0, j + 1, i + 1]
    assert x[k, j, i, 5] == box[-1, j + 1, i + 1]
    assert np.isclose(x[k, j, i, 6], (i + 1) / 6 - 0.5)
    assert np.all(x[..., 10:] == 0)
    # blend: a box whose six faces are constant c gives c everywhere
    cbox = np.full((6, 5, 7), 2.5)
    assert np.allclose(cv.lift(cbox)[..., 9], 2.5)
    # and a face only on i=0 weighs by 1/i against the 6 inverse distances
    fbox = np.zeros((6, 5, 7))
    fbox[1:-1, 1:-1, 0] = 1.0
    b = cv.blend(fbox)
    i, j, kk = 2, 1, 3
    ws = [1 / (i + 1), 1 / (6 - (i + 1)), 1 / (j + 1), 1 / (4 - (j + 1)), 1 / (kk + 1), 1 / (5 - (kk + 1))]
    assert np.isclose(b[kk, j, i], ws[0] / sum(ws))


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(5)
    v = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.0078125, 1.01171875])])
    ref = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cv.bf16_round(v), ref)


def test_network_gradient_matches_finite_differences():
    levels, n = 3, 8
    rng = np.random.default_rng(6)
    box = rng.random((n + 2, n + 2, n + 2))
    target = rng.random((n, n, n))
    theta = cv.init_params(levels, seed=7)
    theta = theta + 0.05 * rng.standard_normal(theta.size)  # non-zero biases
    loss, g, _ = cv.loss_and_grad(theta, box, target, levels, round_bf16=False)
    idx = rng.choice(theta.size, 40, replace=False)
    idx = np.concatenate([idx, [theta.size - 1, theta.size - 2]])
    eps = 1e-6
    for q in idx:
        tp = theta.copy(); tp[q] += eps
        tm = theta.copy(); tm[q] -= eps
        lp = cv.loss_and_grad(tp, box, target, levels, round_bf16=False)[0]
        lm = cv.loss_and_grad(tm, box, target, levels, round_bf16=False)[0]
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[q]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (q, fd, g[q])


def test_adam_matches_torch():
    rng = np.random.default_rng(8)
    theta = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    pt = torch.from_numpy(theta.copy()).requires_grad_()
    opt = torch.optim.Adam([pt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    th = theta.copy()
    for step in range(1, 6):
        g = rng.standard_normal(50)
        th, m, v = cv.adam_step(th, g, m, v, step, 1e-3)
        pt.grad = torch.from_numpy(g.copy())
        opt.step()
    assert np.allclose(th, pt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_low_mode_coefficients_closed_form():
    """The discrete sines are orthogonal: for e = sum_m b_m v_m over the eight
    modes, a_m = b_m * prod over axes of (n+1)/(2n)."""
    shape = (7, 5, 6)
    rng = np.random.default_rng(11)
    b = rng.standard_normal(len(cv.LOW_MODES))
    e = sum(bm * cv.low_mode(shape, m) for bm, m in zip(b, cv.LOW_MODES))
    scale = np.prod([(d + 1) / (2.0 * d) for d in shape])
    assert np.allclose(cv.low_mode_coeffs(e), b * scale, rtol=1e-12, atol=1e-14)
    # a higher mode has no projection on them
    hi = cv.low_mode(shape, (3, 1, 2))
    assert np.allclose(cv.low_mode_coeffs(hi), 0.0, atol=1e-14)


def test_low_mode_loss_gradient_matches_finite_differences():
    levels, n = 2, 8
    rng = np.random.default_rng(12)
    box = rng.random((n + 2, n + 2, n + 2))
    target = rng.random((n, n, n))
    theta = cv.init_params(levels, seed=13) + 0.05 * rng.standard_normal(
        cv.init_params(levels, seed=13).size)
    wlow = 50.0
    loss, g, out = cv.loss_and_grad(theta, box, target, levels, round_bf16=False,
                                    low_weight=wlow)
    a = cv.low_mode_coeffs(out - target)
    assert abs(loss - (np.mean((out - target) ** 2) + wlow * np.sum(a * a))) <= 1e-12 * loss
    idx = np.concatenate([rng.choice(theta.size, 30, replace=False),
                          [theta.size - 1, theta.size - 2]])
    eps = 1e-6
    for q in idx:
        tp = theta.copy(); tp[q] += eps
        tm = theta.copy(); tm[q] -= eps
        lp = cv.loss_and_grad(tp, box, target, levels, round_bf16=False, low_weight=wlow)[0]
        lm = cv.loss_and_grad(tm, box, target, levels, round_bf16=False, low_weight=wlow)[0]
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[q]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (q, fd, g[q])


@pytest.mark.parametrize("stride", [1, 2])
def test_conv3_backward_rounds_only_the_product_operand(stride):
    """With the BF16 rounding of the upstream gradient: an already
    BF16-representable dy gives exactly the unrounded result, db never sees
    the rounding, and dx/dw are torch's conv3d gradients for rnd(dy)."""
    rng = np.random.default_rng(5)
    x = cv.bf16_round(rng.standard_normal((6, 4, 8, 16)))
    w = cv.bf16_round(rng.standard_normal((27, 16, 16)))
    dy = rng.standard_normal((6 // stride, 4 // stride, 8 // stride, 16))
    dyb = cv.bf16_round(dy)
    a = cv.conv3_backward(x, w, dyb, stride, rnd=cv.bf16_round)
    b = cv.conv3_backward(x, w, dyb, stride)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    dx, dw, db = cv.conv3_backward(x, w, dy, stride, rnd=cv.bf16_round)
    assert np.array_equal(db, dy.sum(axis=(0, 1, 2)))
    assert not np.array_equal(dw, cv.conv3_backward(x, w, dy, stride)[1])
    xt = torch.from_numpy(x.transpose(3, 0, 1, 2)[None].copy()).requires_grad_()
    wt = _torch_w(w).requires_grad_()
    yt = torch.nn.functional.conv3d(xt, wt, None, stride=stride, padding=1)
    yt.backward(torch.from_numpy(dyb.transpose(3, 0, 1, 2)[None].copy()))
    assert np.allclose(dx, xt.grad[0].numpy().transpose(1, 2, 3, 0), rtol=1e-11, atol=1e-11)
    gw = wt.grad.numpy().transpose(2, 3, 4, 0, 1).reshape(27, 16, 16)
    assert np.allclose(dw, gw, rtol=1e-11, atol=1e-11)
