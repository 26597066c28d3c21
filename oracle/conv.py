"""FP64 reference of the learned-initial-guess network -- TEST ORACLE.

The learned initial guess is not in the paper: it supplies a starting field for
the Jacobi method of Sect. 1.1.  Architecture (the reading taken here):

* input lift: for interior cell (i,j,k) of an N^3 grid, 16 channels =
  the six face values at its projections onto the boundary faces
  (i=0, i=N+1, j=0, j=N+1, k=0, k=N+1, in that order), the three
  coordinates (i/(N+1) - 1/2, j/(N+1) - 1/2, k/(N+1) - 1/2), the face blend
  b (below), and 6 zeros;
* face blend b(i,j,k) = sum_f g_f w_f / sum_f w_f over the six face values
  g_f at the cell's projections with w_f = 1 / (distance to face f), i.e.
  1/i, 1/(N+1-i), 1/j, ...; the network predicts a correction to it:
  out = b + head(...);
* U-Net with L levels (N, N/2, ..., N/2^(L-1)) and C = 16 channels:
  encoder level l: h = relu(conv(x)); h = relu(conv(h)); skip_l = h;
  if l < L-1: x = relu(conv_stride2(h));
  decoder level l = L-2 .. 0: x = up2(x) + skip_l; x = relu(conv(x));
  x = relu(conv(x));
  head: out = sum_c w_c x_c + b (1x1x1, 16 -> 1);
* every conv is 3x3x3, zero padding 1, stride 1 (or 2 for the down convs),
  with a per-output-channel bias; up2 is nearest-neighbour upsampling by 2;
* loss = mean over the interior of (out - target)^2.

The blend term (not in the first version of this network) was added because
a plain U-Net trained for two epochs left a smooth interior error that the
Jacobi sweeps remove slowest; predicting the correction to the blend keeps
the blend's low-frequency accuracy.

Layout: activations (D, H, W, C) with the channel index last; conv weights
(27, Cout, Cin) with tap index t = (dz+1)*9 + (dy+1)*3 + (dx+1).

Numerics of the GPU network (BF16 weights and activations, FP32 accumulation)
are reproduced by rounding operands with ``bf16_round`` (round to nearest
even) before calling these FP64 functions.  In the backward pass the FP32
upstream gradient of a convolution enters its two matrix products (data and
weight gradient) rounded to BF16, while the bias gradient sums it unrounded.
"""

from __future__ import annotations

import numpy as np

C = 16


def bf16_round(x):
    """Round float values to bfloat16 (round to nearest, ties to even)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32)
    nan = np.isnan(f)
    if np.any(nan):
        out = out.copy()
        out[nan] = np.nan
    return out.astype(np.float64)


def lift(box):
    """Input volume (N, N, N, 16) from a (N+2)^3 box holding the faces."""
    nz2, ny2, nx2 = box.shape
    nz, ny, nx = nz2 - 2, ny2 - 2, nx2 - 2
    x = np.zeros((nz, ny, nx, C))
    x[..., 0] = box[1:-1, 1:-1, 0][:, :, None]
    x[..., 1] = box[1:-1, 1:-1, -1][:, :, None]
    x[..., 2] = box[1:-1, 0, 1:-1][:, None, :]
    x[..., 3] = box[1:-1, -1, 1:-1][:, None, :]
    x[..., 4] = box[0, 1:-1, 1:-1][None, :, :]
    x[..., 5] = box[-1, 1:-1, 1:-1][None, :, :]
    i = np.arange(1, nx + 1) / (nx + 1) - 0.5
    j = np.arange(1, ny + 1) / (ny + 1) - 0.5
    k = np.arange(1, nz + 1) / (nz + 1) - 0.5
    x[..., 6] = i[None, None, :]
    x[..., 7] = j[None, :, None]
    x[..., 8] = k[:, None, None]
    x[..., 9] = blend(box)
    return x


def blend(box):
    """Inverse-distance blend of the six face values at each cell's projections."""
    nz2, ny2, nx2 = box.shape
    nz, ny, nx = nz2 - 2, ny2 - 2, nx2 - 2
    ci = np.arange(1, nx + 1, dtype=np.float64)[None, None, :]
    cj = np.arange(1, ny + 1, dtype=np.float64)[None, :, None]
    ck = np.arange(1, nz + 1, dtype=np.float64)[:, None, None]
    terms = [
        (box[1:-1, 1:-1, 0][:, :, None], 1.0 / ci),
        (box[1:-1, 1:-1, -1][:, :, None], 1.0 / (nx + 1 - ci)),
        (box[1:-1, 0, 1:-1][:, None, :], 1.0 / cj),
        (box[1:-1, -1, 1:-1][:, None, :], 1.0 / (ny + 1 - cj)),
        (box[0, 1:-1, 1:-1][None, :, :], 1.0 / ck),
        (box[-1, 1:-1, 1:-1][None, :, :], 1.0 / (nz + 1 - ck)),
    ]
    num = sum(g * w for g, w in terms)
    den = sum(np.broadcast_to(w, num.shape) for _, w in terms)
    return num / den


def taps():
    return [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1)
            for dx in (-1, 0, 1)]


def conv3(x, w, b, stride=1):
    """y[o] = b + sum_t sum_ci w[t, :, ci] x[stride*o + d_t, ci] (zero pad)."""
    d, h, wd, cin = x.shape
    od, oh, ow = d // stride, h // stride, wd // stride
    xp = np.zeros((d + 2, h + 2, wd + 2, cin))
    xp[1:-1, 1:-1, 1:-1] = x
    y = np.zeros((od, oh, ow, w.shape[1])) + b
    for t, (dz, dy, dx) in enumerate(taps()):
        src = xp[1 + dz: 1 + dz + stride * od: stride,
                 1 + dy: 1 + dy + stride * oh: stride,
                 1 + dx: 1 + dx + stride * ow: stride]
        y = y + src @ w[t].T
    return y


def conv3_backward(x, w, dy, stride=1, rnd=None):
    """Gradients (dx, dw, db) of conv3 for upstream gradient dy.

    With ``rnd`` (the BF16 rounding) the upstream gradient enters the two
    products as rnd(dy), as it does on the GPU, where dx and dw are matrix
    products on BF16 operands; db is a plain sum of the unrounded dy.
    """
    dyp = dy if rnd is None else rnd(dy)
    d, h, wd, cin = x.shape
    od, oh, ow = dy.shape[:3]
    xp = np.zeros((d + 2, h + 2, wd + 2, cin))
    xp[1:-1, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for t, (dz, dy_, dx) in enumerate(taps()):
        sl = (slice(1 + dz, 1 + dz + stride * od, stride),
              slice(1 + dy_, 1 + dy_ + stride * oh, stride),
              slice(1 + dx, 1 + dx + stride * ow, stride))
        src = xp[sl]
        dw[t] = dyp.reshape(-1, dyp.shape[-1]).T @ src.reshape(-1, cin)
        dxp[sl] += dyp @ w[t]
    db = dy.sum(axis=(0, 1, 2))
    return dxp[1:-1, 1:-1, 1:-1], dw, db


def relu(x):
    return np.maximum(x, 0.0)


def up2(x):
    return x.repeat(2, axis=0).repeat(2, axis=1).repeat(2, axis=2)


def up2_backward(dy):
    d, h, w, c = dy.shape
    return dy.reshape(d // 2, 2, h // 2, 2, w // 2, 2, c).sum(axis=(1, 3, 5))


def layer_names(levels):
    names = []
    for l in range(levels):
        names += ["enc%d_a" % l, "enc%d_b" % l]
        if l < levels - 1:
            names.append("down%d" % l)
    for l in range(levels - 2, -1, -1):
        names += ["dec%d_a" % l, "dec%d_b" % l]
    return names


def param_shapes(levels):
    """Ordered (name, shape) of the flat FP32 parameter vector."""
    out = []
    for n in layer_names(levels):
        out.append((n + ".w", (27, C, C)))
        out.append((n + ".b", (C,)))
    out.append(("head.w", (C,)))
    out.append(("head.b", (1,)))
    return out


def unpack(theta, levels):
    p, o = {}, 0
    for name, shp in param_shapes(levels):
        n = int(np.prod(shp))
        p[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return p


def pack(grads, levels):
    return np.concatenate([grads[name].reshape(-1)
                           for name, _ in param_shapes(levels)])


def forward(theta, box, levels, round_bf16=True):
    """Network output (N, N, N) and the cache needed by backward.

    With round_bf16 the weights, the input and every stored activation are
    rounded to bfloat16 as on the GPU (accumulation stays FP64 here); biases,
    the head and the output stay unrounded.
    """
    rnd = bf16_round if round_bf16 else (lambda a: np.asarray(a, np.float64))
    p = unpack(theta, levels)
    w = {k: (rnd(v) if k.endswith(".w") and not k.startswith("head") else v)
         for k, v in p.items()}
    cache = {}
    x = rnd(lift(box))
    cache["in"] = x
    skips = {}
    for l in range(levels):
        h = rnd(relu(conv3(x, w["enc%d_a.w" % l], w["enc%d_a.b" % l])))
        cache["enc%d_a" % l] = (x, h)
        h2 = rnd(relu(conv3(h, w["enc%d_b.w" % l], w["enc%d_b.b" % l])))
        cache["enc%d_b" % l] = (h, h2)
        skips[l] = h2
        if l < levels - 1:
            x = rnd(relu(conv3(h2, w["down%d.w" % l], w["down%d.b" % l], 2)))
            cache["down%d" % l] = (h2, x)
        else:
            x = h2
    for l in range(levels - 2, -1, -1):
        s = rnd(up2(x) + skips[l])
        cache["sum%d" % l] = s
        h = rnd(relu(conv3(s, w["dec%d_a.w" % l], w["dec%d_a.b" % l])))
        cache["dec%d_a" % l] = (s, h)
        h2 = rnd(relu(conv3(h, w["dec%d_b.w" % l], w["dec%d_b.b" % l])))
        cache["dec%d_b" % l] = (h, h2)
        x = h2
    out = x @ p["head.w"] + p["head.b"][0] + blend(box)
    cache["last"] = x
    return out, (cache, w, p)


LOW_MODES = tuple((p, q, r) for p in (1, 2) for q in (1, 2) for r in (1, 2))


def low_mode(shape, pqr):
    """Discrete sine mode sin(p pi i/(n+1)) sin(q pi j/(n+1)) sin(r pi k/(n+1))
    on the interior cells (k, j, i) = 1..n of a (nz, ny, nx) field."""
    nz, ny, nx = shape
    p, q, r = pqr
    si = np.sin(np.pi * p * np.arange(1, nx + 1) / (nx + 1))
    sj = np.sin(np.pi * q * np.arange(1, ny + 1) / (ny + 1))
    sk = np.sin(np.pi * r * np.arange(1, nz + 1) / (nz + 1))
    return sk[:, None, None] * sj[None, :, None] * si[None, None, :]


def low_mode_coeffs(e):
    """a_m = mean over the cells of e * v_m for the modes in LOW_MODES."""
    return np.array([np.mean(e * low_mode(e.shape, m)) for m in LOW_MODES])


def loss_and_grad(theta, box, target, levels, round_bf16=True, low_weight=0.0):
    """Loss and its gradient with respect to the flat parameters.

    loss = mean((out - target)^2) + low_weight * sum_m a_m^2, with a_m the
    mean of (out - target) * v_m over the eight smoothest discrete sine modes
    v_m (p, q, r in {1, 2}).  The Jacobi iteration removes exactly these error
    components slowest (their decay factor per sweep is closest to 1), so
    weighting them sets the sweeps a guess saves; low_weight = 0 is plain
    MSE.
    """
    out, (cache, w, p) = forward(theta, box, levels, round_bf16)
    rnd = bf16_round if round_bf16 else None
    n = out.size
    diff = out - target
    loss = float(np.sum(diff * diff) / n)
    dout = 2.0 * diff / n
    if low_weight:
        a = low_mode_coeffs(diff)
        loss += float(low_weight * np.sum(a * a))
        for am, m in zip(a, LOW_MODES):
            dout = dout + (2.0 * low_weight * am / n) * low_mode(diff.shape, m)
    g = {}
    x = cache["last"]
    g["head.w"] = np.einsum("zyx,zyxc->c", dout, x)
    g["head.b"] = np.array([dout.sum()])
    dx = dout[..., None] * p["head.w"]
    dskip = {}
    # the decoder ran from level L-2 down to 0; walk it back from 0 up
    for l in range(0, levels - 1):
        s, h = cache["dec%d_a" % l]
        h_, h2 = cache["dec%d_b" % l]
        d2 = dx * (h2 > 0)
        dh, g["dec%d_b.w" % l], g["dec%d_b.b" % l] = conv3_backward(h, w["dec%d_b.w" % l], d2, rnd=rnd)
        d1 = dh * (h > 0)
        ds, g["dec%d_a.w" % l], g["dec%d_a.b" % l] = conv3_backward(s, w["dec%d_a.w" % l], d1, rnd=rnd)
        dskip[l] = ds
        dx = up2_backward(ds)
    for l in range(levels - 1, -1, -1):
        if l < levels - 1:
            h2, xo = cache["down%d" % l]
            dd = dx * (xo > 0)
            dh2, g["down%d.w" % l], g["down%d.b" % l] = conv3_backward(
                h2, w["down%d.w" % l], dd, 2, rnd=rnd)
            dh2 = dh2 + dskip[l]
        else:
            dh2 = dx
        h, h2 = cache["enc%d_b" % l]
        d2 = dh2 * (h2 > 0)
        dh, g["enc%d_b.w" % l], g["enc%d_b.b" % l] = conv3_backward(h, w["enc%d_b.w" % l], d2, rnd=rnd)
        x, h_ = cache["enc%d_a" % l]
        d1 = dh * (h > 0)
        dx, g["enc%d_a.w" % l], g["enc%d_a.b" % l] = conv3_backward(x, w["enc%d_a.w" % l], d1, rnd=rnd)
    return loss, pack(g, levels), out


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), bias-corrected; returns new arrays."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(levels, seed):
    """He-normal conv weights, zero biases, small head (numpy PCG64 seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for name, shp in param_shapes(levels):
        if name.endswith(".w") and not name.startswith("head"):
            parts.append(rng.standard_normal(shp).reshape(-1) * np.sqrt(2.0 / (27 * C)))
        elif name == "head.w":
            parts.append(rng.standard_normal(shp).reshape(-1) * np.sqrt(1.0 / C))
        else:
            parts.append(np.zeros(int(np.prod(shp))))
    return np.concatenate(parts)
