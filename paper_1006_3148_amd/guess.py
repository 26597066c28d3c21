"""Python handle over the learned-guess C-ABI (jacobi_guess.h): marshalling
only; every step runs in libjacobi's kernels."""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import check, lib

_h = ctypes.c_void_p
_SIGS = {
    "jg_param_count": ([ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "jg_workspace_size": ([ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
                          ctypes.c_int),
    "jg_create": ([ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                   ctypes.c_void_p, ctypes.POINTER(_h)], ctypes.c_int),
    "jg_forward": ([_h, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "jg_backward": ([_h, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "jg_set_low_mode_weight": ([_h, ctypes.c_double], ctypes.c_int),
    "jg_zero_grads": ([_h], ctypes.c_int),
    "jg_adam": ([_h, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                 ctypes.c_int64], ctypes.c_int),
    "jg_write_guess": ([_h, ctypes.c_void_p], ctypes.c_int),
    "jg_write_blend": ([_h, ctypes.c_void_p], ctypes.c_int),
    "jg_destroy": ([_h], ctypes.c_int),
    "jg_conv3_workspace_size": ([ctypes.c_int64, ctypes.c_int32,
                                 ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "jg_conv3_forward": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                          ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "jg_conv3_backward_data": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
    "jg_conv3_backward_weight": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
}
for _name, (_a, _r) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _a
    _f.restype = _r

EXPORTED = tuple(_SIGS)


def param_count(levels: int) -> int:
    c = ctypes.c_int64()
    check(lib.jg_param_count(levels, ctypes.byref(c)))
    return c.value


def init_params(levels: int, seed: int) -> np.ndarray:
    """Initial parameters: He-normal conv weights (std sqrt(2/(27*16))), zero
    biases, head weights N(0, 1/16), zero head bias; numpy PCG64(seed), drawn
    layer by layer in parameter order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    layers = (param_count(levels) - 17) // (27 * 256 + 16)
    parts = []
    for _ in range(layers):
        parts.append(rng.standard_normal(27 * 256) * np.sqrt(2.0 / (27 * 16)))
        parts.append(np.zeros(16))
    parts.append(rng.standard_normal(16) * np.sqrt(1.0 / 16))
    parts.append(np.zeros(1))
    return np.concatenate(parts)


class GuessNet:
    """The U-Net on the GPU.  ``params`` (numpy FP32/FP64 vector) initialises
    the FP32 master parameters; gradients and Adam moments are allocated
    here (torch tensors)."""

    def __init__(self, n: int, levels: int, params, train: bool = True,
                 stream=None, device: str = "cuda"):
        self.n, self.levels = n, levels
        self.np_ = param_count(levels)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        p = np.asarray(params, dtype=np.float32)
        if p.size != self.np_:
            raise ValueError("expected %d parameters, got %d" % (self.np_, p.size))
        ws = ctypes.c_size_t()
        check(lib.jg_workspace_size(n, levels, ctypes.byref(ws)))
        with torch.cuda.stream(self.stream):
            self.params = torch.from_numpy(p.copy()).to(device)
            self.grads = torch.zeros_like(self.params) if train else None
            self.m = torch.zeros_like(self.params) if train else None
            self.v = torch.zeros_like(self.params) if train else None
            self.ws = torch.empty(ws.value, dtype=torch.uint8, device=device)
            self.out = torch.empty(n ** 3, dtype=torch.float32, device=device)
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        ptr = (lambda t: t.data_ptr() if t is not None else None)
        check(lib.jg_create(n, levels, ptr(self.params), ptr(self.grads), ptr(self.m),
                            ptr(self.v), self.ws.data_ptr(), self.ws.numel(),
                            int(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.step_count = 0

    def forward(self, box: torch.Tensor) -> torch.Tensor:
        """box: dense (n+2)^3 float64 CUDA tensor; returns the n^3 output."""
        check(lib.jg_forward(self._h, box.data_ptr(), self.out.data_ptr()))
        return self.out.view(self.n, self.n, self.n)

    def backward(self, target: torch.Tensor, want_loss: bool = True):
        loss = ctypes.c_double()
        check(lib.jg_backward(self._h, target.data_ptr(),
                              ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def set_low_mode_weight(self, weight: float) -> None:
        """Weight of the low-mode term of the training loss (0: plain MSE)."""
        check(lib.jg_set_low_mode_weight(self._h, float(weight)))

    def zero_grads(self) -> None:
        check(lib.jg_zero_grads(self._h))

    def adam(self, lr: float, beta1=0.9, beta2=0.999, eps=1e-8) -> None:
        self.step_count += 1
        check(lib.jg_adam(self._h, lr, beta1, beta2, eps, self.step_count))

    def write_guess(self, box: torch.Tensor) -> None:
        check(lib.jg_write_guess(self._h, box.data_ptr()))

    def write_blend(self, box: torch.Tensor) -> None:
        """Writes the non-learned face blend of box's faces into its interior."""
        check(lib.jg_write_blend(self._h, box.data_ptr()))

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib.jg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- single convolution layers (jg_conv3_*): BF16 operands are passed as
# int16 tensors holding the bit patterns, everything on the current stream.

def _layer_ws(d: int, stride: int) -> torch.Tensor:
    ws = ctypes.c_size_t()
    check(lib.jg_conv3_workspace_size(d, stride, ctypes.byref(ws)))
    return torch.empty(ws.value, dtype=torch.uint8, device="cuda")


def conv3_forward(x: torch.Tensor, w: torch.Tensor, bias: torch.Tensor,
                  stride: int = 1) -> torch.Tensor:
    """x: (d,d,d,16) int16 BF16 bits; w: (27,16,16) int16 BF16 bits; bias:
    (16,) float32.  Returns the FP32 pre-activation output (d/s,d/s,d/s,16)."""
    d = x.shape[0]
    y = torch.empty((d // stride,) * 3 + (16,), dtype=torch.float32, device=x.device)
    check(lib.jg_conv3_forward(x.data_ptr(), d, w.data_ptr(), bias.data_ptr(), stride,
                               y.data_ptr(), torch.cuda.current_stream().cuda_stream))
    return y


def conv3_backward_data(dy: torch.Tensor, w: torch.Tensor, stride: int = 1) -> torch.Tensor:
    """dy: (d/s,d/s,d/s,16) float32; returns dx (d,d,d,16) float32."""
    d = dy.shape[0] * stride
    dx = torch.empty((d,) * 3 + (16,), dtype=torch.float32, device=dy.device)
    ws = _layer_ws(d, stride)
    check(lib.jg_conv3_backward_data(dy.data_ptr(), d, w.data_ptr(), stride, dx.data_ptr(),
                                     ws.data_ptr(), ws.numel(),
                                     torch.cuda.current_stream().cuda_stream))
    return dx


def conv3_backward_weight(x: torch.Tensor, dy: torch.Tensor, stride: int = 1) -> torch.Tensor:
    """Returns the (27*256 + 16,) float32 weight and bias gradient."""
    d = x.shape[0]
    g = torch.zeros(27 * 256 + 16, dtype=torch.float32, device=x.device)
    ws = _layer_ws(d, stride)
    check(lib.jg_conv3_backward_weight(x.data_ptr(), d, dy.data_ptr(), stride, g.data_ptr(),
                                       ws.data_ptr(), ws.numel(),
                                       torch.cuda.current_stream().cuda_stream))
    return g
