"""Python binding of libctof's convolution, loss, optimiser and sampler
entry points (ctypes; argument marshalling only).

Activations live in channels-last buffers: a torch tensor ``buf`` of shape
[rows, ld] (rows = n * d * h * w) holding BF16 (torch.bfloat16) or float32
elements; a ``Slice`` names channels [c0, c0 + c) of such a buffer.  All
arithmetic runs in the HIP library; this module only passes pointers.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from .ctof import _check, _ConvDesc, _stream_ptr, _Tensor, lib

K3, DN, UP, K1 = 0, 1, 2, 3
KIND = {"k3": K3, "dn": DN, "up": UP, "k1": K1}
TAPS = {K3: 27, DN: 8, UP: 1, K1: 1}


def _torch():
    import torch
    return torch


@dataclass
class Slice:
    buf: object  # torch tensor [rows, ld]
    c0: int = 0
    c: int = -1

    @property
    def ld(self) -> int:
        return int(self.buf.shape[1])

    @property
    def channels(self) -> int:
        return self.ld - self.c0 if self.c < 0 else self.c

    def t(self) -> _Tensor:
        return _Tensor(self.buf.data_ptr(), self.ld, self.c0)


@dataclass(frozen=True)
class Conv:
    kind: int
    n: int
    d: int
    h: int
    w: int
    ci: int
    co: int

    def desc(self) -> _ConvDesc:
        return _ConvDesc(self.kind, self.n, self.d, self.h, self.w, self.ci, self.co)

    def out_grid(self):
        if self.kind == DN:
            return self.n, self.d // 2, self.h // 2, self.w // 2
        if self.kind == UP:
            return self.n, 2 * self.d, 2 * self.h, 2 * self.w
        return self.n, self.d, self.h, self.w

    def out_rows(self) -> int:
        n, d, h, w = self.out_grid()
        return n * d * h * w


# ---- packed weight layout (see include/ctof.h) ------------------------------------

def cip(ci: int) -> int:
    return (ci + 7) // 8 * 8


def copad(co: int) -> int:
    return (co + 15) // 16 * 16


def kpad(kind: int, ci: int) -> int:
    return (TAPS[kind] * cip(ci) + 31) // 32 * 32


def weight_elems(kind: int, co: int, ci: int) -> int:
    n = ctypes.c_size_t()
    d = _ConvDesc(kind, 1, 2, 2, 2, ci, co)
    _check(lib().ctof_conv3d_weight_elems(ctypes.byref(d), ctypes.byref(n)))
    return int(n.value)


def pack_weights(kind: int, W: np.ndarray) -> np.ndarray:
    """Logical weights -> packed float32 layout.  Logical shapes:
    K3 [co,3,3,3,ci], DN [co,2,2,2,ci], UP [2,2,2,co,ci], K1 [co,ci]."""
    W = np.asarray(W, dtype=np.float32)
    if kind == UP:
        co, ci = W.shape[3], W.shape[4]
        out = np.zeros((8, copad(co), kpad(UP, ci)), np.float32)
        out[:, :co, :ci] = W.reshape(8, co, ci)
        return out.reshape(-1)
    co, ci = W.shape[0], W.shape[-1]
    taps = TAPS[kind]
    out = np.zeros((copad(co), kpad(kind, ci)), np.float32)
    cols = np.zeros((co, taps, cip(ci)), np.float32)
    cols[:, :, :ci] = W.reshape(co, taps, ci)
    out[:co, :taps * cip(ci)] = cols.reshape(co, -1)
    return out.reshape(-1)


def unpack_weights(kind: int, packed: np.ndarray, co: int, ci: int) -> np.ndarray:
    """Inverse of pack_weights (drops the padding)."""
    p = np.asarray(packed, dtype=np.float64)
    if kind == UP:
        return p.reshape(8, copad(co), kpad(UP, ci))[:, :co, :ci].reshape(2, 2, 2, co, ci)
    taps = TAPS[kind]
    m = p.reshape(copad(co), kpad(kind, ci))[:co, :taps * cip(ci)].reshape(co, taps, cip(ci))[:, :, :ci]
    return m.reshape((co, 3, 3, 3, ci) if kind == K3 else (co, 2, 2, 2, ci) if kind == DN else (co, ci))


# ---- workspace ------------------------------------------------------------------------

_ws = {}


def workspace(nbytes: int, device="cuda", tag="default"):
    """A grow-only scratch buffer per tag (stream-ordered reuse)."""
    torch = _torch()
    cur = _ws.get(tag)
    if cur is None or cur.numel() < nbytes or cur.device != torch.device(device):
        cur = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _ws[tag] = cur
    return cur


# ---- layer calls ----------------------------------------------------------------------

def conv_fwd(cv: Conv, x: Slice, w_bf16, bias, y: Slice, relu=True, accumulate=False, stream=None):
    y_fp32 = 1 if y.buf.dtype == _torch().float32 else 0
    _check(lib().ctof_conv3d_fwd(ctypes.byref(cv.desc()), ctypes.byref(x.t()), w_bf16.data_ptr(),
                                 bias.data_ptr() if bias is not None else None, ctypes.byref(y.t()),
                                 y_fp32, int(bool(relu)), int(bool(accumulate)), _stream_ptr(stream)))


def conv_bwd_data(cv: Conv, dy: Slice, w_bf16, dx: Slice, accumulate=False, stream=None):
    n = ctypes.c_size_t()
    d = cv.desc()
    _check(lib().ctof_conv3d_bwd_data_ws_bytes(ctypes.byref(d), ctypes.byref(n)))
    ws = workspace(n.value, w_bf16.device, "bwd_data")
    _check(lib().ctof_conv3d_bwd_data(ctypes.byref(d), ctypes.byref(dy.t()), w_bf16.data_ptr(),
                                      ctypes.byref(dx.t()), int(bool(accumulate)), ws.data_ptr(), ws.numel(),
                                      _stream_ptr(stream)))


def conv_bwd_weight(cv: Conv, x: Slice, dy: Slice, dw, db=None, stream=None):
    n = ctypes.c_size_t()
    d = cv.desc()
    _check(lib().ctof_conv3d_bwd_weight_ws_bytes(ctypes.byref(d), ctypes.byref(n)))
    ws = workspace(n.value, dw.device, "bwd_weight")
    _check(lib().ctof_conv3d_bwd_weight(ctypes.byref(d), ctypes.byref(x.t()), ctypes.byref(dy.t()),
                                        dw.data_ptr(), db.data_ptr() if db is not None else None,
                                        ws.data_ptr(), ws.numel(), _stream_ptr(stream)))


def relu_bwd(rows: int, ch: int, dy: Slice, y: Slice, stream=None):
    _check(lib().ctof_relu_bwd(int(rows), int(ch), ctypes.byref(dy.t()), ctypes.byref(y.t()),
                               _stream_ptr(stream)))


def mse(n: int, y: Slice, target, grad: Slice, loss, relu_mask=True, y_scale=1.0, stream=None):
    nb = ctypes.c_size_t()
    _check(lib().ctof_mse_ws_bytes(int(n), ctypes.byref(nb)))
    ws = workspace(nb.value, target.device, "mse")
    _check(lib().ctof_mse(int(n), ctypes.byref(y.t()), float(y_scale), target.data_ptr(), ctypes.byref(grad.t()),
                          int(bool(relu_mask)), loss.data_ptr(), ws.data_ptr(), ws.numel(),
                          _stream_ptr(stream)))


def adam_step(w, g, m, v, w_bf16, lr, step, b1=0.9, b2=0.999, eps=1e-8, grad_scale=1.0, stream=None):
    wb = w_bf16.data_ptr() if w_bf16 is not None else None
    if grad_scale == 1.0:
        _check(lib().ctof_adam_step(int(w.numel()), w.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), wb,
                                    float(lr), float(b1), float(b2), float(eps), int(step), _stream_ptr(stream)))
    else:
        _check(lib().ctof_adam_step_scaled(int(w.numel()), w.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(),
                                           wb, float(lr), float(b1), float(b2), float(eps), int(step),
                                           float(grad_scale), _stream_ptr(stream)))


def sumsq(x, stream=None):
    """FP64 sum of squares of a float tensor (one device double)."""
    torch = _torch()
    nb = ctypes.c_size_t()
    _check(lib().ctof_sumsq_ws_bytes(1, ctypes.byref(nb)))
    ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=x.device)
    out = torch.empty(1, dtype=torch.float64, device=x.device)
    _check(lib().ctof_sumsq(1, int(x.numel()), x.data_ptr(), out.data_ptr(), ws.data_ptr(), ws.numel(),
                            _stream_ptr(stream)))
    return out


def to_channels_last(x, scale: float, out: Slice, zero_rest=False, split=False, stream=None):
    _check(lib().ctof_to_channels_last(int(x.numel()), x.data_ptr(), float(scale), ctypes.byref(out.t()),
                                       int(bool(zero_rest)), int(bool(split)), _stream_ptr(stream)))


def from_channels_last(y: Slice, scale: float, out, stream=None):
    _check(lib().ctof_from_channels_last(int(out.numel()), ctypes.byref(y.t()), float(scale), out.data_ptr(),
                                         _stream_ptr(stream)))


def philox(seed: int, stream_id: int, first: int, n: int, device="cuda", stream=None):
    torch = _torch()
    out = torch.empty((n, 4), dtype=torch.int32, device=device)
    _check(lib().ctof_philox4x32(int(seed), int(stream_id), int(first), int(n), out.data_ptr(),
                                 _stream_ptr(stream)))
    return out


def poisson(lam, seed: int, stream_id: int = 0, out=None, stream=None):
    torch = _torch()
    out = torch.empty_like(lam) if out is None else out
    _check(lib().ctof_poisson(int(lam.numel()), lam.data_ptr(), int(seed), int(stream_id), out.data_ptr(),
                              _stream_ptr(stream)))
    return out


def noisy_histogram(m, peak: float, seed: int, stream_id: int = 0, out=None, stream=None):
    torch = _torch()
    out = torch.empty_like(m) if out is None else out
    nb = ctypes.c_size_t()
    _check(lib().ctof_noisy_histogram_ws_bytes(int(m.numel()), ctypes.byref(nb)))
    ws = workspace(nb.value, m.device, "noisy")
    _check(lib().ctof_noisy_histogram(int(m.numel()), m.data_ptr(), float(peak), int(seed), int(stream_id),
                                      out.data_ptr(), ws.data_ptr(), ws.numel(), _stream_ptr(stream)))
    return out


def warmstart_loss(kernel, nb: int, y: Slice, s, target, w, v, lam: float, grad: Slice, terms,
                   relu_mask=True, stream=None):
    """Operator-weighted start loss (see ctof_warmstart_loss); s (a number
    or nb of them), w, v: host weights; terms: device float64 [>= nb, 2]."""
    nbytes = ctypes.c_size_t()
    _check(lib().ctof_warmstart_loss_ws_bytes(kernel.handle, int(nb), ctypes.byref(nbytes)))
    ws = workspace(nbytes.value, target.device, "start_loss")
    s = [float(s)] * nb if isinstance(s, (int, float)) else [float(x) for x in s]
    sa = (ctypes.c_double * nb)(*s)
    wa = (ctypes.c_double * nb)(*[float(x) for x in w])
    va = (ctypes.c_double * nb)(*[float(x) for x in v])
    _check(lib().ctof_warmstart_loss(kernel.handle, int(nb), ctypes.byref(y.t()), sa, target.data_ptr(), wa,
                                     va, float(lam), int(bool(relu_mask)), ctypes.byref(grad.t()), terms.data_ptr(),
                                     ws.data_ptr(), ws.numel(), _stream_ptr(stream)))


def absmax(x, nb: int, stream=None):
    """max |x[b]| per sample of a float32 tensor with nb leading rows (device
    float32 [nb])."""
    torch = _torch()
    out = torch.empty(nb, dtype=torch.float32, device=x.device)
    nbytes = ctypes.c_size_t()
    _check(lib().ctof_absmax_ws_bytes(int(nb), ctypes.byref(nbytes)))
    ws = workspace(nbytes.value, x.device, "absmax")
    _check(lib().ctof_absmax(int(nb), int(x.numel() // nb), x.data_ptr(), out.data_ptr(), ws.data_ptr(), ws.numel(),
                             _stream_ptr(stream)))
    return out


def depth_resample(x, mode: int, stream=None):
    """x float32 [nb, nz, h, w]: mode 0 sums layer pairs (nz / 2 out), mode 1
    repeats layers (2 nz out)."""
    torch = _torch()
    nb, nz = int(x.shape[0]), int(x.shape[1])
    plane = int(x[0, 0].numel())
    nz_out = nz // 2 if mode == 0 else 2 * nz
    out = torch.empty((nb, nz_out) + tuple(x.shape[2:]), dtype=torch.float32, device=x.device)
    _check(lib().ctof_depth_resample(nb, nz, plane, x.contiguous().data_ptr(), out.data_ptr(), int(mode),
                                     _stream_ptr(stream)))
    return out
