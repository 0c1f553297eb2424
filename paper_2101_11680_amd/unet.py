"""Learned warm start: a 4-level 3D U-Net run on libctof's BF16 kernels.

The network maps the scaled adjoint back-projection x = tau A^T d of a scan
(tau = 1/L, the solver's step) to a non-negative starting volume for the
FISTA reconstruction of the paper's regularised least-squares problem
(section "Reconstruction Algorithm").  Only the start changes: the solver
then runs to the same tolerance, and with warm_start = 2 it discards a start
whose first gradient-mapping ratio is worse than a zero start's.

Architecture (channels c1..c4 = 16/32/64/64 by default; every conv has a
bias and a ReLU):
  encoder level l = 1, 2, 3:  k3 (c_{l-1} -> c_l), k3 (c_l -> c_l) [skip],
                              dn (c_l -> c_l, stride 2)
  level 4:                    k3 (c3 -> c4), k3 (c4 -> c4)
  decoder level l = 3, 2, 1:  up (c_{l+1} -> c_l, stride 2), concatenate
                              [up, skip], k3 (2 c_l -> c_l), k3 (c_l -> c_l)
  head:                       k1 (c1 -> 1)
Activations are BF16 channels-last; the skip of level l is written straight
into the upper half of that level's concatenation buffer.  Parameters are
one flat FP32 master buffer (each layer's packed weights, then its bias) with
a BF16 working copy, FP32 gradients and Adam moments; the optimiser is one
launch over the whole buffer.

Every arithmetic step runs in libctof (conv forward / input gradient /
weight gradient, ReLU mask, loss, Adam, sampling, the operator and the
solver); this module allocates buffers and sequences the calls.
"""

from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import ctof, nn
from .nn import DN, K1, K3, UP, Conv, Slice

DEFAULT_CH = (16, 32, 64, 64)
_KINDS = {"k3": K3, "dn": DN, "up": UP, "k1": K1}


def _torch():
    import torch
    return torch


def layer_list(ch=DEFAULT_CH, c_in: int = 1) -> List[Tuple[str, int, int, int]]:
    """(name, kind, co, ci) in execution order."""
    c1, c2, c3, c4 = ch
    out = []
    prev = c_in
    for lvl, c in ((1, c1), (2, c2), (3, c3)):
        out += [(f"e{lvl}a", K3, c, prev), (f"e{lvl}b", K3, c, c), (f"d{lvl}", DN, c, c)]
        prev = c
    out += [("m4a", K3, c4, c3), ("m4b", K3, c4, c4)]
    below = c4
    for lvl, c in ((3, c3), (2, c2), (1, c1)):
        out += [(f"u{lvl}", UP, c, below), (f"c{lvl}a", K3, c, 2 * c), (f"c{lvl}b", K3, c, c)]
        below = c
    out.append(("head", K1, 1, c1))
    return out


def _align(n: int, a: int = 64) -> int:
    return (n + a - 1) // a * a


@dataclass
class _Param:
    kind: int
    co: int
    ci: int
    w_off: int
    w_len: int
    b_off: int


class UNet:
    """Parameters, activation buffers and the forward/backward sequence."""

    def __init__(self, ch=DEFAULT_CH, device="cuda", seed: int = 0, split_input: bool = True):
        torch = _torch()
        for c in ch:
            if c % 8 or c < 8:
                raise ValueError("channel counts must be multiples of 8")
        self.ch = tuple(int(c) for c in ch)
        self.device = torch.device(device)
        # the input volume enters as a BF16 hi/lo pair (two channels) or as
        # one BF16 channel
        self.split_input = bool(split_input)
        self.c_in = 2 if self.split_input else 1
        self.layers = layer_list(self.ch, self.c_in)
        self.params: Dict[str, _Param] = {}
        off = 0
        for name, kind, co, ci in self.layers:
            wl = nn.weight_elems(kind, co, ci)
            w_off = off
            off += _align(wl)
            b_off = off
            off += _align(co)
            self.params[name] = _Param(kind, co, ci, w_off, wl, b_off)
        self.size = off
        f32 = dict(dtype=torch.float32, device=self.device)
        self.master = torch.zeros(off, **f32)
        self.work = torch.zeros(off, dtype=torch.bfloat16, device=self.device)
        self.grad = torch.zeros(off, **f32)
        self.m = torch.zeros(off, **f32)
        self.v = torch.zeros(off, **f32)
        self.step_count = 0
        # per-sample normalisation: the input is A^T d / max|A^T d| (times
        # in_scale), the start is output * out_scale * tau * max|A^T d|, so the
        # network sees unit-scale inputs whatever the absorbers' depth
        self.in_scale = 1.0
        self.out_scale = 1.0
        self._bufs = None
        self._shape = None
        self.loss_dev = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.init(seed)

    # ---- parameters -----------------------------------------------------------
    def init(self, seed: int) -> None:
        """He-normal weights (fan-in = taps x ci), zero biases."""
        rng = np.random.default_rng(seed)
        logical = {}
        for name, kind, co, ci in self.layers:
            taps = {K3: 27, DN: 8, UP: 1, K1: 1}[kind]
            shape = {K3: (co, 3, 3, 3, ci), DN: (co, 2, 2, 2, ci), UP: (2, 2, 2, co, ci), K1: (co, ci)}[kind]
            logical[name + ".w"] = rng.normal(0.0, math.sqrt(2.0 / (taps * ci)), shape)
            logical[name + ".b"] = np.zeros(co)
        self.load_logical(logical)

    def load_logical(self, P: Dict[str, np.ndarray]) -> None:
        """Set parameters from logical arrays (shapes of the layer kinds)."""
        torch = _torch()
        host = np.zeros(self.size, np.float32)
        for name, p in self.params.items():
            host[p.w_off:p.w_off + p.w_len] = nn.pack_weights(p.kind, P[name + ".w"])
            host[p.b_off:p.b_off + p.co] = np.asarray(P[name + ".b"], np.float32)
        t = torch.from_numpy(host)
        self.master.copy_(t)
        self.work.copy_(t.to(torch.bfloat16))
        self.m.zero_()
        self.v.zero_()
        self.step_count = 0

    def logical(self, which: str = "master") -> Dict[str, np.ndarray]:
        """Parameters ('master') or gradients ('grad') as logical arrays."""
        src = (self.master if which == "master" else self.grad).detach().cpu().numpy()
        out = {}
        for name, p in self.params.items():
            out[name + ".w"] = nn.unpack_weights(p.kind, src[p.w_off:p.w_off + p.w_len], p.co, p.ci)
            out[name + ".b"] = src[p.b_off:p.b_off + p.co].astype(np.float64)
        return out

    def _w(self, name):
        p = self.params[name]
        return self.work[p.w_off:p.w_off + p.w_len], self.master[p.b_off:p.b_off + p.co]

    def _g(self, name):
        p = self.params[name]
        return self.grad[p.w_off:p.w_off + p.w_len], self.grad[p.b_off:p.b_off + p.co]

    # ---- buffers ----------------------------------------------------------------
    def _alloc(self, n: int, D: int, H: int, W: int) -> None:
        if self._shape == (n, D, H, W):
            return
        if D % 8 or H % 8 or W % 8:
            raise ValueError("grid sizes must be divisible by 8 (three stride-2 levels)")
        torch = _torch()
        c1, c2, c3, c4 = self.ch
        rows = [n * D * H * W >> (3 * l) for l in range(4)]
        bf = dict(dtype=torch.bfloat16, device=self.device)

        def z(r, c, dt=None):
            return torch.zeros((r, c), **(bf if dt is None else dict(dtype=dt, device=self.device)))

        A = {"input": z(rows[0], 8)}
        G = {}
        for l, c in ((1, c1), (2, c2), (3, c3)):
            r = rows[l - 1]
            A[f"e{l}a"] = z(r, c)
            A[f"cat{l}"] = z(r, 2 * c)
            A[f"d{l}"] = z(rows[l], c)
            A[f"c{l}a"] = z(r, c)
            A[f"c{l}b"] = z(r, c)
            G[f"e{l}a"] = z(r, c)
            G[f"cat{l}"] = z(r, 2 * c)
            G[f"d{l}"] = z(rows[l], c)
            G[f"c{l}a"] = z(r, c)
            G[f"c{l}b"] = z(r, c)
        A["m4a"] = z(rows[3], c4)
        A["m4b"] = z(rows[3], c4)
        G["m4a"] = z(rows[3], c4)
        G["m4b"] = z(rows[3], c4)
        A["head"] = z(rows[0], 1, torch.float32)
        G["head"] = z(rows[0], 8)
        self._bufs = (A, G)
        self._shape = (n, D, H, W)
        self._grids = [(n, D >> l, H >> l, W >> l) for l in range(4)]

    def _conv(self, name: str, lvl: int) -> Conv:
        """Conv descriptor of a layer whose INPUT is on level lvl (0-based)."""
        p = self.params[name]
        n, d, h, w = self._grids[lvl]
        return Conv(p.kind, n, d, h, w, p.ci, p.co)

    # ---- forward ----------------------------------------------------------------
    def forward(self, x, scale=1.0, stream=None):
        """x: float32 [n, D, H, W] back-projections A^T d; the network input
        is x * scale * in_scale, scale a number or one per sample (tau of the
        scan's class).  Returns the FP32 head buffer [rows, 1] (network
        units: the start volume is head * out_scale)."""
        n, D, H, W = x.shape
        self._alloc(n, D, H, W)
        A, _ = self._bufs
        c = self.ch
        x = x.contiguous()
        if isinstance(scale, (int, float)):
            nn.to_channels_last(x, float(scale) * self.in_scale, Slice(A["input"], 0, self.c_in),
                                split=self.split_input, stream=stream)
        else:
            R = D * H * W
            for i in range(n):
                nn.to_channels_last(x[i], float(scale[i]) * self.in_scale,
                                    Slice(A["input"][i * R:(i + 1) * R], 0, self.c_in), split=self.split_input,
                                    stream=stream)
        run = lambda name, lvl, src, dst: nn.conv_fwd(self._conv(name, lvl), src, *self._w(name), dst,
                                                      relu=True, stream=stream)
        h = Slice(A["input"], 0, self.c_in)
        for l in (1, 2, 3):
            cl = c[l - 1]
            run(f"e{l}a", l - 1, h, Slice(A[f"e{l}a"]))
            run(f"e{l}b", l - 1, Slice(A[f"e{l}a"]), Slice(A[f"cat{l}"], cl, cl))
            run(f"d{l}", l - 1, Slice(A[f"cat{l}"], cl, cl), Slice(A[f"d{l}"]))
            h = Slice(A[f"d{l}"])
        run("m4a", 3, h, Slice(A["m4a"]))
        run("m4b", 3, Slice(A["m4a"]), Slice(A["m4b"]))
        h = Slice(A["m4b"])
        for l in (3, 2, 1):
            cl = c[l - 1]
            run(f"u{l}", l, h, Slice(A[f"cat{l}"], 0, cl))
            run(f"c{l}a", l - 1, Slice(A[f"cat{l}"]), Slice(A[f"c{l}a"]))
            run(f"c{l}b", l - 1, Slice(A[f"c{l}a"]), Slice(A[f"c{l}b"]))
            h = Slice(A[f"c{l}b"])
        run("head", 0, h, Slice(A["head"], 0, 1))
        return A["head"]

    # ---- backward ----------------------------------------------------------------
    def _back(self, name, lvl, x: Slice, dy: Slice, y: Optional[Slice], dx: Optional[Slice], accumulate=False,
              stream=None):
        """ReLU mask of dy by y (unless y is None), weight/bias gradients, and
        the input gradient into dx (unless None)."""
        cv = self._conv(name, lvl)
        if y is not None:
            nn.relu_bwd(cv.out_rows(), cv.co, dy, y, stream=stream)
        gw, gb = self._g(name)
        nn.conv_bwd_weight(cv, x, dy, gw, gb, stream=stream)
        if dx is not None:
            nn.conv_bwd_data(cv, dy, self._w(name)[0], dx, accumulate=accumulate, stream=stream)

    def backward_from_output_grad(self, stream=None) -> None:
        """Backward pass given the head gradient already in G['head'] (channel
        0, the head's ReLU mask applied)."""
        A, G = self._bufs
        c = self.ch
        S = Slice
        self._back("head", 0, S(A["c1b"]), S(G["head"], 0, 1), None, S(G["c1b"]), stream=stream)
        for l in (1, 2, 3):
            cl = c[l - 1]
            self._back(f"c{l}b", l - 1, S(A[f"c{l}a"]), S(G[f"c{l}b"]), S(A[f"c{l}b"]), S(G[f"c{l}a"]),
                       stream=stream)
            self._back(f"c{l}a", l - 1, S(A[f"cat{l}"]), S(G[f"c{l}a"]), S(A[f"c{l}a"]), S(G[f"cat{l}"]),
                       stream=stream)
            src_a, src_g = (A["m4b"], G["m4b"]) if l == 3 else (A[f"c{l + 1}b"], G[f"c{l + 1}b"])
            self._back(f"u{l}", l, S(src_a), S(G[f"cat{l}"], 0, cl), S(A[f"cat{l}"], 0, cl), S(src_g),
                       stream=stream)
        self._back("m4b", 3, S(A["m4a"]), S(G["m4b"]), S(A["m4b"]), S(G["m4a"]), stream=stream)
        self._back("m4a", 3, S(A["d3"]), S(G["m4a"]), S(A["m4a"]), S(G["d3"]), stream=stream)
        for l in (3, 2, 1):
            cl = c[l - 1]
            skip_a, skip_g = S(A[f"cat{l}"], cl, cl), S(G[f"cat{l}"], cl, cl)
            # the dn layer's input gradient is added to the skip's gradient
            self._back(f"d{l}", l - 1, skip_a, S(G[f"d{l}"]), S(A[f"d{l}"]), skip_g, accumulate=True,
                       stream=stream)
            self._back(f"e{l}b", l - 1, S(A[f"e{l}a"]), skip_g, skip_a, S(G[f"e{l}a"]), stream=stream)
            prev_a = S(A["input"], 0, self.c_in) if l == 1 else S(A[f"d{l - 1}"])
            prev_g = None if l == 1 else S(G[f"d{l - 1}"])
            self._back(f"e{l}a", l - 1, prev_a, S(G[f"e{l}a"]), S(A[f"e{l}a"]), prev_g, stream=stream)

    def loss_and_backward(self, target, stream=None):
        """Mean squared error of the start volume (head * out_scale) against
        target (float32 [n, D, H, W], physical units); fills the gradients;
        returns the device loss (double [1])."""
        A, G = self._bufs
        rows = A["head"].shape[0]
        nn.mse(rows, Slice(A["head"], 0, 1), target.contiguous(), Slice(G["head"], 0, 1), self.loss_dev,
               relu_mask=True, y_scale=self.out_scale, stream=stream)
        self.backward_from_output_grad(stream=stream)
        return self.loss_dev

    def start_scales(self, x, tau, stream=None):
        """Per-sample (input scale, output scale) of back-projections x
        [n, ...] for step sizes tau (a number or one per sample)."""
        n = x.shape[0]
        m = nn.absmax(x.contiguous(), n, stream=stream).cpu().numpy().astype(np.float64)
        taus = [float(tau)] * n if isinstance(tau, (int, float)) else [float(t) for t in tau]
        s_in = [self.in_scale / mb if mb > 0 else 0.0 for mb in m]
        s_out = [self.out_scale * t * mb for t, mb in zip(taus, m)]
        return s_in, s_out

    def loss_terms_operator(self, kernel, target, w, v, lam: float, s_out, stream=None):
        """The loss terms (||H e_b||^2, ||e_b||^2) of the current forward
        pass without a backward pass (device [n, 2]); the head gradient
        buffer is overwritten."""
        torch = _torch()
        A, G = self._bufs
        n = self._shape[0]
        if getattr(self, "_terms", None) is None:
            self._terms = torch.zeros((64, 2), dtype=torch.float64, device=self.device)
        nn.warmstart_loss(kernel, n, Slice(A["head"], 0, 1), s_out, target.contiguous(), w, v, lam,
                          Slice(G["head"], 0, 1), self._terms, relu_mask=False, stream=stream)
        return self._terms[:n]

    def loss_and_backward_operator(self, kernel, target, w, v, lam: float, s_out, straight_through: bool = True,
                                   stream=None):
        """Operator-weighted loss w_b ||H e_b||^2 + v_b ||e_b||^2 of the start
        volumes (H = A^T A + lambda I of the scans' handle; e = start -
        target); fills the gradients; returns the device terms [n, 2].  With
        straight_through the head's ReLU passes the gradient where it clamps,
        so outputs pushed below zero can recover."""
        torch = _torch()
        A, G = self._bufs
        n = self._shape[0]
        if getattr(self, "_terms", None) is None:
            self._terms = torch.zeros((64, 2), dtype=torch.float64, device=self.device)
        nn.warmstart_loss(kernel, n, Slice(A["head"], 0, 1), s_out, target.contiguous(), w, v, lam,
                          Slice(G["head"], 0, 1), self._terms, relu_mask=not straight_through, stream=stream)
        self.backward_from_output_grad(stream=stream)
        return self._terms[:n]

    def adam(self, lr: float, grad_scale: float = 1.0, stream=None) -> None:
        self.step_count += 1
        nn.adam_step(self.master, self.grad, self.m, self.v, self.work, lr, self.step_count, grad_scale=grad_scale,
                     stream=stream)

    # ---- inference ----------------------------------------------------------------
    def predict(self, x, tau=1.0, stream=None):
        """Start volumes (float32 [n, D, H, W]) from back-projections A^T d
        (x) of scans with step sizes tau (a number or one per sample)."""
        torch = _torch()
        s_in, s_out = self.start_scales(x, tau, stream=stream)
        head = self.forward(x, s_in, stream=stream)
        out = torch.empty(x.shape, dtype=torch.float32, device=self.device)
        R = int(np.prod(x.shape[1:]))
        for b in range(x.shape[0]):
            nn.from_channels_last(Slice(head[b * R:(b + 1) * R], 0, 1), s_out[b], out[b], stream=stream)
        return out

    # ---- checkpoints ----------------------------------------------------------------
    def save(self, path: str, extra: Optional[dict] = None, weights_only: bool = False) -> None:
        """FP32 master weights, Adam moments (unless weights_only), step and
        scales (npz of plain arrays, no pickles)."""
        meta = dict(ch=list(self.ch), split_input=self.split_input, step=self.step_count, in_scale=self.in_scale,
                    out_scale=self.out_scale)
        meta.update(getattr(self, "meta_extra", {}))
        meta.update(extra or {})
        arrays = dict(master=self.master.cpu().numpy(), meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))
        if not weights_only:
            arrays.update(m=self.m.cpu().numpy(), v=self.v.cpu().numpy())
        np.savez(path, **arrays)

    @classmethod
    def load(cls, path: str, device="cuda") -> "UNet":
        torch = _torch()
        z = np.load(path, allow_pickle=False)
        meta = json.loads(bytes(z["meta"]).decode())
        net = cls(tuple(meta["ch"]), device=device, split_input=bool(meta.get("split_input", False)))
        master = torch.from_numpy(z["master"])
        if master.numel() != net.size:
            raise ValueError("checkpoint does not match the architecture")
        net.master.copy_(master)
        net.work.copy_(master.to(torch.bfloat16))
        if "m" in z.files:
            net.m.copy_(torch.from_numpy(z["m"]))
            net.v.copy_(torch.from_numpy(z["v"]))
        net.step_count = int(meta["step"])
        net.in_scale = float(meta["in_scale"])
        net.out_scale = float(meta["out_scale"])
        net.meta = meta
        net.meta_extra = {k: v for k, v in meta.items()
                          if k not in ("ch", "split_input", "step", "in_scale", "out_scale")}
        return net


WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")
WEIGHTS = os.path.join(WEIGHTS_DIR, "warmstart_64x64x32.npz")


def load_default(device="cuda") -> "UNet":
    """The shipped network trained on the 64 x 64 x 32-layer, 256-bin
    geometry (the checkpoint's metadata holds the recipe)."""
    return UNet.load(WEIGHTS, device=device)


def load_all(device="cuda") -> Dict[int, "UNet"]:
    """Every shipped network, keyed by the layer count it was trained on
    (files warmstart_64x64x<nz>.npz); each runs fully convolutionally on
    any lateral size divisible by 8."""
    nets = {}
    for f in sorted(os.listdir(WEIGHTS_DIR)):
        if f.startswith("warmstart_64x64x") and f.endswith(".npz"):
            nz = int(f[len("warmstart_64x64x"):-4])
            nets[nz] = UNet.load(os.path.join(WEIGHTS_DIR, f), device=device)
    return nets


# ---- data and warm start -------------------------------------------------------------

def warm_start_volumes(net, kernels, ds, taus, max_batch: int = 16, stream=None):
    """Start volumes for a list of scans: the back-projection A^T d of each
    scan, scaled by its class's tau, run through the network in batches of
    one grid shape (at most max_batch scans per batch).  `net` is one UNet
    or a dict {layer count: UNet}.  A layer count without its own network
    but twice one that has one is started through that network on the
    pair-summed back-projection (tau halved), its output repeated into both
    sub-layers; other scans, and grids not divisible by 8, start from zero."""
    torch = _torch()
    out = [None] * len(ds)
    groups: Dict[tuple, List[int]] = {}
    for i, k in enumerate(kernels):
        inf = k.info
        groups.setdefault((inf.nz, inf.ny, inf.nx), []).append(i)
    for (nz, ny, nx), idx in groups.items():
        model = net.get(nz) if isinstance(net, dict) else net
        coarse = False
        if model is None and isinstance(net, dict) and nz % 2 == 0 and (nz // 2) in net:
            model, coarse = net[nz // 2], True
        if model is None or (nz // (2 if coarse else 1)) % 8 or ny % 8 or nx % 8:
            for i in idx:
                out[i] = torch.zeros((nz, ny, nx), dtype=torch.float32, device=ds[i].device)
            continue
        for b0 in range(0, len(idx), max_batch):
            part = idx[b0:b0 + max_batch]
            x = torch.empty((len(part), nz, ny, nx), dtype=torch.float32, device=model.device)
            for j, i in enumerate(part):
                ctof.adjoint(kernels[i], ds[i], out=x[j], stream=stream)
            if coarse:
                pred = model.predict(nn.depth_resample(x, 0, stream=stream), [0.5 * taus[i] for i in part],
                                     stream=stream)
                pred = nn.depth_resample(pred, 1, stream=stream)
            else:
                pred = model.predict(x, [taus[i] for i in part], stream=stream)
            for j, i in enumerate(part):
                out[i] = pred[j]
    return out
