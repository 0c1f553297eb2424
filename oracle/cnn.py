"""FP64 reference for the learned warm start's 3D CNN (test infrastructure).

The network maps the scaled adjoint back-projection tau A^T d of a scan to a
starting volume for the solver (the paper's reconstruction is a regularised
least-squares iteration, section "Reconstruction Algorithm"; a learned
initial guess only changes where it starts).  Everything here is written
from the definitions of the layers, in float64, with plain loops over kernel
taps; nothing is blocked or fused.

Tensors are channels-last: x[n, d, h, w, c].  Layer kinds and weight shapes:

* ``k3``  3x3x3 correlation, stride 1, zero padding 1:  W[co, 3, 3, 3, ci]
          y[b, z, y, x, o] = bias[o] + sum W[o, i, j, k, c] x[b, z+i-1, y+j-1, x+k-1, c]
* ``dn``  2x2x2, stride 2 (down-sampling):              W[co, 2, 2, 2, ci]
          y[b, z, y, x, o] = bias[o] + sum W[o, i, j, k, c] x[b, 2z+i, 2y+j, 2x+k, c]
* ``up``  2x2x2 transposed, stride 2 (up-sampling):      W[2, 2, 2, co, ci]
          y[b, 2z+i, 2y+j, 2x+k, o] = bias[o] + sum_c W[i, j, k, o, c] x[b, z, y, x, c]
* ``k1``  1x1x1:                                         W[co, ci]

Gradients are the transposes of these sums written as scatters (for the
input) and as sums over positions (for the weights), not as derived
convolutions, so they check the GPU's rearranged-weight formulation
independently.

U-Net (4 levels, channels c1..c4): per encoder level two k3 convolutions
with ReLU (the first changes the channel count), the level output kept as a
skip; a dn convolution with ReLU to the next level (channels unchanged);
level 4 is two k3 + ReLU at c4; each decoder level l = 3, 2, 1 applies an
up convolution c_{l+1} -> c_l with ReLU, concatenates [up, skip] along
channels, then two k3 + ReLU (2 c_l -> c_l, c_l -> c_l); a k1 head c1 -> 1
with ReLU makes the output non-negative.

``round_bf16`` rounds float64 values to the nearest bfloat16 (ties to even)
through float32, the storage precision of the GPU's activations, so a
network run here can take the same storage decisions.

Parity unpinned: nothing in the paper fixes the network; the architecture
and its training are this project's design.
"""

from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

KINDS = ("k3", "dn", "up", "k1")


def round_bf16(x):
    """Nearest bfloat16 (ties to even) of float64 values, returned as float64;
    the value is first rounded to float32 (inputs here are float32-exact or
    the rounding to float32 is itself part of the storage model)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    return out.reshape(np.shape(x))


def weight_shape(kind: str, co: int, ci: int) -> Tuple[int, ...]:
    return {"k3": (co, 3, 3, 3, ci), "dn": (co, 2, 2, 2, ci), "up": (2, 2, 2, co, ci), "k1": (co, ci)}[kind]


def out_grid(kind: str, d: int, h: int, w: int) -> Tuple[int, int, int]:
    if kind == "dn":
        return d // 2, h // 2, w // 2
    if kind == "up":
        return 2 * d, 2 * h, 2 * w
    return d, h, w


def conv(kind: str, x, W, bias=None):
    """Forward of one layer (no activation)."""
    x = np.asarray(x, dtype=np.float64)
    n, d, h, w, ci = x.shape
    od, oh, ow = out_grid(kind, d, h, w)
    co = W.shape[-2] if kind == "up" else W.shape[0]
    y = np.zeros((n, od, oh, ow, co))
    if kind == "k3":
        xp = np.zeros((n, d + 2, h + 2, w + 2, ci))
        xp[:, 1:-1, 1:-1, 1:-1] = x
        for i in range(3):
            for j in range(3):
                for k in range(3):
                    y += xp[:, i:i + d, j:j + h, k:k + w] @ W[:, i, j, k, :].T
    elif kind == "dn":
        for i in range(2):
            for j in range(2):
                for k in range(2):
                    y += x[:, i::2, j::2, k::2] @ W[:, i, j, k, :].T
    elif kind == "up":
        for i in range(2):
            for j in range(2):
                for k in range(2):
                    y[:, i::2, j::2, k::2] = x @ W[i, j, k].T
    else:
        y = x @ W.T
    if bias is not None:
        y = y + bias
    return y


def conv_backward(kind: str, x, W, dy, need_dx=True):
    """(dx, dW, dbias) of one layer given the upstream gradient dy."""
    x = np.asarray(x, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    n, d, h, w, ci = x.shape
    dW = np.zeros(W.shape)
    dx = np.zeros(x.shape) if need_dx else None
    if kind == "k3":
        xp = np.zeros((n, d + 2, h + 2, w + 2, ci))
        xp[:, 1:-1, 1:-1, 1:-1] = x
        dxp = np.zeros(xp.shape)
        for i in range(3):
            for j in range(3):
                for k in range(3):
                    win = xp[:, i:i + d, j:j + h, k:k + w]
                    dW[:, i, j, k, :] = np.einsum("bzyxo,bzyxc->oc", dy, win)
                    if need_dx:
                        dxp[:, i:i + d, j:j + h, k:k + w] += dy @ W[:, i, j, k, :]
        if need_dx:
            dx = dxp[:, 1:-1, 1:-1, 1:-1].copy()
    elif kind == "dn":
        for i in range(2):
            for j in range(2):
                for k in range(2):
                    dW[:, i, j, k, :] = np.einsum("bzyxo,bzyxc->oc", dy, x[:, i::2, j::2, k::2])
                    if need_dx:
                        dx[:, i::2, j::2, k::2] += dy @ W[:, i, j, k, :]
    elif kind == "up":
        for i in range(2):
            for j in range(2):
                for k in range(2):
                    g = dy[:, i::2, j::2, k::2]
                    dW[i, j, k] = np.einsum("bzyxo,bzyxc->oc", g, x)
                    if need_dx:
                        dx += g @ W[i, j, k]
    else:
        dW = np.einsum("bzyxo,bzyxc->oc", dy, x)
        if need_dx:
            dx = dy @ W
    db = dy.sum(axis=(0, 1, 2, 3))
    return dx, dW, db


def relu(x):
    return np.maximum(x, 0.0)


# ---- U-Net -----------------------------------------------------------------------

def unet_layers(ch=(16, 32, 64, 64), c_in=1) -> List[Tuple[str, str, int, int]]:
    """(name, kind, co, ci) of every layer, in execution order."""
    c1, c2, c3, c4 = ch
    cs = (c1, c2, c3)
    L = []
    prev = c_in
    for lvl, c in enumerate(cs, start=1):
        L.append((f"e{lvl}a", "k3", c, prev))
        L.append((f"e{lvl}b", "k3", c, c))
        L.append((f"d{lvl}", "dn", c, c))
        prev = c
    L.append(("m4a", "k3", c4, prev))
    L.append(("m4b", "k3", c4, c4))
    up_in = c4
    for lvl in (3, 2, 1):
        c = cs[lvl - 1]
        L.append((f"u{lvl}", "up", c, up_in))
        L.append((f"c{lvl}a", "k3", c, 2 * c))
        L.append((f"c{lvl}b", "k3", c, c))
        up_in = c
    L.append(("head", "k1", 1, c1))
    return L


def init_params(ch=(16, 32, 64, 64), seed=0, c_in=1) -> Dict[str, np.ndarray]:
    """He-normal weights (fan-in = taps * ci), zero biases."""
    rng = np.random.default_rng(seed)
    P = {}
    for name, kind, co, ci in unet_layers(ch, c_in):
        taps = {"k3": 27, "dn": 8, "up": 1, "k1": 1}[kind]
        P[name + ".w"] = rng.normal(0.0, np.sqrt(2.0 / (taps * ci)), weight_shape(kind, co, ci))
        P[name + ".b"] = np.zeros(co)
    return P


def unet_forward(P, x, ch=(16, 32, 64, 64), store=None):
    """Network output and the saved activations.  ``store`` (a rounding
    function or None) is applied to the network input and to every hidden
    layer's post-ReLU output; the head's output is returned unrounded."""
    st = store or (lambda a: a)
    acts = {"input": st(np.asarray(x, dtype=np.float64))}
    kinds = {name: kind for name, kind, _, _ in unet_layers(ch, x.shape[-1])}

    def layer(name, inp, rounded=True):
        out = relu(conv(kinds[name], inp, P[name + ".w"], P[name + ".b"]))
        acts[name] = st(out) if rounded else out
        return acts[name]

    h = acts["input"]
    for lvl in (1, 2, 3):
        h = layer(f"e{lvl}a", h)
        h = layer(f"e{lvl}b", h)
        h = layer(f"d{lvl}", h)
    h = layer("m4a", h)
    h = layer("m4b", h)
    for lvl in (3, 2, 1):
        u = layer(f"u{lvl}", h)
        acts[f"cat{lvl}"] = np.concatenate([u, acts[f"e{lvl}b"]], axis=-1)
        h = layer(f"c{lvl}a", acts[f"cat{lvl}"])
        h = layer(f"c{lvl}b", h)
    y = layer("head", h, rounded=False)
    return y, acts


def unet_backward(P, acts, dy, ch=(16, 32, 64, 64), store=None):
    """Gradients of all parameters given d(loss)/d(output).  ``store`` is
    applied to the incoming gradient and to every propagated input gradient;
    where a skip connection joins, the two contributions are summed before
    a single rounding."""
    st = store or (lambda a: a)
    kinds = {name: kind for name, kind, _, _ in unet_layers(ch, acts["input"].shape[-1])}
    G = {}

    def back(name, inp, g_out, need_dx=True, rounded=True):
        # ReLU: gradient passes where the layer's output is positive
        g = np.where(acts[name] > 0.0, g_out, 0.0)
        dx, dW, db = conv_backward(kinds[name], inp, P[name + ".w"], g, need_dx)
        G[name + ".w"] = dW
        G[name + ".b"] = db
        if not need_dx:
            return None
        return st(dx) if rounded else dx

    g = back("head", acts["c1b"], st(np.asarray(dy, dtype=np.float64)))
    skip = {}
    for lvl in (1, 2, 3):
        c = ch[lvl - 1]
        g = back(f"c{lvl}b", acts[f"c{lvl}a"], g)
        gcat = back(f"c{lvl}a", acts[f"cat{lvl}"], g)
        skip[lvl] = gcat[..., c:]
        src = "m4b" if lvl == 3 else f"c{lvl + 1}b"
        g = back(f"u{lvl}", acts[src], gcat[..., :c])
    # g = d loss / d (m4b output)
    g = back("m4b", acts["m4a"], g)
    g = back("m4a", acts["d3"], g)
    for lvl in (3, 2, 1):
        g = st(back(f"d{lvl}", acts[f"e{lvl}b"], g, rounded=False) + skip[lvl])
        g = back(f"e{lvl}b", acts[f"e{lvl}a"], g)
        prev = "input" if lvl == 1 else f"d{lvl - 1}"
        g = back(f"e{lvl}a", acts[prev], g, need_dx=(lvl > 1))
    return G


def mse(y, t):
    """(mean squared error, its gradient) over all elements."""
    diff = np.asarray(y, dtype=np.float64) - np.asarray(t, dtype=np.float64)
    return float(np.mean(diff * diff)), 2.0 * diff / diff.size


def adam_step(w, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) with bias correction; returns
    (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
