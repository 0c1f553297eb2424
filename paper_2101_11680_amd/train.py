"""Training data, training loop and evaluation of the learned warm start.

Data for one geometry are produced on the GPU with the project's own
kernels: a seeded phantom (absorbers voxelised on the host by the seeded
input generator), its histogram m = A mu (forward model of Eq. 11), Poisson
counting noise d = Poisson(s m) / s at a peak count drawn log-uniformly
(Philox sampler), the back-projection A^T d (adjoint), and as target the
regularised reconstruction mu* itself, solved by the batched FISTA to the
same relative residual the warm start is judged at.  Learning mu* (not the
phantom) makes the network predict the point the solver converges to, which
is what shortens the solve.

The network's input is tau A^T d (tau = 1/L, so its scale is that of the
solver's first iterate); in_scale and out_scale (set from a sample of the
training set) keep the BF16 activations near unit size.
"""

from __future__ import annotations

import math
import time
from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np

from . import ctof, nn, unet


def _torch():
    import torch
    return torch


@dataclass
class Problem:
    geometry: object
    kernel: "ctof.Kernel"
    lipschitz: float
    lam: float

    @property
    def tau(self) -> float:
        return 1.0 / self.lipschitz


def problem(geometry, precision=ctof.FP32, device="cuda") -> Problem:
    """Tabulate the kernel and fix L and lambda (power iteration) once."""
    torch = _torch()
    k = ctof.tabulate(geometry, precision, device=device)
    i = k.info
    d = torch.zeros((i.nt, i.ny, i.nx), dtype=torch.float32, device=device)
    _, rep, _ = ctof.reconstruct(k, d, max_iter=1)
    return Problem(geometry, k, rep.lipschitz, rep.lam)


def simulate(P: Problem, workload: dict, seeds, peak_seed: int, device="cuda"):
    """Noisy histograms d (list of float32 [nt, n, n]) for phantom seeds."""
    from synth import phantoms, workloads
    torch = _torch()
    rng = np.random.Generator(np.random.PCG64(peak_seed))
    out = []
    for s in seeds:
        mu = torch.tensor(phantoms.workload_phantom(workload, P.geometry, int(s)), dtype=torch.float32,
                          device=device)
        m = ctof.forward(P.kernel, mu)
        peak = workloads.draw_peak(workload, rng)
        out.append(nn.noisy_histogram(m, peak, seed=0x5EED0000 + int(s), stream_id=int(s) & 0xFFFFFFFF))
    return out


def back_projections(P: Problem, ds, out=None):
    """A^T d for each scan into out[i] (float32 [N, nz, n, n])."""
    torch = _torch()
    i = P.kernel.info
    if out is None:
        out = torch.empty((len(ds), i.nz, i.ny, i.nx), dtype=torch.float32, device=ds[0].device)
    for j, d in enumerate(ds):
        ctof.adjoint(P.kernel, d, out=out[j])
    return out


def solve(P: Problem, ds, tol: float, max_iter: int, starts=None, warm_start: int = 0, batch: int = 64):
    """Batched FISTA (fixed L, lambda) to gradient-mapping ratio <= tol."""
    mus, reps = [], []
    for b0 in range(0, len(ds), batch):
        part = ds[b0:b0 + batch]
        st = None if starts is None else starts[b0:b0 + batch]
        m, r = ctof.reconstruct_batched([P.kernel] * len(part), part, mus=st, max_iter=max_iter, lam=P.lam,
                                        lipschitz=P.lipschitz, rel_tol=tol, check_every=10,
                                        warm_start=warm_start if st is not None else 0)
        mus += m
        reps += r
    return mus, reps


def sample_maxima(x, chunk: int = 64):
    """max |x[b]| per sample (host float64 [N])."""
    out = []
    for b0 in range(0, x.shape[0], chunk):
        part = x[b0:b0 + chunk]
        out.append(nn.absmax(part, part.shape[0]).cpu().numpy().astype(np.float64))
    return np.concatenate(out)


def set_scales(net: "unet.UNet", P: Problem, xs, targets) -> tuple:
    """Per-sample normalisation constants: in_scale = 1 and out_scale =
    median over the training set of max(mu*) / (tau max|A^T d|), so the
    network's output is of order one.  Returns the per-sample maxima of the
    back-projections and of the targets."""
    mx = sample_maxima(xs)
    mt = sample_maxima(targets)
    ok = mx > 0
    net.in_scale = 1.0
    net.out_scale = float(np.median(mt[ok] / (P.tau * mx[ok]))) if ok.any() else 1.0
    return mx, mt


def target_norms(P: Problem, targets, chunk: int = 32):
    """(||H mu*||^2, ||mu*||^2) per target (host float64 [N, 2]), H = A^T A +
    lambda I, from the loss kernel at a zero start."""
    torch = _torch()
    i = P.kernel.info
    V = i.nz * i.ny * i.nx
    N = targets.shape[0]
    out = np.zeros((N, 2))
    y0 = torch.zeros((chunk * V, 1), dtype=torch.float32, device=targets.device)
    g0 = torch.zeros((chunk * V, 8), dtype=torch.bfloat16, device=targets.device)
    terms = torch.zeros((chunk, 2), dtype=torch.float64, device=targets.device)
    for b0 in range(0, N, chunk):
        nb = min(chunk, N - b0)
        nn.warmstart_loss(P.kernel, nb, nn.Slice(y0, 0, 1), 1.0, targets[b0:b0 + nb], [1.0] * nb, [1.0] * nb,
                          P.lam, nn.Slice(g0, 0, 1), terms)
        out[b0:b0 + nb] = terms[:nb].cpu().numpy()
    return out


def train(net: "unet.UNet", P: Problem, xs, targets, steps: int, batch: int = 8, lr: float = 3e-4,
          lr_min: float = 1e-5, warmup: int = 300, seed: int = 0, log_every: int = 100, log=print,
          loss: str = "operator", alpha: float = 1.0, norms=None, maxima=None,
          floor_pct: float = 10.0, robust: bool = False, clip: float = 0.0) -> List[float]:
    """Adam with cosine learning-rate decay on random minibatches.

    loss = "operator": mean over the batch of ||H e||^2 / ||H mu*||^2 +
    alpha ||e||^2 / ||mu*||^2 (e = start - mu*, H = A^T A + lambda I): the
    first term is, to first order, the squared gradient-mapping ratio of the
    start, which decides whether it is kept; the second keeps the weakly
    observed components, where the solver is slow, in the fit.  Both terms
    are 1 for a zero start.  The per-sample norms are floored at their
    floor_pct-th percentile so that scans whose solution is nearly zero do
    not dominate the gradient.  With robust, each sample's loss enters as
    log(1 + loss_b) (its gradient divided by 1 + loss_b, found by a first
    evaluation of the terms), which bounds the pull of a sample the network
    overshoots.  The learning rate rises linearly over `warmup` steps, then
    follows a cosine to lr_min.  With clip > 0 the gradient is scaled to at
    most clip times the running mean of its norm (an exponential average
    over about 50 steps, of the clipped norms), so a rare minibatch that
    would throw the weights far is taken at a bounded step."""
    torch = _torch()
    g = torch.Generator(device="cpu").manual_seed(seed)
    N = xs.shape[0]
    if loss == "operator" and norms is None:
        norms = target_norms(P, targets)
    if maxima is None:
        maxima = sample_maxima(xs)
    if loss == "operator":
        floors = np.percentile(norms, floor_pct, axis=0)
        norms = np.maximum(norms, floors[None, :])
    losses = []
    gnorm_avg, n_clipped = None, 0
    t0 = time.time()
    for step in range(steps):
        idx_h = torch.randint(0, N, (batch,), generator=g)
        idx = idx_h.to(xs.device)
        xb = xs.index_select(0, idx)
        tb = targets.index_select(0, idx)
        mb = maxima[idx_h.numpy()]
        s_in = [net.in_scale / m if m > 0 else 0.0 for m in mb]
        s_out = [net.out_scale * P.tau * m for m in mb]
        net.forward(xb, s_in)
        if loss == "operator":
            nb = norms[idx_h.numpy()]
            w = 1.0 / np.maximum(nb[:, 0], 1e-300)
            v = alpha / np.maximum(nb[:, 1], 1e-300)
            if robust:
                terms = net.loss_terms_operator(P.kernel, tb, w, v, P.lam, s_out).cpu().numpy()
                f = 1.0 / (1.0 + w * terms[:, 0] + v * terms[:, 1])
                w, v = w * f, v * f
            terms = net.loss_and_backward_operator(P.kernel, tb, w, v, P.lam, s_out)
        else:
            raise ValueError(f"unknown loss {loss!r}")
        if step < warmup:
            cur = lr * (step + 1) / warmup
        else:
            ph = (step - warmup) / max(steps - warmup, 1)
            cur = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * ph))
        gscale = 1.0
        if clip > 0.0:
            gn = math.sqrt(float(nn.sumsq(net.grad).item()))
            if gnorm_avg is None:
                gnorm_avg = gn
            limit = clip * gnorm_avg
            if gn > limit > 0.0:
                gscale = limit / gn
                n_clipped += 1
            gnorm_avg = 0.98 * gnorm_avg + 0.02 * gn * gscale
        net.adam(cur, grad_scale=gscale)
        if (step + 1) % log_every == 0 or step == steps - 1:
            if loss == "operator":
                t = terms.cpu().numpy()
                val = float(np.mean(w * t[:, 0] + v * t[:, 1]))
                extra = f" (H-term {np.mean(w * t[:, 0]):.3e}, plain {np.mean(v * t[:, 1]):.3e})"
            else:
                val = float(terms.item())
                extra = ""
            losses.append(val)
            clipped = f" clipped {n_clipped}" if clip > 0.0 else ""
            log(f"train step {step + 1}/{steps} loss {val:.4e}{extra} lr {cur:.2e}{clipped} "
                f"{(time.time() - t0) / (step + 1) * 1e3:.1f} ms/step")
    return losses


def evaluate(net: "unet.UNet", P: Problem, ds, tol: float = 1e-3, max_iter: int = 3000, batch: int = 64) -> Dict:
    """Iterations and wall time to gradient-mapping ratio <= tol from zero and
    from the learned start (warm_start = 2, CNN time included), and the final
    objectives F = 1/2 ||A mu - d||^2 + lambda/2 ||mu||^2 of both."""
    torch = _torch()
    torch.cuda.synchronize()
    t0 = time.time()
    mz, rz = solve(P, ds, tol, max_iter, batch=batch)
    torch.cuda.synchronize()
    t_zero = time.time() - t0
    t0 = time.time()
    starts = []
    for b0 in range(0, len(ds), 16):
        part = ds[b0:b0 + 16]
        starts += unet.warm_start_volumes(net, [P.kernel] * len(part), part, [P.tau] * len(part))
    torch.cuda.synchronize()
    t_cnn = time.time() - t0
    mw, rw = solve(P, ds, tol, max_iter, starts=starts, warm_start=2, batch=batch)
    torch.cuda.synchronize()
    t_warm = time.time() - t0

    def objective(mu, rep):
        v = mu.cpu().numpy().astype(np.float64)
        return rep.datafit + 0.5 * P.lam * float(np.dot(v.ravel(), v.ravel()))

    fz = np.array([objective(m, r) for m, r in zip(mz, rz)])
    fw = np.array([objective(m, r) for m, r in zip(mw, rw)])
    iz = np.array([r.iters for r in rz])
    iw = np.array([r.iters for r in rw])
    return dict(n=len(ds), tol=tol, iters_zero_mean=float(iz.mean()), iters_warm_mean=float(iw.mean()),
                iters_zero_median=float(np.median(iz)), iters_warm_median=float(np.median(iw)),
                iters_ratio=float(iz.sum() / max(iw.sum(), 1)), fell_back=int(sum(r.fell_back for r in rw)),
                not_converged_zero=int(sum(r.gmap_ratio > tol for r in rz)),
                not_converged_warm=int(sum(r.gmap_ratio > tol for r in rw)),
                seconds_zero=t_zero, seconds_warm=t_warm, seconds_cnn=t_cnn,
                time_ratio=t_zero / max(t_warm, 1e-9),
                objective_rel_diff_max=float(np.max((fw - fz) / np.abs(fz))),
                objective_rel_diff_mean=float(np.mean((fw - fz) / np.abs(fz))))


def build_training_set(P: Problem, workload: dict, seeds, tol: float, max_iter: int, chunk: int = 64,
                       log=print):
    """(back-projections, targets) as float32 [N, nz, n, n] device tensors;
    histograms are generated and dropped chunk by chunk."""
    torch = _torch()
    i = P.kernel.info
    N = len(seeds)
    xs = torch.empty((N, i.nz, i.ny, i.nx), dtype=torch.float32, device="cuda")
    ts = torch.empty_like(xs)
    t0 = time.time()
    iters = []
    for b0 in range(0, N, chunk):
        sd = seeds[b0:b0 + chunk]
        ds = simulate(P, workload, sd, peak_seed=int(sd[0]))
        back_projections(P, ds, out=xs[b0:b0 + len(sd)])
        mus, reps = solve(P, ds, tol, max_iter, batch=chunk)
        for j, m in enumerate(mus):
            ts[b0 + j].copy_(m)
        iters += [r.iters for r in reps]
        log(f"data {b0 + len(sd)}/{N}: median iters {int(np.median(iters))} "
            f"{time.time() - t0:.1f} s")
    return xs, ts


def main(argv=None) -> int:
    import argparse
    import json
    import os
    from synth import workloads
    ap = argparse.ArgumentParser(description="train and evaluate the learned warm start")
    ap.add_argument("--workload", default="learned")
    ap.add_argument("--nz", type=int, default=0, help="layer count (0: the workload's own)")
    ap.add_argument("--n-train", type=int, default=20000)
    ap.add_argument("--n-eval", type=int, default=512)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--max-iter", type=int, default=3000)
    ap.add_argument("--channels", default="16,32,64,64")
    ap.add_argument("--loss", default="operator", choices=("operator",))
    ap.add_argument("--alpha", type=float, default=1.0)
    ap.add_argument("--robust", action="store_true", help="log(1 + loss) per sample")
    ap.add_argument("--clip", type=float, default=0.0,
                    help="scale the gradient to at most CLIP times its running mean norm (0: off)")
    ap.add_argument("--out", default="warmstart.npz")
    ap.add_argument("--report", default="warmstart_report.json")
    a = ap.parse_args(argv)
    torch = _torch()
    log = lambda msg: print(msg, flush=True)
    w = workloads.workload(a.workload)
    geom = workloads.geometry_for(a.workload) if a.nz <= 0 else workloads.geometry_with_layers(a.workload, a.nz)
    P = problem(geom)
    log(f"geometry {geom.nx}x{geom.ny}, {geom.nz} layers {geom.z_mm[0]:g}-{geom.z_mm[-1]:g} mm, {geom.nt} bins")
    log(f"problem: L {P.lipschitz:.6e} lambda {P.lam:.6e}")
    train_seeds = list(range(100000, 100000 + a.n_train))
    eval_seeds = list(range(900000, 900000 + a.n_eval))
    xs, ts = build_training_set(P, w, train_seeds, a.tol, a.max_iter, log=log)
    net = unet.UNet(tuple(int(c) for c in a.channels.split(",")), seed=1)
    mx, _ = set_scales(net, P, xs, ts)
    log(f"scales: in {net.in_scale:.4e} out {net.out_scale:.4e}")
    t0 = time.time()
    losses = train(net, P, xs, ts, a.steps, batch=a.batch, lr=a.lr, log=log, loss=a.loss, alpha=a.alpha,
                   maxima=mx, robust=a.robust, clip=a.clip)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    del xs, ts
    os.makedirs(os.path.dirname(a.out) or ".", exist_ok=True)
    net.save(a.out, extra=dict(workload=a.workload, nz=geom.nz, n_train=a.n_train, steps=a.steps, batch=a.batch,
                               tol=a.tol, lipschitz=P.lipschitz, lam=P.lam, loss=a.loss, alpha=a.alpha, lr=a.lr,
                               robust=a.robust, clip=a.clip))
    ds = simulate(P, w, eval_seeds, peak_seed=eval_seeds[0])
    res = evaluate(net, P, ds, tol=a.tol, max_iter=a.max_iter)
    res.update(train_seconds=t_train, train_steps=a.steps, batch=a.batch, n_train=a.n_train,
               losses=losses[-5:], workload=a.workload, loss=a.loss, alpha=a.alpha)
    log(json.dumps(res))
    with open(a.report, "w") as f:
        json.dump(res, f, indent=1)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
