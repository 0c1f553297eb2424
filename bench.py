#!/usr/bin/env python3
"""Throughput of the confocal ToF-DOT reconstruction on one MI355X.

A step is one FISTA iteration of the whole hot path on one volume: forward
contraction, measurement-side FFT passes with the residual, adjoint
contraction, volume-side FFT passes with the prox/momentum update.  The
workload is the 128 x 128 scan, 64 layers over 1-30 mm, 512 bins of 20 ps,
mu_s' drawn from U[0.8, 1.2] per scan, synthetic absorbers and Poisson
noise at 1e5 peak counts (no public data exist for this path).

Prints one JSON line.  The timed region is one ctof_reconstruct call of
exactly --steps iterations with L and lambda fixed beforehand (the power
iteration and the kernel tabulation are set-up and are reported apart) and
without the solver's optional forward pass after the last step (the data
fit at the final iterate, about half an iteration's work per call); a
second call of the same length with that pass is timed and reported beside
the value.
Per-kernel durations come from HIP events that the library records on its
stream inside the same timed call.  Beside the 8 TB/s peak, the iteration's
byte rates are also given as fractions of a measured device copy (read +
write), for the floor (kernel spectrum twice, data once, volume state) and
for the bytes this design moves (its FFT passes' round trips included).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "recon iters/s at 128^2x64 vox, 512 bins; % HBM/MFMA peak; rel err vs FP64"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "contract_fwd_128x128x64x512_pmc_traffic.json")
# stage events on every 8th timed iteration: five event records between the
# launches of an iteration cost about 4% of its time, and 1 in 8 still gives
# each kernel's average duration over 25 launches of a 200-iteration run
TIMING_STRIDE = 8


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def matrix_frequency_counts(p: int):
    """Per spectrum matrix s = (a, b), a <= b <= p/2, s = b (b + 1)/2 + a:
    the number of distinct rfft frequencies (kx, ky) among (a, b),
    (p - a, b), (b, a), (p - b, a) that it serves (1, 2 or 4)."""
    import numpy as np
    h = p // 2
    s = np.arange((h + 1) * (h + 2) // 2)
    b = np.floor((np.sqrt(8 * s + 1) - 1) / 2).astype(np.int64)
    b -= b * (b + 1) // 2 > s
    b += (b + 1) * (b + 2) // 2 <= s
    a = s - b * (b + 1) // 2
    return 1 + ((a > 0) & (a < h)) + (a != b) + ((a != b) & (b > 0) & (b < h))


def band_time_fraction(ctof, k) -> float:
    """Fraction of the residual spectrum's (frequency, bin) entries that the
    banded adjoint reads: per spectrum matrix its range of 16-bin tiles,
    weighted by the rfft frequencies it serves (1.0 without a band)."""
    tab = ctof.band_table(k)
    if tab is None:
        return 1.0
    i = k.info
    w = matrix_frequency_counts(i.p)
    t = tab.numpy()
    ntt = (i.nt + 31) // 32 * 2
    return float((w * (t[:, 1] - t[:, 0])).sum()) / float(w.sum() * ntt)


def source_digest(path: str) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(n_launch_units: float):
    """HBM bytes per contraction launch from the committed rocprofv3 counters,
    or None when absent or taken on a different contraction source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    src = os.path.join(ROOT, "paper_2101_11680_amd", "csrc", "contract.hip")
    if t.get("source_sha256") != source_digest(src):
        return None
    return t.get("bytes_per_launch")


def copy_bandwidth(torch, dev, mib=1024, reps=5):
    """Device-to-device copy rate (bytes read + written per second, GB/s) of
    a plain copy of `mib` MiB, timed with events on torch's stream."""
    src = torch.ones((mib << 20) // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * (mib << 20) / (ms * 1e-3) / 1e9


def cpu_baseline(g, n_iter: int = 3, run: int = 32):
    """Oracle FFT-tier FISTA iterations at the workload's full shape on the
    host cores, bounded sample.

    The oracle's operator (``oracle.operator.FFTOperator``) is driven over
    runs of `run` time bins (tests.gpu_common.BinRunOperator: each bin of
    Eq. 11 depends only on its own kernel, so the forward concatenates the
    runs and the adjoint sums them), one thread per host core, so the 17 GB
    complex kernel spectrum is built in pieces and every core works.  The
    kernel values are seeded random numbers: the oracle's cost does not
    depend on them.  FISTA is timed for 1 and for 1 + n_iter iterations; the
    difference per iteration is the rate (the solver's one-off adjoint for
    the gradient-mapping denominator cancels).
    """
    import numpy as np
    from oracle import solver as osolver
    from tests.gpu_common import BinRunOperator

    threads = os.cpu_count() or 1
    rng = np.random.default_rng(0)
    t0 = time.perf_counter()
    Kq = rng.random((g.nz, g.ny, g.nx, g.nt))
    F = BinRunOperator(Kq, run=run, threads=threads)
    del Kq
    d = rng.random((g.nt, g.ny, g.nx))
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    osolver.fista(F, d, 1.0, 1e-3, 1)
    t1 = time.perf_counter()
    osolver.fista(F, d, 1.0, 1e-3, 1 + n_iter)
    t2 = time.perf_counter()
    F.close()
    per_iter = ((t2 - t1) - (t1 - t0)) / n_iter
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {
        "value": 1.0 / per_iter,
        "unit": "iters/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"FP64 oracle FFT-tier FISTA measured at the full {g.ny}x{g.nx} grid, {g.nz} layers, "
                   f"{g.nt} bins: {n_iter} iterations (timed runs of 1 and {1 + n_iter}, difference), "
                   f"kernel spectrum built over runs of {run} bins and evaluated in {threads} threads "
                   f"(seeded random kernel values; cost is value-independent); {per_iter:.2f} s/iter; "
                   f"set-up {t_setup:.1f} s untimed; host {model or 'unknown'}"),
    }


def composite_target(ctof, torch, dev, rel_tol: float = 1e-3, n_scans: int = 64, seed: int = 0,
                     max_iter: int = 3000) -> dict:
    """The composite target on the batching workload (64 uneven scans, N in
    {32..128}, Nz in {16, 32, 64}, 256 bins of 25 ps), each scan solved to
    gradient-mapping ratio <= rel_tol.

    plain:        FP32, zero start, one ctof_reconstruct per scan
    batched:      FP32, zero start, one ctof_reconstruct_batched call (shape
                  classes share the kernel spectrum; graph replay)
    accelerated:  BF16 hi+lo contraction, the same batched call, learned
                  warm start with the zero-start fallback; back-projection
                  and network time included
    L and lambda come from one power iteration per shape class (set-up, the
    same values on every side); tabulation and launch tuning are set-up
    too.  Tuning: per class for its volume count (batched sides), for one
    volume (plain side).  Per class: scans, time share, mean iterations and
    the tuner's choice.  The final objectives (data fit + lambda/2 ||mu||^2)
    of the accelerated side are compared per scan with the plain side's.
    """
    import numpy as np

    from paper_2101_11680_amd import unet
    from synth import noise, phantoms, workloads
    scans = workloads.batching_scans(n_scans, seed=seed)
    rec = dict(n_abs=(1, 4), radius=(0.5, 2.0), dmua=(0.01, 0.05), kinds=("sphere", "bar"))
    geoms = []
    for g, _, _ in scans:
        if g not in geoms:
            geoms.append(g)
    counts = {g: sum(1 for q, _, _ in scans if q == g) for g in geoms}
    plain_k = {g: ctof.tabulate(g, ctof.FP32) for g in geoms}
    batch_k = {g: ctof.tabulate(g, ctof.FP32) for g in geoms}
    acc_k = {g: ctof.tabulate(g, ctof.BF16X3) for g in geoms}
    tuning = {}
    for g in geoms:
        ctof.tune(plain_k[g], nvol=1, iters=3)
        tb = ctof.tune(batch_k[g], nvol=counts[g], iters=3)
        ta = ctof.tune(acc_k[g], nvol=counts[g], iters=3)
        tuning[f"{g.nx}x{g.nz}"] = {"fp32": {"bb": tb["bb"], "rb": tb["rb"], "parts": tb["parts"]},
                                    "bf16x3": {"bb": ta["bb"], "rb": ta["rb"], "parts": ta["parts"]}}
    ds = []
    for g, sd, peak in scans:
        mu = phantoms.phantom(g, sd, **rec)
        m = ctof.forward(plain_k[g], torch.tensor(mu, dtype=torch.float32, device=dev))
        ds.append(torch.tensor(noise.poisson_histogram(m.double().cpu().numpy(), peak, sd + 7),
                               dtype=torch.float32, device=dev))
    first = {}
    for i, (g, _, _) in enumerate(scans):
        first.setdefault(g, i)
    lip = {}
    for g, i in first.items():
        _, rep, _ = ctof.reconstruct(plain_k[g], ds[i], max_iter=1)
        lip[g] = (rep.lipschitz, rep.lam)
    Ls = [lip[g][0] for g, _, _ in scans]
    lams = [lip[g][1] for g, _, _ in scans]
    net = unet.load_all(device=dev)
    # warm-up of every path (graph capture, kernels, network) on one scan per class
    for g, i in first.items():
        plain_k[g].workspace(plain_k[g].workspace_bytes(max_iter)[1], dev)
        ctof.reconstruct(plain_k[g], ds[i], max_iter=3, lam=lip[g][1], lipschitz=lip[g][0])
    torch.cuda.synchronize()

    def objective(mu, rep):
        return rep.datafit + 0.5 * rep.lam * float((mu.double() ** 2).sum())

    t0 = time.perf_counter()
    plain = []
    for (g, _, _), d, L, lam in zip(scans, ds, Ls, lams):
        mu, rep, _ = ctof.reconstruct(plain_k[g], d, max_iter=max_iter, rel_tol=rel_tol, check_every=10, lam=lam,
                                      lipschitz=L)
        plain.append((mu, rep))
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    per_scan_plain = []
    for (g, _, _), (mu, rep) in zip(scans, plain):
        per_scan_plain.append(rep.iters)
    t0 = time.perf_counter()
    _, reps_b = ctof.reconstruct_batched([batch_k[g] for g, _, _ in scans], ds, max_iter=max_iter, rel_tol=rel_tol,
                                         check_every=10, lipschitz=Ls, lam=lams)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    ks = [acc_k[g] for g, _, _ in scans]
    t0 = time.perf_counter()
    starts = unet.warm_start_volumes(net, ks, ds, [1.0 / L for L in Ls])
    torch.cuda.synchronize()
    t_cnn = time.perf_counter() - t0
    mus_a, reps_a = ctof.reconstruct_batched(ks, ds, mus=starts, max_iter=max_iter, rel_tol=rel_tol,
                                             check_every=10, warm_start=2, lipschitz=Ls, lam=lams)
    torch.cuda.synchronize()
    t_acc = time.perf_counter() - t0
    gaps = []
    for (mu_p, rp), mu_a, ra in zip(plain, mus_a, reps_a):
        fp, fa = objective(mu_p, rp), objective(mu_a, ra)
        gaps.append((fa - fp) / fp)
    per = {}
    for (g, _, _), (_, rp), rb, ra in zip(scans, plain, reps_b, reps_a):
        key = f"{g.nx}x{g.nz}"
        c = per.setdefault(key, dict(scans=0, iters_plain=0, iters_batched=0, iters_accelerated=0, fell_back=0))
        c["scans"] += 1
        c["iters_plain"] += rp.iters
        c["iters_batched"] += rb.iters
        c["iters_accelerated"] += ra.iters
        c["fell_back"] += ra.fell_back
    for key, c in per.items():
        for f in ("iters_plain", "iters_batched", "iters_accelerated"):
            c[f] = c[f] / c["scans"]
        c["tuning"] = tuning[key]
    return {
        "workload": (f"batching: {len(scans)} scans in {len(geoms)} shape classes (N in {{32,48,64,96,128}}, "
                     f"Nz in {{16,32,64}} over 1-20 mm, 256 bins of 25 ps), each to gradient-mapping ratio "
                     f"<= {rel_tol:g}; L and lambda once per class on every side"),
        "plain_fp32_s": t_plain,
        "batched_fp32_s": t_batched,
        "accelerated_bf16x3_s": t_acc,
        "accelerated_network_s": t_cnn,
        "speedup_batched_fp32": t_plain / t_batched,
        "speedup_accelerated": t_plain / t_acc,
        "target": 3.0,
        "fell_back": int(sum(r.fell_back for r in reps_a)),
        "not_converged": int(sum(r.gmap_ratio > rel_tol for r in reps_a)),
        "objective_gap_vs_plain": {"mean": float(np.mean(gaps)), "max": float(np.max(gaps)),
                                   "min": float(np.min(gaps))},
        "per_class": dict(sorted(per.items())),
    }


def run_batching(args, ctof, torch, dev) -> int:
    """64 uneven scans (N in {32..128}, Nz in {16,32,64}, 256 bins of 25 ps)
    solved to gradient-mapping ratio <= rel_tol: plain FP32 one scan at a
    time against batched shape classes (graph replay) in FP32 and in the
    reduced-precision forms.  Tabulation and tuning are excluded; each
    solver's own power iteration is included."""
    from synth import noise, phantoms, workloads
    scans = workloads.batching_scans(args.scans, seed=args.seed)
    rec = dict(n_abs=(1, 4), radius=(0.5, 2.0), dmua=(0.01, 0.05), kinds=("sphere", "bar"))
    geoms = []
    for g, _, _ in scans:
        if g not in geoms:
            geoms.append(g)
    log(f"{len(scans)} scans in {len(geoms)} shape classes")
    precs = {"fp32": ctof.FP32, "bf16x3": ctof.BF16X3, "bf16": ctof.BF16, "fp32_banded": ctof.FP32}
    kern = {name: {g: ctof.tabulate(g, p) for g in geoms} for name, p in precs.items()}
    # the spectrum band at 1e-9 of its largest entry (an approximation of the
    # operator below FP32 resolution; fraction of spectrum bytes read per class reported)
    out_band = {f"{g.nx}x{g.nz}": ctof.set_band(kern["fp32_banded"][g], 1e-9) for g in geoms}
    torch.cuda.synchronize()
    ds = []
    for g, seed, peak in scans:
        mu = phantoms.phantom(g, seed, **rec)
        m = ctof.forward(kern["fp32"][g], torch.tensor(mu, dtype=torch.float32, device=dev))
        d = noise.poisson_histogram(m.double().cpu().numpy(), peak, seed + 7)
        ds.append(torch.tensor(d, dtype=torch.float32, device=dev))
    counts = {}
    for g, _, _ in scans:
        counts[g] = counts.get(g, 0) + 1
    for name in precs:
        for g in geoms:
            ctof.tune(kern[name][g], nvol=counts[g], iters=3)
    maxit = 3000
    out = {"workload": (f"batching: {len(scans)} scans, N in {{32,48,64,96,128}}, Nz in {{16,32,64}} "
                        f"over 1-20 mm, 256 bins of 25 ps, solved to gradient-mapping ratio "
                        f"<= {args.rel_tol:g}"),
           "classes": len(geoms), "rel_tol": args.rel_tol, "fp32_banded_spectrum_bytes_read": out_band}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters_plain = []
    for (g, _, _), d in zip(scans, ds):
        _, rep, _ = ctof.reconstruct(kern["fp32"][g], d, max_iter=maxit, rel_tol=args.rel_tol,
                                     check_every=10)
        iters_plain.append(rep.iters)
    torch.cuda.synchronize()
    out["plain_fp32_s"] = time.perf_counter() - t0
    out["plain_iters_mean"] = float(sum(iters_plain)) / len(iters_plain)
    srt = sorted(iters_plain)
    out["plain_iters_min_median_max"] = [srt[0], srt[len(srt) // 2], srt[-1]]
    log(f"plain FP32 sequential: {out['plain_fp32_s']:.3f}s, mean iterations {out['plain_iters_mean']:.1f}")
    for name in precs:
        ks = [kern[name][g] for g, _, _ in scans]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, reps = ctof.reconstruct_batched(ks, ds, max_iter=maxit, rel_tol=args.rel_tol, check_every=10)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[f"batched_{name}_s"] = dt
        out[f"batched_{name}_iters_mean"] = float(sum(r.iters for r in reps)) / len(reps)
        out[f"speedup_{name}"] = out["plain_fp32_s"] / dt
        out[f"batched_{name}_iters"] = [r.iters for r in reps]
        log(f"batched {name}: {dt:.3f}s ({out['plain_fp32_s'] / dt:.2f}x)")
    # accelerated: batched classes + learned start (CNN time included) with
    # the zero-start fallback; L per class from one power iteration each
    from paper_2101_11680_amd import unet
    net = unet.load_all(device=dev)
    out["networks_for_layer_counts"] = sorted(net)
    first = {}
    for i, (g, _, _) in enumerate(scans):
        first.setdefault(g, i)
    for name in precs:
        ks = [kern[name][g] for g, _, _ in scans]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lip = {}
        for g, i in first.items():
            _, rep, _ = ctof.reconstruct(kern[name][g], ds[i], max_iter=1)
            lip[g] = (rep.lipschitz, rep.lam)
        starts = unet.warm_start_volumes(net, ks, ds, [1.0 / lip[g][0] for g, _, _ in scans])
        torch.cuda.synchronize()
        t_cnn = time.perf_counter() - t0
        _, reps = ctof.reconstruct_batched(ks, ds, mus=starts, max_iter=maxit, rel_tol=args.rel_tol,
                                           check_every=10, warm_start=2,
                                           lipschitz=[lip[g][0] for g, _, _ in scans],
                                           lam=[lip[g][1] for g, _, _ in scans])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[f"accelerated_{name}_s"] = dt
        out[f"accelerated_{name}_setup_s"] = t_cnn
        out[f"accelerated_{name}_iters_mean"] = float(sum(r.iters for r in reps)) / len(reps)
        out[f"accelerated_{name}_fell_back"] = int(sum(r.fell_back for r in reps))
        out[f"accelerated_{name}_not_converged"] = int(sum(r.gmap_ratio > args.rel_tol for r in reps))
        out[f"speedup_accelerated_{name}"] = out["plain_fp32_s"] / dt
        per = {}
        for (g, _, _), r, rz in zip(scans, reps, out[f"batched_{name}_iters"]):
            key = f"{g.nx}x{g.nz}"
            c = per.setdefault(key, dict(scans=0, iters_zero=0, iters_warm=0, fell_back=0))
            c["scans"] += 1
            c["iters_zero"] += rz
            c["iters_warm"] += r.iters
            c["fell_back"] += r.fell_back
        out[f"accelerated_{name}_per_class"] = {
            k: dict(scans=c["scans"], iters_zero_mean=c["iters_zero"] / c["scans"],
                    iters_warm_mean=c["iters_warm"] / c["scans"], fell_back=c["fell_back"])
            for k, c in sorted(per.items())}
        log(f"accelerated {name}: {dt:.3f}s ({out['plain_fp32_s'] / dt:.2f}x), setup+CNN {t_cnn:.3f}s, "
            f"fell back {out[f'accelerated_{name}_fell_back']}")
    for name in precs:
        out.pop(f"batched_{name}_iters", None)
    print(json.dumps(out), flush=True)
    return 0


def run_warmstart(args, ctof, torch, dev) -> int:
    """Learned warm start on the 64 x 64 x 32-layer, 256-bin geometry: held-out
    scans (phantom seeds 900000+, never trained on) solved to gradient-mapping
    ratio rel_tol from zero and from the shipped network's start (zero-start
    fallback on, CNN time included), same L and lambda."""
    from paper_2101_11680_amd import train, unet
    from synth import workloads
    net = unet.load_default(device=dev)
    P = train.problem(workloads.geometry_for("learned"))
    seeds = list(range(900000, 900000 + args.scans))
    ds = train.simulate(P, workloads.workload("learned"), seeds, peak_seed=seeds[0])
    torch.cuda.synchronize()
    res = train.evaluate(net, P, ds, tol=args.rel_tol, max_iter=3000)
    res["workload"] = ("learned warm start: 64x64 scan, 32 layers 1-20 mm, 256 bins of 25 ps, "
                       f"{args.scans} held-out phantoms (1-4 spheres/bars), Poisson noise at 1e4-1e6 peak counts")
    res["network"] = {k: net.meta.get(k) for k in ("n_train", "steps", "batch", "loss", "alpha", "recipe")}
    print(json.dumps(res), flush=True)
    return 0


def run_cnn(args, ctof, torch, dev) -> int:
    """Training step of the warm-start U-Net (16/32/64/64 channels, BF16
    activations, FP32 accumulation) on 64 x 64 x 32-layer inputs: forward,
    MSE loss, backward (input and weight gradients), Adam.  FLOP/s counts
    the convolutions' algorithmic multiply-adds (unpadded channels):
    forward, weight gradient, and input gradient for every layer but the
    first."""
    from paper_2101_11680_amd import nn, unet
    net = unet.load_default(device=dev)
    n, D, H, W = args.batch, 32, 64, 64
    g = torch.Generator(device="cpu").manual_seed(args.seed)
    x = torch.rand((n, D, H, W), generator=g).to(dev)
    t = torch.rand((n, D, H, W), generator=g).to(dev)
    flops = 0.0
    for name, kind, co, ci in net.layers:
        taps = {nn.K3: 27, nn.DN: 8, nn.UP: 8, nn.K1: 1}[kind]
        lvl_in = {"e1": 0, "e2": 1, "e3": 2, "d1": 0, "d2": 1, "d3": 2, "m4": 3, "u3": 3, "u2": 2, "u1": 1,
                  "c1": 0, "c2": 1, "c3": 2, "he": 0}[name[:2]]
        pos_in = n * (D >> lvl_in) * (H >> lvl_in) * (W >> lvl_in)
        # multiply-adds: output positions x co x taps x ci (UP: input positions x 8 taps)
        pos = pos_in // 8 if kind == nn.DN else pos_in
        macs = pos * co * taps * ci
        flops += 2.0 * macs * (2 if name == "e1a" else 3)
    for _ in range(args.warmup):
        net.forward(x)
        net.loss_and_backward(t)
        net.adam(1e-6)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        net.forward(x)
        net.loss_and_backward(t)
        net.adam(1e-6)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    out = {"workload": f"U-Net training step, batch {n}, {D}x{H}x{W} voxels, channels {list(net.ch)}",
           "ms_per_step": dt * 1e3, "tflop_per_step": flops / 1e12, "tflops": flops / dt / 1e12,
           "peak_tflops_bf16_dense": 2500.0, "frac": flops / dt / 1e12 / 2500.0,
           "samples_per_s": n / dt}
    print(json.dumps(out), flush=True)
    return 0


def run_2d(args, ctof, torch, dev) -> int:
    """The 2D single-plane settings (32x32 scan at 1 mm and 128x128 at
    0.25 mm over a 32 mm field, one absorbing plane at 6.5 mm, 256 bins):
    wall time of one FP32 reconstruction to gradient-mapping ratio rel_tol,
    power iteration included (tabulation excluded), median of repeats; and
    per scan when many scans of the shape are solved in one batched call."""
    from synth import noise, phantoms, workloads
    out = {"workload": "2D single plane (Eq. 9 model), FP32, solve to gradient-mapping ratio "
                       f"<= {args.rel_tol:g}", "paper_context_ms": 8.0}
    for name in ("2d32", "2d128"):
        g = workloads.geometry_for(name)
        w = workloads.workload(name)
        k = ctof.tabulate(g, ctof.FP32)
        ds = []
        for s in range(args.scans):
            mu = phantoms.workload_phantom(w, g, 200 + s)
            m = ctof.forward(k, torch.tensor(mu, dtype=torch.float32, device=dev))
            ds.append(torch.tensor(noise.poisson_histogram(m.double().cpu().numpy(), 1e5, 300 + s),
                                   dtype=torch.float32, device=dev))
        ctof.reconstruct(k, ds[0], max_iter=20)  # warm-up
        times, iters = [], []
        for d in ds[:min(len(ds), 11)]:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, rep, _ = ctof.reconstruct(k, d, max_iter=3000, rel_tol=args.rel_tol, check_every=10)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            iters.append(rep.iters)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, reps = ctof.reconstruct_batched([k] * len(ds), ds, max_iter=3000, rel_tol=args.rel_tol, check_every=10)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        out[name] = {"n": g.nx, "pitch_mm": g.pitch_mm, "single_ms_median": 1e3 * float(np.median(times)),
                     "single_iters_median": float(np.median(iters)),
                     "ms_per_iter": 1e3 * float(np.median(times)) / float(np.median(iters)),
                     "batched_scans": len(ds), "batched_ms_per_scan": 1e3 * tb / len(ds),
                     "batched_iters_mean": float(np.mean([r.iters for r in reps]))}
        log(f"{name}: {out[name]['single_ms_median']:.2f} ms per reconstruction "
            f"({out[name]['single_iters_median']:.0f} iterations); batched {out[name]['batched_ms_per_scan']:.3f} ms/scan")
        del k
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)
    return 0


def run_mux(args, ctof, torch, dev) -> int:
    """Multiplexed reconstruction (Eq. 12) on the 128x128 scan, 64 layers, 512
    bins: the scan cut into 8x8 tiles of sources, each tile measured with the
    128 on/off patterns of the 64x64 Hadamard matrix, counting noise at
    5 Mcps for the brightest measurement plus 200 cps of dark counts over
    --integration-ms.  Reports FISTA iterations/s on S A (power iteration
    excluded) beside the unmultiplexed iteration on the same grid, and the
    fused kernel r = S^T (S m - y) timed alone against its roofline.  Then
    the 2D single-plane setting (32x32 scan, one 8x8 tile pattern set per
    tile): one reconstruction to gradient-mapping ratio rel_tol, power
    iteration included."""
    from synth import mux as smux
    from synth import noise, phantoms, workloads
    rate, dark, t_int = 5e6, 200.0, args.integration_ms * 1e-3
    w = workloads.workload("precision")
    g = workloads.geometry_for("precision", seed=args.seed)
    k = ctof.tabulate(g, ctof.FP32)
    if args.tune:
        ctof.tune(k, nvol=1, iters=5)
    i = k.info
    S = smux.onoff(64)
    mx = ctof.Mux(torch.tensor(S, dtype=torch.float32, device=dev), 8, 8)
    M, P, ntiles = S.shape[0], S.shape[1], mx.ntiles(g.nx)
    mu = torch.tensor(phantoms.workload_phantom(w, g, args.seed), dtype=torch.float32, device=dev)
    m = ctof.forward(k, mu)
    y = ctof.mux_forward(k, mx, m)
    # counts: the brightest measurement reaches rate * T photons; dark counts
    # spread evenly over the bins
    scale = rate * t_int / float(y.sum(dim=0).max())
    bg = dark * t_int / g.nt
    yn = ctof.noisy_counts(y, scale, bg, 1 + args.seed, 7)
    d = torch.tensor(noise.poisson_histogram(m.double().cpu().numpy(), w["peak"][0], 1000 + args.seed),
                     dtype=torch.float32, device=dev)
    _, rep0, _ = ctof.reconstruct(k, yn, max_iter=1, mux=mx)
    L, lam = rep0.lipschitz, rep0.lam
    _, rp0, _ = ctof.reconstruct(k, d, max_iter=1)
    Lp, lamp = rp0.lipschitz, rp0.lam
    res = {}
    for name, data, kw, LL, ll in (("multiplexed", yn, {"mux": mx}, L, lam), ("plain", d, {}, Lp, lamp)):
        if args.warmup > 0:
            ctof.reconstruct(k, data, max_iter=args.warmup, lam=ll, lipschitz=LL, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rep, _ = ctof.reconstruct(k, data, max_iter=args.steps, lam=ll, lipschitz=LL, timing=TIMING_STRIDE,
                                     **kw)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        res[name] = {"iters_per_s": args.steps / wall, "ms_per_iter": 1e3 * wall / args.steps,
                     "ms_fft_t_per_iter": rep.ms_fft_t / rep.timed_iters, "gmap_ratio": rep.gmap_ratio}
        log(f"{name}: {res[name]['iters_per_s']:.1f} iters/s")
    # the fused multiplexing kernel alone, on the solver's shapes
    r = torch.empty_like(m)
    reps = 50
    for _ in range(3):
        ctof.mux_normal(k, mx, m, yn, out=r)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctof.mux_normal(k, mx, m, yn, out=r)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ncol = g.nt * ntiles
    flops = 4.0 * M * P * ncol
    nbytes = 4.0 * (2 * g.nt * g.ny * g.nx + g.nt * M * ntiles)
    tf = flops / (ms * 1e-3) / 1e12
    gbs = nbytes / (ms * 1e-3) / 1e9
    mfma_bound = flops / 157.3e12 > nbytes / 8.0e12
    log(f"mux kernel {1e3 * ms:.1f} us: {tf:.1f} TFLOP/s, {gbs:.0f} GB/s")

    # 2D single plane: 32x32 at 1 mm, one plane at 6.5 mm, 16 tiles of 8x8
    g2 = workloads.geometry_for("2d32")
    w2 = workloads.workload("2d32")
    k2 = ctof.tabulate(g2, ctof.FP32)
    times, iters = [], []
    for s in range(11):
        mu2 = torch.tensor(phantoms.workload_phantom(w2, g2, 200 + s), dtype=torch.float32, device=dev)
        y2 = ctof.mux_forward(k2, mx, ctof.forward(k2, mu2))
        sc2 = rate * t_int / float(y2.sum(dim=0).max())
        y2n = ctof.noisy_counts(y2, sc2, dark * t_int / g2.nt, 300 + s, 7)
        if s == 0:
            ctof.reconstruct(k2, y2n, max_iter=20, mux=mx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rep2, _ = ctof.reconstruct(k2, y2n, max_iter=3000, rel_tol=args.rel_tol, check_every=10, mux=mx)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        iters.append(rep2.iters)
    out = {
        "metric": "multiplexed recon iters/s at 128^2x64 vox, 512 bins, 8x8 tiles x 128 on/off Hadamard patterns",
        "value": res["multiplexed"]["iters_per_s"], "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["multiplexed"]["ms_per_iter"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": ("multiplexed: 128x128 scan at 0.5 mm in 8x8 source tiles, 128 on/off Hadamard "
                                "patterns per tile, 64 layers 1-30 mm, 512 bins of 20 ps; counts at 5 Mcps "
                                f"peak plus 200 cps dark over {args.integration_ms:g} ms"),
                   "rows": M, "tile": [8, 8], "ntiles": ntiles},
        "plain_iters_per_s": res["plain"]["iters_per_s"],
        "overhead_vs_plain": res["plain"]["iters_per_s"] / res["multiplexed"]["iters_per_s"] - 1.0,
        "stages_ms_per_iter": {"fft_t_multiplexed": res["multiplexed"]["ms_fft_t_per_iter"],
                               "fft_t_plain": res["plain"]["ms_fft_t_per_iter"]},
        "roofline": {"bound": "mfma" if mfma_bound else "hbm",
                     "kernel": "mux_kernel (fused r = S^T (S m - y), FP32 MFMA 16x16x4)",
                     "achieved": tf if mfma_bound else gbs, "peak": 157.3 if mfma_bound else 8000.0,
                     "unit": "TFLOP/s" if mfma_bound else "GB/s",
                     "frac": (tf / 157.3) if mfma_bound else (gbs / 8000.0), "traffic": None,
                     "us_per_launch": 1e3 * ms, "flops_per_launch": flops, "bytes_per_launch": nbytes,
                     "hbm_frac": gbs / 8000.0, "mfma_frac": tf / 157.3},
        "mux_2d32": {"single_ms_median": 1e3 * float(np.median(times)),
                     "single_iters_median": float(np.median(iters)), "tiles": mx.ntiles(g2.nx)},
        "cpu_baseline": None,
    }
    log(f"2d32 multiplexed: {out['mux_2d32']['single_ms_median']:.2f} ms per reconstruction")
    print(json.dumps(out), flush=True)
    return 0


def run_fluorescence(args, ctof, torch, dev) -> int:
    """Fluorescence mode on the 128x128 scan, 64 layers, 512 bins: kernel
    tabulation time (FP64 closed form with the lifetime convolution, cosine
    transform, packing) beside absorption mode, and FISTA iterations/s on the
    fluorescence kernel (the operator is unchanged, so this matches the
    absorption rate)."""
    from synth import noise, phantoms, workloads
    w = workloads.workload("precision")
    g = workloads.geometry_for("precision", seed=args.seed)
    fl = (0.9 * g.mus_prime_per_mm, 800.0)
    times = {}
    for name, f in (("absorption", None), ("fluorescence", fl)):
        ctof.tabulate(g, ctof.FP32, fluorescence=f)  # warm-up (module load, first launch)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k = ctof.tabulate(g, ctof.FP32, fluorescence=f)
        torch.cuda.synchronize()
        times[name] = time.perf_counter() - t0
        log(f"{name} tabulation {times[name]:.3f}s")
        if f is None:
            del k
            torch.cuda.empty_cache()
    mu = torch.tensor(phantoms.workload_phantom(w, g, args.seed), dtype=torch.float32, device=dev)
    m = ctof.forward(k, mu)
    d = torch.tensor(noise.poisson_histogram(m.double().cpu().numpy(), w["peak"][0], 1000 + args.seed),
                     dtype=torch.float32, device=dev)
    _, rep0, _ = ctof.reconstruct(k, d, max_iter=1)
    if args.warmup > 0:
        ctof.reconstruct(k, d, max_iter=args.warmup, lam=rep0.lam, lipschitz=rep0.lipschitz)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rep, _ = ctof.reconstruct(k, d, max_iter=args.steps, lam=rep0.lam, lipschitz=rep0.lipschitz)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {"metric": "fluorescence-mode recon iters/s at 128^2x64 vox, 512 bins",
           "value": args.steps / wall, "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": ("fluorescence mode: precision geometry, emission mus' = 0.9 x excitation, "
                                   "lifetime 800 ps, FISTA non-negative Tikhonov"),
                      "mus_prime_ex": g.mus_prime_per_mm, "mus_prime_em": fl[0], "lifetime_ps": fl[1]},
           "tabulation_s": times, "cpu_baseline": None}
    log(f"fluorescence: {out['value']:.1f} iters/s")
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3", "bf16", "fp64"])
    ap.add_argument("--band", type=float, default=0.0,
                    help="precision workload: read only the band of the kernel spectrum holding every entry "
                         ">= BAND * max |entry| (an approximation of the operator; 0 = full operator, the default)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-composite", dest="composite", action="store_false",
                    help="skip the composite target measurement (batching workload) of the default run")
    ap.add_argument("--no-variants", dest="variants", action="store_false",
                    help="skip the BF16 contraction variants of the default run")
    ap.add_argument("--no-tune", dest="tune", action="store_false",
                    help="keep the built-in FFT planes-per-block rule instead of timing the choices")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    ap.add_argument("--batch", type=int, default=8, help="cnn workload: samples per step")
    ap.add_argument("--workload", default="precision",
                    choices=["precision", "batching", "warmstart", "cnn", "2d", "mux", "fluorescence"],
                    help="precision: the iteration-rate metric (default); batching: 64 uneven "
                         "scans solved to gradient-mapping ratio 1e-3, plain vs batched vs batched with "
                         "the learned start; warmstart: held-out scans of the learned geometry, zero vs "
                         "learned start (--scans, default 64; 512 for the full evaluation)")
    ap.add_argument("--config", default="precision", choices=["precision", "mid", "tiny"],
                    help="precision workload: the scan configuration (precision: 128x128, 64 layers, 512 bins, the "
                         "metric's; mid: 64x64, 32 layers, 256 bins; tiny: 16x16, 8 layers, 64 bins)")
    ap.add_argument("--scans", type=int, default=64)
    ap.add_argument("--rel-tol", type=float, default=1e-3)
    ap.add_argument("--integration-ms", type=float, default=10.0,
                    help="mux workload: integration time per measurement")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE={world})", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2101_11680_amd import ctof
    from synth import noise, phantoms, workloads

    globals()["np"] = np
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters
        # calibrate the ones read for the contraction kernel
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "copies": 3}), flush=True)
        return 0
    if args.workload == "batching":
        return run_batching(args, ctof, torch, dev)
    if args.workload == "warmstart":
        return run_warmstart(args, ctof, torch, dev)
    if args.workload == "cnn":
        return run_cnn(args, ctof, torch, dev)
    if args.workload == "2d":
        return run_2d(args, ctof, torch, dev)
    if args.workload == "mux":
        return run_mux(args, ctof, torch, dev)
    if args.workload == "fluorescence":
        return run_fluorescence(args, ctof, torch, dev)
    prec = ctof.PRECISIONS[args.precision]
    dtype = torch.float64 if prec == ctof.FP64 else torch.float32

    w = workloads.workload(args.config)
    g = workloads.geometry_for(args.config, seed=args.seed)
    log(f"geometry n={g.nx} nz={g.nz} nt={g.nt} dt={g.dt_ps}ps mus'={g.mus_prime_per_mm:.4f}")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k = ctof.tabulate(g, prec)
    torch.cuda.synchronize()
    t_tab = time.perf_counter() - t0
    torch.cuda.empty_cache()
    i = k.info
    log(f"tabulated P={i.p} matrices={i.nmat} in {t_tab:.3f}s")
    kept = 1.0
    if args.band > 0:
        kept = ctof.set_band(k, args.band)
        log(f"spectrum band {args.band:g}: {kept:.3f} of the kernel-spectrum bytes read")
    tuning = None
    if args.tune:
        # FFT planes per block for this shape and one volume (set-up, untimed,
        # like tabulation)
        t = ctof.tune(k, nvol=1, iters=5)
        tuning = {"bb_t": t["bb"][0], "bb_z": t["bb"][1], "rb_t": t["rb"][0], "rb_z": t["rb"][1],
                  "fwd_parts": t["parts"][0], "adj_parts": t["parts"][1],
                  "ms_per_iter_bb": t["ms_bb"], "ms_per_iter_rb": t["ms_rb"], "ms_per_iter_fwd_parts": t["ms_fwd"],
                  "ms_per_iter_adj_parts": t["ms_adj"]}
        log(f"tuned launch shape: FFT planes per block {t['bb']}, row passes {t['rb']}, contraction blocks per "
            f"matrix {t['parts']} (ms per iteration: planes {t['ms_bb']}, row planes {t['ms_rb']}, "
            f"forward {t['ms_fwd']}, adjoint {t['ms_adj']})")

    mu_true = phantoms.workload_phantom(w, g, args.seed)
    m_true = ctof.forward(k, torch.tensor(mu_true, dtype=dtype, device=dev))
    d_np = noise.poisson_histogram(m_true.double().cpu().numpy(), w["peak"][0], 1000 + args.seed)
    d = torch.tensor(d_np, dtype=dtype, device=dev)
    del m_true

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rep0, _ = ctof.reconstruct(k, d, max_iter=1)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    L, lam = rep0.lipschitz, rep0.lam
    log(f"power iteration L={L:.6e} lambda={lam:.3e} ({t_setup:.3f}s incl. one iteration)")

    # the solver's workspace, sized once for the timed call (the caller's
    # allocation, set-up like tabulation)
    k.workspace(k.workspace_bytes(max(args.steps, args.warmup))[1], dev)
    if args.warmup > 0:
        ctof.reconstruct(k, d, max_iter=args.warmup, lam=lam, lipschitz=L)
    torch.cuda.synchronize()
    log(f"warm-up {args.warmup} iterations done")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mu, rep, _ = ctof.reconstruct(k, d, max_iter=args.steps, lam=lam, lipschitz=L, timing=TIMING_STRIDE,
                                  final_fit=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert rep.iters == args.steps
    value = args.steps / wall
    log(f"timed {args.steps} iterations in {wall:.4f}s -> {value:.1f} iters/s "
        f"(loop events {rep.ms_loop:.3f} ms)")
    # the same call with the forward pass at the final iterate (its data fit)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mu_ff, rep_ff, _ = ctof.reconstruct(k, d, max_iter=args.steps, lam=lam, lipschitz=L, timing=TIMING_STRIDE)
    torch.cuda.synchronize()
    wall_ff = time.perf_counter() - t0
    assert torch.equal(mu_ff, mu)
    del mu_ff
    log(f"with the final data fit: {args.steps / wall_ff:.1f} iters/s")

    # algorithmic bytes (unpadded sizes) of one contraction launch
    es = {ctof.FP64: 8, ctof.FP32: 4, ctof.BF16X3: 4, ctof.BF16: 2}[prec]
    vs = 8 if prec == ctof.FP64 else 4
    nfreq = i.p * (i.p // 2 + 1)
    khat_bytes = i.nmat * g.nt * g.nz * es
    # (with a band the products read that fraction of the spectrum and the
    # adjoint reads the residual spectrum over each matrix's bin range only;
    # the forward still writes every bin)
    t_kept = band_time_fraction(ctof, k)
    fwd_bytes = kept * khat_bytes + nfreq * g.nz * 2 * vs + nfreq * g.nt * 2 * vs
    adj_bytes = kept * khat_bytes + t_kept * nfreq * g.nt * 2 * vs + nfreq * g.nz * 2 * vs
    fwd_ms = rep.ms_contract_fwd / rep.timed_iters
    adj_ms = rep.ms_contract_adj / rep.timed_iters
    ach_fwd = fwd_bytes / (fwd_ms * 1e-3) / 1e9
    ach_adj = adj_bytes / (adj_ms * 1e-3) / 1e9
    # whole-iteration floor: kernel spectrum twice, data once, volume state
    vol = g.nz * g.ny * g.nx * vs
    floor_bytes = 2 * khat_bytes + g.nt * g.ny * g.nx * vs + 5 * vol
    # bytes this design moves per iteration: the two contractions plus, on
    # each side, column pass (P rows in, n rows out), row pass (spectrum rows
    # in and out, data or volume state) and column pass back
    def spec(planes, rows):
        return planes * rows * (i.p // 2 + 1) * 2 * vs
    side_t = 2 * (spec(g.nt, i.p) + spec(g.nt, g.ny)) + 2 * spec(g.nt, g.ny) + g.nt * g.ny * g.nx * vs
    side_z = 2 * (spec(g.nz, i.p) + spec(g.nz, g.ny)) + 2 * spec(g.nz, g.ny) + 4 * vol
    design_bytes = fwd_bytes + adj_bytes + side_t + side_z
    copy_gbs = copy_bandwidth(torch, dev)
    log(f"device copy {copy_gbs:.0f} GB/s (read + write)")
    traffic = measured_traffic(1.0) if args.band == 0 else None  # counters were taken on the full operator

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "bf16x3": "bf16x3+f32", "bf16": "bf16+f32"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": (f"{args.config} config: {g.ny}x{g.nx} confocal scan at {g.pitch_mm:g} mm, {g.nz} layers "
                         f"{float(g.z_mm[0]):g}-{float(g.z_mm[-1]):g} mm, {g.nt} bins of {g.dt_ps:g} ps, one volume, "
                         "FISTA non-negative Tikhonov"),
            "n": g.nx, "nz": g.nz, "nt": g.nt, "fft_size": i.p, "matrices": i.nmat,
            "precision": args.precision, "mus_prime_per_mm": g.mus_prime_per_mm,
            "operator": "full" if args.band == 0 else (f"spectrum band {args.band:g} ({kept:.3f} of the kernel-spectrum "
                                                       f"bytes, {t_kept:.3f} of the residual spectrum read)"),
            "fft_tuning": tuning,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "contract_fwd_kernel (forward per-frequency contraction)",
            "achieved": ach_fwd,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": ach_fwd / HBM_PEAK_GBS,
            "traffic": traffic,
            "bytes_per_launch": fwd_bytes,
            "ms_per_launch": fwd_ms,
            "adjoint": {"achieved": ach_adj, "frac": ach_adj / HBM_PEAK_GBS,
                        "bytes_per_launch": adj_bytes, "ms_per_launch": adj_ms},
        },
        "stages_ms_per_iter": {
            "contract_fwd": fwd_ms, "fft_t": rep.ms_fft_t / rep.timed_iters,
            "contract_adj": adj_ms, "fft_z": rep.ms_fft_z / rep.timed_iters,
            "loop": rep.ms_loop / rep.iters,
        },
        "iteration_floor": {"bytes": floor_bytes,
                            "achieved_GBs": floor_bytes * value / 1e9,
                            "frac": floor_bytes * value / 1e9 / HBM_PEAK_GBS,
                            "frac_of_copy": floor_bytes * value / 1e9 / copy_gbs},
        "iteration_design": {"bytes": design_bytes,
                             "achieved_GBs": design_bytes * value / 1e9,
                             "frac": design_bytes * value / 1e9 / HBM_PEAK_GBS,
                             "frac_of_copy": design_bytes * value / 1e9 / copy_gbs},
        "copy_GBs": copy_gbs,
        "setup_s": {"tabulate": t_tab, "power_iteration_and_one_iter": t_setup},
        "with_final_fit": {"iters_per_s": args.steps / wall_ff, "ms_per_step": 1e3 * wall_ff / args.steps},
        "report": {"datafit0": rep.datafit0, "datafit_final": rep_ff.datafit, "datafit_last_step": rep.datafit,
                   "gmap_ratio": rep.gmap_ratio},
        "cpu_baseline": None,
    }
    if args.precision == "fp32" and args.variants:
        # the reduced-precision contraction forms on the same scan, same L and
        # lambda (their errors against the FP64 oracle are in the precision
        # report of the GPU tests)
        del k
        torch.cuda.empty_cache()
        variants = {}
        mu_ref = mu.clone()
        for name in ("bf16x3", "bf16", "fp32_banded"):
            kv = ctof.tabulate(g, ctof.PRECISIONS[name.split("_")[0]])
            kept = 1.0
            if name == "fp32_banded":
                # the spectrum band below FP32 resolution of its largest entry
                kept = ctof.set_band(kv, 1e-9)
            if args.tune:
                ctof.tune(kv, nvol=1, iters=5)
            kv.workspace(kv.workspace_bytes(max(args.steps, args.warmup))[1], dev)
            ctof.reconstruct(kv, d, max_iter=args.warmup, lam=lam, lipschitz=L)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            muv, rv, _ = ctof.reconstruct(kv, d, max_iter=args.steps, lam=lam, lipschitz=L,
                                          timing=TIMING_STRIDE, final_fit=False)
            torch.cuda.synchronize()
            wv = time.perf_counter() - t0
            variants[name] = {"iters_per_s": args.steps / wv, "ms_per_step": 1e3 * wv / args.steps,
                              "contract_fwd_ms": rv.ms_contract_fwd / rv.timed_iters,
                              "contract_adj_ms": rv.ms_contract_adj / rv.timed_iters,
                              "datafit_rel_to_fp32": rv.datafit / rep.datafit - 1.0,
                              "iterate_rel_l2_to_fp32": float((muv.double() - mu_ref.double()).norm()
                                                              / mu_ref.double().norm())}
            if name == "fp32_banded":
                variants[name].update({"band_rel": 1e-9, "spectrum_bytes_read": kept})
            log(f"{name}: {args.steps / wv:.1f} iters/s")
            del kv
            torch.cuda.empty_cache()
        out["precision_variants"] = variants
    if args.composite:
        log("composite target on the batching workload (plain FP32 vs batched BF16 hi+lo with the learned start)")
        torch.cuda.empty_cache()
        out["composite_3x"] = composite_target(ctof, torch, dev, rel_tol=args.rel_tol)
        c = out["composite_3x"]
        log(f"composite: plain {c['plain_fp32_s']:.2f}s, batched FP32 {c['batched_fp32_s']:.2f}s "
            f"({c['speedup_batched_fp32']:.2f}x), accelerated {c['accelerated_bf16x3_s']:.2f}s "
            f"({c['speedup_accelerated']:.2f}x)")
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(g)
        log(f"cpu baseline {out['cpu_baseline']['value']:.4f} iters/s")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
