"""Reduce rocprofv3 output to the short summaries kept with the project.

  python -m paper_2101_11680_amd.profiling trace  DIR OUT.txt TITLE COMMAND
      kernel-trace CSV (rocprofv3 --kernel-trace --stats --output-format csv
      -d DIR -o run) -> per-kernel table (calls, average/min duration, share)
  python -m paper_2101_11680_amd.profiling iteration TRACE_DIR FETCH_DIR WRITE_DIR COPY_FETCH_DIR \\
          COPY_WRITE_DIR COPY_MIB MOPS_DIR BUSY_DIR OUT.txt COMMAND...
      the eight stages of an FP32 FISTA iteration picked out of the dispatch
      sequences: duration, calibrated HBM bytes and GB/s per stage, and for the
      contractions SQ_INSTS_VALU_MFMA_MOPS_F32 / SQ_VALU_MFMA_BUSY_CYCLES
  python -m paper_2101_11680_amd.profiling traffic KERNEL COPY_MIB OUT.json \\
          FETCH_DIR WRITE_DIR COPY_FETCH_DIR COPY_WRITE_DIR COMMAND...
      FETCH_SIZE / WRITE_SIZE counter CSVs (one counter per rocprofv3 --pmc
      run) for a kernel and for a plain device copy of COPY_MIB MiB -> HBM
      bytes per launch of the kernel.  Each counter is scaled by the factor
      that maps the copy's reading to its known size (bytes read = written =
      COPY_MIB MiB), and the result is tied to the source file's digest so
      that a changed kernel is not credited with old counters.
  python -m paper_2101_11680_amd.profiling stats STATS_CSV OUT.txt TITLE COMMAND...
      a kernel-stats CSV (rocprofv3 --kernel-trace --stats) -> per-kernel
      totals (calls, total and average duration, share), for runs whose full
      trace is too long to keep
  python -m paper_2101_11680_amd.profiling mfma PMC_DIR STEPS MS_PER_STEP PEAK_TFLOPS OUT.txt TITLE COMMAND...
      one --pmc run holding SQ_INSTS_VALU_MFMA_MOPS_<type> and
      SQ_VALU_MFMA_BUSY_CYCLES over STEPS repetitions of a step that takes
      MS_PER_STEP unprofiled -> executed MFMA TFLOP/s per step against
      PEAK_TFLOPS and the matrix cores' busy share, per kernel and in total
"""

from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def _short(name: str) -> str:
    s = name[name.find("ctof::"):] if "ctof::" in name else name
    s = s.replace("ctof::(anonymous namespace)::", "")
    return s[:s.find("(")] if "(" in s else s


def summarize_trace(d: str, out: str, title: str, command: str) -> str:
    rows = list(csv.DictReader(open(os.path.join(d, "run_kernel_trace.csv"))))
    agg = collections.defaultdict(list)
    meta = {}
    for r in rows:
        key = (_short(r["Kernel_Name"]), r["Grid_Size_X"], r["Grid_Size_Y"])
        agg[key].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1000.0)
        meta[key] = (r["Workgroup_Size_X"], r["VGPR_Count"], r["LDS_Block_Size"])
    tot = sum(sum(v) for v in agg.values())
    lines = [f"# {title}", "", "command (run from /tmp with TMPDIR=/tmp; R = repository root):", f"  {command}", "",
             "rocprofv3 kernel trace, grouped by kernel and grid (durations in microseconds)", "",
             f"{'kernel':58s} {'grid x,y':>16s} {'wg':>4s} {'vgpr':>4s} {'lds':>6s} {'calls':>5s} "
             f"{'avg_us':>10s} {'min_us':>10s} {'share':>6s}"]
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        wg, vg, lds = meta[k]
        lines.append(f"{k[0][:58]:58s} {k[1] + ',' + k[2]:>16s} {wg:>4s} {vg:>4s} {lds:>6s} {len(v):5d} "
                     f"{sum(v) / len(v):10.2f} {min(v):10.2f} {100 * sum(v) / tot:5.1f}%")
    text = "\n".join(lines) + "\n"
    with open(out, "w") as f:
        f.write(text)
    return text


def _counters(d: str):
    path = os.path.join(d, "run_counter_collection.csv")
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        agg[_short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return agg


def _copy_kib(d: str) -> float:
    agg = _counters(d)
    vals = [v for k, vs in agg.items() if "copy" in k.lower() or "elementwise" in k.lower() for v in vs]
    if not vals:
        raise RuntimeError(f"no copy kernel in {d}")
    return max(vals)  # the large copy (3 identical launches)


def traffic(kernel: str, copy_mib: int, out: str, fetch_dir: str, write_dir: str, copy_fetch_dir: str,
            copy_write_dir: str, command: str, source: str) -> dict:
    copy_bytes = copy_mib * (1 << 20)
    f_copy = _copy_kib(copy_fetch_dir)
    w_copy = _copy_kib(copy_write_dir)
    f_fac = copy_bytes / (f_copy * 1024.0)
    w_fac = copy_bytes / (w_copy * 1024.0)
    fk = [v for k, vs in _counters(fetch_dir).items() if k.startswith(kernel) for v in vs]
    wk = [v for k, vs in _counters(write_dir).items() if k.startswith(kernel) for v in vs]
    if not fk or not wk:
        raise RuntimeError(f"kernel {kernel} not found in the counter files")
    fetch = statistics.median(fk) * 1024.0 * f_fac
    write = statistics.median(wk) * 1024.0 * w_fac
    res = dict(kernel=kernel, launches=[len(fk), len(wk)], fetch_kib_median=statistics.median(fk),
               write_kib_median=statistics.median(wk), copy_bytes=copy_bytes, copy_fetch_kib=f_copy,
               copy_write_kib=w_copy, fetch_factor=f_fac, write_factor=w_fac, fetch_bytes_per_launch=fetch,
               write_bytes_per_launch=write, bytes_per_launch=fetch + write,
               source=os.path.relpath(source, os.path.dirname(HERE)),
               source_sha256=hashlib.sha256(open(source, "rb").read()).hexdigest(), command=command)
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
    txt = os.path.splitext(out)[0] + ".txt"
    with open(txt, "w") as f:
        f.write(f"# HBM traffic of {kernel} (rocprofv3 counters, one counter per run)\n\n"
                f"command (run from /tmp with TMPDIR=/tmp; R = repository root):\n  {command}\n\n"
                f"launches measured           {len(fk)} (FETCH_SIZE), {len(wk)} (WRITE_SIZE)\n"
                f"FETCH_SIZE median           {statistics.median(fk):.1f} KiB per launch\n"
                f"WRITE_SIZE median           {statistics.median(wk):.1f} KiB per launch\n"
                f"copy of {copy_mib} MiB: FETCH_SIZE {f_copy:.1f} KiB, WRITE_SIZE {w_copy:.1f} KiB\n"
                f"calibration factors         fetch {f_fac:.4f}, write {w_fac:.4f}\n"
                f"bytes per launch            {fetch:.4e} read + {write:.4e} written = {fetch + write:.4e}\n"
                f"source                      {res['source']} sha256 {res['source_sha256'][:16]}\n")
    return res


FISTA_STAGES = ("contract_fwd", "col_t_inverse", "row_t_residual", "col_t_forward", "contract_adj",
                "col_z_inverse", "row_z_prox", "col_z_forward")
_ADJ = ("contract_adj_kernel<float", "contract_adj_pipe_kernel<float")
_STAGE_KERNELS = ("contract_fwd_kernel<float", "col_pass_kernel<float", "row_pass_kernel<float",
                  "col_pass_kernel<float", _ADJ, "col_pass_kernel<float",
                  "row_pass_kernel<float", "col_pass_kernel<float")


def _dispatches(d: str, counter: bool):
    """[(name, value or duration_us)] in dispatch order."""
    if counter:
        rows = list(csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))))
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        return [(_short(r["Kernel_Name"]), float(r["Counter_Value"])) for r in rows]
    rows = list(csv.DictReader(open(os.path.join(d, "run_kernel_trace.csv"))))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    return [(_short(r["Kernel_Name"]), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1000.0) for r in rows]


def _fista_groups(seq):
    """Values of the eight stages of every FP32 FISTA iteration in a dispatch
    sequence (power-iteration groups end in a reduction, not a column pass)."""
    out = []
    for i in range(len(seq) - 7):
        if all(seq[i + j][0].startswith(_STAGE_KERNELS[j]) for j in range(8)):
            out.append([seq[i + j][1] for j in range(8)])
    return out


def iteration_table(trace_dir, fetch_dir, write_dir, cfetch_dir, cwrite_dir, copy_mib, mops_dir, busy_dir,
                    out, command, clock_hz=2.4e9, simds=1024, hbm_peak=8.0e12, mfma_peak=157.3e12):
    """Per stage of a FISTA iteration: duration (trace), HBM bytes (calibrated
    FETCH_SIZE + WRITE_SIZE), achieved GB/s and share of the HBM peak; for
    the contractions also executed MFMA flops (MOPS x 512), TFLOP/s and the
    MFMA-busy share of the SIMD cycles."""
    copy_bytes = copy_mib * (1 << 20)
    f_fac = copy_bytes / (_copy_kib(cfetch_dir) * 1024.0)
    w_fac = copy_bytes / (_copy_kib(cwrite_dir) * 1024.0)
    med = lambda groups, j: statistics.median(g[j] for g in groups)
    gt = _fista_groups(_dispatches(trace_dir, False))
    gf = _fista_groups(_dispatches(fetch_dir, True))
    gw = _fista_groups(_dispatches(write_dir, True))
    gm = _fista_groups(_dispatches(mops_dir, True))
    gb = _fista_groups(_dispatches(busy_dir, True))
    if not (gt and gf and gw and gm and gb):
        raise RuntimeError("no FISTA iteration found in one of the runs")
    rows = []
    for j, name in enumerate(FISTA_STAGES):
        us = med(gt, j)
        nbytes = med(gf, j) * 1024.0 * f_fac + med(gw, j) * 1024.0 * w_fac
        row = dict(stage=name, us=us, hbm_bytes=nbytes, gbs=nbytes / (us * 1e-6) / 1e9,
                   hbm_frac=nbytes / (us * 1e-6) / hbm_peak)
        if name.startswith("contract"):
            flops = med(gm, j) * 512.0
            row.update(mfma_flops=flops, tflops=flops / (us * 1e-6) / 1e12, mfma_frac=flops / (us * 1e-6) / mfma_peak,
                       mfma_busy=med(gb, j) / (simds * us * 1e-6 * clock_hz))
        rows.append(row)
    tot_us = sum(r["us"] for r in rows)
    tot_b = sum(r["hbm_bytes"] for r in rows)
    lines = ["# FP32 FISTA iteration, 128x128 scan, 64 layers, 512 bins: per-stage HBM and MFMA counters", "",
             "command (run from /tmp with TMPDIR=/tmp; R = repository root):", f"  {command}", "",
             f"iterations found: trace {len(gt)}, FETCH {len(gf)}, WRITE {len(gw)}, MOPS {len(gm)}, BUSY {len(gb)}; "
             f"medians over them", f"HBM bytes = FETCH_SIZE x {f_fac:.4f} + WRITE_SIZE x {w_fac:.4f} (factors from a "
             f"{copy_mib} MiB copy); peaks: HBM 8 TB/s, FP32 MFMA 157.3 TFLOP/s; {simds} SIMDs at "
             f"{clock_hz / 1e9:.1f} GHz", "",
             f"{'stage':16s} {'us':>8s} {'HBM MB':>9s} {'GB/s':>8s} {'%HBM':>6s} {'MFMA TF/s':>10s} {'%MFMA':>6s} "
             f"{'MFMA busy':>9s}"]
    for r in rows:
        extra = (f"{r['tflops']:10.1f} {100 * r['mfma_frac']:5.1f}% {100 * r['mfma_busy']:8.1f}%"
                 if "tflops" in r else f"{'':10s} {'':6s} {'':9s}")
        lines.append(f"{r['stage']:16s} {r['us']:8.1f} {r['hbm_bytes'] / 1e6:9.1f} {r['gbs']:8.0f} "
                     f"{100 * r['hbm_frac']:5.1f}% {extra}")
    lines.append(f"{'iteration':16s} {tot_us:8.1f} {tot_b / 1e6:9.1f} {tot_b / (tot_us * 1e-6) / 1e9:8.0f} "
                 f"{100 * tot_b / (tot_us * 1e-6) / hbm_peak:5.1f}%")
    lines.append("")
    lines.append("MFMA flops are executed flops (MOPS x 512); the contraction fills 8 of the 16 B columns of each "
                 "16x16x4 tile with one volume, so half of them are useful work.")
    text = "\n".join(lines) + "\n"
    with open(out, "w") as f:
        f.write(text)
    with open(os.path.splitext(out)[0] + ".json", "w") as f:
        json.dump(dict(command=command, stages=rows), f, indent=1)
    return text


def summarize_stats(stats_csv: str, out: str, title: str, command: str, top: int = 40) -> str:
    rows = list(csv.DictReader(open(stats_csv)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# {title}", "", "command (run from /tmp with TMPDIR=/tmp; R = repository root):", f"  {command}", "",
             f"rocprofv3 kernel statistics, {len(rows)} kernels, {tot / 1e9:.3f} s of kernel time in all "
             f"(durations in microseconds; the {top} largest totals)", "",
             f"{'kernel':70s} {'calls':>8s} {'total_ms':>10s} {'avg_us':>9s} {'share':>6s}"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:top]:
        lines.append(f"{_short(r['Name'])[:70]:70s} {int(r['Calls']):8d} {float(r['TotalDurationNs']) / 1e6:10.1f} "
                     f"{float(r['AverageNs']) / 1e3:9.1f} {100 * float(r['TotalDurationNs']) / tot:5.1f}%")
    text = "\n".join(lines) + "\n"
    with open(out, "w") as f:
        f.write(text)
    return text


def mfma_table(pmc_dir: str, steps: int, ms_per_step: float, peak_tflops: float, out: str, title: str,
               command: str, clock_hz: float = 2.4e9, simds: int = 1024) -> str:
    """Executed MFMA work per step from one counter run: MOPS x 512 flops and
    the busy cycles of the SIMDs' matrix cores, per kernel name and in total,
    over an unprofiled step time."""
    rows = list(csv.DictReader(open(os.path.join(pmc_dir, "run_counter_collection.csv"))))
    mops = collections.defaultdict(float)
    busy = collections.defaultdict(float)
    mops_name = ""
    for r in rows:
        name, cname, val = _short(r["Kernel_Name"]), r["Counter_Name"], float(r["Counter_Value"])
        if cname.startswith("SQ_INSTS_VALU_MFMA_MOPS"):
            mops[name] += val
            mops_name = cname
        elif cname == "SQ_VALU_MFMA_BUSY_CYCLES":
            busy[name] += val
    t = ms_per_step * 1e-3
    lines = [f"# {title}", "", "command (run from /tmp with TMPDIR=/tmp; R = repository root):", f"  {command}", "",
             f"{mops_name} x 512 = executed MFMA flops; SQ_VALU_MFMA_BUSY_CYCLES over {simds} SIMDs at "
             f"{clock_hz / 1e9:.1f} GHz; per step = counter sums / {steps} steps, over the unprofiled step time "
             f"{ms_per_step:.3f} ms; peak {peak_tflops:g} TFLOP/s", "",
             f"{'kernel':44s} {'GFLOP/step':>11s} {'TFLOP/s':>8s} {'% peak':>7s} {'busy %':>7s}"]
    names = sorted(set(mops) | set(busy), key=lambda n: -mops.get(n, 0.0))
    tot_f = tot_b = 0.0
    for n in names:
        f = mops.get(n, 0.0) * 512.0 / steps
        b = busy.get(n, 0.0) / steps
        if f == 0.0 and b == 0.0:
            continue
        tot_f += f
        tot_b += b
        lines.append(f"{n[:44]:44s} {f / 1e9:11.2f} {f / t / 1e12:8.1f} {100 * f / t / 1e12 / peak_tflops:6.2f}% "
                     f"{100 * b / (simds * clock_hz * t):6.2f}%")
    lines.append(f"{'step total':44s} {tot_f / 1e9:11.2f} {tot_f / t / 1e12:8.1f} "
                 f"{100 * tot_f / t / 1e12 / peak_tflops:6.2f}% {100 * tot_b / (simds * clock_hz * t):6.2f}%")
    text = "\n".join(lines) + "\n"
    with open(out, "w") as fo:
        fo.write(text)
    return text


def main(argv) -> int:
    if len(argv) >= 5 and argv[0] == "trace":
        print(summarize_trace(argv[1], argv[2], argv[3], " ".join(argv[4:])))
        return 0
    if len(argv) >= 9 and argv[0] == "traffic":
        src = os.path.join(HERE, "csrc", "contract.hip")
        print(json.dumps(traffic(argv[1], int(argv[2]), argv[3], argv[4], argv[5], argv[6], argv[7],
                                 " ".join(argv[8:]), src), indent=1))
        return 0
    if len(argv) >= 11 and argv[0] == "iteration":
        print(iteration_table(argv[1], argv[2], argv[3], argv[4], argv[5], int(argv[6]), argv[7], argv[8], argv[9],
                              " ".join(argv[10:])))
        return 0
    if len(argv) >= 5 and argv[0] == "stats":
        print(summarize_stats(argv[1], argv[2], argv[3], " ".join(argv[4:])))
        return 0
    if len(argv) >= 8 and argv[0] == "mfma":
        print(mfma_table(argv[1], int(argv[2]), float(argv[3]), float(argv[4]), argv[5], argv[6],
                         " ".join(argv[7:])))
        return 0
    print(__doc__)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
