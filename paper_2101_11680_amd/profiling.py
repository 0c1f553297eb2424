"""Reduce rocprofv3 output to the short summaries kept with the project.

  python -m paper_2101_11680_amd.profiling trace  DIR OUT.txt TITLE COMMAND
      kernel-trace CSV (rocprofv3 --kernel-trace --stats --output-format csv
      -d DIR -o run) -> per-kernel table (calls, average/min duration, share)
  python -m paper_2101_11680_amd.profiling traffic KERNEL COPY_MIB OUT.json \\
          FETCH_DIR WRITE_DIR COPY_FETCH_DIR COPY_WRITE_DIR COMMAND...
      FETCH_SIZE / WRITE_SIZE counter CSVs (one counter per rocprofv3 --pmc
      run) for a kernel and for a plain device copy of COPY_MIB MiB -> HBM
      bytes per launch of the kernel.  Each counter is scaled by the factor
      that maps the copy's reading to its known size (bytes read = written =
      COPY_MIB MiB), and the result is tied to the source file's digest so
      that a changed kernel is not credited with old counters.
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


def main(argv) -> int:
    if len(argv) >= 5 and argv[0] == "trace":
        print(summarize_trace(argv[1], argv[2], argv[3], " ".join(argv[4:])))
        return 0
    if len(argv) >= 9 and argv[0] == "traffic":
        src = os.path.join(HERE, "csrc", "contract.hip")
        print(json.dumps(traffic(argv[1], int(argv[2]), argv[3], argv[4], argv[5], argv[6], argv[7],
                                 " ".join(argv[8:]), src), indent=1))
        return 0
    print(__doc__)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
