"""Build libctof.so (HIP, gfx950) in-tree with hipcc.

Every translation unit under csrc/ is compiled to an object in parallel and
linked into ``paper_2101_11680_amd/libctof.so``.  Packed FP32 vector
instructions are disabled for all device code.

The compiler's per-kernel resource report is checked on every build: no
kernel may need a dynamic stack (a call the compiler could not resolve,
e.g. recursion, gives every kernel that reaches it a private stack whose
size is unknown at launch), and no kernel of the solver's hot path
(FFT passes, contractions, reductions, tabulation) may use scratch memory
(register spills or local arrays), apart from the documented exceptions in
SCRATCH_ALLOWED.  A violation fails the build.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libctof.so")
OBJ = os.path.join(HERE, "_build")

ARCH = os.environ.get("CTOF_OFFLOAD_ARCH", "gfx950")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


# libraries the link needs beyond HIP's own: roctx (named host ranges for
# tracers)
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
LINK = [f"-L{os.path.join(ROCM, 'lib')}", "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}"]

# translation units whose kernels form the solver's hot path
HOT_SOURCES = ("fft.hip", "contract.hip", "solver.hip", "api.hip", "tabulate.hip")
# kernels allowed to use scratch, by a substring of the mangled name, with the reason
SCRATCH_ALLOWED = {
    # FP64 adjoints for 129-256 layers (12 or 16 z tiles of FP64
    # accumulators): parity configurations, not on the FP32/BF16 hot path
    "contract_adj_kernelIdLi12E": "FP64 adjoint with 12 layer tiles",
    "contract_adj_kernelIdLi16E": "FP64 adjoint with 16 layer tiles",
}

_REMARK = re.compile(r"remark:\s+(Function Name|ScratchSize \[bytes/lane\]|Dynamic Stack):\s*(\S+)")


def resource_report(stderr: str):
    """[(kernel, scratch bytes per lane, dynamic stack)] from the compiler's
    kernel-resource-usage remarks."""
    out, cur = [], None
    for line in stderr.splitlines():
        m = _REMARK.search(line)
        if not m:
            continue
        key, val = m.group(1), m.group(2)
        if key == "Function Name":
            cur = [val, None, None]
            out.append(cur)
        elif cur is not None and key.startswith("ScratchSize"):
            cur[1] = int(val)
        elif cur is not None and key.startswith("Dynamic"):
            cur[2] = val == "True"
    return [tuple(x) for x in out]


def check_resources(src: str, stderr: str) -> None:
    name = os.path.basename(src)
    bad = []
    for fn, scratch, dyn in resource_report(stderr):
        if dyn:
            bad.append(f"{fn}: dynamic stack")
        if name in HOT_SOURCES and scratch and not any(a in fn for a in SCRATCH_ALLOWED):
            bad.append(f"{fn}: {scratch} bytes of scratch per lane")
    if bad:
        raise RuntimeError(f"resource check failed for {name}:\n  " + "\n  ".join(bad))


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found; the HIP toolchain is required to build libctof")
    return path


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [hipcc(), *FLAGS, "-Rpass-analysis=kernel-resource-usage", "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stderr}")
    check_resources(src, res.stderr)
    noise = [ln for ln in res.stderr.splitlines()
             if "packed-fp32-ops" not in ln and "kernel-resource-usage" not in ln
             and not ln.lstrip().startswith(("|", "^")) and not re.match(r"^\s*\d+ \|", ln)]
    if noise:
        sys.stderr.write("\n".join(noise) + "\n")
    return obj


def build(jobs: int | None = None) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    jobs = jobs or min(len(srcs), os.cpu_count() or 4, 8)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, *LINK, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build())
