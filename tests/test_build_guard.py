"""The build's resource check (no GPU): kernels that need a dynamic stack
fail the build, and so do hot-path kernels with scratch memory."""

import os
import shutil
import subprocess

import pytest

from paper_2101_11680_amd import build


def _compile(tmp_path, name, body):
    src = tmp_path / name
    src.write_text(body)
    if not (shutil.which("hipcc") or os.path.exists("/opt/rocm/bin/hipcc")):
        pytest.skip("hipcc not available")
    res = subprocess.run([build.hipcc(), *build.FLAGS, "-Rpass-analysis=kernel-resource-usage", "-c", str(src),
                          "-o", str(tmp_path / (name + ".o"))], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    return str(src), res.stderr


RECURSIVE = """
#include <hip/hip_runtime.h>
__device__ __noinline__ int fib(int n) { return n < 2 ? n : fib(n - 1) + fib(n - 2); }
__global__ void k(int *out, int n) { out[threadIdx.x] = fib(n + threadIdx.x); }
"""

SPILLING = """
#include <hip/hip_runtime.h>
__global__ void k(float *out, const int *idx) {
  float a[64];
  for (int i = 0; i < 64; ++i) a[i] = out[i * 64 + threadIdx.x];
  out[threadIdx.x] = a[idx[threadIdx.x] & 63];
}
"""

PLAIN = """
#include <hip/hip_runtime.h>
__global__ void k(float *out) { out[threadIdx.x] *= 2.0f; }
"""


def test_dynamic_stack_fails_the_build(tmp_path):
    src, err = _compile(tmp_path, "rec.hip", RECURSIVE)
    rep = build.resource_report(err)
    assert rep and any(dyn for _, _, dyn in rep)
    with pytest.raises(RuntimeError, match="dynamic stack"):
        build.check_resources(src, err)


def test_scratch_fails_only_on_the_hot_path(tmp_path):
    src, err = _compile(tmp_path, "fft.hip", SPILLING)
    assert any(s and s > 0 for _, s, _ in build.resource_report(err))
    with pytest.raises(RuntimeError, match="scratch"):
        build.check_resources(src, err)
    # the same kernel in a translation unit off the hot path is accepted
    build.check_resources(str(tmp_path / "rng.hip"), err)


def test_plain_kernel_passes(tmp_path):
    src, err = _compile(tmp_path, "contract.hip", PLAIN)
    rep = build.resource_report(err)
    assert rep == [(rep[0][0], 0, False)]
    build.check_resources(src, err)
