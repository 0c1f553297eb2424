"""The library's host code (argument validation, sizes, errors) under
AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

The boundary's translation units (api.hip, cnn_api.hip) are compiled with
the sanitizers on their host side only (device code is built as usual),
linked with the other translation units into a separate library, and
driven by a C program
(tests/host_validation.c) that calls every validation path reachable
without a GPU: bad geometries, unknown precisions (any 32-bit value a C
caller may pass), NULL and undersized buffers, NULL handles, convolution
descriptors out of range (grids whose row count overflows 64 bits
included).  A sanitizer
report or a wrong status fails the test.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2101_11680_amd")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


def _hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return path if os.path.exists(path) else None


def test_host_validation_under_sanitizers(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    from paper_2101_11680_amd import build as b
    srcs = sorted(f for f in os.listdir(b.CSRC) if f.endswith(".hip"))
    sanitized = ("api.hip", "cnn_api.hip")
    objs = [os.path.join(b.OBJ, f + ".o") for f in srcs if f not in sanitized]
    if not all(os.path.exists(o) for o in objs):
        b.build()
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(hipcc)))
    san_objs = []
    for f in sanitized:
        o = tmp_path / (f + ".san.o")
        res = subprocess.run([hipcc, *b.FLAGS, "-O1", "-g", *SAN, "-Xarch_host", "-fno-omit-frame-pointer", "-c",
                              os.path.join(b.CSRC, f), "-o", str(o)], capture_output=True, text=True)
        assert res.returncode == 0, res.stderr[-4000:]
        san_objs.append(str(o))
    lib = tmp_path / "libctof_san.so"
    res = subprocess.run([hipcc, f"--offload-arch={b.ARCH}", "-shared", "-fPIC", *SAN, *objs, *san_objs, *b.LINK,
                          "-o", str(lib)], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    exe = tmp_path / "host_validation"
    res = subprocess.run([hipcc, "-x", "c", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include"),
                          "-I", os.path.join(ROOT, "include"), *SAN, os.path.join(ROOT, "tests", "host_validation.c"),
                          "-L", str(tmp_path), "-lctof_san", f"-Wl,-rpath,{tmp_path}", "-o", str(exe)],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               HIP_VISIBLE_DEVICES="")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    print(res.stdout, res.stderr[-4000:])
    assert res.returncode == 0, res.stderr[-4000:]
    assert "0 failed" in res.stdout
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr
