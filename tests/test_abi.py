"""C-ABI checks that need no GPU: exported symbols and host-side validation."""

import ctypes
import os
import re

import pytest

from synth.workloads import Geometry, even_layers

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ctof.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ctof_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def ctof():
    from paper_2101_11680_amd import ctof as c
    if not os.path.exists(c.LIB_PATH):
        pytest.skip("libctof.so not built")
    return c


def test_every_declared_symbol_is_exported(ctof):
    lib = ctof.lib()
    names = declared_functions()
    assert "ctof_reconstruct" in names and "ctof_forward" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(ctof.EXPORTS) == set(names)


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2101_11680_amd import ctof as c
    monkeypatch.setattr(c, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(c, "_lib", None)
    with pytest.raises(RuntimeError):
        c.lib()


def _geom(**kw):
    z, dz = even_layers(1.0, 10.0, 4)
    base = dict(nx=16, ny=16, pitch_mm=0.5, z_mm=z, dz_mm=dz, nt=32, dt_ps=25.0)
    base.update(kw)
    return Geometry(**base)


def test_kernel_bytes_sizes(ctof):
    kb32, ws = ctof.kernel_bytes(_geom(), ctof.FP32)
    kb64, _ = ctof.kernel_bytes(_geom(), ctof.FP64)
    kbx3, _ = ctof.kernel_bytes(_geom(), ctof.BF16X3)
    kbh, _ = ctof.kernel_bytes(_geom(), ctof.BF16)
    # P = 32 -> 17*18/2 = 153 matrices, nt padded to 32, nz padded to 16 (32 for bf16)
    assert kb32 == 2 * 153 * 32 * 16 * 4
    assert kb64 == 2 * kb32
    assert kbx3 == 4 * 153 * 32 * 32 * 2
    assert kbh == kbx3 // 2
    assert ws > 0


@pytest.mark.parametrize("bad,status", [
    (dict(nx=0, ny=0), "CTOF_EINVAL"),
    (dict(pitch_mm=0.0), "CTOF_EINVAL"),
    (dict(pitch_mm=float("nan")), "CTOF_EINVAL"),
    (dict(dt_ps=-1.0), "CTOF_EINVAL"),
    (dict(t0_ps=-5.0), "CTOF_EINVAL"),
    (dict(nt=0), "CTOF_EINVAL"),
    (dict(z_mm=(1.0, 3.0, 2.0, 4.0)), "CTOF_EINVAL"),
    (dict(z_mm=(0.0, 1.0, 2.0, 3.0)), "CTOF_EINVAL"),
    (dict(z_mm=(1.0, 2.0, 4.0, 5.0), dz_mm=0.0), "CTOF_EINVAL"),
    (dict(mus_prime_per_mm=0.0), "CTOF_EINVAL"),
    (dict(mua_per_mm=0.0), "CTOF_EINVAL"),
    (dict(n_medium=0.9), "CTOF_EINVAL"),
    (dict(nx=1025, ny=1025), "CTOF_EUNSUPPORTED"),
    (dict(nx=16, ny=1025), "CTOF_EUNSUPPORTED"),
])
def test_geometry_validation(ctof, bad, status):
    with pytest.raises(ctof.CtofError) as ei:
        ctof.kernel_bytes(_geom(**bad), ctof.FP32)
    assert str(ei.value).startswith(status)


def test_single_layer_needs_thickness(ctof):
    g = Geometry(nx=8, ny=8, pitch_mm=1.0, z_mm=(3.0,), dz_mm=0.0, nt=16, dt_ps=50.0)
    with pytest.raises(ctof.CtofError):
        ctof.kernel_bytes(g, ctof.FP32)
    g2 = Geometry(nx=8, ny=8, pitch_mm=1.0, z_mm=(3.0,), dz_mm=1.0, nt=16, dt_ps=50.0)
    assert ctof.kernel_bytes(g2, ctof.FP32)[0] > 0


def test_unknown_precision(ctof):
    with pytest.raises(ctof.CtofError):
        ctof.kernel_bytes(_geom(), 9)


def test_null_arguments_rejected_before_any_launch(ctof):
    lib = ctof.lib()
    gs, _z = ctof._geometry(_geom())
    out = ctypes.c_void_p()
    # NULL device buffers: rejected by validation, no HIP call made
    st = lib.ctof_kernel_tabulate(ctypes.byref(gs), ctof.FP32, None, 1 << 30, None, 1 << 30, None,
                                  ctypes.byref(out))
    assert st == -1
    assert b"NULL" in lib.ctof_last_error()
    # too-small buffers: ENOMEM before any launch
    st = lib.ctof_kernel_tabulate(ctypes.byref(gs), ctof.FP32, ctypes.c_void_p(1 << 20), 16,
                                  ctypes.c_void_p(1 << 20), 16, None, ctypes.byref(out))
    assert st == -2
    assert lib.ctof_forward(None, None, None, None, 0, None) == -1
    assert lib.ctof_reconstruct(None, None, None, None, None, None, 0, None) == -1


def test_non_square_grid_sizes(ctof):
    # ny x nx grids use the FFT size of the longer side on both axes: the
    # spectrum matches the square grid of that side
    kb_sq, _ = ctof.kernel_bytes(_geom(nx=24, ny=24), ctof.FP32)
    kb_ns, _ = ctof.kernel_bytes(_geom(nx=24, ny=9), ctof.FP32)
    kb_ns2, _ = ctof.kernel_bytes(_geom(nx=9, ny=24), ctof.FP32)
    assert kb_ns == kb_sq == kb_ns2


@pytest.mark.parametrize("n,p", [(8, 16), (9, 32), (16, 32), (17, 48), (24, 48), (25, 64), (32, 64), (33, 96),
                                 (48, 96), (49, 128), (64, 128), (65, 192), (96, 192), (97, 256), (128, 256),
                                 (129, 384), (192, 384), (193, 512), (256, 512), (257, 768),
                                 (384, 768), (385, 1024), (512, 1024), (513, 2048)])
def test_fft_size_rule(ctof, n, p):
    # the smallest length >= 2n - 1 among the powers of two (at least 16)
    # and 48, 96, 192, 384, 768; the spectrum holds (p/2 + 1)(p/2 + 2)/2 matrices
    assert max(16, 1 << (2 * n - 2).bit_length()) >= 2 * n - 1
    assert p >= 2 * n - 1
    kb, _ = ctof.kernel_bytes(_geom(nx=n, ny=n), ctof.FP32)
    h = p // 2
    assert kb == 2 * ((h + 1) * (h + 2) // 2) * 32 * 16 * 4
