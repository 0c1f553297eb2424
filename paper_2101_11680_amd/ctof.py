"""Python binding of libctof (ctypes; argument marshalling only).

Every step of the forward model, its adjoint, the kernel tabulation and the
FISTA reconstruction runs in the HIP library; this module allocates device
buffers with torch, passes raw pointers and the current stream, and turns
status codes into exceptions.  It never computes any part of the method and
has no CPU fallback: if the library is missing it raises.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libctof.so")

FP64, FP32, BF16X3, BF16 = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "bf16": BF16}
STATUS = {0: "CTOF_OK", -1: "CTOF_EINVAL", -2: "CTOF_ENOMEM", -3: "CTOF_EHIP",
          -4: "CTOF_ENONFINITE", -5: "CTOF_EUNSUPPORTED", -6: "CTOF_EDIVERGED"}

EXPORTS = ("ctof_kernel_bytes", "ctof_kernel_tabulate", "ctof_kernel_tabulate_quadrant",
           "ctof_kernel_tabulate_fp64_quadrant",
           "ctof_kernel_tabulate_ex", "ctof_kernel_tabulate_quadrant_ex",
           "ctof_kernel_free", "ctof_kernel_info", "ctof_kernel_grid", "ctof_kernel_band_bytes",
           "ctof_kernel_set_band", "ctof_workspace_bytes", "ctof_forward",
           "ctof_adjoint", "ctof_reconstruct", "ctof_workspace_bytes_batched",
           "ctof_reconstruct_batched", "ctof_kernel_set_tuning", "ctof_kernel_get_tuning",
           "ctof_tune_workspace_bytes", "ctof_tune", "ctof_last_error",
           "ctof_conv3d_weight_elems", "ctof_conv3d_fwd", "ctof_conv3d_bwd_data_ws_bytes",
           "ctof_conv3d_bwd_data", "ctof_conv3d_bwd_weight_ws_bytes", "ctof_conv3d_bwd_weight",
           "ctof_relu_bwd", "ctof_mse_ws_bytes", "ctof_mse", "ctof_adam_step",
           "ctof_to_channels_last", "ctof_from_channels_last", "ctof_philox4x32", "ctof_poisson",
           "ctof_noisy_histogram_ws_bytes", "ctof_noisy_histogram", "ctof_warmstart_loss_ws_bytes",
           "ctof_warmstart_loss", "ctof_absmax_ws_bytes", "ctof_absmax", "ctof_depth_resample",
           "ctof_sumsq_ws_bytes", "ctof_sumsq", "ctof_layer_threshold_ws_bytes", "ctof_layer_threshold",
           "ctof_mux_forward", "ctof_mux_adjoint", "ctof_mux_normal_ws_bytes", "ctof_mux_normal",
           "ctof_noisy_counts", "ctof_layer_energy_ws_bytes", "ctof_l1_depth_weights",
           "ctof_forward_noalloc", "ctof_kernel_set_contract_parts", "ctof_kernel_get_contract_parts",
           "ctof_kernel_set_row_tuning", "ctof_kernel_get_row_tuning", "ctof_adam_step_scaled")


class CtofError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class _Geometry(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("pitch_mm", ctypes.c_double),
                ("nz", ctypes.c_int32), ("z_mm", ctypes.POINTER(ctypes.c_double)),
                ("dz_mm", ctypes.c_double), ("nt", ctypes.c_int32), ("dt_ps", ctypes.c_double),
                ("t0_ps", ctypes.c_double), ("mus_prime_per_mm", ctypes.c_double),
                ("mua_per_mm", ctypes.c_double), ("n_medium", ctypes.c_double)]


class _Fluorescence(ctypes.Structure):
    _fields_ = [("mus_prime_em_per_mm", ctypes.c_double), ("lifetime_ps", ctypes.c_double)]


class _Mux(ctypes.Structure):
    _fields_ = [("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32), ("rows", ctypes.c_int32),
                ("s_dev", ctypes.c_void_p)]


class _SolverOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("lambda_tikhonov", ctypes.c_double),
                ("lipschitz", ctypes.c_double), ("power_iters", ctypes.c_int32),
                ("rel_tol", ctypes.c_double), ("check_every", ctypes.c_int32),
                ("warm_start", ctypes.c_int32), ("history_dev", ctypes.c_void_p),
                ("timing", ctypes.c_int32), ("lipschitz_scans", ctypes.POINTER(ctypes.c_double)),
                ("lambda_scans", ctypes.POINTER(ctypes.c_double)),
                ("lambda_l1_z", ctypes.POINTER(ctypes.c_double)),
                ("mux", ctypes.POINTER(_Mux)), ("mu_prev_dev", ctypes.c_void_p),
                ("k0", ctypes.c_int32), ("mu_prev_scans", ctypes.POINTER(ctypes.c_void_p)),
                ("skip_final_fit", ctypes.c_int32)]


class _Tuning(ctypes.Structure):
    _fields_ = [("bb_t", ctypes.c_int32), ("bb_z", ctypes.c_int32), ("fwd_parts", ctypes.c_int32),
                ("adj_parts", ctypes.c_int32), ("ms_bb", ctypes.c_float * 4), ("ms_fwd", ctypes.c_float * 4),
                ("ms_adj", ctypes.c_float * 4), ("rb_t", ctypes.c_int32), ("rb_z", ctypes.c_int32),
                ("ms_rb", ctypes.c_float * 6)]


class _SolverReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("datafit0", ctypes.c_double), ("datafit", ctypes.c_double),
                ("gmap_ratio", ctypes.c_double), ("lipschitz", ctypes.c_double),
                ("lambda_", ctypes.c_double), ("lipschitz_a", ctypes.c_double),
                ("gmap0", ctypes.c_double), ("ms_contract_fwd", ctypes.c_double),
                ("ms_fft_t", ctypes.c_double), ("ms_contract_adj", ctypes.c_double),
                ("ms_fft_z", ctypes.c_double), ("ms_loop", ctypes.c_double),
                ("fell_back", ctypes.c_int32), ("timed_iters", ctypes.c_int32),
                ("fista_k", ctypes.c_int32)]


class _ConvDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int32), ("d", ctypes.c_int32),
                ("h", ctypes.c_int32), ("w", ctypes.c_int32), ("ci", ctypes.c_int32),
                ("co", ctypes.c_int32)]


class _Tensor(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("ld", ctypes.c_int32), ("c0", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libctof.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python paper_2101_11680_amd/build.py`")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32
        gp = ctypes.POINTER(_Geometry)
        L.ctof_kernel_bytes.argtypes = [gp, ctypes.c_int, ctypes.POINTER(sz), ctypes.POINTER(sz)]
        L.ctof_kernel_tabulate.argtypes = [gp, ctypes.c_int, vp, sz, vp, sz, vp, ctypes.POINTER(vp)]
        L.ctof_kernel_tabulate_quadrant.argtypes = [gp, vp, sz, vp]
        L.ctof_kernel_tabulate_fp64_quadrant.argtypes = [gp, vp, vp]
        fp = ctypes.POINTER(_Fluorescence)
        L.ctof_kernel_tabulate_ex.argtypes = [gp, fp, ctypes.c_int, vp, sz, vp, sz, vp, ctypes.POINTER(vp)]
        L.ctof_kernel_tabulate_quadrant_ex.argtypes = [gp, fp, vp, sz, vp]
        L.ctof_kernel_free.argtypes = [vp]
        L.ctof_kernel_free.restype = None
        L.ctof_kernel_info.argtypes = [vp] + [ctypes.POINTER(i32)] * 6
        L.ctof_kernel_grid.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.ctof_kernel_band_bytes.argtypes = [vp, ctypes.POINTER(sz)]
        L.ctof_kernel_set_band.argtypes = [vp, ctypes.c_double, vp, sz, vp]
        L.ctof_workspace_bytes.argtypes = [vp, i32, ctypes.POINTER(sz), ctypes.POINTER(sz)]
        L.ctof_forward.argtypes = [vp, vp, vp, vp, sz, vp]
        L.ctof_adjoint.argtypes = [vp, vp, vp, vp, sz, vp]
        L.ctof_reconstruct.argtypes = [vp, vp, vp, ctypes.POINTER(_SolverOpts),
                                       ctypes.POINTER(_SolverReport), vp, sz, vp]
        kp = ctypes.POINTER(vp)
        L.ctof_workspace_bytes_batched.argtypes = [i32, kp, i32, ctypes.POINTER(sz)]
        L.ctof_reconstruct_batched.argtypes = [i32, kp, kp, kp, ctypes.POINTER(_SolverOpts),
                                               ctypes.POINTER(_SolverReport), vp, sz, vp]
        L.ctof_kernel_set_tuning.argtypes = [vp, i32, i32]
        L.ctof_kernel_get_tuning.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.ctof_tune_workspace_bytes.argtypes = [vp, i32, ctypes.POINTER(sz)]
        L.ctof_tune.argtypes = [vp, i32, i32, vp, sz, vp, ctypes.POINTER(_Tuning)]
        dp = ctypes.POINTER(_ConvDesc)
        tp = ctypes.POINTER(_Tensor)
        i64, u64, u32, f32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_float
        L.ctof_conv3d_weight_elems.argtypes = [dp, ctypes.POINTER(sz)]
        L.ctof_conv3d_fwd.argtypes = [dp, tp, vp, vp, tp, i32, i32, i32, vp]
        L.ctof_conv3d_bwd_data_ws_bytes.argtypes = [dp, ctypes.POINTER(sz)]
        L.ctof_conv3d_bwd_data.argtypes = [dp, tp, vp, tp, i32, vp, sz, vp]
        L.ctof_conv3d_bwd_weight_ws_bytes.argtypes = [dp, ctypes.POINTER(sz)]
        L.ctof_conv3d_bwd_weight.argtypes = [dp, tp, tp, vp, vp, vp, sz, vp]
        L.ctof_relu_bwd.argtypes = [i64, i32, tp, tp, vp]
        L.ctof_mse_ws_bytes.argtypes = [i64, ctypes.POINTER(sz)]
        L.ctof_mse.argtypes = [i64, tp, f32, vp, tp, i32, vp, vp, sz, vp]
        L.ctof_adam_step.argtypes = [i64, vp, vp, vp, vp, vp, f32, f32, f32, f32, i32, vp]
        L.ctof_adam_step_scaled.argtypes = [i64, vp, vp, vp, vp, vp, f32, f32, f32, f32, i32, f32, vp]
        L.ctof_to_channels_last.argtypes = [i64, vp, f32, tp, i32, i32, vp]
        L.ctof_from_channels_last.argtypes = [i64, tp, f32, vp, vp]
        L.ctof_philox4x32.argtypes = [u64, u32, i64, i64, vp, vp]
        L.ctof_poisson.argtypes = [i64, vp, u64, u32, vp, vp]
        L.ctof_noisy_histogram_ws_bytes.argtypes = [i64, ctypes.POINTER(sz)]
        L.ctof_noisy_histogram.argtypes = [i64, vp, ctypes.c_double, u64, u32, vp, vp, sz, vp]
        dptr = ctypes.POINTER(ctypes.c_double)
        L.ctof_warmstart_loss_ws_bytes.argtypes = [vp, i32, ctypes.POINTER(sz)]
        L.ctof_warmstart_loss.argtypes = [vp, i32, tp, dptr, vp, dptr, dptr, ctypes.c_double, i32, tp, vp, vp, sz,
                                          vp]
        L.ctof_absmax_ws_bytes.argtypes = [i32, ctypes.POINTER(sz)]
        L.ctof_absmax.argtypes = [i32, i64, vp, vp, vp, sz, vp]
        L.ctof_depth_resample.argtypes = [i32, i32, i64, vp, vp, i32, vp]
        L.ctof_sumsq_ws_bytes.argtypes = [i32, ctypes.POINTER(sz)]
        L.ctof_sumsq.argtypes = [i32, i64, vp, vp, vp, sz, vp]
        L.ctof_layer_threshold_ws_bytes.argtypes = [i32, ctypes.POINTER(sz)]
        L.ctof_layer_threshold.argtypes = [i32, i64, vp, f32, vp, sz, vp]
        L.ctof_layer_energy_ws_bytes.argtypes = [vp, ctypes.POINTER(sz)]
        L.ctof_forward_noalloc.argtypes = [vp, vp, vp, vp]
        L.ctof_kernel_set_contract_parts.argtypes = [vp, i32, i32]
        L.ctof_kernel_get_contract_parts.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.ctof_kernel_set_row_tuning.argtypes = [vp, i32, i32]
        L.ctof_kernel_get_row_tuning.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.ctof_l1_depth_weights.argtypes = [vp, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_double), vp, sz, vp]
        mp = ctypes.POINTER(_Mux)
        L.ctof_mux_forward.argtypes = [vp, mp, vp, vp, vp]
        L.ctof_mux_adjoint.argtypes = [vp, mp, vp, vp, vp]
        L.ctof_mux_normal_ws_bytes.argtypes = [vp, mp, ctypes.POINTER(sz)]
        L.ctof_mux_normal.argtypes = [vp, mp, vp, vp, vp, vp, vp, sz, vp]
        L.ctof_noisy_counts.argtypes = [i64, vp, ctypes.c_double, ctypes.c_double, u64, u32, vp, vp]
        L.ctof_last_error.argtypes = []
        L.ctof_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name != "ctof_kernel_free" and name != "ctof_last_error":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != 0:
        msg = lib().ctof_last_error().decode(errors="replace")
        raise CtofError(status, msg)


def _geometry(g) -> tuple:
    z = (ctypes.c_double * len(g.z_mm))(*[float(v) for v in g.z_mm])
    s = _Geometry(int(g.nx), int(g.ny), float(g.pitch_mm), len(g.z_mm),
                  ctypes.cast(z, ctypes.POINTER(ctypes.c_double)), float(g.dz_mm), int(g.nt),
                  float(g.dt_ps), float(getattr(g, "t0_ps", 0.0)), float(g.mus_prime_per_mm),
                  float(g.mua_per_mm), float(g.n_medium))
    return s, z  # keep z alive with the struct


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dtype(prec: int):
    torch = _torch()
    return torch.float64 if prec == FP64 else torch.float32


def kernel_bytes(geometry, precision: int) -> tuple:
    gs, _z = _geometry(geometry)
    kb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().ctof_kernel_bytes(ctypes.byref(gs), int(precision), ctypes.byref(kb), ctypes.byref(wb)))
    return kb.value, wb.value


@dataclass
class KernelInfo:
    n: int          # max(ny, nx): the side that sets the FFT size
    nz: int
    nt: int
    p: int
    nmat: int
    precision: int
    ny: int = 0     # scan rows
    nx: int = 0     # scan columns


class Kernel:
    """A tabulated kernel: the host handle plus the device spectrum it refers to."""

    def __init__(self, handle: int, khat, precision: int):
        self._h = ctypes.c_void_p(handle)
        self.khat = khat
        self.precision = precision
        vals = [ctypes.c_int32() for _ in range(6)]
        _check(lib().ctof_kernel_info(self._h, *[ctypes.byref(v) for v in vals]))
        ny, nx = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().ctof_kernel_grid(self._h, ctypes.byref(ny), ctypes.byref(nx)))
        self.info = KernelInfo(*[v.value for v in vals], ny=ny.value, nx=nx.value)
        self._ws = {}
        self._band = None  # device table of the spectrum band, when one is set

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def close(self) -> None:
        if self._h is not None and self._h.value:
            lib().ctof_kernel_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, max_iter: int = 1) -> tuple:
        a, b = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().ctof_workspace_bytes(self._h, int(max_iter), ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def workspace(self, nbytes: int, device, stream=None):
        """The handle's cached workspace of at least nbytes on device, one per
        stream (calls on one stream run in order and may share it; calls on
        different streams may overlap and must not)."""
        torch = _torch()
        key = f"{device}|{_stream_ptr(stream)}"
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
            self._ws[key] = ws
        return ws


def _fluorescence(fl):
    """(mus_prime_em_per_mm, lifetime_ps) -> descriptor pointer, or None (absorption mode)."""
    if fl is None:
        return None
    mus_em, tau = fl
    return ctypes.pointer(_Fluorescence(float(mus_em), float(tau)))


def tabulate(geometry, precision: int = FP32, device="cuda", stream=None, fluorescence=None) -> Kernel:
    """Tabulate the kernel; fluorescence = (emission mus' per mm, lifetime ps)
    for the fluorescence-mode kernel (the geometry's mus' is the excitation one)."""
    torch = _torch()
    gs, _z = _geometry(geometry)
    kb, wb = kernel_bytes(geometry, precision)
    khat = torch.empty(kb, dtype=torch.uint8, device=device)
    ws = torch.empty(max(wb, 256), dtype=torch.uint8, device=device)
    out = ctypes.c_void_p()
    _check(lib().ctof_kernel_tabulate_ex(ctypes.byref(gs), _fluorescence(fluorescence), int(precision),
                                         khat.data_ptr(), kb, ws.data_ptr(), ws.numel(), _stream_ptr(stream),
                                         ctypes.byref(out)))
    del ws
    return Kernel(out.value, khat, precision)


def tabulate_quadrant(geometry, device="cuda", stream=None, fluorescence=None):
    """FP64 kernel values [nz][nt][n][n] for offsets dy, dx >= 0 (test hook)."""
    torch = _torch()
    gs, _z = _geometry(geometry)
    n = max(int(geometry.nx), int(geometry.ny))
    out = torch.empty((len(geometry.z_mm), int(geometry.nt), n, n), dtype=torch.float64, device=device)
    _check(lib().ctof_kernel_tabulate_quadrant_ex(ctypes.byref(gs), _fluorescence(fluorescence), out.data_ptr(),
                                                  out.numel() * 8, _stream_ptr(stream)))
    return out


def _contig(x, dtype, shape):
    if x.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {x.dtype}")
    if tuple(x.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(x.shape)}")
    if not x.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return x


def forward(k: Kernel, mu, out=None, stream=None):
    torch = _torch()
    i = k.info
    mu = _contig(mu, _dtype(k.precision), (i.nz, i.ny, i.nx))
    if out is None:
        out = torch.empty((i.nt, i.ny, i.nx), dtype=mu.dtype, device=mu.device)
    out = _contig(out, mu.dtype, (i.nt, i.ny, i.nx))
    nb, _ = k.workspace_bytes(1)
    ws = k.workspace(nb, mu.device, stream)
    _check(lib().ctof_forward(k.handle, mu.data_ptr(), out.data_ptr(), ws.data_ptr(), ws.numel(),
                              _stream_ptr(stream)))
    return out


def forward_noalloc(k: Kernel, mu, out=None, stream=None):
    """The forward model through ctof_forward_noalloc: the library's fixed
    per-GPU scratch replaces the workspace (raises CtofError with
    CTOF_ENOMEM when the handle's forward needs more than it holds)."""
    torch = _torch()
    i = k.info
    mu = _contig(mu, _dtype(k.precision), (i.nz, i.ny, i.nx))
    if out is None:
        out = torch.empty((i.nt, i.ny, i.nx), dtype=mu.dtype, device=mu.device)
    out = _contig(out, mu.dtype, (i.nt, i.ny, i.nx))
    _check(lib().ctof_forward_noalloc(k.handle, mu.data_ptr(), out.data_ptr(), _stream_ptr(stream)))
    return out


def adjoint(k: Kernel, r, out=None, stream=None):
    torch = _torch()
    i = k.info
    r = _contig(r, _dtype(k.precision), (i.nt, i.ny, i.nx))
    if out is None:
        out = torch.empty((i.nz, i.ny, i.nx), dtype=r.dtype, device=r.device)
    out = _contig(out, r.dtype, (i.nz, i.ny, i.nx))
    nb, _ = k.workspace_bytes(1)
    ws = k.workspace(nb, r.device, stream)
    _check(lib().ctof_adjoint(k.handle, r.data_ptr(), out.data_ptr(), ws.data_ptr(), ws.numel(),
                              _stream_ptr(stream)))
    return out


@dataclass
class Report:
    iters: int
    status: int
    datafit0: float
    datafit: float
    gmap_ratio: float
    lipschitz: float
    lam: float
    lipschitz_a: float
    gmap0: float
    ms_contract_fwd: float = 0.0
    ms_fft_t: float = 0.0
    ms_contract_adj: float = 0.0
    ms_fft_z: float = 0.0
    ms_loop: float = 0.0
    fell_back: int = 0
    timed_iters: int = 0
    fista_k: int = 0


def _l1_array(l1, nz):
    if l1 is None:
        return None
    vals = [float(v) for v in l1]
    if len(vals) != nz:
        raise ValueError(f"need {nz} per-layer L1 weights, got {len(vals)}")
    return (ctypes.c_double * nz)(*vals)


class Mux:
    """Source multiplexing of the measurements (Eq. 12): tiles of tile_x x
    tile_y scan positions combined per time bin by S (rows x tile_x*tile_y),
    held on the device in the data's element type."""

    def __init__(self, S, tile_x: int, tile_y: int):
        if S.dim() != 2 or S.shape[1] != tile_x * tile_y:
            raise ValueError("S must be rows x (tile_x * tile_y)")
        self.S = S.contiguous()
        self.tile_x, self.tile_y = int(tile_x), int(tile_y)
        self.rows = int(S.shape[0])

    def desc(self, k: Kernel) -> _Mux:
        if self.S.dtype != _dtype(k.precision):
            raise TypeError(f"S must be {_dtype(k.precision)} for this kernel")
        return _Mux(self.tile_x, self.tile_y, self.rows, self.S.data_ptr())

    def ntiles(self, ny: int, nx: int | None = None) -> int:
        """Tiles of an ny x nx scan (nx defaults to ny)."""
        nx = ny if nx is None else nx
        return (nx // self.tile_x) * (ny // self.tile_y)


def mux_forward(k: Kernel, mux: Mux, m, out=None, stream=None):
    """y = S m per tile and bin: m [nt][ny][nx] -> y [nt][rows][ntiles]."""
    torch = _torch()
    i = k.info
    m = _contig(m, _dtype(k.precision), (i.nt, i.ny, i.nx))
    shape = (i.nt, mux.rows, mux.ntiles(i.ny, i.nx))
    if out is None:
        out = torch.empty(shape, dtype=m.dtype, device=m.device)
    out = _contig(out, m.dtype, shape)
    desc = mux.desc(k)
    _check(lib().ctof_mux_forward(k.handle, ctypes.byref(desc), m.data_ptr(), out.data_ptr(),
                                  _stream_ptr(stream)))
    return out


def mux_adjoint(k: Kernel, mux: Mux, y, out=None, stream=None):
    """m = S^T y: y [nt][rows][ntiles] -> m [nt][ny][nx]."""
    torch = _torch()
    i = k.info
    y = _contig(y, _dtype(k.precision), (i.nt, mux.rows, mux.ntiles(i.ny, i.nx)))
    if out is None:
        out = torch.empty((i.nt, i.ny, i.nx), dtype=y.dtype, device=y.device)
    out = _contig(out, y.dtype, (i.nt, i.ny, i.nx))
    desc = mux.desc(k)
    _check(lib().ctof_mux_adjoint(k.handle, ctypes.byref(desc), y.data_ptr(), out.data_ptr(),
                                  _stream_ptr(stream)))
    return out


def mux_normal(k: Kernel, mux: Mux, m, y=None, out=None, fit: bool = False, stream=None):
    """r = S^T (S m - y) (y None: S^T S m); returns r, or (r, 1/2 ||S m - y||^2
    as a device float64 scalar) with fit=True.  out may be m itself."""
    torch = _torch()
    i = k.info
    m = _contig(m, _dtype(k.precision), (i.nt, i.ny, i.nx))
    if y is not None:
        y = _contig(y, m.dtype, (i.nt, mux.rows, mux.ntiles(i.ny, i.nx)))
    if out is None:
        out = torch.empty_like(m)
    out = _contig(out, m.dtype, (i.nt, i.ny, i.nx))
    desc = mux.desc(k)
    f = torch.zeros((), dtype=torch.float64, device=m.device) if fit else None
    nb = ctypes.c_size_t()
    _check(lib().ctof_mux_normal_ws_bytes(k.handle, ctypes.byref(desc), ctypes.byref(nb)))
    ws = k.workspace(nb.value, m.device, stream) if fit else None
    _check(lib().ctof_mux_normal(k.handle, ctypes.byref(desc), m.data_ptr(),
                                 y.data_ptr() if y is not None else None, out.data_ptr(),
                                 f.data_ptr() if f is not None else None,
                                 ws.data_ptr() if ws is not None else None, ws.numel() if ws is not None else 0,
                                 _stream_ptr(stream)))
    return (out, f) if fit else out


def noisy_counts(m, scale: float, background: float, seed: int, stream_id: int = 0, out=None, stream=None):
    """(Poisson(scale max(m, 0) + background) - background) / scale, float32."""
    torch = _torch()
    if m.dtype != torch.float32 or not m.is_contiguous():
        raise TypeError("m must be contiguous float32")
    if out is None:
        out = torch.empty_like(m)
    _check(lib().ctof_noisy_counts(m.numel(), m.data_ptr(), float(scale), float(background), int(seed),
                                   int(stream_id), out.data_ptr(), _stream_ptr(stream)))
    return out


def reconstruct(k: Kernel, d, mu=None, max_iter: int = 200, lam: float = -1.0,
                lipschitz: float = 0.0, power_iters: int = 50, rel_tol: float = 0.0,
                check_every: int = 10, warm_start: bool = False, history: bool = False,
                timing: int = 0, l1=None, mux: Optional[Mux] = None, mu_prev=None, k0: int = 0,
                final_fit: bool = True, stream=None):
    """FISTA reconstruction; returns (mu, Report, history or None).  warm_start:
    0/False zero start, 1/True start from ``mu``, 2 start from ``mu`` with the
    zero-start fallback.  l1: per-layer L1 weights (nz numbers) or None.
    mux: a Mux when d holds multiplexed measurements y [nt][rows][ntiles].
    timing: 0 no stage events; n >= 1 (True = 1) events around the stages of
    every n-th iteration, summed in the report's ms_* over timed_iters.
    mu_prev, k0: resumption (a device tensor shaped like mu, in/out): with
    k0 >= 1 (and warm_start = 1) mu holds mu_k0 and mu_prev mu_{k0-1}; on
    return mu_prev holds the iterate before the final one, and the report's
    fista_k is the k0 that resumes the run.  final_fit=False: no forward pass
    after the last step; the report's datafit is then the one at the last
    step's extrapolated point y_K."""
    torch = _torch()
    i = k.info
    if mux is None:
        d = _contig(d, _dtype(k.precision), (i.nt, i.ny, i.nx))
    else:
        d = _contig(d, _dtype(k.precision), (i.nt, mux.rows, mux.ntiles(i.ny, i.nx)))
    if mu is None:
        mu = torch.empty((i.nz, i.ny, i.nx), dtype=d.dtype, device=d.device)
        warm_start = False
    mu = _contig(mu, d.dtype, (i.nz, i.ny, i.nx))
    if mu_prev is not None:
        mu_prev = _contig(mu_prev, d.dtype, (i.nz, i.ny, i.nx))
    hist = torch.zeros((max_iter, 2), dtype=torch.float64, device=d.device) if history else None
    l1a = _l1_array(l1, i.nz)
    mdesc = mux.desc(k) if mux is not None else None
    opts = _SolverOpts(int(max_iter), float(lam), float(lipschitz), int(power_iters),
                       float(rel_tol), int(check_every), int(warm_start),
                       hist.data_ptr() if hist is not None else None, int(timing), None, None, l1a,
                       ctypes.pointer(mdesc) if mdesc is not None else None,
                       mu_prev.data_ptr() if mu_prev is not None else None, int(k0), None,
                       0 if final_fit else 1)
    rep = _SolverReport()
    _, nb = k.workspace_bytes(max_iter)
    ws = k.workspace(nb, d.device, stream)
    _check(lib().ctof_reconstruct(k.handle, d.data_ptr(), mu.data_ptr(), ctypes.byref(opts),
                                  ctypes.byref(rep), ws.data_ptr(), ws.numel(), _stream_ptr(stream)))
    report = _report(rep)
    if hist is not None:
        hist = hist[: rep.iters - rep.fell_back]
    return mu, report, hist


def _report(rep) -> Report:
    return Report(rep.iters, rep.status, rep.datafit0, rep.datafit, rep.gmap_ratio,
                  rep.lipschitz, rep.lambda_, rep.lipschitz_a, rep.gmap0, rep.ms_contract_fwd,
                  rep.ms_fft_t, rep.ms_contract_adj, rep.ms_fft_z, rep.ms_loop, rep.fell_back,
                  rep.timed_iters, rep.fista_k)


def reconstruct_batched(kernels, ds, mus=None, max_iter: int = 200, lam=-1.0, lipschitz=0.0,
                        power_iters: int = 50, rel_tol: float = 0.0, check_every: int = 10,
                        warm_start: bool = False, l1=None, mux: Optional[Mux] = None, mu_prevs=None,
                        k0: int = 0, final_fit: bool = True, stream=None):
    """FISTA for many scans at once; scans sharing a Kernel object form one
    shape class.  lam / lipschitz: one value for all scans or one per scan
    (both sequences, then every scan's pair is used as given).  warm_start as
    in reconstruct.  mux: one Mux for every scan, each ds[i] then holding
    scan i's multiplexed measurements.  mu_prevs, k0: resumption as in
    reconstruct, one mu_prev tensor per scan.  final_fit as in reconstruct.
    Returns (list of mu, list of
    Report)."""
    torch = _torch()
    n = len(ds)
    if len(kernels) != n:
        raise ValueError("one kernel per scan")
    if mus is None:
        mus = [None] * n
        warm_start = False
    outs = []
    for k, d, mu in zip(kernels, ds, mus):
        i = k.info
        if mux is None:
            _contig(d, _dtype(k.precision), (i.nt, i.ny, i.nx))
        else:
            _contig(d, _dtype(k.precision), (i.nt, mux.rows, mux.ntiles(i.ny, i.nx)))
        if mu is None:
            mu = torch.empty((i.nz, i.ny, i.nx), dtype=d.dtype, device=d.device)
        outs.append(_contig(mu, d.dtype, (i.nz, i.ny, i.nx)))
    prev_arr = None
    if mu_prevs is not None:
        if len(mu_prevs) != n:
            raise ValueError("one mu_prev per scan")
        prev_arr = (ctypes.c_void_p * n)(*[
            _contig(p, _dtype(k.precision), (k.info.nz, k.info.ny, k.info.nx)).data_ptr()
            for k, p in zip(kernels, mu_prevs)])
    handles = (ctypes.c_void_p * n)(*[k.handle.value for k in kernels])
    dptr = (ctypes.c_void_p * n)(*[d.data_ptr() for d in ds])
    mptr = (ctypes.c_void_p * n)(*[m.data_ptr() for m in outs])
    nb = ctypes.c_size_t()
    _check(lib().ctof_workspace_bytes_batched(n, handles, int(max_iter), ctypes.byref(nb)))
    ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=ds[0].device)
    per_scan = not isinstance(lipschitz, (int, float))
    l1a = _l1_array(l1, kernels[0].info.nz)
    mdesc = mux.desc(kernels[0]) if mux is not None else None
    mptr_desc = ctypes.pointer(mdesc) if mdesc is not None else None
    if per_scan:
        la = (ctypes.c_double * n)(*[float(x) for x in lipschitz])
        lb = (ctypes.c_double * n)(*[float(x) for x in lam])
        opts = _SolverOpts(int(max_iter), 0.0, 0.0, int(power_iters), float(rel_tol), int(check_every),
                           int(warm_start), None, 0, la, lb, l1a, mptr_desc, None, int(k0), prev_arr,
                           0 if final_fit else 1)
    else:
        opts = _SolverOpts(int(max_iter), float(lam), float(lipschitz), int(power_iters),
                           float(rel_tol), int(check_every), int(warm_start), None, 0, None, None, l1a,
                           mptr_desc, None, int(k0), prev_arr, 0 if final_fit else 1)
    reps = (_SolverReport * n)()
    _check(lib().ctof_reconstruct_batched(n, handles, dptr, mptr, ctypes.byref(opts), reps,
                                          ws.data_ptr(), ws.numel(), _stream_ptr(stream)))
    return outs, [_report(r) for r in reps]


def set_band(k: Kernel, rel: float, stream=None) -> float:
    """Restrict the handle's products to the band of its kernel spectrum
    holding every entry >= rel * max |entry| (rel = 0: full products again).
    Returns the fraction of the forward's kernel-spectrum bytes the products
    still read: per matrix the 16-bin tiles [lo, hi) times the leading
    layers [0, zend) of the band table."""
    torch = _torch()
    if rel == 0.0:
        _check(lib().ctof_kernel_set_band(k.handle, 0.0, None, 0, _stream_ptr(stream)))
        k._band = None
        return 1.0
    nb = ctypes.c_size_t()
    _check(lib().ctof_kernel_band_bytes(k.handle, ctypes.byref(nb)))
    band = torch.zeros(nb.value, dtype=torch.uint8, device="cuda")
    _check(lib().ctof_kernel_set_band(k.handle, float(rel), band.data_ptr(), band.numel(), _stream_ptr(stream)))
    k._band = band  # the handle reads it from now on
    i = k.info
    table = band[: i.nmat * 16].view(torch.int32).view(i.nmat, 4).long()
    ntt = (i.nt + 31) // 32 * 2
    nzp = _layers_packed(i.nz, i.precision)
    kept = ((table[:, 1] - table[:, 0]) * table[:, 2]).sum().item()
    return float(kept) / (i.nmat * ntt * nzp)


def band_table(k: Kernel):
    """The band table of a handle as an (nmat, 3) int64 CPU tensor of
    (lo, hi, zend), or None without a band."""
    if k._band is None:
        return None
    i = k.info
    return k._band[: i.nmat * 16].view(_torch().int32).view(i.nmat, 4)[:, :3].long().cpu()


def _layers_packed(nz: int, prec: int) -> int:
    # layers as the contraction kernels pack them: a multiple of 16 (32 for
    # the BF16 forms) up to 64 layers, of 64 above
    if nz > 64:
        return (nz + 63) // 64 * 64
    m = 32 if prec in (BF16, BF16X3) else 16
    return (nz + m - 1) // m * m


def set_tuning(k: Kernel, bb_t: int, bb_z: int) -> None:
    _check(lib().ctof_kernel_set_tuning(k.handle, int(bb_t), int(bb_z)))
    k._ws = {}


def set_contract_parts(k: Kernel, fwd_parts: int, adj_parts: int) -> None:
    """Blocks per spectrum matrix of the forward / adjoint contraction (0 = rule)."""
    _check(lib().ctof_kernel_set_contract_parts(k.handle, int(fwd_parts), int(adj_parts)))
    k._ws = {}


def set_row_tuning(k: Kernel, rb_t: int, rb_z: int) -> None:
    """Planes per block of the row passes alone (0 = the column passes')."""
    _check(lib().ctof_kernel_set_row_tuning(k.handle, int(rb_t), int(rb_z)))
    k._ws = {}


def get_row_tuning(k: Kernel) -> tuple:
    """The row passes' effective (bin-side, layer-side) planes per block."""
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().ctof_kernel_get_row_tuning(k.handle, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def get_contract_parts(k: Kernel) -> tuple:
    """The effective (forward, adjoint) blocks per spectrum matrix."""
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().ctof_kernel_get_contract_parts(k.handle, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def get_tuning(k: Kernel) -> tuple:
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().ctof_kernel_get_tuning(k.handle, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def tune(k: Kernel, nvol: int = 1, iters: int = 5, cache: Optional[str] = None, stream=None) -> dict:
    """Pick a handle's launch shape for a class of `nvol` volumes by timing
    (ctof_tune: FFT planes per block, the row passes' planes per block, then
    the contractions' blocks per matrix, each judged by the stages it
    changes), with a JSON cache.

    The cache (default: $CTOF_TUNE_CACHE, else no cache) maps
    "arch|grid|nz|nt|precision|nvol" to the choice and its timings.  Returns
    {"bb": (bb_t, bb_z), "rb": (rb_t, rb_z), "parts": (fwd, adj), "ms_bb": [4],
    "ms_rb": [6], "ms_fwd": [4], "ms_adj": [4], "cached": bool} (timings per
    whole iteration; None when taken from the cache).
    """
    import json
    torch = _torch()
    cache = cache if cache is not None else os.environ.get("CTOF_TUNE_CACHE")
    i = k.info
    dev = k.khat.device
    arch = torch.cuda.get_device_properties(dev).gcnArchName.split(":")[0]
    key = f"{arch}|{i.ny}x{i.nx}|{i.nz}|{i.nt}|{i.precision}|{int(nvol)}"
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
        if key in table and "parts" in table[key] and "rb" in table[key]:
            bt, bz = table[key]["bb"]
            rt, rz = table[key]["rb"]
            fp, ap = table[key]["parts"]
            set_tuning(k, bt, bz)
            set_row_tuning(k, rt, rz)
            set_contract_parts(k, fp, ap)
            return {"bb": (bt, bz), "rb": (rt, rz), "parts": (fp, ap), "ms_bb": None, "ms_rb": None,
                    "ms_fwd": None, "ms_adj": None, "cached": True}
    nb = ctypes.c_size_t()
    _check(lib().ctof_tune_workspace_bytes(k.handle, int(nvol), ctypes.byref(nb)))
    ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=dev)
    t = _Tuning()
    _check(lib().ctof_tune(k.handle, int(nvol), int(iters), ws.data_ptr(), ws.numel(), _stream_ptr(stream),
                           ctypes.byref(t)))
    k._ws = {}
    out = {"bb": (t.bb_t, t.bb_z), "rb": (t.rb_t, t.rb_z), "parts": (t.fwd_parts, t.adj_parts),
           "ms_bb": [float(v) for v in t.ms_bb], "ms_rb": [float(v) for v in t.ms_rb],
           "ms_fwd": [float(v) for v in t.ms_fwd], "ms_adj": [float(v) for v in t.ms_adj], "cached": False}
    if cache:
        table[key] = {"bb": list(out["bb"]), "rb": list(out["rb"]), "parts": list(out["parts"]),
                      "ms_bb": out["ms_bb"], "ms_rb": out["ms_rb"], "ms_fwd": out["ms_fwd"], "ms_adj": out["ms_adj"]}
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return out


def _depth_rule(k: Kernel, lam1: float, stream=None):
    import numpy as np
    torch = _torch()
    nz = k.info.nz
    nb = ctypes.c_size_t()
    _check(lib().ctof_layer_energy_ws_bytes(k.handle, ctypes.byref(nb)))
    ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device="cuda")
    e = (ctypes.c_double * nz)()
    w = (ctypes.c_double * nz)()
    _check(lib().ctof_l1_depth_weights(k.handle, float(lam1), e, w, ws.data_ptr(), ws.numel(),
                                       _stream_ptr(stream)))
    return np.array(e[:], dtype=np.float64), [float(v) for v in w]


def layer_energy(k: Kernel, stream=None):
    """Per-layer sensitivity ||A e_z||^2 (host float64 [nz]): the forward
    model's response to a unit absorber at the window centre of each layer,
    squared and summed on the GPU (FP64)."""
    return _depth_rule(k, 0.0, stream)[0]


def l1_depth_weights(k: Kernel, lam1: float, stream=None):
    """Per-layer L1 weights lam1 * e(z) / max e(z), e(z) = ||A e_z||^2, from
    the library (Eq. 10's layer-wise weights: a voxel's soft threshold in
    absorption units, lambda(z) / e(z), is then the same at every depth)."""
    return _depth_rule(k, lam1, stream)[1]


def layer_threshold(mu, frac: float, stream=None):
    """In place: zero the values of each layer of mu (float32 [nz, n, n])
    below frac times the layer's maximum magnitude."""
    torch = _torch()
    nz = int(mu.shape[0])
    nb = ctypes.c_size_t()
    _check(lib().ctof_layer_threshold_ws_bytes(nz, ctypes.byref(nb)))
    ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=mu.device)
    _check(lib().ctof_layer_threshold(nz, int(mu[0].numel()), mu.data_ptr(), float(frac), ws.data_ptr(),
                                      ws.numel(), _stream_ptr(stream)))
    return mu
