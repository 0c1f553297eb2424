"""MI355X (gfx950) implementation of the confocal time-of-flight DOT hot path.

The compute lives in ``libctof.so`` (HIP kernels behind a C ABI declared in
``include/ctof.h``); ``paper_2101_11680_amd.ctof`` is its ctypes binding.
"""

from .ctof import (BF16, BF16X3, FP32, FP64, PRECISIONS, CtofError, Kernel, adjoint,  # noqa: F401
                   forward, kernel_bytes, lib, reconstruct, tabulate, tabulate_quadrant)
