"""Seeded synthetic workloads for confocal time-of-flight DOT.

This package only draws inputs: scan geometries, absorber phantoms, the
Poisson counting noise applied to a histogram that the caller computed, and
the multiplexing patterns S (which sources are on in each measurement).  It
holds none of the method's arithmetic (no Green's function, no kernel, no
convolution, no solver), so both the FP64 oracle and the GPU path can take
their inputs from it without sharing any of the computation being tested.
"""

from .workloads import Geometry, WORKLOADS, workload, geometry_for
from .phantoms import phantom
from .noise import poisson_histogram

__all__ = ["Geometry", "WORKLOADS", "workload", "geometry_for", "phantom",
           "poisson_histogram"]
