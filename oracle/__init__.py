"""FP64 CPU oracle for confocal time-of-flight DOT (test infrastructure).

THIS PACKAGE IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test
suite, the smoke check in ``__graft_entry__`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The GPU library never calls it, shares no code,
tables or constants with it, and must not fall back to it.

What it computes, from the paper (arXiv 2101.11680):

* ``physics``  - the diffusion Green's functions behind the sensitivity
  (Eqs. 3-5), the closed-form time convolution Phi0 (*)_t R of Eq. 5 and its
  per-time-bin integral;
* ``kernel``   - the depth-dependent confocal blur kernel rho_z(x, y, t) of
  Eq. 11, tabulated on the scan grid;
* ``operator`` - the forward model m = sum_z rho_z (*) mu_z (Eq. 11) and its
  adjoint, as a direct spatial sum and an explicit Jacobian (tier 0, tiny
  grids) and as an FP64 FFT evaluation (tier 1, validated against tier 0);
* ``solver``   - power iteration for the step size and FISTA for the
  non-negative Tikhonov-regularised least-squares problem (section
  "Reconstruction Algorithm").

Where the paper is silent, the readings are listed in each module header.
Parity unpinned: absolute kernel values against the paper (it prints none
and its kernels came from Monte Carlo), and which diffusion-coefficient,
source-depth and boundary conventions its authors used.
"""
