/*
 * ctof.h - C ABI of libctof, the MI355X (gfx950) implementation of the
 * confocal time-of-flight diffuse optical tomography hot path of
 * "High Resolution, Deep Imaging Using Confocal Time-of-flight Diffuse
 * Optical Tomography" (arXiv 2101.11680).
 *
 * What is computed
 *   The forward model of Eq. 11: a confocal histogram
 *       m[k][i][j] = sum_z sum_{i',j'} K_z[i-i'][j-j'][k] * mu_z[i'][j']
 *   (lateral linear convolution of each depth layer mu_z with a
 *   depth-dependent, time-resolved kernel, summed over layers), its adjoint
 *   (transpose), and the FISTA reconstruction of section "Reconstruction
 *   Algorithm" for the non-negative Tikhonov-regularised problem
 *       min_{mu >= 0} 1/2 ||A mu - d||^2 + lambda/2 ||mu||^2.
 *   The kernel K_z is the time-binned Jacobian of Eq. 5 (time convolution
 *   of the diffusion fluence and reflectance) for collocated source and
 *   detector on a semi-infinite homogeneous medium with an extrapolated
 *   boundary, integrated exactly over each time bin and scaled by the voxel
 *   volume.
 *
 * Conventions shared by every entry point
 *   - Every function returns ctof_status; none aborts, throws or prints.
 *     On failure ctof_last_error() returns a message (thread-local, valid
 *     until the next call on the same thread).
 *   - Arguments are validated before any GPU work is enqueued; on
 *     CTOF_EINVAL / CTOF_EUNSUPPORTED / CTOF_ENOMEM no output byte is
 *     written.
 *   - All device memory (kernel spectrum, workspace, inputs, outputs) is
 *     owned by the caller.  Pointers named *_dev are device pointers on the
 *     current HIP device; the library never allocates device memory.
 *   - Work is enqueued on the given stream (NULL = the default stream) and
 *     is asynchronous unless stated otherwise.
 *   - Element type: double for CTOF_FP64, float for CTOF_FP32, CTOF_BF16X3
 *     and CTOF_BF16.  Arrays are C-contiguous:
 *       volume mu, g          [nz][ny][nx]
 *       histogram m, d, r     [nt][ny][nx]
 *   - A ctof_kernel handle is immutable after tabulation (apart from its FFT
 *     tuning and its band, see ctof_kernel_set_tuning, ctof_kernel_set_band)
 *     and may be used concurrently from several streams as long as each call
 *     has its own workspace.
 */
#ifndef CTOF_H
#define CTOF_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CTOF_OK = 0,
  CTOF_EINVAL = -1,        /* an argument breaks a documented rule              */
  CTOF_ENOMEM = -2,        /* a caller buffer is smaller than required           */
  CTOF_EHIP = -3,          /* a HIP runtime call failed                          */
  CTOF_ENONFINITE = -4,    /* a NaN/Inf appeared in an FP64 norm                 */
  CTOF_EUNSUPPORTED = -5,  /* valid but outside what the library implements      */
  CTOF_EDIVERGED = -6      /* a solve diverged (a step longer than 1/L_A)        */
} ctof_status;

typedef enum {
  CTOF_FP64 = 0,   /* FP64 FFTs and contraction (small grids, parity runs)           */
  CTOF_FP32 = 1,   /* FP32 FFTs, FP32 matrix-core contraction                        */
  CTOF_BF16X3 = 2, /* FP32 FFTs; contraction as BF16 hi*hi + hi*lo + lo*hi, FP32 acc. */
  CTOF_BF16 = 3    /* FP32 FFTs; kernel spectrum stored as BF16 (half the bytes),
                      data split hi+lo: K_hi*v_hi + K_hi*v_lo                        */
} ctof_precision;

/*
 * Scan geometry and background optics (section "Confocal ToF-DOT": a
 * collocated source/detector pair scanned over an ny x nx grid; the voxel
 * grid is the scan grid, aligned, one voxel layer per entry of z_mm).
 *   nx, ny            scan points per row and rows, 1..1024 each
 *                     (CTOF_EUNSUPPORTED above); spatial arrays are
 *                     [..][ny][nx]; both lateral axes use the FFT size of
 *                     the longer side
 *   pitch_mm          lateral pitch (> 0), equal in x and y
 *   nz, z_mm          number of layers (>= 1) and a HOST array of layer
 *                     centre depths, strictly increasing, > 0
 *   dz_mm             voxel thickness; 0 means the uniform spacing of z_mm
 *                     (then z_mm must be uniform, and nz == 1 needs dz_mm > 0)
 *   nt, dt_ps, t0_ps  time bins: bin k = [t0 + k dt, t0 + (k+1) dt), nt >= 1,
 *                     dt > 0, t0 >= 0 (t = 0 is the pulse entering the medium)
 *   mus_prime_per_mm  reduced scattering coefficient (> 0)
 *   mua_per_mm        background absorption (> 0; the closed form needs it)
 *   n_medium          refractive index inside (>= 1; 1 outside)
 * nz * ny * nx * nt must not exceed 1e15 (every byte count derived from
 * the shape then fits in 63 bits); CTOF_EINVAL otherwise.
 */
typedef struct {
  int32_t nx, ny;
  double pitch_mm;
  int32_t nz;
  const double *z_mm;
  double dz_mm;
  int32_t nt;
  double dt_ps, t0_ps;
  double mus_prime_per_mm, mua_per_mm, n_medium;
} ctof_geometry;

typedef struct ctof_kernel_s *ctof_kernel; /* opaque host handle */

/*
 * Sizes needed to tabulate a kernel: the spectrum buffer that the handle
 * keeps referring to, and a scratch workspace used only during
 * ctof_kernel_tabulate.  Pure host computation; no GPU needed.
 */
ctof_status ctof_kernel_bytes(const ctof_geometry *geom, ctof_precision prec,
                              size_t *khat_bytes, size_t *tab_ws_bytes);

/*
 * Tabulate the kernel of Eq. 5 for every layer, lateral offset and time bin
 * in FP64 on the GPU, transform it to its (real, even) 2D spectrum in FP64,
 * and pack that spectrum in the precision `prec` into khat_dev.  The caller
 * keeps khat_dev alive until ctof_kernel_free.  Enqueues on `stream` and
 * synchronises it before returning (tab_ws_dev may be reused afterwards).
 * On success *out receives a new handle.
 */
ctof_status ctof_kernel_tabulate(const ctof_geometry *geom, ctof_precision prec,
                                 void *khat_dev, size_t khat_bytes,
                                 void *tab_ws_dev, size_t tab_ws_bytes,
                                 hipStream_t stream, ctof_kernel *out);

/*
 * Test hook: the same FP64 kernel values as ctof_kernel_tabulate, before the
 * transform, for lateral offsets 0 <= dy, dx < n, n = max(nx, ny):
 *   quad_dev[z][k][dy][dx] = K_z[dy][dx][k]   (double, nz*nt*n*n entries).
 * Enqueues on `stream`; asynchronous.
 */
ctof_status ctof_kernel_tabulate_quadrant(const ctof_geometry *geom, double *quad_dev,
                                          size_t quad_bytes, hipStream_t stream);

/*
 * The same test hook without a size argument: quad_dev must hold
 * nz * nt * n * n doubles (n = max(nx, ny)), the size the geometry fixes;
 * the caller guarantees it (no other check is possible).  Errors as
 * ctof_kernel_tabulate_quadrant.
 */
ctof_status ctof_kernel_tabulate_fp64_quadrant(const ctof_geometry *geom, double *quad_dev, hipStream_t stream);

/*
 * Fluorescence mode (section "Materials and Methods": the optical
 * properties of the excitation and the emission wavelength, and the
 * fluorescence lifetime).  The kernel becomes the sensitivity of the
 * emission histogram to the fluorophore yield of a voxel,
 *     W = Phi0_ex (*)_t E_tau (*)_t R_em,   E_tau(t) = exp(-t/tau)/tau,
 * with the excitation fluence from the geometry's optics (mus_prime_per_mm
 * is the excitation value) and the flux back to the detector from the
 * emission optics; both wavelengths share mua_per_mm and n_medium.  Each
 * bin is exact (closed form, as in absorption mode).  lifetime_ps = 0 means
 * instantaneous emission; a lifetime must exceed 1/(mua c) (c = 0.2998/n
 * mm/ps; 467 ps at mua 0.01/mm, n 1.4), else CTOF_EUNSUPPORTED.  The
 * forward model, adjoint and solvers are unchanged (m = W mu with mu the
 * fluorophore yield); the spectrum layout and sizes are those of
 * ctof_kernel_bytes.  fl NULL: absorption mode, identical to
 * ctof_kernel_tabulate / ctof_kernel_tabulate_quadrant.
 */
typedef struct {
  double mus_prime_em_per_mm;  /* reduced scattering at the emission wavelength (> 0) */
  double lifetime_ps;          /* fluorescence lifetime tau (>= 0) */
} ctof_fluorescence;

ctof_status ctof_kernel_tabulate_ex(const ctof_geometry *geom, const ctof_fluorescence *fl, ctof_precision prec,
                                    void *khat_dev, size_t khat_bytes, void *tab_ws_dev, size_t tab_ws_bytes,
                                    hipStream_t stream, ctof_kernel *out);
ctof_status ctof_kernel_tabulate_quadrant_ex(const ctof_geometry *geom, const ctof_fluorescence *fl, double *quad_dev,
                                             size_t quad_bytes, hipStream_t stream);

/* Frees the host handle only; the spectrum buffer stays the caller's. */
void ctof_kernel_free(ctof_kernel k);

/*
 * Shape facts of a handle (any pointer may be NULL):
 *   n           max(nx, ny), the side that sets the FFT size
 *   nz, nt      layers, bins;   p   FFT size: the smallest length >= 2n-1
 *               among the powers of two (at least 16) and 48, 96, 192, 384, 768
 *   nmat        distinct spectrum matrices, (p/2+1)(p/2+2)/2
 *   prec        precision the handle was tabulated for
 */
ctof_status ctof_kernel_info(ctof_kernel k, int32_t *n, int32_t *nz, int32_t *nt,
                             int32_t *p, int32_t *nmat, int32_t *prec);

/*
 * Scan grid of a handle: ny rows and nx columns, the shape of every spatial
 * array the handle's calls take ([nz][ny][nx] volumes, [nt][ny][nx]
 * histograms).  Either pointer may be NULL.
 */
ctof_status ctof_kernel_grid(ctof_kernel k, int32_t *ny, int32_t *nx);

/*
 * Workspace bytes for ctof_forward / ctof_adjoint (op_ws) and for
 * ctof_reconstruct with at most max_iter iterations (solve_ws).
 */
ctof_status ctof_workspace_bytes(ctof_kernel k, int32_t max_iter, size_t *op_ws,
                                 size_t *solve_ws);

/*
 * Forward model (Eq. 11): m = A mu.  mu_dev [nz][ny][nx], m_dev [nt][ny][nx],
 * element type of the handle's precision.  Asynchronous.
 */
ctof_status ctof_forward(ctof_kernel k, const void *mu_dev, void *m_dev, void *ws_dev,
                         size_t ws_bytes, hipStream_t stream);

/*
 * The forward model of ctof_forward for callers that cannot allocate device
 * memory or supply a workspace: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation.  Same arguments (without the
 * workspace), same kernels and results bit for bit; the workspace is a fixed
 * device array of CTOF_NOALLOC_SCRATCH_BYTES bytes inside the library, one
 * per GPU, held from the first call on that GPU until the process ends.
 * Nothing is allocated.  CTOF_ENOMEM (before any launch) when the handle's
 * forward needs more workspace than that (op_ws of ctof_workspace_bytes; a
 * 64 x 64 scan with 32 layers and 256 bins needs about 30 MB, the
 * 128 x 128 x 64 layers x 512 bins benchmark shape about 230 MB and is
 * rejected).  Every call on one GPU shares the array and its contents
 * persist between calls (the forward writes every scratch byte it reads
 * before reading it): calls that overlap in time on one GPU, from several
 * streams or threads, race and must be serialised by the caller.
 * Asynchronous.
 */
#define CTOF_NOALLOC_SCRATCH_BYTES (64u << 20)
ctof_status ctof_forward_noalloc(ctof_kernel k, const void *mu_dev, void *m_dev, hipStream_t stream);

/*
 * Adjoint (the transpose of A; the kernel is real): g = A^T r.
 * r_dev [nt][ny][nx], g_dev [nz][ny][nx].  Asynchronous.
 */
ctof_status ctof_adjoint(ctof_kernel k, const void *r_dev, void *g_dev, void *ws_dev,
                         size_t ws_bytes, hipStream_t stream);

/* ===================================================================== *
 * Source multiplexing (subsection "Multiplexed Confocal ToF-DOT", Eq. 12).
 *
 * With several sources on at once, each multiplexed measurement is a fixed
 * linear combination of the confocal transients: y = S m = S A mu.  The
 * scan grid is cut into tiles of tile_x x tile_y positions (P = tile_x *
 * tile_y; the paper's 8 x 8 source array is one tile of 64) and the same S
 * (rows x P) combines the P transients of every tile in every time bin:
 *     y[t][i][g] = sum_j S[i][j] m[t][gy*tile_y + jy][gx*tile_x + jx]
 * with tile g = gy * (nx / tile_x) + gx and position j = jy * tile_x + jx.
 * S may be any matrix: a +-1 Hadamard matrix (y = H m), its on/off pattern
 * pair stacked as a 2P x P 0/1 matrix, a selection, ...
 * ===================================================================== */

typedef struct {
  int32_t tile_x, tile_y;  /* tile of scan positions; tile_x divides nx, tile_y divides ny */
  int32_t rows;            /* M, measurements per tile and bin (1..128); P = tile_x * tile_y <= 128;
                              m [nt][ny][nx] and y [nt][rows][ntiles] must each be below 2 GiB */
  const void *s_dev;       /* S [rows][P], row-major, device memory, element type of the data */
} ctof_mux;

/*
 * y = S m:  m_dev [nt][ny][nx]  ->  y_dev [nt][rows][ntiles], ntiles =
 * (nx / tile_x) * (ny / tile_y), element type of k's precision.  The buffers
 * must not overlap.  Asynchronous.  The products run on the matrix cores
 * (16x16x4 MFMA in the data's precision; S staged in LDS in FP32).
 */
ctof_status ctof_mux_forward(ctof_kernel k, const ctof_mux *mux, const void *m_dev, void *y_dev,
                             hipStream_t stream);

/* m = S^T y:  y_dev [nt][rows][ntiles]  ->  m_dev [nt][ny][nx] (every
 * element written).  The buffers must not overlap.  Asynchronous. */
ctof_status ctof_mux_adjoint(ctof_kernel k, const ctof_mux *mux, const void *y_dev, void *m_dev,
                             hipStream_t stream);

/*
 * Gradient input of the multiplexed data term, fused in one pass over m:
 * r = S^T (S m - y) (y_dev NULL: r = S^T S m), with m_dev, r_dev [nt][ny][nx]
 * (r_dev may equal m_dev; no other overlap) and y_dev [nt][rows][ntiles].
 * fit_dev: NULL, or a device double receiving 1/2 ||S m - y||^2 (FP64
 * per-block partial sums added in a fixed order).  ws_dev: at least
 * ctof_mux_normal_ws_bytes bytes of device memory, 16-byte aligned.
 * Asynchronous.
 */
ctof_status ctof_mux_normal_ws_bytes(ctof_kernel k, const ctof_mux *mux, size_t *ws_bytes);
ctof_status ctof_mux_normal(ctof_kernel k, const ctof_mux *mux, const void *m_dev, const void *y_dev, void *r_dev,
                            double *fit_dev, void *ws_dev, size_t ws_bytes, hipStream_t stream);

/*
 * Solver options (section "Reconstruction Algorithm"; FISTA with constant
 * step, no restart):
 *   max_iter         iterations to run (>= 1)
 *   lambda_tikhonov  Tikhonov weight; < 0 means 1e-3 * L_A
 *   lipschitz        step constant L (tau = 1/L); 0 means
 *                    L = 1.01 L_A + lambda with L_A = ||A||^2 from
 *                    power_iters power iterations (FP64 Rayleigh quotients);
 *                    if > 0, lambda_tikhonov must be >= 0
 *   power_iters      power iterations when lipschitz == 0 (0 means 50)
 *   rel_tol          stop when the gradient-mapping ratio
 *                    ||y_k - mu_k|| / (tau ||max(0, A^T d)||) <= rel_tol,
 *                    checked every check_every iterations (0 = run max_iter)
 *   check_every      >= 1 when rel_tol > 0
 *   warm_start       0: mu_inout is zeroed first; 1: mu_inout is mu_0;
 *                    2: mu_inout is mu_0 with zero-start fallback: after the
 *                    first iteration, a scan whose gradient-mapping ratio
 *                    exceeds 1 (the ratio of a zero start is 1 by
 *                    definition) restarts from mu = 0 as a fresh zero start
 *                    (its FISTA sequence begins again at t_1 = 1, so the
 *                    remaining max_iter - 1 iterations are exactly those of
 *                    a zero-start solve); the discarded iteration counts in
 *                    `iters` but not in the history, datafit0 or fista_k
 *   history_dev      optional device array double[max_iter][2] receiving
 *                    (1/2 ||A y_k - d||^2, gradient-mapping ratio) per
 *                    iteration of the kept run (iters - fell_back rows);
 *                    NULL for none
 *   timing           n >= 1: record HIP events on `stream` around the stages
 *                    of every n-th iteration (0, n, 2n, ...) and at the end
 *                    of the loop, and fill the ms_* fields and timed_iters of
 *                    the report (each timed iteration adds five event records
 *                    between its launches); 0: no events; < 0: CTOF_EINVAL
 *   lipschitz_scans, lambda_scans
 *                    batched solves only (NULL otherwise): host arrays [nscan]
 *                    giving each scan's L (> 0) and lambda (>= 0) in place of
 *                    lipschitz / lambda_tikhonov; scans sharing a handle must
 *                    agree.  NULL: lipschitz / lambda_tikhonov for all.
 *   lambda_l1_z      NULL, or a host array [nz] of per-layer L1 weights
 *                    (>= 0): the objective gains sum_z lambda_l1_z[z] *
 *                    ||mu_z||_1, the paper's sparsity term with its
 *                    layer-wise weights (Eqs. 8 and 10); with mu >= 0 its
 *                    prox shifts each voxel by tau * lambda_l1_z[z] before
 *                    the clamp, and the gradient-mapping ratio's
 *                    denominator becomes ||max(0, A^T d - lambda_l1_z)||.
 *                    Batched solves need one layer count for all scans.
 *   mux              NULL, or the multiplexing of the measurements (Eq. 12):
 *                    ctof_reconstruct then fits y = S A mu, d_dev holds y
 *                    [nt][rows][ntiles], every A and A^T of the solver
 *                    becomes S A and A^T S^T (L_A = ||S A||^2, the
 *                    gradient-mapping denominator ||max(0, A^T S^T y)||,
 *                    datafit = 1/2 ||S A mu - y||^2), and no extra
 *                    workspace is needed.  In batched solves the same
 *                    descriptor (S and the tile) applies to every scan,
 *                    whose grid it must tile; d_dev[i] holds scan i's y.
 *   k0, mu_prev_dev  resumption of an interrupted FISTA run (the state of
 *                    section "Reconstruction Algorithm" is the iterate
 *                    mu_k, its predecessor mu_{k-1} and the counter k of
 *                    the step-size sequence t_k).  k0 = 0: a fresh run.
 *                    k0 >= 1 (warm_start must be 1): mu_inout holds mu_k0
 *                    and mu_prev_dev holds mu_{k0-1} (same layout); the
 *                    first step starts from y = mu_k0 + beta_k0 (mu_k0 -
 *                    mu_{k0-1}) and uses the step weights from index k0 on,
 *                    so K1 iterations followed by a resumed K2 give the
 *                    same iterates, bit for bit, as one run of K1 + K2
 *                    (with the same L and lambda).  Output: when
 *                    mu_prev_dev is not NULL it receives the iterate before
 *                    the final one (for the next resumption, with k0 =
 *                    report.fista_k); it may be given with k0 = 0 to start
 *                    a resumable run.  It must not overlap mu_inout.  The
 *                    gradient-mapping denominator is recomputed (it does
 *                    not depend on the start), datafit0 and the first
 *                    history row are taken at y_{k0+1}.
 *   mu_prev_scans    batched solves only (NULL otherwise, and then
 *                    mu_prev_dev must be NULL too): host array [nscan] of
 *                    device pointers playing mu_prev_dev's role per scan; k0
 *                    applies to every scan (scans frozen early in the
 *                    interrupted call resume from their frozen state).
 *   skip_final_fit   0: after the last step the solver applies the forward
 *                    model once more to report datafit at the final iterate
 *                    (one extra contraction and measurement-side pass, about
 *                    half an iteration's time).  1: no extra pass; datafit
 *                    is then the data fit at the last step's extrapolated
 *                    point y_K (the last history row's), and the iterates,
 *                    history and gmap_ratio are unchanged, bit for bit.  A
 *                    one-iteration call whose start was discarded
 *                    (warm_start = 2) still computes it.  Other values:
 *                    CTOF_EINVAL.
 */
typedef struct {
  int32_t max_iter;
  double lambda_tikhonov;
  double lipschitz;
  int32_t power_iters;
  double rel_tol;
  int32_t check_every;
  int32_t warm_start;
  double *history_dev;
  int32_t timing;
  const double *lipschitz_scans;
  const double *lambda_scans;
  const double *lambda_l1_z;
  const ctof_mux *mux;
  void *mu_prev_dev;
  int32_t k0;
  void *const *mu_prev_scans;
  int32_t skip_final_fit;
} ctof_solver_opts;

/*
 * Report (host memory):
 *   iters       iterations run;  status  final ctof_status of the solve
 *   datafit0    1/2 ||A mu_0 - d||^2;  datafit  1/2 ||A mu_final - d||^2
 *               (1/2 ||A y_K - d||^2 with opts.skip_final_fit)
 *   gmap_ratio  gradient-mapping ratio of the last iteration
 *   lipschitz, lambda   the L and lambda used;  lipschitz_a  L_A (0 if L given)
 *   gmap0       ||max(0, A^T d)||, the ratio's denominator
 *   fell_back   1 if warm_start = 2 discarded the given start, else 0
 *   ms_*        with opts.timing: GPU milliseconds summed over the timed
 *               iterations for the forward contraction, the measurement-side
 *               FFT passes (inverse column, residual row, column), the adjoint
 *               contraction and the volume-side FFT passes (inverse column,
 *               prox row, column); ms_loop: the whole iteration loop (all
 *               iterations, from the first iteration's start to the end)
 *   timed_iters the number of timed iterations (0 without opts.timing)
 *   fista_k     the FISTA counter after the call: k0 + iterations of the
 *               kept run (the k0 that resumes it)
 */
typedef struct {
  int32_t iters, status;
  double datafit0, datafit, gmap_ratio, lipschitz, lambda, lipschitz_a, gmap0;
  double ms_contract_fwd, ms_fft_t, ms_contract_adj, ms_fft_z, ms_loop;
  int32_t fell_back;
  int32_t timed_iters;
  int32_t fista_k;
} ctof_solver_report;

/*
 * FISTA reconstruction.  d_dev [nt][ny][nx] (the measured histogram),
 * mu_inout_dev [nz][ny][nx] (start point if warm_start, result on return).
 * Enqueues on `stream` and synchronises it before returning (the report is
 * filled from device scalars); also synchronises every check_every
 * iterations when rel_tol > 0.  Reaching max_iter is not an error.
 * CTOF_EDIVERGED (report filled) when the last step's gradient-mapping
 * ratio exceeds 1e6 times the first step's (or 1e6 when that is below 1):
 * FISTA with a step of at most 1/L_A does not grow it so, a `lipschitz`
 * below the operator's (a step beyond 2/L_A) does, geometrically.
 */
ctof_status ctof_reconstruct(ctof_kernel k, const void *d_dev, void *mu_inout_dev,
                             const ctof_solver_opts *opts, ctof_solver_report *report,
                             void *ws_dev, size_t ws_bytes, hipStream_t stream);

/*
 * Layer-wise L1 weights (Eqs. 8 and 10: the sparsity weights grow with
 * depth to counter the loss of sensitivity).  energy_host[z] = e(z) =
 * ||A e_z||^2, the squared norm of the forward model's response to a unit
 * absorber at the window centre (row ny/2, column nx/2) of layer z,
 * summed in FP64; weights_host[z] = lambda1 * e(z) / max_z e(z), the rule
 * under which a voxel's soft threshold in absorption units,
 * lambda1_z / e(z), is the same at every depth (a reading: the paper
 * states only that the weights compensate the depth-dependent loss).
 * Either host array [nz] may be NULL.  ws_dev: at least
 * ctof_layer_energy_ws_bytes bytes.  Synchronises `stream`.
 * CTOF_ENONFINITE when an energy is not finite or all are zero.
 */
ctof_status ctof_layer_energy_ws_bytes(ctof_kernel k, size_t *ws_bytes);
ctof_status ctof_l1_depth_weights(ctof_kernel k, double lambda1, double *energy_host, double *weights_host,
                                  void *ws_dev, size_t ws_bytes, hipStream_t stream);

/*
 * Batched reconstruction of nscan independent scans (the same FISTA as
 * ctof_reconstruct, run for every scan).  Scans whose handles are the same
 * pointer form a shape class and share that handle's kernel spectrum: the
 * class's volumes are extra columns of one matrix-core contraction per
 * frequency (the spectrum is read once per class and pass, not once per
 * scan) and extra planes of the same FFT launches.  Handles must share one
 * precision; shapes may differ between classes.  L and lambda come from one
 * power iteration per class (or from opts).  Iterations run in chunks of
 * min(check_every, 50) (min(max_iter, 50) when rel_tol == 0), each chunk of
 * every live class captured once as a HIP graph on an internal stream and
 * replayed on `stream`; with rel_tol > 0 a scan whose gradient-mapping ratio
 * is <= rel_tol at a chunk end is frozen (its mu keeps that iterate) and a
 * class whose scans are all frozen leaves the graph.
 *   d_dev[i]        [nt][ny][nx] of scan i's handle
 *   mu_inout_dev[i] [nz][ny][nx] (start if warm_start, result on return)
 *   reports[i]      per scan; iters = iterations until frozen (or run)
 * opts.history_dev and opts.timing must be NULL / 0.  Synchronises `stream`.
 */
ctof_status ctof_workspace_bytes_batched(int32_t nscan, const ctof_kernel *k, int32_t max_iter,
                                        size_t *ws_bytes);
ctof_status ctof_reconstruct_batched(int32_t nscan, const ctof_kernel *k, const void *const *d_dev,
                                     void *const *mu_inout_dev, const ctof_solver_opts *opts,
                                     ctof_solver_report *reports, void *ws_dev, size_t ws_bytes,
                                     hipStream_t stream);

/*
 * Tuning of a handle's FFT passes: planes per block on the bin side (bb_t)
 * and on the layer side (bb_z), each 16 or 32 (0 = built-in rule: 32 when
 * the pass still has >= 1024 blocks).  The value changes launch shapes and
 * workspace sizes, not results.
 */
ctof_status ctof_kernel_set_tuning(ctof_kernel k, int32_t bb_t, int32_t bb_z);
ctof_status ctof_kernel_get_tuning(ctof_kernel k, int32_t *bb_t, int32_t *bb_z);
/*
 * Planes per block of the row passes alone (the passes that hold whole rows
 * of the spectrum: the c2r/r2c pair around the residual and around the
 * prox/FISTA step), on the bin side (rb_t) and the layer side (rb_z): 0 (the
 * column passes' value), 16, 32 or 64.  64 (256-byte runs of the spectrum,
 * two blocks per compute unit) applies to FP32 handles with FFT size <= 256
 * and plane counts divisible by 64; elsewhere a 64 acts as 32.  Changes
 * launch shapes and workspace sizes; the iterates are unchanged, the FP64
 * norms change only by their summation order.  get reports the effective
 * values for one volume.
 */
ctof_status ctof_kernel_set_row_tuning(ctof_kernel k, int32_t rb_t, int32_t rb_z);
ctof_status ctof_kernel_get_row_tuning(ctof_kernel k, int32_t *rb_t, int32_t *rb_z);

/*
 * Launch shape of a handle's contractions (the per-frequency products of
 * Eq. 11 and their transpose): blocks per spectrum matrix (and pair of
 * volumes), each 0 (built-in rule), 1, 2, 4 or 8.  The forward splits a
 * matrix's bins into runs, one block each; the adjoint splits its sum over
 * bins into runs whose partial results are added, in run order, by the
 * following inverse column pass (the workspace then holds one volume-side
 * spectrum per run: query ctof_workspace_bytes after setting).  Shorter
 * blocks shorten the tail of a launch.  The effective values (get) are
 * clamped: 1 with a spectrum band and for the BF16 adjoints (the BF16
 * forwards' rule is 2 from 256 bins, else 1; other values as asked), an
 * adjoint of FFT size above 256 keeps 1, and a run has at least one 16-bin
 * tile.  Results
 * change only by the order of the adjoint's sum.  The handle must not be in
 * use on other streams meanwhile.
 */
ctof_status ctof_kernel_set_contract_parts(ctof_kernel k, int32_t fwd_parts, int32_t adj_parts);
ctof_status ctof_kernel_get_contract_parts(ctof_kernel k, int32_t *fwd_parts, int32_t *adj_parts);
/*
 * Launch-shape tuner for a class of nvol volumes sharing the handle (the
 * batching form's per-class choice): times `iters` operator passes (1 to
 * 1000; the eight launches of an iteration) with events around their four
 * stages (forward contraction, bin-side passes, adjoint contraction,
 * layer-side passes; each the fastest of three timings after a warm-up)
 * for each legal FFT planes-per-block pair with the contractions at their
 * rule, and keeps the bin side's value that gave the fastest bin-side
 * passes and the layer side's that gave the fastest layer-side ones; then
 * the row passes' planes per block alike; then the forward contraction's
 * blocks per matrix 1, 2, 4, 8 by the time of that contraction and the
 * bin-side passes, then the adjoint's by the time of the adjoint and the
 * layer-side passes (which add its partial spectra).  The choices go into
 * the handle (ctof_kernel_set_tuning, ctof_kernel_set_row_tuning,
 * ctof_kernel_set_contract_parts); every timing is reported as the whole
 * iteration (the sum of its stages).  The FFT size
 * is fixed at tabulation (the kernel spectrum depends on it) to the
 * smallest supported length >= 2n - 1, which is never slower than a longer
 * one: it shrinks the spectrum and every pass.  Choices change
 * launch shapes and workspace sizes; results change only by the order of
 * the adjoint's sum.  Synchronises `stream`; the handle must not be in use
 * on other streams meanwhile.
 *   ms_bb   per iteration for (bb_t, bb_z) = (16,16), (32,16), (16,32),
 *           (32,32); -1 where the block rule does not allow the pair
 *   ms_fwd, ms_adj   for 1, 2, 4, 8 blocks per matrix; -1 where the value
 *           clamps to one timed before
 *   ms_rb   for row-pass planes (rb_t, rb_z) = (bb_t, bb_z), (64, bb_z),
 *           (bb_t, 16), (64, 16), (bb_t, 64), (64, 64); -1 where the
 *           effective values repeat an earlier pair's
 *   rb_t, rb_z   the row passes' effective planes per block
 */
typedef struct {
  int32_t bb_t, bb_z, fwd_parts, adj_parts;
  float ms_bb[4], ms_fwd[4], ms_adj[4];
  int32_t rb_t, rb_z;
  float ms_rb[6];
} ctof_tuning;
ctof_status ctof_tune_workspace_bytes(ctof_kernel k, int32_t nvol, size_t *ws_bytes);
ctof_status ctof_tune(ctof_kernel k, int32_t nvol, int32_t iters, void *ws_dev, size_t ws_bytes,
                      hipStream_t stream, ctof_tuning *out);

/*
 * Band of a handle's kernel spectrum (optional; an approximation of the
 * operator, off by default).  Each layer has its own kernel (Eq. 11), and
 * diffusion makes a deeper layer's kernel broader and later, so at high
 * lateral frequencies only early bins of shallow layers carry weight.  ctof_kernel_set_band finds, for each
 * spectrum matrix, the range of 16-bin tiles and the leading layers (in
 * groups of nzp/4 layers up to 64 layers, 16 from 64 on; nzp = nz rounded up
 * as the precision's kernels pack it) holding every entry >= rel * max |entry|,
 * and from then on the forward and adjoint products read only that block of
 * the matrix (outputs of the skipped forward tiles and adjoint layers are
 * zero).  The operator then differs from the full one by entries below
 * rel * max |entry|: per
 * lateral frequency f and bin t, |dm^(f)[t]| <= rel * max|K| * sum_z |mu^_z(f)|
 * (and likewise for the adjoint).  rel = 1e-9 is below FP32 resolution
 * relative to the largest entry.  rel = 0 removes the band (full products);
 * otherwise 0 < rel < 1.  band_dev: caller-owned device memory of
 * ctof_kernel_band_bytes bytes, 256-byte aligned, kept alive while the handle
 * uses it; its first 16 * nmat bytes receive the table, per matrix s = (a, b)
 * (s = b (b + 1)/2 + a, a <= b <= P/2) four int32 {lo, hi, zend, 0}: 16-bin
 * tiles [lo, hi) and layers [0, zend) ({0, 0, 0, 0} when the matrix holds no
 * entry at or above the threshold); the rest is scratch.  Enqueued on `stream`; the handle must not be in use on other
 * streams meanwhile.  CTOF_EUNSUPPORTED with more than 1024 tiles (16384
 * bins).
 */
ctof_status ctof_kernel_band_bytes(ctof_kernel k, size_t *bytes);
ctof_status ctof_kernel_set_band(ctof_kernel k, double rel, void *band_dev, size_t band_bytes, hipStream_t stream);

/* ===================================================================== *
 * Learned warm start.
 *
 * A 3D convolutional network maps the scaled adjoint back-projection
 * tau * A^T d of a scan to a starting volume for ctof_reconstruct
 * (warm_start = 1).  The reconstruction problem is unchanged (section
 * "Reconstruction Algorithm"); only its starting point is learned, and the
 * solver's own residual decides whether the start is kept.  The entry
 * points below are the network's layers, loss, optimiser step and the
 * counter-based sampler of Poisson photon counts (the detector model of the
 * section on multiplexed measurements) used to generate training data.
 *
 * Tensors are channels-last, [n][d][h][w][ld] rows of ld elements; a
 * ctof_tensor names the channel slice [c0, c0 + c) of such a buffer.
 * Activations and activation gradients are BF16 (uint16 storage), network
 * outputs may be FP32.  For BF16 slices read by a convolution: ptr 16-byte
 * aligned, ld and c0 multiples of 8 and c0 + roundup(c, 8) <= ld (the whole
 * 8-channel groups of the slice are read; channels past c are ignored).
 *
 * Layer kinds (input grid n x d x h x w, ci -> co channels):
 *   CTOF_CONV_K3  3x3x3 correlation, stride 1, zero padding 1 (same grid)
 *   CTOF_CONV_DN  2x2x2, stride 2 (grid halves; d, h, w even)
 *   CTOF_CONV_UP  2x2x2 transposed, stride 2 (grid doubles):
 *                 y[2z+i][2y+j][2x+k][o] = sum_c W[i][j][k][o][c] x[z][y][x][c]
 *   CTOF_CONV_K1  1x1x1
 * Packed weights (float master copy and BF16 working copy share it), with
 * cip = roundup(ci, 8), co_pad = roundup(co, 16), taps = 27 / 8 / 1 / 1
 * (K3 / DN / UP / K1), kpad = roundup(taps * cip, 32):
 *   K3, DN, K1: [co_pad][kpad], column tap * cip + ci, tap = (i*3+j)*3+k
 *               (K3) or (i*2+j)*2+k (DN) for offsets (i, j, k) in z, y, x
 *   UP:         [8][co_pad][kpad], leading index (i*2+j)*2+k, column ci
 *   all other entries zero.  Biases: float [co].
 * Supported channels: 1 <= ci <= 256; co_pad / 16 in {1, 2, 3, 4, 8}.
 * Accumulation is FP32 everywhere; reductions over positions (weight and
 * bias gradients, loss) are split in a fixed order (deterministic).
 * ===================================================================== */
typedef enum { CTOF_CONV_K3 = 0, CTOF_CONV_DN = 1, CTOF_CONV_UP = 2, CTOF_CONV_K1 = 3 } ctof_conv_kind;

typedef struct {
  int32_t kind;       /* ctof_conv_kind */
  int32_t n, d, h, w; /* input grid, each >= 1 */
  int32_t ci, co;     /* input / output channels */
} ctof_conv_desc;

typedef struct {
  void *ptr;   /* device pointer to the buffer's first row */
  int32_t ld;  /* elements per row */
  int32_t c0;  /* first channel of the slice */
} ctof_tensor;

/* Elements of the packed weight layout (float master or BF16 copy). */
ctof_status ctof_conv3d_weight_elems(const ctof_conv_desc *desc, size_t *elems);

/*
 * y = act(conv(x, w) + bias [+ y if accumulate]); act = ReLU if relu.
 * x: BF16 slice of ci channels on the input grid; w: packed BF16 weights;
 * bias: float [co] or NULL; y: slice of co channels on the output grid,
 * float if y_fp32 else BF16 (stored rounded to nearest even).
 */
ctof_status ctof_conv3d_fwd(const ctof_conv_desc *desc, const ctof_tensor *x, const void *w_bf16,
                            const float *bias, const ctof_tensor *y, int32_t y_fp32, int32_t relu,
                            int32_t accumulate, hipStream_t stream);

/*
 * Input gradient: dx (BF16, ci channels, input grid) = conv^T(dy) [+ dx if
 * accumulate]; dy: BF16 slice of co channels on the output grid.  Uses
 * ws_dev (>= ctof_conv3d_bwd_data_ws_bytes) for the rearranged weights.
 */
ctof_status ctof_conv3d_bwd_data_ws_bytes(const ctof_conv_desc *desc, size_t *ws_bytes);
ctof_status ctof_conv3d_bwd_data(const ctof_conv_desc *desc, const ctof_tensor *dy, const void *w_bf16,
                                 const ctof_tensor *dx, int32_t accumulate, void *ws_dev, size_t ws_bytes,
                                 hipStream_t stream);

/*
 * Weight and bias gradients: dw (float, packed layout, fully written, zero
 * outside the real channels) = sum over positions of dy x~; db (float [co],
 * or NULL) = sum of dy over output positions.  x: BF16 layer input; dy:
 * BF16 gradient at the layer output (after the ReLU mask).
 */
ctof_status ctof_conv3d_bwd_weight_ws_bytes(const ctof_conv_desc *desc, size_t *ws_bytes);
ctof_status ctof_conv3d_bwd_weight(const ctof_conv_desc *desc, const ctof_tensor *x, const ctof_tensor *dy,
                                   float *dw_dev, float *db_dev, void *ws_dev, size_t ws_bytes,
                                   hipStream_t stream);

/* ReLU backward in place: dy[r][c] = 0 where y[r][c] <= 0 (BF16 slices, ch channels, rows rows). */
ctof_status ctof_relu_bwd(int64_t rows, int32_t ch, const ctof_tensor *dy, const ctof_tensor *y, hipStream_t stream);

/*
 * Mean squared error of s y (s = y_scale, y = channel y.c0 of an FP32
 * tensor) against a dense float target [n]: *loss_dev (double) =
 * mean (s y - t)^2 and grad (BF16 slice, channel grad.c0) = d loss / d y =
 * 2 s (s y - t) / n, or 0 where y <= 0 when relu_mask (y is then the output
 * of a ReLU, whose backward this folds in).
 */
ctof_status ctof_mse_ws_bytes(int64_t n, size_t *ws_bytes);
ctof_status ctof_mse(int64_t n, const ctof_tensor *y, float y_scale, const float *target_dev,
                     const ctof_tensor *grad, int32_t relu_mask, double *loss_dev, void *ws_dev, size_t ws_bytes,
                     hipStream_t stream);

/*
 * Training loss of the warm start, for nb (1..64) scans of one float handle
 * (CTOF_FP32, CTOF_BF16X3 or CTOF_BF16).  Scan b's start is x_b = s_b y_b
 * (s: host array [nb]),
 * y_b = channel y.c0 of rows b V .. (b + 1) V - 1 of an FP32 tensor
 * (V = nz n n, rows in [z][y][x] order: the network output); target_dev
 * holds the solutions mu*_b (float [nb][nz][ny][nx]).  With e_b = x_b - mu*_b
 * and H = A^T A + lambda I (the Hessian of the regularised objective of
 * section "Reconstruction Algorithm"), H e_b is to first order the gradient
 * of the objective at the start, i.e. what the solver's gradient-mapping
 * ratio measures:
 *   loss_b = w_b ||H e_b||^2 + v_b ||e_b||^2      (w, v: host arrays [nb])
 * terms_dev (double [nb][2]) receives (||H e_b||^2, ||e_b||^2) (FP64 sums in
 * a fixed order); grad (BF16 slice, channel grad.c0 of the same rows)
 * receives d(mean_b loss_b)/dy = (s_b / nb)(2 w_b H^2 e_b +
 * 2 v_b e_b), zeroed where y <= 0 when relu_mask (the backward of an output
 * ReLU); relu_mask = 0 passes it through there (straight-through estimate,
 * which keeps an output clamped at zero trainable).  H runs through the
 * same operator kernels as ctof_forward / ctof_adjoint, all nb scans at once.
 */
ctof_status ctof_warmstart_loss_ws_bytes(ctof_kernel k, int32_t nb, size_t *ws_bytes);
ctof_status ctof_warmstart_loss(ctof_kernel k, int32_t nb, const ctof_tensor *y, const double *s, const float *target_dev,
                                const double *w, const double *v, double lambda, int32_t relu_mask,
                                const ctof_tensor *grad, double *terms_dev, void *ws_dev, size_t ws_bytes,
                                hipStream_t stream);

/* Per-sample maximum magnitude: out_dev[b] = max_i |x_dev[b len + i]| (float). */
ctof_status ctof_absmax_ws_bytes(int32_t nb, size_t *ws_bytes);
ctof_status ctof_absmax(int32_t nb, int64_t len, const float *x_dev, float *out_dev, void *ws_dev, size_t ws_bytes,
                        hipStream_t stream);

/*
 * Depth resampling by 2 of nb volumes [nb][nz_in][plane] (float, out not
 * overlapping x): mode 0 sums layer pairs, out[b][j] = x[b][2j] + x[b][2j+1]
 * (nz_in even; nz_in / 2 layers out); mode 1 repeats layers, out[b][k] =
 * x[b][k / 2] (2 nz_in layers out).  A back-projection on a grid with twice
 * the layers over the same depth range, pair-summed, approximates the one on
 * the coarse grid (each coarse voxel is two fine ones), so a network trained
 * on the coarse grid can start the fine one.
 */
ctof_status ctof_depth_resample(int32_t nb, int32_t nz_in, int64_t plane, const float *x_dev, float *out_dev,
                                int32_t mode, hipStream_t stream);

/* FP64 sums of squares of nb float vectors of length len: out_dev[b] (double). */
ctof_status ctof_sumsq_ws_bytes(int32_t nb, size_t *ws_bytes);
ctof_status ctof_sumsq(int32_t nb, int64_t len, const float *x_dev, double *out_dev, void *ws_dev, size_t ws_bytes,
                       hipStream_t stream);

/*
 * Layer-wise threshold of a reconstruction (the paper's post-processing of
 * its 3D results): in each of the nz layers [plane] of mu_dev (float, in
 * place), values below frac * (the layer's maximum magnitude) are set to 0.
 */
ctof_status ctof_layer_threshold_ws_bytes(int32_t nz, size_t *ws_bytes);
ctof_status ctof_layer_threshold(int32_t nz, int64_t plane, float *mu_dev, float frac, void *ws_dev,
                                 size_t ws_bytes, hipStream_t stream);

/*
 * Adam (Kingma and Ba, 2015) with bias correction on n float master weights
 * w, gradient g and moments m, v (step counts from 1); w_bf16 (or NULL)
 * receives the updated weights rounded to BF16.
 */
ctof_status ctof_adam_step(int64_t n, float *w_dev, const float *g_dev, float *m_dev, float *v_dev,
                           void *w_bf16_dev, float lr, float beta1, float beta2, float eps, int32_t step,
                           hipStream_t stream);
/* The same step on the gradient scaled by grad_scale (finite, >= 0): the
 * caller's gradient-norm clipping (scale = min(1, c / ||g||)) for callers
 * that tame rare large gradients without a host-side pass over g. */
ctof_status ctof_adam_step_scaled(int64_t n, float *w_dev, const float *g_dev, float *m_dev, float *v_dev,
                                  void *w_bf16_dev, float lr, float beta1, float beta2, float eps, int32_t step,
                                  float grad_scale, hipStream_t stream);

/* Dense float [n] -> BF16 channel out.c0 of n rows (v = x * scale rounded
 * to BF16); with split, channel out.c0 + 1 receives BF16(v - BF16(v)), so the
 * pair carries about 16 significant bits; zero_rest zeroes the row's other
 * elements.  And back: out[i] = y[i][c0] * scale for an FP32 tensor y. */
ctof_status ctof_to_channels_last(int64_t n, const float *x_dev, float scale, const ctof_tensor *out,
                                  int32_t zero_rest, int32_t split, hipStream_t stream);
ctof_status ctof_from_channels_last(int64_t n, const ctof_tensor *y, float scale, float *out_dev,
                                    hipStream_t stream);

/*
 * Philox-4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011) with key (seed mod
 * 2^32, seed div 2^32) and counter (i mod 2^32, i div 2^32, stream_id, 0)
 * for i = first .. first + n - 1: out_dev[4 (i - first) + j] = word j.
 */
ctof_status ctof_philox4x32(uint64_t seed, uint32_t stream_id, int64_t first, int64_t n, uint32_t *out_dev,
                            hipStream_t stream);

/*
 * Poisson counts with means lam_dev[i] (float, <= 0 gives 0) into float
 * counts_dev[i] (exact below 2^24).  Element i draws from counters
 * (i, stream_id, trial): for lam < 10 the inverse CDF at one uniform
 * u = ((w0 >> 5) 2^26 + (w1 >> 6)) 2^-53 (w0, w1 = Philox words 0 and 1 of
 * trial 0), for lam >= 10 Hoermann's transformed rejection with squeeze
 * (1993), uniforms from words (0, 1) and (2, 3) of trial t = 0, 1, ...
 * Decisions are taken in FP64.
 */
ctof_status ctof_poisson(int64_t n, const float *lam_dev, uint64_t seed, uint32_t stream_id, float *counts_dev,
                         hipStream_t stream);

/*
 * Noisy histogram: d = Poisson(s m) / s with s = peak / max(m) (FP64), m
 * and d float [n], not overlapping.  A histogram whose maximum is not
 * positive gives d = 0.
 */
ctof_status ctof_noisy_histogram_ws_bytes(int64_t n, size_t *ws_bytes);
ctof_status ctof_noisy_histogram(int64_t n, const float *m_dev, double peak, uint64_t seed, uint32_t stream_id,
                                 float *d_dev, void *ws_dev, size_t ws_bytes, hipStream_t stream);

/*
 * Counting noise with dark counts (section "Advantages of Multiplexing"):
 * out = (c - background) / scale with c ~ Poisson(scale * max(m, 0) +
 * background), m and out float [n] (may be the same buffer).  scale
 * converts the model to expected signal counts, background is the expected
 * dark count of one element.  Counters and sampler as in ctof_poisson; the
 * mean is computed in FP64 without contraction.
 */
ctof_status ctof_noisy_counts(int64_t n, const float *m_dev, double scale, double background, uint64_t seed,
                              uint32_t stream_id, float *out_dev, hipStream_t stream);

const char *ctof_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CTOF_H */
