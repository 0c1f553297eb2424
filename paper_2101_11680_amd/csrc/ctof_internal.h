// Internal declarations shared by the libctof translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "../../include/ctof.h"

namespace ctof {

constexpr int kMaxN = 1024;     // largest scan side (FFT size <= 2048)
constexpr int kMaxLayers = 256; // layer depths travel as a kernel argument
constexpr int kMinP = 16;       // smallest FFT size used
constexpr int kMaxVol = 64;     // volumes of one shape class per batched launch

inline size_t round_up(size_t v, size_t m) { return (v + m - 1) / m * m; }

// Sizes derived from a geometry.  ny x nx: the scan grid (rows, columns);
// n = max(ny, nx) sets the FFT size p (power of two >= 2n-1) of both
// lateral axes, so the spectrum keeps its kx <-> ky symmetry; h = p/2;
// nmat = distinct real spectrum matrices (a <= b <= h); nzp / ntp: layer /
// bin counts padded for the matrix-core tiles.
struct Dims {
  int n, nz, nt, p, h, nmat, nzp, ntp;
  int ny, nx;
};

Dims make_dims(int nx, int ny, int nz, int nt, ctof_precision prec);

// Background optics and the per-voxel constants of the kernel closed form.
struct Optics {
  double c, D, z0, zb, mua, mueff;
};

struct LayerDepths {
  double z[kMaxLayers];
};

struct GaussLegendre16 {
  double x[16], w[16];
};

// Geometry of one tabulation, all on the host side of a launch.
struct TabGeom {
  int n, nz, nt;
  double pitch, dt, t0, dv, rmin;
  Optics o;         // excitation optics (the only optics in absorption mode)
  double Dm, zbm;   // emission diffusion coefficient and boundary (= o.D, o.zb in absorption mode)
  double tau;       // fluorescence lifetime in ps (0: none)
};

// Byte layout of a packed spectrum (offsets into khat_dev).
struct KhatLayout {
  size_t fwd, fwd_lo, adj, adj_lo, total;  // fwd_lo/adj_lo == SIZE_MAX when unused
};

KhatLayout khat_layout(const Dims &d, ctof_precision prec);

// Fragment order of the packed spectrum: every 16-byte vector load of the
// contraction kernels reads one contiguous 1 KB run per wavefront.
//   v     elements per 16 bytes (4 float, 2 double, 8 bf16)
//   kz    forward: layers per lane group per 64-layer chunk (min(nzp,64)/4)
//   tc    adjoint: bins per chunk (16, or 32 for bf16); tl = tc/4 per lane group
// forward element (s, tt, ch, q, lane, e):
//   t = 16 tt + row(lane % 16),  z = 4 kz ch + kz (lane / 16) + v q + e
// adjoint element (s, tc_i, zt, q, lane, e):
//   z = 16 zt + row(lane % 16),  t = tc tc_i + tl (lane / 16) + v q + e
// row() is the identity except for FP64, whose 16x16x4 result interleaves
// rows (item r of lane group g holds row 4r + g): row(i) = 4 (i % 4) + i / 4.
struct Frag {
  int v, kz, tc, tl;
  bool f64;
};

__host__ __device__ inline Frag frag_of(const Dims &d, ctof_precision prec) {
  Frag f;
  f.f64 = prec == CTOF_FP64;
  const bool bf = prec == CTOF_BF16X3 || prec == CTOF_BF16;
  f.v = f.f64 ? 2 : (bf ? 8 : 4);
  f.kz = (d.nzp >= 64 ? 64 : d.nzp) / 4;
  f.tc = bf ? 32 : 16;
  f.tl = f.tc / 4;
  return f;
}

__host__ __device__ inline int frag_row(bool f64, int i) { return f64 ? 4 * (i & 3) + (i >> 2) : i; }

}  // namespace ctof

struct ctof_kernel_s {
  ctof::Dims dims;
  ctof_precision prec;
  ctof::TabGeom geom;
  void *khat;                 // caller-owned device buffer
  ctof::KhatLayout layout;
  int bb_t, bb_z;             // FFT planes per block on the bin / layer side (0 = rule)
  int rb_t = 0, rb_z = 0;     // row passes' planes per block where they differ (0 = bb_t / bb_z)
  const int *band = nullptr;  // caller-owned device table: per matrix {lo, hi, zend, 0} (NULL = all)
  double band_rel = 0.0;      // threshold the table was made with (0 = none)
  int fwd_parts = 0, adj_parts = 0;  // contraction blocks per matrix (0 = rule), see contract_parts
};

namespace ctof {

// ---- tabulation (tabulate.hip) --------------------------------------------
hipError_t launch_tab_values(const TabGeom &g, const LayerDepths &z, const GaussLegendre16 &gl,
                             double *out, size_t s_dy, size_t s_dx, size_t s_z, size_t s_t,
                             hipStream_t st);
// The (p/2 + 1) x n cosine matrix of the kernel spectrum in the operand
// order of launch_gemm_f64 (cosine_matrix_elems doubles).
size_t cosine_matrix_elems(int n, int p);
hipError_t launch_cosine_matrix(int n, int p, double *C, hipStream_t st);
// C[M][N] = A[M][K] * B[K][N] (FP64 on the matrix cores; A in the operand
// order of launch_cosine_matrix, B and C row-major), batched with strides.
hipError_t launch_gemm_f64(int M, long long N, int K, const double *Af, const double *B, long long ldb,
                           long long sB, double *C, long long ldc, long long sC, int batch, hipStream_t st);
hipError_t launch_pack(const Dims &d, ctof_precision prec, const double *k64, void *khat,
                       const KhatLayout &lay, double scale, hipStream_t st);

// ---- FFT passes (fft.hip) ---------------------------------------------------
// Column pass along kx for every ky of a spectrum block.
//   inverse: in [h+1][p][2][B] -> out [h+1][ny][2][B] (rows >= ny dropped)
//   forward: in [h+1][ny][2][B] (rows >= ny are zero) -> out [h+1][p][2][B]
// ppv: planes per volume; active: per-volume flags, blocks of frozen (0)
// volumes do nothing (NULL: all live)
// nsum > 1 (inverse passes of FFT size <= 256 only): the input is the sum of
// nsum spectra `sstride` elements apart, added in order (the partial sums of
// an adjoint contraction split along t).
template <typename T>
hipError_t launch_col_pass(const Dims &d, int B, bool inverse, const T *in, T *out,
                           hipStream_t st, int ppv = 0, int bb = 0, const int *active = nullptr, int nsum = 1,
                           size_t sstride = 0);

enum RowOp : int {
  ROW_SPEC_TO_SPATIAL = 0,   // c2r -> crop -> store spatial (forward/adjoint output)
  ROW_SPATIAL_TO_SPEC = 1,   // spatial (optionally scaled) -> pad -> r2c
  ROW_RESIDUAL = 2,          // c2r -> r = x - d, partial 1/2 r^2 -> r2c
  ROW_PASS = 3,              // c2r -> partial 1/2 x^2 -> r2c (power iteration)
  ROW_FISTA = 4,             // c2r -> prox/FISTA update -> r2c of y_{k+1}
  ROW_POWER_W = 5,           // c2r -> store w, partials |w|^2 and <v, w>
  ROW_GMAP0 = 6,             // c2r -> partial |max(0, x)|^2
  ROW_SCALE_TO_SPEC = 7,     // spatial w * (1/sqrt(scalar)) -> store v -> r2c
  ROW_EXTRAPOLATE = 8,       // y = mu + beta (mu - mu_prev) -> store y -> r2c (resumed FISTA)
  ROW_FIT = 9                // c2r -> r = x - d, partial 1/2 r^2 (data fit only: no r2c, no stores)
};

struct RowArgs {
  int op;
  int B;            // plane-axis length of the spectra (nvol * ppv)
  int ppv;          // spectrum planes per volume (ntp or nzp)
  int nplanes;      // real planes per volume (nt or nz); the rest read as zero
  int nvol;         // volumes (1 for the single-volume entry points)
  int bb;           // planes per block (0 = default rule)
  const void *spec_in;   // [h+1][ny][2][B]
  void *spec_out;        // [h+1][ny][2][B] (may alias spec_in)
  const void *sp_in[kMaxVol];   // per volume spatial input [planes][ny][nx] (d, y, v, ...)
  void *sp_out[kMaxVol];        // per volume spatial output
  void *sp_aux[kMaxVol];        // per volume second spatial buffer (mu for FISTA)
  double *partials;      // per-block FP64 partials (2 per block)
  size_t part_stride;    // doubles per iteration when iter_ctr is set
  const int *iter_ctr;   // device iteration counter: selects partials slot and beta
  const double *beta_tab;  // device FISTA weights, indexed by *iter_ctr (or NULL: beta)
  const int *active;     // per volume: blocks of a frozen (0) volume do nothing (NULL: all live)
  const double *scalar;  // device scalar (ROW_SCALE_TO_SPEC: |w|^2)
  const double *l1;      // device per-layer L1 weights (ROW_FISTA, ROW_GMAP0), or NULL
  double tau, lambda, beta;
  void *sp_prev[kMaxVol];  // ROW_FISTA: per volume, receives mu_{k-1} (the iterate being replaced), or NULL
  const int *beta_off;     // per volume: subtracted from the counter for the beta index (NULL: 0)
  int sp_vec;              // set by launch_row_pass: rows of whole 16-byte words and 16-byte aligned
                           // spatial arrays, accessed with vector loads and stores
  int gmap0_at;            // ROW_FISTA: at this iteration (the counter's value, 0 without one) partial 1
                           // also receives |max(0, -x - l1)|^2, the gradient mapping at zero when y = 0
                           // (x = A^T (A 0 - d) = -A^T d); -1: never
  int spec_of_mu;          // ROW_FISTA: the spectrum written is that of mu_k instead of y_{k+1} (a final step
                           // whose data fit follows; y_{k+1} is still stored)
};

template <typename T>
hipError_t launch_row_pass(const Dims &d, const RowArgs &a, hipStream_t st);
// Blocks of a row pass over B planes with ppv planes per volume and an
// optional planes-per-block override (0 = default rule).
int row_pass_blocks(const Dims &d, int B, int ppv, bool fp64, int bb = 0);
// Planes per block of a row pass: bb = 64 where allowed (FP32, FFT size <=
// 256, 64 | B and 64 | ppv), else the column-pass rule (64 asks for 32 there).
int row_block(const Dims &d, int B, int ppv, bool fp64, int bb = 0);
int batch_block(const Dims &d, int B, int ppv, bool fp64, int bb = 0);

// ---- contraction (contract.hip) ---------------------------------------------
// forward:  out[f][re/im][t] = sum_z K_s(f)[t][z] in[f][re/im][z]
// adjoint:  out[f][re/im][z] = sum_t K_s(f)[t][z] in[f][re/im][t]
// nvol volumes of one shape class share the spectrum; their planes are
// interleaved per frequency as [f][re/im][vol][plane].
// Per matrix s, band[4 s], band[4 s + 1] = the range [lo, hi) of 16-bin tiles
// and band[4 s + 2] = the end zend of the leading layers (a multiple of the
// forward's layers per lane group) holding every entry >= rel * max |entry|
// of the packed spectrum (forward layout; all 0 when none); band[4 s + 3] = 0.
// scratch: one device unsigned int.  At most band_max_tiles() tiles per
// matrix.
hipError_t launch_band(const ctof_kernel_s *k, double rel, int *band, unsigned int *scratch, hipStream_t st);
int band_max_tiles();

// Blocks per (matrix, pair of volumes) of a contraction launch: the forward
// splits a matrix into runs of 16-bin tiles, the adjoint into runs of bin
// chunks whose partial sums go to `parts` consecutive output spectra of
// `pstride` elements each (summed by the following inverse column pass).
int contract_parts(const ctof_kernel_s *k, bool adjoint);
hipError_t launch_contract(const ctof_kernel_s *k, bool adjoint, const void *in, void *out,
                           hipStream_t st, int nvol = 1, const int *active = nullptr, size_t pstride = 0);

// ---- source multiplexing (mux.hip) --------------------------------------------
// Tiles of tx x ty scan positions (P = tx ty) combined per time bin by S
// (M x P, row-major, element type of the data): y[t][i][g] = sum_j S[i][j]
// m[t][pos(g, j)].  MUX_FWD: out = y = S m;  MUX_ADJ: out = m = S^T y (in =
// y);  MUX_NORMAL: out = S^T (S m - y) (y may be NULL: zero), FP64 partials
// (1/2 |S m - y|^2, 0) per block when `partials` is set; out may alias in.
enum { MUX_FWD = 0, MUX_ADJ = 1, MUX_NORMAL = 2 };
constexpr int kMuxMaxDim = 128;  // largest M and P

struct MuxArgs {
  int ny, nx, nt, tx, ty, M, P, ntx, ntiles;  // scan rows and columns; tiles per row, tiles
  const void *S;
  const void *in;    // MUX_FWD, MUX_NORMAL: m [nt][ny][nx];  MUX_ADJ: y [nt][M][ntiles]
  const void *y;     // MUX_NORMAL: y [nt][M][ntiles] or NULL
  void *out;         // MUX_FWD: y;  otherwise [nt][ny][nx]
  double *partials;  // MUX_NORMAL: npart pairs (block b's sum at pair b, zeros past the grid), or NULL
  int npart;         // >= the launch's blocks when partials is set
  int sstr;          // set by launch_mux
  const int *ctr;    // device iteration counter: partials advance by part_stride doubles per count (or NULL)
  size_t part_stride;
  const int *active; // per-volume flags: the launch does nothing when active[vol] == 0 (or NULL)
  int vol;
};

// Grid of a multiplexing launch (persistent blocks, at most one per compute
// unit in FP32).
int mux_default_blocks(const MuxArgs &a, bool f64);
hipError_t launch_mux(int mode, bool f64, const MuxArgs &a, int blocks, hipStream_t st);

// ---- reductions and small kernels (solver.hip) --------------------------------
// sums[j] = sum_i partials[i*stride + j] for j < count, over nrows rows (FP64,
// fixed order).
hipError_t launch_reduce_rows(const double *partials, int nrows, int stride, int count,
                              double *sums, hipStream_t st);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st);
// Per iteration (iters rows of `stride` doubles) and volume: hist[(it*nvol+v)*2] =
// sum of the volume's bin-side partials (data fit), [..+1] = sqrt(sum of its
// layer-side partials) / (tau * sqrt(g0sq[v])) (gradient-mapping ratio).  The
// blocks of volume v are the v-th of nvol equal contiguous ranges.
hipError_t launch_history(const double *partials, int iters, int nvol, int nblk_t, int nblk_z,
                          size_t stride, double tau, const double *g0sq, double *hist, hipStream_t st);
// Freeze check of a batched class after its iteration *ctr - 1: a live volume
// whose gradient-mapping ratio (as launch_history computes it) is finite and
// <= rel_tol gets active[v] = 0 and conv[v] = its iteration count.  g0_part
// (or NULL): the partials of ||max(0, A^T d)||^2 from a zero start's first
// step, summed into g0sq first (as launch_reduce_volumes does).
hipError_t launch_freeze(const double *partials, size_t stride, const int *ctr, int nvol, int nblk_t, int nblk_z,
                         double tau, double *g0sq, const double *g0_part, double rel_tol, int *active, int *conv,
                         hipStream_t st);
// The end-of-solve values in one place, so that one copy reads them back:
// out[0..3] = scal[0..3], out[4..5] = history row 0 and out[6..7] row
// kept - 1 (zeros when kept = 0), out[8] = g0sq[0].
hipError_t launch_pack_report(const double *scal, const double *hist, int kept, const double *g0sq, double *out,
                              hipStream_t st);
// out[v] = sum of partial 0 over the v-th of nvol equal block ranges
hipError_t launch_reduce_volumes(const double *partials, int nblk, int nvol, double *out, hipStream_t st);
hipError_t launch_increment(int *ctr, hipStream_t st);
// beta[j] = beta_{first + j} of FISTA's step sequence, j < count
hipError_t launch_beta_table(double *beta, int first, int count, hipStream_t st);
hipError_t launch_fill_int(int *p, int n, int v, hipStream_t st);
hipError_t launch_fill_value(float *p, size_t n, float v, hipStream_t st);
hipError_t launch_fill_value_f64(double *p, size_t n, double v, hipStream_t st);


// Thread-local error message of the C ABI (returns s).
ctof_status set_error(ctof_status s, const char *fmt, ...);
const char *last_error();

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return ::ctof::set_error(CTOF_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));  \
  } while (0)

// ---- learned warm start: 3D convolution layers and sampling ------------------------
enum { CNN_K3 = 0, CNN_DN = 1, CNN_UP = 2, CNN_K1 = 3 };

struct ConvArgs {
  int kind, n, d, h, w, ci, co;  // input grid and channels
  int cip, co_pad, kpad;         // packed-weight layout
  const __bf16 *x;
  int x_ld, x_c0;
  const __bf16 *wt;
  const float *bias;
  void *y;
  int y_ld, y_c0, y_fp32, relu, accumulate;
};

struct WgradArgs {
  const __bf16 *dy;
  int dy_ld, dy_c0;
  float *part;
  int nparts;
  long long per_part;
};

int cnn_cip(int ci);
int cnn_copad(int co);
int cnn_kpad(int kind, int ci);
size_t cnn_weight_elems(int kind, int co, int ci);
void conv_fill_layout(ConvArgs &a);
long long conv_gemm_positions(const ConvArgs &a);
long long conv_output_rows(const ConvArgs &a);
ConvArgs conv_transposed(const ConvArgs &f);
bool conv_co_supported(int co);
hipError_t launch_conv_fwd(const ConvArgs &a, hipStream_t st);
size_t conv_transposed_weight_bytes(const ConvArgs &f);
hipError_t launch_transpose_weights(const ConvArgs &f, const __bf16 *w, __bf16 *wt, hipStream_t st);
size_t conv_wgrad_ws_bytes(const ConvArgs &a);
hipError_t launch_conv_wgrad(const ConvArgs &a, const __bf16 *dy, int dy_ld, int dy_c0, float *dw, float *db,
                             float *ws, hipStream_t st);
hipError_t launch_relu_mask(__bf16 *dy, int dld, int dc0, const __bf16 *y, int yld, int yc0, long long nrows,
                            int ch, hipStream_t st);
size_t mse_ws_bytes(long long n);
hipError_t launch_mse(const float *y, int yld, int yc0, float ys, const float *t, long long n, __bf16 *g, int gld,
                      int gc0, int relu_mask, double *part, double *loss, hipStream_t st);
hipError_t launch_adam(float *w, const float *g, float *m, float *v, __bf16 *wb, long long n, float lr, float b1,
                       float b2, float eps, int step, float gscale, hipStream_t st);
hipError_t launch_to_channels_last(const float *x, long long n, float scale, __bf16 *out, int ld, int c0,
                                   int zero_rest, int split, hipStream_t st);
hipError_t launch_from_channels_last(const float *y, int ld, int c0, long long n, float scale, float *out,
                                     hipStream_t st);

size_t sumsq_ws_bytes(int nb);
hipError_t launch_layer_threshold(float *mu, int nz, long long plane, const float *maxes, float frac, hipStream_t st);

struct StartCoef {
  float s[kMaxVol], ch[kMaxVol], ce[kMaxVol];
};
hipError_t launch_start_error(const float *y, int ld, int c0, const StartCoef &cf, long long V, const float *t,
                              long long n, float *e, hipStream_t st);
size_t absmax_ws_bytes(int nb);
hipError_t launch_depth_resample(const float *x, float *out, int nb, int nz_in, long long plane, int mode,
                                 hipStream_t st);
hipError_t launch_absmax(const float *x, long long V, int nb, float *part, float *out, hipStream_t st);
hipError_t launch_axpy(long long n, float a, const float *x, float *y, hipStream_t st);
hipError_t launch_sumsq(const float *u, const float *v, long long V, int nb, double *part, double *out,
                        hipStream_t st);
hipError_t launch_start_grad(long long n, long long V, const StartCoef &cf, const float *u, const float *e,
                             const float *y, int yld, int yc0, int relu_mask, __bf16 *g, int gld, int gc0,
                             hipStream_t st);

hipError_t launch_philox(uint64_t seed, uint32_t stream_id, long long first, long long n, uint32_t *out,
                         hipStream_t st);
hipError_t launch_poisson(const float *lam, long long n, uint64_t seed, uint32_t stream_id, float *counts,
                          hipStream_t st);
hipError_t launch_noisy_counts(const float *m, long long n, double scale, double background, uint64_t seed,
                               uint32_t stream_id, float *out, hipStream_t st);
size_t noisy_histogram_ws_bytes(long long n);
hipError_t launch_noisy_histogram(const float *m, long long n, double peak, uint64_t seed, uint32_t stream_id,
                                  float *d, void *ws, hipStream_t st);

}  // namespace ctof
