// Host side of libctof: argument validation, sizes, handles and the
// stream-ordered drivers of the forward model, its adjoint and FISTA.
//
// Operator (Eq. 11, evaluated per frequency):
//   mu [nz][n][n] --row pass r2c--> xz --column FFT--> yhat
//   yhat --contraction--> mhat --inverse column FFT--> xt --row pass c2r--> m
// and the mirror image for the adjoint.  The reconstruction runs FISTA
// (section "Reconstruction Algorithm") with constant step 1/L on
//   1/2 ||A mu - d||^2 + lambda/2 ||mu||^2,  mu >= 0,
// eight launches per iteration: contraction, inverse column FFT, residual
// row pass, column FFT, adjoint contraction, inverse column FFT, prox/FISTA
// row pass, column FFT.  The FISTA momentum weights do not depend on the
// data, so they are computed on the host and passed as launch arguments.
#include "ctof_internal.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

namespace ctof {

thread_local std::string g_err;

ctof_status set_error(ctof_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

const char *last_error() { return g_err.c_str(); }

}  // namespace ctof

namespace {

using ctof::set_error;

int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// FFT size of an n-point scan side: the smallest length >= 2n - 1 (the
// circular convolution then equals the linear one on the scan) among the
// powers of two and 48, 96, 192, 384, 768 (radix-3 first stages), at least
// kMinP.  3 * 2^k sizes cut the kernel spectrum by up to 44% (n = 96: 4,753
// instead of 8,385 matrices) and every FFT pass by up to a quarter.
int fft_size(int n) {
  const int need = 2 * n - 1;
  int p = std::max(ctof::kMinP, next_pow2(need));
  for (int q : {48, 96, 192, 384, 768})
    if (q >= need && q < p) p = q;
  return p;
}

bool finite(double v) { return std::isfinite(v); }

// Legendre-Gauss nodes and weights on [-1, 1] by Newton's method on P_16.
ctof::GaussLegendre16 gauss_legendre16() {
  ctof::GaussLegendre16 gl;
  const int n = 16;
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (x * p1 - p0) / (x * x - 1.0);
    gl.x[i] = x;
    gl.w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  return gl;
}

// Validates a geometry; on success fills the derived tabulation geometry.
ctof_status check_geometry(const ctof_geometry *g, ctof::TabGeom *tg, ctof::LayerDepths *zs) {
  if (!g) return set_error(CTOF_EINVAL, "geometry is NULL");
  if (g->nx <= 0 || g->ny <= 0) return set_error(CTOF_EINVAL, "nx, ny must be >= 1");
  if (g->nz <= 0) return set_error(CTOF_EINVAL, "nz must be >= 1");
  if (g->nt <= 0) return set_error(CTOF_EINVAL, "nt must be >= 1");
  if (!g->z_mm) return set_error(CTOF_EINVAL, "z_mm is NULL");
  if (!(finite(g->pitch_mm) && g->pitch_mm > 0)) return set_error(CTOF_EINVAL, "pitch_mm must be > 0");
  if (!(finite(g->dt_ps) && g->dt_ps > 0)) return set_error(CTOF_EINVAL, "dt_ps must be > 0");
  if (!(finite(g->t0_ps) && g->t0_ps >= 0)) return set_error(CTOF_EINVAL, "t0_ps must be >= 0");
  if (!(finite(g->mus_prime_per_mm) && g->mus_prime_per_mm > 0))
    return set_error(CTOF_EINVAL, "mus_prime_per_mm must be > 0");
  if (!(finite(g->mua_per_mm) && g->mua_per_mm > 0)) return set_error(CTOF_EINVAL, "mua_per_mm must be > 0");
  if (!(finite(g->n_medium) && g->n_medium >= 1)) return set_error(CTOF_EINVAL, "n_medium must be >= 1");
  if (!(finite(g->dz_mm) && g->dz_mm >= 0)) return set_error(CTOF_EINVAL, "dz_mm must be >= 0");
  for (int k = 0; k < g->nz; ++k) {
    if (!(finite(g->z_mm[k]) && g->z_mm[k] > 0)) return set_error(CTOF_EINVAL, "z_mm[%d] must be > 0", k);
    if (k > 0 && !(g->z_mm[k] > g->z_mm[k - 1]))
      return set_error(CTOF_EINVAL, "z_mm must be strictly increasing (index %d)", k);
  }
  double dz = g->dz_mm;
  if (dz == 0.0) {
    if (g->nz < 2) return set_error(CTOF_EINVAL, "nz == 1 needs dz_mm > 0");
    const double step = (g->z_mm[g->nz - 1] - g->z_mm[0]) / (g->nz - 1);
    for (int k = 1; k < g->nz; ++k)
      if (std::fabs((g->z_mm[k] - g->z_mm[k - 1]) - step) > 1e-9 * std::max(1.0, step))
        return set_error(CTOF_EINVAL, "dz_mm == 0 needs uniformly spaced z_mm");
    dz = step;
  }
  // every byte count derived from the shape (kernel spectrum, spectra,
  // workspaces: at most a few dozen bytes per voxel-bin) then fits in 63 bits
  const double total = (double)g->nz * g->nx * g->ny * (double)g->nt;
  if (total > 1.0e15) return set_error(CTOF_EINVAL, "nz*ny*nx*nt = %g exceeds 1e15", total);
  if (g->nx > ctof::kMaxN || g->ny > ctof::kMaxN)
    return set_error(CTOF_EUNSUPPORTED, "a scan side above %d needs an FFT size above 2048", ctof::kMaxN);
  if (g->nz > ctof::kMaxLayers) return set_error(CTOF_EUNSUPPORTED, "nz > %d", ctof::kMaxLayers);
  if (g->nt > (1 << 20)) return set_error(CTOF_EUNSUPPORTED, "nt > 2^20");
  if (tg) {
    const double n = g->n_medium;
    const double mus = g->mus_prime_per_mm, mua = g->mua_per_mm;
    ctof::Optics o;
    o.c = 0.299792458 / n;
    o.D = 1.0 / (3.0 * (mua + mus));
    o.z0 = 1.0 / (mua + mus);
    const double reff = -1.440 / (n * n) + 0.710 / n + 0.668 + 0.0636 * n;
    const double A = (1.0 + reff) / (1.0 - reff);
    o.zb = 2.0 * A * o.D;
    o.mua = mua;
    o.mueff = std::sqrt(mua / o.D);
    tg->n = std::max(g->nx, g->ny);  // kernel offsets cover the longer side in both axes
    tg->nz = g->nz;
    tg->nt = g->nt;
    tg->pitch = g->pitch_mm;
    tg->dt = g->dt_ps;
    tg->t0 = g->t0_ps;
    tg->dv = g->pitch_mm * g->pitch_mm * dz;
    tg->rmin = std::cbrt(3.0 * tg->dv / (4.0 * M_PI));
    tg->o = o;
    tg->Dm = o.D;
    tg->zbm = o.zb;
    tg->tau = 0.0;
  }
  if (zs) {
    for (int k = 0; k < ctof::kMaxLayers; ++k) zs->z[k] = k < g->nz ? g->z_mm[k] : 0.0;
  }
  return CTOF_OK;
}

// Fluorescence mode: emission optics and lifetime on top of a checked geometry.
ctof_status apply_fluorescence(const ctof_geometry *g, const ctof_fluorescence *fl, ctof::TabGeom *tg) {
  if (!fl) return CTOF_OK;
  if (!(std::isfinite(fl->mus_prime_em_per_mm) && fl->mus_prime_em_per_mm > 0))
    return set_error(CTOF_EINVAL, "mus_prime_em_per_mm must be > 0");
  if (!(std::isfinite(fl->lifetime_ps) && fl->lifetime_ps >= 0))
    return set_error(CTOF_EINVAL, "lifetime_ps must be >= 0");
  const double c = 0.299792458 / g->n_medium;
  if (fl->lifetime_ps > 0 && !(1.0 / fl->lifetime_ps < g->mua_per_mm * c))
    return set_error(CTOF_EUNSUPPORTED,
                     "lifetime %g ps is not above 1/(mu_a c) = %g ps (the closed form then needs the complex "
                     "error function)", fl->lifetime_ps, 1.0 / (g->mua_per_mm * c));
  if (tg) {
    const double n = g->n_medium;
    const double reff = -1.440 / (n * n) + 0.710 / n + 0.668 + 0.0636 * n;
    const double A = (1.0 + reff) / (1.0 - reff);
    tg->Dm = 1.0 / (3.0 * (g->mua_per_mm + fl->mus_prime_em_per_mm));
    tg->zbm = 2.0 * A * tg->Dm;
    tg->tau = fl->lifetime_ps;
  }
  return CTOF_OK;
}

size_t elem_size(ctof_precision p) { return p == CTOF_FP64 ? 8 : 4; }

// A caller may pass any 32-bit value where a ctof_precision is expected (C
// and foreign-function callers do); reading an enum object outside its
// enumerators' range is undefined in C++, so an argument is read through
// its bytes (its address) until it is known to be valid.
int32_t prec_value(const ctof_precision *prec) {
  int32_t p;
  static_assert(sizeof(p) == sizeof(*prec), "ctof_precision is 32 bits wide");
  std::memcpy(&p, prec, sizeof p);
  return p;
}
bool valid_prec(const ctof_precision *prec) {
  const int32_t p = prec_value(prec);
  return p >= CTOF_FP64 && p <= CTOF_BF16;
}

// A named host-side range for tracers (rocprofv3 --marker-trace): it spans
// the enqueueing of a call's GPU work, which runs asynchronously; without a
// tracer attached a push or pop costs a call through a null hook.
struct TraceRange {
  bool open;
  explicit TraceRange(const char *name) : open(true) { roctxRangePushA(name); }
  void end() {
    if (open) {
      roctxRangePop();
      open = false;
    }
  }
  ~TraceRange() { end(); }
  TraceRange(const TraceRange &) = delete;
  TraceRange &operator=(const TraceRange &) = delete;
};

struct TabWs {
  size_t q, t1, cm, total;  // offsets
};

TabWs tab_ws(const ctof::Dims &d) {
  TabWs w;
  const size_t per = (size_t)d.nt * d.nz;
  const size_t q = std::max((size_t)d.n * d.n, (size_t)(d.h + 1) * (d.h + 1)) * per * 8;
  const size_t t1 = (size_t)d.n * (d.h + 1) * per * 8;
  const size_t cm = ctof::cosine_matrix_elems(d.n, d.p) * 8;
  w.q = 0;
  w.t1 = ctof::round_up(q, 256);
  w.cm = w.t1 + ctof::round_up(t1, 256);
  w.total = w.cm + ctof::round_up(cm, 256);
  return w;
}

// Workspace of one shape class holding nvol volumes: spectra and column-pass
// intermediates carry every volume's planes, solver state is per volume.
struct ClassWs {
  size_t yhat, mhat, xt, xz, op_total;
  size_t yhat_elems;  // elements of one volume-side spectrum set (the adjoint's parts follow each other)
  int adj_parts;
  size_t y, v, w, hist, scal, g0sq, part, beta, ctr, active, boff, conv, l1, solve_total;
  int nblk_t, nblk_z;
  size_t part_stride;  // doubles per iteration
};

// planes per block of a handle's row passes on the bin (tside) or layer side
int row_planes(const ctof_kernel_s *k, bool tside) {
  const int rb = tside ? k->rb_t : k->rb_z;
  return rb ? rb : (tside ? k->bb_t : k->bb_z);
}

ClassWs class_ws(const ctof_kernel_s *k, int nvol, int max_iter) {
  const ctof::Dims &d = k->dims;
  ClassWs o;
  const size_t es = elem_size(k->prec);
  const bool f64 = k->prec == CTOF_FP64;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += ctof::round_up(bytes, 256);
    return at;
  };
  // the adjoint contraction split along t writes one spectrum set per part
  o.adj_parts = ctof::contract_parts(k, true);
  o.yhat_elems = (size_t)(d.h + 1) * d.p * 2 * nvol * d.nzp;
  o.yhat = take(o.yhat_elems * es * o.adj_parts);
  o.mhat = take((size_t)(d.h + 1) * d.p * 2 * nvol * d.ntp * es);
  o.xt = take((size_t)(d.h + 1) * d.ny * 2 * nvol * d.ntp * es);
  o.xz = take((size_t)(d.h + 1) * d.ny * 2 * nvol * d.nzp * es);
  o.op_total = off;
  const size_t vol = (size_t)d.nz * d.ny * d.nx * es;
  o.y = take(vol * nvol);
  o.v = take(vol);
  o.w = take(vol);
  o.nblk_t = ctof::row_pass_blocks(d, nvol * d.ntp, d.ntp, f64, row_planes(k, true));
  o.nblk_z = ctof::row_pass_blocks(d, nvol * d.nzp, d.nzp, f64, row_planes(k, false));
  o.part_stride = 2 * (size_t)(o.nblk_t + o.nblk_z);
  const int iters = std::max(max_iter, 1);
  o.hist = take((size_t)iters * nvol * 2 * 8);
  o.scal = take((size_t)(64 + nvol) * 8);  // [0..7] scalars, [8..8+nvol) final fits
  o.g0sq = take((size_t)nvol * 8);
  o.part = take((size_t)(iters + 2) * o.part_stride * 8);
  o.beta = take((size_t)iters * 8);
  o.ctr = take(64);
  o.active = take((size_t)nvol * 4);
  o.boff = take((size_t)nvol * 4);
  o.conv = take((size_t)nvol * 4);
  o.l1 = take((size_t)d.nz * 8);
  o.solve_total = off;
  return o;
}

// Launch helpers for one shape class (nvol volumes, one kernel spectrum).
template <typename T>
struct Engine {
  const ctof_kernel_s *k;
  int nvol;
  char *ws;
  ClassWs L;
  hipStream_t st;
  const int *live = nullptr;  // per-volume flags honoured by every launch (batched solves)
  const double *l1dev = nullptr;  // per-layer L1 weights in the workspace when the objective has them
  const ctof::MuxArgs *mux = nullptr;  // source multiplexing of the measurements (Eq. 12), or NULL

  const ctof::Dims &dm() const { return k->dims; }
  T *yhat() const { return reinterpret_cast<T *>(ws + L.yhat); }
  T *mhat() const { return reinterpret_cast<T *>(ws + L.mhat); }
  T *xt() const { return reinterpret_cast<T *>(ws + L.xt); }
  T *xz() const { return reinterpret_cast<T *>(ws + L.xz); }
  T *y(int v) const { return reinterpret_cast<T *>(ws + L.y) + (size_t)v * dm().nz * dm().ny * dm().nx; }
  T *pv() const { return reinterpret_cast<T *>(ws + L.v); }
  T *pw() const { return reinterpret_cast<T *>(ws + L.w); }
  double *hist() const { return reinterpret_cast<double *>(ws + L.hist); }
  double *scal() const { return reinterpret_cast<double *>(ws + L.scal); }
  double *g0sq() const { return reinterpret_cast<double *>(ws + L.g0sq); }
  double *part() const { return reinterpret_cast<double *>(ws + L.part); }
  double *beta() const { return reinterpret_cast<double *>(ws + L.beta); }
  int *ctr() const { return reinterpret_cast<int *>(ws + L.ctr); }
  int *active() const { return reinterpret_cast<int *>(ws + L.active); }
  int *boff() const { return reinterpret_cast<int *>(ws + L.boff); }
  int *conv() const { return reinterpret_cast<int *>(ws + L.conv); }
  double *l1() const { return reinterpret_cast<double *>(ws + L.l1); }
  int Bt() const { return nvol * dm().ntp; }
  int Bz() const { return nvol * dm().nzp; }

  ctof::RowArgs row(int op, bool tside) const {
    ctof::RowArgs a;
    std::memset(&a, 0, sizeof(a));
    a.op = op;
    a.B = tside ? Bt() : Bz();
    a.ppv = tside ? dm().ntp : dm().nzp;
    a.nplanes = tside ? dm().nt : dm().nz;
    a.nvol = nvol;
    a.bb = row_planes(k, tside);
    a.spec_in = tside ? (void *)xt() : (void *)xz();
    a.spec_out = const_cast<void *>(a.spec_in);
    a.l1 = tside ? nullptr : l1dev;
    a.gmap0_at = -1;
    return a;
  }
  hipError_t run_row(const ctof::RowArgs &a) const { return ctof::launch_row_pass<T>(dm(), a, st); }
  // t side: inverse mhat -> xt, forward xt -> mhat;  z side: inverse yhat -> xz, forward xz -> yhat
  hipError_t col_t(bool inverse) const {
    return inverse ? ctof::launch_col_pass<T>(dm(), Bt(), true, mhat(), xt(), st, dm().ntp, k->bb_t, live)
                   : ctof::launch_col_pass<T>(dm(), Bt(), false, xt(), mhat(), st, dm().ntp, k->bb_t, live);
  }
  hipError_t col_z(bool inverse) const {
    // (the inverse pass follows an adjoint contraction and adds its parts)
    return inverse ? ctof::launch_col_pass<T>(dm(), Bz(), true, yhat(), xz(), st, dm().nzp, k->bb_z, live,
                                              L.adj_parts, L.yhat_elems)
                   : ctof::launch_col_pass<T>(dm(), Bz(), false, xz(), yhat(), st, dm().nzp, k->bb_z, live);
  }
  hipError_t contract(bool adjoint) const {
    return adjoint ? ctof::launch_contract(k, true, mhat(), yhat(), st, nvol, live, L.yhat_elems)
                   : ctof::launch_contract(k, false, yhat(), mhat(), st, nvol, live);
  }
  // spatial volume(s) -> yhat
  hipError_t mu_to_spec(const ctof::RowArgs &a) const {
    hipError_t e = run_row(a);
    return e != hipSuccess ? e : col_z(false);
  }
  // yhat -> mhat -> xt
  hipError_t fwd_to_xt() const {
    hipError_t e = contract(false);
    return e != hipSuccess ? e : col_t(true);
  }
  // xt (row-pass output) -> mhat -> yhat -> xz
  hipError_t adj_to_xz() const {
    hipError_t e = col_t(false);
    if (e != hipSuccess) return e;
    e = contract(true);
    return e != hipSuccess ? e : col_z(true);
  }
};

// Multiplexing descriptor -> kernel arguments (sizes from the kernel handle).
ctof_status make_mux(const ctof_kernel_s *k, const ctof_mux *mx, ctof::MuxArgs *a) {
  if (!mx) return set_error(CTOF_EINVAL, "mux is NULL");
  const int ny = k->dims.ny, nx = k->dims.nx;
  if (mx->tile_x < 1 || mx->tile_y < 1 || nx % mx->tile_x != 0 || ny % mx->tile_y != 0)
    return set_error(CTOF_EINVAL, "mux tile %dx%d must divide the %dx%d scan (columns x rows)", mx->tile_x,
                     mx->tile_y, nx, ny);
  const int P = mx->tile_x * mx->tile_y;
  if (P > ctof::kMuxMaxDim)
    return set_error(CTOF_EINVAL, "mux tile of %d positions exceeds %d", P, ctof::kMuxMaxDim);
  if (mx->rows < 1 || mx->rows > ctof::kMuxMaxDim)
    return set_error(CTOF_EINVAL, "mux rows %d must be in [1, %d]", mx->rows, ctof::kMuxMaxDim);
  const size_t es = k->prec == CTOF_FP64 ? 8 : 4;
  if (!mx->s_dev || (reinterpret_cast<uintptr_t>(mx->s_dev) % es) != 0)
    return set_error(CTOF_EINVAL, "mux s_dev is NULL or not aligned to its element");
  std::memset(a, 0, sizeof(*a));
  a->ny = ny;
  a->nx = nx;
  a->nt = k->dims.nt;
  a->tx = mx->tile_x;
  a->ty = mx->tile_y;
  a->M = mx->rows;
  a->P = P;
  a->ntx = nx / mx->tile_x;
  a->ntiles = a->ntx * (ny / mx->tile_y);
  a->S = mx->s_dev;
  if ((long long)a->nt * a->M * a->ntiles * (long long)es >= (1LL << 31) ||
      (long long)a->nt * ny * nx * (long long)es >= (1LL << 31))
    return set_error(CTOF_EINVAL, "multiplexed arrays must stay below 2 GiB");
  return CTOF_OK;
}

bool overlaps(const void *a, const void *b, size_t bytes) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + bytes && y < x + bytes;
}

// Resumption fields shared by both solvers (see ctof_solver_opts).
// Divergence of a FISTA run from its first and last gradient-mapping ratios:
// with a step of at most 1/L_A the ratio does not grow by orders of
// magnitude; with a step beyond 2/L_A it grows geometrically.
constexpr double kDivergence = 1e6;
bool diverged(double first_ratio, double last_ratio) {
  return last_ratio > kDivergence * std::max(1.0, first_ratio);
}

ctof_status check_resume(const ctof_solver_opts *o, bool have_prev) {
  if (o->k0 < 0 || o->k0 > (1 << 30) - o->max_iter)
    return set_error(CTOF_EINVAL, "k0 must be in [0, 2^30 - max_iter]");
  if (o->k0 > 0 && o->warm_start != 1)
    return set_error(CTOF_EINVAL, "a resumed solve (k0 > 0) needs warm_start = 1");
  if (o->k0 > 0 && !have_prev) return set_error(CTOF_EINVAL, "a resumed solve (k0 > 0) needs mu_{k0-1}");
  return CTOF_OK;
}

ctof_status check_kernel(ctof_kernel k) {
  if (!k) return set_error(CTOF_EINVAL, "kernel handle is NULL");
  if (!k->khat) return set_error(CTOF_EINVAL, "kernel handle has no spectrum");
  return CTOF_OK;
}

template <typename T>
Engine<T> engine(const ctof_kernel_s *k, int nvol, void *ws, int max_iter, hipStream_t st) {
  return Engine<T>{k, nvol, reinterpret_cast<char *>(ws), class_ws(k, nvol, max_iter), st};
}

// ---- fixed device scratch for the allocation-free forward entry point ----------
// One array per GPU (each device holds its own copy of a __device__ variable),
// kept until the process ends.  Host code must not pass the array's name to
// a kernel: on the host it is only a stand-in for the symbol, so its device
// address is looked up once per device and used everywhere instead.
static __device__ __align__(256) unsigned char scratch[CTOF_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call per device, with that device current).
ctof_status scratch_address(void **out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return set_error(CTOF_EUNSUPPORTED, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return set_error(CTOF_EHIP, "hipGetSymbolAddress gave no address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CTOF_OK;
}

template <typename T>
ctof_status run_forward(ctof_kernel k, const void *mu, void *m, void *ws, hipStream_t st) {
  const Engine<T> E = engine<T>(k, 1, ws, 1, st);
  ctof::RowArgs a = E.row(ctof::ROW_SPATIAL_TO_SPEC, false);
  a.sp_in[0] = mu;
  HIP_TRY(E.mu_to_spec(a));
  HIP_TRY(E.fwd_to_xt());
  ctof::RowArgs b = E.row(ctof::ROW_SPEC_TO_SPATIAL, true);
  b.sp_out[0] = m;
  HIP_TRY(E.run_row(b));
  return CTOF_OK;
}

template <typename T>
ctof_status run_adjoint(ctof_kernel k, const void *r, void *g, void *ws, hipStream_t st) {
  const Engine<T> E = engine<T>(k, 1, ws, 1, st);
  ctof::RowArgs a = E.row(ctof::ROW_SPATIAL_TO_SPEC, true);
  a.sp_in[0] = r;
  HIP_TRY(E.run_row(a));
  HIP_TRY(E.adj_to_xz());
  ctof::RowArgs b = E.row(ctof::ROW_SPEC_TO_SPATIAL, false);
  b.sp_out[0] = g;
  HIP_TRY(E.run_row(b));
  return CTOF_OK;
}

// out_v = A^T A in_v for the engine's volumes (spatial [nz][ny][nx])
template <typename T>
ctof_status enqueue_normal(const Engine<T> &E, const void *const *in, void *const *out) {
  ctof::RowArgs a = E.row(ctof::ROW_SPATIAL_TO_SPEC, false);
  for (int v = 0; v < E.nvol; ++v) a.sp_in[v] = in[v];
  HIP_TRY(E.mu_to_spec(a));
  HIP_TRY(E.fwd_to_xt());
  HIP_TRY(E.run_row(E.row(ctof::ROW_PASS, true)));
  HIP_TRY(E.adj_to_xz());
  ctof::RowArgs b = E.row(ctof::ROW_SPEC_TO_SPATIAL, false);
  for (int v = 0; v < E.nvol; ++v) b.sp_out[v] = out[v];
  HIP_TRY(E.run_row(b));
  return CTOF_OK;
}

// Warm-start training loss (see ctof_warmstart_loss).  Workspace: operator
// regions for nb volumes, then e, h = H e, u = H h (float [nb][V] each) and
// the FP64 partial sums.
struct StartLossWs {
  size_t op, e, h, u, part, total;
};

StartLossWs start_loss_ws(const ctof_kernel_s *k, int nb) {
  StartLossWs o;
  const ClassWs L = class_ws(k, nb, 1);
  const ctof::Dims &d = k->dims;
  const size_t vol = (size_t)nb * d.nz * d.ny * d.nx * sizeof(float);
  size_t off = ctof::round_up(L.op_total, 256);
  o.op = 0;
  o.e = off;
  off += ctof::round_up(vol, 256);
  o.h = off;
  off += ctof::round_up(vol, 256);
  o.u = off;
  off += ctof::round_up(vol, 256);
  o.part = off;
  off += ctof::round_up(ctof::sumsq_ws_bytes(nb), 256);
  o.total = off;
  return o;
}

ctof_status run_start_loss(const ctof_kernel_s *k, int nb, const ctof_tensor *y, const double *s, const float *target,
                           const double *w, const double *v, double lambda, int relu_mask, const ctof_tensor *grad,
                           double *terms, void *ws, hipStream_t st) {
  const ctof::Dims &d = k->dims;
  const long long V = (long long)d.nz * d.ny * d.nx;
  const long long n = V * nb;
  const StartLossWs o = start_loss_ws(k, nb);
  char *base = reinterpret_cast<char *>(ws);
  float *e = reinterpret_cast<float *>(base + o.e);
  float *h = reinterpret_cast<float *>(base + o.h);
  float *u = reinterpret_cast<float *>(base + o.u);
  const Engine<float> E = engine<float>(k, nb, base + o.op, 1, st);
  const float *yv = reinterpret_cast<const float *>(y->ptr);
  ctof::StartCoef cf{};
  for (int b = 0; b < nb; ++b) {
    cf.s[b] = (float)s[b];
    cf.ch[b] = (float)(2.0 * s[b] * w[b] / nb);
    cf.ce[b] = (float)(2.0 * s[b] * v[b] / nb);
  }
  HIP_TRY(ctof::launch_start_error(yv, y->ld, y->c0, cf, V, target, n, e, st));
  std::vector<const void *> ein(nb), hin(nb);
  std::vector<void *> hout(nb), uout(nb);
  for (int b = 0; b < nb; ++b) {
    ein[b] = e + (size_t)b * V;
    hout[b] = h + (size_t)b * V;
    hin[b] = h + (size_t)b * V;
    uout[b] = u + (size_t)b * V;
  }
  if (ctof_status r = enqueue_normal(E, ein.data(), hout.data()); r != CTOF_OK) return r;
  HIP_TRY(ctof::launch_axpy(n, (float)lambda, e, h, st));
  if (ctof_status r = enqueue_normal(E, hin.data(), uout.data()); r != CTOF_OK) return r;
  HIP_TRY(ctof::launch_axpy(n, (float)lambda, h, u, st));
  HIP_TRY(ctof::launch_sumsq(h, e, V, nb, reinterpret_cast<double *>(base + o.part), terms, st));
  HIP_TRY(ctof::launch_start_grad(n, V, cf, u, e, yv, y->ld, y->c0, relu_mask, reinterpret_cast<__bf16 *>(grad->ptr),
                                  grad->ld, grad->c0, st));
  return CTOF_OK;
}

// FISTA's step weights beta_k = (t_k - 1) / t_{k+1} (t_1 = 1,
// t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2), for k = first .. first + count - 1
std::vector<double> fista_betas(int first, int count) {
  std::vector<double> b(count);
  double t = 1.0;
  for (int k = 0; k < first + count; ++k) {
    const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
    if (k >= first) b[k - first] = (t - 1.0) / tn;
    t = tn;
  }
  return b;
}

// Bin-side pass of a multiplexed solve (Eq. 12): the spectra in xt back to
// the histograms m_v (held in the idle mhat buffer), r_v = S^T (S m_v - y_v)
// in place (y NULL: r = S^T S m), FP64 half squares of S m - y into
// `partials` (nblk_t pairs, each volume's run of nblk_t / nvol in turn) when
// given, and r back to spectra in xt.  by_counter: inside a captured
// iteration, partials advance with the device counter and frozen volumes are
// skipped.
template <typename T>
ctof_status enqueue_mux_residual(const Engine<T> &E, const void *const *y, double *partials, bool by_counter) {
  const ctof::Dims &dm = E.dm();
  const size_t vt = (size_t)dm.nt * dm.ny * dm.nx;
  ctof::RowArgs a = E.row(ctof::ROW_SPEC_TO_SPATIAL, true);
  for (int v = 0; v < E.nvol; ++v) a.sp_out[v] = E.mhat() + (size_t)v * vt;
  if (by_counter) a.active = E.live;
  HIP_TRY(E.run_row(a));
  const int per = E.L.nblk_t / E.nvol;
  for (int v = 0; v < E.nvol; ++v) {
    ctof::MuxArgs m = *E.mux;
    m.in = E.mhat() + (size_t)v * vt;
    m.out = E.mhat() + (size_t)v * vt;
    m.y = y ? y[v] : nullptr;
    m.partials = partials ? partials + 2 * (size_t)v * per : nullptr;
    m.npart = per;
    if (by_counter) {
      m.ctr = E.ctr();
      m.part_stride = E.L.part_stride;
      m.active = E.live;
      m.vol = v;
    }
    const int blocks = std::min(ctof::mux_default_blocks(m, sizeof(T) == 8), per);
    HIP_TRY(ctof::launch_mux(ctof::MUX_NORMAL, sizeof(T) == 8, m, blocks, E.st));
  }
  ctof::RowArgs b = E.row(ctof::ROW_SPATIAL_TO_SPEC, true);
  for (int v = 0; v < E.nvol; ++v) b.sp_in[v] = E.mhat() + (size_t)v * vt;
  if (by_counter) b.active = E.live;
  HIP_TRY(E.run_row(b));
  return CTOF_OK;
}

// S^T y_v of every volume into its histogram slot of mhat (set-up of a
// multiplexed solve: the gradient-mapping denominator needs A^T S^T y)
template <typename T>
ctof_status enqueue_mux_adjoint_data(const Engine<T> &E, const void *const *y, std::vector<const void *> &sty) {
  const ctof::Dims &dm = E.dm();
  const size_t vt = (size_t)dm.nt * dm.ny * dm.nx;
  sty.resize(E.nvol);
  for (int v = 0; v < E.nvol; ++v) {
    ctof::MuxArgs a = *E.mux;
    a.in = y[v];
    a.out = E.mhat() + (size_t)v * vt;
    sty[v] = a.out;
    HIP_TRY(ctof::launch_mux(ctof::MUX_ADJ, sizeof(T) == 8, a, ctof::mux_default_blocks(a, sizeof(T) == 8), E.st));
  }
  return CTOF_OK;
}

// L_A of one class by power iteration on a single vector (FP64 Rayleigh
// quotients); enqueued on the engine's stream, result in scal()[1].
template <typename T>
ctof_status enqueue_power_iteration(const Engine<T> &E1, int iters) {
  const ctof::Dims &dm = E1.dm();
  const size_t vol = (size_t)dm.nz * dm.ny * dm.nx;
  if (sizeof(T) == 8)
    HIP_TRY(ctof::launch_fill_value_f64(reinterpret_cast<double *>(E1.pv()), vol, 1.0 / std::sqrt((double)vol), E1.st));
  else
    HIP_TRY(ctof::launch_fill_value(reinterpret_cast<float *>(E1.pv()), vol, (float)(1.0 / std::sqrt((double)vol)), E1.st));
  for (int j = 0; j < iters; ++j) {
    ctof::RowArgs a = E1.row(j == 0 ? ctof::ROW_SPATIAL_TO_SPEC : ctof::ROW_SCALE_TO_SPEC, false);
    a.sp_in[0] = j == 0 ? (const void *)E1.pv() : (const void *)E1.pw();
    a.sp_out[0] = E1.pv();
    a.scalar = E1.scal() + 0;
    HIP_TRY(E1.mu_to_spec(a));
    HIP_TRY(E1.fwd_to_xt());
    if (E1.mux) {
      if (ctof_status s = enqueue_mux_residual(E1, nullptr, nullptr, false); s != CTOF_OK) return s;
    } else {
      HIP_TRY(E1.run_row(E1.row(ctof::ROW_PASS, true)));
    }
    HIP_TRY(E1.adj_to_xz());
    ctof::RowArgs c = E1.row(ctof::ROW_POWER_W, false);
    c.sp_in[0] = E1.pv();
    c.sp_out[0] = E1.pw();
    c.partials = E1.part();
    HIP_TRY(E1.run_row(c));
    HIP_TRY(ctof::launch_reduce_rows(E1.part(), E1.L.nblk_z, 2, 2, E1.scal() + 0, E1.st));
  }
  return CTOF_OK;
}

// Per-layer sensitivity e(z) = ||A e_z||^2 of a unit absorber at the window
// centre of layer z, into e_dev[z] (FP64): the forward model's bin-side
// spectrum goes through the row pass that sums 1/2 x^2 per block.
template <typename T>
ctof_status enqueue_layer_energy(const Engine<T> &E, double *e_dev) {
  const ctof::Dims &dm = E.dm();
  const size_t vol = (size_t)dm.nz * dm.ny * dm.nx;
  T *unit = E.pv();
  for (int z = 0; z < dm.nz; ++z) {
    HIP_TRY(ctof::launch_fill_zero(unit, vol * sizeof(T), E.st));
    T *at = unit + ((size_t)z * dm.ny + dm.ny / 2) * dm.nx + dm.nx / 2;
    if (sizeof(T) == 8)
      HIP_TRY(ctof::launch_fill_value_f64(reinterpret_cast<double *>(at), 1, 1.0, E.st));
    else
      HIP_TRY(ctof::launch_fill_value(reinterpret_cast<float *>(at), 1, 1.0f, E.st));
    ctof::RowArgs a = E.row(ctof::ROW_SPATIAL_TO_SPEC, false);
    a.sp_in[0] = unit;
    HIP_TRY(E.mu_to_spec(a));
    HIP_TRY(E.fwd_to_xt());
    ctof::RowArgs b = E.row(ctof::ROW_PASS, true);
    b.partials = E.part();
    HIP_TRY(E.run_row(b));
    HIP_TRY(ctof::launch_reduce_rows(E.part(), E.L.nblk_t, 2, 1, e_dev + z, E.st));
  }
  return CTOF_OK;
}

// ||max(0, A^T d_v)||^2 per volume into g0sq()[v]
template <typename T>
ctof_status enqueue_gmap0(const Engine<T> &E, const void *const *d) {
  ctof::RowArgs a = E.row(ctof::ROW_SPATIAL_TO_SPEC, true);
  for (int v = 0; v < E.nvol; ++v) a.sp_in[v] = d[v];
  HIP_TRY(E.run_row(a));
  HIP_TRY(E.adj_to_xz());
  ctof::RowArgs b = E.row(ctof::ROW_GMAP0, false);
  b.partials = E.part();
  HIP_TRY(E.run_row(b));
  HIP_TRY(ctof::launch_reduce_volumes(E.part(), E.L.nblk_z, E.nvol, E.g0sq(), E.st));
  return CTOF_OK;
}

// one FISTA iteration of every volume of the class; partials and beta come
// from the device iteration counter when `by_counter`, else from `it`
template <typename T>
ctof_status enqueue_iteration(const Engine<T> &E, const void *const *d, void *const *mu, double tau,
                              double lam, bool by_counter, int it, double beta, void *const *prev = nullptr,
                              bool g0_first = false) {
  HIP_TRY(E.contract(false));
  HIP_TRY(E.col_t(true));
  if (E.mux) {
    if (ctof_status s = enqueue_mux_residual(E, d, E.part() + (by_counter ? 0 : (size_t)it * E.L.part_stride),
                                             by_counter);
        s != CTOF_OK)
      return s;
  } else {
    ctof::RowArgs a = E.row(ctof::ROW_RESIDUAL, true);
    for (int v = 0; v < E.nvol; ++v) a.sp_in[v] = d[v];
    a.partials = E.part() + (by_counter ? 0 : (size_t)it * E.L.part_stride);
    if (by_counter) {
      a.iter_ctr = E.ctr();
      a.part_stride = E.L.part_stride;
      a.active = E.live;
    }
    HIP_TRY(E.run_row(a));
  }
  HIP_TRY(E.col_t(false));
  HIP_TRY(E.contract(true));
  HIP_TRY(E.col_z(true));
  ctof::RowArgs b = E.row(ctof::ROW_FISTA, false);
  for (int v = 0; v < E.nvol; ++v) {
    b.sp_in[v] = E.y(v);
    b.sp_out[v] = E.y(v);
    b.sp_aux[v] = mu[v];
    b.sp_prev[v] = prev ? prev[v] : nullptr;
  }
  b.partials = E.part() + 2 * (size_t)E.L.nblk_t + (by_counter ? 0 : (size_t)it * E.L.part_stride);
  b.tau = tau;
  b.lambda = lam;
  b.beta = beta;
  if (g0_first) b.gmap0_at = 0;
  if (by_counter) {
    b.iter_ctr = E.ctr();
    b.part_stride = E.L.part_stride;
    b.beta_tab = E.beta();
    b.beta_off = E.boff();
    b.active = E.live;
  }
  HIP_TRY(E.run_row(b));
  HIP_TRY(E.col_z(false));
  if (by_counter) HIP_TRY(ctof::launch_increment(E.ctr(), E.st));
  return CTOF_OK;
}

// y_v = mu_v (zeroed first for a cold start) and the spectrum of y (the
// spectrum of a cold start is zero and is written as such)
template <typename T>
ctof_status enqueue_start(const Engine<T> &E, void *const *mu, bool warm) {
  const ctof::Dims &dm = E.dm();
  const size_t vol = (size_t)dm.nz * dm.ny * dm.nx;
  if (!warm) {
    for (int v = 0; v < E.nvol; ++v) {
      HIP_TRY(ctof::launch_fill_zero(mu[v], vol * sizeof(T), E.st));
      HIP_TRY(ctof::launch_fill_zero(E.y(v), vol * sizeof(T), E.st));
    }
    HIP_TRY(ctof::launch_fill_zero(E.yhat(), E.L.yhat_elems * sizeof(T), E.st));
    return CTOF_OK;
  }
  for (int v = 0; v < E.nvol; ++v)
    HIP_TRY(hipMemcpyAsync(E.y(v), mu[v], vol * sizeof(T), hipMemcpyDeviceToDevice, E.st));
  ctof::RowArgs a = E.row(ctof::ROW_SPATIAL_TO_SPEC, false);
  for (int v = 0; v < E.nvol; ++v) a.sp_in[v] = E.y(v);
  HIP_TRY(E.mu_to_spec(a));
  return CTOF_OK;
}

// Resumed start: y_v = mu_v + beta (mu_v - prev_v) (mu_v = mu_k0, prev_v =
// mu_{k0-1}, beta = beta_{k0}) and the spectrum of y.
template <typename T>
ctof_status enqueue_resume(const Engine<T> &E, void *const *mu, const void *const *prev, double beta) {
  ctof::RowArgs a = E.row(ctof::ROW_EXTRAPOLATE, false);
  for (int v = 0; v < E.nvol; ++v) {
    a.sp_in[v] = mu[v];
    a.sp_aux[v] = const_cast<void *>(prev[v]);
    a.sp_out[v] = E.y(v);
  }
  a.beta = beta;
  HIP_TRY(E.mu_to_spec(a));
  return CTOF_OK;
}

// Zero-start fallback: the flagged volumes restart from mu = 0 (mu and y
// zeroed, spectrum of y recomputed for the class).
template <typename T>
ctof_status restart_from_zero(const Engine<T> &E, void *const *mu, const std::vector<int> &reset) {
  const ctof::Dims &dm = E.dm();
  const size_t vol = (size_t)dm.nz * dm.ny * dm.nx;
  bool any = false;
  for (int v = 0; v < E.nvol; ++v)
    if (reset[v]) {
      any = true;
      HIP_TRY(ctof::launch_fill_zero(mu[v], vol * sizeof(T), E.st));
      HIP_TRY(ctof::launch_fill_zero(E.y(v), vol * sizeof(T), E.st));
    }
  if (!any) return CTOF_OK;
  ctof::RowArgs a = E.row(ctof::ROW_SPATIAL_TO_SPEC, false);
  for (int v = 0; v < E.nvol; ++v) a.sp_in[v] = E.y(v);
  HIP_TRY(E.mu_to_spec(a));
  return CTOF_OK;
}

// 1/2 ||A mu_v - d_v||^2 per volume into out[v] (device)
template <typename T>
ctof_status enqueue_final_fit(const Engine<T> &E, const void *const *d, void *const *mu, double *pf,
                              double *out, bool have_spec = false) {
  // (have_spec: the spectrum buffer already holds that of mu)
  if (!have_spec) {
    ctof::RowArgs a = E.row(ctof::ROW_SPATIAL_TO_SPEC, false);
    for (int v = 0; v < E.nvol; ++v) a.sp_in[v] = mu[v];
    HIP_TRY(E.mu_to_spec(a));
  }
  HIP_TRY(E.fwd_to_xt());
  if (E.mux) {
    if (ctof_status s = enqueue_mux_residual(E, d, pf, false); s != CTOF_OK) return s;
  } else {
    // only the norm is needed: no spectrum of the residual
    ctof::RowArgs b = E.row(ctof::ROW_FIT, true);
    for (int v = 0; v < E.nvol; ++v) b.sp_in[v] = d[v];
    b.partials = pf;
    HIP_TRY(E.run_row(b));
  }
  HIP_TRY(ctof::launch_reduce_volumes(pf, E.L.nblk_t, E.nvol, out, E.st));
  return CTOF_OK;
}

template <typename T>
ctof_status run_reconstruct(ctof_kernel k, const void *d, void *mu, const ctof_solver_opts *opt,
                            ctof_solver_report *rep, void *ws, hipStream_t st) {
  TraceRange trace("ctof_reconstruct");
  const ctof::Dims &dm = k->dims;
  Engine<T> E = engine<T>(k, 1, ws, opt->max_iter, st);
  const void *dd[1] = {d};
  void *mm[1] = {mu};
  double *scal = E.scal();
  const int K = opt->max_iter;
  const int k0 = opt->k0;
  const size_t vol = (size_t)dm.nz * dm.ny * dm.nx;
  // scalars: [0] |w|^2  [1] <v,w>  [3] final fit  [5..6] last history row  [16..24] packed report
  HIP_TRY(ctof::launch_fill_zero(scal, 64 * 8, st));
  if (opt->lambda_l1_z) {
    HIP_TRY(hipMemcpyAsync(E.l1(), opt->lambda_l1_z, (size_t)dm.nz * sizeof(double), hipMemcpyHostToDevice, st));
    E.l1dev = E.l1();
  }
  ctof::MuxArgs mux;
  if (opt->mux) {
    if (ctof_status s = make_mux(k, opt->mux, &mux); s != CTOF_OK) return s;
    E.mux = &mux;
  }
  // A zero start takes its first step from y = 0, where the gradient is
  // -A^T d: the gradient-mapping denominator ||max(0, A^T d)|| is then
  // accumulated inside that step instead of by a separate adjoint.
  const bool fused_g0 = opt->warm_start == 0 && k0 == 0;
  if (!fused_g0) {
    if (E.mux) {
      // the gradient-mapping denominator needs A^T S^T y: S^T y into mhat first
      std::vector<const void *> sty;
      if (ctof_status s = enqueue_mux_adjoint_data(E, dd, sty); s != CTOF_OK) return s;
      if (ctof_status s = enqueue_gmap0(E, sty.data()); s != CTOF_OK) return s;
    } else {
      if (ctof_status s = enqueue_gmap0(E, dd); s != CTOF_OK) return s;
    }
  }

  double lam = opt->lambda_tikhonov, Lip = opt->lipschitz, LA = 0.0;
  if (Lip == 0.0) {
    TraceRange tp("power iteration");
    if (ctof_status s = enqueue_power_iteration(E, opt->power_iters > 0 ? opt->power_iters : 50); s != CTOF_OK)
      return s;
    double hs[2];
    HIP_TRY(hipMemcpyAsync(hs, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    LA = hs[1];
    if (!std::isfinite(LA) || !(LA > 0)) {
      rep->status = CTOF_ENONFINITE;
      return set_error(CTOF_ENONFINITE, "power iteration gave a non-positive or non-finite ||A||^2 (%g)", LA);
    }
    if (lam < 0) lam = 1e-3 * LA;
    Lip = 1.01 * LA + lam;
  }
  const double tau = 1.0 / Lip;
  rep->lipschitz = Lip;
  rep->lambda = lam;
  rep->lipschitz_a = LA;

  // step weights beta_k for k = kb .. k0 + K - 1 (beta_{k0-1} extrapolates a resumed start)
  const int kb = std::max(k0 - 1, 0);
  const std::vector<double> btab = fista_betas(kb, k0 + K - kb);
  auto beta_at = [&](int kk) { return btab[(size_t)(kk - kb)]; };
  if (k0 > 0) {
    const void *prev[1] = {opt->mu_prev_dev};
    if (ctof_status s = enqueue_resume(E, mm, prev, beta_at(k0 - 1)); s != CTOF_OK) return s;
  } else {
    if (ctof_status s = enqueue_start(E, mm, opt->warm_start != 0); s != CTOF_OK) return s;
  }
  // optional stage timing: events around the contraction and FFT groups of
  // every `timing`-th iteration (0, n, 2n, ...) and one at the loop's end
  const int tstride = opt->timing;
  const int nsamp = tstride > 0 ? (K + tstride - 1) / tstride : 0;
  std::vector<hipEvent_t> ev;
  struct EventGuard {
    std::vector<hipEvent_t> *v;
    ~EventGuard() {
      for (hipEvent_t e : *v) (void)hipEventDestroy(e);
    }
  } guard{&ev};
  if (tstride > 0) {
    ev.resize((size_t)nsamp * 5 + 1, nullptr);
    for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
  }
  auto mark = [&](int it, int j) -> hipError_t {
    return (tstride > 0 && it % tstride == 0) ? hipEventRecord(ev[(size_t)(it / tstride) * 5 + j], st)
                                              : hipSuccess;
  };
  // iterations after which the loop may stop: there mu_{k-1} is kept for a
  // later resumption
  int done = 0;
  int base = 0;  // first iteration of the kept run (1 after a zero-start fallback)
  auto may_stop = [&](int it) {
    return it == K - 1 || (opt->rel_tol > 0 && (it + 1 - base) % opt->check_every == 0);
  };
  TraceRange tl("iterations");
  for (int it = 0; it < K; ++it) {
    double *pk = E.part() + (size_t)it * E.L.part_stride;
    HIP_TRY(mark(it, 0));
    HIP_TRY(E.contract(false));
    HIP_TRY(mark(it, 1));
    HIP_TRY(E.col_t(true));
    if (E.mux) {
      if (ctof_status s = enqueue_mux_residual(E, dd, pk, false); s != CTOF_OK) return s;
    } else {
      ctof::RowArgs a = E.row(ctof::ROW_RESIDUAL, true);
      a.sp_in[0] = d;
      a.partials = pk;
      HIP_TRY(E.run_row(a));
    }
    HIP_TRY(E.col_t(false));
    HIP_TRY(mark(it, 2));
    HIP_TRY(E.contract(true));
    HIP_TRY(mark(it, 3));
    HIP_TRY(E.col_z(true));
    ctof::RowArgs b = E.row(ctof::ROW_FISTA, false);
    b.sp_in[0] = E.y(0);
    b.sp_out[0] = E.y(0);
    b.sp_aux[0] = mu;
    if (opt->mu_prev_dev && may_stop(it)) b.sp_prev[0] = opt->mu_prev_dev;
    b.partials = pk + 2 * (size_t)E.L.nblk_t;
    b.tau = tau;
    b.lambda = lam;
    b.beta = beta_at(k0 + it - base);
    if (fused_g0 && it == 0) b.gmap0_at = 0;
    // the last step transforms mu_K itself: the final data fit needs its
    // spectrum, and no step follows that would use the one of y_{K+1}
    b.spec_of_mu = it == K - 1;
    HIP_TRY(E.run_row(b));
    if (fused_g0 && it == 0)
      HIP_TRY(ctof::launch_reduce_volumes(pk + 2 * (size_t)E.L.nblk_t + 1, E.L.nblk_z, 1, E.g0sq(), st));
    HIP_TRY(E.col_z(false));
    HIP_TRY(mark(it, 4));
    done = it + 1;
    if (opt->warm_start == 2 && it == 0) {
      HIP_TRY(ctof::launch_history(E.part(), 1, 1, E.L.nblk_t, E.L.nblk_z, E.L.part_stride, tau, E.g0sq(),
                                   scal + 5, st));
      double h1[2];
      HIP_TRY(hipMemcpyAsync(h1, scal + 5, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (!(h1[1] <= 1.0)) {
        // a fresh zero start: the next step is the first of its sequence
        rep->fell_back = 1;
        base = 1;
        if (ctof_status s = restart_from_zero(E, mm, std::vector<int>{1}); s != CTOF_OK) return s;
      }
    }
    // checks follow the kept run's count (a restarted scan stops where a zero start would)
    if (opt->rel_tol > 0 && done > base && ((done - base) % opt->check_every == 0) && done < K) {
      HIP_TRY(ctof::launch_history(E.part() + (size_t)it * E.L.part_stride, 1, 1, E.L.nblk_t, E.L.nblk_z,
                                   E.L.part_stride, tau, E.g0sq(), scal + 5, st));
      double h2[2];
      HIP_TRY(hipMemcpyAsync(h2, scal + 5, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (!std::isfinite(h2[0]) || !std::isfinite(h2[1])) break;
      if (h2[1] <= opt->rel_tol) break;
    }
  }
  tl.end();
  if (tstride > 0) HIP_TRY(hipEventRecord(ev[(size_t)nsamp * 5], st));  // end of the loop
  const int kept = done - base;
  HIP_TRY(ctof::launch_history(E.part() + (size_t)base * E.L.part_stride, kept, 1, E.L.nblk_t, E.L.nblk_z,
                               E.L.part_stride, tau, E.g0sq(), E.hist(), st));
  if (opt->history_dev && kept > 0)
    HIP_TRY(hipMemcpyAsync(opt->history_dev, E.hist(), (size_t)kept * 2 * sizeof(double),
                           hipMemcpyDeviceToDevice, st));
  // after all K steps the spectrum buffer holds that of mu_K (also after a
  // fallback in a one-step call: mu = y = 0 and their spectrum recomputed);
  // a call that skips the final fit reports the last history row's instead
  // (a one-step call that fell back has no kept row: it still computes it)
  const bool final_fit = !opt->skip_final_fit || kept == 0;
  if (final_fit)
    if (ctof_status s = enqueue_final_fit(E, dd, mm, E.part() + (size_t)K * E.L.part_stride, scal + 3, done == K);
        s != CTOF_OK)
      return s;
  // scalars, first and last history rows and ||G(0)||^2, read back with one copy
  double pk[9];
  HIP_TRY(ctof::launch_pack_report(scal, E.hist(), kept, E.g0sq(), scal + 16, st));
  HIP_TRY(hipMemcpyAsync(pk, scal + 16, sizeof(pk), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const double *hs = pk, *h0 = pk + 4, *hl = pk + 6;
  const double g0 = pk[8];
  if (tstride > 0 && done > 0) {
    // iterations 0, n, ... below `done` were timed (an early stop leaves the
    // later samples unrecorded)
    const int ntimed = (done + tstride - 1) / tstride;
    double acc[4] = {0, 0, 0, 0};
    for (int q = 0; q < ntimed; ++q) {
      for (int j = 0; j < 4; ++j) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ev[(size_t)q * 5 + j], ev[(size_t)q * 5 + j + 1]));
        acc[j] += ms;
      }
    }
    float loop = 0.f;
    HIP_TRY(hipEventElapsedTime(&loop, ev[0], ev[(size_t)nsamp * 5]));
    rep->ms_contract_fwd = acc[0];
    rep->ms_fft_t = acc[1];
    rep->ms_contract_adj = acc[2];
    rep->ms_fft_z = acc[3];
    rep->ms_loop = loop;
    rep->timed_iters = ntimed;
  }
  rep->iters = done;
  rep->fista_k = k0 + kept;
  rep->datafit0 = h0[0];
  rep->datafit = final_fit ? hs[3] : hl[0];
  rep->gmap_ratio = hl[1];
  if (kept == 0) {
    // a one-iteration call that fell back returns the zero start itself,
    // whose ratio is 1 by the definition of the denominator
    rep->datafit0 = hs[3];
    rep->gmap_ratio = 1.0;
  }
  rep->gmap0 = std::sqrt(g0);
  rep->status = CTOF_OK;
  (void)vol;
  if (!std::isfinite(rep->datafit) || !std::isfinite(rep->datafit0) || !std::isfinite(rep->gmap_ratio) ||
      !std::isfinite(rep->gmap0)) {
    rep->status = CTOF_ENONFINITE;
    return set_error(CTOF_ENONFINITE, "non-finite FP64 norm during the solve (stopped after %d iterations)", done);
  }
  if (kept > 0 && diverged(h0[1], hl[1])) {
    rep->status = CTOF_EDIVERGED;
    return set_error(CTOF_EDIVERGED, "the solve diverged: gradient-mapping ratio %g after %d iterations, %g after the "
                     "first (is lipschitz below the operator's?)", hl[1], kept, h0[1]);
  }
  return CTOF_OK;
}

// ---- batched reconstruction -----------------------------------------------------
struct ClassPlan {
  const ctof_kernel_s *k;
  std::vector<int> scans;
  size_t off;
  ClassWs L;
  double tau, lam, lip, lip_a;
  bool active;
};

std::vector<ClassPlan> plan_classes(int nscan, const ctof_kernel *ks, int max_iter, size_t *total) {
  std::vector<ClassPlan> cls;
  for (int i = 0; i < nscan; ++i) {
    ClassPlan *c = nullptr;
    for (auto &x : cls)
      if (x.k == ks[i] && (int)x.scans.size() < ctof::kMaxVol) c = &x;
    if (!c) {
      cls.push_back(ClassPlan{ks[i], {}, 0, ClassWs{}, 0, 0, 0, 0, true});
      c = &cls.back();
    }
    c->scans.push_back(i);
  }
  size_t off = 0;
  for (auto &c : cls) {
    c.L = class_ws(c.k, (int)c.scans.size(), max_iter);
    c.off = off;
    off += ctof::round_up(c.L.solve_total, 256);
  }
  if (total) *total = off;
  return cls;
}

// Internal streams and events for graph capture; destroyed on every exit.
constexpr int kBranches = 4;
struct StreamGuard {
  hipStream_t s = nullptr;
  hipStream_t br[kBranches] = {};
  hipEvent_t fork = nullptr, join[kBranches] = {};
  hipEvent_t chunk_end[2] = {};
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
  // graphs replaced while a launch of theirs may still run: destroyed at the end
  std::vector<hipGraphExec_t> old_x;
  std::vector<hipGraph_t> old_g;
  void reset_graph() {
    if (x) old_x.push_back(x);
    if (g) old_g.push_back(g);
    x = nullptr;
    g = nullptr;
  }
  ~StreamGuard() {
    reset_graph();
    for (hipGraphExec_t e : old_x) (void)hipGraphExecDestroy(e);
    for (hipGraph_t e : old_g) (void)hipGraphDestroy(e);
    for (hipEvent_t e : chunk_end)
      if (e) (void)hipEventDestroy(e);
    for (int b = 0; b < kBranches; ++b) {
      if (join[b]) (void)hipEventDestroy(join[b]);
      if (br[b]) (void)hipStreamDestroy(br[b]);
    }
    if (fork) (void)hipEventDestroy(fork);
    if (s) (void)hipStreamDestroy(s);
  }
};

template <typename T>
ctof_status run_batched(int nscan, const ctof_kernel *ks, const void *const *d, void *const *mu,
                        const ctof_solver_opts *opt, ctof_solver_report *rep, void *ws, hipStream_t st) {
  TraceRange trace("ctof_reconstruct_batched");
  const int K = opt->max_iter;
  std::vector<ClassPlan> cls = plan_classes(nscan, ks, K, nullptr);
  char *base = reinterpret_cast<char *>(ws);
  std::vector<Engine<T>> E;
  std::vector<std::vector<const void *>> dv(cls.size());
  std::vector<std::vector<void *>> mv(cls.size()), pv(cls.size());
  const int k0 = opt->k0;
  // a zero start accumulates ||max(0, A^T d)|| inside its first step (see run_reconstruct)
  const bool fused_g0 = opt->warm_start == 0 && k0 == 0;
  std::vector<ctof::MuxArgs> muxes(cls.size());  // sized once: the engines keep pointers into it
  for (size_t c = 0; c < cls.size(); ++c) {
    E.push_back(Engine<T>{cls[c].k, (int)cls[c].scans.size(), base + cls[c].off, cls[c].L, st});
    if (opt->mux) {
      if (ctof_status s = make_mux(cls[c].k, opt->mux, &muxes[c]); s != CTOF_OK) return s;
      E.back().mux = &muxes[c];
    }
    if (opt->lambda_l1_z) {
      HIP_TRY(hipMemcpyAsync(E.back().l1(), opt->lambda_l1_z, (size_t)cls[c].k->dims.nz * sizeof(double),
                             hipMemcpyHostToDevice, st));
      E.back().l1dev = E.back().l1();
    }
    for (int i : cls[c].scans) {
      dv[c].push_back(d[i]);
      mv[c].push_back(mu[i]);
      pv[c].push_back(opt->mu_prev_scans ? opt->mu_prev_scans[i] : nullptr);
    }
  }
  auto prev_of = [&](size_t c) -> void *const * { return opt->mu_prev_scans ? pv[c].data() : nullptr; };
  // set-up: ||G(0)|| per volume and L_A per class (one vector per class)
  for (size_t c = 0; c < cls.size(); ++c) {
    HIP_TRY(ctof::launch_fill_zero(E[c].scal(), 64 * 8, st));
    if (fused_g0) {
      // nothing here: the first step fills g0sq
    } else if (E[c].mux) {
      std::vector<const void *> sty;
      if (ctof_status s = enqueue_mux_adjoint_data(E[c], dv[c].data(), sty); s != CTOF_OK) return s;
      if (ctof_status s = enqueue_gmap0(E[c], sty.data()); s != CTOF_OK) return s;
    } else {
      if (ctof_status s = enqueue_gmap0(E[c], dv[c].data()); s != CTOF_OK) return s;
    }
    if (opt->lipschitz == 0.0 && !opt->lipschitz_scans) {
      Engine<T> E1 = E[c];
      const bool f64 = E1.k->prec == CTOF_FP64;
      E1.nvol = 1;
      E1.L.nblk_t = ctof::row_pass_blocks(E1.dm(), E1.dm().ntp, E1.dm().ntp, f64, row_planes(E1.k, true));
      E1.L.nblk_z = ctof::row_pass_blocks(E1.dm(), E1.dm().nzp, E1.dm().nzp, f64, row_planes(E1.k, false));
      if (ctof_status s = enqueue_power_iteration(E1, opt->power_iters > 0 ? opt->power_iters : 50); s != CTOF_OK)
        return s;
    }
  }
  for (size_t c = 0; c < cls.size(); ++c) {
    double lam = opt->lambda_tikhonov, lip = opt->lipschitz, la = 0.0;
    if (opt->lipschitz_scans) {
      lip = opt->lipschitz_scans[cls[c].scans[0]];
      lam = opt->lambda_scans[cls[c].scans[0]];
      for (int i : cls[c].scans)
        if (opt->lipschitz_scans[i] != lip || opt->lambda_scans[i] != lam)
          return set_error(CTOF_EINVAL, "scans %d and %d share a handle but not L / lambda", cls[c].scans[0], i);
    } else if (lip == 0.0) {
      double hs[2];
      HIP_TRY(hipMemcpyAsync(hs, E[c].scal(), 2 * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      la = hs[1];
      if (!std::isfinite(la) || !(la > 0))
        return set_error(CTOF_ENONFINITE, "power iteration of class %zu gave ||A||^2 = %g", c, la);
      if (lam < 0) lam = 1e-3 * la;
      lip = 1.01 * la + lam;
    }
    cls[c].lam = lam;
    cls[c].lip = lip;
    cls[c].lip_a = la;
    cls[c].tau = 1.0 / lip;
    if (k0 > 0) {
      std::vector<const void *> prev(pv[c].begin(), pv[c].end());
      if (ctof_status s = enqueue_resume(E[c], mv[c].data(), prev.data(), fista_betas(k0 - 1, 1)[0]); s != CTOF_OK)
        return s;
    } else {
      if (ctof_status s = enqueue_start(E[c], mv[c].data(), opt->warm_start != 0); s != CTOF_OK) return s;
    }
    HIP_TRY(ctof::launch_beta_table(E[c].beta(), k0, K, st));
    HIP_TRY(ctof::launch_fill_int(E[c].ctr(), 1, 0, st));
    HIP_TRY(ctof::launch_fill_int(E[c].active(), E[c].nvol, 1, st));
    HIP_TRY(ctof::launch_fill_int(E[c].boff(), E[c].nvol, 0, st));
    HIP_TRY(ctof::launch_fill_int(E[c].conv(), E[c].nvol, 0, st));
  }
  // ||max(0, A^T d_v)||^2 from the partials of the first step of a zero start
  bool g0_pending = fused_g0;
  auto reduce_g0 = [&]() -> ctof_status {
    if (!g0_pending) return CTOF_OK;
    for (size_t c = 0; c < cls.size(); ++c)
      HIP_TRY(ctof::launch_reduce_volumes(E[c].part() + 2 * (size_t)cls[c].L.nblk_t + 1, cls[c].L.nblk_z,
                                          E[c].nvol, E[c].g0sq(), st));
    g0_pending = false;
    return CTOF_OK;
  };
  // iterations: chunks of `chunk` iterations of every live class, captured once
  // as a graph on an internal stream and replayed on the caller's stream
  const int chunk = std::max(1, std::min(opt->rel_tol > 0 ? opt->check_every : K, 50));
  StreamGuard sg;
  HIP_TRY(hipStreamCreateWithFlags(&sg.s, hipStreamNonBlocking));
  for (int b = 0; b < kBranches; ++b) {
    HIP_TRY(hipStreamCreateWithFlags(&sg.br[b], hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&sg.join[b], hipEventDisableTiming));
  }
  HIP_TRY(hipEventCreateWithFlags(&sg.fork, hipEventDisableTiming));
  for (hipEvent_t &e : sg.chunk_end) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  bool recapture = true;
  std::vector<std::vector<int>> conv(cls.size()), fell(cls.size());
  for (size_t c = 0; c < cls.size(); ++c) {
    conv[c].assign(E[c].nvol, 0);
    fell[c].assign(E[c].nvol, 0);
  }
  int done = 0;
  if (opt->warm_start == 2) {
    // first iteration from the given starts; a volume whose gradient-mapping
    // ratio exceeds that of a zero start (1) restarts from zero
    std::vector<std::vector<double>> first(cls.size());
    for (size_t c = 0; c < cls.size(); ++c) {
      Engine<T> Ec = E[c];
      Ec.live = E[c].active();
      if (ctof_status s = enqueue_iteration(Ec, dv[c].data(), mv[c].data(), cls[c].tau, cls[c].lam, true, 0, 0.0,
                                            prev_of(c));
          s != CTOF_OK)
        return s;
      const ClassWs &L = cls[c].L;
      HIP_TRY(ctof::launch_history(E[c].part(), 1, E[c].nvol, L.nblk_t, L.nblk_z, L.part_stride, cls[c].tau,
                                   E[c].g0sq(), E[c].hist(), st));
      first[c].resize((size_t)E[c].nvol * 2);
      HIP_TRY(hipMemcpyAsync(first[c].data(), E[c].hist(), first[c].size() * sizeof(double),
                             hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    for (size_t c = 0; c < cls.size(); ++c) {
      for (int v = 0; v < E[c].nvol; ++v) fell[c][v] = (first[c][2 * v + 1] <= 1.0) ? 0 : 1;
      if (ctof_status s = restart_from_zero(E[c], mv[c].data(), fell[c]); s != CTOF_OK) return s;
      // a restarted volume begins its own step sequence: beta index = counter - 1
      HIP_TRY(hipMemcpyAsync(E[c].boff(), fell[c].data(), fell[c].size() * sizeof(int), hipMemcpyHostToDevice, st));
    }
    HIP_TRY(hipStreamSynchronize(st));  // the host flags above are copied before they go out of scope
    done = 1;
  }
  // With a tolerance every chunk ends with a device-side freeze check of each
  // live class (freeze_kernel: the same ratio launch_history reports).  The
  // host launches chunk j + 1 before it reads back the flags that chunk j
  // left, so the device never waits for the host; a class the host finds
  // all frozen leaves the graph from the next capture on (a chunk launched
  // meanwhile skips its frozen volumes).
  const bool freeze = opt->rel_tol > 0;
  std::vector<std::vector<int>> host_active(cls.size());
  auto enqueue_freeze = [&](size_t c, hipStream_t s) -> ctof_status {
    const ClassWs &L = cls[c].L;
    HIP_TRY(ctof::launch_freeze(E[c].part(), L.part_stride, E[c].ctr(), E[c].nvol, L.nblk_t, L.nblk_z, cls[c].tau,
                                E[c].g0sq(), fused_g0 ? E[c].part() + 2 * (size_t)L.nblk_t + 1 : nullptr,
                                opt->rel_tol, E[c].active(), E[c].conv(), s));
    return CTOF_OK;
  };
  // read back the flags of the chunk that ended at event `ev` (blocks the
  // host until that chunk is done, not the later ones)
  auto read_flags = [&](hipEvent_t ev) -> ctof_status {
    HIP_TRY(hipStreamWaitEvent(sg.s, ev, 0));
    for (size_t c = 0; c < cls.size(); ++c) {
      if (!cls[c].active) continue;
      host_active[c].resize(E[c].nvol);
      HIP_TRY(hipMemcpyAsync(host_active[c].data(), E[c].active(), (size_t)E[c].nvol * sizeof(int),
                             hipMemcpyDeviceToHost, sg.s));
    }
    HIP_TRY(hipStreamSynchronize(sg.s));
    for (size_t c = 0; c < cls.size(); ++c) {
      if (!cls[c].active) continue;
      int live = 0;
      for (int v = 0; v < E[c].nvol; ++v) live += host_active[c][v] != 0;
      if (live == 0) {
        cls[c].active = false;
        recapture = true;
      }
    }
    return CTOF_OK;
  };
  int nchunk = 0;
  TraceRange tl("iterations");
  while (done < K) {
    bool any = false;
    for (auto &c : cls) any = any || c.active;
    if (!any) break;
    const int n_this = std::min(chunk, K - done);
    if (n_this == chunk) {
      if (recapture) {
        // live classes go to up to kBranches parallel branches (greedy by
        // estimated bytes per iteration); each branch runs its classes'
        // iterations in order, branches join at the end of the chunk
        sg.reset_graph();
        std::vector<int> order;
        for (size_t c = 0; c < cls.size(); ++c)
          if (cls[c].active) order.push_back((int)c);
        auto cost = [&](int c) {
          const ctof::Dims &q = cls[c].k->dims;
          return (double)q.nmat * q.ntp * q.nzp + (double)E[c].nvol * (q.h + 1) * q.p * (q.ntp + q.nzp);
        };
        std::sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
        const int nb = std::min<int>(kBranches, (int)order.size());
        std::vector<std::vector<int>> branch(nb);
        std::vector<double> load(nb, 0.0);
        for (int c : order) {
          const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
          branch[b].push_back(c);
          load[b] += cost(c);
        }
        HIP_TRY(hipStreamBeginCapture(sg.s, hipStreamCaptureModeThreadLocal));
        ctof_status cap = CTOF_OK;
        hipError_t ce = hipEventRecord(sg.fork, sg.s);
        for (int b = 0; b < nb && ce == hipSuccess; ++b) ce = hipStreamWaitEvent(sg.br[b], sg.fork, 0);
        for (int b = 0; b < nb && ce == hipSuccess && cap == CTOF_OK; ++b) {
          for (int i = 0; i < chunk && cap == CTOF_OK; ++i)
            for (int c : branch[b]) {
              Engine<T> Ec = E[c];
              Ec.st = sg.br[b];
              Ec.live = E[c].active();
              cap = enqueue_iteration(Ec, dv[c].data(), mv[c].data(), cls[c].tau, cls[c].lam, true, 0, 0.0,
                                      prev_of(c), fused_g0);
              if (cap != CTOF_OK) break;
            }
          if (freeze)
            for (int c : branch[b])
              if (cap == CTOF_OK) cap = enqueue_freeze((size_t)c, sg.br[b]);
        }
        for (int b = 0; b < nb && ce == hipSuccess; ++b) {
          ce = hipEventRecord(sg.join[b], sg.br[b]);
          if (ce == hipSuccess) ce = hipStreamWaitEvent(sg.s, sg.join[b], 0);
        }
        hipGraph_t g = nullptr;
        const hipError_t ee = hipStreamEndCapture(sg.s, &g);
        sg.g = g;
        if (cap != CTOF_OK) return cap;
        HIP_TRY(ce);
        HIP_TRY(ee);
        HIP_TRY(hipGraphInstantiate(&sg.x, sg.g, nullptr, nullptr, 0));
        recapture = false;
      }
      HIP_TRY(hipGraphLaunch(sg.x, st));
    } else {
      // the last, shorter chunk ends at max_iter: no check follows it
      for (int i = 0; i < n_this; ++i)
        for (size_t c = 0; c < cls.size(); ++c)
          if (cls[c].active) {
            Engine<T> Ec = E[c];
            Ec.live = E[c].active();
            if (ctof_status s = enqueue_iteration(Ec, dv[c].data(), mv[c].data(), cls[c].tau, cls[c].lam,
                                                  true, 0, 0.0, prev_of(c), fused_g0);
                s != CTOF_OK)
              return s;
          }
    }
    if (ctof_status s = reduce_g0(); s != CTOF_OK) return s;
    done += n_this;
    if (freeze && n_this == chunk) {
      HIP_TRY(hipEventRecord(sg.chunk_end[nchunk & 1], st));
      // the previous chunk's flags, read while this one runs
      if (nchunk > 0)
        if (ctof_status s = read_flags(sg.chunk_end[(nchunk - 1) & 1]); s != CTOF_OK) return s;
      ++nchunk;
    }
  }
  tl.end();
  // conv per volume (device): iterations until frozen, 0 for volumes still live
  for (size_t c = 0; c < cls.size(); ++c) {
    if (!freeze) break;
    HIP_TRY(hipMemcpyAsync(conv[c].data(), E[c].conv(), (size_t)E[c].nvol * sizeof(int), hipMemcpyDeviceToHost,
                           st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  if (ctof_status s = reduce_g0(); s != CTOF_OK) return s;
  // reports: full history, final data fit per volume (skipped on request,
  // except in a one-step call with the fallback, where a volume that fell
  // back has no kept history row)
  const bool skip_fit = opt->skip_final_fit && !(K == 1 && opt->warm_start == 2);
  std::vector<std::vector<double>> hist(cls.size()), fit(cls.size()), g0(cls.size());
  for (size_t c = 0; c < cls.size(); ++c) {
    const ClassWs &L = cls[c].L;
    const int its = std::max(1, std::min(done, K));
    HIP_TRY(ctof::launch_history(E[c].part(), its, E[c].nvol, L.nblk_t, L.nblk_z, L.part_stride, cls[c].tau,
                                 E[c].g0sq(), E[c].hist(), st));
    if (!skip_fit)
      if (ctof_status s = enqueue_final_fit(E[c], dv[c].data(), mv[c].data(),
                                            E[c].part() + (size_t)K * L.part_stride, E[c].scal() + 8);
          s != CTOF_OK)
        return s;
    hist[c].resize((size_t)its * E[c].nvol * 2);
    fit[c].resize(E[c].nvol);
    g0[c].resize(E[c].nvol);
    HIP_TRY(hipMemcpyAsync(hist[c].data(), E[c].hist(), hist[c].size() * sizeof(double), hipMemcpyDeviceToHost, st));
    if (!skip_fit)
      HIP_TRY(hipMemcpyAsync(fit[c].data(), E[c].scal() + 8, fit[c].size() * sizeof(double), hipMemcpyDeviceToHost,
                             st));
    HIP_TRY(hipMemcpyAsync(g0[c].data(), E[c].g0sq(), g0[c].size() * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  ctof_status worst = CTOF_OK;
  for (size_t c = 0; c < cls.size(); ++c) {
    const int nv = E[c].nvol;
    for (int v = 0; v < nv; ++v) {
      ctof_solver_report &r = rep[cls[c].scans[v]];
      std::memset(&r, 0, sizeof(r));
      const int its = conv[c][v] > 0 ? conv[c][v] : std::max(1, done);
      r.iters = its;
      r.fista_k = k0 + its - fell[c][v];
      // the kept run of a restarted volume begins at its second row
      r.datafit0 = hist[c][((size_t)fell[c][v] * nv + v) * 2];
      r.gmap_ratio = hist[c][((size_t)(its - 1) * nv + v) * 2 + 1];
      // (without the final fit: the data fit at the last step's extrapolated point)
      r.datafit = skip_fit ? hist[c][((size_t)(its - 1) * nv + v) * 2] : fit[c][v];
      r.lipschitz = cls[c].lip;
      r.lambda = cls[c].lam;
      r.lipschitz_a = cls[c].lip_a;
      r.gmap0 = std::sqrt(g0[c][v]);
      r.fell_back = fell[c][v];
      r.status = CTOF_OK;
      if (!std::isfinite(r.datafit) || !std::isfinite(r.datafit0) || !std::isfinite(r.gmap_ratio)) {
        r.status = CTOF_ENONFINITE;
        worst = CTOF_ENONFINITE;
      } else if (its > fell[c][v] && diverged(hist[c][((size_t)fell[c][v] * nv + v) * 2 + 1], r.gmap_ratio)) {
        r.status = CTOF_EDIVERGED;
        if (worst == CTOF_OK) worst = CTOF_EDIVERGED;
      }
    }
  }
  if (worst == CTOF_ENONFINITE) return set_error(worst, "non-finite FP64 norm in a batched solve");
  if (worst == CTOF_EDIVERGED)
    return set_error(worst, "a scan of the batched solve diverged (is its lipschitz below the operator's?)");
  return CTOF_OK;
}

// Launch-shape tuner: times the operator passes of one class (the eight
// launches of an iteration) for the FFT planes-per-block pairs, then, with
// the fastest pair, for the forward and the adjoint contraction's blocks per
// matrix in turn, and keeps the fastest of each in the handle.
template <typename T>
ctof_status run_tune(ctof_kernel_s *k, int nvol, int iters, void *ws, hipStream_t st, ctof_tuning *out) {
  const int cand[4][2] = {{16, 16}, {32, 16}, {16, 32}, {32, 32}};
  const int parts[4] = {1, 2, 4, 8};
  // events at the stage boundaries of every timed iteration: before the
  // forward contraction, the bin-side passes, the adjoint contraction and the
  // layer-side passes, and one at the end
  std::vector<hipEvent_t> evs((size_t)4 * iters + 1, nullptr);
  struct Ev {
    std::vector<hipEvent_t> *v;
    ~Ev() {
      for (hipEvent_t e : *v)
        if (e) (void)hipEventDestroy(e);
    }
  } ev_guard{&evs};
  for (auto &e : evs) HIP_TRY(hipEventCreate(&e));
  // milliseconds per iteration of each stage of the handle's current launch
  // shape, [0] forward contraction, [1] bin-side passes, [2] adjoint
  // contraction, [3] layer-side passes: each the fastest of three timed
  // passes after a warm-up pass.  A choice is judged by the stages it
  // changes, whose times are far less noisy than the whole iteration's.
  auto time_stages = [&](float (&ms)[4]) -> ctof_status {
    const Engine<T> E = engine<T>(k, nvol, ws, 1, st);
    HIP_TRY(ctof::launch_fill_zero(E.ws, E.L.op_total, st));
    float best[4] = {1e30f, 1e30f, 1e30f, 1e30f};
    for (int rep = 0; rep < 4; ++rep) {
      for (int i = 0; i < iters; ++i) {
        const ctof::RowArgs a = E.row(ctof::ROW_PASS, true);
        const ctof::RowArgs b = E.row(ctof::ROW_PASS, false);
        HIP_TRY(hipEventRecord(evs[(size_t)4 * i], st));
        HIP_TRY(E.contract(false));
        HIP_TRY(hipEventRecord(evs[(size_t)4 * i + 1], st));
        HIP_TRY(E.col_t(true));
        HIP_TRY(E.run_row(a));
        HIP_TRY(E.col_t(false));
        HIP_TRY(hipEventRecord(evs[(size_t)4 * i + 2], st));
        HIP_TRY(E.contract(true));
        HIP_TRY(hipEventRecord(evs[(size_t)4 * i + 3], st));
        HIP_TRY(E.col_z(true));
        HIP_TRY(E.run_row(b));
        HIP_TRY(E.col_z(false));
      }
      HIP_TRY(hipEventRecord(evs[(size_t)4 * iters], st));
      HIP_TRY(hipEventSynchronize(evs[(size_t)4 * iters]));
      float acc[4] = {0.f, 0.f, 0.f, 0.f};
      for (int i = 0; i < iters; ++i)
        for (int j = 0; j < 4; ++j) {
          float t = 0.f;
          HIP_TRY(hipEventElapsedTime(&t, evs[(size_t)4 * i + j], evs[(size_t)4 * i + j + 1]));
          acc[j] += t;
        }
      if (rep > 0)
        for (int j = 0; j < 4; ++j) best[j] = std::min(best[j], acc[j]);
    }
    for (int j = 0; j < 4; ++j) ms[j] = best[j] / std::max(iters, 1);
    return CTOF_OK;
  };
  auto total = [](const float (&ms)[4]) { return ms[0] + ms[1] + ms[2] + ms[3]; };
  std::memset(out, 0, sizeof(*out));
  // 1. FFT planes per block, row passes alike, contractions at the built-in
  // rule: the bin side's value by the bin-side passes' time, the layer
  // side's by theirs
  k->fwd_parts = 0;
  k->adj_parts = 0;
  k->rb_t = 0;
  k->rb_z = 0;
  float bt[2] = {1e30f, 1e30f}, bz[2] = {1e30f, 1e30f};  // [0]: 16 planes, [1]: 32
  const bool f64 = k->prec == CTOF_FP64;
  for (int c = 0; c < 4; ++c) {
    k->bb_t = cand[c][0];
    k->bb_z = cand[c][1];
    const Engine<T> E = engine<T>(k, nvol, ws, 1, st);
    // skip choices the block rule would not honour (it falls back to 16)
    if (ctof::batch_block(E.dm(), E.Bt(), E.dm().ntp, f64, cand[c][0]) != cand[c][0] ||
        ctof::batch_block(E.dm(), E.Bz(), E.dm().nzp, f64, cand[c][1]) != cand[c][1]) {
      out->ms_bb[c] = -1.f;
      continue;
    }
    float ms[4];
    if (ctof_status s = time_stages(ms); s != CTOF_OK) return s;
    out->ms_bb[c] = total(ms);
    float &t = bt[cand[c][0] == 32], &z = bz[cand[c][1] == 32];
    t = std::min(t, ms[1]);
    z = std::min(z, ms[3]);
  }
  k->bb_t = bt[1] < bt[0] ? 32 : 16;
  k->bb_z = bz[1] < bz[0] ? 32 : 16;
  // 2. the row passes' planes per block: the column passes' or 64 on the
  // bin side, the column passes', 16 or 64 on the layer side (pairs whose
  // effective values repeat an earlier pair's are skipped; the first repeats
  // the choice above), each side by its own passes' time
  const int rcand[6][2] = {{0, 0}, {64, 0}, {0, 16}, {64, 16}, {0, 64}, {64, 64}};
  {
    int rt = 0, rz = 0;
    float bestt = 1e30f, bestz = 1e30f;
    int seen[6][2];
    for (int c = 0; c < 6; ++c) {
      k->rb_t = rcand[c][0];
      k->rb_z = rcand[c][1];
      const Engine<T> E = engine<T>(k, nvol, ws, 1, st);
      seen[c][0] = ctof::row_block(E.dm(), E.Bt(), E.dm().ntp, f64, row_planes(k, true));
      seen[c][1] = ctof::row_block(E.dm(), E.Bz(), E.dm().nzp, f64, row_planes(k, false));
      bool dup = false;
      for (int r = 0; r < c; ++r) dup = dup || (seen[r][0] == seen[c][0] && seen[r][1] == seen[c][1]);
      if (dup) {
        out->ms_rb[c] = -1.f;
        continue;
      }
      float ms[4];
      if (ctof_status s = time_stages(ms); s != CTOF_OK) return s;
      out->ms_rb[c] = total(ms);
      if (ms[1] < bestt) {
        bestt = ms[1];
        rt = rcand[c][0];
      }
      if (ms[3] < bestz) {
        bestz = ms[3];
        rz = rcand[c][1];
      }
    }
    k->rb_t = rt;
    k->rb_z = rz;
  }
  // 3. forward, then 4. adjoint blocks per matrix, each by the time of its
  // contraction and the passes after it (the adjoint's partial spectra are
  // added by the layer-side inverse column pass); values that clamp to one
  // already timed are skipped
  for (int dir = 0; dir < 2; ++dir) {
    float *row = dir == 0 ? out->ms_fwd : out->ms_adj;
    int chosen = 0, seen[4] = {0, 0, 0, 0};
    float bestp = 1e30f;
    for (int q = 0; q < 4; ++q) {
      if (dir == 0) k->fwd_parts = parts[q];
      else k->adj_parts = parts[q];
      const int eff = ctof::contract_parts(k, dir == 1);
      bool dup = false;
      for (int r = 0; r < q; ++r) dup = dup || seen[r] == eff;
      seen[q] = eff;
      if (dup) {
        row[q] = -1.f;
        continue;
      }
      float ms[4];
      if (ctof_status s = time_stages(ms); s != CTOF_OK) return s;
      row[q] = total(ms);
      const float judged = dir == 0 ? ms[0] + ms[1] : ms[2] + ms[3];
      if (judged < bestp) {
        bestp = judged;
        chosen = parts[q];
      }
    }
    if (dir == 0) k->fwd_parts = chosen;
    else k->adj_parts = chosen;
  }
  out->bb_t = k->bb_t;
  out->bb_z = k->bb_z;
  out->rb_t = row_planes(k, true);
  out->rb_z = row_planes(k, false);
  out->fwd_parts = ctof::contract_parts(k, false);
  out->adj_parts = ctof::contract_parts(k, true);
  return CTOF_OK;
}

}  // namespace

namespace ctof {

Dims make_dims(int nx, int ny, int nz, int nt, ctof_precision prec) {
  Dims d;
  const int n = std::max(nx, ny);
  d.n = n;
  d.ny = ny;
  d.nx = nx;
  d.nz = nz;
  d.nt = nt;
  d.p = fft_size(n);
  d.h = d.p / 2;
  d.nmat = (d.h + 1) * (d.h + 2) / 2;
  const bool bf = prec == CTOF_BF16X3 || prec == CTOF_BF16;
  d.nzp = nz <= 64 ? (int)round_up(nz, bf ? 32 : 16) : (int)round_up(nz, 64);
  d.ntp = (int)round_up(nt, 32);
  return d;
}

KhatLayout khat_layout(const Dims &d, ctof_precision prec) {
  KhatLayout L;
  const size_t per = (size_t)d.nmat * d.ntp * d.nzp;
  const size_t none = std::numeric_limits<size_t>::max();
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += round_up(bytes, 256);
    return at;
  };
  if (prec == CTOF_FP64 || prec == CTOF_FP32) {
    const size_t es = prec == CTOF_FP64 ? 8 : 4;
    L.fwd = take(per * es);
    L.adj = take(per * es);
    L.fwd_lo = L.adj_lo = none;
  } else if (prec == CTOF_BF16X3) {
    L.fwd = take(per * 2);
    L.fwd_lo = take(per * 2);
    L.adj = take(per * 2);
    L.adj_lo = take(per * 2);
  } else {
    L.fwd = take(per * 2);
    L.adj = take(per * 2);
    L.fwd_lo = L.adj_lo = none;
  }
  L.total = off;
  return L;
}

}  // namespace ctof

extern "C" {

ctof_status ctof_warmstart_loss_ws_bytes(ctof_kernel k, int32_t nb, size_t *ws_bytes) {
  if (ctof_status s = check_kernel(k); s != CTOF_OK) return s;
  if (nb < 1 || nb > ctof::kMaxVol) return set_error(CTOF_EINVAL, "nb must be in [1, %d]", ctof::kMaxVol);
  if (!ws_bytes) return set_error(CTOF_EINVAL, "ws_bytes is NULL");
  *ws_bytes = start_loss_ws(k, nb).total;
  return CTOF_OK;
}

ctof_status ctof_warmstart_loss(ctof_kernel k, int32_t nb, const ctof_tensor *y, const double *s, const float *target_dev,
                                const double *w, const double *v, double lambda, int32_t relu_mask,
                                const ctof_tensor *grad, double *terms_dev, void *ws_dev, size_t ws_bytes,
                                hipStream_t stream) {
  if (ctof_status r = check_kernel(k); r != CTOF_OK) return r;
  if (k->prec == CTOF_FP64) return set_error(CTOF_EUNSUPPORTED, "the warm-start loss takes float handles");
  if (nb < 1 || nb > ctof::kMaxVol) return set_error(CTOF_EINVAL, "nb must be in [1, %d]", ctof::kMaxVol);
  if (!y || !y->ptr || !grad || !grad->ptr || !target_dev || !s || !w || !v || !terms_dev || !ws_dev)
    return set_error(CTOF_EINVAL, "NULL argument");
  if (y->c0 < 0 || y->c0 >= y->ld || grad->c0 < 0 || grad->c0 >= grad->ld)
    return set_error(CTOF_EINVAL, "channel outside the row");
  if (!std::isfinite(lambda) || lambda < 0) return set_error(CTOF_EINVAL, "lambda must be finite and >= 0");
  for (int b = 0; b < nb; ++b)
    if (!std::isfinite(s[b]) || !std::isfinite(w[b]) || !std::isfinite(v[b]))
      return set_error(CTOF_EINVAL, "scales and weights must be finite");
  const size_t need = start_loss_ws(k, nb).total;
  if (ws_bytes < need) return set_error(CTOF_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
  return run_start_loss(k, nb, y, s, target_dev, w, v, lambda, relu_mask ? 1 : 0, grad, terms_dev, ws_dev, stream);
}

const char *ctof_last_error(void) { return ctof::last_error(); }

ctof_status ctof_kernel_bytes(const ctof_geometry *geom, ctof_precision prec, size_t *khat_bytes,
                              size_t *tab_ws_bytes) {
  ctof_status s = check_geometry(geom, nullptr, nullptr);
  if (s != CTOF_OK) return s;
  if (!valid_prec(&prec)) return set_error(CTOF_EINVAL, "unknown precision %d", (int)prec_value(&prec));
  const ctof::Dims d = ctof::make_dims(geom->nx, geom->ny, geom->nz, geom->nt, prec);
  if (khat_bytes) *khat_bytes = ctof::khat_layout(d, prec).total;
  if (tab_ws_bytes) *tab_ws_bytes = tab_ws(d).total;
  return CTOF_OK;
}

ctof_status ctof_kernel_tabulate(const ctof_geometry *geom, ctof_precision prec, void *khat_dev,
                                 size_t khat_bytes, void *tab_ws_dev, size_t tab_ws_bytes,
                                 hipStream_t stream, ctof_kernel *out) {
  if (!valid_prec(&prec)) return set_error(CTOF_EINVAL, "unknown precision %d", (int)prec_value(&prec));
  return ctof_kernel_tabulate_ex(geom, nullptr, prec, khat_dev, khat_bytes, tab_ws_dev, tab_ws_bytes, stream, out);
}

ctof_status ctof_kernel_tabulate_ex(const ctof_geometry *geom, const ctof_fluorescence *fl, ctof_precision prec,
                                    void *khat_dev, size_t khat_bytes, void *tab_ws_dev, size_t tab_ws_bytes,
                                    hipStream_t stream, ctof_kernel *out) {
  TraceRange trace("ctof_kernel_tabulate");
  ctof::TabGeom tg;
  ctof::LayerDepths zs;
  ctof_status s = check_geometry(geom, &tg, &zs);
  if (s != CTOF_OK) return s;
  if ((s = apply_fluorescence(geom, fl, &tg)) != CTOF_OK) return s;
  if (!valid_prec(&prec)) return set_error(CTOF_EINVAL, "unknown precision %d", (int)prec_value(&prec));
  if (!out) return set_error(CTOF_EINVAL, "out handle pointer is NULL");
  if (!khat_dev || !tab_ws_dev) return set_error(CTOF_EINVAL, "device buffer is NULL");
  const ctof::Dims d = ctof::make_dims(geom->nx, geom->ny, geom->nz, geom->nt, prec);
  const ctof::KhatLayout lay = ctof::khat_layout(d, prec);
  const TabWs tw = tab_ws(d);
  if (khat_bytes < lay.total) return set_error(CTOF_ENOMEM, "khat buffer %zu < %zu bytes", khat_bytes, lay.total);
  if (tab_ws_bytes < tw.total)
    return set_error(CTOF_ENOMEM, "tabulation workspace %zu < %zu bytes", tab_ws_bytes, tw.total);
  char *ws = reinterpret_cast<char *>(tab_ws_dev);
  double *Q = reinterpret_cast<double *>(ws + tw.q);
  double *T1 = reinterpret_cast<double *>(ws + tw.t1);
  double *C = reinterpret_cast<double *>(ws + tw.cm);
  const size_t per = (size_t)d.nt * d.nz;
  const ctof::GaussLegendre16 gl = gauss_legendre16();
  // Q[dy][dx][k][z]
  HIP_TRY(ctof::launch_tab_values(tg, zs, gl, Q, (size_t)d.n * per, per, 1, (size_t)d.nz, stream));
  HIP_TRY(ctof::launch_cosine_matrix(d.n, d.p, C, stream));
  // T1[dy][b][k][z] = sum_dx C[b][dx] Q[dy][dx][k][z]
  HIP_TRY(ctof::launch_gemm_f64(d.h + 1, (long long)per, d.n, C, Q, (long long)per, (long long)(d.n * per), T1,
                                (long long)per, (long long)((d.h + 1) * per), d.n, stream));
  // K64[a][b][k][z] = sum_dy C[a][dy] T1[dy][b][k][z]   (written over Q)
  const long long N2 = (long long)(d.h + 1) * (long long)per;
  HIP_TRY(ctof::launch_gemm_f64(d.h + 1, N2, d.n, C, T1, N2, 0, Q, N2, 0, 1, stream));
  HIP_TRY(ctof::launch_pack(d, prec, Q, khat_dev, lay, 1.0 / ((double)d.p * (double)d.p), stream));
  HIP_TRY(hipStreamSynchronize(stream));
  ctof_kernel_s *k = new (std::nothrow) ctof_kernel_s;
  if (!k) return set_error(CTOF_ENOMEM, "host allocation of the handle failed");
  k->dims = d;
  k->prec = prec;
  k->geom = tg;
  k->khat = khat_dev;
  k->layout = lay;
  k->bb_t = 0;
  k->bb_z = 0;
  *out = k;
  return CTOF_OK;
}

ctof_status ctof_kernel_tabulate_quadrant(const ctof_geometry *geom, double *quad_dev, size_t quad_bytes,
                                          hipStream_t stream) {
  return ctof_kernel_tabulate_quadrant_ex(geom, nullptr, quad_dev, quad_bytes, stream);
}

ctof_status ctof_kernel_tabulate_fp64_quadrant(const ctof_geometry *geom, double *quad_dev, hipStream_t stream) {
  if (!geom) return set_error(CTOF_EINVAL, "geometry is NULL");
  // the buffer size the geometry fixes (geometry errors are reported below)
  const size_t n = (size_t)std::max(std::max(geom->nx, geom->ny), 0);
  const size_t need = (size_t)std::max(geom->nz, 0) * (size_t)std::max(geom->nt, 0) * n * n * sizeof(double);
  return ctof_kernel_tabulate_quadrant_ex(geom, nullptr, quad_dev, need, stream);
}

ctof_status ctof_kernel_tabulate_quadrant_ex(const ctof_geometry *geom, const ctof_fluorescence *fl, double *quad_dev,
                                             size_t quad_bytes, hipStream_t stream) {
  ctof::TabGeom tg;
  ctof::LayerDepths zs;
  ctof_status s = check_geometry(geom, &tg, &zs);
  if (s != CTOF_OK) return s;
  if ((s = apply_fluorescence(geom, fl, &tg)) != CTOF_OK) return s;
  if (!quad_dev) return set_error(CTOF_EINVAL, "quad_dev is NULL");
  const size_t n = tg.n;  // max(nx, ny)
  const size_t need = (size_t)geom->nz * geom->nt * n * n * sizeof(double);
  if (quad_bytes < need) return set_error(CTOF_ENOMEM, "quadrant buffer %zu < %zu bytes", quad_bytes, need);
  const ctof::GaussLegendre16 gl = gauss_legendre16();
  // [z][k][dy][dx]
  HIP_TRY(ctof::launch_tab_values(tg, zs, gl, quad_dev, n, 1, (size_t)geom->nt * n * n, n * n, stream));
  return CTOF_OK;
}

void ctof_kernel_free(ctof_kernel k) { delete k; }

ctof_status ctof_kernel_info(ctof_kernel k, int32_t *n, int32_t *nz, int32_t *nt, int32_t *p, int32_t *nmat,
                             int32_t *prec) {
  ctof_status s = check_kernel(k);
  if (s != CTOF_OK) return s;
  if (n) *n = k->dims.n;
  if (nz) *nz = k->dims.nz;
  if (nt) *nt = k->dims.nt;
  if (p) *p = k->dims.p;
  if (nmat) *nmat = k->dims.nmat;
  if (prec) *prec = (int32_t)k->prec;
  return CTOF_OK;
}

ctof_status ctof_kernel_band_bytes(ctof_kernel k, size_t *bytes) {
  ctof_status s = check_kernel(k);
  if (s != CTOF_OK) return s;
  if (!bytes) return set_error(CTOF_EINVAL, "bytes is NULL");
  *bytes = ctof::round_up((size_t)k->dims.nmat * 4 * sizeof(int32_t), 256) + 256;  // table, scratch word
  return CTOF_OK;
}

ctof_status ctof_kernel_set_band(ctof_kernel k, double rel, void *band_dev, size_t band_bytes, hipStream_t stream) {
  ctof_status s = check_kernel(k);
  if (s != CTOF_OK) return s;
  if (rel == 0.0) {
    k->band = nullptr;
    k->band_rel = 0.0;
    return CTOF_OK;
  }
  if (!(std::isfinite(rel) && rel > 0.0 && rel < 1.0)) return set_error(CTOF_EINVAL, "rel must be 0 or in (0, 1)");
  if (!band_dev || (reinterpret_cast<uintptr_t>(band_dev) & 255))
    return set_error(CTOF_EINVAL, "band_dev is NULL or not 256-byte aligned");
  const size_t table = (size_t)k->dims.nmat * 4 * sizeof(int32_t);
  const size_t need = ctof::round_up(table, 256) + 256;
  if (band_bytes < need) return set_error(CTOF_ENOMEM, "band buffer %zu < %zu bytes", band_bytes, need);
  if (k->dims.ntp / 16 > ctof::band_max_tiles())
    return set_error(CTOF_EUNSUPPORTED, "a band covers at most %d tiles of 16 bins", ctof::band_max_tiles());
  int *band = reinterpret_cast<int *>(band_dev);
  unsigned int *scratch = reinterpret_cast<unsigned int *>(reinterpret_cast<char *>(band_dev) + ctof::round_up(table, 256));
  HIP_TRY(ctof::launch_band(k, rel, band, scratch, stream));
  k->band = band;
  k->band_rel = rel;
  return CTOF_OK;
}

ctof_status ctof_kernel_grid(ctof_kernel k, int32_t *ny, int32_t *nx) {
  ctof_status s = check_kernel(k);
  if (s != CTOF_OK) return s;
  if (ny) *ny = k->dims.ny;
  if (nx) *nx = k->dims.nx;
  return CTOF_OK;
}

ctof_status ctof_workspace_bytes(ctof_kernel k, int32_t max_iter, size_t *op_ws_bytes, size_t *solve_ws) {
  ctof_status s = check_kernel(k);
  if (s != CTOF_OK) return s;
  if (max_iter < 0) return set_error(CTOF_EINVAL, "max_iter must be >= 0");
  const ClassWs o = class_ws(k, 1, max_iter);
  if (op_ws_bytes) *op_ws_bytes = o.op_total;
  if (solve_ws) *solve_ws = o.solve_total;
  return CTOF_OK;
}

ctof_status ctof_forward(ctof_kernel k, const void *mu_dev, void *m_dev, void *ws_dev, size_t ws_bytes,
                         hipStream_t stream) {
  TraceRange trace("ctof_forward");
  ctof_status s = check_kernel(k);
  if (s != CTOF_OK) return s;
  if (!mu_dev || !m_dev || !ws_dev) return set_error(CTOF_EINVAL, "device pointer is NULL");
  const ClassWs o = class_ws(k, 1, 1);
  if (ws_bytes < o.op_total) return set_error(CTOF_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, o.op_total);
  if (k->prec == CTOF_FP64) return run_forward<double>(k, mu_dev, m_dev, ws_dev, stream);
  return run_forward<float>(k, mu_dev, m_dev, ws_dev, stream);
}

ctof_status ctof_forward_noalloc(ctof_kernel k, const void *mu_dev, void *m_dev, hipStream_t stream) {
  ctof_status s = check_kernel(k);
  if (s != CTOF_OK) return s;
  if (!mu_dev || !m_dev) return set_error(CTOF_EINVAL, "device pointer is NULL");
  const ClassWs o = class_ws(k, 1, 1);
  if (o.op_total > (size_t)CTOF_NOALLOC_SCRATCH_BYTES)
    return set_error(CTOF_ENOMEM, "the forward model needs %zu bytes of workspace, the fixed scratch holds %zu",
                     o.op_total, (size_t)CTOF_NOALLOC_SCRATCH_BYTES);
  void *ws = nullptr;
  if (ctof_status e = scratch_address(&ws); e != CTOF_OK) return e;
  if (k->prec == CTOF_FP64) return run_forward<double>(k, mu_dev, m_dev, ws, stream);
  return run_forward<float>(k, mu_dev, m_dev, ws, stream);
}

ctof_status ctof_adjoint(ctof_kernel k, const void *r_dev, void *g_dev, void *ws_dev, size_t ws_bytes,
                         hipStream_t stream) {
  TraceRange trace("ctof_adjoint");
  ctof_status s = check_kernel(k);
  if (s != CTOF_OK) return s;
  if (!r_dev || !g_dev || !ws_dev) return set_error(CTOF_EINVAL, "device pointer is NULL");
  const ClassWs o = class_ws(k, 1, 1);
  if (ws_bytes < o.op_total) return set_error(CTOF_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, o.op_total);
  if (k->prec == CTOF_FP64) return run_adjoint<double>(k, r_dev, g_dev, ws_dev, stream);
  return run_adjoint<float>(k, r_dev, g_dev, ws_dev, stream);
}

ctof_status ctof_mux_forward(ctof_kernel k, const ctof_mux *mux, const void *m_dev, void *y_dev,
                             hipStream_t stream) {
  if (ctof_status s = check_kernel(k); s != CTOF_OK) return s;
  ctof::MuxArgs a;
  if (ctof_status s = make_mux(k, mux, &a); s != CTOF_OK) return s;
  if (!m_dev || !y_dev || (reinterpret_cast<uintptr_t>(m_dev) & 15))
    return set_error(CTOF_EINVAL, "m or y is NULL, or m is not 16-byte aligned");
  a.in = m_dev;
  a.out = y_dev;
  HIP_TRY(ctof::launch_mux(ctof::MUX_FWD, k->prec == CTOF_FP64, a, ctof::mux_default_blocks(a, k->prec == CTOF_FP64),
                           stream));
  return CTOF_OK;
}

ctof_status ctof_mux_adjoint(ctof_kernel k, const ctof_mux *mux, const void *y_dev, void *m_dev,
                             hipStream_t stream) {
  if (ctof_status s = check_kernel(k); s != CTOF_OK) return s;
  ctof::MuxArgs a;
  if (ctof_status s = make_mux(k, mux, &a); s != CTOF_OK) return s;
  if (!m_dev || !y_dev || (reinterpret_cast<uintptr_t>(m_dev) & 15))
    return set_error(CTOF_EINVAL, "m or y is NULL, or m is not 16-byte aligned");
  a.in = y_dev;
  a.out = m_dev;
  HIP_TRY(ctof::launch_mux(ctof::MUX_ADJ, k->prec == CTOF_FP64, a, ctof::mux_default_blocks(a, k->prec == CTOF_FP64),
                           stream));
  return CTOF_OK;
}

ctof_status ctof_mux_normal_ws_bytes(ctof_kernel k, const ctof_mux *mux, size_t *ws_bytes) {
  if (ctof_status s = check_kernel(k); s != CTOF_OK) return s;
  ctof::MuxArgs a;
  if (ctof_status s = make_mux(k, mux, &a); s != CTOF_OK) return s;
  if (!ws_bytes) return set_error(CTOF_EINVAL, "ws_bytes is NULL");
  *ws_bytes = ctof::round_up((size_t)ctof::mux_default_blocks(a, k->prec == CTOF_FP64) * 2 * sizeof(double), 256);
  return CTOF_OK;
}

ctof_status ctof_mux_normal(ctof_kernel k, const ctof_mux *mux, const void *m_dev, const void *y_dev, void *r_dev,
                            double *fit_dev, void *ws_dev, size_t ws_bytes, hipStream_t stream) {
  if (ctof_status s = check_kernel(k); s != CTOF_OK) return s;
  ctof::MuxArgs a;
  if (ctof_status s = make_mux(k, mux, &a); s != CTOF_OK) return s;
  if (!m_dev || !r_dev || (reinterpret_cast<uintptr_t>(m_dev) & 15) || (reinterpret_cast<uintptr_t>(r_dev) & 15))
    return set_error(CTOF_EINVAL, "m or r is NULL or not 16-byte aligned");
  const int blocks = ctof::mux_default_blocks(a, k->prec == CTOF_FP64);
  const size_t need = (size_t)blocks * 2 * sizeof(double);
  if (fit_dev) {
    if (!ws_dev || (reinterpret_cast<uintptr_t>(ws_dev) & 15))
      return set_error(CTOF_EINVAL, "workspace NULL or not 16-byte aligned");
    if (ws_bytes < need) return set_error(CTOF_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
  }
  a.in = m_dev;
  a.y = y_dev;
  a.out = r_dev;
  a.partials = fit_dev ? reinterpret_cast<double *>(ws_dev) : nullptr;
  a.npart = blocks;
  HIP_TRY(ctof::launch_mux(ctof::MUX_NORMAL, k->prec == CTOF_FP64, a, blocks, stream));
  if (fit_dev) HIP_TRY(ctof::launch_reduce_rows(a.partials, blocks, 2, 1, fit_dev, stream));
  return CTOF_OK;
}

ctof_status ctof_reconstruct(ctof_kernel k, const void *d_dev, void *mu_inout_dev, const ctof_solver_opts *opts,
                             ctof_solver_report *report, void *ws_dev, size_t ws_bytes, hipStream_t stream) {
  ctof_status s = check_kernel(k);
  if (s != CTOF_OK) return s;
  if (!opts || !report) return set_error(CTOF_EINVAL, "opts/report is NULL");
  if (!d_dev || !mu_inout_dev || !ws_dev) return set_error(CTOF_EINVAL, "device pointer is NULL");
  if (opts->max_iter < 1) return set_error(CTOF_EINVAL, "max_iter must be >= 1");
  if (!std::isfinite(opts->lambda_tikhonov)) return set_error(CTOF_EINVAL, "lambda_tikhonov must be finite");
  if (!(std::isfinite(opts->lipschitz) && opts->lipschitz >= 0)) return set_error(CTOF_EINVAL, "lipschitz must be >= 0");
  if (opts->lipschitz > 0 && opts->lambda_tikhonov < 0)
    return set_error(CTOF_EINVAL, "an explicit lipschitz needs lambda_tikhonov >= 0");
  if (opts->power_iters < 0) return set_error(CTOF_EINVAL, "power_iters must be >= 0");
  if (!(std::isfinite(opts->rel_tol) && opts->rel_tol >= 0)) return set_error(CTOF_EINVAL, "rel_tol must be >= 0");
  if (opts->rel_tol > 0 && opts->check_every < 1) return set_error(CTOF_EINVAL, "check_every must be >= 1");
  if (opts->warm_start < 0 || opts->warm_start > 2) return set_error(CTOF_EINVAL, "warm_start must be 0, 1 or 2");
  if (opts->timing < 0) return set_error(CTOF_EINVAL, "timing must be >= 0");
  if (opts->lipschitz_scans || opts->lambda_scans || opts->mu_prev_scans)
    return set_error(CTOF_EINVAL, "lipschitz_scans / lambda_scans / mu_prev_scans are batched options");
  if (ctof_status e = check_resume(opts, opts->mu_prev_dev != nullptr); e != CTOF_OK) return e;
  if (opts->skip_final_fit != 0 && opts->skip_final_fit != 1)
    return set_error(CTOF_EINVAL, "skip_final_fit must be 0 or 1");
  if (opts->mu_prev_dev &&
      overlaps(opts->mu_prev_dev, mu_inout_dev, (size_t)k->dims.nz * k->dims.ny * k->dims.nx * elem_size(k->prec)))
    return set_error(CTOF_EINVAL, "mu_prev_dev overlaps mu_inout_dev");
  if (opts->lambda_l1_z)
    for (int z = 0; z < k->dims.nz; ++z)
      if (!(std::isfinite(opts->lambda_l1_z[z]) && opts->lambda_l1_z[z] >= 0))
        return set_error(CTOF_EINVAL, "lambda_l1_z[%d] must be finite and >= 0", z);
  if (opts->mux) {
    ctof::MuxArgs m;
    if (ctof_status e = make_mux(k, opts->mux, &m); e != CTOF_OK) return e;
  }
  const ClassWs o = class_ws(k, 1, opts->max_iter);
  if (ws_bytes < o.solve_total) return set_error(CTOF_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, o.solve_total);
  std::memset(report, 0, sizeof(*report));
  if (k->prec == CTOF_FP64) return run_reconstruct<double>(k, d_dev, mu_inout_dev, opts, report, ws_dev, stream);
  return run_reconstruct<float>(k, d_dev, mu_inout_dev, opts, report, ws_dev, stream);
}

ctof_status ctof_layer_energy_ws_bytes(ctof_kernel k, size_t *ws_bytes) {
  if (ctof_status s = check_kernel(k); s != CTOF_OK) return s;
  if (!ws_bytes) return set_error(CTOF_EINVAL, "ws_bytes is NULL");
  *ws_bytes = class_ws(k, 1, k->dims.nz).solve_total;
  return CTOF_OK;
}

ctof_status ctof_l1_depth_weights(ctof_kernel k, double lambda1, double *energy, double *weights, void *ws_dev,
                                  size_t ws_bytes, hipStream_t stream) {
  if (ctof_status s = check_kernel(k); s != CTOF_OK) return s;
  if (!(std::isfinite(lambda1) && lambda1 >= 0)) return set_error(CTOF_EINVAL, "lambda1 must be finite and >= 0");
  if (!ws_dev) return set_error(CTOF_EINVAL, "workspace is NULL");
  const ClassWs o = class_ws(k, 1, k->dims.nz);
  if (ws_bytes < o.solve_total) return set_error(CTOF_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, o.solve_total);
  const int nz = k->dims.nz;
  std::vector<double> e((size_t)nz);
  if (k->prec == CTOF_FP64) {
    const Engine<double> E = engine<double>(k, 1, ws_dev, nz, stream);
    if (ctof_status s = enqueue_layer_energy(E, E.hist()); s != CTOF_OK) return s;
    HIP_TRY(hipMemcpyAsync(e.data(), E.hist(), (size_t)nz * sizeof(double), hipMemcpyDeviceToHost, stream));
  } else {
    const Engine<float> E = engine<float>(k, 1, ws_dev, nz, stream);
    if (ctof_status s = enqueue_layer_energy(E, E.hist()); s != CTOF_OK) return s;
    HIP_TRY(hipMemcpyAsync(e.data(), E.hist(), (size_t)nz * sizeof(double), hipMemcpyDeviceToHost, stream));
  }
  HIP_TRY(hipStreamSynchronize(stream));
  double emax = 0.0;
  for (int z = 0; z < nz; ++z) {
    e[z] *= 2.0;  // the row pass sums 1/2 x^2
    if (!std::isfinite(e[z])) return set_error(CTOF_ENONFINITE, "non-finite layer energy at layer %d", z);
    emax = std::max(emax, e[z]);
  }
  if (!(emax > 0)) return set_error(CTOF_ENONFINITE, "every layer energy is zero");
  for (int z = 0; z < nz; ++z) {
    if (energy) energy[z] = e[z];
    if (weights) weights[z] = lambda1 * e[z] / emax;
  }
  return CTOF_OK;
}

ctof_status ctof_workspace_bytes_batched(int32_t nscan, const ctof_kernel *k, int32_t max_iter,
                                        size_t *ws_bytes) {
  if (nscan < 1 || !k) return set_error(CTOF_EINVAL, "need at least one scan and a handle array");
  if (max_iter < 1) return set_error(CTOF_EINVAL, "max_iter must be >= 1");
  for (int i = 0; i < nscan; ++i)
    if (ctof_status s = check_kernel(k[i]); s != CTOF_OK) return s;
  size_t total = 0;
  plan_classes(nscan, k, max_iter, &total);
  if (ws_bytes) *ws_bytes = total;
  return CTOF_OK;
}

ctof_status ctof_reconstruct_batched(int32_t nscan, const ctof_kernel *k, const void *const *d_dev,
                                     void *const *mu_inout_dev, const ctof_solver_opts *opts,
                                     ctof_solver_report *reports, void *ws_dev, size_t ws_bytes,
                                     hipStream_t stream) {
  if (nscan < 1 || !k || !d_dev || !mu_inout_dev || !opts || !reports || !ws_dev)
    return set_error(CTOF_EINVAL, "NULL argument or no scans");
  const ctof_precision prec = k[0] ? k[0]->prec : CTOF_FP32;
  for (int i = 0; i < nscan; ++i) {
    if (ctof_status s = check_kernel(k[i]); s != CTOF_OK) return s;
    if (k[i]->prec != prec) return set_error(CTOF_EINVAL, "all handles of a batch need one precision");
    if (!d_dev[i] || !mu_inout_dev[i]) return set_error(CTOF_EINVAL, "device pointer of scan %d is NULL", i);
  }
  if (opts->mux)
    for (int i = 0; i < nscan; ++i) {
      ctof::MuxArgs m;
      if (ctof_status e = make_mux(k[i], opts->mux, &m); e != CTOF_OK) return e;
    }
  if (opts->max_iter < 1) return set_error(CTOF_EINVAL, "max_iter must be >= 1");
  if (!std::isfinite(opts->lambda_tikhonov)) return set_error(CTOF_EINVAL, "lambda_tikhonov must be finite");
  if (!(std::isfinite(opts->lipschitz) && opts->lipschitz >= 0)) return set_error(CTOF_EINVAL, "lipschitz must be >= 0");
  if (opts->lipschitz > 0 && opts->lambda_tikhonov < 0)
    return set_error(CTOF_EINVAL, "an explicit lipschitz needs lambda_tikhonov >= 0");
  if (!(std::isfinite(opts->rel_tol) && opts->rel_tol >= 0)) return set_error(CTOF_EINVAL, "rel_tol must be >= 0");
  if (opts->rel_tol > 0 && opts->check_every < 1) return set_error(CTOF_EINVAL, "check_every must be >= 1");
  if (opts->warm_start < 0 || opts->warm_start > 2) return set_error(CTOF_EINVAL, "warm_start must be 0, 1 or 2");
  if (opts->history_dev || opts->timing || opts->mu_prev_dev)
    return set_error(CTOF_EINVAL, "history_dev, timing and mu_prev_dev are single-scan options");
  {
    bool all_prev = opts->mu_prev_scans != nullptr;
    if (opts->mu_prev_scans)
      for (int i = 0; i < nscan; ++i) {
        const size_t vb = (size_t)k[i]->dims.nz * k[i]->dims.ny * k[i]->dims.nx * elem_size(prec);
        if (!opts->mu_prev_scans[i]) all_prev = false;
        else if (overlaps(opts->mu_prev_scans[i], mu_inout_dev[i], vb))
          return set_error(CTOF_EINVAL, "mu_prev_scans[%d] overlaps mu_inout_dev[%d]", i, i);
      }
    if (opts->mu_prev_scans && !all_prev) return set_error(CTOF_EINVAL, "mu_prev_scans has a NULL entry");
    if (ctof_status e = check_resume(opts, all_prev); e != CTOF_OK) return e;
    if (opts->skip_final_fit != 0 && opts->skip_final_fit != 1)
      return set_error(CTOF_EINVAL, "skip_final_fit must be 0 or 1");
  }
  if ((opts->lipschitz_scans == nullptr) != (opts->lambda_scans == nullptr))
    return set_error(CTOF_EINVAL, "lipschitz_scans and lambda_scans go together");
  if (opts->lambda_l1_z) {
    for (int i = 1; i < nscan; ++i)
      if (k[i]->dims.nz != k[0]->dims.nz)
        return set_error(CTOF_EINVAL, "per-layer L1 weights need one layer count for all scans");
    for (int z = 0; z < k[0]->dims.nz; ++z)
      if (!(std::isfinite(opts->lambda_l1_z[z]) && opts->lambda_l1_z[z] >= 0))
        return set_error(CTOF_EINVAL, "lambda_l1_z[%d] must be finite and >= 0", z);
  }
  if (opts->lipschitz_scans)
    for (int i = 0; i < nscan; ++i)
      if (!(std::isfinite(opts->lipschitz_scans[i]) && opts->lipschitz_scans[i] > 0) ||
          !(std::isfinite(opts->lambda_scans[i]) && opts->lambda_scans[i] >= 0))
        return set_error(CTOF_EINVAL, "scan %d: need L > 0 and lambda >= 0", i);
  size_t need = 0;
  plan_classes(nscan, k, opts->max_iter, &need);
  if (ws_bytes < need) return set_error(CTOF_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
  if (prec == CTOF_FP64)
    return run_batched<double>(nscan, k, d_dev, mu_inout_dev, opts, reports, ws_dev, stream);
  return run_batched<float>(nscan, k, d_dev, mu_inout_dev, opts, reports, ws_dev, stream);
}

ctof_status ctof_kernel_set_tuning(ctof_kernel k, int32_t bb_t, int32_t bb_z) {
  if (ctof_status s = check_kernel(k); s != CTOF_OK) return s;
  auto ok = [](int32_t v) { return v == 0 || v == 16 || v == 32; };
  if (!ok(bb_t) || !ok(bb_z)) return set_error(CTOF_EINVAL, "planes per block must be 0, 16 or 32");
  k->bb_t = bb_t;
  k->bb_z = bb_z;
  return CTOF_OK;
}

ctof_status ctof_kernel_set_row_tuning(ctof_kernel k, int32_t rb_t, int32_t rb_z) {
  if (ctof_status s = check_kernel(k); s != CTOF_OK) return s;
  auto ok = [](int32_t v) { return v == 0 || v == 16 || v == 32 || v == 64; };
  if (!ok(rb_t) || !ok(rb_z)) return set_error(CTOF_EINVAL, "row-pass planes per block must be 0, 16, 32 or 64");
  k->rb_t = rb_t;
  k->rb_z = rb_z;
  return CTOF_OK;
}

ctof_status ctof_kernel_get_row_tuning(ctof_kernel k, int32_t *rb_t, int32_t *rb_z) {
  if (ctof_status s = check_kernel(k); s != CTOF_OK) return s;
  const ctof::Dims &d = k->dims;
  const bool f64 = k->prec == CTOF_FP64;
  if (rb_t) *rb_t = ctof::row_block(d, d.ntp, d.ntp, f64, row_planes(k, true));
  if (rb_z) *rb_z = ctof::row_block(d, d.nzp, d.nzp, f64, row_planes(k, false));
  return CTOF_OK;
}

ctof_status ctof_kernel_set_contract_parts(ctof_kernel k, int32_t fwd_parts, int32_t adj_parts) {
  if (ctof_status s = check_kernel(k); s != CTOF_OK) return s;
  auto ok = [](int32_t v) { return v == 0 || v == 1 || v == 2 || v == 4 || v == 8; };
  if (!ok(fwd_parts) || !ok(adj_parts)) return set_error(CTOF_EINVAL, "parts must be 0, 1, 2, 4 or 8");
  k->fwd_parts = fwd_parts;
  k->adj_parts = adj_parts;
  return CTOF_OK;
}

ctof_status ctof_kernel_get_contract_parts(ctof_kernel k, int32_t *fwd_parts, int32_t *adj_parts) {
  if (ctof_status s = check_kernel(k); s != CTOF_OK) return s;
  if (fwd_parts) *fwd_parts = ctof::contract_parts(k, false);
  if (adj_parts) *adj_parts = ctof::contract_parts(k, true);
  return CTOF_OK;
}

ctof_status ctof_kernel_get_tuning(ctof_kernel k, int32_t *bb_t, int32_t *bb_z) {
  if (ctof_status s = check_kernel(k); s != CTOF_OK) return s;
  if (bb_t) *bb_t = k->bb_t;
  if (bb_z) *bb_z = k->bb_z;
  return CTOF_OK;
}

// largest workspace over the launch shapes the tuner tries
static size_t tune_ws_bytes(ctof_kernel_s *k, int nvol) {
  const int32_t save_t = k->bb_t, save_z = k->bb_z, save_a = k->adj_parts, save_rt = k->rb_t, save_rz = k->rb_z;
  size_t need = 0;
  for (int bt : {16, 32})
    for (int bz : {16, 32})
      for (int rb : {0, 16, 64})
        for (int ap : {1, 2, 4, 8}) {
          k->bb_t = bt;
          k->bb_z = bz;
          k->rb_t = rb;
          k->rb_z = rb;
          k->adj_parts = ap;
          need = std::max(need, class_ws(k, nvol, 1).solve_total);
        }
  k->bb_t = save_t;
  k->bb_z = save_z;
  k->rb_t = save_rt;
  k->rb_z = save_rz;
  k->adj_parts = save_a;
  return need;
}

ctof_status ctof_tune(ctof_kernel k, int32_t nvol, int32_t iters, void *ws_dev, size_t ws_bytes,
                      hipStream_t stream, ctof_tuning *out) {
  TraceRange trace("ctof_tune");
  if (ctof_status s = check_kernel(k); s != CTOF_OK) return s;
  if (nvol < 1 || nvol > ctof::kMaxVol) return set_error(CTOF_EINVAL, "nvol must be in [1, %d]", ctof::kMaxVol);
  if (iters < 1 || iters > 1000) return set_error(CTOF_EINVAL, "iters must be in [1, 1000]");
  if (!ws_dev || !out) return set_error(CTOF_EINVAL, "workspace or result is NULL");
  const size_t need = tune_ws_bytes(k, nvol);
  if (ws_bytes < need) return set_error(CTOF_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
  if (k->prec == CTOF_FP64) return run_tune<double>(k, nvol, iters, ws_dev, stream, out);
  return run_tune<float>(k, nvol, iters, ws_dev, stream, out);
}

ctof_status ctof_tune_workspace_bytes(ctof_kernel k, int32_t nvol, size_t *ws_bytes) {
  if (ctof_status s = check_kernel(k); s != CTOF_OK) return s;
  if (nvol < 1 || nvol > ctof::kMaxVol) return set_error(CTOF_EINVAL, "nvol must be in [1, %d]", ctof::kMaxVol);
  if (ws_bytes) *ws_bytes = tune_ws_bytes(k, nvol);
  return CTOF_OK;
}

}  // extern "C"
