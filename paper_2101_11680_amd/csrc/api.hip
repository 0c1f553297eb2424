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

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

namespace {

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

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return set_error(CTOF_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));         \
  } while (0)

int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
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
  const double total = (double)g->nz * g->nx * g->ny * (double)g->nt;
  if (total > 9.0e18) return set_error(CTOF_EINVAL, "nz*ny*nx*nt overflows");
  if (g->nx != g->ny) return set_error(CTOF_EUNSUPPORTED, "only square scan grids (nx == ny) are implemented");
  if (g->nx > ctof::kMaxN) return set_error(CTOF_EUNSUPPORTED, "n > %d needs an FFT size above 256", ctof::kMaxN);
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
    tg->n = g->nx;
    tg->nz = g->nz;
    tg->nt = g->nt;
    tg->pitch = g->pitch_mm;
    tg->dt = g->dt_ps;
    tg->t0 = g->t0_ps;
    tg->dv = g->pitch_mm * g->pitch_mm * dz;
    tg->rmin = std::cbrt(3.0 * tg->dv / (4.0 * M_PI));
    tg->o = o;
  }
  if (zs) {
    for (int k = 0; k < ctof::kMaxLayers; ++k) zs->z[k] = k < g->nz ? g->z_mm[k] : 0.0;
  }
  return CTOF_OK;
}

size_t elem_size(ctof_precision p) { return p == CTOF_FP64 ? 8 : 4; }

bool valid_prec(int p) { return p >= CTOF_FP64 && p <= CTOF_BF16; }

struct TabWs {
  size_t q, t1, cm, total;  // offsets
};

TabWs tab_ws(const ctof::Dims &d) {
  TabWs w;
  const size_t per = (size_t)d.nt * d.nz;
  const size_t q = std::max((size_t)d.n * d.n, (size_t)(d.h + 1) * (d.h + 1)) * per * 8;
  const size_t t1 = (size_t)d.n * (d.h + 1) * per * 8;
  const size_t cm = (size_t)(d.h + 1) * d.n * 8;
  w.q = 0;
  w.t1 = ctof::round_up(q, 256);
  w.cm = w.t1 + ctof::round_up(t1, 256);
  w.total = w.cm + ctof::round_up(cm, 256);
  return w;
}

// Workspace carve-up for forward/adjoint/reconstruct.
struct OpWs {
  size_t yhat, mhat, xt, xz, op_total;
  size_t y, v, w, hist, scal, part, solve_total;
  int nblk_t, nblk_z;
  size_t part_stride;  // doubles per iteration
};

OpWs op_ws(const ctof::Dims &d, ctof_precision prec, int max_iter) {
  OpWs o;
  const size_t es = elem_size(prec);
  const bool f64 = prec == CTOF_FP64;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += ctof::round_up(bytes, 256);
    return at;
  };
  o.yhat = take((size_t)(d.h + 1) * d.p * 2 * d.nzp * es);
  o.mhat = take((size_t)(d.h + 1) * d.p * 2 * d.ntp * es);
  o.xt = take((size_t)(d.h + 1) * d.n * 2 * d.ntp * es);
  o.xz = take((size_t)(d.h + 1) * d.n * 2 * d.nzp * es);
  o.op_total = off;
  const size_t vol = (size_t)d.nz * d.n * d.n * es;
  o.y = take(vol);
  o.v = take(vol);
  o.w = take(vol);
  o.nblk_t = ctof::row_pass_blocks(d, d.ntp, f64);
  o.nblk_z = ctof::row_pass_blocks(d, d.nzp, f64);
  o.part_stride = 2 * (size_t)(o.nblk_t + o.nblk_z);
  const int iters = std::max(max_iter, 1);
  o.hist = take((size_t)iters * 2 * 8);
  o.scal = take(64 * 8);
  o.part = take((size_t)(iters + 2) * o.part_stride * 8);
  o.solve_total = off;
  return o;
}

template <typename T>
struct Ops {
  const ctof_kernel_s *k;
  char *ws;
  OpWs lay;
  hipStream_t st;

  T *yhat() const { return reinterpret_cast<T *>(ws + lay.yhat); }
  T *mhat() const { return reinterpret_cast<T *>(ws + lay.mhat); }
  T *xt() const { return reinterpret_cast<T *>(ws + lay.xt); }
  T *xz() const { return reinterpret_cast<T *>(ws + lay.xz); }

  ctof::RowArgs row(int op, bool tside) const {
    ctof::RowArgs a;
    std::memset(&a, 0, sizeof(a));
    a.op = op;
    a.B = tside ? k->dims.ntp : k->dims.nzp;
    a.nplanes = tside ? k->dims.nt : k->dims.nz;
    a.spec_in = tside ? (void *)xt() : (void *)xz();
    a.spec_out = a.spec_in == nullptr ? nullptr : const_cast<void *>(a.spec_in);
    return a;
  }

  // spatial volume -> yhat
  hipError_t mu_to_spec(ctof::RowArgs a) const {
    hipError_t e = ctof::launch_row_pass<T>(k->dims, a, st);
    if (e != hipSuccess) return e;
    return ctof::launch_col_pass<T>(k->dims, k->dims.nzp, false, xz(), yhat(), st);
  }
  // yhat -> (contraction) -> mhat -> xt (inverse column pass)
  hipError_t fwd_to_xt() const {
    hipError_t e = ctof::launch_contract(k, false, yhat(), mhat(), st);
    if (e != hipSuccess) return e;
    return ctof::launch_col_pass<T>(k->dims, k->dims.ntp, true, mhat(), xt(), st);
  }
  // xt (row-pass output spectrum) -> mhat -> (adjoint contraction) -> yhat -> xz
  hipError_t adj_to_xz() const {
    hipError_t e = ctof::launch_col_pass<T>(k->dims, k->dims.ntp, false, xt(), mhat(), st);
    if (e != hipSuccess) return e;
    e = ctof::launch_contract(k, true, mhat(), yhat(), st);
    if (e != hipSuccess) return e;
    return ctof::launch_col_pass<T>(k->dims, k->dims.nzp, true, yhat(), xz(), st);
  }
};

ctof_status check_kernel(ctof_kernel k) {
  if (!k) return set_error(CTOF_EINVAL, "kernel handle is NULL");
  if (!k->khat) return set_error(CTOF_EINVAL, "kernel handle has no spectrum");
  return CTOF_OK;
}

template <typename T>
ctof_status run_forward(ctof_kernel k, const void *mu, void *m, void *ws, hipStream_t st) {
  Ops<T> ops{k, reinterpret_cast<char *>(ws), op_ws(k->dims, k->prec, 1), st};
  ctof::RowArgs a = ops.row(ctof::ROW_SPATIAL_TO_SPEC, false);
  a.sp_in = mu;
  HIP_TRY(ops.mu_to_spec(a));
  HIP_TRY(ops.fwd_to_xt());
  ctof::RowArgs b = ops.row(ctof::ROW_SPEC_TO_SPATIAL, true);
  b.sp_out = m;
  HIP_TRY(ctof::launch_row_pass<T>(k->dims, b, st));
  return CTOF_OK;
}

template <typename T>
ctof_status run_adjoint(ctof_kernel k, const void *r, void *g, void *ws, hipStream_t st) {
  Ops<T> ops{k, reinterpret_cast<char *>(ws), op_ws(k->dims, k->prec, 1), st};
  ctof::RowArgs a = ops.row(ctof::ROW_SPATIAL_TO_SPEC, true);
  a.sp_in = r;
  HIP_TRY(ctof::launch_row_pass<T>(k->dims, a, st));
  HIP_TRY(ops.adj_to_xz());
  ctof::RowArgs b = ops.row(ctof::ROW_SPEC_TO_SPATIAL, false);
  b.sp_out = g;
  HIP_TRY(ctof::launch_row_pass<T>(k->dims, b, st));
  return CTOF_OK;
}

std::vector<double> fista_betas(int iters) {
  std::vector<double> b(iters);
  double t = 1.0;
  for (int k = 0; k < iters; ++k) {
    const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
    b[k] = (t - 1.0) / tn;
    t = tn;
  }
  return b;
}

template <typename T>
ctof_status run_reconstruct(ctof_kernel k, const void *d, void *mu, const ctof_solver_opts *opt,
                            ctof_solver_report *rep, void *ws, hipStream_t st) {
  const ctof::Dims &dm = k->dims;
  const OpWs L = op_ws(dm, k->prec, opt->max_iter);
  Ops<T> ops{k, reinterpret_cast<char *>(ws), L, st};
  char *base = reinterpret_cast<char *>(ws);
  T *y = reinterpret_cast<T *>(base + L.y);
  T *v = reinterpret_cast<T *>(base + L.v);
  T *w = reinterpret_cast<T *>(base + L.w);
  double *hist = reinterpret_cast<double *>(base + L.hist);
  double *scal = reinterpret_cast<double *>(base + L.scal);
  double *part = reinterpret_cast<double *>(base + L.part);
  const size_t vol = (size_t)dm.nz * dm.n * dm.n;
  const int K = opt->max_iter;
  // scalars: [0] |w|^2  [1] <v,w>  [2] |max(0, A^T d)|^2  [3..4] final fit  [5..6] last hist
  HIP_TRY(ctof::launch_fill_zero(scal, 64 * 8, st));
  if (!opt->warm_start) HIP_TRY(ctof::launch_fill_zero(mu, vol * sizeof(T), st));

  // ||G(0)|| = ||max(0, A^T d)||
  {
    ctof::RowArgs a = ops.row(ctof::ROW_SPATIAL_TO_SPEC, true);
    a.sp_in = d;
    HIP_TRY(ctof::launch_row_pass<T>(dm, a, st));
    HIP_TRY(ops.adj_to_xz());
    ctof::RowArgs b = ops.row(ctof::ROW_GMAP0, false);
    b.partials = part;
    HIP_TRY(ctof::launch_row_pass<T>(dm, b, st));
    HIP_TRY(ctof::launch_reduce_rows(part, L.nblk_z, 2, 1, scal + 2, st));
  }

  double lam = opt->lambda_tikhonov, Lip = opt->lipschitz, LA = 0.0;
  if (Lip == 0.0) {
    const int iters = opt->power_iters > 0 ? opt->power_iters : 50;
    if (sizeof(T) == 8)
      HIP_TRY(ctof::launch_fill_value_f64(reinterpret_cast<double *>(v), vol, 1.0 / std::sqrt((double)vol), st));
    else
      HIP_TRY(ctof::launch_fill_value(reinterpret_cast<float *>(v), vol, (float)(1.0 / std::sqrt((double)vol)), st));
    for (int j = 0; j < iters; ++j) {
      ctof::RowArgs a = ops.row(j == 0 ? ctof::ROW_SPATIAL_TO_SPEC : ctof::ROW_SCALE_TO_SPEC, false);
      a.sp_in = j == 0 ? (const void *)v : (const void *)w;
      a.sp_out = v;
      a.scalar = scal + 0;
      HIP_TRY(ops.mu_to_spec(a));
      HIP_TRY(ops.fwd_to_xt());
      ctof::RowArgs b = ops.row(ctof::ROW_PASS, true);
      HIP_TRY(ctof::launch_row_pass<T>(dm, b, st));
      HIP_TRY(ops.adj_to_xz());
      ctof::RowArgs c = ops.row(ctof::ROW_POWER_W, false);
      c.sp_in = v;
      c.sp_out = w;
      c.partials = part;
      HIP_TRY(ctof::launch_row_pass<T>(dm, c, st));
      HIP_TRY(ctof::launch_reduce_rows(part, L.nblk_z, 2, 2, scal + 0, st));
    }
    double hs[3];
    HIP_TRY(hipMemcpyAsync(hs, scal, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
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

  // FISTA: y_1 = mu_0
  HIP_TRY(hipMemcpyAsync(y, mu, vol * sizeof(T), hipMemcpyDeviceToDevice, st));
  {
    ctof::RowArgs a = ops.row(ctof::ROW_SPATIAL_TO_SPEC, false);
    a.sp_in = y;
    HIP_TRY(ops.mu_to_spec(a));
  }
  const std::vector<double> beta = fista_betas(K);
  // optional stage timing: five events per iteration on the caller's stream
  std::vector<hipEvent_t> ev;
  struct EventGuard {
    std::vector<hipEvent_t> *v;
    ~EventGuard() {
      for (hipEvent_t e : *v) (void)hipEventDestroy(e);
    }
  } guard{&ev};
  if (opt->timing) {
    ev.resize((size_t)K * 5, nullptr);
    for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
  }
  auto mark = [&](int it, int j) -> hipError_t {
    return opt->timing ? hipEventRecord(ev[(size_t)it * 5 + j], st) : hipSuccess;
  };
  int done = 0;
  for (int it = 0; it < K; ++it) {
    double *pk = part + (size_t)it * L.part_stride;
    HIP_TRY(mark(it, 0));
    HIP_TRY(ctof::launch_contract(k, false, ops.yhat(), ops.mhat(), st));
    HIP_TRY(mark(it, 1));
    HIP_TRY(ctof::launch_col_pass<T>(dm, dm.ntp, true, ops.mhat(), ops.xt(), st));
    ctof::RowArgs a = ops.row(ctof::ROW_RESIDUAL, true);
    a.sp_in = d;
    a.partials = pk;
    HIP_TRY(ctof::launch_row_pass<T>(dm, a, st));
    HIP_TRY(ctof::launch_col_pass<T>(dm, dm.ntp, false, ops.xt(), ops.mhat(), st));
    HIP_TRY(mark(it, 2));
    HIP_TRY(ctof::launch_contract(k, true, ops.mhat(), ops.yhat(), st));
    HIP_TRY(mark(it, 3));
    HIP_TRY(ctof::launch_col_pass<T>(dm, dm.nzp, true, ops.yhat(), ops.xz(), st));
    ctof::RowArgs b = ops.row(ctof::ROW_FISTA, false);
    b.sp_in = y;
    b.sp_out = y;
    b.sp_aux = mu;
    b.partials = pk + 2 * (size_t)L.nblk_t;
    b.tau = tau;
    b.lambda = lam;
    b.beta = beta[it];
    HIP_TRY(ctof::launch_row_pass<T>(dm, b, st));
    HIP_TRY(ctof::launch_col_pass<T>(dm, dm.nzp, false, ops.xz(), ops.yhat(), st));
    HIP_TRY(mark(it, 4));
    done = it + 1;
    if (opt->rel_tol > 0 && (done % opt->check_every == 0) && done < K) {
      HIP_TRY(ctof::launch_history_k(part + (size_t)it * L.part_stride, 1, L.nblk_t, L.nblk_z, tau,
                                     scal + 2, scal + 5, nullptr, st));
      double h2[2];
      HIP_TRY(hipMemcpyAsync(h2, scal + 5, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (!std::isfinite(h2[0]) || !std::isfinite(h2[1])) break;
      if (h2[1] <= opt->rel_tol) break;
    }
  }
  HIP_TRY(ctof::launch_history_k(part, done, L.nblk_t, L.nblk_z, tau, scal + 2, hist, scal + 5, st));
  if (opt->history_dev)
    HIP_TRY(hipMemcpyAsync(opt->history_dev, hist, (size_t)done * 2 * sizeof(double),
                           hipMemcpyDeviceToDevice, st));
  // final data fit 1/2 ||A mu - d||^2
  {
    double *pf = part + (size_t)(K) * L.part_stride;
    ctof::RowArgs a = ops.row(ctof::ROW_SPATIAL_TO_SPEC, false);
    a.sp_in = mu;
    HIP_TRY(ops.mu_to_spec(a));
    HIP_TRY(ops.fwd_to_xt());
    ctof::RowArgs b = ops.row(ctof::ROW_RESIDUAL, true);
    b.sp_in = d;
    b.partials = pf;
    HIP_TRY(ctof::launch_row_pass<T>(dm, b, st));
    HIP_TRY(ctof::launch_reduce_rows(pf, L.nblk_t, 2, 1, scal + 3, st));
  }
  double hs[8];
  double h0[2];
  HIP_TRY(hipMemcpyAsync(hs, scal, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(h0, hist, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (opt->timing && done > 0) {
    double acc[4] = {0, 0, 0, 0};
    for (int it = 0; it < done; ++it) {
      for (int j = 0; j < 4; ++j) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ev[(size_t)it * 5 + j], ev[(size_t)it * 5 + j + 1]));
        acc[j] += ms;
      }
    }
    float loop = 0.f;
    HIP_TRY(hipEventElapsedTime(&loop, ev[0], ev[(size_t)(done - 1) * 5 + 4]));
    rep->ms_contract_fwd = acc[0];
    rep->ms_fft_t = acc[1];
    rep->ms_contract_adj = acc[2];
    rep->ms_fft_z = acc[3];
    rep->ms_loop = loop;
  }
  rep->iters = done;
  rep->datafit0 = h0[0];
  rep->datafit = hs[3];
  rep->gmap_ratio = hs[6];
  rep->gmap0 = std::sqrt(hs[2]);
  rep->status = CTOF_OK;
  if (!std::isfinite(rep->datafit) || !std::isfinite(rep->datafit0) || !std::isfinite(rep->gmap_ratio) ||
      !std::isfinite(rep->gmap0)) {
    rep->status = CTOF_ENONFINITE;
    return set_error(CTOF_ENONFINITE, "non-finite FP64 norm during the solve");
  }
  return CTOF_OK;
}

}  // namespace

namespace ctof {

Dims make_dims(int n, int nz, int nt, ctof_precision prec) {
  Dims d;
  d.n = n;
  d.nz = nz;
  d.nt = nt;
  d.p = std::max(kMinP, next_pow2(2 * n - 1));
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

const char *ctof_last_error(void) { return g_err.c_str(); }

ctof_status ctof_kernel_bytes(const ctof_geometry *geom, ctof_precision prec, size_t *khat_bytes,
                              size_t *tab_ws_bytes) {
  ctof_status s = check_geometry(geom, nullptr, nullptr);
  if (s != CTOF_OK) return s;
  if (!valid_prec(prec)) return set_error(CTOF_EINVAL, "unknown precision %d", (int)prec);
  const ctof::Dims d = ctof::make_dims(geom->nx, geom->nz, geom->nt, prec);
  if (khat_bytes) *khat_bytes = ctof::khat_layout(d, prec).total;
  if (tab_ws_bytes) *tab_ws_bytes = tab_ws(d).total;
  return CTOF_OK;
}

ctof_status ctof_kernel_tabulate(const ctof_geometry *geom, ctof_precision prec, void *khat_dev,
                                 size_t khat_bytes, void *tab_ws_dev, size_t tab_ws_bytes,
                                 hipStream_t stream, ctof_kernel *out) {
  ctof::TabGeom tg;
  ctof::LayerDepths zs;
  ctof_status s = check_geometry(geom, &tg, &zs);
  if (s != CTOF_OK) return s;
  if (!valid_prec(prec)) return set_error(CTOF_EINVAL, "unknown precision %d", (int)prec);
  if (!out) return set_error(CTOF_EINVAL, "out handle pointer is NULL");
  if (!khat_dev || !tab_ws_dev) return set_error(CTOF_EINVAL, "device buffer is NULL");
  const ctof::Dims d = ctof::make_dims(geom->nx, geom->nz, geom->nt, prec);
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
  HIP_TRY(ctof::launch_gemm_f64(d.h + 1, (long long)per, d.n, C, d.n, 0, Q, (long long)per, (long long)(d.n * per),
                                T1, (long long)per, (long long)((d.h + 1) * per), d.n, stream));
  // K64[a][b][k][z] = sum_dy C[a][dy] T1[dy][b][k][z]   (written over Q)
  const long long N2 = (long long)(d.h + 1) * (long long)per;
  HIP_TRY(ctof::launch_gemm_f64(d.h + 1, N2, d.n, C, d.n, 0, T1, N2, 0, Q,
                                N2, 0, 1, stream));
  HIP_TRY(ctof::launch_pack(d, prec, Q, khat_dev, lay, 1.0 / ((double)d.p * (double)d.p), stream));
  HIP_TRY(hipStreamSynchronize(stream));
  ctof_kernel_s *k = new (std::nothrow) ctof_kernel_s;
  if (!k) return set_error(CTOF_ENOMEM, "host allocation of the handle failed");
  k->dims = d;
  k->prec = prec;
  k->geom = tg;
  k->khat = khat_dev;
  k->layout = lay;
  *out = k;
  return CTOF_OK;
}

ctof_status ctof_kernel_tabulate_quadrant(const ctof_geometry *geom, double *quad_dev, size_t quad_bytes,
                                          hipStream_t stream) {
  ctof::TabGeom tg;
  ctof::LayerDepths zs;
  ctof_status s = check_geometry(geom, &tg, &zs);
  if (s != CTOF_OK) return s;
  if (!quad_dev) return set_error(CTOF_EINVAL, "quad_dev is NULL");
  const size_t n = geom->nx;
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

ctof_status ctof_workspace_bytes(ctof_kernel k, int32_t max_iter, size_t *op_ws_bytes, size_t *solve_ws) {
  ctof_status s = check_kernel(k);
  if (s != CTOF_OK) return s;
  if (max_iter < 0) return set_error(CTOF_EINVAL, "max_iter must be >= 0");
  const OpWs o = op_ws(k->dims, k->prec, max_iter);
  if (op_ws_bytes) *op_ws_bytes = o.op_total;
  if (solve_ws) *solve_ws = o.solve_total;
  return CTOF_OK;
}

ctof_status ctof_forward(ctof_kernel k, const void *mu_dev, void *m_dev, void *ws_dev, size_t ws_bytes,
                         hipStream_t stream) {
  ctof_status s = check_kernel(k);
  if (s != CTOF_OK) return s;
  if (!mu_dev || !m_dev || !ws_dev) return set_error(CTOF_EINVAL, "device pointer is NULL");
  const OpWs o = op_ws(k->dims, k->prec, 1);
  if (ws_bytes < o.op_total) return set_error(CTOF_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, o.op_total);
  if (k->prec == CTOF_FP64) return run_forward<double>(k, mu_dev, m_dev, ws_dev, stream);
  return run_forward<float>(k, mu_dev, m_dev, ws_dev, stream);
}

ctof_status ctof_adjoint(ctof_kernel k, const void *r_dev, void *g_dev, void *ws_dev, size_t ws_bytes,
                         hipStream_t stream) {
  ctof_status s = check_kernel(k);
  if (s != CTOF_OK) return s;
  if (!r_dev || !g_dev || !ws_dev) return set_error(CTOF_EINVAL, "device pointer is NULL");
  const OpWs o = op_ws(k->dims, k->prec, 1);
  if (ws_bytes < o.op_total) return set_error(CTOF_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, o.op_total);
  if (k->prec == CTOF_FP64) return run_adjoint<double>(k, r_dev, g_dev, ws_dev, stream);
  return run_adjoint<float>(k, r_dev, g_dev, ws_dev, stream);
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
  if (opts->warm_start != 0 && opts->warm_start != 1) return set_error(CTOF_EINVAL, "warm_start must be 0 or 1");
  const OpWs o = op_ws(k->dims, k->prec, opts->max_iter);
  if (ws_bytes < o.solve_total) return set_error(CTOF_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, o.solve_total);
  std::memset(report, 0, sizeof(*report));
  if (k->prec == CTOF_FP64) return run_reconstruct<double>(k, d_dev, mu_inout_dev, opts, report, ws_dev, stream);
  return run_reconstruct<float>(k, d_dev, mu_inout_dev, opts, report, ws_dev, stream);
}

}  // extern "C"
