// FP64 tabulation of the confocal kernel and its real 2D spectrum (gfx950).
//
// Kernel values follow Eq. 5 of the paper (the time-resolved Jacobian as
// the time convolution of the diffusion fluence Phi0 from the source and
// the reflectance R back to the detector), for a collocated source and
// detector on a semi-infinite homogeneous medium with an extrapolated
// boundary.  The convolution has a closed form: with a = r1 + r2 (source or
// its image to the voxel, plus voxel or its image to the detector) each of
// the four image terms is
//   amp * t^(-3/2) exp(-alpha/t - beta t) (2 alpha/t + g - 1),
//   alpha = a^2/(4 D c), beta = mu_a c, g = a / r2,
// whose integral from 0 to T is
//   F(T) = 2 e(T)/sqrt(T) + g I_{3/2}(T) + 2 beta I_{1/2}(T),
// where I_nu(T) = int_0^T s^(-nu) exp(-alpha/s - beta s) ds are written
// with erfcx/erfc (device math library).  A bin is F(hi) - F(lo) while that
// difference does not cancel (F(lo) <= 100 |F(hi) - F(lo)|), else 16-point
// Gauss-Legendre on the integrand.  Each value is scaled by the voxel
// volume.
//
// Fluorescence mode (section "Materials and Methods": excitation and
// emission optics, lifetime convolution): the fluence comes from the
// excitation optics, the flux back to the detector from the emission
// optics, and the emission is delayed by E_tau(t) = exp(-t/tau)/tau.  With
// a shared mu_a the two diffusion wavenumbers are proportional, so every
// image term keeps the form above with D = D_em, a = r1 sqrt(D_em/D_ex) + r2
// and amp = sigma w / (16 pi^2 D_ex r1 r2^2) (absorption mode is D_em = D_ex).
// The lifetime convolution h = k (*) E_tau of a term has the exact
// antiderivative
//   Q(T) = F_beta(T) - exp(-T/tau) F_beta'(T),   beta' = beta - 1/tau > 0,
// since h(T) = exp(-T/tau) F_beta'(T) / tau; bins use Q like F above, with
// Gauss-Legendre on h where the difference cancels.
//
// The kernel is even in both lateral offsets, so its spectrum on a P x P
// torus is real and equals a cosine transform:
//   Khat(a, b) = sum_{dy, dx} w_dy w_dx K[dy][dx] cos(2 pi a dy / P) cos(2 pi b dx / P)
// with w_0 = 1, w_{>0} = 2 over the quadrant dy, dx in [0, n).  It is
// evaluated as two FP64 GEMMs with the cosine matrix C[a][d] = w_d cos(2 pi a d / P).
#include "ctof_internal.h"

#include <cmath>

namespace ctof {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrtPi = 1.77245385090551602730;

__device__ inline double antiderivative(double alpha, double sqrt_alpha, double beta,
                                        double sqrt_beta, double g, double T) {
  if (!(T > 0.0)) return 0.0;
  const double x = sqrt(alpha / T);
  const double y = sqrt(beta * T);
  const double E = exp(-x * x - y * y);
  const double ep = E * erfcx(x + y);
  const double em = (x >= y) ? E * erfcx(x - y) : exp(-2.0 * x * y) * erfc(x - y);
  const double i32 = kSqrtPi / (2.0 * sqrt_alpha) * (em + ep);
  const double i12 = kSqrtPi / (2.0 * sqrt_beta) * (em - ep);
  return 2.0 * E / sqrt(T) + g * i32 + 2.0 * beta * i12;
}

__device__ inline double integrand(double alpha, double beta, double g, double s) {
  const double inv = 1.0 / s;
  return inv * sqrt(inv) * exp(-alpha * inv - beta * s) * (2.0 * alpha * inv + g - 1.0);
}

// Antiderivative of a term's bin integrand: F (no lifetime) or Q (lifetime).
struct TermCurve {
  double alpha, sa, g, beta, sb, betap, sbp, tau;
  __device__ double prim(double T) const {
    const double f = antiderivative(alpha, sa, beta, sb, g, T);
    if (tau == 0.0) return f;
    return f - exp(-T / tau) * antiderivative(alpha, sa, betap, sbp, g, T);
  }
  __device__ double density(double s) const {
    if (tau == 0.0) return integrand(alpha, beta, g, s);
    return exp(-s / tau) * antiderivative(alpha, sa, betap, sbp, g, s) / tau;
  }
};

// One thread per (layer, dy, dx); loops over the time bins so that F at the
// upper edge of bin k is reused as the lower edge of bin k+1.
__global__ void __launch_bounds__(128)
tab_values_kernel(TabGeom g, LayerDepths zs, GaussLegendre16 gl, double *__restrict__ out,
                  size_t s_dy, size_t s_dx, size_t s_z, size_t s_t, int z_fastest) {
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)g.nz * g.n * g.n;
  if (tid >= total) return;
  int z, dy, dx;
  if (z_fastest) {
    z = (int)(tid % g.nz);
    const size_t r = tid / g.nz;
    dx = (int)(r % g.n);
    dy = (int)(r / g.n);
  } else {
    dx = (int)(tid % g.n);
    const size_t r = tid / g.n;
    dy = (int)(r % g.n);
    z = (int)(r / g.n);
  }
  const Optics o = g.o;
  const double zz = zs.z[z];
  const double rho2 = g.pitch * g.pitch * (double)(dy * dy + dx * dx);
  const double Dc = g.Dm * o.c;
  const double beta = o.mua * o.c;
  const double norm = 1.0 / (2.0 * sqrt(kPi * Dc));
  const double scale = sqrt(g.Dm / o.D);  // exactly 1 in absorption mode

  const double r11 = fmax(sqrt(rho2 + (zz - o.z0) * (zz - o.z0)), g.rmin);
  const double zs1 = zz + o.z0 + 2.0 * o.zb;
  const double r12 = sqrt(rho2 + zs1 * zs1);
  const double zi = zz + 2.0 * g.zbm;
  const double r21 = sqrt(rho2 + zz * zz);
  const double r22 = sqrt(rho2 + zi * zi);

  double amp[4], flo[4];
  TermCurve tc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double sigma = (q < 2) ? 1.0 : -1.0;
    const double r1 = (q < 2) ? r11 : r12;
    const double w = (q & 1) ? zi : zz;
    const double r2 = (q & 1) ? r22 : r21;
    const double a = r1 * scale + r2;
    amp[q] = sigma * w / (16.0 * kPi * kPi * o.D * r1 * r2 * r2) * norm;
    tc[q].alpha = a * a / (4.0 * Dc);
    tc[q].sa = sqrt(tc[q].alpha);
    tc[q].g = a / r2;
    tc[q].beta = beta;
    tc[q].sb = sqrt(beta);
    tc[q].tau = g.tau;
    tc[q].betap = g.tau > 0.0 ? beta - 1.0 / g.tau : beta;
    tc[q].sbp = sqrt(tc[q].betap);
    flo[q] = tc[q].prim(g.t0);
  }
  double *dst = out + (size_t)dy * s_dy + (size_t)dx * s_dx + (size_t)z * s_z;
  for (int k = 0; k < g.nt; ++k) {
    const double tlo = g.t0 + (double)k * g.dt;
    const double thi = g.t0 + (double)(k + 1) * g.dt;
    const double mid = 0.5 * (thi + tlo);
    const double half = 0.5 * (thi - tlo);
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double fhi = tc[q].prim(thi);
      const double df = fhi - flo[q];
      double bin;
      if (flo[q] <= 100.0 * fabs(df)) {
        bin = df;
      } else {
        double acc = 0.0;
#pragma unroll 4
        for (int e = 0; e < 16; ++e) acc += gl.w[e] * tc[q].density(mid + half * gl.x[e]);
        bin = acc * half;
      }
      sum += amp[q] * bin;
      flo[q] = fhi;
    }
    dst[(size_t)k * s_t] = g.dv * sum;
  }
}

// The cosine matrix C[a][d] = w_d cos(2 pi a d / p), a in [0, h], d in
// [0, n) (w_0 = 1, else 2), written in the GEMM's operand order: entry
// (t ks + s) 64 + lane holds C[16 t + lane % 16][4 s + lane / 16], ks =
// ceil(n / 4) steps of depth 4 per tile of 16 rows, zero past h and n.
__global__ void cosine_kernel(int n, int p, double *__restrict__ C) {
  const int h = p / 2;
  const int ks = (n + 3) / 4;
  const long long total = (long long)((h + 1 + 15) / 16) * ks * 64;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int lane = (int)(idx & 63);
  const long long ts = idx >> 6;
  const int t = (int)(ts / ks), st = (int)(ts % ks);
  const int a = 16 * t + (lane & 15);
  const int d = 4 * st + (lane >> 4);
  double v = 0.0;
  if (a <= h && d < n) {
    const long long m = (2LL * a * d) % (2LL * p);
    v = ((d == 0) ? 1.0 : 2.0) * cospi((double)m / (double)p);
  }
  C[idx] = v;
}

// FP64 GEMM on the matrix cores, C = A B: A [M][K] in the operand order of
// cosine_kernel (Af), B [K][N] row-major (row stride ldb), C [M][N]
// row-major (ldc), batch z offset by sB and sC.  A wave owns 16 columns of
// C and a group of up to GMT row tiles of 16 (the cosine transform's M =
// P/2 + 1 rows fit one group up to P = 286): per 4-deep step of K it loads
// one B fragment (4 rows x 16 columns, the streamed operand, read once per
// group) and one A fragment per row tile (512 contiguous bytes; A is at most
// a few MB and stays in the caches), and issues one 16x16x4 FP64 MFMA per
// row tile; the next step's operands are loaded before the current step's
// products.  Operand lanes: A row i = lane % 16 and B column j = lane % 16,
// both at depth lane / 16; the result item r of lane group g is row 4r + g
// of the tile.
typedef double gemm_v4d __attribute__((ext_vector_type(4)));
constexpr int GMT = 9;

__global__ void __launch_bounds__(256)
gemm_f64_kernel(int M, long long N, int K, const double *__restrict__ Af, const double *__restrict__ B,
                long long ldb, long long sB, double *__restrict__ C, long long ldc, long long sC) {
  const int l = threadIdx.x & 63;
  const int c = l & 15, g = l >> 4;
  const long long col = ((long long)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16 + c;
  const int mt0 = blockIdx.y * GMT;                     // first row tile of the group
  const int nmt = min(GMT, (M + 15) / 16 - mt0);        // row tiles in the group
  const int ks = (K + 3) / 4;
  B += sB * blockIdx.z;
  C += sC * blockIdx.z;
  const bool con = col < N;
  gemm_v4d acc[GMT];
#pragma unroll
  for (int t = 0; t < GMT; ++t) acc[t] = {0.0, 0.0, 0.0, 0.0};
  // operands of step k0 + 4 are loaded before the products of step k0
  auto load = [&](int k0, double &b, double (&a)[GMT]) {
    const int k = k0 + g;
    b = (con && k < K) ? B[(long long)k * ldb + col] : 0.0;
#pragma unroll
    for (int t = 0; t < GMT; ++t)
      a[t] = t < nmt ? Af[((size_t)(mt0 + t) * ks + k0 / 4) * 64 + l] : 0.0;
  };
  double b0, a0[GMT], b1, a1[GMT];
  load(0, b0, a0);
  for (int k0 = 0; k0 < K; k0 += 8) {
    if (k0 + 4 < K) load(k0 + 4, b1, a1);
#pragma unroll
    for (int t = 0; t < GMT; ++t)
      if (t < nmt) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[t], b0, acc[t], 0, 0, 0);
    if (k0 + 4 >= K) break;
    if (k0 + 8 < K) load(k0 + 8, b0, a0);
#pragma unroll
    for (int t = 0; t < GMT; ++t)
      if (t < nmt) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[t], b1, acc[t], 0, 0, 0);
  }
  if (!con) return;
#pragma unroll
  for (int t = 0; t < GMT; ++t) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * (mt0 + t) + 4 * r + g;
      if (t < nmt && row < M) C[(long long)row * ldc + col] = acc[t][r];
    }
  }
}

__device__ inline void matrix_ab(int s, int &a, int &b) {
  int bb = (int)((sqrt(8.0 * (double)s + 1.0) - 1.0) * 0.5);
  while ((bb + 1) * (bb + 2) / 2 <= s) ++bb;
  while (bb * (bb + 1) / 2 > s) --bb;
  b = bb;
  a = s - bb * (bb + 1) / 2;
}

// Pack the FP64 spectrum k64[a][b][k][z] (a, b in [0, h]) into the
// fragment-ordered forward and adjoint layouts (see Frag), s = b(b+1)/2 + a
// for a <= b, scaled by `scale` (the 1/p^2 of the unnormalised inverse FFTs);
// padded bins and layers are zero.  One thread per packed element.
template <int KIND>  // 0 double, 1 float, 2 bf16 hi+lo, 3 bf16 hi
__global__ void __launch_bounds__(256)
pack_kernel(Dims d, Frag fr, const double *__restrict__ k64, char *__restrict__ khat,
            KhatLayout lay, double scale, int adjoint) {
  const size_t per = (size_t)d.ntp * d.nzp;
  const size_t total = (size_t)d.nmat * per;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int s = (int)(idx / per);
  size_t r = idx % per;
  const int e = (int)(r % fr.v);
  r /= fr.v;
  const int lane = (int)(r % 64);
  r /= 64;
  int t, z;
  if (!adjoint) {
    const int nq = fr.kz / fr.v;
    const int nch = d.nzp / (4 * fr.kz);
    const int q = (int)(r % nq);
    r /= nq;
    const int ch = (int)(r % nch);
    const int tt = (int)(r / nch);
    t = 16 * tt + frag_row(fr.f64, lane % 16);
    z = 4 * fr.kz * ch + fr.kz * (lane / 16) + fr.v * q + e;
  } else {
    const int nq = fr.tl / fr.v;
    const int nzt = d.nzp / 16;
    const int q = (int)(r % nq);
    r /= nq;
    const int zt = (int)(r % nzt);
    const int tci = (int)(r / nzt);
    z = 16 * zt + frag_row(fr.f64, lane % 16);
    t = fr.tc * tci + fr.tl * (lane / 16) + fr.v * q + e;
  }
  int a, b;
  matrix_ab(s, a, b);
  double v = 0.0;
  if (t < d.nt && z < d.nz) v = k64[(((size_t)a * (d.h + 1) + b) * d.nt + t) * d.nz + z] * scale;
  const size_t off = adjoint ? lay.adj : lay.fwd;
  if (KIND == 0) {
    reinterpret_cast<double *>(khat + off)[idx] = v;
  } else if (KIND == 1) {
    reinterpret_cast<float *>(khat + off)[idx] = (float)v;
  } else {
    const __bf16 hi = (__bf16)(float)v;
    reinterpret_cast<__bf16 *>(khat + off)[idx] = hi;
    if (KIND == 2) {
      const size_t lo = adjoint ? lay.adj_lo : lay.fwd_lo;
      reinterpret_cast<__bf16 *>(khat + lo)[idx] = (__bf16)(float)(v - (double)(float)hi);
    }
  }
}

}  // namespace

hipError_t launch_tab_values(const TabGeom &g, const LayerDepths &z, const GaussLegendre16 &gl,
                             double *out, size_t s_dy, size_t s_dx, size_t s_z, size_t s_t,
                             hipStream_t st) {
  const size_t total = (size_t)g.nz * g.n * g.n;
  const int z_fastest = (s_z == 1) ? 1 : 0;
  const unsigned blocks = (unsigned)((total + 127) / 128);
  hipLaunchKernelGGL(tab_values_kernel, dim3(blocks), dim3(128), 0, st, g, z, gl, out, s_dy, s_dx,
                     s_z, s_t, z_fastest);
  return hipGetLastError();
}

size_t cosine_matrix_elems(int n, int p) { return (size_t)((p / 2 + 1 + 15) / 16) * ((n + 3) / 4) * 64; }

hipError_t launch_cosine_matrix(int n, int p, double *C, hipStream_t st) {
  const size_t total = cosine_matrix_elems(n, p);
  hipLaunchKernelGGL(cosine_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n, p, C);
  return hipGetLastError();
}

hipError_t launch_gemm_f64(int M, long long N, int K, const double *Af, const double *B, long long ldb,
                           long long sB, double *C, long long ldc, long long sC, int batch, hipStream_t st) {
  // 64 columns (four waves of 16) per block; one block row per group of row tiles
  const int groups = ((M + 15) / 16 + GMT - 1) / GMT;
  dim3 grid((unsigned)((N + 63) / 64), (unsigned)groups, (unsigned)batch);
  hipLaunchKernelGGL(gemm_f64_kernel, grid, dim3(256), 0, st, M, N, K, Af, B, ldb, sB, C, ldc, sC);
  return hipGetLastError();
}

hipError_t launch_pack(const Dims &d, ctof_precision prec, const double *k64, void *khat,
                       const KhatLayout &lay, double scale, hipStream_t st) {
  const size_t total = (size_t)d.nmat * d.ntp * d.nzp;
  const dim3 grid((unsigned)((total + 255) / 256));
  const Frag fr = frag_of(d, prec);
  char *kh = reinterpret_cast<char *>(khat);
  for (int adj = 0; adj < 2; ++adj) {
    switch (prec) {
      case CTOF_FP64:
        hipLaunchKernelGGL(pack_kernel<0>, grid, dim3(256), 0, st, d, fr, k64, kh, lay, scale, adj);
        break;
      case CTOF_FP32:
        hipLaunchKernelGGL(pack_kernel<1>, grid, dim3(256), 0, st, d, fr, k64, kh, lay, scale, adj);
        break;
      case CTOF_BF16X3:
        hipLaunchKernelGGL(pack_kernel<2>, grid, dim3(256), 0, st, d, fr, k64, kh, lay, scale, adj);
        break;
      default:
        hipLaunchKernelGGL(pack_kernel<3>, grid, dim3(256), 0, st, d, fr, k64, kh, lay, scale, adj);
        break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace ctof
