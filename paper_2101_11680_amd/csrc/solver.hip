// FP64 reductions and small helper kernels for the FISTA driver (gfx950).
//
// Every norm the solver reports (data fit, gradient mapping, power-iteration
// Rayleigh quotients) is accumulated per block in FP64 by the FFT row pass
// and summed here in a fixed order, so repeated runs are bitwise identical.
#include "ctof_internal.h"

namespace ctof {

namespace {

__device__ inline double block_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// sums[j] = sum_i partials[i * stride + j]
__global__ void __launch_bounds__(256)
reduce_rows_kernel(const double *__restrict__ partials, int nrows, int stride, int count,
                   double *__restrict__ sums) {
  __shared__ double red[256];
  for (int j = 0; j < count; ++j) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < nrows; i += blockDim.x) acc += partials[(size_t)i * stride + j];
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) sums[j] = tot;
  }
}

// Block (it, v): data fit and gradient-mapping ratio of volume v at iteration it.
__global__ void __launch_bounds__(256)
history_kernel(const double *__restrict__ partials, int nvol, int nblk_t, int nblk_z, size_t stride,
               double tau, const double *__restrict__ g0sq, double *__restrict__ hist) {
  __shared__ double red[256];
  const int it = blockIdx.x, v = blockIdx.y;
  const double *pt = partials + (size_t)it * stride;
  const double *pz = pt + 2 * (size_t)nblk_t;
  const int bt = nblk_t / nvol, bz = nblk_z / nvol;
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < bt; i += blockDim.x) a += pt[2 * ((size_t)v * bt + i)];
  for (int i = threadIdx.x; i < bz; i += blockDim.x) b += pz[2 * ((size_t)v * bz + i)];
  const double fit = block_sum(a, red);
  const double gm = block_sum(b, red);
  if (threadIdx.x == 0) {
    const double g0 = sqrt(g0sq[v]);
    const double ratio = g0 > 0.0 ? sqrt(gm) / (tau * g0) : 0.0;
    hist[2 * ((size_t)it * nvol + v)] = fit;
    hist[2 * ((size_t)it * nvol + v) + 1] = ratio;
  }
}

// Block v: the gradient-mapping ratio of volume v at the last completed
// iteration (*ctr - 1), summed exactly as history_kernel does; a live volume
// whose ratio is finite and <= rel_tol is frozen (active = 0) and its
// iteration count recorded.
// g0_part (or NULL): the first step's partials of ||max(0, A^T d)||^2 (a zero
// start), summed into g0sq[v] first exactly as reduce_volumes_kernel does.
__global__ void __launch_bounds__(256)
freeze_kernel(const double *__restrict__ partials, size_t stride, const int *__restrict__ ctr, int nvol,
              int nblk_t, int nblk_z, double tau, double *__restrict__ g0sq, const double *__restrict__ g0_part,
              double rel_tol, int *__restrict__ active, int *__restrict__ conv) {
  __shared__ double red[256];
  const int v = blockIdx.x;
  if (active[v] == 0) return;  // (the same value for every thread of the block)
  const int bz = nblk_z / nvol;
  double g0s = 0.0;
  if (g0_part != nullptr) {
    double a = 0.0;
    for (int i = threadIdx.x; i < bz; i += blockDim.x) a += g0_part[2 * ((size_t)v * bz + i)];
    g0s = block_sum(a, red);
  }
  const int it = *ctr - 1;
  const double *pz = partials + (size_t)it * stride + 2 * (size_t)nblk_t;
  double b = 0.0;
  for (int i = threadIdx.x; i < bz; i += blockDim.x) b += pz[2 * ((size_t)v * bz + i)];
  const double gm = block_sum(b, red);
  if (threadIdx.x == 0) {
    if (g0_part != nullptr) g0sq[v] = g0s;
    const double g0 = sqrt(g0_part != nullptr ? g0s : g0sq[v]);
    const double ratio = g0 > 0.0 ? sqrt(gm) / (tau * g0) : 0.0;
    if (isfinite(ratio) && ratio <= rel_tol) {
      active[v] = 0;
      conv[v] = it + 1;
    }
  }
}

__global__ void __launch_bounds__(256)
reduce_volumes_kernel(const double *__restrict__ partials, int nblk, int nvol, double *__restrict__ out) {
  __shared__ double red[256];
  const int v = blockIdx.x;
  const int per = nblk / nvol;
  double a = 0.0;
  for (int i = threadIdx.x; i < per; i += blockDim.x) a += partials[2 * ((size_t)v * per + i)];
  const double tot = block_sum(a, red);
  if (threadIdx.x == 0) out[v] = tot;
}

__global__ void increment_kernel(int *ctr) {
  if (threadIdx.x == 0) *ctr += 1;
}

// beta_k = (t_k - 1) / t_{k+1}, t_1 = 1, t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2;
// entries first .. first + count - 1 go to beta[0 ..)
__global__ void beta_table_kernel(double *beta, int first, int count) {
  if (threadIdx.x != 0) return;
  double t = 1.0;
  for (int k = 0; k < first + count; ++k) {
    const double tn = (1.0 + sqrt(1.0 + 4.0 * t * t)) / 2.0;
    if (k >= first) beta[k - first] = (t - 1.0) / tn;
    t = tn;
  }
}

__global__ void pack_report_kernel(const double *__restrict__ scal, const double *__restrict__ hist, int kept,
                                   const double *__restrict__ g0sq, double *__restrict__ out) {
  if (threadIdx.x != 0) return;
  for (int j = 0; j < 4; ++j) out[j] = scal[j];
  const size_t last = kept > 0 ? 2 * (size_t)(kept - 1) : 0;
  out[4] = kept > 0 ? hist[0] : 0.0;
  out[5] = kept > 0 ? hist[1] : 0.0;
  out[6] = kept > 0 ? hist[last] : 0.0;
  out[7] = kept > 0 ? hist[last + 1] : 0.0;
  out[8] = g0sq[0];
}

__global__ void fill_int_kernel(int *p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void fill_zero_kernel(uint4 *__restrict__ p, size_t n16, unsigned char *tail, size_t ntail) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n16) p[i] = make_uint4(0, 0, 0, 0);
  if (i < ntail) tail[i] = 0;
}

template <typename T>
__global__ void fill_value_kernel(T *__restrict__ p, size_t n, T v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_reduce_rows(const double *partials, int nrows, int stride, int count,
                              double *sums, hipStream_t st) {
  hipLaunchKernelGGL(reduce_rows_kernel, dim3(1), dim3(256), 0, st, partials, nrows, stride, count,
                     sums);
  return hipGetLastError();
}

hipError_t launch_history(const double *partials, int iters, int nvol, int nblk_t, int nblk_z,
                          size_t stride, double tau, const double *g0sq, double *hist, hipStream_t st) {
  if (iters <= 0) return hipSuccess;
  hipLaunchKernelGGL(history_kernel, dim3((unsigned)iters, (unsigned)nvol), dim3(256), 0, st, partials,
                     nvol, nblk_t, nblk_z, stride, tau, g0sq, hist);
  return hipGetLastError();
}

hipError_t launch_freeze(const double *partials, size_t stride, const int *ctr, int nvol, int nblk_t, int nblk_z,
                         double tau, double *g0sq, const double *g0_part, double rel_tol, int *active, int *conv,
                         hipStream_t st) {
  hipLaunchKernelGGL(freeze_kernel, dim3((unsigned)nvol), dim3(256), 0, st, partials, stride, ctr, nvol, nblk_t,
                     nblk_z, tau, g0sq, g0_part, rel_tol, active, conv);
  return hipGetLastError();
}

hipError_t launch_pack_report(const double *scal, const double *hist, int kept, const double *g0sq, double *out,
                              hipStream_t st) {
  hipLaunchKernelGGL(pack_report_kernel, dim3(1), dim3(64), 0, st, scal, hist, kept, g0sq, out);
  return hipGetLastError();
}

hipError_t launch_reduce_volumes(const double *partials, int nblk, int nvol, double *out, hipStream_t st) {
  hipLaunchKernelGGL(reduce_volumes_kernel, dim3((unsigned)nvol), dim3(256), 0, st, partials, nblk, nvol, out);
  return hipGetLastError();
}

hipError_t launch_increment(int *ctr, hipStream_t st) {
  hipLaunchKernelGGL(increment_kernel, dim3(1), dim3(64), 0, st, ctr);
  return hipGetLastError();
}

hipError_t launch_beta_table(double *beta, int first, int count, hipStream_t st) {
  hipLaunchKernelGGL(beta_table_kernel, dim3(1), dim3(64), 0, st, beta, first, count);
  return hipGetLastError();
}

hipError_t launch_fill_int(int *p, int n, int v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st) {
  // p is 16-byte aligned by construction of every workspace region
  const size_t n16 = bytes / 16;
  const size_t ntail = bytes % 16;
  unsigned char *tail = reinterpret_cast<unsigned char *>(p) + n16 * 16;
  const size_t n = n16 > ntail ? n16 : ntail;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     reinterpret_cast<uint4 *>(p), n16, tail, ntail);
  return hipGetLastError();
}

hipError_t launch_fill_value(float *p, size_t n, float v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_value_kernel<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_value_f64(double *p, size_t n, double v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_value_kernel<double>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     st, p, n, v);
  return hipGetLastError();
}

}  // namespace ctof
