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

// Per iteration k (one block each): hist[k] = (sum of t-side partial 0,
// sqrt(sum of z-side partial 0) * gscale), gscale = 1 / (tau * ||G(0)||).
__global__ void __launch_bounds__(256)
history_kernel(const double *__restrict__ partials, int nblk_t, int nblk_z, double tau,
               const double *__restrict__ g0sq, double *__restrict__ hist, double *__restrict__ last,
               int iters) {
  __shared__ double red[256];
  const int k = blockIdx.x;
  const size_t stride = 2 * (size_t)(nblk_t + nblk_z);
  const double *pt = partials + (size_t)k * stride;
  const double *pz = pt + 2 * (size_t)nblk_t;
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nblk_t; i += blockDim.x) a += pt[2 * i];
  for (int i = threadIdx.x; i < nblk_z; i += blockDim.x) b += pz[2 * i];
  const double fit = block_sum(a, red);
  const double gm = block_sum(b, red);
  if (threadIdx.x == 0) {
    const double g0 = sqrt(*g0sq);
    const double ratio = g0 > 0.0 ? sqrt(gm) / (tau * g0) : 0.0;
    hist[2 * (size_t)k] = fit;
    hist[2 * (size_t)k + 1] = ratio;
    if (k == iters - 1 && last) {
      last[0] = fit;
      last[1] = ratio;
    }
  }
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

hipError_t launch_history_k(const double *partials, int iters, int nblk_t, int nblk_z, double tau,
                            const double *g0sq, double *hist, double *last, hipStream_t st) {
  hipLaunchKernelGGL(history_kernel, dim3((unsigned)iters), dim3(256), 0, st, partials, nblk_t,
                     nblk_z, tau, g0sq, hist, last, iters);
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
