// Counter-based random numbers and Poisson photon counts (gfx950).
//
// Training data for the learned warm start are histograms of the forward
// model scaled to a peak count with Poisson counting noise (the detector
// model of the paper's section on multiplexed measurements).  Every element
// draws from its own counter, so results do not depend on the launch shape:
//   Philox-4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011), key = (seed lo,
//   seed hi), counter = (i lo, i hi, stream, trial);
//   u = ((w_hi >> 5) 2^26 + (w_lo >> 6)) 2^-53 in [0, 1);
//   Poisson(lam): for lam < 10 the smallest k with u <= F(k), F accumulated
//   from p_k = p_{k-1} lam / k (at most 1000 steps); for lam >= 10 the
//   transformed rejection method with squeeze (Hoermann 1993), one Philox
//   block per trial, at most 1024 trials (then the rounded mean).
// All decisions are taken in FP64 with contraction disabled, so the samples
// follow the scalar definition term by term.
#include <cstdint>

#include "ctof_internal.h"

namespace ctof {

namespace {

struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
    const uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

__device__ __forceinline__ U4 draw(uint64_t seed, long long i, uint32_t stream, uint32_t trial) {
  const uint64_t u = (uint64_t)i;
  return philox4x32_10(U4{(uint32_t)u, (uint32_t)(u >> 32), stream, trial}, (uint32_t)seed,
                       (uint32_t)(seed >> 32));
}

__device__ double uniform53(uint32_t hi, uint32_t lo) {
#pragma clang fp contract(off)
  return ((double)(hi >> 5) * 67108864.0 + (double)(lo >> 6)) * (1.0 / 9007199254740992.0);
}

__device__ double poisson_one(double lam, uint64_t seed, long long i, uint32_t stream) {
#pragma clang fp contract(off)
  if (!(lam > 0.0)) return 0.0;
  if (lam < 10.0) {
    const U4 w = draw(seed, i, stream, 0);
    const double u = uniform53(w.x, w.y);
    double p = exp(-lam), F = p;
    int k = 0;
    while (u > F && k < 1000) {
      ++k;
      p = p * lam / (double)k;
      F = F + p;
    }
    return (double)k;
  }
  const double smu = sqrt(lam);
  const double b = 0.931 + 2.53 * smu;
  const double a = -0.059 + 0.02483 * b;
  const double inv_alpha = 1.1239 + 1.1328 / (b - 3.4);
  const double vr = 0.9277 - 3.6224 / (b - 2.0);
  const double log_lam = log(lam);
  for (uint32_t trial = 0; trial < 1024; ++trial) {
    const U4 w = draw(seed, i, stream, trial);
    const double U = uniform53(w.x, w.y) - 0.5;
    const double V = uniform53(w.z, w.w);
    const double us = 0.5 - fabs(U);
    const double kf = floor((2.0 * a / us + b) * U + lam + 0.43);
    if (us >= 0.07 && V <= vr) return kf;
    if (kf < 0.0 || (us < 0.013 && V > us)) continue;
    const double lhs = log(V * inv_alpha / (a / (us * us) + b));
    const double rhs = -lam + kf * log_lam - lgamma(kf + 1.0);
    if (lhs <= rhs) return kf;
  }
  return floor(lam + 0.5);
}

__global__ void philox_kernel(uint64_t seed, uint32_t stream, long long first, long long n,
                              uint32_t *__restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const U4 w = draw(seed, first + i, stream, 0);
  uint4 *o = reinterpret_cast<uint4 *>(out);
  o[i] = make_uint4(w.x, w.y, w.z, w.w);
}

__global__ void poisson_kernel(const float *__restrict__ lam, long long n, uint64_t seed, uint32_t stream,
                               float *__restrict__ counts) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  counts[i] = (float)poisson_one((double)lam[i], seed, i, stream);
}

constexpr int kMaxBlocks = 1024;

__global__ void __launch_bounds__(256)
max_partial_kernel(const float *__restrict__ m, long long n, float *__restrict__ part) {
  __shared__ float red[256];
  float v = 0.0f;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    v = fmaxf(v, m[i]);
  red[threadIdx.x] = v;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + k]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// d = Poisson(s m) / s with s = peak / max(m); a non-positive maximum gives d = 0.
__global__ void __launch_bounds__(256)
noisy_kernel(const float *__restrict__ m, long long n, const float *__restrict__ part, int nparts, double peak,
             uint64_t seed, uint32_t stream, float *__restrict__ d) {
  __shared__ float red[256];
  float v = 0.0f;
  for (int i = threadIdx.x; i < nparts; i += 256) v = fmaxf(v, part[i]);
  red[threadIdx.x] = v;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + k]);
    __syncthreads();
  }
  const double mx = (double)red[0];
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!(mx > 0.0)) {
    d[i] = 0.0f;
    return;
  }
  const double s = peak / mx;
  const double mi = (double)m[i];
  const double lam = (mi > 0.0 ? mi : 0.0) * s;
  d[i] = (float)(poisson_one(lam, seed, i, stream) / s);
}

// out = (Poisson(scale max(m, 0) + background) - background) / scale: counts
// of a measurement with a dark-count background, offset and scaled back.
__global__ void __launch_bounds__(256)
noisy_counts_kernel(const float *m, long long n, double scale, double background, uint64_t seed,
                    uint32_t stream, float *out) {
#pragma clang fp contract(off)
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double mi = (double)m[i];
  const double lam = (mi > 0.0 ? mi : 0.0) * scale + background;
  out[i] = (float)((poisson_one(lam, seed, i, stream) - background) / scale);
}

inline unsigned blocks_for(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_philox(uint64_t seed, uint32_t stream_id, long long first, long long n, uint32_t *out,
                         hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(philox_kernel, dim3(blocks_for(n)), dim3(256), 0, st, seed, stream_id, first, n, out);
  return hipGetLastError();
}

hipError_t launch_poisson(const float *lam, long long n, uint64_t seed, uint32_t stream_id, float *counts,
                          hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(poisson_kernel, dim3(blocks_for(n)), dim3(256), 0, st, lam, n, seed, stream_id, counts);
  return hipGetLastError();
}

hipError_t launch_noisy_counts(const float *m, long long n, double scale, double background, uint64_t seed,
                               uint32_t stream_id, float *out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(noisy_counts_kernel, dim3(blocks_for(n)), dim3(256), 0, st, m, n, scale, background, seed,
                     stream_id, out);
  return hipGetLastError();
}

size_t noisy_histogram_ws_bytes(long long) { return kMaxBlocks * sizeof(float); }

hipError_t launch_noisy_histogram(const float *m, long long n, double peak, uint64_t seed, uint32_t stream_id,
                                  float *d, void *ws, hipStream_t st) {
  if (n == 0) return hipSuccess;
  float *part = reinterpret_cast<float *>(ws);
  const long long nb = (long long)blocks_for(n);
  const int nparts = (int)(nb < kMaxBlocks ? nb : kMaxBlocks);
  hipLaunchKernelGGL(max_partial_kernel, dim3((unsigned)nparts), dim3(256), 0, st, m, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(noisy_kernel, dim3(blocks_for(n)), dim3(256), 0, st, m, n, part, nparts, peak, seed,
                     stream_id, d);
  return hipGetLastError();
}

}  // namespace ctof
