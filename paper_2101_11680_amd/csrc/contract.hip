// Per-frequency contraction with the real kernel spectrum on the matrix
// cores (gfx950).
//
// In the Fourier domain Eq. 11 becomes, for every lateral frequency f,
//   m^(f)[t] = sum_z Khat_z(f)[t] mu^_z(f)        (forward)
// and the adjoint (section "Faster forward models": the transpose of the
// operator) is
//   g^_z(f) = sum_t Khat_z(f)[t] r^(f)[t].
// Khat is real and even in kx and ky, and symmetric under kx <-> ky on the
// square grid, so one real Nt x Nz matrix K_s with s = (a, b), a <= b <= P/2
// serves up to four rfft frequencies (kx, ky) = (a, b), (P-a, b), (b, a),
// (P-b, a).  Their real and imaginary parts are 8 real columns, so each
// matrix is one small dense GEMM:
//   forward  [Nt x Nz] x [Nz x 8],  adjoint  [Nz x Nt] x [Nt x 8].
// One workgroup streams one matrix (read once per pass: the kernel spectrum
// is the dominant HBM traffic of an iteration).  MFMA 16x16x4 (FP32, FP64)
// or 16x16x32 (BF16) tiles: the matrix occupies the A operand, the 8 columns
// the first 8 of the 16 B columns.  The reduction dimension is assigned so
// that every lane reads a contiguous run of the matrix row (vector loads):
// in k-step kk, lane group g = lane/16 carries index g * KC + kk.
//
// Layouts (element type by precision):
//   khat fwd / adj   per matrix, fragment order (see Frag): each 16-byte
//                    vector load reads one contiguous 1 KB run per wave,
//                    streamed with non-temporal loads (read once per pass)
//   mu side    [ky][kx][re/im][nzp]  t side [ky][kx][re/im][ntp]
#include "ctof_internal.h"

namespace ctof {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ inline void matrix_ab(int s, int &a, int &b) {
  int bb = (int)((sqrt(8.0 * (double)s + 1.0) - 1.0) * 0.5);
  while ((bb + 1) * (bb + 2) / 2 <= s) ++bb;
  while (bb * (bb + 1) / 2 > s) --bb;
  b = bb;
  a = s - bb * (bb + 1) / 2;
}

// Frequency index and validity of slot q (0..3) of matrix s = (a, b):
// (kx, ky) = (a, b), (P-a, b), (b, a), (P-b, a); duplicates are invalid.
// Selected with conditionals so the lane's slot never indexes a local array
// (which would live in scratch memory).
__device__ inline int matrix_slot(int s, int h, int p, int q, bool &valid) {
  int a, b;
  matrix_ab(s, a, b);
  const int lo = (q < 2) ? a : b;   // kx before reflection
  const int ky = (q < 2) ? b : a;
  const bool refl = (q & 1) != 0;
  const int kx = refl ? p - lo : lo;
  valid = (q == 0) || (q == 1 && a > 0 && a < h) || (q == 2 && a != b) ||
          (q == 3 && a != b && b > 0 && b < h);
  return ky * p + kx;
}

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef v4f acc_t;
  // output item r of lane group g is row 4g + r
  __device__ static int row_of(int i) { return i; }
  __device__ static acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<double> {
  typedef v4d acc_t;
  // the f64 16x16x4 result holds row 4r + g in item r of lane group g; feed
  // A-row i with matrix row 4(i%4) + i/4 so that item r is row 4g + r
  __device__ static int row_of(int i) { return 4 * (i & 3) + (i >> 2); }
  __device__ static acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef unsigned int nt_u4 __attribute__((ext_vector_type(4)));

// N contiguous elements (16-byte words) through the regular cache path
template <typename T, int N>
__device__ __forceinline__ void load_run(const T *__restrict__ p, T (&v)[N]) {
  constexpr int PER = 16 / sizeof(T);
  static_assert(N % PER == 0, "vector runs are whole 16-byte words");
#pragma unroll
  for (int q = 0; q < N / PER; ++q) {
    if constexpr (sizeof(T) == 4) {
      const float4 w = *reinterpret_cast<const float4 *>(p + q * PER);
      v[q * 4 + 0] = w.x;
      v[q * 4 + 1] = w.y;
      v[q * 4 + 2] = w.z;
      v[q * 4 + 3] = w.w;
    } else {
      const double2 w = *reinterpret_cast<const double2 *>(p + q * PER);
      v[q * 2 + 0] = w.x;
      v[q * 2 + 1] = w.y;
    }
  }
}

// N elements of one lane from a fragment block: word q sits at (q*64 + lane)
template <typename T, int N>
__device__ __forceinline__ void load_frag(const T *__restrict__ blk, int lane, T (&v)[N]) {
  constexpr int PER = 16 / sizeof(T);
  static_assert(N % PER == 0, "fragments are whole 16-byte words");
#pragma unroll
  for (int q = 0; q < N / PER; ++q) {
    const T *p = blk + ((size_t)q * 64 + lane) * PER;
    if constexpr (sizeof(T) == 4) {
      const nt_f4 w = __builtin_nontemporal_load(reinterpret_cast<const nt_f4 *>(p));
      v[q * 4 + 0] = w[0];
      v[q * 4 + 1] = w[1];
      v[q * 4 + 2] = w[2];
      v[q * 4 + 3] = w[3];
    } else {
      const nt_d2 w = __builtin_nontemporal_load(reinterpret_cast<const nt_d2 *>(p));
      v[q * 2 + 0] = w[0];
      v[q * 2 + 1] = w[1];
    }
  }
}

template <typename T>
__device__ __forceinline__ void store4(T *p, const typename Mfma<T>::acc_t &a) {
  if constexpr (sizeof(T) == 4) {
    *reinterpret_cast<float4 *>(p) = make_float4(a[0], a[1], a[2], a[3]);
  } else {
    *reinterpret_cast<double2 *>(p) = make_double2(a[0], a[1]);
    *reinterpret_cast<double2 *>(p + 2) = make_double2(a[2], a[3]);
  }
}

// ---- FP32 / FP64, forward: M = t (tiles of 16), K = z --------------------------
template <typename T, int KZ>
__global__ void __launch_bounds__(256)
contract_fwd_kernel(const T *__restrict__ khat, const T *__restrict__ vin, T *__restrict__ vout,
                    int h, int p, int nzp, int ntp) {
  using M = Mfma<T>;
  const int s = blockIdx.x;
  const int w = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  const int c = l & 15, g = l >> 4;
  const int q = (c >> 1) & 3;
  bool slot_ok;
  const int f = matrix_slot(s, h, p, q, slot_ok);
  const bool col = (c < 8) && slot_ok;
  const int nchunk = nzp / (4 * KZ);
  const T *vcol = vin + ((size_t)f * 2 + (c & 1)) * nzp;
  T *ocol = vout + ((size_t)f * 2 + (c & 1)) * ntp;
  const int ntt = ntp / 16;
  for (int ch = 0; ch < nchunk; ++ch) {
    T bv[KZ];
    if (col) {
      load_run<T, KZ>(vcol + ch * 4 * KZ + g * KZ, bv);
    } else {
#pragma unroll
      for (int kk = 0; kk < KZ; ++kk) bv[kk] = (T)0;
    }
    for (int tt = w; tt < ntp / 16; tt += 4) {
      const int t0 = tt * 16;
      T av[KZ];
      load_frag<T, KZ>(khat + (((size_t)s * ntt + tt) * nchunk + ch) * (64 * KZ), l, av);
      typename M::acc_t acc = {0, 0, 0, 0};
      if (ch > 0 && col) {
        // accumulate onto the previous z-chunk's partial result
        const T *o = ocol + t0 + 4 * g;
        acc[0] = o[0]; acc[1] = o[1]; acc[2] = o[2]; acc[3] = o[3];
      }
#pragma unroll
      for (int kk = 0; kk < KZ; ++kk) acc = M::step(av[kk], bv[kk], acc);
      if (col) store4<T>(ocol + t0 + 4 * g, acc);
    }
  }
}

// ---- FP32 / FP64, adjoint: M = z (tiles of 16), K = t (chunks of 16) -----------
template <typename T, int ZT>
__global__ void __launch_bounds__(256)
contract_adj_kernel(const T *__restrict__ khat, const T *__restrict__ vin, T *__restrict__ vout,
                    int h, int p, int nzp, int ntp) {
  using M = Mfma<T>;
  extern __shared__ unsigned char smem_raw[];
  T *red = reinterpret_cast<T *>(smem_raw);  // [4 waves][ZT][64 lanes][4]
  const int s = blockIdx.x;
  const int w = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  const int c = l & 15, g = l >> 4;
  const int q = (c >> 1) & 3;
  bool slot_ok;
  const int f = matrix_slot(s, h, p, q, slot_ok);
  const bool col = (c < 8) && slot_ok;
  const T *vcol = vin + ((size_t)f * 2 + (c & 1)) * ntp;
  typename M::acc_t acc[ZT];
#pragma unroll
  for (int zt = 0; zt < ZT; ++zt) acc[zt] = {0, 0, 0, 0};
  for (int ch = w; ch < ntp / 16; ch += 4) {
    const int t0 = ch * 16 + 4 * g;
    T bv[4];
    if (col) {
      load_run<T, 4>(vcol + t0, bv);
    } else {
      bv[0] = bv[1] = bv[2] = bv[3] = (T)0;
    }
#pragma unroll
    for (int zt = 0; zt < ZT; ++zt) {
      T av[4];
      load_frag<T, 4>(khat + (((size_t)s * (ntp / 16) + ch) * ZT + zt) * 256, l, av);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) acc[zt] = M::step(av[kk], bv[kk], acc[zt]);
    }
  }
  // sum the four waves' partial products (fixed order); output rows 4g..4g+3
  // of every tile sit in lane group g, so all 64 lanes take part
#pragma unroll
  for (int zt = 0; zt < ZT; ++zt)
#pragma unroll
    for (int r = 0; r < 4; ++r) red[((w * ZT + zt) * 64 + l) * 4 + r] = acc[zt][r];
  __syncthreads();
  if (w == 0 && col) {
    T *ocol = vout + ((size_t)f * 2 + (c & 1)) * nzp;
#pragma unroll
    for (int zt = 0; zt < ZT; ++zt) {
      typename M::acc_t o;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        T v = red[((0 * ZT + zt) * 64 + l) * 4 + r];
        v += red[((1 * ZT + zt) * 64 + l) * 4 + r];
        v += red[((2 * ZT + zt) * 64 + l) * 4 + r];
        v += red[((3 * ZT + zt) * 64 + l) * 4 + r];
        o[r] = v;
      }
      store4<T>(ocol + zt * 16 + 4 * g, o);
    }
  }
}

// ---- BF16 split forms -----------------------------------------------------------
// KIND 2: K_hi v_hi + K_hi v_lo + K_lo v_hi;  KIND 3 (hi-only K): K_hi v_hi + K_hi v_lo.
__device__ inline void split_bf16(float v, __bf16 &hi, __bf16 &lo) {
  hi = (__bf16)v;
  lo = (__bf16)(v - (float)hi);
}

__device__ __forceinline__ v8bf load_bf8(const __bf16 *p) {
  const nt_u4 u = __builtin_nontemporal_load(reinterpret_cast<const nt_u4 *>(p));
  v8bf r;
  __builtin_memcpy(&r, &u, 16);
  return r;
}

template <int KIND, int KZ>  // KZ: z per lane group per chunk (multiple of 8)
__global__ void __launch_bounds__(256)
contract_fwd_bf16_kernel(const __bf16 *__restrict__ khi, const __bf16 *__restrict__ klo,
                         const float *__restrict__ vin, float *__restrict__ vout, int h, int p,
                         int nzp, int ntp) {
  const int s = blockIdx.x;
  const int w = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  const int c = l & 15, g = l >> 4;
  const int q = (c >> 1) & 3;
  bool slot_ok;
  const int f = matrix_slot(s, h, p, q, slot_ok);
  const bool col = (c < 8) && slot_ok;
  const int nchunk = nzp / (4 * KZ);
  const float *vcol = vin + ((size_t)f * 2 + (c & 1)) * nzp;
  float *ocol = vout + ((size_t)f * 2 + (c & 1)) * ntp;
  const int ntt = ntp / 16;
  for (int ch = 0; ch < nchunk; ++ch) {
    v8bf bh[KZ / 8], bl[KZ / 8];
#pragma unroll
    for (int e = 0; e < KZ / 8; ++e) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const float v = col ? vcol[ch * 4 * KZ + g * KZ + e * 8 + u] : 0.0f;
        __bf16 hi, lo;
        split_bf16(v, hi, lo);
        bh[e][u] = hi;
        bl[e][u] = lo;
      }
    }
    for (int tt = w; tt < ntp / 16; tt += 4) {
      const int t0 = tt * 16;
      const size_t blk = (((size_t)s * ntt + tt) * nchunk + ch) * (64 * KZ);
      v4f acc = {0, 0, 0, 0};
      if (ch > 0 && col) {
        const float *o = ocol + t0 + 4 * g;
        acc[0] = o[0]; acc[1] = o[1]; acc[2] = o[2]; acc[3] = o[3];
      }
#pragma unroll
      for (int e = 0; e < KZ / 8; ++e) {
        const size_t off = blk + ((size_t)e * 64 + l) * 8;
        const v8bf ah = load_bf8(khi + off);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[e], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[e], acc, 0, 0, 0);
        if (KIND == 2) {
          const v8bf al = load_bf8(klo + off);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[e], acc, 0, 0, 0);
        }
      }
      if (col) *reinterpret_cast<float4 *>(ocol + t0 + 4 * g) = make_float4(acc[0], acc[1], acc[2], acc[3]);
    }
  }
}

template <int KIND, int ZT>
__global__ void __launch_bounds__(256)
contract_adj_bf16_kernel(const __bf16 *__restrict__ khi, const __bf16 *__restrict__ klo,
                         const float *__restrict__ vin, float *__restrict__ vout, int h, int p,
                         int nzp, int ntp) {
  extern __shared__ unsigned char smem_raw[];
  float *red = reinterpret_cast<float *>(smem_raw);
  const int s = blockIdx.x;
  const int w = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  const int c = l & 15, g = l >> 4;
  const int q = (c >> 1) & 3;
  bool slot_ok;
  const int f = matrix_slot(s, h, p, q, slot_ok);
  const bool col = (c < 8) && slot_ok;
  const float *vcol = vin + ((size_t)f * 2 + (c & 1)) * ntp;
  v4f acc[ZT];
#pragma unroll
  for (int zt = 0; zt < ZT; ++zt) acc[zt] = {0, 0, 0, 0};
  for (int ch = w; ch < ntp / 32; ch += 4) {
    const int t0 = ch * 32 + 8 * g;
    v8bf bh, bl;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float v = col ? vcol[t0 + u] : 0.0f;
      __bf16 hi, lo;
      split_bf16(v, hi, lo);
      bh[u] = hi;
      bl[u] = lo;
    }
#pragma unroll
    for (int zt = 0; zt < ZT; ++zt) {
      const size_t off = (((size_t)s * (ntp / 32) + ch) * ZT + zt) * 512 + (size_t)l * 8;
      const v8bf ah = load_bf8(khi + off);
      acc[zt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[zt], 0, 0, 0);
      acc[zt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[zt], 0, 0, 0);
      if (KIND == 2) {
        const v8bf al = load_bf8(klo + off);
        acc[zt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[zt], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int zt = 0; zt < ZT; ++zt)
#pragma unroll
    for (int r = 0; r < 4; ++r) red[((w * ZT + zt) * 64 + l) * 4 + r] = acc[zt][r];
  __syncthreads();
  if (w == 0 && col) {
    float *ocol = vout + ((size_t)f * 2 + (c & 1)) * nzp;
#pragma unroll
    for (int zt = 0; zt < ZT; ++zt) {
      float o[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float v = red[((0 * ZT + zt) * 64 + l) * 4 + r];
        v += red[((1 * ZT + zt) * 64 + l) * 4 + r];
        v += red[((2 * ZT + zt) * 64 + l) * 4 + r];
        v += red[((3 * ZT + zt) * 64 + l) * 4 + r];
        o[r] = v;
      }
      *reinterpret_cast<float4 *>(ocol + zt * 16 + 4 * g) = make_float4(o[0], o[1], o[2], o[3]);
    }
  }
}

template <typename T>
hipError_t launch_plain(const ctof_kernel_s *k, bool adjoint, const void *in, void *out,
                        hipStream_t st) {
  const Dims &d = k->dims;
  const char *kh = reinterpret_cast<const char *>(k->khat);
  const T *vin = reinterpret_cast<const T *>(in);
  T *vout = reinterpret_cast<T *>(out);
  const dim3 grid((unsigned)d.nmat), block(256);
  if (!adjoint) {
    const T *K = reinterpret_cast<const T *>(kh + k->layout.fwd);
    const int kz = (d.nzp >= 64 ? 64 : d.nzp) / 4;
    switch (kz) {
      case 4: hipLaunchKernelGGL((contract_fwd_kernel<T, 4>), grid, block, 0, st, K, vin, vout, d.h, d.p, d.nzp, d.ntp); break;
      case 8: hipLaunchKernelGGL((contract_fwd_kernel<T, 8>), grid, block, 0, st, K, vin, vout, d.h, d.p, d.nzp, d.ntp); break;
      case 12: hipLaunchKernelGGL((contract_fwd_kernel<T, 12>), grid, block, 0, st, K, vin, vout, d.h, d.p, d.nzp, d.ntp); break;
      case 16: hipLaunchKernelGGL((contract_fwd_kernel<T, 16>), grid, block, 0, st, K, vin, vout, d.h, d.p, d.nzp, d.ntp); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    const T *K = reinterpret_cast<const T *>(kh + k->layout.adj);
    const int zt = d.nzp / 16;
    const size_t shm = (size_t)4 * zt * 64 * 4 * sizeof(T);
    switch (zt) {
      case 1: hipLaunchKernelGGL((contract_adj_kernel<T, 1>), grid, block, shm, st, K, vin, vout, d.h, d.p, d.nzp, d.ntp); break;
      case 2: hipLaunchKernelGGL((contract_adj_kernel<T, 2>), grid, block, shm, st, K, vin, vout, d.h, d.p, d.nzp, d.ntp); break;
      case 3: hipLaunchKernelGGL((contract_adj_kernel<T, 3>), grid, block, shm, st, K, vin, vout, d.h, d.p, d.nzp, d.ntp); break;
      case 4: hipLaunchKernelGGL((contract_adj_kernel<T, 4>), grid, block, shm, st, K, vin, vout, d.h, d.p, d.nzp, d.ntp); break;
      case 8: hipLaunchKernelGGL((contract_adj_kernel<T, 8>), grid, block, shm, st, K, vin, vout, d.h, d.p, d.nzp, d.ntp); break;
      case 12: hipLaunchKernelGGL((contract_adj_kernel<T, 12>), grid, block, shm, st, K, vin, vout, d.h, d.p, d.nzp, d.ntp); break;
      case 16: hipLaunchKernelGGL((contract_adj_kernel<T, 16>), grid, block, shm, st, K, vin, vout, d.h, d.p, d.nzp, d.ntp); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template <int KIND>
hipError_t launch_bf16(const ctof_kernel_s *k, bool adjoint, const void *in, void *out,
                       hipStream_t st) {
  const Dims &d = k->dims;
  const char *kh = reinterpret_cast<const char *>(k->khat);
  const float *vin = reinterpret_cast<const float *>(in);
  float *vout = reinterpret_cast<float *>(out);
  const dim3 grid((unsigned)d.nmat), block(256);
  if (!adjoint) {
    const __bf16 *hi = reinterpret_cast<const __bf16 *>(kh + k->layout.fwd);
    const __bf16 *lo = KIND == 2 ? reinterpret_cast<const __bf16 *>(kh + k->layout.fwd_lo) : hi;
    const int kz = (d.nzp >= 64 ? 64 : d.nzp) / 4;
    switch (kz) {
      case 8: hipLaunchKernelGGL((contract_fwd_bf16_kernel<KIND, 8>), grid, block, 0, st, hi, lo, vin, vout, d.h, d.p, d.nzp, d.ntp); break;
      case 16: hipLaunchKernelGGL((contract_fwd_bf16_kernel<KIND, 16>), grid, block, 0, st, hi, lo, vin, vout, d.h, d.p, d.nzp, d.ntp); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    const __bf16 *hi = reinterpret_cast<const __bf16 *>(kh + k->layout.adj);
    const __bf16 *lo = KIND == 2 ? reinterpret_cast<const __bf16 *>(kh + k->layout.adj_lo) : hi;
    const int zt = d.nzp / 16;
    const size_t shm = (size_t)4 * zt * 64 * 4 * sizeof(float);
    switch (zt) {
      case 2: hipLaunchKernelGGL((contract_adj_bf16_kernel<KIND, 2>), grid, block, shm, st, hi, lo, vin, vout, d.h, d.p, d.nzp, d.ntp); break;
      case 4: hipLaunchKernelGGL((contract_adj_bf16_kernel<KIND, 4>), grid, block, shm, st, hi, lo, vin, vout, d.h, d.p, d.nzp, d.ntp); break;
      case 8: hipLaunchKernelGGL((contract_adj_bf16_kernel<KIND, 8>), grid, block, shm, st, hi, lo, vin, vout, d.h, d.p, d.nzp, d.ntp); break;
      case 12: hipLaunchKernelGGL((contract_adj_bf16_kernel<KIND, 12>), grid, block, shm, st, hi, lo, vin, vout, d.h, d.p, d.nzp, d.ntp); break;
      case 16: hipLaunchKernelGGL((contract_adj_bf16_kernel<KIND, 16>), grid, block, shm, st, hi, lo, vin, vout, d.h, d.p, d.nzp, d.ntp); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_contract(const ctof_kernel_s *k, bool adjoint, const void *in, void *out,
                           hipStream_t st) {
  switch (k->prec) {
    case CTOF_FP64: return launch_plain<double>(k, adjoint, in, out, st);
    case CTOF_FP32: return launch_plain<float>(k, adjoint, in, out, st);
    case CTOF_BF16X3: return launch_bf16<2>(k, adjoint, in, out, st);
    case CTOF_BF16: return launch_bf16<3>(k, adjoint, in, out, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ctof
