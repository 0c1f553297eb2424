// Batched 2D real FFT passes for the lateral convolution (gfx950).
//
// The forward model of Eq. 11 is evaluated in the Fourier domain (section
// "Computational Complexity Analysis": convolution by FFT).  Each 2D
// transform on the P x P torus is split into passes that touch HBM once:
//
//   column pass  complex DFT of length P along kx for every ky column,
//                for a block of BB planes at once (planes are the fastest
//                index of every spectrum, so a block load is BB contiguous
//                values per row);
//   row pass     per scan row i: inverse real DFT along ky (c2r) of the
//                column-pass output, crop to n samples, a pointwise step
//                (residual, prox update, store, ...), zero-pad, forward
//                real DFT (r2c), again for BB planes at once.
//
// Spectra are laid out [ky][row][re/im][plane] with ky in [0, P/2].  All
// transforms are unnormalised; the 1/P^2 of the inverse is folded into the
// packed kernel spectrum.  A length-R DFT (R <= 16) runs in registers
// (radix-2, fully unrolled); a length-P pass is two such stages through
// LDS with a twiddle table built per block in double precision.  Real DFTs
// of length P use one complex DFT of length P/2 plus the standard
// even/odd split.
#include "ctof_internal.h"

namespace ctof {

namespace {

__host__ __device__ constexpr double cos16(int k) {
  // cos(2 pi k / 16)
  return k == 0 ? 1.0 : k == 1 ? 0.92387953251128675613 : k == 2 ? 0.70710678118654752440
       : k == 3 ? 0.38268343236508977173 : k == 4 ? 0.0 : k == 5 ? -0.38268343236508977173
       : k == 6 ? -0.70710678118654752440 : k == 7 ? -0.92387953251128675613 : -1.0;
}
__host__ __device__ constexpr double sin16(int k) {
  // sin(2 pi k / 16), k in [0, 8)
  return k == 0 ? 0.0 : k == 1 ? 0.38268343236508977173 : k == 2 ? 0.70710678118654752440
       : k == 3 ? 0.92387953251128675613 : k == 4 ? 1.0 : k == 5 ? 0.92387953251128675613
       : k == 6 ? 0.70710678118654752440 : 0.38268343236508977173;
}

template <int R>
__host__ __device__ constexpr int bitrev(int i) {
  int r = 0;
  for (int b = 1, q = R >> 1; b < R; b <<= 1, q >>= 1)
    if (i & b) r |= q;
  return r;
}

// In-register DFT of length R (power of two <= 16):
//   X[k] = sum_n x[n] exp(DIR * 2 pi i n k / R)   (DIR = -1 forward, +1 inverse)
template <typename T, int R, int DIR>
__device__ __forceinline__ void dft_reg(T (&xr)[R], T (&xi)[R]) {
  T tr[R], ti[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    tr[bitrev<R>(i)] = xr[i];
    ti[bitrev<R>(i)] = xi[i];
  }
#pragma unroll
  for (int len = 2; len <= R; len <<= 1) {
#pragma unroll
    for (int s = 0; s < R; s += len) {
#pragma unroll
      for (int j = 0; j < len / 2; ++j) {
        const int idx = j * (16 / len);
        const int a = s + j, b = s + j + len / 2;
        T vr, vi;
        if (idx == 0) {
          vr = tr[b];
          vi = ti[b];
        } else if (idx == 4) {  // multiply by DIR * i
          vr = (T)(-DIR) * ti[b];
          vi = (T)DIR * tr[b];
        } else {
          const T wr = (T)cos16(idx);
          const T wi = (T)(DIR * sin16(idx));
          vr = tr[b] * wr - ti[b] * wi;
          vi = tr[b] * wi + ti[b] * wr;
        }
        const T ur = tr[a], ui = ti[a];
        tr[a] = ur + vr;
        ti[a] = ui + vi;
        tr[b] = ur - vr;
        ti[b] = ui - vi;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < R; ++i) {
    xr[i] = tr[i];
    xi[i] = ti[i];
  }
}

// twc[m] = cos(2 pi m / P), tws[m] = sin(2 pi m / P), m < P.
template <typename T, int P>
__device__ __forceinline__ void build_twiddles(T *twc, T *tws) {
  for (int m = threadIdx.x; m < P; m += blockDim.x) {
    double s, c;
    sincospi(2.0 * (double)m / (double)P, &s, &c);
    twc[m] = (T)c;
    tws[m] = (T)s;
  }
}

// Stage 1 of a length-L = R1*R2 DFT along rows of (br, bi)[row*ld + b] for
// BB columns: for each (n2, b), DFT_R1 over rows R2*n1 + n2, multiply by
// W_L^(n2 k1), write back in place.  `tstep` maps W_L^m onto the P-table.
template <typename T, int R1, int R2, int BB, int DIR>
__device__ __forceinline__ void dft_stage1(T *br, T *bi, int ld, const T *twc, const T *tws,
                                           int tstep, int tmask) {
  for (int u = threadIdx.x; u < R2 * BB; u += blockDim.x) {
    const int b = u % BB, n2 = u / BB;
    T xr[R1], xi[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) {
      xr[n1] = br[(R2 * n1 + n2) * ld + b];
      xi[n1] = bi[(R2 * n1 + n2) * ld + b];
    }
    dft_reg<T, R1, DIR>(xr, xi);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      T yr = xr[k1], yi = xi[k1];
      if (k1 != 0) {
        const int m = (n2 * k1 * tstep) & tmask;
        const T c = twc[m], s = (T)DIR * tws[m];
        const T tr = yr * c - yi * s;
        yi = yr * s + yi * c;
        yr = tr;
      }
      br[(R2 * k1 + n2) * ld + b] = yr;
      bi[(R2 * k1 + n2) * ld + b] = yi;
    }
  }
}

// Stage 2 for one unit (k1, b): DFT_R2 over rows R2*k1 + n2; output index
// k1 + R1*k2 holds (zr[k2], zi[k2]).
template <typename T, int R1, int R2, int DIR>
__device__ __forceinline__ void dft_stage2_unit(const T *br, const T *bi, int ld, int k1, int b,
                                                T (&zr)[R2], T (&zi)[R2]) {
#pragma unroll
  for (int n2 = 0; n2 < R2; ++n2) {
    zr[n2] = br[(R2 * k1 + n2) * ld + b];
    zi[n2] = bi[(R2 * k1 + n2) * ld + b];
  }
  dft_reg<T, R2, DIR>(zr, zi);
}

template <int P>
struct Fac {
  static constexpr int R1 = P == 256 ? 16 : P == 128 ? 16 : P == 64 ? 8 : P == 32 ? 8 : P == 16 ? 4 : P == 8 ? 4 : 2;
  static constexpr int R2 = P / R1;
};

// ---- column pass ---------------------------------------------------------------
template <typename T, int P, int BB, bool INV>
__global__ void __launch_bounds__(256)
col_pass_kernel(int n, int B, const T *__restrict__ in, T *__restrict__ out) {
  constexpr int R1 = Fac<P>::R1, R2 = Fac<P>::R2;
  constexpr int DIR = INV ? 1 : -1;
  constexpr int ld = BB + 1;
  extern __shared__ unsigned char smem_raw[];
  T *br = reinterpret_cast<T *>(smem_raw);
  T *bi = br + P * ld;
  T *twc = bi + P * ld;
  T *tws = twc + P;
  const int ky = blockIdx.x;
  const int b0 = blockIdx.y * BB;
  const int rows_in = INV ? P : n;
  const int rows_out = INV ? n : P;
  build_twiddles<T, P>(twc, tws);
  const T *src = in + (size_t)ky * rows_in * 2 * B + b0;
  for (int e = threadIdx.x; e < P * 2 * BB; e += blockDim.x) {
    const int b = e % BB;
    const int r = e / BB;
    const int row = r >> 1, reim = r & 1;
    T v = (T)0;
    if (row < rows_in) v = src[((size_t)row * 2 + reim) * B + b];
    (reim ? bi : br)[row * ld + b] = v;
  }
  __syncthreads();
  dft_stage1<T, R1, R2, BB, DIR>(br, bi, ld, twc, tws, 1, P - 1);
  __syncthreads();
  T *dst = out + (size_t)ky * rows_out * 2 * B + b0;
  for (int u = threadIdx.x; u < R1 * BB; u += blockDim.x) {
    const int b = u % BB, k1 = u / BB;
    T zr[R2], zi[R2];
    dft_stage2_unit<T, R1, R2, DIR>(br, bi, ld, k1, b, zr, zi);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) {
      const int row = k1 + R1 * k2;
      if (row < rows_out) {
        dst[((size_t)row * 2) * B + b] = zr[k2];
        dst[((size_t)row * 2 + 1) * B + b] = zi[k2];
      }
    }
  }
}

// ---- row pass --------------------------------------------------------------------
template <typename T, int P, int BB>
__global__ void __launch_bounds__(256)
row_pass_kernel(int n, RowArgs a) {
  constexpr int H = P / 2;
  constexpr int R1 = Fac<H>::R1, R2 = Fac<H>::R2;
  constexpr int ld = BB + 1;
  extern __shared__ unsigned char smem_raw[];
  T *xr = reinterpret_cast<T *>(smem_raw);
  T *xi = xr + (H + 1) * ld;
  T *wr = xi + (H + 1) * ld;
  T *wi = wr + H * ld;
  T *twc = wi + H * ld;
  T *tws = twc + P;
  double *red = reinterpret_cast<double *>(tws + P + (P & 1));

  const int op = a.op;
  const int i = blockIdx.x;
  const int b0 = blockIdx.y * BB;
  const int B = a.B;
  const bool spec_in = (op != ROW_SPATIAL_TO_SPEC) && (op != ROW_SCALE_TO_SPEC);
  const bool spec_out = (op == ROW_SPATIAL_TO_SPEC) || (op == ROW_SCALE_TO_SPEC) ||
                        (op == ROW_RESIDUAL) || (op == ROW_PASS) || (op == ROW_FISTA);
  const int nh = (n + 1) / 2;
  build_twiddles<T, P>(twc, tws);

  if (spec_in) {
    const T *src = reinterpret_cast<const T *>(a.spec_in) + b0;
    for (int e = threadIdx.x; e < (H + 1) * 2 * BB; e += blockDim.x) {
      const int b = e % BB;
      const int r = e / BB;
      const int ky = r >> 1, reim = r & 1;
      const T v = src[(((size_t)ky * n + i) * 2 + reim) * B + b];
      (reim ? xi : xr)[ky * ld + b] = v;
    }
    __syncthreads();
    // Z[k] = A[k] + i B[k], A = X[k] + conj(X[H-k]), B = (X[k] - conj(X[H-k])) e^{+2 pi i k/P}
    for (int u = threadIdx.x; u < H * BB; u += blockDim.x) {
      const int b = u % BB, k = u / BB;
      const T x1r = xr[k * ld + b], x1i = xi[k * ld + b];
      const T x2r = xr[(H - k) * ld + b], x2i = -xi[(H - k) * ld + b];
      const T ar = x1r + x2r, ai = x1i + x2i;
      const T dr = x1r - x2r, di = x1i - x2i;
      const T c = twc[k], s = tws[k];
      const T br_ = dr * c - di * s, bi_ = dr * s + di * c;
      wr[k * ld + b] = ar - bi_;
      wi[k * ld + b] = ai + br_;
    }
    __syncthreads();
    dft_stage1<T, R1, R2, BB, 1>(wr, wi, ld, twc, tws, 2, P - 1);
    __syncthreads();
    for (int u = threadIdx.x; u < R1 * BB; u += blockDim.x) {
      const int b = u % BB, k1 = u / BB;
      T zr[R2], zi[R2];
      dft_stage2_unit<T, R1, R2, 1>(wr, wi, ld, k1, b, zr, zi);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) {
        const int m = k1 + R1 * k2;
        xr[m * ld + b] = zr[k2];
        xi[m * ld + b] = zi[k2];
      }
    }
    __syncthreads();
  }

  // pointwise step on the cropped real row x[j], j < n
  double acc0 = 0.0, acc1 = 0.0;
  const T tau = (T)a.tau, lam = (T)a.lambda, beta = (T)a.beta;
  T scale = (T)1;
  if (op == ROW_SCALE_TO_SPEC) scale = (T)(1.0 / sqrt(*a.scalar));
  const T *sp_in = reinterpret_cast<const T *>(a.sp_in);
  T *sp_out = reinterpret_cast<T *>(a.sp_out);
  T *sp_aux = reinterpret_cast<T *>(a.sp_aux);
  for (int u = threadIdx.x; u < n * BB; u += blockDim.x) {
    const int j = u % n, b = u / n;
    const int pl = b0 + b;
    const bool valid = pl < a.nplanes;
    const size_t idx = ((size_t)pl * n + i) * n + j;
    T x = (T)0;
    if (spec_in) x = (j & 1) ? xi[(j >> 1) * ld + b] : xr[(j >> 1) * ld + b];
    T r = (T)0;
    switch (op) {
      case ROW_SPEC_TO_SPATIAL:
        if (valid) sp_out[idx] = x;
        break;
      case ROW_SPATIAL_TO_SPEC:
        r = valid ? sp_in[idx] : (T)0;
        break;
      case ROW_SCALE_TO_SPEC:
        if (valid) {
          r = sp_in[idx] * scale;
          sp_out[idx] = r;
        }
        break;
      case ROW_RESIDUAL:
        if (valid) {
          r = x - sp_in[idx];
          acc0 += 0.5 * (double)r * (double)r;
        }
        break;
      case ROW_PASS:
        if (valid) {
          r = x;
          acc0 += 0.5 * (double)x * (double)x;
        }
        break;
      case ROW_FISTA:
        if (valid) {
          const T yk = sp_in[idx];
          const T mprev = sp_aux[idx];
          T mu = yk - tau * (x + lam * yk);
          mu = mu > (T)0 ? mu : (T)0;
          const T ynew = mu + beta * (mu - mprev);
          sp_aux[idx] = mu;
          sp_out[idx] = ynew;
          const double dd = (double)yk - (double)mu;
          acc0 += dd * dd;
          r = ynew;
        }
        break;
      case ROW_POWER_W:
        if (valid) {
          sp_out[idx] = x;
          acc0 += (double)x * (double)x;
          acc1 += (double)sp_in[idx] * (double)x;
        }
        break;
      case ROW_GMAP0:
        if (valid) {
          const double g = x > (T)0 ? (double)x : 0.0;
          acc0 += g * g;
        }
        break;
      default:
        break;
    }
    if (spec_out) {
      if (j & 1)
        wi[(j >> 1) * ld + b] = r;
      else
        wr[(j >> 1) * ld + b] = r;
    }
  }
  if (spec_out) {
    // zero the padded part of the half-length sequence
    for (int u = threadIdx.x; u < H * BB; u += blockDim.x) {
      const int b = u % BB, m = u / BB;
      if (m >= nh) {
        wr[m * ld + b] = (T)0;
        wi[m * ld + b] = (T)0;
      } else if ((n & 1) && m == nh - 1) {
        wi[m * ld + b] = (T)0;
      }
    }
  }
  if (a.partials) {
    red[threadIdx.x] = acc0;
    red[blockDim.x + threadIdx.x] = acc1;
  }
  __syncthreads();
  if (a.partials) {
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) {
        red[threadIdx.x] += red[threadIdx.x + s];
        red[blockDim.x + threadIdx.x] += red[blockDim.x + threadIdx.x + s];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const size_t blk = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
      a.partials[2 * blk] = red[0];
      a.partials[2 * blk + 1] = red[blockDim.x];
    }
  }
  if (!spec_out) return;

  // r2c: Z' = DFT_H(r_even + i r_odd); X'[k] = Ev[k] + e^{-2 pi i k/P} Od[k]
  dft_stage1<T, R1, R2, BB, -1>(wr, wi, ld, twc, tws, 2, P - 1);
  __syncthreads();
  for (int u = threadIdx.x; u < R1 * BB; u += blockDim.x) {
    const int b = u % BB, k1 = u / BB;
    T zr[R2], zi[R2];
    dft_stage2_unit<T, R1, R2, -1>(wr, wi, ld, k1, b, zr, zi);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) {
      const int m = k1 + R1 * k2;
      xr[m * ld + b] = zr[k2];
      xi[m * ld + b] = zi[k2];
    }
  }
  __syncthreads();
  T *dst = reinterpret_cast<T *>(a.spec_out) + b0;
  for (int u = threadIdx.x; u < (H + 1) * BB; u += blockDim.x) {
    const int b = u % BB, k = u / BB;
    const int k1 = (k == H) ? 0 : k;
    const int k2 = (k == 0) ? 0 : H - k;
    const T z1r = xr[k1 * ld + b], z1i = xi[k1 * ld + b];
    const T z2r = xr[k2 * ld + b], z2i = -xi[k2 * ld + b];
    const T evr = (T)0.5 * (z1r + z2r), evi = (T)0.5 * (z1i + z2i);
    // Od = (Z1 - conj(Z2)) / (2 i)
    const T dr = z1r - z2r, di = z1i - z2i;
    const T odr = (T)0.5 * di, odi = (T)(-0.5) * dr;
    const T c = twc[k], s = -tws[k];
    const T outr = evr + odr * c - odi * s;
    const T outi = evi + odr * s + odi * c;
    dst[(((size_t)k * n + i) * 2) * B + b] = outr;
    dst[(((size_t)k * n + i) * 2 + 1) * B + b] = outi;
  }
}

template <typename T>
constexpr int pick_bb(int B) {
  return sizeof(T) == 8 ? 16 : ((B % 32) == 0 ? 32 : 16);
}

template <typename T, int P, int BB>
hipError_t col_dispatch_bb(const Dims &d, int B, bool inverse, const T *in, T *out,
                           hipStream_t st) {
  const size_t shm = (size_t)(2 * P * (BB + 1) + 2 * P) * sizeof(T);
  dim3 grid((unsigned)(d.h + 1), (unsigned)(B / BB));
  if (inverse)
    hipLaunchKernelGGL((col_pass_kernel<T, P, BB, true>), grid, dim3(256), shm, st, d.n, B, in, out);
  else
    hipLaunchKernelGGL((col_pass_kernel<T, P, BB, false>), grid, dim3(256), shm, st, d.n, B, in, out);
  return hipGetLastError();
}

template <typename T, int P>
hipError_t col_dispatch(const Dims &d, int B, bool inverse, const T *in, T *out, hipStream_t st) {
  if (pick_bb<T>(B) == 32) return col_dispatch_bb<T, P, 32>(d, B, inverse, in, out, st);
  return col_dispatch_bb<T, P, 16>(d, B, inverse, in, out, st);
}

template <typename T, int P, int BB>
hipError_t row_dispatch_bb(const Dims &d, const RowArgs &a, hipStream_t st) {
  constexpr int H = P / 2;
  const size_t shm = (size_t)((2 * (H + 1) + 2 * H) * (BB + 1) + 2 * P + 1) * sizeof(T) +
                     2 * 256 * sizeof(double) + 16;
  dim3 grid((unsigned)d.n, (unsigned)(a.B / BB));
  hipLaunchKernelGGL((row_pass_kernel<T, P, BB>), grid, dim3(256), shm, st, d.n, a);
  return hipGetLastError();
}

template <typename T, int P>
hipError_t row_dispatch(const Dims &d, const RowArgs &a, hipStream_t st) {
  if (pick_bb<T>(a.B) == 32) return row_dispatch_bb<T, P, 32>(d, a, st);
  return row_dispatch_bb<T, P, 16>(d, a, st);
}

}  // namespace

template <typename T>
hipError_t launch_col_pass(const Dims &d, int B, bool inverse, const T *in, T *out,
                           hipStream_t st) {
  switch (d.p) {
    case 16: return col_dispatch<T, 16>(d, B, inverse, in, out, st);
    case 32: return col_dispatch<T, 32>(d, B, inverse, in, out, st);
    case 64: return col_dispatch<T, 64>(d, B, inverse, in, out, st);
    case 128: return col_dispatch<T, 128>(d, B, inverse, in, out, st);
    case 256: return col_dispatch<T, 256>(d, B, inverse, in, out, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_row_pass(const Dims &d, const RowArgs &a, hipStream_t st) {
  switch (d.p) {
    case 16: return row_dispatch<T, 16>(d, a, st);
    case 32: return row_dispatch<T, 32>(d, a, st);
    case 64: return row_dispatch<T, 64>(d, a, st);
    case 128: return row_dispatch<T, 128>(d, a, st);
    case 256: return row_dispatch<T, 256>(d, a, st);
    default: return hipErrorInvalidValue;
  }
}

int row_pass_blocks(const Dims &d, int B, bool fp64) {
  const int bb = fp64 ? 16 : ((B % 32) == 0 ? 32 : 16);
  return d.n * (B / bb);
}

template hipError_t launch_col_pass<float>(const Dims &, int, bool, const float *, float *, hipStream_t);
template hipError_t launch_col_pass<double>(const Dims &, int, bool, const double *, double *, hipStream_t);
template hipError_t launch_row_pass<float>(const Dims &, const RowArgs &, hipStream_t);
template hipError_t launch_row_pass<double>(const Dims &, const RowArgs &, hipStream_t);

}  // namespace ctof
