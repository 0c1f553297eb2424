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
// packed kernel spectrum.  A length-R DFT (R <= 32) runs in registers
// (radix-2, fully unrolled); a length-P pass is two such stages through
// LDS with a twiddle table built per block in double precision (P = 512:
// 16 x 32, P = 1024: 32 x 32, with the column held in LDS whole).  Real DFTs of length P use
// one complex DFT of length P/2 plus the standard even/odd split.
#include "ctof_internal.h"

namespace ctof {

namespace {

// cos(2 pi k / 32) and sin(2 pi k / 32) for k in [0, 16], written out (no
// recursion: the unrolled DFTs fold every call into a literal)
__host__ __device__ constexpr double cos32(int k) {
  return k == 0 ? 1.0 : k == 1 ? 0.98078528040323044913 : k == 2 ? 0.92387953251128675613
       : k == 3 ? 0.83146961230254523708 : k == 4 ? 0.70710678118654752440 : k == 5 ? 0.55557023301960222474
       : k == 6 ? 0.38268343236508977173 : k == 7 ? 0.19509032201612826785 : k == 8 ? 0.0
       : k == 9 ? -0.19509032201612826785 : k == 10 ? -0.38268343236508977173 : k == 11 ? -0.55557023301960222474
       : k == 12 ? -0.70710678118654752440 : k == 13 ? -0.83146961230254523708 : k == 14 ? -0.92387953251128675613
       : k == 15 ? -0.98078528040323044913 : -1.0;
}
__host__ __device__ constexpr double sin32(int k) {
  return k == 0 ? 0.0 : k == 1 ? 0.19509032201612826785 : k == 2 ? 0.38268343236508977173
       : k == 3 ? 0.55557023301960222474 : k == 4 ? 0.70710678118654752440 : k == 5 ? 0.83146961230254523708
       : k == 6 ? 0.92387953251128675613 : k == 7 ? 0.98078528040323044913 : k == 8 ? 1.0
       : k == 9 ? 0.98078528040323044913 : k == 10 ? 0.92387953251128675613 : k == 11 ? 0.83146961230254523708
       : k == 12 ? 0.70710678118654752440 : k == 13 ? 0.55557023301960222474 : k == 14 ? 0.38268343236508977173
       : k == 15 ? 0.19509032201612826785 : 0.0;
}

// cos(2 pi j / 24) and sin(2 pi j / 24) for j in [0, 24) (the twiddles of
// the radix-3 DFT lengths 3, 6, 12 and 24)
__host__ __device__ constexpr double cos24_half(int j) {  // j in [0, 12]
  return j == 0 ? 1.0 : j == 1 ? 0.96592582628906828675 : j == 2 ? 0.86602540378443864676
       : j == 3 ? 0.70710678118654752440 : j == 4 ? 0.5 : j == 5 ? 0.25881904510252076235 : j == 6 ? 0.0
       : j == 7 ? -0.25881904510252076235 : j == 8 ? -0.5 : j == 9 ? -0.70710678118654752440
       : j == 10 ? -0.86602540378443864676 : j == 11 ? -0.96592582628906828675 : -1.0;
}
__host__ __device__ constexpr double cos24(int j) { return j <= 12 ? cos24_half(j) : cos24_half(24 - j); }
__host__ __device__ constexpr double sin24(int j) { return cos24((j + 18) % 24); }

// m mod L for m >= 0 (a mask when L is a power of two)
template <int L>
__device__ __forceinline__ int wrap(int m) {
  if constexpr ((L & (L - 1)) == 0) return m & (L - 1);
  else return m % L;
}

template <int R>
__host__ __device__ constexpr int bitrev(int i) {
  int r = 0;
  for (int b = 1, q = R >> 1; b < R; b <<= 1, q >>= 1)
    if (i & b) r |= q;
  return r;
}

// In-register DFT of length R (a power of two <= 32, or 3, 6, 12, 24):
//   X[k] = sum_n x[n] exp(DIR * 2 pi i n k / R)   (DIR = -1 forward, +1 inverse)
template <typename T, int R, int DIR>
__device__ __forceinline__ void dft_reg(T (&xr)[R], T (&xi)[R]) {
  static_assert(R >= 1 && ((R <= 32 && (R & (R - 1)) == 0) || R == 3 || R == 6 || R == 12 || R == 24),
                "a power of two up to 32, or 3, 6, 12, 24");
  if constexpr (R % 3 == 0) {
    // decimation in time by 3: the DFTs E_r of x[3n + r] (length M = R/3),
    // then X[k + q M] = E_0 + w^q W^k E_1 + w^{2q} W^{2k} E_2 with
    // W = exp(DIR 2 pi i / R) and w = W^M = -1/2 + DIR i sqrt(3)/2
    constexpr int M = R / 3;
    T er[3][M], ei[3][M];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int n = 0; n < M; ++n) {
        er[r][n] = xr[3 * n + r];
        ei[r][n] = xi[3 * n + r];
      }
      if constexpr (M > 1) dft_reg<T, M, DIR>(er[r], ei[r]);
    }
    constexpr T c3 = (T)(DIR * 0.86602540378443864676);
#pragma unroll
    for (int k = 0; k < M; ++k) {
      T t1r = er[1][k], t1i = ei[1][k], t2r = er[2][k], t2i = ei[2][k];
      if (k != 0) {
        const int j1 = (k * (24 / R)) % 24, j2 = (2 * k * (24 / R)) % 24;
        const T c1 = (T)cos24(j1), s1 = (T)(DIR * sin24(j1));
        const T c2 = (T)cos24(j2), s2 = (T)(DIR * sin24(j2));
        const T ar = t1r * c1 - t1i * s1, ai = t1r * s1 + t1i * c1;
        const T br = t2r * c2 - t2i * s2, bi = t2r * s2 + t2i * c2;
        t1r = ar;
        t1i = ai;
        t2r = br;
        t2i = bi;
      }
      const T sr = t1r + t2r, si = t1i + t2i, dr = t1r - t2r, di = t1i - t2i;
      const T mr = er[0][k] - (T)0.5 * sr, mi = ei[0][k] - (T)0.5 * si;
      xr[k] = er[0][k] + sr;
      xi[k] = ei[0][k] + si;
      xr[k + M] = mr - c3 * di;
      xi[k + M] = mi + c3 * dr;
      xr[k + 2 * M] = mr + c3 * di;
      xi[k + 2 * M] = mi - c3 * dr;
    }
    return;
  } else if constexpr (R == 32) {
    // two length-16 DFTs of the even and odd samples, then one radix-2 step
    // (keeps the live values near 2R instead of the fully unrolled tree's)
    T er[16], ei[16], orr[16], oi[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      er[i] = xr[2 * i];
      ei[i] = xi[2 * i];
      orr[i] = xr[2 * i + 1];
      oi[i] = xi[2 * i + 1];
    }
    dft_reg<T, 16, DIR>(er, ei);
    dft_reg<T, 16, DIR>(orr, oi);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      T vr, vi;
      if (k == 0) {
        vr = orr[k];
        vi = oi[k];
      } else if (k == 8) {  // multiply by DIR * i
        vr = (T)(-DIR) * oi[k];
        vi = (T)DIR * orr[k];
      } else {
        const T wr = (T)cos32(k);
        const T wi = (T)(DIR * sin32(k));
        vr = orr[k] * wr - oi[k] * wi;
        vi = orr[k] * wi + oi[k] * wr;
      }
      xr[k] = er[k] + vr;
      xi[k] = ei[k] + vi;
      xr[k + 16] = er[k] - vr;
      xi[k + 16] = ei[k] - vi;
    }
    return;
  }
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
        const int idx = j * (32 / len);  // W_len^j = exp(DIR 2 pi i idx / 32)
        const int a = s + j, b = s + j + len / 2;
        T vr, vi;
        if (idx == 0) {
          vr = tr[b];
          vi = ti[b];
        } else if (idx == 8) {  // multiply by DIR * i
          vr = (T)(-DIR) * ti[b];
          vi = (T)DIR * tr[b];
        } else {
          const T wr = (T)cos32(idx);
          const T wi = (T)(DIR * sin32(idx));
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

// twc[m] = cos(2 pi m / P), tws[m] = sin(2 pi m / P), m < P.  FP32 tables
// come from the FP32 sincospi (about one unit in the last place), FP64
// tables from the FP64 one.
template <typename T, int P>
__device__ __forceinline__ void build_twiddles(T *twc, T *tws) {
  for (int m = threadIdx.x; m < P; m += blockDim.x) {
    if constexpr (sizeof(T) == 4) {
      float s, c;
      sincospif(2.0f * (float)m / (float)P, &s, &c);
      twc[m] = c;
      tws[m] = s;
    } else {
      double s, c;
      sincospi(2.0 * (double)m / (double)P, &s, &c);
      twc[m] = c;
      tws[m] = s;
    }
  }
}

// Stage 1 of a length-L = R1*R2 DFT along rows of (br, bi)[row*ld + b] for
// BB columns: for each (n2, b), DFT_R1 over rows R2*n1 + n2, multiply by
// W_L^(n2 k1), write back in place.  Entry TSTEP m of the TSIZE-entry table is W_L^m.
template <typename T, int R1, int R2, int BB, int DIR, int TSTEP, int TSIZE>
__device__ __forceinline__ void dft_stage1(T *br, T *bi, int ld, const T *twc, const T *tws) {
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
        const int m = wrap<TSIZE>(n2 * k1 * TSTEP);
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
  // (lengths 3 * 2^k: a radix-12 or, at 768, radix-24 first stage)
  static constexpr int R1 = P == 768 ? 24 : (P == 384 || P == 192 || P == 96 || P == 48 || P == 24) ? 12
                           : P == 1024 ? 32 : P == 512 ? 16 : P == 256 ? 16 : P == 128 ? 16 : P == 64 ? 8 : P == 32 ? 8
                           : P == 16 ? 4 : P == 8 ? 4 : 2;
  static constexpr int R2 = P / R1;
};

// ---- column pass ---------------------------------------------------------------
// One block per (ky, BB planes).  Stage 1 reads its R1 inputs straight from
// global memory into registers (lanes run along the planes, so every load
// instruction covers contiguous runs), stage 2 gets its inputs through LDS.
// The exchange goes through one real-valued LDS array, first the real then
// the imaginary parts, to keep the block's LDS small.
template <typename T, int P, int BB, bool INV>
__global__ void __launch_bounds__(512)
col_pass_kernel(int ny, int B, const T *__restrict__ in, T *__restrict__ out, int ppv,
                const int *__restrict__ active, int nsum, size_t sstride) {
  constexpr int R1 = Fac<P>::R1, R2 = Fac<P>::R2;
  constexpr int DIR = INV ? 1 : -1;
  constexpr int ld = BB + 1;
  static_assert(R1 * BB <= 512 && R2 * BB <= 512, "one unit per thread");
  __shared__ T lds[P * ld];
  __shared__ T twc[P], tws[P];
  const int ky = blockIdx.x;
  const int b0 = blockIdx.y * BB;
  if (active != nullptr && active[b0 / ppv] == 0) return;  // frozen volume
  const int rows_in = INV ? P : ny;
  const int rows_out = INV ? ny : P;
  const int tid = threadIdx.x;
  build_twiddles<T, P>(twc, tws);
  const T *src = in + (size_t)ky * rows_in * 2 * B + b0;
  const bool act1 = tid < R2 * BB;
  const int b1 = tid % BB, n2 = tid / BB;
  T yr[R1], yi[R1];
  if (act1) {
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) {
      const int row = R2 * n1 + n2;
      if (row < rows_in) {
        yr[n1] = src[((size_t)row * 2) * B + b1];
        yi[n1] = src[((size_t)row * 2 + 1) * B + b1];
        // partial spectra of a split adjoint, added in part order
        for (int q = 1; q < nsum; ++q) {
          yr[n1] += src[(size_t)q * sstride + ((size_t)row * 2) * B + b1];
          yi[n1] += src[(size_t)q * sstride + ((size_t)row * 2 + 1) * B + b1];
        }
      } else {
        yr[n1] = (T)0;
        yi[n1] = (T)0;
      }
    }
  }
  __syncthreads();  // twiddle table ready
  if (act1) {
    dft_reg<T, R1, DIR>(yr, yi);
#pragma unroll
    for (int k1 = 1; k1 < R1; ++k1) {
      const int m = wrap<P>(n2 * k1);
      const T c = twc[m], sn = (T)DIR * tws[m];
      const T tr = yr[k1] * c - yi[k1] * sn;
      yi[k1] = yr[k1] * sn + yi[k1] * c;
      yr[k1] = tr;
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) lds[(R2 * k1 + n2) * ld + b1] = yr[k1];
  }
  __syncthreads();
  const bool act2 = tid < R1 * BB;
  const int b2 = tid % BB, k1 = tid / BB;
  T zr[R2], zi[R2];
  if (act2) {
#pragma unroll
    for (int m = 0; m < R2; ++m) zr[m] = lds[(R2 * k1 + m) * ld + b2];
  }
  __syncthreads();
  if (act1) {
#pragma unroll
    for (int kk = 0; kk < R1; ++kk) lds[(R2 * kk + n2) * ld + b1] = yi[kk];
  }
  __syncthreads();
  if (act2) {
#pragma unroll
    for (int m = 0; m < R2; ++m) zi[m] = lds[(R2 * k1 + m) * ld + b2];
    dft_reg<T, R2, DIR>(zr, zi);
    T *dst = out + (size_t)ky * rows_out * 2 * B + b0;
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) {
      const int row = k1 + R1 * k2;
      if (row < rows_out) {
        if constexpr (!INV) {
          // the forward pass's spectrum goes to memory at once (non-temporal):
          // the contraction that reads it next then starts without this
          // pass's dirty lines draining from the L2 under its reads
          __builtin_nontemporal_store(zr[k2], &dst[((size_t)row * 2) * B + b2]);
          __builtin_nontemporal_store(zi[k2], &dst[((size_t)row * 2 + 1) * B + b2]);
        } else {
          dst[((size_t)row * 2) * B + b2] = zr[k2];
          dst[((size_t)row * 2 + 1) * B + b2] = zi[k2];
        }
      }
    }
  }
}

// Two-stage length-H DFT in place on (wr, wi)[m * ld + b], natural order in
// and out, for blocks of NT threads; a thread holds its NU stage-2 units in
// registers between the two barriers.
template <typename T, int H, int BB, int DIR, int TSTEP = 2, int NT = 512>
__device__ __forceinline__ void dft_lds_inplace(T *wr, T *wi, const T *twc, const T *tws) {
  constexpr int R1 = Fac<H>::R1, R2 = Fac<H>::R2;
  constexpr int ld = BB + 1;
  constexpr int NU = (R1 * BB + NT - 1) / NT;
  // stage-1 twiddles W_H^m live at index TSTEP m of the length-(TSTEP H) table
  dft_stage1<T, R1, R2, BB, DIR, TSTEP, TSTEP * H>(wr, wi, ld, twc, tws);
  __syncthreads();
  const int tid = threadIdx.x;
  T zr[NU][R2], zi[NU][R2];
#pragma unroll
  for (int q = 0; q < NU; ++q) {
    const int u = tid + q * NT;
    if (u < R1 * BB) dft_stage2_unit<T, R1, R2, DIR>(wr, wi, ld, u / BB, u % BB, zr[q], zi[q]);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NU; ++q) {
    const int u = tid + q * NT;
    if (u < R1 * BB) {
      const int b = u % BB, k1 = u / BB;
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) {
        const int m = k1 + R1 * k2;
        wr[m * ld + b] = zr[q][k2];
        wi[m * ld + b] = zi[q][k2];
      }
    }
  }
  __syncthreads();
}

// Column pass for FFT sizes above 256: a radix-32 stage does not fit in the
// registers beside its global addresses, so the block's columns (P x BB
// complex) go through LDS whole and the DFT runs in place there.
template <typename T, int P, int BB, bool INV>
__global__ void __launch_bounds__(512)
col_pass_lds_kernel(int ny, int B, const T *__restrict__ in, T *__restrict__ out, int ppv,
                    const int *__restrict__ active) {
  constexpr int DIR = INV ? 1 : -1;
  constexpr int ld = BB + 1;
  constexpr int NT = 512;
  __shared__ T wr[P * ld], wi[P * ld];
  __shared__ T twc[P], tws[P];
  const int ky = blockIdx.x;
  const int b0 = blockIdx.y * BB;
  if (active != nullptr && active[b0 / ppv] == 0) return;  // frozen volume
  const int rows_in = INV ? P : ny;
  const int rows_out = INV ? ny : P;
  const int tid = threadIdx.x;
  build_twiddles<T, P>(twc, tws);
  const T *src = in + (size_t)ky * rows_in * 2 * B + b0;
#pragma unroll 4
  for (int u = tid; u < P * BB; u += NT) {
    const int b = u % BB, row = u / BB;
    T xr = (T)0, xi = (T)0;
    if (row < rows_in) {
      xr = src[((size_t)row * 2) * B + b];
      xi = src[((size_t)row * 2 + 1) * B + b];
    }
    wr[row * ld + b] = xr;
    wi[row * ld + b] = xi;
  }
  __syncthreads();
  dft_lds_inplace<T, P, BB, DIR, 1>(wr, wi, twc, tws);
  T *dst = out + (size_t)ky * rows_out * 2 * B + b0;
#pragma unroll 4
  for (int u = tid; u < rows_out * BB; u += NT) {
    const int b = u % BB, row = u / BB;
    dst[((size_t)row * 2) * B + b] = wr[row * ld + b];
    dst[((size_t)row * 2 + 1) * B + b] = wi[row * ld + b];
  }
}

// Length-64 DFTs in place on 32 blocks of 64 consecutive rows (block s
// covers rows 64 s .. 64 s + 63), BB planes each, natural order in and out,
// as two radix-8 steps; W_64^m is entry (P/64) m of the length-P table.
// Every thread keeps at most two units of the second step in registers.
template <typename T, int P, int BB, int DIR>
__device__ __forceinline__ void dft64_blocks(T *wr, T *wi, const T *twc, const T *tws) {
  constexpr int ld = BB + 1;
  constexpr int NU = 32 * 8 * BB;  // (block, n2 or k1, plane) units of each step
  constexpr int NT = 512;
  static_assert(NU <= 2 * NT, "two units per thread");
  const int tid = threadIdx.x;
  for (int u = tid; u < NU; u += NT) {
    const int b = u % BB, n2 = (u / BB) % 8, sb = u / (8 * BB);
    T xr[8], xi[8];
#pragma unroll
    for (int n1 = 0; n1 < 8; ++n1) {
      xr[n1] = wr[(64 * sb + 8 * n1 + n2) * ld + b];
      xi[n1] = wi[(64 * sb + 8 * n1 + n2) * ld + b];
    }
    dft_reg<T, 8, DIR>(xr, xi);
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) {
      T yr = xr[k1], yi = xi[k1];
      if (k1 != 0) {
        const int m = (n2 * k1 * (P / 64)) & (P - 1);
        const T c = twc[m], sn = (T)DIR * tws[m];
        const T tr = yr * c - yi * sn;
        yi = yr * sn + yi * c;
        yr = tr;
      }
      wr[(64 * sb + 8 * k1 + n2) * ld + b] = yr;
      wi[(64 * sb + 8 * k1 + n2) * ld + b] = yi;
    }
  }
  __syncthreads();
  T zr[2][8], zi[2][8];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int u = tid + h * NT;
    if (u < NU) {
      const int b = u % BB, k1 = (u / BB) % 8, sb = u / (8 * BB);
#pragma unroll
      for (int n2 = 0; n2 < 8; ++n2) {
        zr[h][n2] = wr[(64 * sb + 8 * k1 + n2) * ld + b];
        zi[h][n2] = wi[(64 * sb + 8 * k1 + n2) * ld + b];
      }
      dft_reg<T, 8, DIR>(zr[h], zi[h]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int u = tid + h * NT;
    if (u < NU) {
      const int b = u % BB, k1 = (u / BB) % 8, sb = u / (8 * BB);
#pragma unroll
      for (int k2 = 0; k2 < 8; ++k2) {
        wr[(64 * sb + k1 + 8 * k2) * ld + b] = zr[h][k2];
        wi[(64 * sb + k1 + 8 * k2) * ld + b] = zi[h][k2];
      }
    }
  }
  __syncthreads();
}

// Column pass for FFT size 2048: 32 x 64 through LDS (a radix-32 step with
// twiddles, then the 64-point blocks of dft64_blocks); output row
// r = k1 + 32 k2 sits in LDS row 64 k1 + k2.
template <typename T, int BB, bool INV>
__global__ void __launch_bounds__(512)
col_pass_2048_kernel(int ny, int B, const T *__restrict__ in, T *__restrict__ out, int ppv,
                     const int *__restrict__ active) {
  constexpr int P = 2048;
  constexpr int DIR = INV ? 1 : -1;
  constexpr int ld = BB + 1;
  constexpr int NT = 512;
  __shared__ T wr[P * ld], wi[P * ld];
  __shared__ T twc[P], tws[P];
  const int ky = blockIdx.x;
  const int b0 = blockIdx.y * BB;
  if (active != nullptr && active[b0 / ppv] == 0) return;  // frozen volume
  const int rows_in = INV ? P : ny;
  const int rows_out = INV ? ny : P;
  const int tid = threadIdx.x;
  build_twiddles<T, P>(twc, tws);
  const T *src = in + (size_t)ky * rows_in * 2 * B + b0;
#pragma unroll 4
  for (int u = tid; u < P * BB; u += NT) {
    const int b = u % BB, row = u / BB;
    T xr = (T)0, xi = (T)0;
    if (row < rows_in) {
      xr = src[((size_t)row * 2) * B + b];
      xi = src[((size_t)row * 2 + 1) * B + b];
    }
    wr[row * ld + b] = xr;
    wi[row * ld + b] = xi;
  }
  __syncthreads();
  dft_stage1<T, 32, 64, BB, DIR, 1, P>(wr, wi, ld, twc, tws);
  __syncthreads();
  dft64_blocks<T, P, BB, DIR>(wr, wi, twc, tws);
  T *dst = out + (size_t)ky * rows_out * 2 * B + b0;
#pragma unroll 4
  for (int u = tid; u < rows_out * BB; u += NT) {
    const int b = u % BB, r = u / BB;
    const int lr = 64 * (r & 31) + (r >> 5);
    dst[((size_t)r * 2) * B + b] = wr[lr * ld + b];
    dst[((size_t)r * 2 + 1) * B + b] = wi[lr * ld + b];
  }
}

// FISTA's extrapolation y = mu + beta (mu - mu_prev), one rounding of the
// product-sum (the same expression wherever a step is taken or resumed, so a
// resumed solve reproduces an uninterrupted one bit for bit).
template <typename T>
__device__ __forceinline__ T fista_extrapolate(T mu, T mprev, T beta) {
  if constexpr (sizeof(T) == 8) return __builtin_fma(beta, mu - mprev, mu);
  else return __builtin_fmaf(beta, mu - mprev, mu);
}

// ---- row pass --------------------------------------------------------------------
// One block per (scan row i, BB planes): c2r along ky, crop, pointwise step,
// pad, r2c.  A real DFT of length P is a complex DFT of length H = P/2 on
// (even, odd) sample pairs; the pre/post-processing pairs bins k and H - k.
template <typename T, int P, int BB>
__global__ void __launch_bounds__(512)
row_pass_kernel(int ny, int nx, RowArgs a) {
  constexpr int H = P / 2;
  constexpr int ld = BB + 1;
  constexpr int NT = 512;
  constexpr int V = 16 / (int)sizeof(T);  // elements per 16-byte access
  constexpr int BQ = BB / V;              // 16-byte words per plane run
  static_assert(BB % V == 0, "plane blocks are whole 16-byte words");
  typedef T VT __attribute__((ext_vector_type(V)));
  __shared__ T wr[H * ld], wi[H * ld];
  __shared__ T twc[P], tws[P];
  __shared__ double red[2 * (NT / 64)];

  const int op = a.op;
  const int i = blockIdx.x;
  const int b0 = blockIdx.y * BB;
  const int B = a.B;
  const int tid = threadIdx.x;
  // a block's planes all belong to one volume (BB divides the planes per volume)
  const int vol = b0 / a.ppv;
  const int pb0 = b0 - vol * a.ppv;
  const bool vol_on = vol < a.nvol;
  if (a.active != nullptr && vol_on && a.active[vol] == 0) return;  // frozen volume
  const int it = a.iter_ctr ? *a.iter_ctr : 0;
  const bool spec_in = (op != ROW_SPATIAL_TO_SPEC) && (op != ROW_SCALE_TO_SPEC) && (op != ROW_EXTRAPOLATE);
  const bool spec_out = (op == ROW_SPATIAL_TO_SPEC) || (op == ROW_SCALE_TO_SPEC) ||
                        (op == ROW_RESIDUAL) || (op == ROW_PASS) || (op == ROW_FISTA) ||
                        (op == ROW_EXTRAPOLATE);
  // the gradient mapping at zero rides along the first step of a zero start
  const bool g0acc = op == ROW_FISTA && a.gmap0_at >= 0 && it == a.gmap0_at;
  const int nh = (nx + 1) / 2;
  build_twiddles<T, P>(twc, tws);
  __syncthreads();

  if (spec_in) {
    // Z[k] = A + i B,  A = X[k] + conj(X[H-k]),  B = (X[k] - conj(X[H-k])) e^{+2 pi i k/P}
    // A unit is (k, V consecutive planes): four 16-byte loads (X[k] and
    // X[H-k], real and imaginary rows); two rounds of units are loaded
    // before either is used (indices clamped into range, so every load is in
    // bounds).
    const T *src = reinterpret_cast<const T *>(a.spec_in) + b0;
    constexpr int NUV = (H / 2 + 1) * BQ;
#pragma unroll 1
    for (int u0 = tid; u0 < NUV; u0 += 2 * NT) {
      VT xv[2][4];
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const int u = min(u0 + jj * NT, NUV - 1);
        const int q = u % BQ, k = u / BQ;
        const size_t o1 = (((size_t)k * ny + i) * 2) * B + q * V;
        const size_t o2 = (((size_t)(H - k) * ny + i) * 2) * B + q * V;
        xv[jj][0] = *reinterpret_cast<const VT *>(src + o1);
        xv[jj][1] = *reinterpret_cast<const VT *>(src + o1 + B);
        xv[jj][2] = *reinterpret_cast<const VT *>(src + o2);
        xv[jj][3] = *reinterpret_cast<const VT *>(src + o2 + B);
      }
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const int u = u0 + jj * NT;
        if (u >= NUV) continue;
        const int q = u % BQ, k = u / BQ;
        const T c = twc[k], s = tws[k];
        const int kk = H - k;
        const T cc = twc[wrap<P>(kk)], ss = tws[wrap<P>(kk)];
#pragma unroll
        for (int e = 0; e < V; ++e) {
          const int b = q * V + e;
          const T x1r = xv[jj][0][e], x1i = xv[jj][1][e];
          const T x2r = xv[jj][2][e], x2i = xv[jj][3][e];
          {
            const T ar = x1r + x2r, ai = x1i - x2i;
            const T dr = x1r - x2r, di = x1i + x2i;
            const T br_ = dr * c - di * s, bi_ = dr * s + di * c;
            wr[k * ld + b] = ar - bi_;
            wi[k * ld + b] = ai + br_;
          }
          if (k > 0 && k < H / 2) {
            const T ar = x2r + x1r, ai = x2i - x1i;
            const T dr = x2r - x1r, di = x2i + x1i;
            const T br_ = dr * cc - di * ss, bi_ = dr * ss + di * cc;
            wr[kk * ld + b] = ar - bi_;
            wi[kk * ld + b] = ai + br_;
          }
        }
      }
    }
    __syncthreads();
    dft_lds_inplace<T, H, BB, 1>(wr, wi, twc, tws);
  }

  // pointwise step on the cropped real row x[j], j < n (in place: the value
  // x[j] lives in the slot that receives r[j])
  double acc0 = 0.0, acc1 = 0.0;
  const T tau = (T)a.tau, lam = (T)a.lambda;
  const int boff = (a.beta_off != nullptr && vol_on) ? a.beta_off[vol] : 0;
  const T beta = a.beta_tab ? (T)a.beta_tab[it - boff] : (T)a.beta;
  T scale = (T)1;
  if (op == ROW_SCALE_TO_SPEC) scale = (T)(1.0 / sqrt(*a.scalar));
  const T *sp_in = vol_on ? reinterpret_cast<const T *>(a.sp_in[vol]) : nullptr;
  T *sp_out = vol_on ? reinterpret_cast<T *>(a.sp_out[vol]) : nullptr;
  T *sp_aux = vol_on ? reinterpret_cast<T *>(a.sp_aux[vol]) : nullptr;
  T *sp_prev = vol_on ? reinterpret_cast<T *>(a.sp_prev[vol]) : nullptr;
  // One element of the pointwise step: x is the c2r value (spec_in ops),
  // yi / ya the spatial inputs; r receives the value for the r2c, o and oa
  // the spatial outputs (sp_out, sp_aux) of the ops that write them.
  auto point = [&](T x, T yi, T ya, int pl, T &r, T &o, T &oa) {
    switch (op) {
      case ROW_SPEC_TO_SPATIAL:
        o = x;
        break;
      case ROW_SPATIAL_TO_SPEC:
        r = yi;
        break;
      case ROW_SCALE_TO_SPEC:
        r = yi * scale;
        o = r;
        break;
      case ROW_RESIDUAL:
      case ROW_FIT:
        r = x - yi;
        acc0 += 0.5 * (double)r * (double)r;
        break;
      case ROW_PASS:
        r = x;
        acc0 += 0.5 * (double)x * (double)x;
        break;
      case ROW_FISTA: {
        T mu = yi - tau * (x + lam * yi);
        if (a.l1) mu -= tau * (T)a.l1[pl];  // prox of the per-layer L1 term
        mu = mu < (T)0 ? (T)0 : mu;  // a NaN stays NaN (the solve's checks then stop it)
        const T ynew = fista_extrapolate(mu, ya, beta);
        oa = mu;
        o = ynew;
        const double dd = (double)yi - (double)mu;
        acc0 += dd * dd;
        if (g0acc) {
          // y = 0 here, so x = -A^T d exactly (negation is exact in every step)
          const double v = -(double)x - (a.l1 ? a.l1[pl] : 0.0);
          const double gz = v > 0.0 ? v : 0.0;
          acc1 += gz * gz;
        }
        r = a.spec_of_mu ? mu : ynew;
        break;
      }
      case ROW_EXTRAPOLATE:
        o = fista_extrapolate(yi, ya, beta);
        r = o;
        break;
      case ROW_POWER_W:
        o = x;
        acc0 += (double)x * (double)x;
        acc1 += (double)yi * (double)x;
        break;
      case ROW_GMAP0: {
        const double v = (double)x - (a.l1 ? a.l1[pl] : 0.0);
        const double g = v > 0.0 ? v : 0.0;
        acc0 += g * g;
        break;
      }
      default:
        break;
    }
  };
  const bool rd_in = op == ROW_SPATIAL_TO_SPEC || op == ROW_SCALE_TO_SPEC || op == ROW_RESIDUAL ||
                     op == ROW_FIT || op == ROW_FISTA || op == ROW_POWER_W || op == ROW_EXTRAPOLATE;
  const bool rd_aux = op == ROW_FISTA || op == ROW_EXTRAPOLATE;
  const bool wr_out = op == ROW_SPEC_TO_SPATIAL || op == ROW_SCALE_TO_SPEC || op == ROW_FISTA ||
                      op == ROW_EXTRAPOLATE || op == ROW_POWER_W;
  const bool wr_aux = op == ROW_FISTA;
  const bool wr_prev = op == ROW_FISTA && sp_prev != nullptr;
  // Each element is read and written by one thread, so outputs that alias
  // an input (FISTA's y) stay correct.
  if (a.sp_vec) {
    // rows of whole 16-byte words: a unit is V consecutive samples of one
    // plane row, read and written with one vector access per array; two
    // rounds of units are loaded before either is used
    const int nxv = nx / V;
    const int NPV = nxv * BB;
#pragma unroll 1
    for (int u0 = tid; u0 < NPV; u0 += 2 * NT) {
      VT yin[2], yaux[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int u = u0 + q * NT;
        const int pl = pb0 + u / nxv;
        const bool ok = u < NPV && vol_on && pl < a.nplanes;
        const size_t idx = ((size_t)pl * ny + i) * nx + (size_t)(u % nxv) * V;
        yin[q] = (rd_in && ok) ? *reinterpret_cast<const VT *>(sp_in + idx) : VT{};
        yaux[q] = (rd_aux && ok) ? *reinterpret_cast<const VT *>(sp_aux + idx) : VT{};
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int u = u0 + q * NT;
        if (u >= NPV) break;
        const int jq = u % nxv, b = u / nxv;
        const int pl = pb0 + b;
        const bool valid = vol_on && pl < a.nplanes;
        const size_t idx = ((size_t)pl * ny + i) * nx + (size_t)jq * V;
        VT o{}, oa{};
#pragma unroll
        for (int e = 0; e < V; ++e) {
          const int j = jq * V + e;
          T *slot = ((j & 1) ? wi : wr) + (j >> 1) * ld + b;
          T x = (T)0;
          if (spec_in) x = *slot;
          T r = (T)0, ov = (T)0, oav = (T)0;
          if (valid) point(x, yin[q][e], yaux[q][e], pl, r, ov, oav);
          o[e] = ov;
          oa[e] = oav;
          if (spec_out) *slot = r;
        }
        if (valid) {
          if (wr_prev) *reinterpret_cast<VT *>(sp_prev + idx) = yaux[q];
          if (wr_aux) *reinterpret_cast<VT *>(sp_aux + idx) = oa;
          if (wr_out) *reinterpret_cast<VT *>(sp_out + idx) = o;
        }
      }
    }
  } else {
    // any row length: one sample per unit, four rounds loaded before use
    constexpr int NQ = 4;
    const int NP = nx * BB;
    for (int u0 = tid; u0 < NP; u0 += NQ * NT) {
      T yin[NQ], yaux[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int u = u0 + q * NT;
        const int pl = pb0 + u / nx;
        const bool ok = u < NP && vol_on && pl < a.nplanes;
        const size_t idx = ((size_t)pl * ny + i) * nx + u % nx;
        yin[q] = (rd_in && ok) ? sp_in[idx] : (T)0;
        yaux[q] = (rd_aux && ok) ? sp_aux[idx] : (T)0;
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int u = u0 + q * NT;
        if (u >= NP) break;
        const int j = u % nx, b = u / nx;
        const int pl = pb0 + b;
        const bool valid = vol_on && pl < a.nplanes;
        const size_t idx = ((size_t)pl * ny + i) * nx + j;
        T *slot = ((j & 1) ? wi : wr) + (j >> 1) * ld + b;
        T x = (T)0;
        if (spec_in) x = *slot;
        T r = (T)0, ov = (T)0, oav = (T)0;
        if (valid) {
          point(x, yin[q], yaux[q], pl, r, ov, oav);
          if (wr_prev) sp_prev[idx] = yaux[q];
          if (wr_aux) sp_aux[idx] = oav;
          if (wr_out) sp_out[idx] = ov;
        }
        if (spec_out) *slot = r;
      }
    }
  }
  if (spec_out) {
    for (int u = tid; u < H * BB; u += NT) {
      const int b = u % BB, m = u / BB;
      if (m >= nh) {
        wr[m * ld + b] = (T)0;
        wi[m * ld + b] = (T)0;
      } else if ((nx & 1) && m == nh - 1) {
        wi[m * ld + b] = (T)0;
      }
    }
  }
  constexpr int NW = NT / 64;
  if (a.partials) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      acc0 += __shfl_xor(acc0, off, 64);
      acc1 += __shfl_xor(acc1, off, 64);
    }
    if ((tid & 63) == 0) {
      red[tid >> 6] = acc0;
      red[NW + (tid >> 6)] = acc1;
    }
  }
  __syncthreads();
  if (a.partials && tid == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int w = 0; w < NW; ++w) {
      s0 += red[w];
      s1 += red[NW + w];
    }
    const size_t blk = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    double *part = a.partials + (a.iter_ctr ? (size_t)it * a.part_stride : 0);
    part[2 * blk] = s0;
    part[2 * blk + 1] = s1;
  }
  if (!spec_out) return;

  // r2c: Z' = DFT_H(r_even + i r_odd); X'[k] = Ev[k] + e^{-2 pi i k/P} Od[k]
  dft_lds_inplace<T, H, BB, -1>(wr, wi, twc, tws);
  T *dst = reinterpret_cast<T *>(a.spec_out) + b0;
  // a unit is (k, V consecutive planes): bins k, H - k (and H with k = 0)
  // for V planes, each stored with 16-byte writes
  for (int u = tid; u < (H / 2 + 1) * BQ; u += NT) {
    const int q = u % BQ, k = u / BQ;
    const int k2 = (k == 0) ? 0 : H - k;
    const T c = twc[k], s = -tws[k];
    const T c2 = twc[k2], s2 = -tws[k2];
    VT pr, pi, qr, qi, hr, hi;
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const int b = q * V + e;
      const T z1r = wr[k * ld + b], z1i = wi[k * ld + b];
      const T z2r = wr[k2 * ld + b], z2i = wi[k2 * ld + b];
      // bin k from (Z'[k], Z'[H-k]); bin H-k from the same pair swapped
      // (bin H from Z'[0] with e^{-i pi} = -1)
      const T evr = (T)0.5 * (z1r + z2r), evi = (T)0.5 * (z1i - z2i);
      const T odr = (T)0.5 * (z1i + z2i), odi = (T)(-0.5) * (z1r - z2r);
      pr[e] = evr + odr * c - odi * s;
      pi[e] = evi + odr * s + odi * c;
      hr[e] = evr - odr;
      hi[e] = evi - odi;
      const T evr2 = (T)0.5 * (z2r + z1r), evi2 = (T)0.5 * (z2i - z1i);
      const T odr2 = (T)0.5 * (z2i + z1i), odi2 = (T)(-0.5) * (z2r - z1r);
      qr[e] = evr2 + odr2 * c2 - odi2 * s2;
      qi[e] = evi2 + odr2 * s2 + odi2 * c2;
    }
    const size_t ok_ = (((size_t)k * ny + i) * 2) * B + q * V;
    *reinterpret_cast<VT *>(dst + ok_) = pr;
    *reinterpret_cast<VT *>(dst + ok_ + B) = pi;
    if (k == 0) {
      const size_t oh = (((size_t)H * ny + i) * 2) * B + q * V;
      *reinterpret_cast<VT *>(dst + oh) = hr;
      *reinterpret_cast<VT *>(dst + oh + B) = hi;
    }
    if (k > 0 && k < H / 2) {
      const size_t ok2 = (((size_t)k2 * ny + i) * 2) * B + q * V;
      *reinterpret_cast<VT *>(dst + ok2) = qr;
      *reinterpret_cast<VT *>(dst + ok2 + B) = qi;
    }
  }
}

template <typename T, int P, int BB>
hipError_t col_dispatch_bb(const Dims &d, int B, bool inverse, const T *in, T *out,
                           hipStream_t st, int ppv, const int *active, int nsum, size_t sstride) {
  dim3 grid((unsigned)(d.h + 1), (unsigned)(B / BB));
  if constexpr (P > 256) {
    if (nsum != 1) return hipErrorInvalidValue;
    if (inverse)
      hipLaunchKernelGGL((col_pass_lds_kernel<T, P, BB, true>), grid, dim3(512), 0, st, d.ny, B, in, out, ppv, active);
    else
      hipLaunchKernelGGL((col_pass_lds_kernel<T, P, BB, false>), grid, dim3(512), 0, st, d.ny, B, in, out, ppv, active);
  } else {
    if (inverse)
      hipLaunchKernelGGL((col_pass_kernel<T, P, BB, true>), grid, dim3(512), 0, st, d.ny, B, in, out, ppv, active,
                         nsum, sstride);
    else
      hipLaunchKernelGGL((col_pass_kernel<T, P, BB, false>), grid, dim3(512), 0, st, d.ny, B, in, out, ppv, active,
                         nsum, sstride);
  }
  return hipGetLastError();
}

template <typename T, int P>
hipError_t col_dispatch(const Dims &d, int B, bool inverse, const T *in, T *out, hipStream_t st,
                        int ppv, int bb, const int *active, int nsum, size_t sstride) {
  ppv = ppv ? ppv : B;
  if (nsum < 1 || (nsum > 1 && (!inverse || P > 256))) return hipErrorInvalidValue;
  if constexpr (P == 2048) {
    // three-stage column DFT, the whole block in LDS: 4 FP32 or 2 FP64 planes
    constexpr int BB = sizeof(T) == 8 ? 2 : 4;
    dim3 grid((unsigned)(d.h + 1), (unsigned)(B / BB));
    if (inverse)
      hipLaunchKernelGGL((col_pass_2048_kernel<T, BB, true>), grid, dim3(512), 0, st, d.ny, B, in, out, ppv, active);
    else
      hipLaunchKernelGGL((col_pass_2048_kernel<T, BB, false>), grid, dim3(512), 0, st, d.ny, B, in, out, ppv, active);
    return hipGetLastError();
  } else if constexpr (P > 512) {
    // the whole column block lives in LDS: 16 FP32 or 4 FP64 planes fit
    if constexpr (sizeof(T) == 8) return col_dispatch_bb<T, P, 4>(d, B, inverse, in, out, st, ppv, active, nsum, sstride);
    else return col_dispatch_bb<T, P, 16>(d, B, inverse, in, out, st, ppv, active, nsum, sstride);
  }
  else {
    // 32 planes per block only where every thread still holds one DFT unit
    if constexpr (Fac<P>::R1 * 32 <= 512 && Fac<P>::R2 * 32 <= 512) {
      if (batch_block(d, B, ppv, sizeof(T) == 8, bb) == 32)
        return col_dispatch_bb<T, P, 32>(d, B, inverse, in, out, st, ppv, active, nsum, sstride);
    }
    return col_dispatch_bb<T, P, 16>(d, B, inverse, in, out, st, ppv, active, nsum, sstride);
  }
}

template <typename T, int P, int BB>
hipError_t row_dispatch_bb(const Dims &d, const RowArgs &a, hipStream_t st) {
  dim3 grid((unsigned)d.ny, (unsigned)(a.B / BB));
  hipLaunchKernelGGL((row_pass_kernel<T, P, BB>), grid, dim3(512), 0, st, d.ny, d.nx, a);
  return hipGetLastError();
}

template <typename T, int P>
hipError_t row_dispatch(const Dims &d, const RowArgs &a, hipStream_t st) {
  if constexpr (P > 512) {
    if constexpr (sizeof(T) == 8) return row_dispatch_bb<T, P, 4>(d, a, st);
    else return row_dispatch_bb<T, P, 16>(d, a, st);
  }
  else {
    if constexpr (P <= 256) {
      // (row_pass_blocks counts the blocks with the same rule)
      const int rb = row_block(d, a.B, a.ppv, sizeof(T) == 8, a.bb);
      if constexpr (sizeof(T) == 4) {
        if (rb == 64) return row_dispatch_bb<T, P, 64>(d, a, st);
      }
      if (rb == 32) return row_dispatch_bb<T, P, 32>(d, a, st);
    }
    return row_dispatch_bb<T, P, 16>(d, a, st);
  }
}

}  // namespace

template <typename T>
hipError_t launch_col_pass(const Dims &d, int B, bool inverse, const T *in, T *out,
                           hipStream_t st, int ppv, int bb, const int *active, int nsum, size_t sstride) {
  switch (d.p) {
    case 16: return col_dispatch<T, 16>(d, B, inverse, in, out, st, ppv, bb, active, nsum, sstride);
    case 32: return col_dispatch<T, 32>(d, B, inverse, in, out, st, ppv, bb, active, nsum, sstride);
    case 64: return col_dispatch<T, 64>(d, B, inverse, in, out, st, ppv, bb, active, nsum, sstride);
    case 48: return col_dispatch<T, 48>(d, B, inverse, in, out, st, ppv, bb, active, nsum, sstride);
    case 96: return col_dispatch<T, 96>(d, B, inverse, in, out, st, ppv, bb, active, nsum, sstride);
    case 128: return col_dispatch<T, 128>(d, B, inverse, in, out, st, ppv, bb, active, nsum, sstride);
    case 192: return col_dispatch<T, 192>(d, B, inverse, in, out, st, ppv, bb, active, nsum, sstride);
    case 384: return col_dispatch<T, 384>(d, B, inverse, in, out, st, ppv, bb, active, nsum, sstride);
    case 768: return col_dispatch<T, 768>(d, B, inverse, in, out, st, ppv, bb, active, nsum, sstride);
    case 256: return col_dispatch<T, 256>(d, B, inverse, in, out, st, ppv, bb, active, nsum, sstride);
    case 512: return col_dispatch<T, 512>(d, B, inverse, in, out, st, ppv, bb, active, nsum, sstride);
    case 1024: return col_dispatch<T, 1024>(d, B, inverse, in, out, st, ppv, bb, active, nsum, sstride);
    case 2048: return col_dispatch<T, 2048>(d, B, inverse, in, out, st, ppv, bb, active, nsum, sstride);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_row_pass(const Dims &d, const RowArgs &a0, hipStream_t st) {
  // vector access to the spatial arrays when every row is whole 16-byte
  // words and every array starts on a 16-byte boundary
  RowArgs a = a0;
  const int V = 16 / (int)sizeof(T);
  bool vec = d.nx % V == 0;
  for (int v = 0; v < a.nvol && v < kMaxVol; ++v)
    for (const void *p : {a.sp_in[v], (const void *)a.sp_out[v], (const void *)a.sp_aux[v],
                          (const void *)a.sp_prev[v]})
      vec = vec && (reinterpret_cast<uintptr_t>(p) & 15) == 0;
  a.sp_vec = vec ? 1 : 0;
  switch (d.p) {
    case 16: return row_dispatch<T, 16>(d, a, st);
    case 32: return row_dispatch<T, 32>(d, a, st);
    case 64: return row_dispatch<T, 64>(d, a, st);
    case 48: return row_dispatch<T, 48>(d, a, st);
    case 96: return row_dispatch<T, 96>(d, a, st);
    case 128: return row_dispatch<T, 128>(d, a, st);
    case 192: return row_dispatch<T, 192>(d, a, st);
    case 384: return row_dispatch<T, 384>(d, a, st);
    case 768: return row_dispatch<T, 768>(d, a, st);
    case 256: return row_dispatch<T, 256>(d, a, st);
    case 512: return row_dispatch<T, 512>(d, a, st);
    case 1024: return row_dispatch<T, 1024>(d, a, st);
    case 2048: return row_dispatch<T, 2048>(d, a, st);
    default: return hipErrorInvalidValue;
  }
}

// Planes per block: 32 (128-byte runs) when that still gives enough blocks to
// fill the chip, else 16; FP64 and FFT sizes above 256 (a radix-32 column
// stage) always 16; at FFT size 1024 the column block lives in LDS whole,
// which holds 16 FP32 or 4 FP64 planes.  A block never straddles two volumes
// (the choice divides the planes per volume).
int batch_block(const Dims &d, int B, int ppv, bool fp64, int bb) {
  if (d.p > 512) return fp64 ? 4 : 16;
  if (fp64 || d.p > 256 || (B % 32) != 0 || (ppv % 32) != 0) return 16;
  if (bb == 16 || bb == 32) return bb;
  return ((d.h + 1) * (B / 32) >= 1024) ? 32 : 16;
}

// A row pass also takes 64 planes per block (256-byte runs of the spectrum,
// 67 KB of LDS: two blocks per compute unit) where asked for: FP32 at FFT
// sizes up to 256 with 64 dividing the planes per volume.
int row_block(const Dims &d, int B, int ppv, bool fp64, int bb) {
  if (bb == 64 && !fp64 && d.p <= 256 && B % 64 == 0 && ppv % 64 == 0) return 64;
  return batch_block(d, B, ppv, fp64, bb == 64 ? 32 : bb);
}

int row_pass_blocks(const Dims &d, int B, int ppv, bool fp64, int bb) {
  return d.ny * (B / row_block(d, B, ppv, fp64, bb));
}

template hipError_t launch_col_pass<float>(const Dims &, int, bool, const float *, float *, hipStream_t, int, int,
                                           const int *, int, size_t);
template hipError_t launch_col_pass<double>(const Dims &, int, bool, const double *, double *, hipStream_t, int,
                                            int, const int *, int, size_t);
template hipError_t launch_row_pass<float>(const Dims &, const RowArgs &, hipStream_t);
template hipError_t launch_row_pass<double>(const Dims &, const RowArgs &, hipStream_t);

}  // namespace ctof
