// Source multiplexing (Eq. 12) on gfx950.
//
// With several sources on at once, each multiplexed measurement is a fixed
// linear combination S (M x P) of the confocal transients of one tile of P
// scan positions, the same S in every tile and time bin:
//   y[t][i][g] = sum_j S[i][j] m[t][gy ty + jy][gx tx + jx]
// with tile g = gy (n / tx) + gx and position j = jy tx + jx inside it.
// A column is one (bin, tile) pair: P values of m in, M values of y out.
//
// A block of 256 threads (4 wavefronts) takes 64 columns at a time.  Both
// products are matrix-core contractions, U (M x 64) = S (M x P) X (P x 64)
// and R (P x 64) = S^T (P x M) U, in 16x16x4 MFMA tiles (FP32 or FP64).
// The block's fragments of S and S^T are loaded into registers once; the
// 64 columns of X, and then of U, are staged in LDS column-major ([col][k],
// padded rows) so that each lane fetches the four k values of its next four
// MFMA steps with one vector read: in step s of a 16-wide k block b, lane
// group g = lane/16 carries k = 16 b + 4 g + s.  Wavefront w owns the
// 16-row tiles w and w + 4 of each product.  X is read with one 16-byte
// load per lane (4 consecutive positions of a tile row) when the tile width
// and the scan side are multiples of 4.  The solver's mode fuses the
// residual U = S X - Y, its FP64 half sum of squares and R = S^T U (the
// input of A^T for the composed operator S A) into one pass over X; R may
// overwrite X.
#include <algorithm>

#include "ctof_internal.h"

namespace ctof {

namespace {

constexpr int kCols = 64;      // columns per group
constexpr int kThreads = 256;  // four wavefronts

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <typename T>
struct Mma;
template <>
struct Mma<float> {
  typedef v4f acc_t;
  typedef v4f quad_t;
  static constexpr int kPad = 4;  // row stride = 4 words mod 32 banks: conflict-free quads
  // item r of lane group g is row 4g + r
  __device__ static int row_of(int i) { return i; }
  __device__ static acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mma<double> {
  typedef v4d acc_t;
  typedef v4d quad_t;
  static constexpr int kPad = 0;  // keeps 128-row FP64 staging within 64 KB
  // the f64 result holds row 4r + g in item r of lane group g; A-row i is
  // fed with matrix row 4(i%4) + i/4 so that item r is row 4g + r
  __device__ static int row_of(int i) { return 4 * (i & 3) + (i >> 2); }
  __device__ static acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <typename T>
__device__ __forceinline__ typename Mma<T>::quad_t lds_quad(const T *p) {
  return *reinterpret_cast<const typename Mma<T>::quad_t *>(p);
}
template <typename T>
__device__ __forceinline__ void lds_store_quad(T *p, typename Mma<T>::quad_t v) {
  *reinterpret_cast<typename Mma<T>::quad_t *>(p) = v;
}

// offset of position j of a tile from the tile's first position
__device__ __forceinline__ long long pos_off(int j, int tx, int n) {
  const int jy = j / tx;
  return (long long)jy * n + (j - jy * tx);
}

struct Column {
  long long base, ybase;  // m[t][tile origin], y[t][0][tile]
  bool valid;
};

__device__ __forceinline__ Column column(const MuxArgs &a, long long c, long long ncol) {
  Column k{0, 0, c < ncol};
  if (k.valid) {
    const int ci = (int)c;  // nt * ntiles < 2^31 (checked by the callers)
    const int t = ci / a.ntiles;
    const int tile = ci - t * a.ntiles;
    const int gy = tile / a.ntx, gx = tile - gy * a.ntx;
    k.base = ((long long)t * a.n + (long long)gy * a.ty) * a.n + (long long)gx * a.tx;
    k.ybase = (long long)t * a.M * a.ntiles + tile;
  }
  return k;
}

// KB1 = 16-wide k blocks of the first product (>= ceil(P/16)), KB2 = of the
// second (>= ceil(M/16)); a wavefront holds NT1 row tiles of the first
// product (2 when M > 64) and NT2 of the second (2 when P > 64).
template <typename T, int MODE, int KB1, int KB2>
__global__ void __launch_bounds__(kThreads)
mux_kernel(MuxArgs a) {
  constexpr int NT1 = KB2 == 8 ? 2 : 1;
  constexpr int NT2 = KB1 == 8 ? 2 : 1;
  constexpr bool kPre = sizeof(T) == 4;  // FP32: S fragments live in registers
  constexpr int STR1 = 16 * KB1 + Mma<T>::kPad, STR2 = 16 * KB2 + Mma<T>::kPad;
  typedef typename Mma<T>::acc_t acc_t;
  typedef typename Mma<T>::quad_t quad_t;
  extern __shared__ __align__(16) unsigned char smem[];
  T *buf = reinterpret_cast<T *>(smem);  // [64][STR1] X, then [64][STR2] U
  const T *__restrict__ S = static_cast<const T *>(a.S);
  const int lane = threadIdx.x & 63, g = lane >> 4, i16 = lane & 15;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int M = a.M, P = a.P, MT = (M + 15) / 16, PT = (P + 15) / 16;
  const long long ncol = (long long)a.nt * a.ntiles;
  const long long ngroups = (ncol + kCols - 1) / kCols;
  const bool vec = (a.tx & 3) == 0 && (a.n & 3) == 0;

  // S fragments: first product row tile w + 4 t1, k block b, step s ->
  // S[16 rt + row_of(i16)][16 b + 4 g + s]; second product (S^T) row tile
  // w + 4 t2 -> S[16 b + 4 g + s][16 rt + row_of(i16)]
  auto s1 = [&](int t1, int b, int st) -> T {
    const int i = 16 * (w + 4 * t1) + Mma<T>::row_of(i16), j = 16 * b + 4 * g + st;
    return (i < M && j < P) ? S[(long long)i * P + j] : T(0);
  };
  auto s2 = [&](int t2, int b, int st) -> T {
    const int j = 16 * (w + 4 * t2) + Mma<T>::row_of(i16), i = 16 * b + 4 * g + st;
    return (i < M && j < P) ? S[(long long)i * P + j] : T(0);
  };
  T sa1[kPre && MODE != MUX_ADJ ? NT1 : 1][kPre && MODE != MUX_ADJ ? KB1 : 1][4];
  T sa2[kPre && MODE != MUX_FWD ? NT2 : 1][kPre && MODE != MUX_FWD ? KB2 : 1][4];
  if constexpr (kPre && MODE != MUX_ADJ) {
#pragma unroll
    for (int t1 = 0; t1 < NT1; ++t1)
#pragma unroll
      for (int b = 0; b < KB1; ++b)
#pragma unroll
        for (int st = 0; st < 4; ++st) sa1[t1][b][st] = s1(t1, b, st);
  }
  if constexpr (kPre && MODE != MUX_FWD) {
#pragma unroll
    for (int t2 = 0; t2 < NT2; ++t2)
#pragma unroll
      for (int b = 0; b < KB2; ++b)
#pragma unroll
        for (int st = 0; st < 4; ++st) sa2[t2][b][st] = s2(t2, b, st);
  }
  // padded k rows are multiplied by zero fragments; clear the buffer once so
  // that they never hold a non-finite pattern
  {
    const int total = kCols * (STR1 > STR2 ? STR1 : STR2);
    for (int e = threadIdx.x; e < total; e += kThreads) buf[e] = T(0);
  }
  __syncthreads();

  double fit = 0.0;
  for (long long grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const long long c0 = grp * kCols;
    // columns of this lane in the MFMA layout (16 ct + i16)
    Column cm[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) cm[ct] = column(a, c0 + 16 * ct + i16, ncol);

    if constexpr (MODE == MUX_ADJ) {
      // stage U = Y: lane = column, wavefront w takes rows w, w + 4, ...
      const Column cl = column(a, c0 + lane, ncol);
      const T *yin = static_cast<const T *>(a.in);
      for (int i = w; i < M; i += 4)
        buf[lane * STR2 + i] = cl.valid ? yin[cl.ybase + (long long)i * a.ntiles] : T(0);
      __syncthreads();
    } else {
      // stage X: lane = column, wavefront w takes k quads w, w + 4, ...
      const Column cl = column(a, c0 + lane, ncol);
      const T *m = static_cast<const T *>(a.in);
      for (int q = w; 4 * q < P; q += 4) {
        quad_t v;
        if (vec && 4 * q + 3 < P) {
          v = cl.valid ? *reinterpret_cast<const quad_t *>(m + cl.base + pos_off(4 * q, a.tx, a.n)) : quad_t(0);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int j = 4 * q + e;
            v[e] = (cl.valid && j < P) ? m[cl.base + pos_off(j, a.tx, a.n)] : T(0);
          }
        }
        lds_store_quad<T>(buf + lane * STR1 + 4 * q, v);
      }
      __syncthreads();

      // first product: U = S X for the wavefront's row tiles
      acc_t acc[NT1][4];
#pragma unroll
      for (int t1 = 0; t1 < NT1; ++t1)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[t1][ct] = acc_t(0);
#pragma unroll
      for (int b = 0; b < KB1; ++b) {
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
          const quad_t xv = lds_quad<T>(buf + (16 * ct + i16) * STR1 + 16 * b + 4 * g);
#pragma unroll
          for (int t1 = 0; t1 < NT1; ++t1) {
            if (w + 4 * t1 >= MT) continue;
#pragma unroll
            for (int st = 0; st < 4; ++st) {
              T sv;
              if constexpr (kPre) sv = sa1[t1][b][st]; else sv = s1(t1, b, st);
              acc[t1][ct] = Mma<T>::step(sv, xv[st], acc[t1][ct]);
            }
          }
        }
      }
      if constexpr (MODE == MUX_FWD) {
        T *yo = static_cast<T *>(a.out);
#pragma unroll
        for (int t1 = 0; t1 < NT1; ++t1)
#pragma unroll
          for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = 16 * (w + 4 * t1) + 4 * g + r;
              if (i < M && cm[ct].valid) yo[cm[ct].ybase + (long long)i * a.ntiles] = acc[t1][ct][r];
            }
      } else {
        const T *yv = static_cast<const T *>(a.y);
#pragma unroll
        for (int t1 = 0; t1 < NT1; ++t1)
#pragma unroll
          for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = 16 * (w + 4 * t1) + 4 * g + r;
              T u = T(0);
              if (i < M && cm[ct].valid) {
                u = acc[t1][ct][r];
                if (yv) u -= yv[cm[ct].ybase + (long long)i * a.ntiles];
              }
              acc[t1][ct][r] = u;
              fit += 0.5 * (double)u * (double)u;
            }
        __syncthreads();  // X is no longer read
#pragma unroll
        for (int t1 = 0; t1 < NT1; ++t1) {
          if (w + 4 * t1 >= MT) continue;
#pragma unroll
          for (int ct = 0; ct < 4; ++ct)
            lds_store_quad<T>(buf + (16 * ct + i16) * STR2 + 16 * (w + 4 * t1) + 4 * g, acc[t1][ct]);
        }
        __syncthreads();
      }
    }

    if constexpr (MODE != MUX_FWD) {
      // second product: R = S^T U for the wavefront's row tiles
      acc_t acc2[NT2][4];
#pragma unroll
      for (int t2 = 0; t2 < NT2; ++t2)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc2[t2][ct] = acc_t(0);
#pragma unroll
      for (int b = 0; b < KB2; ++b) {
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
          const quad_t uv = lds_quad<T>(buf + (16 * ct + i16) * STR2 + 16 * b + 4 * g);
#pragma unroll
          for (int t2 = 0; t2 < NT2; ++t2) {
            if (w + 4 * t2 >= PT) continue;
#pragma unroll
            for (int st = 0; st < 4; ++st) {
              T sv;
              if constexpr (kPre) sv = sa2[t2][b][st]; else sv = s2(t2, b, st);
              acc2[t2][ct] = Mma<T>::step(sv, uv[st], acc2[t2][ct]);
            }
          }
        }
      }
      T *ro = static_cast<T *>(a.out);
#pragma unroll
      for (int t2 = 0; t2 < NT2; ++t2) {
        const int j0 = 16 * (w + 4 * t2) + 4 * g;
        if (w + 4 * t2 >= PT) continue;
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
          if (!cm[ct].valid) continue;
          if (vec && j0 + 3 < P) {
            *reinterpret_cast<quad_t *>(ro + cm[ct].base + pos_off(j0, a.tx, a.n)) = acc2[t2][ct];
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (j0 + r < P) ro[cm[ct].base + pos_off(j0 + r, a.tx, a.n)] = acc2[t2][ct][r];
          }
        }
      }
    }
    __syncthreads();  // the buffer is refilled by the next group
  }
  if constexpr (MODE == MUX_NORMAL) {
    if (a.partials) {
      double *red = reinterpret_cast<double *>(smem);  // the staging buffer is free now
      red[threadIdx.x] = fit;
      __syncthreads();
      for (int st = kThreads / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
      }
      if (threadIdx.x == 0) {
        a.partials[2 * (size_t)blockIdx.x] = red[0];
        a.partials[2 * (size_t)blockIdx.x + 1] = 0.0;
      }
    }
  }
}

inline int kblocks(int k) {
  const int b = (k + 15) / 16;
  return b <= 1 ? 1 : b <= 2 ? 2 : b <= 4 ? 4 : 8;
}

template <typename T, int MODE, int KB1, int KB2>
hipError_t launch_one(const MuxArgs &a, int blocks, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL((mux_kernel<T, MODE, KB1, KB2>), dim3((unsigned)blocks), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

template <typename T, int MODE, int KB1>
hipError_t launch_kb2(const MuxArgs &a, int blocks, size_t lds, hipStream_t st) {
  switch (kblocks(a.M)) {
    case 1: return launch_one<T, MODE, KB1, 1>(a, blocks, lds, st);
    case 2: return launch_one<T, MODE, KB1, 2>(a, blocks, lds, st);
    case 4: return launch_one<T, MODE, KB1, 4>(a, blocks, lds, st);
    default: return launch_one<T, MODE, KB1, 8>(a, blocks, lds, st);
  }
}

template <typename T, int MODE>
hipError_t launch_kb1(const MuxArgs &a, int blocks, size_t lds, hipStream_t st) {
  switch (kblocks(a.P)) {
    case 1: return launch_kb2<T, MODE, 1>(a, blocks, lds, st);
    case 2: return launch_kb2<T, MODE, 2>(a, blocks, lds, st);
    case 4: return launch_kb2<T, MODE, 4>(a, blocks, lds, st);
    default: return launch_kb2<T, MODE, 8>(a, blocks, lds, st);
  }
}

}  // namespace

size_t mux_lds_bytes(int M, int P, bool f64) {
  const int pad = f64 ? Mma<double>::kPad : Mma<float>::kPad;
  const int str = 16 * std::max(kblocks(M), kblocks(P)) + pad;
  return std::max<size_t>((size_t)kCols * str * (f64 ? 8 : 4), kThreads * sizeof(double));
}

int mux_default_blocks(const MuxArgs &a) {
  const long long ngroups = ((long long)a.nt * a.ntiles + kCols - 1) / kCols;
  return (int)std::min<long long>(std::max<long long>(ngroups, 1), 4096);
}

hipError_t launch_mux(int mode, bool f64, const MuxArgs &a, int blocks, hipStream_t st) {
  if (a.M < 1 || a.P < 1 || a.M > kMuxMaxDim || a.P > kMuxMaxDim || blocks < 1) return hipErrorInvalidValue;
  const size_t lds = mux_lds_bytes(a.M, a.P, f64);
  if (f64) {
    if (mode == MUX_FWD) return launch_kb1<double, MUX_FWD>(a, blocks, lds, st);
    if (mode == MUX_ADJ) return launch_kb1<double, MUX_ADJ>(a, blocks, lds, st);
    return launch_kb1<double, MUX_NORMAL>(a, blocks, lds, st);
  }
  if (mode == MUX_FWD) return launch_kb1<float, MUX_FWD>(a, blocks, lds, st);
  if (mode == MUX_ADJ) return launch_kb1<float, MUX_ADJ>(a, blocks, lds, st);
  return launch_kb1<float, MUX_NORMAL>(a, blocks, lds, st);
}

}  // namespace ctof
