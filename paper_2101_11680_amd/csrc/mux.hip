// Source multiplexing (Eq. 12) on gfx950.
//
// With several sources on at once, each multiplexed measurement is a fixed
// linear combination S (M x P) of the confocal transients of one tile of P
// scan positions, the same S in every tile and time bin:
//   y[t][i][g] = sum_j S[i][j] m[t][gy ty + jy][gx tx + jx]
// with tile g = gy (n / tx) + gx and position j = jy tx + jx inside it.
// A column is one (bin, tile) pair: P values of m in, M values of y out.
//
// Both products are matrix-core contractions in 16x16x4 MFMA tiles (FP32 or
// FP64): U (M x 16) = S (M x P) X (P x 16) and R (P x 16) = S^T (P x M) U.
// Each wavefront owns 16 columns at a time and keeps them in registers from
// load to store: its X columns are loaded straight into B operands (one
// 16-byte load per lane for four consecutive positions of a tile row), and
// because in step s of a 16-wide k block b lane group g = lane/16 carries
// k = 16 b + 4 g + s, the accumulator of the first product's row tile b is
// already the B operand of the second product's k block b: U never leaves
// the registers.  S is staged once per block in LDS (FP32; rows padded so
// that each lane's four-value A fragment is one conflict-free vector read)
// and read from the caches in FP64.  Blocks are persistent (16 wavefronts
// in FP32, one block per compute unit) and take column tiles in a strided
// loop without barriers.  The solver's mode fuses the residual U = S X - Y,
// its FP64 half sum of squares and R = S^T U (the input of A^T for the
// composed operator S A) into one pass over X; R may overwrite X.
#include <algorithm>

#include "ctof_internal.h"

namespace ctof {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <typename T>
struct Mma;
template <>
struct Mma<float> {
  typedef v4f acc_t;
  typedef v4f quad_t;
  static constexpr int kWaves = 16;  // 1024 threads: four wavefronts per SIMD
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
  static constexpr int kWaves = 4;
  // the f64 result holds row 4r + g in item r of lane group g; A-row i is
  // fed with matrix row 4(i%4) + i/4 so that item r is row 4g + r
  __device__ static int row_of(int i) { return 4 * (i & 3) + (i >> 2); }
  __device__ static acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// Element offsets fit in 32 bits (every array is below 2 GiB, checked by the
// callers), so loads and stores address a uniform base plus a 32-bit lane
// offset.
struct Column {
  uint32_t base, ybase;  // m[t][tile origin], y[t][0][tile]
  bool valid;
};

__device__ __forceinline__ Column column(const MuxArgs &a, long long c, long long ncol) {
  Column k{0u, 0u, c < ncol};
  if (k.valid) {
    const int ci = (int)c;  // nt * ntiles < 2^31
    const int t = ci / a.ntiles;
    const int tile = ci - t * a.ntiles;
    const int gy = tile / a.ntx, gx = tile - gy * a.ntx;
    k.base = ((uint32_t)t * a.ny + (uint32_t)(gy * a.ty)) * (uint32_t)a.nx + (uint32_t)(gx * a.tx);
    k.ybase = (uint32_t)t * (uint32_t)a.M * (uint32_t)a.ntiles + (uint32_t)tile;
  }
  return k;
}

// offset of tile position j (row j / tx, column j % tx) from the tile origin
// on a grid of nx columns
__device__ __forceinline__ uint32_t pos_off32(int j, int tx, int nx) {
  const int jy = j / tx;
  return (uint32_t)(jy * nx + (j - jy * tx));
}

template <typename V, typename T>
__device__ __forceinline__ V ld(const T *p, uint32_t off) {
  return *reinterpret_cast<const V *>(reinterpret_cast<const char *>(p) + (size_t)off * sizeof(T));
}
template <typename V, typename T>
__device__ __forceinline__ void st(T *p, uint32_t off, V v) {
  *reinterpret_cast<V *>(reinterpret_cast<char *>(p) + (size_t)off * sizeof(T)) = v;
}

// KB1: 16-wide k blocks of the first product (>= ceil(P/16)), which are also
// the second product's row tiles; the first product's row tiles (ceil(M/16))
// are a runtime loop.
// VEC: tile width and scan side are multiples of 4 (16-byte column runs).
template <typename T, int MODE, int KB1, bool VEC>
__global__ void __launch_bounds__(64 * Mma<T>::kWaves)
mux_kernel(MuxArgs a) {
  constexpr int kWaves = Mma<T>::kWaves;
  constexpr bool kLds = sizeof(T) == 4;
  typedef typename Mma<T>::acc_t acc_t;
  typedef typename Mma<T>::quad_t quad_t;
  extern __shared__ __align__(16) unsigned char smem[];
  T *Ssh = reinterpret_cast<T *>(smem);  // [16 ceil(M/16)][sstr], zero padded
  const T *__restrict__ S = static_cast<const T *>(a.S);
  const int lane = threadIdx.x & 63, g = lane >> 4, i16 = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (a.active != nullptr && a.active[a.vol] == 0) return;  // frozen volume (uniform)
  const int M = a.M, P = a.P, MT = (M + 15) / 16;
  const int str = a.sstr;
  if constexpr (kLds) {
    for (int e = threadIdx.x; e < 16 * MT * str; e += 64 * kWaves) {
      const int i = e / str, j = e - (e / str) * str;
      Ssh[e] = (i < M && j < P) ? S[(long long)i * P + j] : T(0);
    }
    __syncthreads();
  }
  // first product, row tile rt, k block b: lane holds S[16 rt + row_of(i16)][16 b + 4 g + s], s = 0..3
  auto a1 = [&](int rt, int b) -> quad_t {
    const int i = 16 * rt + Mma<T>::row_of(i16), j = 16 * b + 4 * g;
    if constexpr (kLds) {
      return *reinterpret_cast<const quad_t *>(Ssh + i * str + j);
    } else {
      quad_t v;
#pragma unroll
      for (int st = 0; st < 4; ++st) v[st] = (i < M && j + st < P) ? S[(long long)i * P + j + st] : T(0);
      return v;
    }
  };
  // second product (S^T), row tile jt, k block b, step s: S[16 b + 4 g + s][16 jt + row_of(i16)]
  auto a2 = [&](int jt, int b, int st) -> T {
    const int i = 16 * b + 4 * g + st, j = 16 * jt + Mma<T>::row_of(i16);
    if constexpr (kLds) return Ssh[i * str + j];
    else return (i < M && j < P) ? S[(long long)i * P + j] : T(0);
  };

  const long long ncol = (long long)a.nt * a.ntiles;
  const int ntile16 = (int)((ncol + 15) / 16);
  const T *m = static_cast<const T *>(a.in);
  const T *yv = static_cast<const T *>(MODE == MUX_ADJ ? a.in : a.y);
  T *out = static_cast<T *>(a.out);
  const uint32_t nti = (uint32_t)a.ntiles;
  double fit = 0.0;
  for (int q = blockIdx.x * kWaves + wave; q < ntile16; q += gridDim.x * kWaves) {
    const Column cl = column(a, 16LL * q + i16, ncol);
    // X columns as the first product's B operands
    quad_t xb[MODE == MUX_ADJ ? 1 : KB1];
    if constexpr (MODE != MUX_ADJ) {
#pragma unroll
      for (int b = 0; b < KB1; ++b) {
        const int j0 = 16 * b + 4 * g;
        if constexpr (VEC) {
          // P is a multiple of 4: a quad is wholly inside or outside; loads
          // outside read element 0 and are discarded (no branch)
          const bool in = cl.valid && j0 < P;
          const quad_t v = ld<quad_t>(m, in ? cl.base + pos_off32(j0, a.tx, a.nx) : 0u);
          xb[b] = in ? v : quad_t(0);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const bool in = cl.valid && j0 + e < P;
            const T v = ld<T>(m, in ? cl.base + pos_off32(j0 + e, a.tx, a.nx) : 0u);
            xb[b][e] = in ? v : T(0);
          }
        }
      }
    }
    // the second product accumulates as each row tile of U is formed
    acc_t rv[MODE == MUX_FWD ? 1 : KB1];
#pragma unroll
    for (int jt = 0; jt < (MODE == MUX_FWD ? 1 : KB1); ++jt) rv[jt] = acc_t(0);
    // one row tile of U at a time (the loop is not unrolled: only this
    // tile's fragments of S are in flight); the first product's chain is
    // split over even and odd k blocks and the second product's steps cycle
    // through its accumulators, so consecutive MFMAs are independent
#pragma unroll 1
    for (int b = 0; b < MT; ++b) {
      acc_t ub = acc_t(0);
      if constexpr (MODE != MUX_ADJ) {
        acc_t uo = acc_t(0);
        // k blocks past P hold zero fragments of S and zero X (no branch)
#pragma unroll
        for (int kb = 0; kb < KB1; ++kb) {
          const quad_t av = a1(b, kb);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            if (kb & 1) uo = Mma<T>::step(av[e], xb[kb][e], uo);
            else ub = Mma<T>::step(av[e], xb[kb][e], ub);
          }
        }
        ub += uo;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * b + 4 * g + r;
        const bool live = i < M && cl.valid;
        const uint32_t yo = cl.ybase + (uint32_t)i * nti;
        if constexpr (MODE == MUX_FWD) {
          if (live) st<T>(out, yo, ub[r]);
        } else if constexpr (MODE == MUX_ADJ) {
          const T v = ld<T>(yv, live ? yo : 0u);
          ub[r] = live ? v : T(0);
        } else {
          const T d = yv ? ld<T>(yv, live ? yo : 0u) : T(0);
          const T v = live ? ub[r] - d : T(0);
          ub[r] = v;
          fit += 0.5 * (double)v * (double)v;
        }
      }
      if constexpr (MODE != MUX_FWD) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
#pragma unroll
          for (int jt = 0; jt < KB1; ++jt) rv[jt] = Mma<T>::step(a2(jt, b, e), ub[e], rv[jt]);
        }
      }
    }
    if constexpr (MODE != MUX_FWD) {
      if (cl.valid) {
#pragma unroll
        for (int jt = 0; jt < KB1; ++jt) {
          const int j0 = 16 * jt + 4 * g;
          if constexpr (VEC) {
            if (j0 < P) st<quad_t>(out, cl.base + pos_off32(j0, a.tx, a.nx), rv[jt]);
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (j0 + r < P) st<T>(out, cl.base + pos_off32(j0 + r, a.tx, a.nx), rv[jt][r]);
          }
        }
      }
    }
  }
  if constexpr (MODE == MUX_NORMAL) {
    if (a.partials) {
      // fixed-order sums: lanes by a butterfly, wavefronts in index order
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) fit += __shfl_xor(fit, off, 64);
      __syncthreads();  // S is no longer read: its LDS holds the wavefront sums
      double *red = reinterpret_cast<double *>(smem);
      if (lane == 0) red[wave] = fit;
      __syncthreads();
      if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < kWaves; ++w) tot += red[w];
        double *part = a.partials + (a.ctr ? (size_t)(*a.ctr) * a.part_stride : 0);
        for (int b = blockIdx.x; b < a.npart; b += gridDim.x) {
          part[2 * (size_t)b] = b == (int)blockIdx.x ? tot : 0.0;
          part[2 * (size_t)b + 1] = 0.0;
        }
      }
    }
  }
}

inline int kblocks(int k) {
  const int b = (k + 15) / 16;
  return b <= 1 ? 1 : b <= 2 ? 2 : b <= 4 ? 4 : 8;
}

// LDS row stride of S (elements): the padded width plus 4 (conflict-free A
// reads) when the copy then fits in 64 KB
inline int lds_stride(int M, int P) {
  const int cols = 16 * kblocks(P), rows = 16 * ((M + 15) / 16);
  return (size_t)rows * (cols + 4) * 4 <= 65536 ? cols + 4 : cols;
}

template <typename T, int MODE, int KB1>
hipError_t launch_one(const MuxArgs &a, int blocks, size_t lds, hipStream_t st) {
  if ((a.tx & 3) == 0 && (a.nx & 3) == 0)
    hipLaunchKernelGGL((mux_kernel<T, MODE, KB1, true>), dim3((unsigned)blocks), dim3(64 * Mma<T>::kWaves), lds, st,
                       a);
  else
    hipLaunchKernelGGL((mux_kernel<T, MODE, KB1, false>), dim3((unsigned)blocks), dim3(64 * Mma<T>::kWaves), lds,
                       st, a);
  return hipGetLastError();
}

template <typename T, int MODE>
hipError_t launch_kb1(const MuxArgs &a, int blocks, size_t lds, hipStream_t st) {
  switch (kblocks(a.P)) {
    case 1: return launch_one<T, MODE, 1>(a, blocks, lds, st);
    case 2: return launch_one<T, MODE, 2>(a, blocks, lds, st);
    case 4: return launch_one<T, MODE, 4>(a, blocks, lds, st);
    default: return launch_one<T, MODE, 8>(a, blocks, lds, st);
  }
}

}  // namespace

int mux_default_blocks(const MuxArgs &a, bool f64) {
  const int waves = f64 ? Mma<double>::kWaves : Mma<float>::kWaves;
  const long long tiles16 = ((long long)a.nt * a.ntiles + 15) / 16;
  const long long need = (tiles16 + waves - 1) / waves;
  const long long cap = f64 ? 1024 : 256;  // FP32: one 1024-thread block per compute unit
  return (int)std::min<long long>(std::max<long long>(need, 1), cap);
}

hipError_t launch_mux(int mode, bool f64, const MuxArgs &a_in, int blocks, hipStream_t st) {
  if (a_in.M < 1 || a_in.P < 1 || a_in.M > kMuxMaxDim || a_in.P > kMuxMaxDim || blocks < 1)
    return hipErrorInvalidValue;
  MuxArgs a = a_in;
  if (a.partials && a.npart < blocks) return hipErrorInvalidValue;
  a.sstr = lds_stride(a.M, a.P);
  const size_t lds = std::max<size_t>(f64 ? 0 : (size_t)16 * ((a.M + 15) / 16) * a.sstr * sizeof(float),
                                      (size_t)(f64 ? Mma<double>::kWaves : Mma<float>::kWaves) * sizeof(double));
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
