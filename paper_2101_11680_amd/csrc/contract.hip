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
// One workgroup streams one matrix for one pair of volumes (the FP32/FP64
// forward splits the matrix into up to four runs of t rows, one workgroup
// each, which shortens the drain at the end of the launch): the matrix is the A operand,
// the pair's 2 x 8 real columns fill the 16 B columns of an MFMA 16x16x4
// (FP32, FP64) or 16x16x32 (BF16) tile.  A single volume leaves the second
// half empty.  With several pairs (volumes of one shape class share
// the kernel spectrum) the workgroups of one matrix are mapped to the same
// XCD, so the matrix comes from HBM once and from that XCD's L2 afterwards;
// with one pair it is streamed with non-temporal loads (read once per pass:
// the kernel spectrum is the dominant HBM traffic of an iteration).  The reduction dimension is assigned so
// that every lane reads a contiguous run of the matrix row (vector loads):
// in k-step kk, lane group g = lane/16 carries index g * KC + kk.
//
// Layouts (element type by precision):
//   khat fwd / adj   per matrix, fragment order (see Frag): each 16-byte
//                    vector load reads one contiguous 1 KB run per wave,
//                    streamed with non-temporal loads (read once per pass)
//   mu side    [ky][kx][re/im][nzp]  t side [ky][kx][re/im][ntp]
#include "ctof_internal.h"

#include <algorithm>

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
template <typename T, int N, bool NT>
__device__ __forceinline__ void load_frag(const T *__restrict__ blk, int lane, T (&v)[N]) {
  constexpr int PER = 16 / sizeof(T);
  static_assert(N % PER == 0, "fragments are whole 16-byte words");
#pragma unroll
  for (int q = 0; q < N / PER; ++q) {
    const T *p = blk + ((size_t)q * 64 + lane) * PER;
    if constexpr (sizeof(T) == 4) {
      const nt_f4 w = NT ? __builtin_nontemporal_load(reinterpret_cast<const nt_f4 *>(p))
                         : *reinterpret_cast<const nt_f4 *>(p);
      v[q * 4 + 0] = w[0];
      v[q * 4 + 1] = w[1];
      v[q * 4 + 2] = w[2];
      v[q * 4 + 3] = w[3];
    } else {
      const nt_d2 w = NT ? __builtin_nontemporal_load(reinterpret_cast<const nt_d2 *>(p))
                         : *reinterpret_cast<const nt_d2 *>(p);
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

// Launch geometry shared by all contraction kernels.
struct CArgs {
  const void *khat, *khat_lo;  // forward or adjoint layout (bf16: hi and lo parts)
  const void *vin;
  void *vout;
  int h, p, nzp, ntp, nmat;
  int nvol, npairs;
  int parts;          // blocks per (matrix, pair): forward, each a contiguous run of t tiles; adjoint,
                      // each a contiguous run of bin chunks writing its partial sums to output part `part`
  size_t pstride;     // adjoint: elements between the output spectra of consecutive parts
  const int *active;  // per volume, 0 = frozen (no loads, no stores); NULL = all live
  const int *band;    // per matrix {lo, hi, zend, 0}: 16-bin tiles [lo, hi) and layers [0, zend)
                      // holding its significant entries; NULL = all
};

// Tiles [lo, hi) and layers [0, zend) of matrix s inside the band (all of
// [0, ntt) x [0, nzp) without one).  BAND: the kernel is launched with a band
// table; kernels without one compile without any of its logic.
template <bool BAND>
__device__ inline void band_of(const CArgs &a, int s, int ntt, int &lo, int &hi, int &zend) {
  lo = 0;
  hi = ntt;
  zend = a.nzp;
  if (BAND) {
    const int4 b = *reinterpret_cast<const int4 *>(a.band + 4 * s);
    lo = b.x;
    hi = b.y;
    zend = b.z;
  }
}

// Block -> (matrix, pair, part): block L runs on XCD L % 8; all pairs and
// parts of matrix s get blocks with the same residue so they share an L2.
__device__ inline bool map_block(const CArgs &a, int &s, int &pair, int &part) {
  const int L = blockIdx.x;
  const int xcd = L & 7;
  const int r = L >> 3;
  const int q = r / a.parts;
  part = r - q * a.parts;
  const int grp = q / a.npairs;
  pair = q - grp * a.npairs;
  s = grp * 8 + xcd;
  return s < a.nmat;
}

// Column c of the B tile: volume 2 pair + c/8, slot (c%8)/2, real/imag c%2.
struct Col {
  int f, vol, reim;
  bool on;
};

__device__ inline Col column_of(const CArgs &a, int s, int pair, int c) {
  Col k;
  k.vol = 2 * pair + (c >> 3);
  const int cc = c & 7;
  k.reim = cc & 1;
  bool ok;
  k.f = matrix_slot(s, a.h, a.p, cc >> 1, ok);
  k.on = ok && k.vol < a.nvol && (a.active == nullptr || a.active[k.vol] != 0);
  return k;
}

// true when neither volume of the pair takes part (the block has no work)
__device__ inline bool pair_idle(const CArgs &a, int pair) {
  if (a.active == nullptr) return false;
  const int v0 = 2 * pair, v1 = 2 * pair + 1;
  const bool on0 = v0 < a.nvol && a.active[v0] != 0;
  const bool on1 = v1 < a.nvol && a.active[v1] != 0;
  return !on0 && !on1;
}

// ---- FP32 / FP64, forward: M = t (tiles of 16), K = z --------------------------
template <typename T, int KZ, bool NT, bool BAND>
__global__ void __launch_bounds__(256)
contract_fwd_kernel(CArgs a) {
  using M = Mfma<T>;
  int s, pair, part;
  if (!map_block(a, s, pair, part) || pair_idle(a, pair)) return;
  const int w = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  const int c = l & 15, g = l >> 4;
  const Col k = column_of(a, s, pair, c);
  const int nzp = a.nzp, ntp = a.ntp;
  const int nchunk = nzp / (4 * KZ);
  const T *vcol = reinterpret_cast<const T *>(a.vin) + ((size_t)k.f * 2 + k.reim) * a.nvol * nzp +
                  (size_t)k.vol * nzp;
  T *ocol = reinterpret_cast<T *>(a.vout) + ((size_t)k.f * 2 + k.reim) * a.nvol * ntp +
            (size_t)k.vol * ntp;
  const T *khat = reinterpret_cast<const T *>(a.khat);
  const int ntt = ntp / 16;
  int blo0, bhi0, zend;
  band_of<BAND>(a, s, ntt, blo0, bhi0, zend);
  for (int ch = 0; ch < nchunk; ++ch) {
    // layer chunks past the band's layers add nothing (the first one still
    // runs: it writes the tiles)
    if (BAND && ch > 0 && ch * 4 * KZ >= zend) break;
    // this lane group's layers hold significant entries
    const bool zon = !BAND || ch * 4 * KZ + g * KZ < zend;
    T bv[KZ];
    if (k.on) {
      load_run<T, KZ>(vcol + ch * 4 * KZ + g * KZ, bv);
    } else {
#pragma unroll
      for (int kk = 0; kk < KZ; ++kk) bv[kk] = (T)0;
    }
    // the next tile's kernel fragment is loaded before the current one's
    // products, so each wave keeps a tile of loads in flight
    auto frag = [&](int tt) { return khat + (((size_t)s * ntt + tt) * nchunk + ch) * (64 * KZ); };
    auto tile = [&](int tt, const T (&av)[KZ]) {
      const int t0 = tt * 16;
      typename M::acc_t acc = {0, 0, 0, 0};
      if (ch > 0 && k.on) {
        // accumulate onto the previous layer chunk's partial result
        const T *o = ocol + t0 + 4 * g;
        acc[0] = o[0]; acc[1] = o[1]; acc[2] = o[2]; acc[3] = o[3];
      }
#pragma unroll
      for (int kk = 0; kk < KZ; ++kk) acc = M::step(av[kk], bv[kk], acc);
      if (k.on) store4<T>(ocol + t0 + 4 * g, acc);
    };
    // this block's run of t tiles, restricted to the matrix's band; tiles
    // outside it are written as zeros (with the first layer chunk)
    const int r0 = part * ntt / a.parts, r1 = (part + 1) * ntt / a.parts;
    const int blo = max(blo0, r0);
    const int bhi = max(blo, min(bhi0, r1));
    if (ch == 0 && k.on && (blo > r0 || bhi < r1)) {
      const typename M::acc_t zero = {0, 0, 0, 0};
      for (int zt = r0 + w; zt < r1; zt += 4)
        if (zt < blo || zt >= bhi) store4<T>(ocol + zt * 16 + 4 * g, zero);
    }
    const int tend = bhi;
    // lane groups past the band's layers read nothing and multiply zeros
    auto fetch = [&](int t, T (&av)[KZ]) {
      if (!BAND || zon) {
        load_frag<T, KZ, NT>(frag(t), l, av);
      } else {
#pragma unroll
        for (int kk = 0; kk < KZ; ++kk) av[kk] = (T)0;
      }
    };
    T a0[KZ], a1[KZ];
    int tt = blo + w;
    if (tt < tend) fetch(tt, a0);
    for (; tt < tend; tt += 8) {
      if (tt + 4 < tend) fetch(tt + 4, a1);
      tile(tt, a0);
      if (tt + 4 >= tend) break;
      if (tt + 8 < tend) fetch(tt + 8, a0);
      tile(tt + 4, a1);
    }
  }
}

// ---- FP32 / FP64 adjoint without a band: software-pipelined form ---------------
// The steady state of each wave's loop is straight-line code: every load of
// the next chunk is issued unconditionally (columns without a frequency read
// a valid address and multiply zeros), so the compiler's wait before a
// chunk's products covers exactly that chunk's loads and the next chunk's
// loads stay in flight during the products (conditional loads made it wait
// for the prefetched chunk as well).  The sums are taken in the same order
// as in contract_adj_kernel.  (The same form of the forward was slower: its
// output stores, interleaved with the kernel-spectrum reads, dominate.)

// FP32 / FP64 adjoint: wave w takes bin chunks c0 + w, c0 + w + 4, ... of
// the block's run; partial products of the four waves are summed in a fixed
// order through LDS.
template <typename T, int ZT, bool NT>
__global__ void __launch_bounds__(256)
contract_adj_pipe_kernel(CArgs a) {
  using M = Mfma<T>;
  extern __shared__ unsigned char smem_raw[];
  T *red = reinterpret_cast<T *>(smem_raw);  // [4 waves][ZT][64 lanes][4]
  int s, pair, part;
  if (!map_block(a, s, pair, part) || pair_idle(a, pair)) return;
  const int w = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  const int c = l & 15, g = l >> 4;
  const Col k = column_of(a, s, pair, c);
  const int nzp = a.nzp, ntp = a.ntp;
  const T *vcol = k.on ? reinterpret_cast<const T *>(a.vin) + ((size_t)k.f * 2 + k.reim) * a.nvol * ntp +
                             (size_t)k.vol * ntp + 4 * g
                       : reinterpret_cast<const T *>(a.vin);
  const int vstep = k.on ? 16 : 0;
  const T *khat = reinterpret_cast<const T *>(a.khat);
  typename M::acc_t acc[ZT];
#pragma unroll
  for (int zt = 0; zt < ZT; ++zt) acc[zt] = {0, 0, 0, 0};
  const int nch = ntp / 16;
  const int c0 = part * nch / a.parts, c1 = (part + 1) * nch / a.parts;
  const int ch0 = c0 + w;
  const int n = ch0 < c1 ? (c1 - ch0 + 3) / 4 : 0;
  auto load_chunk = [&](int ch, T (&av)[ZT][4], T (&bv)[4]) {
    load_run<T, 4>(vcol + ch * vstep, bv);
#pragma unroll
    for (int zt = 0; zt < ZT; ++zt) load_frag<T, 4, NT>(khat + (((size_t)s * nch + ch) * ZT + zt) * 256, l, av[zt]);
  };
  auto mul_chunk = [&](const T (&av)[ZT][4], const T (&bv)[4]) {
    T b[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) b[kk] = k.on ? bv[kk] : (T)0;
#pragma unroll
    for (int zt = 0; zt < ZT; ++zt)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) acc[zt] = M::step(av[zt][kk], b[kk], acc[zt]);
  };
  if (n > 0) {
    T a0[ZT][4], a1[ZT][4], b0[4], b1[4];
    load_chunk(ch0, a0, b0);
    int i = 0;
    for (; i + 2 < n; i += 2) {
      load_chunk(ch0 + 4 * (i + 1), a1, b1);
      __builtin_amdgcn_sched_barrier(0);
      mul_chunk(a0, b0);
      __builtin_amdgcn_sched_barrier(0);
      load_chunk(ch0 + 4 * (i + 2), a0, b0);
      __builtin_amdgcn_sched_barrier(0);
      mul_chunk(a1, b1);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (i + 1 < n) {
      load_chunk(ch0 + 4 * (i + 1), a1, b1);
      __builtin_amdgcn_sched_barrier(0);
      mul_chunk(a0, b0);
      mul_chunk(a1, b1);
    } else {
      mul_chunk(a0, b0);
    }
  }
#pragma unroll
  for (int zt = 0; zt < ZT; ++zt)
#pragma unroll
    for (int r = 0; r < 4; ++r) red[((w * ZT + zt) * 64 + l) * 4 + r] = acc[zt][r];
  __syncthreads();
  if (w == 0 && k.on) {
    T *ocol = reinterpret_cast<T *>(a.vout) + (size_t)part * a.pstride +
              ((size_t)k.f * 2 + k.reim) * a.nvol * nzp + (size_t)k.vol * nzp;
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

// ---- FP32 / FP64, adjoint: M = z (tiles of 16), K = t (chunks of 16) -----------
template <typename T, int ZT, bool NT, bool BAND>
__global__ void __launch_bounds__(256)
contract_adj_kernel(CArgs a) {
  using M = Mfma<T>;
  extern __shared__ unsigned char smem_raw[];
  T *red = reinterpret_cast<T *>(smem_raw);  // [4 waves][ZT][64 lanes][4]
  int s, pair, part;
  if (!map_block(a, s, pair, part) || pair_idle(a, pair)) return;
  const int w = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  const int c = l & 15, g = l >> 4;
  const Col k = column_of(a, s, pair, c);
  const int nzp = a.nzp, ntp = a.ntp;
  const T *vcol = reinterpret_cast<const T *>(a.vin) + ((size_t)k.f * 2 + k.reim) * a.nvol * ntp +
                  (size_t)k.vol * ntp;
  const T *khat = reinterpret_cast<const T *>(a.khat);
  typename M::acc_t acc[ZT];
#pragma unroll
  for (int zt = 0; zt < ZT; ++zt) acc[zt] = {0, 0, 0, 0};
  // next chunk's kernel fragments and data are loaded before the current
  // chunk's products (one chunk of loads in flight per wave)
  const int nch = ntp / 16;
  // chunks of 16 bins and z tiles inside the matrix's band (the rest of the
  // sum is below the band's threshold; z tiles past it stay zero), and of
  // this block's run of chunks
  int c0, c1, zend;
  band_of<BAND>(a, s, nch, c0, c1, zend);
  c0 = max(c0, part * nch / a.parts);
  c1 = min(c1, (part + 1) * nch / a.parts);
  auto load_chunk = [&](int ch, T (&av)[ZT][4], T (&bv)[4]) {
    if (k.on) {
      load_run<T, 4>(vcol + ch * 16 + 4 * g, bv);
    } else {
      bv[0] = bv[1] = bv[2] = bv[3] = (T)0;
    }
#pragma unroll
    for (int zt = 0; zt < ZT; ++zt)
      if (!BAND || zt * 16 < zend) load_frag<T, 4, NT>(khat + (((size_t)s * nch + ch) * ZT + zt) * 256, l, av[zt]);
  };
  auto mul_chunk = [&](const T (&av)[ZT][4], const T (&bv)[4]) {
#pragma unroll
    for (int zt = 0; zt < ZT; ++zt)
      if (!BAND || zt * 16 < zend)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) acc[zt] = M::step(av[zt][kk], bv[kk], acc[zt]);
  };
  T a0[ZT][4], a1[ZT][4], b0[4], b1[4];
  int ch = c0 + w;
  if (ch < c1) load_chunk(ch, a0, b0);
  for (; ch < c1; ch += 8) {
    if (ch + 4 < c1) load_chunk(ch + 4, a1, b1);
    mul_chunk(a0, b0);
    if (ch + 4 >= c1) break;
    if (ch + 8 < c1) load_chunk(ch + 8, a0, b0);
    mul_chunk(a1, b1);
  }
  // sum the four waves' partial products (fixed order); output rows 4g..4g+3
  // of every tile sit in lane group g, so all 64 lanes take part
#pragma unroll
  for (int zt = 0; zt < ZT; ++zt)
#pragma unroll
    for (int r = 0; r < 4; ++r) red[((w * ZT + zt) * 64 + l) * 4 + r] = acc[zt][r];
  __syncthreads();
  if (w == 0 && k.on) {
    T *ocol = reinterpret_cast<T *>(a.vout) + (size_t)part * a.pstride +
              ((size_t)k.f * 2 + k.reim) * a.nvol * nzp + (size_t)k.vol * nzp;
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

template <bool NT>
__device__ __forceinline__ v8bf load_bf8(const __bf16 *p) {
  const nt_u4 u = NT ? __builtin_nontemporal_load(reinterpret_cast<const nt_u4 *>(p))
                     : *reinterpret_cast<const nt_u4 *>(p);
  v8bf r;
  __builtin_memcpy(&r, &u, 16);
  return r;
}

template <int KIND, int KZ, bool NT, bool BAND>  // KZ: z per lane group per chunk (multiple of 8)
__global__ void __launch_bounds__(256)
contract_fwd_bf16_kernel(CArgs a) {
  int s, pair, part;
  if (!map_block(a, s, pair, part) || pair_idle(a, pair)) return;
  const int w = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  const int c = l & 15, g = l >> 4;
  const Col k = column_of(a, s, pair, c);
  const int nzp = a.nzp, ntp = a.ntp;
  const int nchunk = nzp / (4 * KZ);
  const float *vcol = reinterpret_cast<const float *>(a.vin) +
                      ((size_t)k.f * 2 + k.reim) * a.nvol * nzp + (size_t)k.vol * nzp;
  float *ocol = reinterpret_cast<float *>(a.vout) + ((size_t)k.f * 2 + k.reim) * a.nvol * ntp +
                (size_t)k.vol * ntp;
  const __bf16 *khi = reinterpret_cast<const __bf16 *>(a.khat);
  const __bf16 *klo = reinterpret_cast<const __bf16 *>(a.khat_lo);
  const int ntt = ntp / 16;
  int blo0, bhi0, zend;
  band_of<BAND>(a, s, ntt, blo0, bhi0, zend);
  for (int ch = 0; ch < nchunk; ++ch) {
    if (BAND && ch > 0 && ch * 4 * KZ >= zend) break;
    const bool zon = !BAND || ch * 4 * KZ + g * KZ < zend;
    // the lane group's KZ layers of its column, read in 16-byte words
    float vz[KZ];
    if (k.on) {
      load_run<float, KZ>(vcol + ch * 4 * KZ + g * KZ, vz);
    } else {
#pragma unroll
      for (int u = 0; u < KZ; ++u) vz[u] = 0.0f;
    }
    v8bf bh[KZ / 8], bl[KZ / 8];
#pragma unroll
    for (int e = 0; e < KZ / 8; ++e) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        __bf16 hi, lo;
        split_bf16(vz[e * 8 + u], hi, lo);
        bh[e][u] = hi;
        bl[e][u] = lo;
      }
    }
    const int r0 = part * ntt / a.parts, r1 = (part + 1) * ntt / a.parts;
    const int blo = max(blo0, r0);
    const int bhi = max(blo, min(bhi0, r1));
    if (ch == 0 && k.on && (blo > r0 || bhi < r1)) {
      for (int zt = r0 + w; zt < r1; zt += 4)
        if (zt < blo || zt >= bhi) *reinterpret_cast<float4 *>(ocol + zt * 16 + 4 * g) = make_float4(0, 0, 0, 0);
    }
    const int tend = bhi;
    constexpr int NF = KIND == 2 ? 2 : 1;  // fragments per layer group: hi (and lo)
    // the kernel fragments of tile tt (zeros past the band's layers)
    auto fetch = [&](int tt, v8bf (&af)[KZ / 8][NF]) {
      const size_t blk = (((size_t)s * ntt + tt) * nchunk + ch) * (64 * KZ);
#pragma unroll
      for (int e = 0; e < KZ / 8; ++e) {
        const size_t off = blk + ((size_t)e * 64 + l) * 8;
        const v8bf zero8 = {};
        af[e][0] = (!BAND || zon) ? load_bf8<NT>(khi + off) : zero8;
        if constexpr (KIND == 2) af[e][1] = (!BAND || zon) ? load_bf8<NT>(klo + off) : zero8;
      }
    };
    auto tile = [&](int tt, const v8bf (&af)[KZ / 8][NF]) {
      const int t0 = tt * 16;
      v4f acc = {0, 0, 0, 0};
      if (ch > 0 && k.on) {
        const float *o = ocol + t0 + 4 * g;
        acc[0] = o[0]; acc[1] = o[1]; acc[2] = o[2]; acc[3] = o[3];
      }
#pragma unroll
      for (int e = 0; e < KZ / 8; ++e) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[e][0], bh[e], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[e][0], bl[e], acc, 0, 0, 0);
        if constexpr (KIND == 2) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[e][1], bh[e], acc, 0, 0, 0);
      }
      if (k.on) *reinterpret_cast<float4 *>(ocol + t0 + 4 * g) = make_float4(acc[0], acc[1], acc[2], acc[3]);
    };
    // the next tile's fragments are loaded before the current one's
    // products, so each wave keeps a tile of loads in flight
    v8bf a0[KZ / 8][NF], a1[KZ / 8][NF];
    int tt = blo + w;
    if (tt < tend) fetch(tt, a0);
    for (; tt < tend; tt += 8) {
      if (tt + 4 < tend) fetch(tt + 4, a1);
      tile(tt, a0);
      if (tt + 4 >= tend) break;
      if (tt + 8 < tend) fetch(tt + 8, a0);
      tile(tt + 4, a1);
    }
  }
}

template <int KIND, int ZT, bool NT, bool BAND>
__global__ void __launch_bounds__(256)
contract_adj_bf16_kernel(CArgs a) {
  extern __shared__ unsigned char smem_raw[];
  float *red = reinterpret_cast<float *>(smem_raw);
  int s, pair, part;
  if (!map_block(a, s, pair, part) || pair_idle(a, pair)) return;
  const int w = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  const int c = l & 15, g = l >> 4;
  const Col k = column_of(a, s, pair, c);
  const int nzp = a.nzp, ntp = a.ntp;
  const float *vcol = reinterpret_cast<const float *>(a.vin) +
                      ((size_t)k.f * 2 + k.reim) * a.nvol * ntp + (size_t)k.vol * ntp;
  const __bf16 *khi = reinterpret_cast<const __bf16 *>(a.khat);
  const __bf16 *klo = reinterpret_cast<const __bf16 *>(a.khat_lo);
  v4f acc[ZT];
#pragma unroll
  for (int zt = 0; zt < ZT; ++zt) acc[zt] = {0, 0, 0, 0};
  // chunks of 32 bins covering the matrix's band of 16-bin tiles
  int c0, c1, zend;
  band_of<BAND>(a, s, ntp / 16, c0, c1, zend);
  c0 = c0 / 2;
  c1 = (c1 + 1) / 2;
  for (int ch = c0 + w; ch < c1; ch += 4) {
    const int t0 = ch * 32 + 8 * g;
    v8bf bh, bl;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float v = k.on ? vcol[t0 + u] : 0.0f;
      __bf16 hi, lo;
      split_bf16(v, hi, lo);
      bh[u] = hi;
      bl[u] = lo;
    }
#pragma unroll
    for (int zt = 0; zt < ZT; ++zt) {
      if (BAND && zt * 16 >= zend) continue;  // z tiles past the band stay zero
      const size_t off = (((size_t)s * (ntp / 32) + ch) * ZT + zt) * 512 + (size_t)l * 8;
      const v8bf ah = load_bf8<NT>(khi + off);
      acc[zt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[zt], 0, 0, 0);
      acc[zt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[zt], 0, 0, 0);
      if (KIND == 2) {
        const v8bf al = load_bf8<NT>(klo + off);
        acc[zt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[zt], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int zt = 0; zt < ZT; ++zt)
#pragma unroll
    for (int r = 0; r < 4; ++r) red[((w * ZT + zt) * 64 + l) * 4 + r] = acc[zt][r];
  __syncthreads();
  if (w == 0 && k.on) {
    float *ocol = reinterpret_cast<float *>(a.vout) + ((size_t)k.f * 2 + k.reim) * a.nvol * nzp +
                  (size_t)k.vol * nzp;
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

template <typename T, bool NT, bool BAND>
hipError_t launch_plain(const ctof_kernel_s *k, bool adjoint, const CArgs &a, hipStream_t st) {
  const Dims &d = k->dims;
  const dim3 grid((unsigned)(8 * ((d.nmat + 7) / 8) * a.npairs * a.parts)), block(256);
  if constexpr (!BAND) {
    if (adjoint && (d.nzp / 16) <= 4) {
      const size_t shm = (size_t)4 * (d.nzp / 16) * 64 * 4 * sizeof(T);
      switch (d.nzp / 16) {
        case 1: hipLaunchKernelGGL((contract_adj_pipe_kernel<T, 1, NT>), grid, block, shm, st, a); break;
        case 2: hipLaunchKernelGGL((contract_adj_pipe_kernel<T, 2, NT>), grid, block, shm, st, a); break;
        case 3: hipLaunchKernelGGL((contract_adj_pipe_kernel<T, 3, NT>), grid, block, shm, st, a); break;
        case 4: hipLaunchKernelGGL((contract_adj_pipe_kernel<T, 4, NT>), grid, block, shm, st, a); break;
        default: return hipErrorInvalidValue;
      }
      return hipGetLastError();
    }
  }
  if (!adjoint) {
    const int kz = (d.nzp >= 64 ? 64 : d.nzp) / 4;
    switch (kz) {
      case 4: hipLaunchKernelGGL((contract_fwd_kernel<T, 4, NT, BAND>), grid, block, 0, st, a); break;
      case 8: hipLaunchKernelGGL((contract_fwd_kernel<T, 8, NT, BAND>), grid, block, 0, st, a); break;
      case 12: hipLaunchKernelGGL((contract_fwd_kernel<T, 12, NT, BAND>), grid, block, 0, st, a); break;
      case 16: hipLaunchKernelGGL((contract_fwd_kernel<T, 16, NT, BAND>), grid, block, 0, st, a); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    const int zt = d.nzp / 16;
    const size_t shm = (size_t)4 * zt * 64 * 4 * sizeof(T);
    switch (zt) {
      case 1: hipLaunchKernelGGL((contract_adj_kernel<T, 1, NT, BAND>), grid, block, shm, st, a); break;
      case 2: hipLaunchKernelGGL((contract_adj_kernel<T, 2, NT, BAND>), grid, block, shm, st, a); break;
      case 3: hipLaunchKernelGGL((contract_adj_kernel<T, 3, NT, BAND>), grid, block, shm, st, a); break;
      case 4: hipLaunchKernelGGL((contract_adj_kernel<T, 4, NT, BAND>), grid, block, shm, st, a); break;
      case 8: hipLaunchKernelGGL((contract_adj_kernel<T, 8, NT, BAND>), grid, block, shm, st, a); break;
      case 12: hipLaunchKernelGGL((contract_adj_kernel<T, 12, NT, BAND>), grid, block, shm, st, a); break;
      case 16: hipLaunchKernelGGL((contract_adj_kernel<T, 16, NT, BAND>), grid, block, shm, st, a); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

// BF16 split adjoint without a band, software-pipelined as
// contract_adj_pipe_kernel: every load of a wave's next 32-bin chunk (its
// residual values and the chunk's hi / lo fragments) is issued before the
// current chunk's products, unconditionally (columns without a frequency
// read a valid address and multiply zeros).  The products are taken in the
// order of contract_adj_bf16_kernel, so the results are bitwise the same.
template <int KIND, int ZT, bool NT>
__global__ void __launch_bounds__(256)
contract_adj_bf16_pipe_kernel(CArgs a) {
  extern __shared__ unsigned char smem_raw[];
  float *red = reinterpret_cast<float *>(smem_raw);
  int s, pair, part;
  if (!map_block(a, s, pair, part) || pair_idle(a, pair)) return;
  const int w = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  const int c = l & 15, g = l >> 4;
  const Col k = column_of(a, s, pair, c);
  const int nzp = a.nzp, ntp = a.ntp;
  const float *vcol = k.on ? reinterpret_cast<const float *>(a.vin) + ((size_t)k.f * 2 + k.reim) * a.nvol * ntp +
                                 (size_t)k.vol * ntp + 8 * g
                           : reinterpret_cast<const float *>(a.vin);
  const int vstep = k.on ? 32 : 0;
  const __bf16 *khi = reinterpret_cast<const __bf16 *>(a.khat);
  const __bf16 *klo = reinterpret_cast<const __bf16 *>(a.khat_lo);
  constexpr int NF = KIND == 2 ? 2 : 1;  // fragments per z tile: hi (and lo)
  v4f acc[ZT];
#pragma unroll
  for (int zt = 0; zt < ZT; ++zt) acc[zt] = {0, 0, 0, 0};
  const int nch = ntp / 32;
  const int ch0 = w;
  const int n = ch0 < nch ? (nch - ch0 + 3) / 4 : 0;
  auto load_chunk = [&](int ch, v8bf (&af)[ZT][NF], float (&bv)[8]) {
    load_run<float, 8>(vcol + ch * vstep, bv);
#pragma unroll
    for (int zt = 0; zt < ZT; ++zt) {
      const size_t off = (((size_t)s * nch + ch) * ZT + zt) * 512 + (size_t)l * 8;
      af[zt][0] = load_bf8<NT>(khi + off);
      if constexpr (KIND == 2) af[zt][1] = load_bf8<NT>(klo + off);
    }
  };
  auto mul_chunk = [&](const v8bf (&af)[ZT][NF], const float (&bv)[8]) {
    v8bf bh, bl;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      __bf16 hi, lo;
      split_bf16(k.on ? bv[u] : 0.0f, hi, lo);
      bh[u] = hi;
      bl[u] = lo;
    }
#pragma unroll
    for (int zt = 0; zt < ZT; ++zt) {
      acc[zt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[zt][0], bh, acc[zt], 0, 0, 0);
      acc[zt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[zt][0], bl, acc[zt], 0, 0, 0);
      if constexpr (KIND == 2) acc[zt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[zt][1], bh, acc[zt], 0, 0, 0);
    }
  };
  if (n > 0) {
    v8bf a0[ZT][NF], a1[ZT][NF];
    float b0[8], b1[8];
    load_chunk(ch0, a0, b0);
    int i = 0;
    for (; i + 2 < n; i += 2) {
      load_chunk(ch0 + 4 * (i + 1), a1, b1);
      __builtin_amdgcn_sched_barrier(0);
      mul_chunk(a0, b0);
      __builtin_amdgcn_sched_barrier(0);
      load_chunk(ch0 + 4 * (i + 2), a0, b0);
      __builtin_amdgcn_sched_barrier(0);
      mul_chunk(a1, b1);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (i + 1 < n) {
      load_chunk(ch0 + 4 * (i + 1), a1, b1);
      __builtin_amdgcn_sched_barrier(0);
      mul_chunk(a0, b0);
      mul_chunk(a1, b1);
    } else {
      mul_chunk(a0, b0);
    }
  }
#pragma unroll
  for (int zt = 0; zt < ZT; ++zt)
#pragma unroll
    for (int r = 0; r < 4; ++r) red[((w * ZT + zt) * 64 + l) * 4 + r] = acc[zt][r];
  __syncthreads();
  if (w == 0 && k.on) {
    float *ocol = reinterpret_cast<float *>(a.vout) + ((size_t)k.f * 2 + k.reim) * a.nvol * nzp +
                  (size_t)k.vol * nzp;
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

template <int KIND, bool NT, bool BAND>
hipError_t launch_bf16(const ctof_kernel_s *k, bool adjoint, const CArgs &a0, hipStream_t st) {
  const Dims &d = k->dims;
  // the adjoints keep one block per matrix; the forwards split a matrix
  // into the handle's runs of bins (contract_parts)
  CArgs a = a0;
  if (adjoint) a.parts = 1;
  const dim3 grid((unsigned)(8 * ((d.nmat + 7) / 8) * a.npairs * a.parts)), block(256);
  if (!adjoint) {
    const int kz = (d.nzp >= 64 ? 64 : d.nzp) / 4;
    switch (kz) {
      case 8: hipLaunchKernelGGL((contract_fwd_bf16_kernel<KIND, 8, NT, BAND>), grid, block, 0, st, a); break;
      case 16: hipLaunchKernelGGL((contract_fwd_bf16_kernel<KIND, 16, NT, BAND>), grid, block, 0, st, a); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    const int zt = d.nzp / 16;
    const size_t shm = (size_t)4 * zt * 64 * 4 * sizeof(float);
    if constexpr (!BAND) {
      if (zt <= 4) {
        if (zt == 2) hipLaunchKernelGGL((contract_adj_bf16_pipe_kernel<KIND, 2, NT>), grid, block, shm, st, a);
        else if (zt == 4) hipLaunchKernelGGL((contract_adj_bf16_pipe_kernel<KIND, 4, NT>), grid, block, shm, st, a);
        else return hipErrorInvalidValue;
        return hipGetLastError();
      }
    }
    switch (zt) {
      case 2: hipLaunchKernelGGL((contract_adj_bf16_kernel<KIND, 2, NT, BAND>), grid, block, shm, st, a); break;
      case 4: hipLaunchKernelGGL((contract_adj_bf16_kernel<KIND, 4, NT, BAND>), grid, block, shm, st, a); break;
      case 8: hipLaunchKernelGGL((contract_adj_bf16_kernel<KIND, 8, NT, BAND>), grid, block, shm, st, a); break;
      case 12: hipLaunchKernelGGL((contract_adj_bf16_kernel<KIND, 12, NT, BAND>), grid, block, shm, st, a); break;
      case 16: hipLaunchKernelGGL((contract_adj_bf16_kernel<KIND, 16, NT, BAND>), grid, block, shm, st, a); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template <bool NT, bool BAND>
hipError_t dispatch_prec(const ctof_kernel_s *k, bool adjoint, const CArgs &a, hipStream_t st) {
  switch (k->prec) {
    case CTOF_FP64: return launch_plain<double, NT, BAND>(k, adjoint, a, st);
    case CTOF_FP32: return launch_plain<float, NT, BAND>(k, adjoint, a, st);
    case CTOF_BF16X3: return launch_bf16<2, NT, BAND>(k, adjoint, a, st);
    case CTOF_BF16: return launch_bf16<3, NT, BAND>(k, adjoint, a, st);
    default: return hipErrorInvalidValue;
  }
}

template <bool NT>
hipError_t dispatch(const ctof_kernel_s *k, bool adjoint, const CArgs &a, hipStream_t st) {
  if (a.band != nullptr) return dispatch_prec<NT, true>(k, adjoint, a, st);
  return dispatch_prec<NT, false>(k, adjoint, a, st);
}

}  // namespace

int contract_parts(const ctof_kernel_s *k, bool adjoint) {
  const Dims &d = k->dims;
  const bool bf = k->prec == CTOF_BF16X3 || k->prec == CTOF_BF16;
  if (k->band || (bf && adjoint)) return 1;  // (the BF16 adjoints keep one block per matrix)
  if (bf) {
    // the BF16 forwards: up to two blocks per matrix, at least 8 t tiles each
    // (each block splits its data columns into hi and lo parts, from 16-byte
    // loads; at 512 bins two blocks measured fastest for both forms)
    const int rule = std::max(1, std::min(2, d.ntp / 128));
    return k->fwd_parts > 0 ? std::max(1, std::min(k->fwd_parts, d.ntp / 16)) : rule;
  }
  if (!adjoint) {
    // up to four blocks per matrix, at least 8 t tiles (2 per wave) each:
    // shorter blocks shorten the tail of the launch
    const int rule = std::max(1, std::min(4, d.ntp / 128));
    return k->fwd_parts > 0 ? std::max(1, std::min(k->fwd_parts, d.ntp / 16)) : rule;
  }
  // the partial sums are added by the inverse column pass (FFT sizes <= 256)
  if (d.p > 256) return 1;
  return k->adj_parts > 0 ? std::max(1, std::min(k->adj_parts, d.ntp / 16)) : 1;
}

hipError_t launch_contract(const ctof_kernel_s *k, bool adjoint, const void *in, void *out,
                           hipStream_t st, int nvol, const int *active, size_t pstride) {
  const Dims &d = k->dims;
  const char *kh = reinterpret_cast<const char *>(k->khat);
  CArgs a;
  a.khat = kh + (adjoint ? k->layout.adj : k->layout.fwd);
  const size_t lo = adjoint ? k->layout.adj_lo : k->layout.fwd_lo;
  a.khat_lo = (k->prec == CTOF_BF16X3) ? kh + lo : a.khat;
  a.vin = in;
  a.vout = out;
  a.h = d.h;
  a.p = d.p;
  a.nzp = d.nzp;
  a.ntp = d.ntp;
  a.nmat = d.nmat;
  a.nvol = nvol;
  a.npairs = (nvol + 1) / 2;
  a.band = k->band;
  // (with a band most tiles are skipped, and one block per matrix avoids
  // blocks that only write zeros: 83 against 170 us at the benchmark shape)
  a.parts = contract_parts(k, adjoint);
  a.pstride = pstride;
  if (adjoint && a.parts > 1 && pstride == 0) return hipErrorInvalidValue;
  a.active = active;
  if (a.npairs == 1) return dispatch<true>(k, adjoint, a, st);
  return dispatch<false>(k, adjoint, a, st);
}

// ---- band of significant tiles ---------------------------------------------------
// The entries of a matrix's 16-bin tile (s, tt) are contiguous in the forward
// layout: elements [(s ntt + tt) 16 nzp, + 16 nzp).  Inside a tile, layer
// chunk ch holds 64 KZ elements in 16-byte words, word q of lane l at
// (64 q + l); lane group g = l / 16 carries the layers 4 KZ ch + KZ g ..
// + KZ - 1, layer group ch * 4 + g.  |x| of a non-negative float orders like
// its bit pattern as an unsigned integer, so an integer maximum over the bits
// is the float maximum (order-independent).
namespace {

template <typename E>
__device__ inline float mag(E x) {
  return fabsf((float)x);
}

template <typename E>
__global__ void __launch_bounds__(256) band_absmax_kernel(const E *__restrict__ k, size_t n, unsigned int *out) {
  __shared__ float red[256];
  float m = 0.f;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) m = fmaxf(m, mag(k[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, __float_as_uint(red[0]));
}

// One block per matrix: band[4 s] = first tile, band[4 s + 1] = one past the
// last tile, band[4 s + 2] = one past the last layer group, in layers (a
// multiple of kz), holding an entry >= rel * max |entry|; all 0 when none
// does.  Threads only ever set a flag to 1, so their stores may race.
template <typename E>
__global__ void __launch_bounds__(256) band_range_kernel(const E *__restrict__ k, int nmat, int ntt, int tile_elems,
                                                         int kz, double rel, const unsigned int *gmax, int *band) {
  constexpr int PER = 16 / (int)sizeof(E);
  __shared__ int ton[1024];
  __shared__ int zon[16];
  const int s = blockIdx.x;
  if (s >= nmat) return;
  for (int i = threadIdx.x; i < ntt; i += 256) ton[i] = 0;
  if (threadIdx.x < 16) zon[threadIdx.x] = 0;
  __syncthreads();
  const float thr = (float)(rel * (double)__uint_as_float(*gmax));
  const E *base = k + (size_t)s * ntt * tile_elems;
  const int chunk = 64 * kz;
  for (int tt = 0; tt < ntt; ++tt) {
    const E *t = base + (size_t)tt * tile_elems;
    for (int r = threadIdx.x; r < tile_elems; r += 256) {
      const float v = mag(t[r]);
      if (v >= thr && v > 0.f) {
        const int ch = r / chunk;
        const int lane = ((r - ch * chunk) / PER) & 63;
        ton[tt] = 1;
        zon[ch * 4 + (lane >> 4)] = 1;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int lo = -1, hi = -1, zg = 0;
    for (int tt = 0; tt < ntt; ++tt)
      if (ton[tt]) {
        if (lo < 0) lo = tt;
        hi = tt + 1;
      }
    for (int q = 0; q < 16; ++q)
      if (zon[q]) zg = q + 1;
    band[4 * s] = lo < 0 ? 0 : lo;
    band[4 * s + 1] = lo < 0 ? 0 : hi;
    band[4 * s + 2] = lo < 0 ? 0 : zg * kz;
    band[4 * s + 3] = 0;
  }
}

template <typename E>
hipError_t band_typed(const ctof_kernel_s *k, double rel, int *band, unsigned int *scratch, hipStream_t st) {
  const Dims &d = k->dims;
  const int ntt = d.ntp / 16;
  const int tile = 16 * d.nzp;
  // layers per lane group and chunk, as the forward kernels are launched
  const int kz = (d.nzp >= 64 ? 64 : d.nzp) / 4;
  if (d.nzp / kz > 16) return hipErrorInvalidValue;
  const E *kh = reinterpret_cast<const E *>(reinterpret_cast<const char *>(k->khat) + k->layout.fwd);
  const size_t n = (size_t)d.nmat * ntt * tile;
  hipError_t e = launch_fill_zero(scratch, sizeof(unsigned int), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(band_absmax_kernel<E>, dim3(2048), dim3(256), 0, st, kh, n, scratch);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(band_range_kernel<E>, dim3((unsigned)d.nmat), dim3(256), 0, st, kh, d.nmat, ntt, tile, kz, rel,
                     scratch, band);
  return hipGetLastError();
}

}  // namespace

int band_max_tiles() { return 1024; }

hipError_t launch_band(const ctof_kernel_s *k, double rel, int *band, unsigned int *scratch, hipStream_t st) {
  if (k->dims.ntp / 16 > band_max_tiles()) return hipErrorInvalidValue;
  switch (k->prec) {
    case CTOF_FP64: return band_typed<double>(k, rel, band, scratch, st);
    case CTOF_FP32: return band_typed<float>(k, rel, band, scratch, st);
    case CTOF_BF16X3:
    case CTOF_BF16: return band_typed<__bf16>(k, rel, band, scratch, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ctof
