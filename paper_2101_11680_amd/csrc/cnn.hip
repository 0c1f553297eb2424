// 3D convolution layers of the learned warm start (gfx950).
//
// A small 3D U-Net maps the scaled adjoint back-projection of a scan to a
// starting volume for the regularised least-squares iteration.  Activations
// are BF16, channels-last [n][d][h][w][ld]; a tensor is a channel slice
// [c0, c0 + c) of such a buffer, which is how skip concatenations are held
// without copies.  Accumulation is FP32.  Four layer kinds:
//   K3  3x3x3, stride 1, zero padding 1     (output grid = input grid)
//   DN  2x2x2, stride 2                     (output grid = input grid / 2)
//   UP  2x2x2 transposed, stride 2          (output grid = input grid * 2)
//   K1  1x1x1
// Packed weights (FP32 master and BF16 working copy share the layout):
//   K3, DN, K1: [co_pad][kpad], column k = tap * cip + ci
//   UP:         [8][co_pad][kpad], column k = ci
// with cip = roundup(ci, 8), co_pad = roundup(co, 16), kpad = roundup(taps *
// cip, 32) (taps = 27, 8, 1; 1 for UP, whose taps are the leading index);
// entries outside the real channels are zero.
//
// Forward is an implicit GEMM on the matrix cores: Y[pos][co] = sum_k
// W[co][k] X~[pos][k], X~ gathered on the fly, one 16x16x32 BF16 MFMA tile =
// 16 output channels x 16 positions x 32 columns.  The input gradient runs the
// same kernel with rearranged weights (K3: taps mirrored, channel roles
// swapped; a DN layer's input gradient is an UP layer and vice versa).  The
// weight gradient sums dY[pos][co] X~[pos][k] over positions in FP32 on the
// matrix cores, with per-wave partial sums reduced in a fixed order.
#include <cstdint>

#include "ctof_internal.h"

namespace ctof {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ v8bf load8(const __bf16 *p) {
  const uint4 u = *reinterpret_cast<const uint4 *>(p);
  v8bf r;
  __builtin_memcpy(&r, &u, 16);
  return r;
}

__device__ __forceinline__ v8bf zero8() {
  v8bf r;
#pragma unroll
  for (int i = 0; i < 8; ++i) r[i] = (__bf16)0.0f;
  return r;
}

struct Pos {
  int b, z, y, x;
};

__device__ __forceinline__ Pos unflatten(long long p, int d, int h, int w) {
  Pos q;
  q.x = (int)(p % w);
  p /= w;
  q.y = (int)(p % h);
  p /= h;
  q.z = (int)(p % d);
  q.b = (int)(p / d);
  return q;
}

__device__ __forceinline__ long long flat(int d, int h, int w, int b, int z, int y, int x) {
  return (((long long)b * d + z) * h + y) * w + x;
}

__device__ __forceinline__ void advance(Pos &q, int d, int h, int w) {
  if (++q.x == w) {
    q.x = 0;
    if (++q.y == h) {
      q.y = 0;
      if (++q.z == d) {
        q.z = 0;
        ++q.b;
      }
    }
  }
}

__host__ __device__ __forceinline__ int ntaps_of(int kind) {
  return kind == CNN_K3 ? 27 : (kind == CNN_DN ? 8 : 1);
}

// taps of the weight-gradient column space (UP's 8 taps included)
__host__ __device__ __forceinline__ int wg_taps(int kind) { return kind == CNN_UP ? 8 : ntaps_of(kind); }

// Row of the input feeding GEMM position q through `tap` (-1: zero padding).
// For K3/DN/K1 q runs over the output grid; for UP over the input grid.
__device__ __forceinline__ long long source_row(const ConvArgs &a, const Pos &q, int tap) {
  if (a.kind == CNN_K3) {
    const int zz = q.z + tap / 9 - 1, yy = q.y + (tap / 3) % 3 - 1, xx = q.x + tap % 3 - 1;
    if (zz < 0 || zz >= a.d || yy < 0 || yy >= a.h || xx < 0 || xx >= a.w) return -1;
    return flat(a.d, a.h, a.w, q.b, zz, yy, xx);
  }
  if (a.kind == CNN_DN)
    return flat(a.d, a.h, a.w, q.b, 2 * q.z + tap / 4, 2 * q.y + (tap / 2) % 2, 2 * q.x + tap % 2);
  return flat(a.d, a.h, a.w, q.b, q.z, q.y, q.x);
}

// Row of the output that GEMM position q feeds through `tap` (UP), else q.
__device__ __forceinline__ long long target_row(const ConvArgs &a, const Pos &q, long long qflat, int tap) {
  if (a.kind != CNN_UP) return qflat;
  return flat(2 * a.d, 2 * a.h, 2 * a.w, q.b, 2 * q.z + tap / 4, 2 * q.y + (tap / 2) % 2, 2 * q.x + tap % 2);
}

__device__ __forceinline__ void gemm_grid(const ConvArgs &a, int &gd, int &gh, int &gw) {
  if (a.kind == CNN_DN) {
    gd = a.d / 2;
    gh = a.h / 2;
    gw = a.w / 2;
  } else {
    gd = a.d;
    gh = a.h;
    gw = a.w;
  }
}

// ---- forward (and input-gradient) implicit GEMM ----------------------------------
// Block: 4 waves x 16 GEMM positions; a wave keeps CT accumulators of 16
// output channels.  For UP, blockIdx.y is the tap (it fixes the output parity).
template <int CT>
__global__ void __launch_bounds__(256)
conv_fwd_kernel(ConvArgs a) {
  const int wave = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  const int col = l & 15, g = l >> 4;
  int gd, gh, gw;
  gemm_grid(a, gd, gh, gw);
  const long long npos = (long long)a.n * gd * gh * gw;
  const long long qf = ((long long)blockIdx.x * 4 + wave) * 16 + col;
  const bool ok = qf < npos;
  const Pos q = unflatten(ok ? qf : 0, gd, gh, gw);
  const int tap_up = blockIdx.y;
  const int ntap = ntaps_of(a.kind);
  const __bf16 *wb = a.wt + (a.kind == CNN_UP ? (size_t)tap_up * a.co_pad * a.kpad : 0);
  v4f acc[CT];
#pragma unroll
  for (int t = 0; t < CT; ++t) acc[t] = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < a.kpad; k0 += 32) {
    const int k = k0 + 8 * g;  // this lane group's 8 consecutive columns
    const int tap = k / a.cip, ci = k - tap * a.cip;
    v8bf bx = zero8();
    if (ok && tap < ntap) {
      const long long src = source_row(a, q, tap);
      if (src >= 0) {
        bx = load8(a.x + (size_t)src * a.x_ld + a.x_c0 + ci);
        if (ci + 8 > a.ci) {
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (ci + u >= a.ci) bx[u] = (__bf16)0.0f;
        }
      }
    }
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      const v8bf aw = load8(wb + (size_t)(16 * t + col) * a.kpad + k);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw, bx, acc[t], 0, 0, 0);
    }
  }
  if (!ok) return;
  const long long dst = target_row(a, q, qf, tap_up);
#pragma unroll
  for (int t = 0; t < CT; ++t) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int co = 16 * t + 4 * g + r;
      if (co >= a.co) continue;
      float v = acc[t][r] + (a.bias ? a.bias[co] : 0.0f);
      const size_t o = (size_t)dst * a.y_ld + a.y_c0 + co;
      if (a.y_fp32) {
        float *yo = reinterpret_cast<float *>(a.y);
        if (a.accumulate) v += yo[o];
        if (a.relu) v = v > 0.0f ? v : 0.0f;
        yo[o] = v;
      } else {
        __bf16 *yo = reinterpret_cast<__bf16 *>(a.y);
        if (a.accumulate) v += (float)yo[o];
        if (a.relu) v = v > 0.0f ? v : 0.0f;
        yo[o] = (__bf16)v;
      }
    }
  }
}

constexpr int kK3Chunk = 32;  // input channels per LDS stage of the 3x3x3 kernels

// ---- forward (and input-gradient) 3x3x3 layers, staged in LDS -----------------------
// A block owns one spatial tile of ry whole rows of one plane, ry * w = 64 *
// NPT positions (NPT 16-position tiles per wave), and every output channel.
// Per 32-channel input chunk it copies the input halo (3 planes x (ry + 2)
// rows x (w + 2) columns x 32 channels, zero outside the grid and past ci)
// into LDS with 16-byte moves; each wave then runs the 27 taps with one
// 16-byte LDS read per position tile (8 channels of one position per lane:
// the B operand) and one 16-byte weight read per output-channel tile (the A
// operand, shared by the block's waves through L1), CT x NPT MFMAs per tap
// and chunk.
template <int CT, int NPT>
__global__ void __launch_bounds__(256)
conv_fwd_k3_kernel(ConvArgs a, int ry) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __bf16 *halo = reinterpret_cast<__bf16 *>(lds_raw);
  const int W2 = a.w + 2, R2 = ry + 2;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, col = l & 15, g = l >> 4;
  const int tiles_per_plane = a.h / ry;
  const long long plane = blockIdx.x / tiles_per_plane;
  const int y0 = (int)(blockIdx.x % tiles_per_plane) * ry;
  const int b = (int)(plane / a.d), z = (int)(plane % a.d);
  // this lane's position in each of its tiles
  int pr[NPT], px[NPT];
#pragma unroll
  for (int p = 0; p < NPT; ++p) {
    const int q = 16 * (wave * NPT + p) + col;
    pr[p] = q / a.w;
    px[p] = q - pr[p] * a.w;
  }
  v4f acc[NPT][CT];
#pragma unroll
  for (int p = 0; p < NPT; ++p)
#pragma unroll
    for (int t = 0; t < CT; ++t) acc[p][t] = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int cc0 = 0; cc0 < a.ci; cc0 += kK3Chunk) {
    __syncthreads();  // the previous chunk's halo is no longer read
    const int nsite = 3 * R2 * W2;
    for (int v = threadIdx.x; v < nsite * 4; v += 256) {
      const int site = v >> 2, q = v & 3;
      const int pl = site / (R2 * W2), rem = site - pl * (R2 * W2);
      const int hr = rem / W2, hc = rem - hr * W2;
      const int zz = z + pl - 1, yy = y0 + hr - 1, xx = hc - 1;
      const int c = cc0 + 8 * q;
      v8bf val = zero8();
      if (zz >= 0 && zz < a.d && yy >= 0 && yy < a.h && xx >= 0 && xx < a.w && c < a.ci) {
        const long long row = (((long long)b * a.d + zz) * a.h + yy) * a.w + xx;
        val = load8(a.x + (size_t)row * a.x_ld + a.x_c0 + c);
        if (c + 8 > a.ci) {
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (c + u >= a.ci) val[u] = (__bf16)0.0f;
        }
      }
      *reinterpret_cast<v8bf *>(halo + (size_t)site * kK3Chunk + 8 * q) = val;
    }
    __syncthreads();
    // weight columns of this lane group: tap * cip + cc0 + 8 g (none past cip)
    const int kc = cc0 + 8 * g;
    const bool kin = kc < a.cip;
    for (int tap = 0; tap < 27; ++tap) {
      const int dz = tap / 9, dyy = (tap / 3) % 3, dxx = tap % 3;
      v8bf bv[NPT];
#pragma unroll
      for (int p = 0; p < NPT; ++p)
        bv[p] = *reinterpret_cast<const v8bf *>(
            halo + ((size_t)(dz * R2 + pr[p] + dyy) * W2 + px[p] + dxx) * kK3Chunk + 8 * g);
#pragma unroll
      for (int t = 0; t < CT; ++t) {
        const v8bf aw = kin ? load8(a.wt + (size_t)(16 * t + col) * a.kpad + tap * a.cip + kc) : zero8();
#pragma unroll
        for (int p = 0; p < NPT; ++p)
          acc[p][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw, bv[p], acc[p][t], 0, 0, 0);
      }
    }
  }
  const long long row0 = ((long long)plane * a.h + y0) * a.w;
#pragma unroll
  for (int p = 0; p < NPT; ++p) {
    const long long dst = row0 + (long long)pr[p] * a.w + px[p];
#pragma unroll
    for (int t = 0; t < CT; ++t) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int co = 16 * t + 4 * g + r;
        if (co >= a.co) continue;
        float v = acc[p][t][r] + (a.bias ? a.bias[co] : 0.0f);
        const size_t o = (size_t)dst * a.y_ld + a.y_c0 + co;
        if (a.y_fp32) {
          float *yo = reinterpret_cast<float *>(a.y);
          if (a.accumulate) v += yo[o];
          if (a.relu) v = v > 0.0f ? v : 0.0f;
          yo[o] = v;
        } else {
          __bf16 *yo = reinterpret_cast<__bf16 *>(a.y);
          if (a.accumulate) v += (float)yo[o];
          if (a.relu) v = v > 0.0f ? v : 0.0f;
          yo[o] = (__bf16)v;
        }
      }
    }
  }
}

// ---- weight gradient --------------------------------------------------------------
// Tiles: (16 output channels) x (tap, 16 input channels).  A wave owns
// kWgTiles tiles of one output-channel tile over one range of GEMM positions
// and writes FP32 partial sums part[wpart][co_pad][taps][cit * 16];
// wgrad_reduce_kernel sums the parts in order into the packed weight layout.
constexpr int kWgTiles = 8;

__global__ void __launch_bounds__(256)
conv_wgrad_kernel(ConvArgs a, WgradArgs w) {
  const int wave = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  const int col = l & 15, g = l >> 4;
  const int part = blockIdx.x * 4 + wave;
  if (part >= w.nparts) return;
  const int taps = wg_taps(a.kind);
  const int cit = (a.ci + 15) / 16;
  const int ktiles = taps * cit;
  const int kgroups = (ktiles + kWgTiles - 1) / kWgTiles;
  const int cot = blockIdx.y / kgroups;
  const int kt0 = (blockIdx.y % kgroups) * kWgTiles;
  const int co0 = cot * 16;
  int gd, gh, gw;
  gemm_grid(a, gd, gh, gw);
  const long long npos = (long long)a.n * gd * gh * gw;
  const long long p_begin = (long long)part * w.per_part;
  const long long p_end = p_begin + w.per_part < npos ? p_begin + w.per_part : npos;
  const int co = co0 + col;
  v4f acc[kWgTiles];
#pragma unroll
  for (int t = 0; t < kWgTiles; ++t) acc[t] = {0.0f, 0.0f, 0.0f, 0.0f};
  for (long long p0 = p_begin; p0 < p_end; p0 += 32) {
    const long long qf0 = p0 + 8 * g;
    Pos qs[8];
    Pos q = unflatten(qf0 < npos ? qf0 : 0, gd, gh, gw);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      qs[j] = q;
      advance(q, gd, gh, gw);
    }
    v8bf av = zero8();
    if (a.kind != CNN_UP && co < a.co) {
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (qf0 + j < p_end) av[j] = w.dy[(size_t)(qf0 + j) * w.dy_ld + w.dy_c0 + co];
    }
#pragma unroll
    for (int t = 0; t < kWgTiles; ++t) {
      const int kt = kt0 + t;
      if (kt < ktiles) {
        const int tap = kt / cit;
        const int ci = (kt - tap * cit) * 16 + col;
        v8bf bv = zero8();
        if (a.kind == CNN_UP && co < a.co) {
#pragma unroll
          for (int j = 0; j < 8; ++j)
            if (qf0 + j < p_end)
              av[j] = w.dy[(size_t)target_row(a, qs[j], qf0 + j, tap) * w.dy_ld + w.dy_c0 + co];
        }
        if (ci < a.ci) {
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            if (qf0 + j < p_end) {
              const long long src = source_row(a, qs[j], tap);
              if (src >= 0) bv[j] = a.x[(size_t)src * a.x_ld + a.x_c0 + ci];
            }
          }
        }
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[t], 0, 0, 0);
      }
    }
  }
  const size_t rowlen = (size_t)taps * cit * 16;
  float *pp = w.part + (size_t)part * a.co_pad * rowlen;
#pragma unroll
  for (int t = 0; t < kWgTiles; ++t) {
    const int kt = kt0 + t;
    if (kt < ktiles) {
      const int tap = kt / cit;
      const int cc = (kt - tap * cit) * 16 + col;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        pp[(size_t)(co0 + 4 * g + r) * rowlen + (size_t)tap * cit * 16 + cc] = acc[t][r];
    }
  }
}

// ---- weight gradient of 3x3x3 layers, staged in LDS -----------------------------------
// A block owns one 16-channel output tile, one chunk of up to 32 input
// channels and a contiguous range of spatial tiles; a spatial tile is ry
// whole rows of one plane (ry * w positions, a multiple of 32).  Per tile
// the block copies the input halo (3 planes x (ry + 2) rows x (w + 2)
// columns x 32 channels, zero outside the grid) and dY (positions x 16
// channels) into LDS, channels-last, with 16-byte moves; each wave then adds
// its (tap, 16 input channels) tiles with one MFMA per 32 positions, both
// operands read from LDS (8 positions of one channel per lane).  Partial
// sums use the layout of conv_wgrad_kernel and the same reduction.
constexpr int kK3WaveTiles = 14;  // ceil(27 taps * 2 channel tiles / 4 waves)

__global__ void __launch_bounds__(256)
conv_wgrad_k3_kernel(ConvArgs a, WgradArgs w, int ry, long long ntiles, long long tpb) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __bf16 *halo = reinterpret_cast<__bf16 *>(lds_raw);
  const int W2 = a.w + 2, R2 = ry + 2;
  __bf16 *dys = halo + (size_t)3 * R2 * W2 * kK3Chunk;
  const int tpos = ry * a.w;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, col = l & 15, g = l >> 4;
  const int co_tiles = a.co_pad / 16;
  const int cot = blockIdx.y % co_tiles, chunk = blockIdx.y / co_tiles;
  const int co0 = cot * 16, cc0 = chunk * kK3Chunk;
  const int rem_ci = a.ci - cc0;
  const int citc = rem_ci >= 32 ? 2 : (rem_ci + 15) / 16;
  const int ntl = 27 * citc;
  const int tiles_per_plane = a.h / ry;
  const long long t_begin = (long long)blockIdx.x * tpb;
  const long long t_end = t_begin + tpb < ntiles ? t_begin + tpb : ntiles;
  v4f acc[kK3WaveTiles];
#pragma unroll
  for (int i = 0; i < kK3WaveTiles; ++i) acc[i] = {0.0f, 0.0f, 0.0f, 0.0f};
  for (long long st = t_begin; st < t_end; ++st) {
    const long long plane = st / tiles_per_plane;
    const int y0 = (int)(st % tiles_per_plane) * ry;
    const int b = (int)(plane / a.d), z = (int)(plane % a.d);
    __syncthreads();
    const int nsite = 3 * R2 * W2;
    for (int v = threadIdx.x; v < nsite * 4; v += 256) {
      const int site = v >> 2, q = v & 3;
      const int pl = site / (R2 * W2), rem = site - pl * (R2 * W2);
      const int hr = rem / W2, hc = rem - hr * W2;
      const int zz = z + pl - 1, yy = y0 + hr - 1, xx = hc - 1;
      const int c = cc0 + 8 * q;
      v8bf val = zero8();
      if (zz >= 0 && zz < a.d && yy >= 0 && yy < a.h && xx >= 0 && xx < a.w && c < a.ci) {
        const long long row = (((long long)b * a.d + zz) * a.h + yy) * a.w + xx;
        val = load8(a.x + (size_t)row * a.x_ld + a.x_c0 + c);
        if (c + 8 > a.ci) {
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (c + u >= a.ci) val[u] = (__bf16)0.0f;
        }
      }
      *reinterpret_cast<v8bf *>(halo + (size_t)site * kK3Chunk + 8 * q) = val;
    }
    const long long prow0 = ((long long)plane * a.h + y0) * a.w;
    for (int v = threadIdx.x; v < tpos * 2; v += 256) {
      const int pp = v >> 1, q = v & 1;
      const int co = co0 + 8 * q;
      v8bf val = zero8();
      const __bf16 *src = w.dy + (size_t)(prow0 + pp) * w.dy_ld + w.dy_c0 + co;
      if (co + 8 <= a.co) {
        val = load8(src);
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (co + u < a.co) val[u] = src[u];
      }
      *reinterpret_cast<v8bf *>(dys + (size_t)pp * 16 + 8 * q) = val;
    }
    __syncthreads();
    for (int s = 0; s < tpos / 32; ++s) {
      const int q0 = 32 * s + 8 * g;
      const int r = q0 / a.w, x0 = q0 - r * a.w;
      v8bf av;
#pragma unroll
      for (int j = 0; j < 8; ++j) av[j] = dys[(size_t)(q0 + j) * 16 + col];
#pragma unroll
      for (int i = 0; i < kK3WaveTiles; ++i) {
        const int t = wave + 4 * i;
        if (t < ntl) {
          const int tap = t / citc, cib = t - tap * citc;
          const int dz = tap / 9, dyy = (tap / 3) % 3, dxx = tap % 3;
          const __bf16 *hb = halo + ((size_t)(dz * R2 + r + dyy) * W2 + x0 + dxx) * kK3Chunk + cib * 16 + col;
          v8bf bv;
#pragma unroll
          for (int j = 0; j < 8; ++j) bv[j] = hb[j * kK3Chunk];
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[i], 0, 0, 0);
        }
      }
    }
  }
  const int cit = (a.ci + 15) / 16;
  const size_t rowlen = (size_t)27 * cit * 16;
  float *pp = w.part + (size_t)blockIdx.x * a.co_pad * rowlen;
#pragma unroll
  for (int i = 0; i < kK3WaveTiles; ++i) {
    const int t = wave + 4 * i;
    if (t < ntl) {
      const int tap = t / citc, cib = t - tap * citc;
      const int ci = cc0 + cib * 16 + col;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr)
        pp[(size_t)(co0 + 4 * g + rr) * rowlen + (size_t)tap * cit * 16 + ci] = acc[i][rr];
    }
  }
}

// dw (packed layout) = sum over parts.  T threads per element (a power of
// two dividing 256): thread t sums parts t, t + T, ... in order, then the T
// sums are added pairwise in a fixed tree (deterministic).
__global__ void __launch_bounds__(256)
wgrad_reduce_kernel(ConvArgs a, const float *__restrict__ part, int nparts, size_t elems, int T,
                    float *__restrict__ dw) {
  __shared__ float red[256];
  const int per_block = 256 / T;
  const int t = threadIdx.x % T;
  const size_t e = (size_t)blockIdx.x * per_block + threadIdx.x / T;
  const int taps = wg_taps(a.kind);
  const int cit = (a.ci + 15) / 16;
  int co, tap, ci;
  if (a.kind == CNN_UP) {
    tap = (int)(e / ((size_t)a.co_pad * a.kpad));
    const size_t r = e % ((size_t)a.co_pad * a.kpad);
    co = (int)(r / a.kpad);
    ci = (int)(r % a.kpad);
  } else {
    co = (int)(e / a.kpad);
    const int k = (int)(e % a.kpad);
    tap = k / a.cip;
    ci = k - tap * a.cip;
  }
  float s = 0.0f;
  if (e < elems && co < a.co && tap < taps && ci < a.ci) {
    const size_t rowlen = (size_t)taps * cit * 16;
    const size_t off = (size_t)co * rowlen + (size_t)tap * cit * 16 + ci;
    const size_t stride = (size_t)a.co_pad * rowlen;
    for (int p = t; p < nparts; p += T) s += part[(size_t)p * stride + off];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = T / 2; k > 0; k >>= 1) {
    if (t < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (t == 0 && e < elems) dw[e] = red[threadIdx.x];
}

// Bias gradient: per-block partial sums over a range of output rows, then a
// fixed-order sum over blocks.
constexpr int kBiasBlocks = 2048;

__global__ void __launch_bounds__(256)
bias_partial_kernel(const __bf16 *__restrict__ dy, int ld, int c0, long long nrows, int co, long long per,
                    float *__restrict__ part) {
  __shared__ float red[16][17];
  const int c16 = threadIdx.x & 15, rr = threadIdx.x >> 4;
  const long long r0 = (long long)blockIdx.x * per;
  const long long r1 = r0 + per < nrows ? r0 + per : nrows;
  for (int cb = 0; cb < co; cb += 16) {
    const int c = cb + c16;
    float s = 0.0f;
    if (c < co)
      for (long long r = r0 + rr; r < r1; r += 16) s += (float)dy[(size_t)r * ld + c0 + c];
    red[rr][c16] = s;
    __syncthreads();
    if (rr == 0) {
      float t = 0.0f;
      for (int i = 0; i < 16; ++i) t += red[i][c16];
      if (c < co) part[(size_t)blockIdx.x * co + c] = t;
    }
    __syncthreads();
  }
}

// Block c: thread b loads partial b of channel c; fixed-order tree sum.
__global__ void __launch_bounds__(256)
bias_reduce_kernel(const float *__restrict__ part, int nblk, int co, float *__restrict__ db) {
  __shared__ float red[256];
  const int c = blockIdx.x;
  float s = 0.0f;
  for (int b = threadIdx.x; b < nblk; b += 256) s += part[(size_t)b * co + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[c] = red[0];
}

// Input-gradient weights t from forward weights f (layouts of the file header):
//   K3 -> K3: wt[ci][tap][co] = w[co][26 - tap][ci]      K1 -> K1: wt[ci][co] = w[co][ci]
//   DN -> UP: wt[tap][ci][co] = w[co][tap][ci]          UP -> DN: wt[ci][tap][co] = w[tap][co][ci]
__global__ void transpose_weights_kernel(ConvArgs f, ConvArgs t, const __bf16 *__restrict__ w,
                                         __bf16 *__restrict__ wt, size_t elems) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= elems) return;
  int oc, tap, ic;  // target output channel (forward ci), tap, target input channel (forward co)
  if (t.kind == CNN_UP) {
    tap = (int)(e / ((size_t)t.co_pad * t.kpad));
    const size_t r = e % ((size_t)t.co_pad * t.kpad);
    oc = (int)(r / t.kpad);
    ic = (int)(r % t.kpad);
  } else {
    oc = (int)(e / t.kpad);
    const int k = (int)(e % t.kpad);
    tap = k / t.cip;
    ic = k - tap * t.cip;
  }
  float v = 0.0f;
  if (oc < t.co && ic < t.ci && tap < wg_taps(t.kind)) {
    size_t s;
    if (f.kind == CNN_K3) s = (size_t)ic * f.kpad + (size_t)(26 - tap) * f.cip + oc;
    else if (f.kind == CNN_K1) s = (size_t)ic * f.kpad + oc;
    else if (f.kind == CNN_DN) s = (size_t)ic * f.kpad + (size_t)tap * f.cip + oc;
    else s = ((size_t)tap * f.co_pad + ic) * f.kpad + oc;
    v = (float)w[s];
  }
  wt[e] = (__bf16)v;
}

// dy[row][c] = 0 where y[row][c] <= 0
__global__ void relu_mask_kernel(__bf16 *__restrict__ dy, int dld, int dc0, const __bf16 *__restrict__ y, int yld,
                                 int yc0, long long nrows, int ch) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows * ch) return;
  const long long r = i / ch;
  const int c = (int)(i - r * ch);
  if (!((float)y[(size_t)r * yld + yc0 + c] > 0.0f)) dy[(size_t)r * dld + dc0 + c] = (__bf16)0.0f;
}

// Mean squared error of ys * (channel yc0 of an FP32 tensor) against a dense
// FP32 target: gradient 2 ys (ys y - t) / n into a BF16 slice (zero where
// y <= 0 when relu_mask: y is then a ReLU output), FP64 partial sums.
__global__ void __launch_bounds__(256)
mse_kernel(const float *__restrict__ y, int yld, int yc0, float ys, const float *__restrict__ tg, long long n,
           __bf16 *__restrict__ g, int gld, int gc0, int relu_mask, double *__restrict__ part) {
  __shared__ double red[256];
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double e = 0.0;
  if (i < n) {
    const float yi = y[(size_t)i * yld + yc0];
    const float d = ys * yi - tg[i];
    e = (double)d * (double)d;
    g[(size_t)i * gld + gc0] = (relu_mask && !(yi > 0.0f)) ? (__bf16)0.0f : (__bf16)(2.0f * ys * d / (float)n);
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256)
mse_total_kernel(const double *__restrict__ part, int nblk, long long n, double *__restrict__ loss) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] / (double)n;
}

// Adam with bias correction on FP32 master weights; optional BF16 copy.
__global__ void adam_kernel(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, __bf16 *__restrict__ wb, long long n, float lr, float b1,
                            float b2, float eps, float c1, float c2, float gs) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i] * gs;
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  if (wb) wb[i] = (__bf16)wi;
}

// Dense FP32 volume -> BF16 channel c0 of rows of length ld (other channels
// of each row zeroed when zero_rest), times scale; with split, channel c0 + 1
// receives the BF16 rounding of the remainder (a hi/lo pair carrying ~16
// significant bits).
__global__ void to_channels_last_kernel(const float *__restrict__ x, long long n, float scale,
                                        __bf16 *__restrict__ out, int ld, int c0, int zero_rest, int split) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (zero_rest)
    for (int c = 0; c < ld; ++c)
      if (c != c0 && !(split && c == c0 + 1)) out[(size_t)i * ld + c] = (__bf16)0.0f;
  const float v = x[i] * scale;
  const __bf16 hi = (__bf16)v;
  out[(size_t)i * ld + c0] = hi;
  if (split) out[(size_t)i * ld + c0 + 1] = (__bf16)(v - (float)hi);
}

__global__ void from_channels_last_kernel(const float *__restrict__ y, int ld, int c0, long long n, float scale,
                                          float *__restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = y[(size_t)i * ld + c0] * scale;
}

// ---- warm-start training loss helpers --------------------------------------------
// e[b][i] = s_b * y[(b V + i) ld + c0] - t[b][i]
__global__ void start_error_kernel(const float *__restrict__ y, int ld, int c0, StartCoef cf, long long V,
                                   const float *__restrict__ t, long long n, float *__restrict__ e) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  e[i] = cf.s[i / V] * y[(size_t)i * ld + c0] - t[i];
}

// y[i] += a * x[i]
__global__ void axpy_kernel(long long n, float a, const float *__restrict__ x, float *__restrict__ y) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

// Block (c, b): FP64 partial sums of u^2 and v^2 over chunk c of sample b.
constexpr int kSqChunks = 64;
__global__ void __launch_bounds__(256)
sumsq_partial_kernel(const float *__restrict__ u, const float *__restrict__ v, long long V,
                     double *__restrict__ part) {
  __shared__ double ra[256], rb[256];
  const int c = blockIdx.x, b = blockIdx.y;
  const long long per = (V + kSqChunks - 1) / kSqChunks;
  const long long i0 = (long long)c * per, i1 = i0 + per < V ? i0 + per : V;
  double a = 0.0, q = 0.0;
  for (long long i = i0 + threadIdx.x; i < i1; i += 256) {
    const double x = u[(size_t)b * V + i], z = v[(size_t)b * V + i];
    a += x * x;
    q += z * z;
  }
  ra[threadIdx.x] = a;
  rb[threadIdx.x] = q;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      ra[threadIdx.x] += ra[threadIdx.x + k];
      rb[threadIdx.x] += rb[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((size_t)b * kSqChunks + c) * 2] = ra[0];
    part[((size_t)b * kSqChunks + c) * 2 + 1] = rb[0];
  }
}

__global__ void sumsq_total_kernel(const double *__restrict__ part, int nb, double *__restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  double a = 0.0, q = 0.0;
  for (int c = 0; c < kSqChunks; ++c) {
    a += part[((size_t)b * kSqChunks + c) * 2];
    q += part[((size_t)b * kSqChunks + c) * 2 + 1];
  }
  out[2 * b] = a;
  out[2 * b + 1] = q;
}

// grad[(b V + i) gld + gc0] = ch[b] u[b][i] + ce[b] e[b][i], zeroed where y <= 0
// when relu_mask
__global__ void start_grad_kernel(long long n, long long V, StartCoef cf, const float *__restrict__ u,
                                  const float *__restrict__ e, const float *__restrict__ y, int yld, int yc0,
                                  int relu_mask, __bf16 *__restrict__ g, int gld, int gc0) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int b = (int)(i / V);
  const float yi = y[(size_t)i * yld + yc0];
  const float v = (yi > 0.0f || !relu_mask) ? cf.ch[b] * u[i] + cf.ce[b] * e[i] : 0.0f;
  g[(size_t)i * gld + gc0] = (__bf16)v;
}

// Depth resampling of [nb][nz][plane] volumes by a factor 2:
// mode 0: out[b][j] = x[b][2j] + x[b][2j + 1]  (nz even, nz / 2 layers out)
// mode 1: out[b][k] = x[b][k / 2]              (2 nz layers out)
__global__ void depth_resample_kernel(const float *__restrict__ x, float *__restrict__ out, int nz_out,
                                      long long plane, long long n, int mode) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long p = i % plane;
  const long long bz = i / plane;
  const int k = (int)(bz % nz_out);
  const long long b = bz / nz_out;
  if (mode == 0) {
    const long long nz_in = 2LL * nz_out;
    const float *src = x + (b * nz_in + 2 * k) * plane + p;
    out[i] = src[0] + src[plane];
  } else {
    const long long nz_in = nz_out / 2;
    out[i] = x[(b * nz_in + k / 2) * plane + p];
  }
}

// Block (c, b): max |x| over chunk c of sample b; then per sample.
constexpr int kAbsChunks = 64;
__global__ void __launch_bounds__(256)
absmax_partial_kernel(const float *__restrict__ x, long long V, float *__restrict__ part) {
  __shared__ float red[256];
  const int c = blockIdx.x, b = blockIdx.y;
  const long long per = (V + kAbsChunks - 1) / kAbsChunks;
  const long long i0 = (long long)c * per, i1 = i0 + per < V ? i0 + per : V;
  float m = 0.0f;
  for (long long i = i0 + threadIdx.x; i < i1; i += 256) m = fmaxf(m, fabsf(x[(size_t)b * V + i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + k]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)b * kAbsChunks + c] = red[0];
}

__global__ void absmax_total_kernel(const float *__restrict__ part, int nb, float *__restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  float m = 0.0f;
  for (int c = 0; c < kAbsChunks; ++c) m = fmaxf(m, part[(size_t)b * kAbsChunks + c]);
  out[b] = m;
}

// mu[z][i] = 0 where |mu[z][i]| < frac * maxes[z]
__global__ void layer_threshold_kernel(float *__restrict__ mu, long long plane, long long n,
                                       const float *__restrict__ maxes, float frac) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float t = frac * maxes[i / plane];
  if (fabsf(mu[i]) < t) mu[i] = 0.0f;
}

inline unsigned blocks_for(long long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_layer_threshold(float *mu, int nz, long long plane, const float *maxes, float frac,
                                  hipStream_t st) {
  const long long n = (long long)nz * plane;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(layer_threshold_kernel, dim3(blocks_for(n)), dim3(256), 0, st, mu, plane, n, maxes, frac);
  return hipGetLastError();
}

size_t absmax_ws_bytes(int nb) { return (size_t)nb * kAbsChunks * sizeof(float); }

hipError_t launch_depth_resample(const float *x, float *out, int nb, int nz_in, long long plane, int mode,
                                 hipStream_t st) {
  const int nz_out = mode == 0 ? nz_in / 2 : 2 * nz_in;
  const long long n = (long long)nb * nz_out * plane;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(depth_resample_kernel, dim3(blocks_for(n)), dim3(256), 0, st, x, out, nz_out, plane, n, mode);
  return hipGetLastError();
}

hipError_t launch_absmax(const float *x, long long V, int nb, float *part, float *out, hipStream_t st) {
  if (V == 0 || nb == 0) return hipSuccess;
  hipLaunchKernelGGL(absmax_partial_kernel, dim3(kAbsChunks, (unsigned)nb), dim3(256), 0, st, x, V, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(absmax_total_kernel, dim3((unsigned)((nb + 63) / 64)), dim3(64), 0, st, part, nb, out);
  return hipGetLastError();
}

hipError_t launch_start_error(const float *y, int ld, int c0, const StartCoef &cf, long long V, const float *t,
                              long long n, float *e, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(start_error_kernel, dim3(blocks_for(n)), dim3(256), 0, st, y, ld, c0, cf, V, t, n, e);
  return hipGetLastError();
}

hipError_t launch_axpy(long long n, float a, const float *x, float *y, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(axpy_kernel, dim3(blocks_for(n)), dim3(256), 0, st, n, a, x, y);
  return hipGetLastError();
}

size_t sumsq_ws_bytes(int nb) { return (size_t)nb * kSqChunks * 2 * sizeof(double); }

hipError_t launch_sumsq(const float *u, const float *v, long long V, int nb, double *part, double *out,
                        hipStream_t st) {
  hipLaunchKernelGGL(sumsq_partial_kernel, dim3(kSqChunks, (unsigned)nb), dim3(256), 0, st, u, v, V, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sumsq_total_kernel, dim3(1), dim3(64), 0, st, part, nb, out);
  return hipGetLastError();
}

hipError_t launch_start_grad(long long n, long long V, const StartCoef &cf, const float *u, const float *e,
                             const float *y, int yld, int yc0, int relu_mask, __bf16 *g, int gld, int gc0,
                             hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(start_grad_kernel, dim3(blocks_for(n)), dim3(256), 0, st, n, V, cf, u, e, y, yld, yc0,
                     relu_mask, g, gld, gc0);
  return hipGetLastError();
}

int cnn_cip(int ci) { return (ci + 7) / 8 * 8; }
int cnn_copad(int co) { return (co + 15) / 16 * 16; }
int cnn_kpad(int kind, int ci) { return (ntaps_of(kind) * cnn_cip(ci) + 31) / 32 * 32; }
size_t cnn_weight_elems(int kind, int co, int ci) {
  return (size_t)(kind == CNN_UP ? 8 : 1) * cnn_copad(co) * cnn_kpad(kind, ci);
}

void conv_fill_layout(ConvArgs &a) {
  a.cip = cnn_cip(a.ci);
  a.co_pad = cnn_copad(a.co);
  a.kpad = cnn_kpad(a.kind, a.ci);
}

long long conv_gemm_positions(const ConvArgs &a) {
  if (a.kind == CNN_DN) return (long long)a.n * (a.d / 2) * (a.h / 2) * (a.w / 2);
  return (long long)a.n * a.d * a.h * a.w;
}

long long conv_output_rows(const ConvArgs &a) {
  if (a.kind == CNN_UP) return (long long)a.n * 8 * a.d * a.h * a.w;
  return conv_gemm_positions(a);
}

ConvArgs conv_transposed(const ConvArgs &f) {
  ConvArgs t{};
  t.kind = f.kind == CNN_DN ? CNN_UP : (f.kind == CNN_UP ? CNN_DN : f.kind);
  t.n = f.n;
  if (f.kind == CNN_DN) {
    t.d = f.d / 2;
    t.h = f.h / 2;
    t.w = f.w / 2;
  } else if (f.kind == CNN_UP) {
    t.d = 2 * f.d;
    t.h = 2 * f.h;
    t.w = 2 * f.w;
  } else {
    t.d = f.d;
    t.h = f.h;
    t.w = f.w;
  }
  t.ci = f.co;
  t.co = f.ci;
  conv_fill_layout(t);
  return t;
}

// Rows per tile of the LDS-staged 3x3x3 forward kernel (ry * w = 64 * npt),
// or false when the layer does not fit it (then the generic kernel runs):
// at least 32 input channels, rows of 8 to 64 columns, 16-byte rows.
static bool k3f_plan(const ConvArgs &a, int &ry, int &npt, size_t &lds) {
  const int ct = a.co_pad / 16;
  // below 32 input channels a 32-channel stage would be half empty (the
  // generic kernel packs the taps' channels densely into its k steps)
  if (a.kind != CNN_K3 || a.ci < kK3Chunk || a.w % 8 != 0 || (a.x_ld % 8) || (a.x_c0 % 8) || ct < 1 || ct > 4 ||
      (reinterpret_cast<uintptr_t>(a.x) & 15))
    return false;
  for (npt = 2; npt >= 1; --npt) {
    const int pos = 64 * npt;
    if (pos % a.w) continue;
    ry = pos / a.w;
    if (ry > a.h || a.h % ry) continue;
    lds = (size_t)3 * (ry + 2) * (a.w + 2) * kK3Chunk * sizeof(__bf16);
    if (lds <= 64 * 1024) return true;
  }
  return false;
}

template <int CT>
static void launch_k3f(const ConvArgs &a, int ry, int npt, size_t lds, unsigned blocks, hipStream_t st) {
  if (npt == 2)
    hipLaunchKernelGGL((conv_fwd_k3_kernel<CT, 2>), dim3(blocks), dim3(256), lds, st, a, ry);
  else
    hipLaunchKernelGGL((conv_fwd_k3_kernel<CT, 1>), dim3(blocks), dim3(256), lds, st, a, ry);
}

hipError_t launch_conv_fwd(const ConvArgs &a, hipStream_t st) {
  const long long npos = conv_gemm_positions(a);
  if (npos == 0) return hipSuccess;
  int ry, npt;
  size_t lds;
  if (k3f_plan(a, ry, npt, lds)) {
    const unsigned blocks = (unsigned)((long long)a.n * a.d * (a.h / ry));
    switch (a.co_pad / 16) {
      case 1: launch_k3f<1>(a, ry, npt, lds, blocks, st); break;
      case 2: launch_k3f<2>(a, ry, npt, lds, blocks, st); break;
      case 3: launch_k3f<3>(a, ry, npt, lds, blocks, st); break;
      default: launch_k3f<4>(a, ry, npt, lds, blocks, st); break;
    }
    return hipGetLastError();
  }
  const dim3 grid(blocks_for(npos, 64), a.kind == CNN_UP ? 8 : 1);
  switch (a.co_pad / 16) {
    case 1: hipLaunchKernelGGL(conv_fwd_kernel<1>, grid, dim3(256), 0, st, a); break;
    case 2: hipLaunchKernelGGL(conv_fwd_kernel<2>, grid, dim3(256), 0, st, a); break;
    case 3: hipLaunchKernelGGL(conv_fwd_kernel<3>, grid, dim3(256), 0, st, a); break;
    case 4: hipLaunchKernelGGL(conv_fwd_kernel<4>, grid, dim3(256), 0, st, a); break;
    case 8: hipLaunchKernelGGL(conv_fwd_kernel<8>, grid, dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

bool conv_co_supported(int co) {
  const int t = cnn_copad(co) / 16;
  return t == 1 || t == 2 || t == 3 || t == 4 || t == 8;
}

size_t conv_transposed_weight_bytes(const ConvArgs &f) {
  const ConvArgs t = conv_transposed(f);
  return cnn_weight_elems(t.kind, t.co, t.ci) * sizeof(__bf16);
}

hipError_t launch_transpose_weights(const ConvArgs &f, const __bf16 *w, __bf16 *wt, hipStream_t st) {
  const ConvArgs t = conv_transposed(f);
  const size_t elems = cnn_weight_elems(t.kind, t.co, t.ci);
  hipLaunchKernelGGL(transpose_weights_kernel, dim3(blocks_for((long long)elems)), dim3(256), 0, st, f, t, w, wt,
                     elems);
  return hipGetLastError();
}

static void wgrad_plan(const ConvArgs &a, int &nparts, long long &per_part, int &groups, size_t &part_elems) {
  const int taps = wg_taps(a.kind);
  const int cit = (a.ci + 15) / 16;
  const int ktiles = taps * cit;
  groups = (a.co_pad / 16) * ((ktiles + kWgTiles - 1) / kWgTiles);
  const long long npos = conv_gemm_positions(a);
  part_elems = (size_t)a.co_pad * taps * cit * 16;
  long long want = (4096 + groups - 1) / groups;
  if (want > 1024) want = 1024;
  const long long cap_mem = (long long)((size_t)(16u << 20) / part_elems);
  const long long cap_pos = (npos + 255) / 256;
  if (want > cap_mem) want = cap_mem;
  if (want > cap_pos) want = cap_pos;
  if (want < 1) want = 1;
  per_part = ((npos + want - 1) / want + 31) / 32 * 32;
  if (per_part < 32) per_part = 32;
  nparts = (int)((npos + per_part - 1) / per_part);
  if (nparts < 1) nparts = 1;
}

// Plan of the LDS-staged 3x3x3 weight gradient, or false when the layer
// does not fit it (then the generic kernel runs).
struct K3Plan {
  int ry, groups, nparts;
  long long ntiles, tpb;
  size_t lds;
};

static bool k3_plan(const ConvArgs &a, int dy_ld, int dy_c0, K3Plan &p) {
  if (a.kind != CNN_K3 || a.w % 8 != 0 || (dy_ld % 8) || (dy_c0 % 8)) return false;
  int ry = a.w >= 128 ? 1 : 128 / a.w;
  if (ry > a.h) ry = a.h;
  while (ry > 1 && a.h % ry) --ry;
  if ((ry * a.w) % 32 || a.h % ry) return false;
  p.ry = ry;
  p.lds = ((size_t)3 * (ry + 2) * (a.w + 2) * kK3Chunk + (size_t)ry * a.w * 16) * sizeof(__bf16);
  if (p.lds > 64 * 1024) return false;
  p.groups = (a.co_pad / 16) * ((a.ci + kK3Chunk - 1) / kK3Chunk);
  p.ntiles = (long long)a.n * a.d * (a.h / ry);
  const size_t part_elems = (size_t)a.co_pad * 27 * ((a.ci + 15) / 16) * 16;
  long long want = (2048 + p.groups - 1) / p.groups;
  const long long cap_mem = (long long)((size_t)(16u << 20) / part_elems);
  if (want > cap_mem) want = cap_mem;
  if (want > p.ntiles) want = p.ntiles;
  if (want < 1) want = 1;
  p.tpb = (p.ntiles + want - 1) / want;
  p.nparts = (int)((p.ntiles + p.tpb - 1) / p.tpb);
  return p.ntiles > 0;
}

size_t conv_wgrad_ws_bytes(const ConvArgs &a) {
  int nparts, groups;
  long long per;
  size_t part_elems;
  wgrad_plan(a, nparts, per, groups, part_elems);
  K3Plan kp;
  if (k3_plan(a, 8, 0, kp) && kp.nparts > nparts) nparts = kp.nparts;
  return ((size_t)nparts * part_elems + (size_t)kBiasBlocks * a.co) * sizeof(float);
}

hipError_t launch_conv_wgrad(const ConvArgs &a, const __bf16 *dy, int dy_ld, int dy_c0, float *dw, float *db,
                             float *ws, hipStream_t st) {
  int nparts, groups;
  long long per;
  size_t part_elems;
  wgrad_plan(a, nparts, per, groups, part_elems);
  const long long npos = conv_gemm_positions(a);
  const size_t elems = cnn_weight_elems(a.kind, a.co, a.ci);
  hipError_t e;
  K3Plan kp;
  const bool staged = npos > 0 && k3_plan(a, dy_ld, dy_c0, kp) &&
                      (reinterpret_cast<uintptr_t>(dy) & 15) == 0 && (reinterpret_cast<uintptr_t>(a.x) & 15) == 0;
  if (staged) {
    WgradArgs w{dy, dy_ld, dy_c0, ws, kp.nparts, 0};
    hipLaunchKernelGGL(conv_wgrad_k3_kernel, dim3((unsigned)kp.nparts, (unsigned)kp.groups), dim3(256), kp.lds, st,
                       a, w, kp.ry, kp.ntiles, kp.tpb);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    nparts = kp.nparts;
  } else if (npos > 0) {
    WgradArgs w{dy, dy_ld, dy_c0, ws, nparts, per};
    hipLaunchKernelGGL(conv_wgrad_kernel, dim3((unsigned)((nparts + 3) / 4), (unsigned)groups), dim3(256), 0, st,
                       a, w);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // threads per element: enough to keep about 64K threads busy, at most 64
  const int np_eff = npos > 0 ? nparts : 0;
  int T = 1;
  while (T < 64 && (size_t)T * elems < 65536 && T < np_eff) T *= 2;
  const size_t per_block = 256 / T;
  hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((unsigned)((elems + per_block - 1) / per_block)), dim3(256), 0, st,
                     a, ws, np_eff, elems, T, dw);
  e = hipGetLastError();
  if (e != hipSuccess || !db) return e;
  float *bpart = ws + (size_t)nparts * part_elems;
  const long long rows = conv_output_rows(a);
  const long long bper = rows > 0 ? (rows + kBiasBlocks - 1) / kBiasBlocks : 1;
  const int nblk = rows > 0 ? (int)((rows + bper - 1) / bper) : 0;
  if (nblk > 0) {
    hipLaunchKernelGGL(bias_partial_kernel, dim3((unsigned)nblk), dim3(256), 0, st, dy, dy_ld, dy_c0, rows, a.co,
                       bper, bpart);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(bias_reduce_kernel, dim3((unsigned)a.co), dim3(256), 0, st, bpart, nblk, a.co, db);
  return hipGetLastError();
}

hipError_t launch_relu_mask(__bf16 *dy, int dld, int dc0, const __bf16 *y, int yld, int yc0, long long nrows,
                            int ch, hipStream_t st) {
  if (nrows * ch == 0) return hipSuccess;
  hipLaunchKernelGGL(relu_mask_kernel, dim3(blocks_for(nrows * ch)), dim3(256), 0, st, dy, dld, dc0, y, yld, yc0,
                     nrows, ch);
  return hipGetLastError();
}

size_t mse_ws_bytes(long long n) { return (size_t)blocks_for(n) * sizeof(double); }

hipError_t launch_mse(const float *y, int yld, int yc0, float ys, const float *t, long long n, __bf16 *g, int gld,
                      int gc0, int relu_mask, double *part, double *loss, hipStream_t st) {
  const unsigned nb = blocks_for(n);
  hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(256), 0, st, y, yld, yc0, ys, t, n, g, gld, gc0, relu_mask, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mse_total_kernel, dim3(1), dim3(256), 0, st, part, (int)nb, n, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float *w, const float *g, float *m, float *v, __bf16 *wb, long long n, float lr, float b1,
                       float b2, float eps, int step, float gscale, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const float c1 = (float)(1.0 - pow((double)b1, (double)step));
  const float c2 = (float)(1.0 - pow((double)b2, (double)step));
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(256), 0, st, w, g, m, v, wb, n, lr, b1, b2, eps, c1,
                     c2, gscale);
  return hipGetLastError();
}

hipError_t launch_to_channels_last(const float *x, long long n, float scale, __bf16 *out, int ld, int c0,
                                   int zero_rest, int split, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(to_channels_last_kernel, dim3(blocks_for(n)), dim3(256), 0, st, x, n, scale, out, ld, c0,
                     zero_rest, split);
  return hipGetLastError();
}

hipError_t launch_from_channels_last(const float *y, int ld, int c0, long long n, float scale, float *out,
                                     hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(from_channels_last_kernel, dim3(blocks_for(n)), dim3(256), 0, st, y, ld, c0, n, scale, out);
  return hipGetLastError();
}

}  // namespace ctof
