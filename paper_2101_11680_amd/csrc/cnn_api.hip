// C ABI of the learned warm start's layers, loss, optimiser and sampler.
// Every entry point validates its arguments before enqueueing any work.
#include <cmath>
#include <cstdint>

#include "ctof_internal.h"

namespace {

using ctof::ConvArgs;
using ctof::set_error;

constexpr int kMaxChannels = 256;
constexpr long long kMaxRows = 1LL << 40;

ctof_status check_desc(const ctof_conv_desc *d) {
  if (!d) return set_error(CTOF_EINVAL, "conv descriptor is NULL");
  if (d->kind < CTOF_CONV_K3 || d->kind > CTOF_CONV_K1) return set_error(CTOF_EINVAL, "unknown conv kind %d", d->kind);
  if (d->n < 1 || d->d < 1 || d->h < 1 || d->w < 1) return set_error(CTOF_EINVAL, "grid sizes must be >= 1");
  // the row count, built up factor by factor so that no product overflows
  long long rows = d->kind == CTOF_CONV_UP ? 8 : 1;
  for (const int f : {d->n, d->d, d->h, d->w}) {
    if (f > kMaxRows / rows) return set_error(CTOF_EINVAL, "grid too large");
    rows *= f;
  }
  if (d->kind == CTOF_CONV_DN && ((d->d | d->h | d->w) & 1))
    return set_error(CTOF_EINVAL, "a stride-2 layer needs even d, h, w");
  if (d->ci < 1 || d->ci > kMaxChannels) return set_error(CTOF_EINVAL, "ci must be in [1, %d]", kMaxChannels);
  if (d->co < 1 || d->co > kMaxChannels) return set_error(CTOF_EINVAL, "co must be in [1, %d]", kMaxChannels);
  if (!ctof::conv_co_supported(d->co))
    return set_error(CTOF_EUNSUPPORTED, "co = %d: roundup(co, 16) / 16 must be 1, 2, 3, 4 or 8", d->co);
  return CTOF_OK;
}

ConvArgs args_of(const ctof_conv_desc *d) {
  ConvArgs a{};
  a.kind = d->kind;
  a.n = d->n;
  a.d = d->d;
  a.h = d->h;
  a.w = d->w;
  a.ci = d->ci;
  a.co = d->co;
  ctof::conv_fill_layout(a);
  return a;
}

// A BF16 slice of c channels read in whole 8-channel groups by 16-byte loads.
ctof_status check_read(const ctof_tensor *t, int c, const char *name) {
  if (!t || !t->ptr) return set_error(CTOF_EINVAL, "%s: tensor or pointer is NULL", name);
  if ((reinterpret_cast<uintptr_t>(t->ptr) & 15) != 0) return set_error(CTOF_EINVAL, "%s: pointer not 16-byte aligned", name);
  if (t->ld % 8 != 0 || t->c0 % 8 != 0 || t->c0 < 0)
    return set_error(CTOF_EINVAL, "%s: ld and c0 must be non-negative multiples of 8", name);
  if (t->c0 + ctof::cnn_cip(c) > t->ld) return set_error(CTOF_EINVAL, "%s: c0 + roundup(c, 8) exceeds ld", name);
  return CTOF_OK;
}

ctof_status check_write(const ctof_tensor *t, int c, int elem_bytes, const char *name) {
  if (!t || !t->ptr) return set_error(CTOF_EINVAL, "%s: tensor or pointer is NULL", name);
  if ((reinterpret_cast<uintptr_t>(t->ptr) % elem_bytes) != 0) return set_error(CTOF_EINVAL, "%s: misaligned pointer", name);
  if (t->c0 < 0 || t->ld < 1 || t->c0 + c > t->ld) return set_error(CTOF_EINVAL, "%s: slice exceeds the row", name);
  return CTOF_OK;
}

inline const __bf16 *bf(const void *p) { return reinterpret_cast<const __bf16 *>(p); }
inline __bf16 *bfw(void *p) { return reinterpret_cast<__bf16 *>(p); }

#define CHECK(expr)                  \
  do {                               \
    const ctof_status s_ = (expr);   \
    if (s_ != CTOF_OK) return s_;    \
  } while (0)

}  // namespace

extern "C" {

ctof_status ctof_conv3d_weight_elems(const ctof_conv_desc *desc, size_t *elems) {
  CHECK(check_desc(desc));
  if (!elems) return set_error(CTOF_EINVAL, "elems is NULL");
  *elems = ctof::cnn_weight_elems(desc->kind, desc->co, desc->ci);
  return CTOF_OK;
}

ctof_status ctof_conv3d_fwd(const ctof_conv_desc *desc, const ctof_tensor *x, const void *w_bf16, const float *bias,
                            const ctof_tensor *y, int32_t y_fp32, int32_t relu, int32_t accumulate,
                            hipStream_t stream) {
  CHECK(check_desc(desc));
  CHECK(check_read(x, desc->ci, "x"));
  CHECK(check_write(y, desc->co, y_fp32 ? 4 : 2, "y"));
  if (!w_bf16 || (reinterpret_cast<uintptr_t>(w_bf16) & 15)) return set_error(CTOF_EINVAL, "w: NULL or not 16-byte aligned");
  ConvArgs a = args_of(desc);
  a.x = bf(x->ptr);
  a.x_ld = x->ld;
  a.x_c0 = x->c0;
  a.wt = bf(w_bf16);
  a.bias = bias;
  a.y = y->ptr;
  a.y_ld = y->ld;
  a.y_c0 = y->c0;
  a.y_fp32 = y_fp32 ? 1 : 0;
  a.relu = relu ? 1 : 0;
  a.accumulate = accumulate ? 1 : 0;
  HIP_TRY(ctof::launch_conv_fwd(a, stream));
  return CTOF_OK;
}

ctof_status ctof_conv3d_bwd_data_ws_bytes(const ctof_conv_desc *desc, size_t *ws_bytes) {
  CHECK(check_desc(desc));
  if (!ws_bytes) return set_error(CTOF_EINVAL, "ws_bytes is NULL");
  *ws_bytes = (ctof::conv_transposed_weight_bytes(args_of(desc)) + 255) / 256 * 256;
  return CTOF_OK;
}

ctof_status ctof_conv3d_bwd_data(const ctof_conv_desc *desc, const ctof_tensor *dy, const void *w_bf16,
                                 const ctof_tensor *dx, int32_t accumulate, void *ws_dev, size_t ws_bytes,
                                 hipStream_t stream) {
  CHECK(check_desc(desc));
  if (!ctof::conv_co_supported(desc->ci))
    return set_error(CTOF_EUNSUPPORTED, "input gradient with ci = %d: roundup(ci, 16) / 16 must be 1, 2, 3, 4 or 8",
                     desc->ci);
  CHECK(check_read(dy, desc->co, "dy"));
  CHECK(check_write(dx, desc->ci, 2, "dx"));
  if (!w_bf16 || (reinterpret_cast<uintptr_t>(w_bf16) & 15)) return set_error(CTOF_EINVAL, "w: NULL or not 16-byte aligned");
  const ConvArgs f = args_of(desc);
  const size_t need = ctof::conv_transposed_weight_bytes(f);
  if (!ws_dev || (reinterpret_cast<uintptr_t>(ws_dev) & 15)) return set_error(CTOF_EINVAL, "workspace NULL or misaligned");
  if (ws_bytes < need) return set_error(CTOF_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
  ConvArgs t = ctof::conv_transposed(f);
  HIP_TRY(ctof::launch_transpose_weights(f, bf(w_bf16), bfw(ws_dev), stream));
  t.x = bf(dy->ptr);
  t.x_ld = dy->ld;
  t.x_c0 = dy->c0;
  t.wt = bf(ws_dev);
  t.bias = nullptr;
  t.y = dx->ptr;
  t.y_ld = dx->ld;
  t.y_c0 = dx->c0;
  t.y_fp32 = 0;
  t.relu = 0;
  t.accumulate = accumulate ? 1 : 0;
  HIP_TRY(ctof::launch_conv_fwd(t, stream));
  return CTOF_OK;
}

ctof_status ctof_conv3d_bwd_weight_ws_bytes(const ctof_conv_desc *desc, size_t *ws_bytes) {
  CHECK(check_desc(desc));
  if (!ws_bytes) return set_error(CTOF_EINVAL, "ws_bytes is NULL");
  *ws_bytes = (ctof::conv_wgrad_ws_bytes(args_of(desc)) + 255) / 256 * 256;
  return CTOF_OK;
}

ctof_status ctof_conv3d_bwd_weight(const ctof_conv_desc *desc, const ctof_tensor *x, const ctof_tensor *dy,
                                   float *dw_dev, float *db_dev, void *ws_dev, size_t ws_bytes,
                                   hipStream_t stream) {
  CHECK(check_desc(desc));
  CHECK(check_read(x, desc->ci, "x"));
  CHECK(check_write(dy, desc->co, 2, "dy"));
  if (!dw_dev) return set_error(CTOF_EINVAL, "dw is NULL");
  const ConvArgs base = args_of(desc);
  const size_t need = ctof::conv_wgrad_ws_bytes(base);
  if (!ws_dev || (reinterpret_cast<uintptr_t>(ws_dev) & 15)) return set_error(CTOF_EINVAL, "workspace NULL or misaligned");
  if (ws_bytes < need) return set_error(CTOF_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
  ConvArgs a = base;
  a.x = bf(x->ptr);
  a.x_ld = x->ld;
  a.x_c0 = x->c0;
  HIP_TRY(ctof::launch_conv_wgrad(a, bf(dy->ptr), dy->ld, dy->c0, dw_dev, db_dev, reinterpret_cast<float *>(ws_dev),
                                  stream));
  return CTOF_OK;
}

ctof_status ctof_relu_bwd(int64_t rows, int32_t ch, const ctof_tensor *dy, const ctof_tensor *y, hipStream_t stream) {
  if (rows < 0 || rows > kMaxRows || ch < 1 || ch > kMaxChannels) return set_error(CTOF_EINVAL, "bad rows / ch");
  CHECK(check_write(dy, ch, 2, "dy"));
  CHECK(check_write(y, ch, 2, "y"));
  HIP_TRY(ctof::launch_relu_mask(bfw(dy->ptr), dy->ld, dy->c0, bf(y->ptr), y->ld, y->c0, rows, ch, stream));
  return CTOF_OK;
}

ctof_status ctof_mse_ws_bytes(int64_t n, size_t *ws_bytes) {
  if (n < 1 || n > kMaxRows) return set_error(CTOF_EINVAL, "n must be >= 1");
  if (!ws_bytes) return set_error(CTOF_EINVAL, "ws_bytes is NULL");
  *ws_bytes = (ctof::mse_ws_bytes(n) + 255) / 256 * 256;
  return CTOF_OK;
}

ctof_status ctof_mse(int64_t n, const ctof_tensor *y, float y_scale, const float *target_dev, const ctof_tensor *grad,
                     int32_t relu_mask, double *loss_dev, void *ws_dev, size_t ws_bytes, hipStream_t stream) {
  if (n < 1 || n > kMaxRows) return set_error(CTOF_EINVAL, "n must be >= 1");
  CHECK(check_write(y, 1, 4, "y"));
  CHECK(check_write(grad, 1, 2, "grad"));
  if (!target_dev || !loss_dev) return set_error(CTOF_EINVAL, "target or loss is NULL");
  const size_t need = ctof::mse_ws_bytes(n);
  if (!ws_dev || (reinterpret_cast<uintptr_t>(ws_dev) & 7)) return set_error(CTOF_EINVAL, "workspace NULL or misaligned");
  if (ws_bytes < need) return set_error(CTOF_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
  if (!std::isfinite(y_scale)) return set_error(CTOF_EINVAL, "y_scale must be finite");
  HIP_TRY(ctof::launch_mse(reinterpret_cast<const float *>(y->ptr), y->ld, y->c0, y_scale, target_dev, n, bfw(grad->ptr),
                           grad->ld, grad->c0, relu_mask ? 1 : 0, reinterpret_cast<double *>(ws_dev),
                           loss_dev, stream));
  return CTOF_OK;
}

ctof_status ctof_adam_step(int64_t n, float *w_dev, const float *g_dev, float *m_dev, float *v_dev, void *w_bf16_dev,
                           float lr, float beta1, float beta2, float eps, int32_t step, hipStream_t stream) {
  if (n < 0 || n > kMaxRows) return set_error(CTOF_EINVAL, "bad n");
  if (!w_dev || !g_dev || !m_dev || !v_dev) return set_error(CTOF_EINVAL, "w, g, m or v is NULL");
  if (step < 1) return set_error(CTOF_EINVAL, "step counts from 1");
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f && lr >= 0.0f))
    return set_error(CTOF_EINVAL, "need 0 <= beta < 1, eps > 0, lr >= 0");
  HIP_TRY(ctof::launch_adam(w_dev, g_dev, m_dev, v_dev, bfw(w_bf16_dev), n, lr, beta1, beta2, eps, step, 1.0f,
                            stream));
  return CTOF_OK;
}

ctof_status ctof_adam_step_scaled(int64_t n, float *w_dev, const float *g_dev, float *m_dev, float *v_dev,
                                  void *w_bf16_dev, float lr, float beta1, float beta2, float eps, int32_t step,
                                  float grad_scale, hipStream_t stream) {
  if (!(grad_scale >= 0.0f && grad_scale <= 1e30f)) return set_error(CTOF_EINVAL, "grad_scale must be finite, >= 0");
  if (n < 0 || n > kMaxRows) return set_error(CTOF_EINVAL, "bad n");
  if (!w_dev || !g_dev || !m_dev || !v_dev) return set_error(CTOF_EINVAL, "w, g, m or v is NULL");
  if (step < 1) return set_error(CTOF_EINVAL, "step counts from 1");
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f && lr >= 0.0f))
    return set_error(CTOF_EINVAL, "need 0 <= beta < 1, eps > 0, lr >= 0");
  HIP_TRY(ctof::launch_adam(w_dev, g_dev, m_dev, v_dev, bfw(w_bf16_dev), n, lr, beta1, beta2, eps, step, grad_scale,
                            stream));
  return CTOF_OK;
}

ctof_status ctof_to_channels_last(int64_t n, const float *x_dev, float scale, const ctof_tensor *out,
                                  int32_t zero_rest, int32_t split, hipStream_t stream) {
  if (n < 0 || n > kMaxRows) return set_error(CTOF_EINVAL, "bad n");
  if (!x_dev) return set_error(CTOF_EINVAL, "x is NULL");
  CHECK(check_write(out, split ? 2 : 1, 2, "out"));
  HIP_TRY(ctof::launch_to_channels_last(x_dev, n, scale, bfw(out->ptr), out->ld, out->c0, zero_rest ? 1 : 0,
                                        split ? 1 : 0, stream));
  return CTOF_OK;
}

ctof_status ctof_from_channels_last(int64_t n, const ctof_tensor *y, float scale, float *out_dev, hipStream_t stream) {
  if (n < 0 || n > kMaxRows) return set_error(CTOF_EINVAL, "bad n");
  if (!out_dev) return set_error(CTOF_EINVAL, "out is NULL");
  CHECK(check_write(y, 1, 4, "y"));
  HIP_TRY(ctof::launch_from_channels_last(reinterpret_cast<const float *>(y->ptr), y->ld, y->c0, n, scale, out_dev,
                                          stream));
  return CTOF_OK;
}

ctof_status ctof_philox4x32(uint64_t seed, uint32_t stream_id, int64_t first, int64_t n, uint32_t *out_dev,
                            hipStream_t stream) {
  if (n < 0 || first < 0 || n > kMaxRows) return set_error(CTOF_EINVAL, "bad first / n");
  if (!out_dev || (reinterpret_cast<uintptr_t>(out_dev) & 15)) return set_error(CTOF_EINVAL, "out NULL or not 16-byte aligned");
  HIP_TRY(ctof::launch_philox(seed, stream_id, first, n, out_dev, stream));
  return CTOF_OK;
}

ctof_status ctof_poisson(int64_t n, const float *lam_dev, uint64_t seed, uint32_t stream_id, float *counts_dev,
                         hipStream_t stream) {
  if (n < 0 || n > kMaxRows) return set_error(CTOF_EINVAL, "bad n");
  if (!lam_dev || !counts_dev) return set_error(CTOF_EINVAL, "lam or counts is NULL");
  HIP_TRY(ctof::launch_poisson(lam_dev, n, seed, stream_id, counts_dev, stream));
  return CTOF_OK;
}

ctof_status ctof_noisy_histogram_ws_bytes(int64_t n, size_t *ws_bytes) {
  if (n < 0 || n > kMaxRows) return set_error(CTOF_EINVAL, "bad n");
  if (!ws_bytes) return set_error(CTOF_EINVAL, "ws_bytes is NULL");
  *ws_bytes = (ctof::noisy_histogram_ws_bytes(n) + 255) / 256 * 256;
  return CTOF_OK;
}

ctof_status ctof_noisy_histogram(int64_t n, const float *m_dev, double peak, uint64_t seed, uint32_t stream_id,
                                 float *d_dev, void *ws_dev, size_t ws_bytes, hipStream_t stream) {
  if (n < 0 || n > kMaxRows) return set_error(CTOF_EINVAL, "bad n");
  if (!m_dev || !d_dev) return set_error(CTOF_EINVAL, "m or d is NULL");
  if (!(peak > 0.0 && peak < 1e15)) return set_error(CTOF_EINVAL, "peak must be in (0, 1e15)");
  const size_t need = ctof::noisy_histogram_ws_bytes(n);
  if (!ws_dev || (reinterpret_cast<uintptr_t>(ws_dev) & 15)) return set_error(CTOF_EINVAL, "workspace NULL or misaligned");
  if (ws_bytes < need) return set_error(CTOF_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
  HIP_TRY(ctof::launch_noisy_histogram(m_dev, n, peak, seed, stream_id, d_dev, ws_dev, stream));
  return CTOF_OK;
}

ctof_status ctof_noisy_counts(int64_t n, const float *m_dev, double scale, double background, uint64_t seed,
                              uint32_t stream_id, float *out_dev, hipStream_t stream) {
  if (n < 0 || n > kMaxRows) return set_error(CTOF_EINVAL, "bad n");
  if (!m_dev || !out_dev) return set_error(CTOF_EINVAL, "m or out is NULL");
  if (!(scale > 0.0 && scale < 1e15)) return set_error(CTOF_EINVAL, "scale must be in (0, 1e15)");
  if (!(background >= 0.0 && background < 1e15)) return set_error(CTOF_EINVAL, "background must be in [0, 1e15)");
  HIP_TRY(ctof::launch_noisy_counts(m_dev, n, scale, background, seed, stream_id, out_dev, stream));
  return CTOF_OK;
}

ctof_status ctof_absmax_ws_bytes(int32_t nb, size_t *ws_bytes) {
  if (nb < 1 || nb > 65535) return set_error(CTOF_EINVAL, "nb must be in [1, 65535]");
  if (!ws_bytes) return set_error(CTOF_EINVAL, "ws_bytes is NULL");
  *ws_bytes = (ctof::absmax_ws_bytes(nb) + 255) / 256 * 256;
  return CTOF_OK;
}

ctof_status ctof_absmax(int32_t nb, int64_t len, const float *x_dev, float *out_dev, void *ws_dev, size_t ws_bytes,
                        hipStream_t stream) {
  if (nb < 1 || nb > 65535 || len < 0 || len > kMaxRows) return set_error(CTOF_EINVAL, "bad nb / len");
  if (!x_dev || !out_dev || !ws_dev) return set_error(CTOF_EINVAL, "NULL argument");
  const size_t need = ctof::absmax_ws_bytes(nb);
  if (ws_bytes < need) return set_error(CTOF_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
  HIP_TRY(ctof::launch_absmax(x_dev, len, nb, reinterpret_cast<float *>(ws_dev), out_dev, stream));
  return CTOF_OK;
}

ctof_status ctof_depth_resample(int32_t nb, int32_t nz_in, int64_t plane, const float *x_dev, float *out_dev,
                                int32_t mode, hipStream_t stream) {
  if (nb < 1 || nz_in < 1 || plane < 1 || (long long)nb * nz_in * plane > kMaxRows / 2)
    return set_error(CTOF_EINVAL, "bad sizes");
  if (mode != 0 && mode != 1) return set_error(CTOF_EINVAL, "mode must be 0 (sum pairs) or 1 (repeat)");
  if (mode == 0 && (nz_in & 1)) return set_error(CTOF_EINVAL, "summing layer pairs needs an even nz");
  if (!x_dev || !out_dev) return set_error(CTOF_EINVAL, "NULL argument");
  HIP_TRY(ctof::launch_depth_resample(x_dev, out_dev, nb, nz_in, plane, mode, stream));
  return CTOF_OK;
}

ctof_status ctof_sumsq_ws_bytes(int32_t nb, size_t *ws_bytes) {
  if (nb < 1 || nb > 65535) return set_error(CTOF_EINVAL, "nb must be in [1, 65535]");
  if (!ws_bytes) return set_error(CTOF_EINVAL, "ws_bytes is NULL");
  *ws_bytes = (ctof::sumsq_ws_bytes(nb) + 255) / 256 * 256;
  return CTOF_OK;
}

ctof_status ctof_sumsq(int32_t nb, int64_t len, const float *x_dev, double *out_dev, void *ws_dev, size_t ws_bytes,
                       hipStream_t stream) {
  if (nb < 1 || nb > 65535 || len < 1 || len > kMaxRows) return set_error(CTOF_EINVAL, "bad nb / len");
  if (!x_dev || !out_dev || !ws_dev) return set_error(CTOF_EINVAL, "NULL argument");
  if (ws_bytes < ctof::sumsq_ws_bytes(nb)) return set_error(CTOF_ENOMEM, "workspace too small");
  HIP_TRY(ctof::launch_sumsq(x_dev, x_dev, len, nb, reinterpret_cast<double *>(ws_dev), out_dev, stream));
  return CTOF_OK;
}

ctof_status ctof_layer_threshold_ws_bytes(int32_t nz, size_t *ws_bytes) {
  if (nz < 1 || nz > 65535) return set_error(CTOF_EINVAL, "nz must be in [1, 65535]");
  if (!ws_bytes) return set_error(CTOF_EINVAL, "ws_bytes is NULL");
  *ws_bytes = (ctof::absmax_ws_bytes(nz) + (size_t)nz * sizeof(float) + 511) / 256 * 256;
  return CTOF_OK;
}

ctof_status ctof_layer_threshold(int32_t nz, int64_t plane, float *mu_dev, float frac, void *ws_dev,
                                 size_t ws_bytes, hipStream_t stream) {
  if (nz < 1 || nz > 65535 || plane < 1 || (long long)nz * plane > kMaxRows) return set_error(CTOF_EINVAL, "bad sizes");
  if (!mu_dev || !ws_dev) return set_error(CTOF_EINVAL, "NULL argument");
  if (!(frac >= 0.0f && frac <= 1.0f)) return set_error(CTOF_EINVAL, "frac must be in [0, 1]");
  const size_t part = (ctof::absmax_ws_bytes(nz) + 255) / 256 * 256;
  if (ws_bytes < part + (size_t)nz * sizeof(float)) return set_error(CTOF_ENOMEM, "workspace too small");
  float *partials = reinterpret_cast<float *>(ws_dev);
  float *maxes = reinterpret_cast<float *>(reinterpret_cast<char *>(ws_dev) + part);
  HIP_TRY(ctof::launch_absmax(mu_dev, plane, nz, partials, maxes, stream));
  HIP_TRY(ctof::launch_layer_threshold(mu_dev, nz, plane, maxes, frac, stream));
  return CTOF_OK;
}

}  // extern "C"
