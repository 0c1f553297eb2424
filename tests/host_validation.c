/*
 * Host-side argument validation of libctof, run without a GPU: every call
 * below must return its documented status before any HIP call.  Built
 * together with the library's host code under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_host_sanitize.py.
 */
#include <math.h>
#include <stdio.h>
#include <string.h>
#include "ctof.h"

static int fails = 0;
#define EXPECT(cond) do { if (!(cond)) { fprintf(stderr, "FAILED %s:%d %s\n", __FILE__, __LINE__, #cond); ++fails; } } while (0)

int main(void) {
  double z[4] = {1.0, 2.0, 3.0, 4.0};
  ctof_geometry g;
  memset(&g, 0, sizeof(g));
  g.nx = 24; g.ny = 20; g.pitch_mm = 0.5; g.nz = 4; g.z_mm = z; g.dz_mm = 1.0; g.nt = 48; g.dt_ps = 25.0;
  g.mus_prime_per_mm = 1.0; g.mua_per_mm = 0.01; g.n_medium = 1.4;
  size_t kb = 0, wb = 0;
  for (int p = 0; p < 4; ++p) {
    EXPECT(ctof_kernel_bytes(&g, (ctof_precision)p, &kb, &wb) == CTOF_OK);
    EXPECT(kb > 0 && wb > 0);
  }
  EXPECT(ctof_kernel_bytes(&g, (ctof_precision)7, &kb, &wb) == CTOF_EINVAL);
  EXPECT(ctof_kernel_bytes(NULL, CTOF_FP32, &kb, &wb) == CTOF_EINVAL);
  ctof_geometry b = g; b.nx = 0;           EXPECT(ctof_kernel_bytes(&b, CTOF_FP32, &kb, &wb) == CTOF_EINVAL);
  b = g; b.pitch_mm = -1.0;                EXPECT(ctof_kernel_bytes(&b, CTOF_FP32, &kb, &wb) == CTOF_EINVAL);
  b = g; b.dt_ps = NAN;                    EXPECT(ctof_kernel_bytes(&b, CTOF_FP32, &kb, &wb) == CTOF_EINVAL);
  double zb[4] = {1.0, 3.0, 2.0, 4.0};
  b = g; b.z_mm = zb;                      EXPECT(ctof_kernel_bytes(&b, CTOF_FP32, &kb, &wb) == CTOF_EINVAL);
  b = g; b.z_mm = NULL;                    EXPECT(ctof_kernel_bytes(&b, CTOF_FP32, &kb, &wb) == CTOF_EINVAL);
  b = g; b.nx = 1025;                      EXPECT(ctof_kernel_bytes(&b, CTOF_FP32, &kb, &wb) != CTOF_OK);
  b = g; b.n_medium = 0.5;                 EXPECT(ctof_kernel_bytes(&b, CTOF_FP32, &kb, &wb) == CTOF_EINVAL);
  b = g; b.nx = b.ny = 1024; b.nt = 2147483647;
  EXPECT(ctof_kernel_bytes(&b, CTOF_FP32, &kb, &wb) == CTOF_EINVAL);  /* beyond 1e15 voxel-bins */
  b = g; b.nx = b.ny = 1024; b.nt = 16384;
  EXPECT(ctof_kernel_bytes(&b, CTOF_FP64, &kb, &wb) == CTOF_OK && kb > ((size_t)1 << 36));
  EXPECT(strlen(ctof_last_error()) > 0);
  ctof_kernel k = NULL;
  EXPECT(ctof_kernel_tabulate(NULL, CTOF_FP32, NULL, 0, NULL, 0, NULL, &k) == CTOF_EINVAL);
  EXPECT(ctof_kernel_tabulate(&g, (ctof_precision)9, (void *)16, 1 << 30, (void *)16, 1 << 30, NULL, &k) == CTOF_EINVAL);
  EXPECT(ctof_kernel_tabulate(&g, CTOF_FP32, NULL, 0, NULL, 0, NULL, &k) == CTOF_EINVAL);
  EXPECT(ctof_kernel_tabulate(&g, CTOF_FP32, (void *)16, 0, (void *)16, 0, NULL, NULL) == CTOF_EINVAL);
  EXPECT(ctof_kernel_tabulate(&g, CTOF_FP32, (void *)16, 1, (void *)16, 1, NULL, &k) == CTOF_ENOMEM);
  EXPECT(ctof_kernel_tabulate_fp64_quadrant(NULL, NULL, NULL) == CTOF_EINVAL);
  EXPECT(ctof_kernel_tabulate_fp64_quadrant(&g, NULL, NULL) == CTOF_EINVAL);
  EXPECT(ctof_kernel_tabulate_quadrant(&g, (double *)16, 8, NULL) == CTOF_ENOMEM);
  size_t ws = 0;
  EXPECT(ctof_workspace_bytes(NULL, 10, &ws, &ws) == CTOF_EINVAL);
  ctof_solver_opts o;
  memset(&o, 0, sizeof(o));
  o.max_iter = 10;
  ctof_solver_report r;
  EXPECT(ctof_reconstruct(NULL, (void *)16, (void *)16, &o, &r, (void *)16, 1 << 20, NULL) == CTOF_EINVAL);
  EXPECT(ctof_forward(NULL, (void *)16, (void *)16, (void *)16, 1 << 20, NULL) == CTOF_EINVAL);
  EXPECT(ctof_adjoint(NULL, (void *)16, (void *)16, (void *)16, 1 << 20, NULL) == CTOF_EINVAL);
  const ctof_kernel ks[2] = {NULL, NULL};
  EXPECT(ctof_workspace_bytes_batched(2, ks, 10, &ws) == CTOF_EINVAL);
  EXPECT(ctof_workspace_bytes_batched(0, ks, 10, &ws) == CTOF_EINVAL);
  /* the network's layers */
  ctof_conv_desc cd = {CTOF_CONV_K3, 2, 8, 8, 8, 16, 16};
  size_t el = 0;
  EXPECT(ctof_conv3d_weight_elems(&cd, &el) == CTOF_OK && el > 0);
  EXPECT(ctof_conv3d_weight_elems(NULL, &el) == CTOF_EINVAL);
  ctof_conv_desc cb = cd; cb.kind = 9;                 EXPECT(ctof_conv3d_weight_elems(&cb, &el) == CTOF_EINVAL);
  cb = cd; cb.n = 0;                                   EXPECT(ctof_conv3d_weight_elems(&cb, &el) == CTOF_EINVAL);
  cb = cd; cb.ci = 0;                                  EXPECT(ctof_conv3d_weight_elems(&cb, &el) == CTOF_EINVAL);
  cb = cd; cb.kind = CTOF_CONV_DN; cb.w = 7;           EXPECT(ctof_conv3d_weight_elems(&cb, &el) == CTOF_EINVAL);
  cb = cd; cb.n = cb.d = cb.h = cb.w = 1 << 30;        EXPECT(ctof_conv3d_weight_elems(&cb, &el) == CTOF_EINVAL);
  cb = cd; cb.kind = CTOF_CONV_UP; cb.n = cb.d = cb.h = cb.w = 2147483647;
  EXPECT(ctof_conv3d_weight_elems(&cb, &el) == CTOF_EINVAL);
  cb = cd; cb.co = 80;                                 EXPECT(ctof_conv3d_weight_elems(&cb, &el) != CTOF_OK);
  size_t cws = 0;
  EXPECT(ctof_conv3d_bwd_data_ws_bytes(&cd, &cws) == CTOF_OK);
  EXPECT(ctof_conv3d_bwd_weight_ws_bytes(&cd, &cws) == CTOF_OK);
  EXPECT(ctof_conv3d_bwd_weight_ws_bytes(NULL, &cws) == CTOF_EINVAL);
  ctof_tensor tx = {NULL, 16, 0};
  EXPECT(ctof_conv3d_fwd(&cd, &tx, NULL, NULL, &tx, 0, 1, 0, NULL) == CTOF_EINVAL);
  EXPECT(ctof_conv3d_fwd(&cd, NULL, NULL, NULL, NULL, 0, 1, 0, NULL) == CTOF_EINVAL);
  EXPECT(ctof_relu_bwd(-1, 16, &tx, &tx, NULL) != CTOF_OK);
  EXPECT(ctof_mse_ws_bytes(-5, &cws) != CTOF_OK);
  ctof_kernel_free(NULL);
  printf("host validation checks: %d failed\n", fails);
  return fails != 0;
}
