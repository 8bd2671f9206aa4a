/* Test infrastructure: drives the host side of the C ABI (argument checks,
 * error strings, option and configuration bookkeeping, the batch driver's
 * checks) with no GPU, for a library whose host sources are built with
 * AddressSanitizer and UndefinedBehaviorSanitizer. None of these calls
 * reaches the HIP runtime. Prints "ok" and returns 0 on success. */
#include <stdio.h>
#include <string.h>

#include "bms.h"

static int bad = 0;
#define EXPECT(cond)                                         \
  do {                                                       \
    if (!(cond)) {                                           \
      printf("FAILED line %d: %s\n", __LINE__, #cond);       \
      bad = 1;                                               \
    }                                                        \
  } while (0)

int main(void) {
  bms_opts o;
  bms_default_opts(&o);
  EXPECT(o.precision == BMS_PREC_F64 && o.check_interval >= 1);
  for (int code = 0; code > -8; --code) EXPECT(strlen(bms_error_string(code)) > 0);
  EXPECT(strstr(bms_error_string(-99), "unknown") != NULL);
  EXPECT(strcmp(bms_last_error(NULL), "") == 0);

  const int bad_dims[4] = {3, 4, 4, 4}, dims[4] = {4, 4, 4, 4}, bc[4] = {1, 1, 1, -1};
  bms_ctx* ctx = NULL;
  EXPECT(bms_create(&ctx, bad_dims, bc, NULL) == BMS_EINVAL && ctx == NULL);
  EXPECT(bms_create(&ctx, dims, bc, NULL) == BMS_OK && ctx != NULL);
  bms_ctx* ctx2 = NULL;
  const int dims2[4] = {2, 2, 2, 2};
  EXPECT(bms_create(&ctx2, dims2, bc, NULL) == BMS_OK && ctx2 != NULL);

  void* dummy = (void*)0x1000;
  void* other = (void*)0x2000;
  const double sh[2] = {0.1, 0.2}, neg[2] = {0.1, -0.2};
  EXPECT(bms_apply_hop(ctx, 2, 1, dummy, other, 0) == BMS_EINVAL);
  EXPECT(bms_apply_hop(ctx, 1, 33, dummy, other, 0) == BMS_EINVAL);
  EXPECT(bms_apply_mdagm(ctx, 0.1, 0.0, 1, dummy, other, 2) == BMS_EINVAL);
  EXPECT(strstr(bms_last_error(ctx), "precision") != NULL);
  EXPECT(bms_solve(ctx, 0.1, 0, 2, sh, 1e-8, 100, NULL, dummy, other, NULL) == BMS_EINVAL);
  EXPECT(bms_solve(ctx, 0.1, 1, 2, sh, 1.5, 100, NULL, dummy, other, NULL) == BMS_EINVAL);
  EXPECT(bms_solve(ctx, 0.1, 1, 2, neg, 1e-8, 100, NULL, dummy, other, NULL) == BMS_EINVAL);
  EXPECT(bms_solve(ctx, 0.1, 1, 65, sh, 1e-8, 100, NULL, dummy, other, NULL) == BMS_EINVAL);
  o.qr_passes = 3;
  EXPECT(bms_solve(ctx, 0.1, 1, 2, sh, 1e-8, 100, &o, dummy, other, NULL) == BMS_EINVAL);
  bms_default_opts(&o);
  o.check_interval = 0;
  EXPECT(bms_solve(ctx, 0.1, 1, 2, sh, 1e-8, 100, &o, dummy, other, NULL) == BMS_EINVAL);
  bms_default_opts(&o);
  EXPECT(bms_force(ctx, 1, 2, sh, dummy, other, 7) == BMS_EINVAL);
  EXPECT(bms_set_gauge(ctx, NULL) == BMS_EINVAL);
  EXPECT(bms_set_gauge_improved(ctx, NULL, dummy) == BMS_EINVAL);
  EXPECT(bms_set_variant(ctx, BMS_KERNEL_UPDATE, 9) == BMS_EINVAL);
  /* well-formed calls need a gauge field first */
  EXPECT(bms_apply_hop(ctx, 1, 1, dummy, other, 0) == BMS_ESTATE);
  EXPECT(bms_solve(ctx, 0.1, 1, 2, sh, 1e-8, 100, NULL, dummy, other, NULL) == BMS_ESTATE);
  EXPECT(bms_force(ctx, 1, 2, sh, dummy, other, 0) == BMS_ESTATE);
  double S[2];
  EXPECT(bms_action(ctx, 1, 2, 1.0, sh, dummy, other, S) == BMS_ESTATE);
  EXPECT(strstr(bms_last_error(ctx), "gauge") != NULL);
  /* host-only bookkeeping */
  EXPECT(bms_timing_enable(ctx, 1) == BMS_OK);
  double ms = -1, by = -1;
  long long nl = -1;
  EXPECT(bms_timing_read(ctx, BMS_KERNEL_HOP, &ms, &nl, &by) == BMS_OK);
  EXPECT(ms == 0.0 && nl == 0 && by == 0.0);
  EXPECT(bms_timing_read(ctx, 99, NULL, NULL, NULL) == BMS_EINVAL);
  double fl = -1;
  EXPECT(bms_timing_floor(ctx, BMS_KERNEL_UPDATE, 8e12, 78.6e12, 157.3e12, &fl) == BMS_OK);
  EXPECT(fl == 0.0);
  EXPECT(bms_timing_floor(ctx, BMS_KERNEL_UPDATE, -1.0, 1.0, 1.0, &fl) == BMS_EINVAL);
  EXPECT(bms_timing_floor(ctx, BMS_KERNEL_UPDATE, 1.0, 1.0, 1.0, NULL) == BMS_EINVAL);
  int rows = 0;
  double dev = 0;
  EXPECT(bms_get_link_rows(ctx, &rows, &dev) == BMS_OK && rows == 3 && dev == -1.0);
  EXPECT(bms_get_link_rows(ctx, &rows, NULL) == BMS_OK);
  EXPECT(bms_set_link_rows(ctx, 1) == BMS_EINVAL);
  EXPECT(bms_set_link_rows(ctx, 3) == BMS_OK && bms_set_link_rows(ctx, 2) == BMS_OK);
  EXPECT(bms_set_variant(ctx, BMS_KERNEL_UPDATE, 4) == BMS_OK);
  int v = -5;
  EXPECT(bms_get_variant(ctx, BMS_KERNEL_UPDATE, &v) == BMS_OK && v == 4);
  int cfg[5] = {8, 8, 4, 2, 1}, got[5] = {0, 0, 0, 0, 0};
  EXPECT(bms_set_hop_config(ctx, BMS_PREC_F64, cfg) == BMS_OK);
  EXPECT(bms_get_hop_config(ctx, BMS_PREC_F64, got) == BMS_OK && memcmp(cfg, got, sizeof cfg) == 0);
  int badcfg[5] = {8, 8, 4, 2, 2};
  EXPECT(bms_set_hop_config(ctx, BMS_PREC_F64, badcfg) == BMS_EINVAL);
  EXPECT(bms_set_tune_cache(ctx, "/nonexistent/dir/cache.json") == BMS_OK);
  EXPECT(bms_autotune(ctx, 0.1, 1, 2, sh, BMS_PREC_F32, 8, dummy, other) == BMS_EINVAL);
  EXPECT(bms_autotune(ctx, 0.1, 1, 2, sh, BMS_PREC_F64, 0, dummy, other) == BMS_EINVAL);
  EXPECT(bms_autotune(ctx, 0.1, 1, 2, sh, BMS_PREC_F64, 8, dummy, other) == BMS_ESTATE);
  /* RHMC parameters: the defaults with no rational approximations */
  bms_rhmc_params p;
  bms_rhmc_result r;
  bms_default_rhmc_params(&p);
  EXPECT(bms_rhmc_trajectory(ctx, &p, dummy, other, dummy, &r) == BMS_EINVAL);
  p.n = 0;
  p.tau = -1;
  EXPECT(bms_rhmc_trajectory(ctx, &p, dummy, other, NULL, &r) == BMS_EINVAL);
  /* batch: argument checks, then per-problem status */
  bms_ctx* ctxs[2] = {ctx, ctx2};
  bms_ctx* same[2] = {ctx, ctx};
  const double mass[2] = {0.1, 0.1}, tol[2] = {1e-8, 1e-8};
  const int n[2] = {1, 1}, nsh[2] = {2, 2}, mi[2] = {100, 100};
  const double* shp[2] = {sh, sh};
  const void* Bp[2] = {(void*)0x1000, (void*)0x3000};
  void* Xp[2] = {(void*)0x2000, (void*)0x4000};
  int status[2] = {7, 7};
  EXPECT(bms_solve_batch(0, ctxs, mass, n, nsh, shp, tol, mi, NULL, Bp, Xp, NULL, status) ==
         BMS_EINVAL);
  EXPECT(bms_solve_batch(2, same, mass, n, nsh, shp, tol, mi, NULL, Bp, Xp, NULL, status) ==
         BMS_EINVAL);
  EXPECT(bms_solve_batch(2, ctxs, mass, n, nsh, shp, tol, mi, NULL, Bp, Xp, NULL, status) ==
         BMS_ESTATE);
  EXPECT(status[0] == BMS_ESTATE && status[1] == BMS_ESTATE);
  EXPECT(bms_destroy(ctx) == BMS_OK);
  EXPECT(bms_destroy(ctx2) == BMS_OK);
  EXPECT(bms_destroy(NULL) == BMS_EINVAL);
  if (!bad) printf("ok\n");
  return bad;
}
