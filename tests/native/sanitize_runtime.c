/*
 * Driver of the library's host code for sanitizer builds (test infrastructure only).
 *
 * Linked with the runtime units compiled for the host only under AddressSanitizer and
 * UndefinedBehaviorSanitizer, and run where no GPU is present: every call here either
 * fails before touching a device (parameter validation, NULL or invalid contexts), fails
 * cleanly when the device is missing (context creation), or is host-only (lattice tables,
 * status strings, the warm-start features and order scaling).  Exits 0 when every status
 * is as documented in include/lbm.h, lbm_batch.h and lbm_nn.h; the sanitizers abort on
 * the first error they find.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm.h"
#include "lbm_batch.h"
#include "lbm_nn.h"

static int failures = 0;
#define EXPECT(cond)                                                   \
  do {                                                                 \
    if (!(cond)) {                                                     \
      fprintf(stderr, "line %d: %s (last error: %s)\n", __LINE__, #cond, \
              lbm_last_error());                                       \
      ++failures;                                                      \
    }                                                                  \
  } while (0)

static lbm_params base_params(void) {
  lbm_params p;
  memset(&p, 0, sizeof(p));
  p.lattice = LBM_D3Q19;
  p.collision = LBM_SMRT;
  p.storage = LBM_F32_SHIFTED;
  p.nx = 16;
  p.ny = 8;
  p.nz = 4;
  p.tau[2] = 0.6;
  p.tau[3] = 0.9;
  p.tau[4] = 1.0;
  p.rho0 = 1.0;
  return p;
}

int main(void) {
  /* status strings and version */
  for (int s = -6; s <= 2; ++s) EXPECT(lbm_strerror(s) != NULL && strlen(lbm_strerror(s)) > 0);
  EXPECT(lbm_version() > 0);
  /* lattice tables (host only) */
  for (int l = 0; l < 4; ++l) {
    int32_t D = 0, Q = 0, e[39 * 3];
    double w[39], sum = 0.0;
    EXPECT(lbm_lattice_info(l, &D, &Q, e, w) == LBM_OK);
    for (int i = 0; i < Q; ++i) sum += w[i];
    EXPECT(fabs(sum - 1.0) < 1e-15 && (D == 2 || D == 3));
  }
  EXPECT(lbm_lattice_info(4, NULL, NULL, NULL, NULL) == LBM_EINVAL);

  /* parameter validation: every one fails before any allocation */
  lbm_ctx *c = (lbm_ctx *)0x1;
  lbm_params p;
  p = base_params(); p.tau[2] = 0.5;
  EXPECT(lbm_init(&p, NULL, NULL, NULL, &c) == LBM_EINVAL && c == NULL);
  p = base_params(); p.tau[4] = 0.9;
  EXPECT(lbm_init(&p, NULL, NULL, NULL, &c) == LBM_EINVAL);
  p = base_params(); p.nx = 0;
  EXPECT(lbm_init(&p, NULL, NULL, NULL, &c) == LBM_EINVAL);
  p = base_params(); p.lattice = 7;
  EXPECT(lbm_init(&p, NULL, NULL, NULL, &c) == LBM_EINVAL);
  p = base_params(); p.mach_limit = NAN;
  EXPECT(lbm_init(&p, NULL, NULL, NULL, &c) == LBM_EINVAL);
  p = base_params(); p.g_kind = LBM_G_FIELD; p.g_data = NULL;
  EXPECT(lbm_init(&p, NULL, NULL, NULL, &c) == LBM_EINVAL);
  p = base_params(); p.nx = 2048; p.ny = 2048; p.nz = 1024;
  EXPECT(lbm_init(&p, NULL, NULL, NULL, &c) == LBM_EINVAL);
  p = base_params(); p.lattice = LBM_D3Q39; p.nz = 2;
  EXPECT(lbm_init(&p, NULL, NULL, NULL, &c) == LBM_EINVAL);
  p = base_params(); p.lattice = LBM_D3Q39; p.bc[1] = LBM_WALLS;
  EXPECT(lbm_init(&p, NULL, NULL, NULL, &c) == LBM_EINVAL);
  p = base_params(); p.lattice = LBM_D3Q39; p.collision = LBM_SMRT; p.force_order = 4;
  EXPECT(lbm_init(&p, NULL, NULL, NULL, &c) == LBM_EINVAL);
  p = base_params(); p.collision = LBM_BGK; p.force_order = 4;
  EXPECT(lbm_init(&p, NULL, NULL, NULL, &c) == LBM_EINVAL);
  EXPECT(lbm_init(NULL, NULL, NULL, NULL, &c) == LBM_EINVAL);
  EXPECT(lbm_init(&p, NULL, NULL, NULL, NULL) == LBM_EINVAL);
  /* a valid context where there is no device: a device error, nothing leaked */
  p = base_params();
  {
    uint8_t solid[16 * 8 * 4];
    double g[3 * 16 * 8 * 4];
    for (int n = 0; n < 16 * 8 * 4; ++n) {
      solid[n] = (uint8_t)(n % 9 == 0);
      g[n] = 1e-5;
      g[512 + n] = 0;
      g[1024 + n] = 0;
    }
    p.solid = solid;
    p.g_kind = LBM_G_FIELD;
    p.g_data = g;
    p.monitor_every = 3;
    const int rc = lbm_init(&p, NULL, NULL, NULL, &c);
    EXPECT(rc == LBM_EDEVICE || rc == LBM_ENOMEM);
    EXPECT(c == NULL);
  }
  /* calls on NULL contexts */
  lbm_monitors m;
  double buf[64];
  int64_t t = 0;
  size_t bytes = 0;
  lbm_tuning tu = {256, 1, 0};
  EXPECT(lbm_step(NULL, 1, NULL) == LBM_ESTATE);
  EXPECT(lbm_moments(NULL, 1.0, buf, buf) == LBM_ESTATE);
  EXPECT(lbm_monitors_get(NULL, &m) == LBM_ESTATE);
  EXPECT(lbm_get_populations(NULL, 1, NULL, buf) == LBM_ESTATE);
  EXPECT(lbm_get_populations_noalloc(NULL, 1, NULL, buf) == LBM_ESTATE);
  EXPECT(lbm_set_populations(NULL, buf) == LBM_ESTATE);
  EXPECT(lbm_set_waves(NULL, 0, NULL, NULL, NULL) == LBM_ESTATE);
  EXPECT(lbm_time(NULL, &t) == LBM_ESTATE);
  EXPECT(lbm_device_bytes(NULL, &bytes) == LBM_ESTATE);
  EXPECT(lbm_save(NULL, "x") == LBM_ESTATE && lbm_load(NULL, "x") == LBM_ESTATE);
  EXPECT(lbm_set_tuning(NULL, &tu) == LBM_ESTATE && lbm_get_tuning(NULL, &tu) == LBM_ESTATE);
  EXPECT(lbm_autotune(NULL, 1, NULL, NULL) == LBM_ESTATE);
  EXPECT(lbm_free(NULL) == LBM_ESTATE);
  EXPECT(lbm_copy_probe(NULL, NULL, 16, 1, 256, 0, NULL) == LBM_EINVAL);
  EXPECT(lbm_copy_probe(buf, buf, 17, 1, 256, 0, NULL) == LBM_EINVAL);

  /* the batched engine */
  lbm_domain d[2];
  memset(d, 0, sizeof(d));
  for (int k = 0; k < 2; ++k) {
    d[k].nx = 32;
    d[k].ny = 16 + k;
    d[k].nz = 1;
    d[k].tau[2] = 0.7;
    d[k].tau[3] = 1.0;
    d[k].tau[4] = 1.0;
  }
  lbm_batch *b = NULL;
  d[1].tau[2] = 0.4;
  EXPECT(lbm_batch_init(d, 2, LBM_D2Q9, LBM_SMRT, LBM_F32_SHIFTED, 1.0, NULL, &b) == LBM_EINVAL);
  d[1].tau[2] = 0.7;
  {
    const int rc = lbm_batch_init(d, 2, LBM_D2Q9, LBM_SMRT, LBM_F32_SHIFTED, 1.0, NULL, &b);
    EXPECT(rc == LBM_EDEVICE || rc == LBM_ENOMEM);
    EXPECT(b == NULL);
  }
  int64_t steps[2];
  double resid[2];
  int32_t status[2];
  EXPECT(lbm_batch_step(NULL, 10, 1e-8, steps, resid) == LBM_ESTATE);
  EXPECT(lbm_batch_run(NULL, 10, 1e-8, 2, 1, steps, resid, status) == LBM_ESTATE);
  EXPECT(lbm_batch_status(NULL, status) == LBM_ESTATE);
  EXPECT(lbm_batch_advance(NULL, 1) == LBM_ESTATE && lbm_batch_free(NULL) == LBM_ESTATE);

  /* warm start: wave bounds, features and order scaling (host only) */
  EXPECT(lbm_ws_max_waves(4, 4) > lbm_ws_max_waves(4, 3) && lbm_ws_max_waves(9, 1) == 0);
  lbm_ws_problem pr;
  memset(&pr, 0, sizeof(pr));
  pr.tau2 = 0.8;
  pr.nmodes = 4;
  for (int j = 0; j < 4; ++j) {
    pr.k[j][0] = 1 + j;
    pr.k[j][1] = j % 2;
    pr.p[j][2] = 1.0;
    pr.amp[j] = 1e-6 * (j + 1);
  }
  const int Q = 27, nw = 12;
  double *amp = calloc((size_t)nw * Q * 2, sizeof(double));
  const int32_t ends[4] = {4, 8, 10, 12};
  for (int k = 0; k < nw * Q * 2; ++k) amp[k] = 1e-3 / (1 + k % 7);
  float feat[LBM_WS_RESUM_FEATURES];
  double sigma = 0.0;
  EXPECT(lbm_ws_resum_features(&pr, 128, Q, amp, ends, feat, &sigma) == LBM_OK && sigma > 0);
  for (int f = 0; f < LBM_WS_RESUM_FEATURES; ++f) EXPECT(isfinite(feat[f]));
  const double cfac[4] = {1.0, 1.0, 0.9, 0.8};
  const double before = amp[10 * Q * 2];
  EXPECT(lbm_ws_scale_orders(amp, Q, ends, cfac) == LBM_OK);
  EXPECT(amp[10 * Q * 2] == before * 0.8);
  const int32_t bad_ends[4] = {4, 2, 10, 12};
  EXPECT(lbm_ws_scale_orders(amp, Q, bad_ends, cfac) == LBM_EINVAL);
  pr.nmodes = 3;
  EXPECT(lbm_ws_resum_features(&pr, 128, Q, amp, ends, feat, &sigma) == LBM_EINVAL);
  free(amp);
  lbm_mlp *net = NULL;
  const int32_t widths[3] = {4, 8, 2};
  EXPECT(lbm_mlp_create(widths, 0, 16, NULL, &net) == LBM_EINVAL && net == NULL);

  printf("%d failures\n", failures);
  return failures ? 1 : 0;
}
