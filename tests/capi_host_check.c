/* Host-side paths of the C ABI driven from C: rate tables, velocity sets,
 * workspace sizes (up to lattices of nearly 2^31 nodes), and argument
 * validation of the entry points, all of which return before any device
 * call.  Built and run with AddressSanitizer and UndefinedBehaviorSanitizer on
 * the host code (tests/test_capi_host_sanitized.py); prints "ok" on success. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "lbm_capi.h"

static int failures = 0;

#define CHECK(cond)                                                        \
  do {                                                                     \
    if (!(cond)) {                                                         \
      fprintf(stderr, "check failed at line %d: %s (last error: %s)\n",   \
              __LINE__, #cond, lbm_last_error(NULL));                      \
      ++failures;                                                          \
    }                                                                      \
  } while (0)

static lbm_grid grid3(int nx, int ny, int nz, int bx, int by, int bz) {
  lbm_grid g;
  g.n[0] = nx;
  g.n[1] = ny;
  g.n[2] = nz;
  g.bc[0] = bx;
  g.bc[1] = by;
  g.bc[2] = bz;
  return g;
}

static lbm_params flow_params(int storage, double gamma) {
  lbm_params p;
  memset(&p, 0, sizeof p);
  p.storage = storage;
  p.gamma = gamma;
  lbm_default_rates(0.1, gamma, 0, 0.0, p.s);
  p.rho0 = 1.0;
  p.force_mode = LBM_FORCE_UNIFORM;
  p.force_const[0] = 1e-5;
  p.mu = 1.0;
  p.check_every = 10;
  p.history_len = 64;
  return p;
}

static void rates_and_velocities(void) {
  double s[19];
  CHECK(lbm_default_rates(0.131, 0.1, 0, 0.0, s) == LBM_OK);
  for (int k = 0; k < 19; ++k) CHECK(s[k] > 0.0 && s[k] < 2.0);
  CHECK(lbm_default_rates(0.131, 0.5, 1, 3.0 / 16.0, s) == LBM_OK);
  CHECK(lbm_default_rates(-1.0, 0.5, 0, 0.0, s) == LBM_EINVAL);
  CHECK(lbm_default_rates(0.1, 0.0, 0, 0.0, s) == LBM_EINVAL);
  CHECK(lbm_default_rates(0.1, 1.5, 0, 0.0, s) == LBM_EINVAL);
  CHECK(lbm_default_rates(0.1, 0.5, 1, -1.0, s) == LBM_EINVAL);
  double s9[9];
  CHECK(lbm_default_rates_d2q9(0.1, 0.3, 0, 0.0, s9) == LBM_OK);
  CHECK(lbm_default_rates_d2q9(0.1, 0.3, 1, 3.0 / 16.0, s9) == LBM_OK);
  const int qs[4] = {19, 9, 7, 5};
  for (int i = 0; i < 4; ++i) {
    int32_t e[19 * 3];
    const int q = qs[i];
    CHECK(lbm_lattice_velocities(q, e) == LBM_OK);
    /* the rest direction first, every other direction has its opposite */
    CHECK(e[0] == 0 && e[1] == 0 && e[2] == 0);
    for (int a = 1; a < q; ++a) {
      int found = 0;
      for (int b = 1; b < q; ++b)
        found |= e[3 * b] == -e[3 * a] && e[3 * b + 1] == -e[3 * a + 1] &&
                 e[3 * b + 2] == -e[3 * a + 2];
      CHECK(found);
    }
  }
  int32_t e[3 * 19];
  CHECK(lbm_lattice_velocities(15, e) == LBM_EINVAL);
  CHECK(lbm_lattice_velocities(19, NULL) == LBM_EINVAL);
}

static void workspace_sizes(void) {
  size_t b = 0, prev = 0;
  const int storages[4] = {LBM_F64, LBM_F32, LBM_BF16, LBM_F16};
  for (int i = 0; i < 4; ++i) {
    lbm_grid g = grid3(64, 48, 40, LBM_PERIODIC, LBM_WALL, LBM_WALL);
    lbm_params p = flow_params(storages[i], 0.5);
    CHECK(lbm_workspace_bytes(&g, &p, &b) == LBM_OK);
    CHECK(b >= (size_t)2 * 19 * 64 * 48 * 40 * 2);
  }
  /* lattices of nearly 2^31 nodes: sizes beyond 2^32 bytes, no overflow */
  {
    lbm_grid g = grid3(2048, 1024, 1023, LBM_PERIODIC, LBM_WALL, LBM_WALL);
    lbm_params p = flow_params(LBM_F64, 1.0);
    CHECK(lbm_workspace_bytes(&g, &p, &b) == LBM_OK);
    CHECK(b >= (size_t)2 * 19 * 8 * (size_t)2048 * 1024 * 1023);
    p.storage = LBM_F32;
    prev = b;
    CHECK(lbm_workspace_bytes(&g, &p, &b) == LBM_OK);
    CHECK(b < prev && b >= (size_t)2 * 19 * 4 * (size_t)2048 * 1024 * 1023);
    p.mhd = 1;
    p.gamma_m = 0.5;
    p.chi = 0.1;
    p.eta = 0.02;
    p.B0[1] = 0.01;
    CHECK(lbm_workspace_bytes(&g, &p, &b) == LBM_OK);
    CHECK(b >= (size_t)2 * (19 + 21) * 4 * (size_t)2048 * 1024 * 1023);
  }
  /* 2^31 nodes or more: rejected */
  {
    lbm_grid g = grid3(2048, 1024, 1024, LBM_PERIODIC, LBM_WALL, LBM_WALL);
    lbm_params p = flow_params(LBM_F32, 1.0);
    CHECK(lbm_workspace_bytes(&g, &p, &b) == LBM_EINVAL);
    g = grid3(65536, 65536, 65536, LBM_PERIODIC, LBM_WALL, LBM_WALL);
    CHECK(lbm_workspace_bytes(&g, &p, &b) == LBM_EINVAL);
  }
  /* D2Q9, with and without induction */
  {
    lbm_grid g = grid3(4096, 4096, 1, LBM_PERIODIC, LBM_WALL, LBM_PERIODIC);
    lbm_params p = flow_params(LBM_F32, 0.1);
    p.lattice = LBM_D2Q9;
    lbm_default_rates_d2q9(0.1, 0.1, 0, 0.0, p.s);
    CHECK(lbm_workspace_bytes(&g, &p, &b) == LBM_OK);
    p.mhd = 1;
    p.gamma_m = 0.1;
    p.chi = 0.01;
    p.eta = 0.025;
    p.B0[1] = 0.01;
    CHECK(lbm_workspace_bytes(&g, &p, &b) == LBM_OK);
    g.n[2] = 2;
    CHECK(lbm_workspace_bytes(&g, &p, &b) == LBM_EINVAL);
  }
  /* batches */
  {
    lbm_grid g = grid3(4, 4, 64, LBM_PERIODIC, LBM_PERIODIC, LBM_WALL);
    CHECK(lbm_batch_workspace_bytes(&g, LBM_F64, 10, &b) == LBM_OK);
    CHECK(b >= (size_t)10 * 1024 * (2 * 19 * 8 + 3 * 8));
    CHECK(lbm_batch_workspace_bytes(&g, 9, 10, &b) == LBM_EINVAL);
    CHECK(lbm_batch_workspace_bytes(&g, LBM_F64, 0, &b) == LBM_EINVAL);
    CHECK(lbm_batch_workspace_bytes(&g, LBM_F64, 1 << 30, &b) == LBM_EINVAL);
  }
}

static void validation(void) {
  size_t b = 0;
  lbm_grid g = grid3(16, 8, 8, LBM_PERIODIC, LBM_WALL, LBM_WALL);
  lbm_params p;
  p = flow_params(7, 0.5);
  CHECK(lbm_workspace_bytes(&g, &p, &b) == LBM_EINVAL);
  p = flow_params(LBM_F32, 0.0);
  CHECK(lbm_workspace_bytes(&g, &p, &b) == LBM_EINVAL);
  p = flow_params(LBM_F32, 0.5);
  p.s[9] = 2.5;
  CHECK(lbm_workspace_bytes(&g, &p, &b) == LBM_EINVAL);
  p = flow_params(LBM_F32, 0.5);
  p.launch.waves = 2;
  CHECK(lbm_workspace_bytes(&g, &p, &b) == LBM_EINVAL);
  p = flow_params(LBM_F32, 0.5);
  p.launch.store = 3;
  CHECK(lbm_workspace_bytes(&g, &p, &b) == LBM_EINVAL);
  p = flow_params(LBM_F32, 0.5);
  p.mhd = 1;
  p.gamma_m = 0.5;
  p.chi = 0.0;
  p.eta = 0.02;
  CHECK(lbm_workspace_bytes(&g, &p, &b) == LBM_EINVAL);
  p = flow_params(LBM_F32, 0.5);
  p.rounding = LBM_ROUND_STOCHASTIC;
  CHECK(lbm_workspace_bytes(&g, &p, &b) == LBM_EINVAL);
  p = flow_params(LBM_F32, 0.5);
  p.history_len = 0;
  CHECK(lbm_workspace_bytes(&g, &p, &b) == LBM_EINVAL);
  lbm_grid bad = grid3(0, 8, 8, LBM_PERIODIC, LBM_WALL, LBM_WALL);
  p = flow_params(LBM_F32, 0.5);
  CHECK(lbm_workspace_bytes(&bad, &p, &b) == LBM_EINVAL);
  bad = grid3(8, 8, 8, LBM_PERIODIC, 5, LBM_WALL);
  CHECK(lbm_workspace_bytes(&bad, &p, &b) == LBM_EINVAL);
  CHECK(lbm_workspace_bytes(NULL, &p, &b) == LBM_EINVAL);
  CHECK(lbm_workspace_bytes(&g, NULL, &b) == LBM_EINVAL);
  CHECK(lbm_workspace_bytes(&g, &p, NULL) == LBM_EINVAL);
  /* lbm_create: invalid parameters and a missing workspace, before any device call */
  lbm_ctx* ctx = (lbm_ctx*)&b;
  p = flow_params(LBM_F32, 2.0);
  CHECK(lbm_create(&g, &p, NULL, NULL, 0, NULL, &ctx) == LBM_EINVAL && ctx == NULL);
  p = flow_params(LBM_F32, 0.5);
  CHECK(lbm_create(&g, &p, NULL, NULL, 0, NULL, &ctx) == LBM_ENOWS && ctx == NULL);
  CHECK(strlen(lbm_last_error(NULL)) > 0);
  /* the calibration copy: argument checks (these pointers are never dereferenced) */
  void* fake = (void*)(uintptr_t)4096;
  CHECK(lbm_bandwidth_probe(9, fake, fake, 64, 4, 4, 0, 2, 8, NULL) == LBM_EINVAL);
  CHECK(lbm_bandwidth_probe(3, fake, fake, 96, 4, 4, 0, 2, 8, NULL) == LBM_EINVAL);
  CHECK(lbm_bandwidth_probe(4, fake, fake, 1024, 1024, 64, 0, 2, 8, NULL) == LBM_EINVAL);
  CHECK(lbm_bandwidth_probe(1, fake, fake, 1 << 12, 1 << 12, 1 << 8, 0, 2, 8, NULL) == LBM_EINVAL);
  /* batches: a member with a rate out of range, then no workspace */
  lbm_grid gb = grid3(4, 4, 64, LBM_PERIODIC, LBM_PERIODIC, LBM_WALL);
  lbm_member m[2];
  memset(m, 0, sizeof m);
  for (int i = 0; i < 2; ++i) {
    m[i].gamma = 0.5;
    lbm_default_rates(0.1, 0.5, 0, 0.0, m[i].s);
  }
  m[1].s[9] = 2.5;
  lbm_member_result r[2];
  CHECK(lbm_batch_run(&gb, LBM_F64, 1.0, 2, m, NULL, 0, NULL, 1e-9, 100, 10, 100, NULL, r) ==
        LBM_EINVAL);
  CHECK(strstr(lbm_last_error(NULL), "member 1") != NULL);
  m[1].s[9] = 1.0;
  CHECK(lbm_batch_run(&gb, LBM_F64, 1.0, 2, m, NULL, 0, NULL, 1e-9, 100, 10, 100, NULL, r) ==
        LBM_ENOWS);
  /* no-allocation reductions: sizes beyond the static scratch are rejected */
  lbm_grid big = grid3(1024, 1024, 64, LBM_PERIODIC, LBM_WALL, LBM_WALL);
  double out[2];
  p = flow_params(LBM_F32, 0.5);
  CHECK(lbm_reductions_noalloc(&big, &p, fake, NULL, NULL, out) == LBM_ENOWS);
}

int main(void) {
  rates_and_velocities();
  workspace_sizes();
  validation();
  if (failures) {
    fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  printf("ok\n");
  return 0;
}
