// sanitize_host_driver.cpp -- test driver for the address and undefined-behaviour sanitizer
// build of the host side of the HIP library (include/lbm.h).  On a machine without a GPU it
// runs every host-only path: parameter validation of lbm_create and lbm_batch_create, the
// surface-tension conversions, the per-cell collision compiled for the host
// (lbm_selftest_collide_host) on interface, bulk, zero- and tiny-gradient cells, the tile
// cover of the step's launches (lbm_selftest_tile_sets_host), error text and NULL handling.  Exit status 0 when every call returns what it should.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "lbm.h"

static int failures = 0;
#define EXPECT(cond)                                                   \
  do {                                                                 \
    if (!(cond)) {                                                     \
      std::fprintf(stderr, "%s:%d: failed: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                      \
    }                                                                  \
  } while (0)

static lbm_params base() {
  lbm_params p;
  std::memset(&p, 0, sizeof(p));
  p.nx = 16; p.ny = 12; p.nz = 20;
  p.rho_r0 = 1.6; p.rho_b0 = 1.0; p.nu_r = 0.02; p.nu_b = 0.01; p.A = 0.01; p.beta = 0.7;
  p.face[4] = LBM_FREESLIP; p.face[5] = LBM_OUTFLOW;
  p.force = 1; p.g[2] = 1e-5; p.rho_ref = 1.0;
  p.storage = LBM_F16;
  return p;
}

int main() {
  lbm_ctx* ctx = nullptr;
  // invalid parameters are rejected before any device call
  lbm_params p = base();
  p.nu_r = 0.0;
  EXPECT(lbm_create(&p, nullptr, &ctx) == LBM_EINVAL && ctx == nullptr);
  EXPECT(std::strlen(lbm_last_error(nullptr)) > 0);
  p = base(); p.beta = 2.0;
  EXPECT(lbm_create(&p, nullptr, &ctx) == LBM_EINVAL);
  p = base(); p.rho_r0 = 0.5;
  EXPECT(lbm_create(&p, nullptr, &ctx) == LBM_EINVAL);
  p = base(); p.face[0] = LBM_FREESLIP;
  EXPECT(lbm_create(&p, nullptr, &ctx) == LBM_EINVAL);
  p = base(); p.nx = 19884108; p.ny = 1; p.nz = 3;
  EXPECT(lbm_create(&p, nullptr, &ctx) == LBM_EINVAL);
  p = base(); p.s[26] = 1.5;
  EXPECT(lbm_create(&p, nullptr, &ctx) == LBM_EINVAL);
  EXPECT(lbm_create(nullptr, nullptr, &ctx) == LBM_EINVAL);
  lbm_params two[2] = {base(), base()};
  two[0].storage = 7;  // the first case is validated first
  lbm_batch* batch = nullptr;
  EXPECT(lbm_batch_create(two, 2, nullptr, &batch) == LBM_EINVAL && batch == nullptr);
  EXPECT(lbm_batch_create(two, 0, nullptr, &batch) == LBM_EINVAL);
  // a valid lattice passes validation; without a GPU the device is then reported missing
  p = base();
  p.face[0] = p.face[1] = LBM_FREESLIP;
  const lbm_status st = lbm_create(&p, nullptr, &ctx);
  EXPECT(st == LBM_EDEVICE || st == LBM_OK);
  if (ctx) lbm_destroy(ctx);
  // NULL contexts
  lbm_destroy(nullptr);
  lbm_batch_destroy(nullptr);
  EXPECT(lbm_step(nullptr, 1) == LBM_EINVAL && lbm_sync(nullptr) == LBM_EINVAL);
  EXPECT(lbm_state_bytes(nullptr) == 0 && lbm_batch_size(nullptr) == 0);
  // surface tension, Eq. (sigma)
  EXPECT(std::fabs(lbm_A_from_sigma(lbm_sigma_from_A(0.01, 0.05), 0.05) - 0.01) < 1e-17);
  EXPECT(std::isnan(lbm_sigma_from_A(0.01, 0.0)) && std::isnan(lbm_A_from_sigma(-1.0, 0.1)));
  // the collision on the host: an interface cell, a pure cell, zero and tiny gradients
  p = base();
  double fr[27], fb[27], outr[27], outb[27];
  const double w[4] = {8.0 / 27, 2.0 / 27, 1.0 / 54, 1.0 / 216};
  const int shell[27] = {0, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3, 3};
  const double grads[4][3] = {{0.1, -0.05, 0.2}, {0.0, 0.0, 0.0}, {1e-25, 0.0, 0.0}, {3e-9, 1e-9, -2e-9}};
  const double fracs[3] = {0.5, 0.0, 1e-9};
  for (double a : fracs)
    for (const auto& gp : grads) {
      for (int i = 0; i < 27; ++i) {
        fr[i] = 1.3 * a * w[shell[i]];
        fb[i] = 1.1 * (1.0 - a) * w[shell[i]] * (1.0 + 0.01 * (i % 3));
      }
      const double grho[3] = {0.01, 0.0, -0.02};
      EXPECT(lbm_selftest_collide_host(&p, fr, fb, gp, grho, outr, outb) == LBM_OK);
      double mr = 0.0, mb = 0.0;
      for (int i = 0; i < 27; ++i) {
        EXPECT(std::isfinite(outr[i]) && std::isfinite(outb[i]));
        mr += outr[i];
        mb += outb[i];
      }
      double r0 = 0.0, b0 = 0.0;
      for (int i = 0; i < 27; ++i) {
        r0 += fr[i];
        b0 += fb[i];
      }
      EXPECT(std::fabs(mr - r0) < 1e-6 && std::fabs(mb - b0) < 1e-6);
    }
  EXPECT(lbm_selftest_collide_host(nullptr, fr, fb, grads[0], grads[0], outr, outb) == LBM_EINVAL);

  // tile cover of the step's launches, with and without lateral walls, for the per-axis and
  // the per-wall (FP16) split of the frame: every tile once
  const int shapes[5][2] = {{32, 4}, {32, 8}, {64, 4}, {64, 8}, {32, 16}};
  for (int walls = 0; walls < 4; ++walls)
    for (const auto& sh : shapes) {
      lbm_params q = base();
      q.nx = 200; q.ny = 72;
      q.storage = (walls & 2) ? LBM_F32 : LBM_F16;
      if (walls & 1) q.face[0] = q.face[1] = q.face[2] = q.face[3] = LBM_FREESLIP;
      const int tx = (q.nx + sh[0] - 1) / sh[0], ty = (q.ny + sh[1] - 1) / sh[1], nt = tx * ty;
      int counts[3 * 7 * 18];
      EXPECT(3 * nt <= (int)(sizeof(counts) / sizeof(int)));
      EXPECT(lbm_selftest_tile_sets_host(&q, sh[0], sh[1], counts) == LBM_OK);
      for (int t = 0; t < nt; ++t) EXPECT(counts[t] + counts[nt + t] + counts[2 * nt + t] == 1);
    }
  {
    lbm_params q = base();
    int counts[3 * 64];
    EXPECT(lbm_selftest_tile_sets_host(&q, 16, 16, counts) == LBM_EINVAL);
    EXPECT(lbm_selftest_tile_sets_host(nullptr, 32, 8, counts) == LBM_EINVAL);
    EXPECT(lbm_selftest_tile_sets_host(&q, 32, 8, nullptr) == LBM_EINVAL);
  }
  std::printf("host sanitizer driver: %d failures\n", failures);
  return failures ? 1 : 0;
}
