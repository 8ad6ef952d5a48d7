/*
 * sanitize_driver.c -- TEST INFRASTRUCTURE ONLY: a driver for the address and undefined-
 * behaviour sanitizer build of the FP64 oracle (lbm_oracle.c).  It runs small lattices through
 * every code path of the oracle -- all face rules (periodic, bounce-back, free-slip on every
 * axis, convective outflow), the inflow disk with noise, the body force, user and default
 * relaxation rates, read-back of fields, populations and gradients -- and checks that the
 * per-colour masses stay finite.  Exit status 0 on success; a sanitizer report aborts.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm_oracle.c"

static int run(oracle_params *p, int steps, const char *name) {
  oracle *o = NULL;
  if (oracle_create(p, &o) != 0) {
    fprintf(stderr, "%s: oracle_create failed\n", name);
    return 1;
  }
  const long n = (long)p->nx * p->ny * p->nz;
  double *rr = malloc(sizeof(double) * n), *rb = malloc(sizeof(double) * n), *u = calloc(3 * n, sizeof(double));
  for (long c = 0; c < n; c++) {
    const int x = (int)(c % p->nx), z = (int)(c / ((long)p->nx * p->ny));
    const double t = tanh((x - 0.5 * p->nx) / 2.0 + 0.3 * (z - 0.5 * p->nz));
    rr[c] = 0.5 * p->rho_r0 * (1.0 - t);
    rb[c] = 0.5 * p->rho_b0 * (1.0 + t);
    u[2 * n + c] = 0.01;
  }
  oracle_init(o, rr, rb, u);
  oracle_step(o, steps);
  double *f = malloc(sizeof(double) * 2 * Q * n), *g = malloc(sizeof(double) * 3 * n);
  oracle_fields(o, rr, rb, u);
  oracle_populations(o, f);
  oracle_set_populations(o, f);
  oracle_gradient(o, rr, g);
  double mr = 0, mb = 0;
  for (long c = 0; c < n; c++) {
    mr += rr[c];
    mb += rb[c];
  }
  const int ok = isfinite(mr) && isfinite(mb) && oracle_step_count(o) == steps;
  printf("%s: %d steps, mass red %.6f blue %.6f%s\n", name, steps, mr, mb, ok ? "" : " NOT FINITE");
  free(rr); free(rb); free(u); free(f); free(g);
  oracle_destroy(o);
  return ok ? 0 : 1;
}

int main(void) {
  int bad = 0;
  oracle_params p;
  memset(&p, 0, sizeof(p));
  p.nx = 7; p.ny = 6; p.nz = 9;
  p.rho_r0 = 1.6; p.rho_b0 = 1.0; p.nu_r = 0.02; p.nu_b = 0.01; p.A = 0.01; p.beta = 0.7;
  p.gphi_cut = 1e-12;
  bad |= run(&p, 5, "periodic");
  for (int k = 0; k < 6; k++) p.face[k] = FACE_FREESLIP;
  p.force_model = 1; p.g[0] = 1e-5; p.g[1] = -1e-5; p.g[2] = 2e-5; p.rho_ref = 1.0;
  bad |= run(&p, 5, "free-slip box with a body force");
  p.face[4] = p.face[5] = FACE_BOUNCEBACK;
  for (int j = 4; j < Q; j++) p.s[j] = 1.2;
  bad |= run(&p, 5, "bounce-back z, free-slip x and y, user rates");
  memset(p.s, 0, sizeof(p.s));
  for (int k = 0; k < 4; k++) p.face[k] = FACE_PERIODIC;
  p.face[4] = FACE_FREESLIP; p.face[5] = FACE_OUTFLOW;
  p.inflow = 1; p.xc = 3.0; p.yc = 2.5; p.diameter = 4.0; p.u_in = 0.04; p.noise_rel = 0.01; p.seed = 3;
  bad |= run(&p, 6, "jet: inflow disk with noise, convective outflow");
  p.gnx = 14; p.gny = 12; p.gnz = 18; p.ox = 2; p.oy = 1; p.oz = 0;
  bad |= run(&p, 3, "window of a larger domain");
  return bad;
}
