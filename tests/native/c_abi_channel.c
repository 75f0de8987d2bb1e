/* A plain C99 user of the library's C ABI (no Python, no HIP headers): a
 * forced FP64 channel nx x ny x nz with walls in y, started at rest, run for
 * a number of steps; prints the x-z mean of u_x per y row, the mass and the
 * x-momentum, one value per line, for the test that checks it against the
 * oracle.  Usage: c_abi_channel nx ny nz steps.  Exit code: 0, or the
 * library's error code (its text on stderr). */
#include <stdio.h>
#include <stdlib.h>

#include "lbm.h"

static int fail(lbm_ctx* c, int rc, const char* what) {
  fprintf(stderr, "%s: %d %s\n", what, rc, lbm_last_error(c));
  if (c) lbm_destroy(c);
  return rc < 0 ? -rc : 1;
}

int main(int argc, char** argv) {
  if (argc != 5) {
    fprintf(stderr, "usage: %s nx ny nz steps\n", argv[0]);
    return 2;
  }
  lbm_config cfg;
  lbm_config_default(&cfg);
  cfg.nx = atoi(argv[1]);
  cfg.ny = atoi(argv[2]);
  cfg.nz = atoi(argv[3]);
  const long steps = atol(argv[4]);
  cfg.storage = LBM_F64;
  cfg.walls_y = 1;
  cfg.nu = 0.02;
  cfg.force[0] = 1e-5;
  lbm_ctx* c = NULL;
  int rc = lbm_create(&cfg, &c);
  if (rc) return fail(NULL, rc, "lbm_create");
  if ((rc = lbm_init(c, NULL, NULL))) return fail(c, rc, "lbm_init");
  if ((rc = lbm_step(c, steps))) return fail(c, rc, "lbm_step");
  const long n = (long)cfg.nx * cfg.ny * cfg.nz;
  double* rho = malloc(sizeof(double) * n);
  double* u = malloc(sizeof(double) * 3 * n);
  if (!rho || !u) return fail(c, -2, "malloc");
  if ((rc = lbm_moments(c, rho, u))) return fail(c, rc, "lbm_moments");
  for (int y = 0; y < cfg.ny; ++y) {
    double s = 0.0;
    for (int z = 0; z < cfg.nz; ++z)
      for (int x = 0; x < cfg.nx; ++x) s += u[((long)z * cfg.ny + y) * cfg.nx + x];
    printf("%.17g\n", s / ((double)cfg.nx * cfg.nz));
  }
  lbm_diag d;
  if ((rc = lbm_diagnostics(c, &d))) return fail(c, rc, "lbm_diagnostics");
  printf("%.17g\n%.17g\n", d.mass, d.momentum[0]);
  free(rho);
  free(u);
  lbm_destroy(c);
  return 0;
}
