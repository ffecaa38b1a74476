/*
 * Runs every entry point of the FP64 oracle on small systems, for a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py).
 * Test infrastructure: it includes the oracle's source as one translation
 * unit and checks a few facts of each result, so that a call that silently
 * did nothing would fail too.  Exit status 0 when every check holds.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/tbsma_oracle.c"

static int failures = 0;

static void check(int ok, const char *what) {
  if (!ok) {
    fprintf(stderr, "oracle driver: check failed: %s\n", what);
    failures++;
  }
}

int main(void) {
  const orc_pot P = {0.2061, 1.790, 10.229, 4.036, 2.884, 6.5, 7.0};
  /* wires: count, then fill; with and without the ring notch; cap 0 */
  int64_t n = orc_build_wire(4.08, 20.0, 30.6, 2, 0, 0.0, NULL, NULL, NULL,
                             NULL, 0);
  check(n > 100, "wire count");
  double *x = malloc(n * sizeof(double)), *y = malloc(n * sizeof(double)),
         *z = malloc(n * sizeof(double));
  uint8_t *flag = malloc(n);
  check(orc_build_wire(4.08, 20.0, 30.6, 2, 0, 0.0, x, y, z, flag, n) == n,
        "wire fill");
  int64_t nn = orc_build_wire(4.08, 20.0, 30.6, 2, 3, 4.08, NULL, NULL, NULL,
                              NULL, 0);
  check(nn < n, "notch removes atoms");
  /* a capacity short by one writes only cap atoms */
  double *xs = malloc((n - 1) * sizeof(double)),
         *ys = malloc((n - 1) * sizeof(double)),
         *zs = malloc((n - 1) * sizeof(double));
  uint8_t *fs = malloc(n - 1);
  check(orc_build_wire(4.08, 20.0, 30.6, 2, 0, 0.0, xs, ys, zs, fs, n - 1) ==
            n,
        "short capacity still counts");
  free(xs);
  free(ys);
  free(zs);
  free(fs);

  /* energies and forces: brute force, cell list, sampled, pair counts */
  double *e = malloc(n * sizeof(double)), *rho = malloc(n * sizeof(double));
  double *fx = malloc(n * sizeof(double)), *fy = malloc(n * sizeof(double)),
         *fz = malloc(n * sizeof(double));
  double w6[6];
  double E0 = orc_forces(&P, n, x, y, z, 0, rho, e, fx, fy, fz, w6);
  double E1 = orc_forces(&P, n, x, y, z, 1, NULL, NULL, NULL, NULL, NULL,
                         NULL);
  check(fabs(E0 - E1) < 1e-9 * fabs(E0), "brute force == cell list");
  double sfx = 0.0;
  for (int64_t i = 0; i < n; i++) sfx += fx[i];
  check(fabs(sfx) < 1e-9, "forces sum to zero");
  int64_t idx[3] = {0, n / 2, n - 1};
  double sx[3], sy[3], sz[3], se[3], sr[3];
  orc_forces_sampled(&P, n, x, y, z, 3, idx, sx, sy, sz, se, sr);
  check(fabs(sx[1] - fx[n / 2]) < 1e-12 && fabs(se[2] - e[n - 1]) < 1e-12,
        "sampled forces");
  int32_t *cnt = malloc(n * sizeof(int32_t));
  check(orc_count_pairs(n, x, y, z, 8.0, cnt) > 0, "pair counts");
  /* empty and single-atom systems */
  check(orc_forces(&P, 0, x, y, z, 1, NULL, NULL, NULL, NULL, NULL, w6) == 0.0,
        "empty system");
  check(orc_forces(&P, 1, x, y, z, 1, rho, e, fx, fy, fz, w6) == 0.0,
        "single atom");
  double d;
  check(orc_radial_eval(&P, 0, 8.0, &d) == 0.0 && d == 0.0, "beyond r_cut");

  /* random numbers */
  uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
  orc_philox4x32_10(ctr, key, out);
  double u[4], g[3];
  orc_uniform4(99, 1, 2, 3, 0, u);
  check(u[0] > 0.0 && u[0] < 1.0, "uniform in (0, 1)");
  orc_gauss3(99, 1, 2, 3, 0, g);
  check(isfinite(g[0] + g[1] + g[2]), "normals finite");

  /* dynamics: Langevin pulled, Nose-Hoover stepwise, barostat with a ramp */
  double *vx = calloc(n, sizeof(double)), *vy = calloc(n, sizeof(double)),
         *vz = calloc(n, sizeof(double)), *z0 = malloc(n * sizeof(double));
  double zlo = 0.0, zhi = 1e9;
  for (int64_t i = 0; i < n; i++) {
    if (flag[i] == 1 && z[i] > zlo) zlo = z[i];
    if (flag[i] == 2 && z[i] < zhi) zhi = z[i];
  }
  orc_md M;
  memset(&M, 0, sizeof(M));
  M.dt = 0.002;
  M.gamma = 1.0;
  M.T = 298.0;
  M.v_pull = 0.5;
  M.z_lo = zlo;
  M.z_hi = zhi;
  M.mass = 196.96657;
  M.seed = 13113890000ull;
  M.rep_id = 3;
  orc_init_state(&M, n, x, y, z, vx, vy, vz, flag, 0.02);
  memcpy(z0, z, n * sizeof(double));
  orc_forces(&P, n, x, y, z, 1, NULL, e, fx, fy, fz, NULL);
  double zeta = 0.0, eta = 0.0, piston[2] = {0.0, 0.0};
  orc_run(&P, &M, n, x, y, z, vx, vy, vz, z0, flag, fx, fy, fz, e, 0, 10, 1,
          &zeta, &eta, piston);
  double obs[8];
  orc_observe(&P, &M, n, x, y, z, vx, vy, vz, flag, 10, 1000.0, 30.6, piston,
              obs);
  check(obs[2] > 100.0 && obs[2] < 600.0, "Langevin temperature");
  M.gamma = 0.0;
  M.nh_tau = 0.1;
  M.grip_step = 0.05;
  M.grip_hold = 4;
  orc_run(&P, &M, n, x, y, z, vx, vy, vz, z0, flag, fx, fy, fz, e, 10, 10, 0,
          &zeta, &eta, piston);
  check(zeta != 0.0 && eta != 0.0, "Nose-Hoover variables move");
  M.grip_hold = 0;
  M.grip_step = 0.0;
  M.baro_mass = 300.0;
  M.baro_damp = 2.0;
  M.T_start = 20.0;
  M.ramp_steps = 20;
  orc_run(&P, &M, n, x, y, z, vx, vy, vz, z0, flag, fx, fy, fz, e, 20, 10, 1,
          &zeta, &eta, piston);
  orc_observe(&P, &M, n, x, y, z, vx, vy, vz, flag, 30, 1000.0, 30.6, piston,
              obs);
  check(piston[0] != 0.0 && fabs(obs[7] - 2.0 * piston[0]) < 1e-15,
        "barostat elongation");
  check(orc_target_temperature(&M, 10.0) > 20.0 &&
            orc_target_temperature(&M, 10.0) < 298.0,
        "ramp target");
  check(orc_num_threads() >= 1, "threads");

  free(x);
  free(y);
  free(z);
  free(flag);
  free(e);
  free(rho);
  free(fx);
  free(fy);
  free(fz);
  free(cnt);
  free(vx);
  free(vy);
  free(vz);
  free(z0);
  if (failures) return 1;
  printf("oracle driver: all checks passed (%lld atoms)\n", (long long)n);
  return 0;
}
