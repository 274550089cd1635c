/*
 * Driver for an AddressSanitizer + UndefinedBehaviorSanitizer build of the
 * 3D FP64 oracle (host code only; test infrastructure): a few steps of
 * channels and ducts with both wall schemes and every collision operator on
 * small and degenerate grids, from a perturbed rest state.  The state must
 * stay finite, and link-walled runs keep their mass.
 *
 *   gcc -std=c11 -O1 -g -fsanitize=address,undefined -fno-sanitize-recover=all \
 *       -fno-omit-frame-pointer tests/native/oracle3_sanitize.c -lm
 */
#include "../../oracle/lks_oracle3.c"

#include <stdio.h>

static double frand(uint32_t *s) {
  *s = *s * 1664525u + 1013904223u;
  return (double)(*s >> 8) / 16777216.0;
}

static int run_case(const char *name, orc3_params p, int steps) {
  const size_t N = (size_t)p.nx * p.ny * p.nz, n = (size_t)NPL3 * N;
  double *a = malloc(n * sizeof(double)), *b = malloc(n * sizeof(double));
  double *obs = malloc(10 * N * sizeof(double));
  if (!a || !b || !obs) return 1;
  orc3_init(&p, 1.0, a);
  uint32_t seed = 777u;
  for (size_t i = 0; i < n; ++i) a[i] *= 1.0 + 0.02 * (frand(&seed) - 0.5);
  double m0 = 0.0, m1 = 0.0;
  for (size_t i = 0; i < NQF * N; ++i) m0 += a[i];
  orc3_run(&p, a, b, steps, 1);
  int finite = 1;
  for (size_t i = 0; i < n; ++i) finite &= isfinite(a[i]) != 0;
  for (size_t i = 0; i < NQF * N; ++i) m1 += a[i];
  orc3_observe(&p, a, obs);
  for (size_t i = 0; i < 10 * N; ++i) finite &= isfinite(obs[i]) != 0;
  double pops[40];
  orc3_gather(&p, a, p.nx - 1, p.ny - 1, p.nz - 1, pops);
  const double drift = fabs(m1 - m0) / m0;
  const int ok = finite && (p.bc != 0 || drift < 1e-12);
  printf("%-22s %dx%dx%d finite=%d mass drift=%.2e %s\n", name, p.nx, p.ny, p.nz, finite, drift,
         ok ? "ok" : "FAIL");
  free(a);
  free(b);
  free(obs);
  return ok ? 0 : 1;
}

int main(void) {
  orc3_params base;
  memset(&base, 0, sizeof base);
  base.tau_f = 0.8;
  base.tau_m = 0.9;
  base.b0 = 0.03;
  base.fx = 1e-5;
  base.fz = 2e-6;
  base.c_lo = 0.4;
  base.c_hi = INFINITY;
  base.u_hi = 0.03;
  base.tau_fm = 0.8;
  base.tau_mp = 0.9;
  base.s_fe = 1.19;
  base.s_feps = 1.4;
  base.s_fq = 1.2;
  base.s_md = 1.6;
  int bad = 0;
  const int sizes[][3] = {{1, 3, 1}, {2, 3, 2}, {4, 5, 3}};
  for (int si = 0; si < 3; ++si)
    for (int bc = 0; bc < 2; ++bc)
      for (int coll = 0; coll < 3; ++coll)
        for (int duct = 0; duct < 2; ++duct) {
          if (duct && (bc != 0 || sizes[si][2] < 2)) continue; /* ducts: link walls, nz >= 2 */
          orc3_params p = base;
          p.nx = sizes[si][0];
          p.ny = sizes[si][1];
          p.nz = sizes[si][2];
          p.bc = bc;
          p.collision = coll;
          p.side_walls = duct;
          p.cs_lo = 0.5;
          p.cs_hi = 0.0;
          p.a = bc == 0 ? p.ny / 2.0 : (p.ny - 1) / 2.0;
          char name[48];
          snprintf(name, sizeof name, "%s %s%s", bc ? "moment" : "link",
                   coll == 0 ? "BGK" : (coll == 1 ? "TRT" : "MRT"), duct ? " duct" : "");
          bad += run_case(name, p, 12);
        }
  printf("%s\n", bad ? "FAILED" : "all ok");
  return bad ? 1 : 0;
}
