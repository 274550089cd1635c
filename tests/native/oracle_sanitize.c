/*
 * Driver for an AddressSanitizer + UndefinedBehaviorSanitizer build of the
 * 2D FP64 oracle (host code only; test infrastructure).  It runs a few steps
 * of every wall scheme, collision operator and boundary variant on small and
 * degenerate grids from a perturbed rest state, and checks that the state
 * stays finite and that link-walled channels keep their mass.  Any
 * out-of-bounds access, use of uninitialised stack memory through a bad
 * index, signed overflow or similar undefined behaviour aborts the run.
 *
 *   gcc -std=c11 -O1 -g -fsanitize=address,undefined -fno-sanitize-recover=all \
 *       -fno-omit-frame-pointer tests/native/oracle_sanitize.c -lm
 */
#include "../../oracle/lks_oracle.c"

#include <stdio.h>

static double frand(uint32_t *s) {
  *s = *s * 1664525u + 1013904223u;
  return (double)(*s >> 8) / 16777216.0;
}

static int run_case(const char *name, orc_params p, int steps) {
  const size_t n = (size_t)NPLANES * (size_t)p.nx * (size_t)p.ny;
  double *a = malloc(n * sizeof(double)), *b = malloc(n * sizeof(double));
  if (!a || !b) return 1;
  orc_init(&p, 1.0, a);
  uint32_t seed = 12345u;
  for (size_t i = 0; i < n; ++i) a[i] *= 1.0 + 0.02 * (frand(&seed) - 0.5);
  double m0 = 0.0;
  for (size_t i = 0; i < 9 * (size_t)p.nx * p.ny; ++i) m0 += a[i];
  orc_run(&p, a, b, steps, 1);
  double m1 = 0.0;
  int finite = 1;
  for (size_t i = 0; i < n; ++i) finite &= isfinite(a[i]) != 0;
  for (size_t i = 0; i < 9 * (size_t)p.nx * p.ny; ++i) m1 += a[i];
  double *obs = malloc(6 * (size_t)p.nx * p.ny * sizeof(double));
  const size_t k = (size_t)p.nx * p.ny;
  orc_observe(&p, a, obs, obs + k, obs + 2 * k, obs + 3 * k, obs + 4 * k, obs + 5 * k);
  for (size_t i = 0; i < 6 * k; ++i) finite &= isfinite(obs[i]) != 0;
  double pops[19];
  orc_gather(&p, a, p.nx - 1, p.ny - 1, pops);
  const int link = p.bc == ORC_LINK;
  const double drift = fabs(m1 - m0) / m0;
  const int ok = finite && (!link || drift < 1e-12);
  printf("%-34s nx=%-3d ny=%-3d finite=%d mass drift=%.2e %s\n", name, p.nx, p.ny, finite, drift,
         ok ? "ok" : "FAIL");
  free(a);
  free(b);
  free(obs);
  return ok ? 0 : 1;
}

int main(void) {
  orc_params base;
  memset(&base, 0, sizeof base);
  base.tau_f = 0.8;
  base.tau_m = 0.9;
  base.b0 = 0.03;
  base.fx = 1e-5;
  base.c_lo = 0.3;
  base.c_hi = INFINITY;
  base.u_hi = 0.04;
  base.tau_fm = 0.8;
  base.tau_mp = 0.9;
  base.q_lo = base.q_hi = 0.5;
  base.s_fe = 1.64;
  base.s_feps = 1.54;
  base.s_fq = 1.2;
  base.s_me = 1.1;
  base.s_md = 1.3;
  int bad = 0;
  const int sizes[][2] = {{1, 3}, {2, 3}, {5, 7}, {17, 4}};
  for (int si = 0; si < 4; ++si)
    for (int bc = 0; bc < 2; ++bc)
      for (int coll = 0; coll < 3; ++coll) {
        orc_params p = base;
        p.nx = sizes[si][0];
        p.ny = sizes[si][1];
        p.bc = bc;
        p.collision = coll;
        p.a = bc == ORC_LINK ? p.ny / 2.0 : (p.ny - 1) / 2.0;
        char name[64];
        snprintf(name, sizeof name, "%s %s", bc ? "moment" : "link",
                 coll == 0 ? "BGK" : (coll == 1 ? "TRT" : "MRT"));
        bad += run_case(name, p, 25);
      }
  /* limits of the conductance ratio on both walls */
  const double cs[] = {0.0, 1e-3, INFINITY};
  for (int i = 0; i < 3; ++i)
    for (int bc = 0; bc < 2; ++bc) {
      orc_params p = base;
      p.nx = 6;
      p.ny = 5;
      p.bc = bc;
      p.c_lo = p.c_hi = cs[i];
      p.u_lo = -0.02;
      p.a = bc == ORC_LINK ? p.ny / 2.0 : (p.ny - 1) / 2.0;
      bad += run_case(bc ? "moment, equal c" : "link, equal c", p, 25);
    }
  /* enclosure (x walls, link) */
  for (int coll = 0; coll < 3; ++coll) {
    orc_params p = base;
    p.nx = 4;
    p.ny = 5;
    p.x_walls = 1;
    p.cx_lo = 0.5;
    p.cx_hi = INFINITY;
    p.collision = coll;
    p.a = p.ny / 2.0;
    bad += run_case("enclosure", p, 25);
  }
  /* link walls at cut distances (three rows or more) */
  const double qs[][2] = {{0.25, 0.75}, {1.0, 0.3}};
  for (int i = 0; i < 2; ++i) {
    orc_params p = base;
    p.nx = 5;
    p.ny = 4;
    p.q_lo = qs[i][0];
    p.q_hi = qs[i][1];
    p.c_hi = 2.0;
    p.a = (p.ny - 1 + p.q_lo + p.q_hi) / 2.0;
    bad += run_case("cut-distance walls", p, 25);
  }
  /* solid bodies (curved walls): a rotating disc and a half-plane */
  for (int coll = 0; coll < 3; ++coll) {
    orc_params p = base;
    p.nx = 14;
    p.ny = 12;
    p.collision = coll;
    p.c_hi = 0.5;
    p.a = p.ny / 2.0;
    p.nsolid = 2;
    p.solid[0].kind = ORC_SOLID_DISC;
    p.solid[0].cx = 6.3;
    p.solid[0].cy = 6.1;
    p.solid[0].r = 2.7;
    p.solid[0].omega = 0.01;
    p.solid[1].kind = ORC_SOLID_BELOW;
    p.solid[1].cy = 1.4;
    p.solid[1].u = 0.01;
    /* curved walls leak a little mass: finiteness only */
    const orc_params q = p;
    const size_t n = (size_t)NPLANES * q.nx * q.ny;
    double *a = malloc(n * sizeof(double)), *b = malloc(n * sizeof(double));
    orc_init(&q, 1.0, a);
    orc_run(&q, a, b, 25, 1);
    int finite = 1;
    for (size_t i = 0; i < n; ++i) finite &= isfinite(a[i]) != 0;
    printf("%-34s nx=%-3d ny=%-3d finite=%d %s\n", "solid bodies", q.nx, q.ny, finite,
           finite ? "ok" : "FAIL");
    bad += !finite;
    free(a);
    free(b);
  }
  printf("%s\n", bad ? "FAILED" : "all ok");
  return bad ? 1 : 0;
}
