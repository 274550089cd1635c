/*
 * FP64 CPU oracle for the lattice-kinetic MHD time step with Shercliff
 * thin-conducting-wall closures (Yahia & Premnath, arXiv 2112.13930).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header or table with the HIP
 * library: the lattice constants below are typed in here from the paper.
 *
 * It is deliberately plain: separate pull-stream, wall-closure, moment,
 * local-solve and collision stages per node, double precision throughout,
 * built with -O2 -ffp-contract=off (no fused multiply-add, no fast-math).
 * Rows may be split over OpenMP threads; every node is computed from the
 * previous state only, so the result does not depend on the thread count.
 *
 * State layout: post-collision populations in one array of 19 planes,
 * plane-major, each plane [ny][nx] with x fastest:
 *   planes 0..8   f_alpha        (D2Q9, Sec. V)
 *   planes 9..13  g_{alpha x}    (D2Q5 vector distribution, x component)
 *   planes 14..18 g_{alpha y}    (D2Q5, y component)
 * x is periodic (a channel) or bounded by stationary link-closed Shercliff
 * walls at x = -1/2 and nx - 1/2 (an enclosure); the Hartmann walls bound
 * y: row 0 is the lower wall side (y = -a), row ny-1 the upper (y = +a).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NQ9 9
#define NQ5 5
#define NPLANES 19

/* D2Q9 velocity set.  The paper's lattice figure is missing from the text; the
 * numbering is fixed by the moment sums of App. A (Pi_10, Pi_01, Pi_20 in terms
 * of f_1..f_8) and by the lower-wall unknowns being {2,5,6}. */
static const int EX9[NQ9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY9[NQ9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* Weights of Sec. V. */
static const double W9[NQ9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                               1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                               1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP9[NQ9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

/* D2Q5 velocity set for the vector distribution (Sec. IV); numbering fixed by
 * Lambda_yx = g_2x - g_4x in the moment closure (Sec. VII) and e_4y = -1
 * (App. B.1). */
static const int EX5[NQ5] = {0, 1, 0, -1, 0};
static const int EY5[NQ5] = {0, 0, 1, 0, -1};
static const double W5[NQ5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0,
                               1.0 / 6.0};
static const int OPP5[NQ5] = {0, 3, 4, 1, 2};

static const double CS2 = 1.0 / 3.0;  /* c_s^2, Sec. V */
static const double CSM2 = 1.0 / 3.0; /* c_sm^2, Sec. IV */

enum { ORC_LINK = 0, ORC_MOMENT = 1 };
enum { ORC_LOWER = 0, ORC_UPPER = 1 };
/* Collision operator: the paper's single-relaxation-time (BGK) form, or the
 * two-relaxation-time form it names as a drop-in replacement (Secs. V and
 * IX).  Under TRT the rates that set the transport coefficients keep their
 * meaning: tau_f relaxes the even (symmetric) part of f, giving nu, and
 * tau_m the odd (antisymmetric) part of g, giving eta; tau_fm and tau_mp are
 * the free rates of the other halves. */
enum { ORC_BGK = 0, ORC_TRT = 1, ORC_MRT = 2 };

typedef struct {
  int32_t nx, ny, bc, collision;
  double tau_f, tau_m; /* relaxation times of f and g */
  double b0;           /* imposed field, along +y */
  double fx, fy;       /* external body force F_ext */
  double c_lo, c_hi;   /* wall conductance ratios c_w (0 .. INFINITY) */
  double u_lo, u_hi;   /* wall velocities along x */
  double a;            /* half-width H = a entering theta and 1/(c_w a) */
  double tau_fm;       /* TRT: relaxation time of the odd part of f */
  double tau_mp;       /* TRT: relaxation time of the even part of g */
  int32_t x_walls, pad_; /* 1: an enclosure, stationary walls at x = -1/2 and nx - 1/2 */
  double cx_lo, cx_hi;   /* their wall conductance ratios (0 .. INFINITY) */
  double q_lo, q_hi;     /* link scheme: distance of each Hartmann wall from its
                            wall row, in (0, 1]; 1/2 is the paper's half-way wall */
  double s_fe, s_feps, s_fq; /* MRT rates of f's e, epsilon and q moments */
  double s_me, s_md;         /* MRT rates of g's epsilon and d moments */
  int32_t nsolid, pad2_;     /* solid bodies (curved walls), at most ORC_MAX_SOLIDS */
  struct orc_solid {
    int32_t kind, pad_;      /* ORC_SOLID_* */
    double cx, cy, r;        /* circle: centre and radius; half-plane: cy = its edge y0 */
    double omega;            /* circle: angular velocity of its surface (counterclockwise) */
    double u;                /* half-plane: its velocity along x */
  } solid[4];
} orc_params;

/* Solid bodies, in lattice units with node (i, j) at the point (i, j); x is
 * periodic, so a circle also covers its images one period away.  A node is
 * solid if it lies strictly inside a body.  DISC: solid inside the circle;
 * BORE: solid outside it; BELOW / ABOVE: solid where y < cy / y > cy. */
enum { ORC_SOLID_DISC = 1, ORC_SOLID_BORE = 2, ORC_SOLID_BELOW = 3, ORC_SOLID_ABOVE = 4 };
#define ORC_MAX_SOLIDS 4

/* ---------------------------------------------------------------------- */
/* Equilibria and source (Secs. IV and V)                                 */
/* ---------------------------------------------------------------------- */

/* f^eq of Sec. V: w rho [1 + e.u/cs2 + (e.u)^2/(2 cs2^2) - u.u/(2 cs2)]. */
void orc_feq(double rho, double ux, double uy, double *feq) {
  const double uu = ux * ux + uy * uy;
  for (int q = 0; q < NQ9; ++q) {
    const double eu = EX9[q] * ux + EY9[q] * uy;
    feq[q] = W9[q] * rho *
             (1.0 + eu / CS2 + (eu * eu) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
  }
}

/* g^eq of Sec. IV, Eq. (geqmagneticfield):
 *   g^eq_{alpha i} = W_alpha { B_i + e_{alpha j} (u_j B_i - B_j u_i) / cs2m }
 * written with the sum over j spelled out. */
void orc_geq(double bx, double by, double ux, double uy, double *geqx,
             double *geqy) {
  const double u[2] = {ux, uy};
  const double b[2] = {bx, by};
  for (int q = 0; q < NQ5; ++q) {
    const int e[2] = {EX5[q], EY5[q]};
    double out[2];
    for (int i = 0; i < 2; ++i) {
      double flux = 0.0;
      for (int j = 0; j < 2; ++j) flux += e[j] * (u[j] * b[i] - b[j] * u[i]);
      out[i] = W5[q] * (b[i] + flux / CSM2);
    }
    geqx[q] = out[0];
    geqy[q] = out[1];
  }
}

/* Source of Sec. V: S_alpha = (e_alpha - u).F f^eq_alpha / (rho cs2). */
void orc_source(double rho, double ux, double uy, double Fx, double Fy,
                const double *feq, double *S) {
  for (int q = 0; q < NQ9; ++q) {
    const double dot = (EX9[q] - ux) * Fx + (EY9[q] - uy) * Fy;
    S[q] = dot * feq[q] / (rho * CS2);
  }
}

/* ---------------------------------------------------------------------- */
/* Coupled local solve for u and J_z                                      */
/* ---------------------------------------------------------------------- */
/*
 * The velocity uses the half-force correction rho u = sum f e + F/2 (Sec. V),
 * the force contains the Lorentz part J x B (Sec. II), and J_z comes from the
 * non-equilibrium part of Lambda (Sec. IV):
 *   J_z = dB_y/dx - dB_x/dy
 *       = -(1/(tau_m cs2m)) [ (Lambda_xy - L0_xy) - (Lambda_yx - L0_yx) ],
 *   L0_ji = u_j B_i - B_j u_i.
 * The paper does not say how the implicit u <-> J dependence is resolved; this
 * oracle takes the three relations as simultaneous linear equations in
 * (u_x, u_y, J_z) and solves them by Gaussian elimination with partial
 * pivoting:
 *   rho u_x + (B_y/2) J_z                    = m_x + F_ext,x/2
 *   rho u_y - (B_x/2) J_z                    = m_y + F_ext,y/2
 *   -2k B_y u_x + 2k B_x u_y + J_z           = -k (Lambda_xy - Lambda_yx)
 * with k = 1/(tau_m cs2m).
 */
void orc_local_solve(double rho, double mx, double my, double bx, double by,
                     double lxy, double lyx, double tau_m, double fex,
                     double fey, double *out /* ux, uy, jz */) {
  const double k = 1.0 / (tau_m * CSM2);
  double M[3][4] = {
      {rho, 0.0, by / 2.0, mx + fex / 2.0},
      {0.0, rho, -bx / 2.0, my + fey / 2.0},
      {-2.0 * k * by, 2.0 * k * bx, 1.0, -k * (lxy - lyx)},
  };
  for (int c = 0; c < 3; ++c) {
    int piv = c;
    for (int r = c + 1; r < 3; ++r)
      if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
    if (piv != c)
      for (int k2 = 0; k2 < 4; ++k2) {
        const double t = M[c][k2];
        M[c][k2] = M[piv][k2];
        M[piv][k2] = t;
      }
    for (int r = c + 1; r < 3; ++r) {
      const double fac = M[r][c] / M[c][c];
      for (int k2 = c; k2 < 4; ++k2) M[r][k2] -= fac * M[c][k2];
    }
  }
  double x[3];
  for (int r = 2; r >= 0; --r) {
    double s = M[r][3];
    for (int k2 = r + 1; k2 < 3; ++k2) s -= M[r][k2] * x[k2];
    x[r] = s / M[r][r];
  }
  out[0] = x[0];
  out[1] = x[1];
  out[2] = x[2];
}

/* ---------------------------------------------------------------------- */
/* Wall closures                                                          */
/* ---------------------------------------------------------------------- */

/*
 * Link-based closures (Sec. VI, App. B.1).  The wall sits half-way between
 * the wall-row node x_f and the ghost node.  `own` holds the node's own
 * post-collision populations of the previous step (all 19 planes); the
 * incoming populations (those whose upstream node is the ghost) are set in
 * f, gx, gy.
 *   f:    half-way bounce-back with the moving-wall momentum term of App. B.1,
 *         f_alpha = f~_abar + 2 w_alpha e_{alpha x} U_w / cs2.
 *   g_x:  Shercliff closure, Eq. (movingwalllinkbasedclosure):
 *         g_alpha = ((theta-1)/(theta+1)) g~_abar
 *                   - (2 theta/(theta+1)) W_alpha (e_{alpha y}/cs2m) B0 U_w,
 *         theta = c_w a / (tau_m - 1/2)   (Eq. weightingfactor, H = a);
 *         c_w = INFINITY takes the perfectly conducting limit of App. B.1(b).
 *   g_y:  Dirichlet B_y = B0 from Eq. (magneticfieldanditsgradientrelation1):
 *         g_alpha = -g~_abar + 2 W_alpha B0.  (The upper-wall example prints
 *         the outgoing population as g~_4y; the outgoing direction at the
 *         upper wall is 2, so g~_2y is used.)
 */
void orc_link_closure(const orc_params *p, int wall, const double *own,
                      double *f, double *gx, double *gy) {
  const int ey_in = (wall == ORC_LOWER) ? +1 : -1; /* incoming e_y */
  const double cw = (wall == ORC_LOWER) ? p->c_lo : p->c_hi;
  const double uw = (wall == ORC_LOWER) ? p->u_lo : p->u_hi;
  for (int q = 0; q < NQ9; ++q) {
    if (EY9[q] != ey_in) continue;
    f[q] = own[OPP9[q]] + 2.0 * W9[q] * EX9[q] * uw / CS2;
  }
  for (int q = 0; q < NQ5; ++q) {
    if (EY5[q] != ey_in) continue;
    const double gbar_x = own[9 + OPP5[q]];
    const double gbar_y = own[14 + OPP5[q]];
    const double moving = W5[q] * (EY5[q] / CSM2) * p->b0 * uw;
    if (isinf(cw)) {
      gx[q] = gbar_x - 2.0 * moving;
    } else {
      const double theta = cw * p->a / (p->tau_m - 0.5);
      gx[q] = ((theta - 1.0) / (theta + 1.0)) * gbar_x -
              (2.0 * theta / (theta + 1.0)) * moving;
    }
    gy[q] = -gbar_y + 2.0 * W5[q] * p->b0;
  }
}

/*
 * Link-based closure with the Hartmann wall at a distance q (0 < q <= 1)
 * from the wall row instead of half-way (the paper names link-based walls at
 * other cut distances as future work, Sec. IX).  in is the whole
 * post-collision state and (x, y) the wall-row node; the closure reads the
 * node itself and the next nodes into the fluid along the wall normal.
 *   f: linear interpolated bounce-back (Bouzidi, Firdaouss and Lallemand,
 *      Phys. Fluids 13 (2001) 3452) with the moving-wall term scaled as in
 *      Lallemand and Luo, J. Comput. Phys. 184 (2003) 406:
 *        q <  1/2: f_a = 2q f~_abar + (1-2q) f~_abar(x + e_a) + 2 w e_ax U / cs2
 *        q >= 1/2: f_a = f~_abar / (2q) + (1 - 1/(2q)) f~_a + w e_ax U / (q cs2)
 *   g, a field component with the wall value zero (the normal component's
 *      induced part, or any component at an insulating wall): interpolated
 *      anti-bounce-back, exact for linear profiles,
 *        q <  1/2: g_a = -2q g~_abar + (2q-1) g~_abar(x + e_a)
 *        q >= 1/2: g_a = -g~_abar / (2q) + (1 - 1/(2q)) g~_a
 *      (induced parts: g_y is taken minus W B0 on both sides).
 *   g, the tangential component at a conducting wall (0 < c <= inf).  Its
 *      outgoing post-collision populations at the wall row and the next two
 *      nodes, o0, o1, o2, give the closure
 *        g_a = r o0 + kappa (o2 - 2 o1 + o0) - (1 + r) W (e_ay/cs2m) B0 U.
 *      With the first-order Chapman-Enskog populations
 *      g~ = g^eq - (tau_m - 1) W e.grad b of a quadratic profile and the
 *      thin-wall condition c a db/dn + b = 0 at the wall, the first two
 *      Taylor orders fix
 *        r = (C + q - tau_m) / (C + q + tau_m - 1),   C = c a (r = 1 at c = inf),
 *        kappa = Bt - r B0 - (1 - r) K,
 *        B0 = q^2/2 + (tau_m-1) q,  Bt = (1-q)^2/2 + (tau_m-1)(1-q),
 *        K = 1/8 + (tau_m-1)/2,
 *      which cancels the curvature term of order c a (1/2 - q) b'' that
 *      would otherwise make the wall condition first order.  At q = 1/2,
 *      kappa = 0 and r = (theta-1)/(theta+1), theta = c a / (tau_m - 1/2):
 *      the paper's closure.  The moving-wall term is the paper's with the
 *      factor 1 + r.
 */
static inline size_t idx(const orc_params *p, int plane, int y, int x);

void orc_link_closure_q(const orc_params *p, int wall, const double *in, int x, int y,
                        double *f, double *gx, double *gy) {
  const int ey_in = (wall == ORC_LOWER) ? +1 : -1;
  const double cw = (wall == ORC_LOWER) ? p->c_lo : p->c_hi;
  const double uw = (wall == ORC_LOWER) ? p->u_lo : p->u_hi;
  const double q = (wall == ORC_LOWER) ? p->q_lo : p->q_hi;
  const double tau = p->tau_m;
#define ST(plane, yy, xx) in[idx(p, (plane), (yy), ((xx) % p->nx + p->nx) % p->nx)]
  double defect = 0.0, win = 0.0;
  for (int a = 0; a < NQ9; ++a) {
    if (EY9[a] != ey_in) continue;
    const double ladd = 2.0 * W9[a] * EX9[a] * uw / CS2;
    const double out0 = ST(OPP9[a], y, x);
    if (q < 0.5)
      f[a] = 2.0 * q * out0 + (1.0 - 2.0 * q) * ST(OPP9[a], y + EY9[a], x + EX9[a]) + ladd;
    else
      f[a] = out0 / (2.0 * q) + (1.0 - 1.0 / (2.0 * q)) * ST(a, y, x) + ladd / (2.0 * q);
    defect += out0 - f[a];
    win += W9[a];
  }
  /* the mass the wall would let through (non-zero when the post-collision
   * populations are asymmetric about the wall normal, as under a normal
   * force) goes back into the incoming populations in proportion to their
   * weights, so that no mass crosses the wall, as with bounce-back */
  for (int a = 0; a < NQ9; ++a)
    if (EY9[a] == ey_in) f[a] += defect * W9[a] / win;
  /* the D2Q5 link entering from the wall: a = 2 (lower) or 4 (upper) */
  const int a = (wall == ORC_LOWER) ? 2 : 4, o = OPP5[a];
  const double wb0 = W5[a] * p->b0;
  /* interpolated anti-bounce-back of a field component with wall value 0;
   * dev is subtracted from every population (W B0 for g_y) */
  double zero_wall[2];
  for (int i = 0; i < 2; ++i) {
    const int base = 9 + 5 * i;
    const double dev = (i == 1) ? wb0 : 0.0;
    const double o0 = ST(base + o, y, x) - dev;
    if (q < 0.5)
      zero_wall[i] = -2.0 * q * o0 + (2.0 * q - 1.0) * (ST(base + o, y + ey_in, x) - dev) + dev;
    else
      zero_wall[i] = -o0 / (2.0 * q) + (1.0 - 1.0 / (2.0 * q)) * (ST(base + a, y, x) - dev) + dev;
  }
  gy[a] = zero_wall[1];
  if (cw == 0.0) {
    gx[a] = zero_wall[0];
  } else {
    const double C = cw * p->a;
    const double r = isinf(cw) ? 1.0 : (C + q - tau) / (C + q + tau - 1.0);
    const double B0c = 0.5 * q * q + (tau - 1.0) * q;
    const double Btc = 0.5 * (1.0 - q) * (1.0 - q) + (tau - 1.0) * (1.0 - q);
    const double K = 0.125 + 0.5 * (tau - 1.0);
    const double kappa = Btc - r * B0c - (1.0 - r) * K;
    const double o0 = ST(9 + o, y, x), o1 = ST(9 + o, y + ey_in, x),
                 o2 = ST(9 + o, y + 2 * ey_in, x);
    const double moving = W5[a] * (EY5[a] / CSM2) * p->b0 * uw;
    /* the flux part 3 W e_y B0 u_x of the equilibria leaves, through the
     * wall-normal shear du/dn = (u_x - U)/q, a mismatch (1/2 - q)(1 + r)
     * times 3 W e_y B0 du/dn; u_x is the node's velocity from its
     * post-collision momentum */
    double rho_n = 0.0, mx_n = 0.0;
    for (int b = 0; b < NQ9; ++b) {
      rho_n += ST(b, y, x);
      mx_n += EX9[b] * ST(b, y, x);
    }
    const double dudn = (mx_n / rho_n - uw) / q;
    const double shear = (0.5 - q) * (1.0 + r) * W5[a] * (EY5[a] / CSM2) * p->b0 * dudn;
    gx[a] = r * o0 + kappa * (o2 - 2.0 * o1 + o0) - (1.0 + r) * moving + shear;
  }
#undef ST
}

/*
 * Walls of an enclosure at x = -1/2 (lower, wall = ORC_LOWER) and
 * x = nx - 1/2 (upper), parallel to the imposed field: stationary,
 * link-based, applied to every link whose source lies behind the wall:
 *   f:   half-way bounce-back;
 *   g_y: the tangential component; the theta-weighted Shercliff closure of
 *        Sec. VI on the induced field b_y = B_y - B0,
 *          g_in,y - W B0 = r (g~_out,y - W B0),  r = (theta-1)/(theta+1),
 *        theta = c_w a / (tau_m - 1/2) with the Hartmann half-width a;
 *        c_w = INFINITY gives r = 1;
 *   g_x: the normal component; anti-bounce-back to B_x = 0,
 *          g_in,x = -g~_out,x.
 * At a corner the links that also cross a Hartmann wall are closed by that
 * wall afterwards (its moving-wall term included), which keeps the moving
 * wall's mass balance.
 */
void orc_xwall_closure(const orc_params *p, int wall, const double *own, double *f,
                       double *gx, double *gy) {
  const int ex_in = (wall == ORC_LOWER) ? +1 : -1;
  const double cw = (wall == ORC_LOWER) ? p->cx_lo : p->cx_hi;
  double r = 1.0;
  if (!isinf(cw)) {
    const double theta = cw * p->a / (p->tau_m - 0.5);
    r = (theta - 1.0) / (theta + 1.0);
  }
  for (int q = 0; q < NQ9; ++q)
    if (EX9[q] == ex_in) f[q] = own[OPP9[q]];
  for (int q = 0; q < NQ5; ++q) {
    if (EX5[q] != ex_in) continue;
    const double wb0 = W5[q] * p->b0;
    gy[q] = r * (own[14 + OPP5[q]] - wb0) + wb0;
    gx[q] = -own[9 + OPP5[q]];
  }
}

/*
 * On-node ("wet") moment-based closures (Sec. VII, App. A, App. B.2).
 * f, gx, gy hold the post-streaming populations at the wall node; the
 * unknowns are overwritten.
 *   f:   constraints Pi_10 = rho U_w, Pi_01 = 0, Pi_20 = rho (cs2 + U_w^2)
 *        with rho from the known populations; closures of App. A (stationary)
 *        and App. B.2 (moving upper wall).  App. B.2 prints the first two
 *        constraints with Pi_10 and Pi_01 swapped; the printed closures satisfy
 *        the reading used here.  The moving lower wall is the mirror image.
 *   g_x: Shercliff constraint with Lambda_yx = g_2x - g_4x:
 *          lower:  A (g_2x - g_4x + B0 U) + C sum_a g_ax = 0
 *          upper: -A (g_2x - g_4x + B0 U) + C sum_a g_ax = 0
 *        A = 1/(tau_m cs2m), C = 1/(c_w a), solved for the unknown as in
 *        Eqs. (momentbasedBCslowerboundary), (momentbasedBCsupperboundary) and
 *        (momentbasedclosureformovingwall); c_w = 0 and c_w = INFINITY take the
 *        limits printed after them.
 *   g_y: sum_a g_ay = B0.
 */
void orc_moment_closure(const orc_params *p, int wall, double *f, double *gx,
                        double *gy) {
  const double cw = (wall == ORC_LOWER) ? p->c_lo : p->c_hi;
  const double U = (wall == ORC_LOWER) ? p->u_lo : p->u_hi;
  const double A = 1.0 / (p->tau_m * CSM2);
  if (wall == ORC_LOWER) {
    const double rho = f[0] + f[1] + f[3] + 2.0 * (f[4] + f[7] + f[8]);
    f[2] = -rho * (CS2 + U * U) + f[1] + f[3] + f[4] + 2.0 * (f[7] + f[8]);
    f[5] = 0.5 * rho * (CS2 + U * U + U) - (f[1] + f[8]);
    f[6] = 0.5 * rho * (CS2 + U * U - U) - (f[3] + f[7]);
    const double others = gx[0] + gx[1] + gx[3];
    if (cw == 0.0) {
      gx[2] = -(others + gx[4]);
    } else if (isinf(cw)) {
      gx[2] = gx[4] - p->b0 * U;
    } else {
      const double C = 1.0 / (cw * p->a);
      gx[2] = ((A - C) * gx[4] - C * others - A * p->b0 * U) / (A + C);
    }
    gy[2] = p->b0 - (gy[0] + gy[1] + gy[3] + gy[4]);
  } else {
    const double rho = f[0] + f[1] + f[3] + 2.0 * (f[2] + f[5] + f[6]);
    f[4] = -rho * (CS2 + U * U) + f[1] + f[2] + f[3] + 2.0 * (f[5] + f[6]);
    f[7] = 0.5 * rho * (CS2 + U * U - U) - (f[3] + f[6]);
    f[8] = 0.5 * rho * (CS2 + U * U + U) - (f[1] + f[5]);
    const double others = gx[0] + gx[1] + gx[3];
    if (cw == 0.0) {
      gx[4] = -(others + gx[2]);
    } else if (isinf(cw)) {
      gx[4] = gx[2] + p->b0 * U;
    } else {
      const double C = 1.0 / (cw * p->a);
      gx[4] = ((A - C) * gx[2] - C * others + A * p->b0 * U) / (A + C);
    }
    gy[4] = p->b0 - (gy[0] + gy[1] + gy[2] + gy[3]);
  }
}

/* ---------------------------------------------------------------------- */
/* Curved walls: link-based closures on the surfaces of solid bodies       */
/* ---------------------------------------------------------------------- */
/*
 * The paper closes straight Hartmann walls only and names curved walls,
 * walls that cut the links at distances other than one half, as future work
 * (Sec. IX).  This is the reading taken here.  A fluid node's population f_a
 * whose upstream node x - e_a is solid is closed on that link, with q the
 * fraction of the link from the node to the surface (0 < q <= 1):
 *   f: linear interpolated bounce-back (Bouzidi, Firdaouss and Lallemand
 *      2001) with the moving-wall term 2 w_a e_a.u_w / cs2 at the crossing
 *      point (scaled by 1/(2q) on the far branch, as for the straight walls
 *      at a cut distance above):
 *        q <  1/2: f_a = 2q f~_abar + (1-2q) f~_abar(x + e_a) + m_a
 *        q >= 1/2: f_a = f~_abar / (2q) + (1 - 1/(2q)) f~_a + m_a / (2q)
 *      and half-way bounce-back f~_abar + m_a where q < 1/2 but x + e_a is
 *      solid too.  Unlike bounce-back (q = 1/2) the interpolation does not
 *      conserve mass exactly; the straight cut walls above return the mass
 *      defect to the closed populations, but on a curved surface that
 *      correction acts as a spurious local source and spoils the order of
 *      convergence (circular Couette flow: 2-6% errors that do not fall with
 *      resolution, against 0.7%, 0.14%, 0.026% without it), so here none
 *      is applied;
 *   g: the body holds the induced field at zero, B = (0, B0) on its surface
 *      (an insulating body that field lines cross undisturbed): interpolated
 *      anti-bounce-back of each component's deviation from W_a B_wall on the
 *      D2Q5 links, with the same branches.
 * At q = 1/2 this is the paper's link-based closure of an insulating
 * (c_w = 0) Hartmann wall (Sec. VI): half-way bounce-back with Ladd's term
 * and anti-bounce-back of g to B_x = 0, B_y = B0.
 */
static inline size_t idx(const orc_params *p, int plane, int y, int x) {
  return ((size_t)plane * (size_t)p->ny + (size_t)y) * (size_t)p->nx + (size_t)x;
}

/* x offset of a point from a circle's centre, taken to the nearest image. */
static double body_dx(const orc_params *p, double X, double cx) {
  double dx = X - cx;
  if (!p->x_walls) {
    const double L = (double)p->nx;
    dx -= L * floor(dx / L + 0.5);
  }
  return dx;
}

static int inside_body(const orc_params *p, const struct orc_solid *b, double X, double Y) {
  switch (b->kind) {
  case ORC_SOLID_DISC:
  case ORC_SOLID_BORE: {
    const double dx = body_dx(p, X, b->cx), dy = Y - b->cy;
    const double d2 = dx * dx + dy * dy, r2 = b->r * b->r;
    return b->kind == ORC_SOLID_DISC ? d2 < r2 : d2 > r2;
  }
  case ORC_SOLID_BELOW: return Y < b->cy;
  case ORC_SOLID_ABOVE: return Y > b->cy;
  default: return 0;
  }
}

int orc_is_solid(const orc_params *p, int x, int y) {
  for (int k = 0; k < p->nsolid; ++k)
    if (inside_body(p, &p->solid[k], (double)x, (double)y)) return 1;
  return 0;
}

/* The link from fluid node (x, y) towards its upstream node (x, y) - e_a:
 * returns 1 and the surface distance q (fraction of the link) and the
 * surface velocity where a body contains the upstream node, the nearest
 * crossing if several do. */
int orc_link_cut(const orc_params *p, int x, int y, int a, double *q, double *uwx,
                 double *uwy) {
  const double ex = EX9[a], ey = EY9[a];
  const double ux = x - ex, uy = y - ey; /* upstream point */
  int found = 0;
  double best = 2.0;
  for (int k = 0; k < p->nsolid; ++k) {
    const struct orc_solid *b = &p->solid[k];
    if (!inside_body(p, b, ux, uy)) continue;
    double t, wx = 0.0, wy = 0.0;
    if (b->kind == ORC_SOLID_DISC || b->kind == ORC_SOLID_BORE) {
      /* |P - t e - c| = r along the link from the node (P) */
      const double px = body_dx(p, (double)x, b->cx), py = (double)y - b->cy;
      const double ee = ex * ex + ey * ey, pe = px * ex + py * ey;
      const double disc = pe * pe - ee * (px * px + py * py - b->r * b->r);
      const double sq = sqrt(disc > 0.0 ? disc : 0.0);
      /* entering a disc: the first root; leaving a bore: the second */
      t = (b->kind == ORC_SOLID_DISC ? pe - sq : pe + sq) / ee;
      wx = -b->omega * (py - t * ey);
      wy = b->omega * (px - t * ex);
    } else {
      t = ((double)y - b->cy) / ey;
      wx = b->u;
    }
    if (t <= 0.0) t = 1e-12; /* a node on the surface itself */
    if (t > 1.0) t = 1.0;
    if (t < best) {
      best = t;
      *uwx = wx;
      *uwy = wy;
      found = 1;
    }
  }
  if (found) *q = best;
  return found;
}

/* Closure of every link of fluid node (x, y) that comes from a solid node;
 * `in` is the whole post-collision state. */
static void curved_closure(const orc_params *p, const double *in, int x, int y, double *f,
                           double *gx, double *gy) {
#define ST(plane, yy, xx) in[idx(p, (plane), (yy), ((xx) % p->nx + p->nx) % p->nx)]
  int cut[NQ9] = {0};
  double qa[NQ9] = {0.0};
  int nearok[NQ9] = {0};
  for (int a = 1; a < NQ9; ++a) {
    double q, uwx = 0.0, uwy = 0.0;
    if (!orc_link_cut(p, x, y, a, &q, &uwx, &uwy)) continue;
    cut[a] = 1;
    qa[a] = q;
    const int nxp = x + EX9[a], nyp = y + EY9[a]; /* next node into the fluid */
    nearok[a] = q < 0.5 && nyp >= 0 && nyp < p->ny &&
                !orc_is_solid(p, ((nxp % p->nx) + p->nx) % p->nx, nyp);
    const double m = 2.0 * W9[a] * (EX9[a] * uwx + EY9[a] * uwy) / CS2;
    const double o = ST(OPP9[a], y, x);
    if (nearok[a])
      f[a] = 2.0 * q * o + (1.0 - 2.0 * q) * ST(OPP9[a], nyp, nxp) + m;
    else if (q >= 0.5)
      f[a] = o / (2.0 * q) + (1.0 - 1.0 / (2.0 * q)) * ST(a, y, x) + m / (2.0 * q);
    else
      f[a] = o + m;
  }
  /* D2Q5: the axis links 1..4 (same directions as D2Q9's) */
  for (int a = 1; a < NQ5; ++a) {
    if (!cut[a]) continue;
    const double q = qa[a];
    const int o = OPP5[a];
    double *g[2] = {gx, gy};
    for (int i = 0; i < 2; ++i) {
      const int base = 9 + 5 * i;
      const double dev = (i == 1) ? W5[a] * p->b0 : 0.0; /* W_a B_wall,i */
      const double ov = ST(base + o, y, x) - dev;
      double v;
      if (nearok[a])
        v = -2.0 * q * ov + (2.0 * q - 1.0) * (ST(base + o, y + EY5[a], x + EX5[a]) - dev);
      else if (q >= 0.5)
        v = -ov / (2.0 * q) + (1.0 - 1.0 / (2.0 * q)) * (ST(base + a, y, x) - dev);
      else
        v = -ov;
      g[i][a] = v + dev;
    }
  }
#undef ST
}

/* ---------------------------------------------------------------------- */
/* One node: stream, close, moments, solve; optionally collide            */
/* ---------------------------------------------------------------------- */

typedef struct {
  double f[NQ9], gx[NQ5], gy[NQ5];
  double rho, ux, uy, bx, by, jz, Fx, Fy;
} node_t;

/* Rest state of a solid node: equilibrium at rho = 1, u = 0, B = (0, B0). */
static void rest_node(const orc_params *p, node_t *n) {
  orc_feq(1.0, 0.0, 0.0, n->f);
  orc_geq(0.0, p->b0, 0.0, 0.0, n->gx, n->gy);
  n->rho = 1.0;
  n->ux = n->uy = n->jz = n->Fx = n->Fy = 0.0;
  n->bx = 0.0;
  n->by = p->b0;
}

static void gather_node(const orc_params *p, const double *in, int x, int y,
                        node_t *n) {
  if (p->nsolid > 0 && orc_is_solid(p, x, y)) {
    rest_node(p, n);
    return;
  }
  /* S1: pull streaming, f_alpha(x) = f~_alpha(x - e_alpha) (Eqs.
   * LBMforflowfield, LKSformagneticfield); x periodic, or bounded by walls
   * in an enclosure. */
  for (int q = 0; q < NQ9; ++q) {
    const int sy = y - EY9[q];
    const int rx = x - EX9[q];
    const int inx = !p->x_walls || (rx >= 0 && rx < p->nx);
    const int sx = (rx % p->nx + p->nx) % p->nx;
    n->f[q] = (sy >= 0 && sy < p->ny && inx) ? in[idx(p, q, sy, sx)] : NAN;
  }
  for (int q = 0; q < NQ5; ++q) {
    const int sy = y - EY5[q];
    const int rx = x - EX5[q];
    const int inx = !p->x_walls || (rx >= 0 && rx < p->nx);
    const int sx = (rx % p->nx + p->nx) % p->nx;
    const int ok = (sy >= 0 && sy < p->ny && inx);
    n->gx[q] = ok ? in[idx(p, 9 + q, sy, sx)] : NAN;
    n->gy[q] = ok ? in[idx(p, 14 + q, sy, sx)] : NAN;
  }
  /* S2: wall closures; enclosure walls first, the Hartmann walls then take
   * the corner links that cross them. */
  const int xwall = p->x_walls && ((x == 0) || (x == p->nx - 1));
  const int nwall = (y == 0) + (y == p->ny - 1);
  if (xwall) {
    double own[NPLANES];
    for (int k = 0; k < NPLANES; ++k) own[k] = in[idx(p, k, y, x)];
    if (x == 0) orc_xwall_closure(p, ORC_LOWER, own, n->f, n->gx, n->gy);
    if (x == p->nx - 1) orc_xwall_closure(p, ORC_UPPER, own, n->f, n->gx, n->gy);
  }
  if (nwall) {
    double own[NPLANES];
    for (int k = 0; k < NPLANES; ++k) own[k] = in[idx(p, k, y, x)];
    for (int w = 0; w < 2; ++w) {
      if (!(w == ORC_LOWER ? y == 0 : y == p->ny - 1)) continue;
      const double qw = (w == ORC_LOWER) ? p->q_lo : p->q_hi;
      if (p->bc != ORC_LINK) {
        orc_moment_closure(p, w, n->f, n->gx, n->gy);
      } else if (qw == 0.5) {
        orc_link_closure(p, w, own, n->f, n->gx, n->gy);
      } else {
        orc_link_closure_q(p, w, in, x, y, n->f, n->gx, n->gy);
      }
    }
  }
  /* S2b: links from solid bodies (curved walls) */
  if (p->nsolid > 0) curved_closure(p, in, x, y, n->f, n->gx, n->gy);
  /* S3: moments (Secs. IV, V). */
  double rho = 0.0, mx = 0.0, my = 0.0;
  for (int q = 0; q < NQ9; ++q) {
    rho += n->f[q];
    mx += n->f[q] * EX9[q];
    my += n->f[q] * EY9[q];
  }
  double bx = 0.0, by = 0.0, lam[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int q = 0; q < NQ5; ++q) {
    const int e[2] = {EX5[q], EY5[q]};
    const double g[2] = {n->gx[q], n->gy[q]};
    bx += g[0];
    by += g[1];
    for (int j = 0; j < 2; ++j)
      for (int i = 0; i < 2; ++i) lam[j][i] += e[j] * g[i]; /* Lambda_ji */
  }
  n->rho = rho;
  n->bx = bx;
  n->by = by;
  if (nwall && p->bc == ORC_MOMENT) {
    /* Wet wall node: the closure has fixed its velocity through the moments,
     * sum f e = rho (U_w, 0) (App. A, App. B.2).  It is a Dirichlet node: no
     * force enters its collision, u = sum f e / rho, and J_z follows from the
     * non-equilibrium part of Lambda with that u (Sec. IV). */
    const double k = 1.0 / (p->tau_m * CSM2);
    n->ux = mx / rho;
    n->uy = my / rho;
    const double l0xy = n->ux * by - bx * n->uy; /* u_x B_y - B_x u_y */
    const double l0yx = n->uy * bx - by * n->ux; /* u_y B_x - B_y u_x */
    n->jz = -k * ((lam[0][1] - l0xy) - (lam[1][0] - l0yx));
    n->Fx = 0.0;
    n->Fy = 0.0;
    return;
  }
  /* S4: coupled local solve and total force. */
  double sol[3];
  orc_local_solve(rho, mx, my, bx, by, lam[0][1], lam[1][0], p->tau_m, p->fx,
                  p->fy, sol);
  n->ux = sol[0];
  n->uy = sol[1];
  n->jz = sol[2];
  n->Fx = p->fx - sol[2] * by; /* (J x B)_x = -J_z B_y */
  n->Fy = p->fy + sol[2] * bx; /* (J x B)_y = +J_z B_x */
}

/* S5: collide one node (Eqs. LBMforflowfield and LKSformagneticfield).
 * f, gx, gy are the post-streaming, post-closure populations; rho, u, B and
 * F the fields of S3-S4.  out receives the 19 post-collision values in plane
 * order.
 *
 * BGK: every population relaxes to its equilibrium at 1/tau, and the source
 * enters with the weight 1 - 1/(2 tau) (Sec. V).
 * TRT: each population splits into the parts even and odd under e -> -e,
 *   h+_a = (h_a + h_abar)/2,  h-_a = (h_a - h_abar)/2,
 * for h = f, f^eq, S (and g, g^eq), and each part relaxes at its own rate,
 * the source part with the matching weight 1 - 1/(2 tau+-).  The rest
 * population is even.
 * MRT: populations map to moments (the bases above); each moment's
 * non-equilibrium part relaxes at its own rate, the source's moment with the
 * matching weight, and the moments map back.  The paper names multiple
 * relaxation times as a replacement for BGK (Secs. V and IX) without fixing
 * a basis; these are the usual orthogonal ones. */
/* MRT moment bases.  f (D2Q9, Lallemand & Luo 2000): rows rho, e, epsilon,
 * j_x, q_x, j_y, q_y, p_xx, p_xy.  g (D2Q5, each component): rows B,
 * Lambda_x, Lambda_y, epsilon, d.  The rows of each are orthogonal, so
 * M^-1 = M^T diag(1 / |row|^2). */
static const double MRT9[NQ9][NQ9] = {{1, 1, 1, 1, 1, 1, 1, 1, 1},
                                      {-4, -1, -1, -1, -1, 2, 2, 2, 2},
                                      {4, -2, -2, -2, -2, 1, 1, 1, 1},
                                      {0, 1, 0, -1, 0, 1, -1, -1, 1},
                                      {0, -2, 0, 2, 0, 1, -1, -1, 1},
                                      {0, 0, 1, 0, -1, 1, 1, -1, -1},
                                      {0, 0, -2, 0, 2, 1, 1, -1, -1},
                                      {0, 1, -1, 1, -1, 0, 0, 0, 0},
                                      {0, 0, 0, 0, 0, 1, -1, 1, -1}};
static const double MRT5[NQ5][NQ5] = {{1, 1, 1, 1, 1},
                                      {0, 1, 0, -1, 0},
                                      {0, 0, 1, 0, -1},
                                      {-4, 1, 1, 1, 1},
                                      {0, 1, -1, 1, -1}};

/* One MRT update of n populations h with basis rows M (n x n, row-major):
 * the non-equilibrium part of moment k relaxes at rate s[k] and the
 * source's moment k (src may be NULL) enters with weight 1 - s[k]/2. */
static void mrt_update(int n, const double *M, const double *s, const double *h,
                       const double *heq, const double *src, double *out) {
  double c[NQ9];
  for (int k = 0; k < n; ++k) {
    double neq = 0.0, ms = 0.0, norm = 0.0;
    for (int a = 0; a < n; ++a) {
      neq += M[k * n + a] * (h[a] - heq[a]);
      if (src) ms += M[k * n + a] * src[a];
      norm += M[k * n + a] * M[k * n + a];
    }
    c[k] = (-s[k] * neq + (1.0 - 0.5 * s[k]) * ms) / norm;
  }
  for (int a = 0; a < n; ++a) {
    double d = 0.0;
    for (int k = 0; k < n; ++k) d += M[k * n + a] * c[k];
    out[a] = h[a] + d;
  }
}

void orc_collide(const orc_params *p, const double *f, const double *gx,
                 const double *gy, double rho, double ux, double uy, double bx,
                 double by, double Fx, double Fy, double *out) {
  double feq[NQ9], S[NQ9], geqx[NQ5], geqy[NQ5];
  orc_feq(rho, ux, uy, feq);
  orc_source(rho, ux, uy, Fx, Fy, feq, S);
  orc_geq(bx, by, ux, uy, geqx, geqy);
  if (p->collision == ORC_MRT) {
    /* f: p_xx and p_xy at s_nu = 1/tau_f (viscosity); e, epsilon, q at their
     * own rates.  rho and j: their non-equilibrium parts are 0 and -F/2 and
     * the forced j update is F at any rate, so their rates do not matter;
     * they take s_nu and s_fq, with which s_fe = s_feps = s_nu is TRT. */
    const double snu = 1.0 / p->tau_f;
    const double sf[NQ9] = {snu, p->s_fe, p->s_feps, p->s_fq, p->s_fq, p->s_fq, p->s_fq, snu, snu};
    mrt_update(NQ9, &MRT9[0][0], sf, f, feq, S, out);
    /* g: Lambda at 1/tau_m (magnetic diffusivity); epsilon and d at their
     * own rates; B (no non-equilibrium part) takes s_me. */
    const double sm[NQ5] = {p->s_me, 1.0 / p->tau_m, 1.0 / p->tau_m, p->s_me, p->s_md};
    mrt_update(NQ5, &MRT5[0][0], sm, gx, geqx, NULL, out + 9);
    mrt_update(NQ5, &MRT5[0][0], sm, gy, geqy, NULL, out + 14);
    return;
  }
  if (p->collision != ORC_TRT) {
    for (int q = 0; q < NQ9; ++q)
      out[q] = f[q] - (f[q] - feq[q]) / p->tau_f +
               (1.0 - 1.0 / (2.0 * p->tau_f)) * S[q];
    for (int q = 0; q < NQ5; ++q) {
      out[9 + q] = gx[q] - (gx[q] - geqx[q]) / p->tau_m;
      out[14 + q] = gy[q] - (gy[q] - geqy[q]) / p->tau_m;
    }
    return;
  }
  /* f: even part at tau_f (viscosity), odd part at tau_fm. */
  const double tfe = p->tau_f, tfo = p->tau_fm;
  for (int q = 0; q < NQ9; ++q) {
    const int r = OPP9[q];
    const double fe = 0.5 * (f[q] + f[r]), fo = 0.5 * (f[q] - f[r]);
    const double ee = 0.5 * (feq[q] + feq[r]), eo = 0.5 * (feq[q] - feq[r]);
    const double se = 0.5 * (S[q] + S[r]), so = 0.5 * (S[q] - S[r]);
    out[q] = f[q] - (fe - ee) / tfe - (fo - eo) / tfo +
             (1.0 - 1.0 / (2.0 * tfe)) * se + (1.0 - 1.0 / (2.0 * tfo)) * so;
  }
  /* g: odd part at tau_m (magnetic diffusivity), even part at tau_mp. */
  const double tme = p->tau_mp, tmo = p->tau_m;
  for (int q = 0; q < NQ5; ++q) {
    const int r = OPP5[q];
    const double *g[2] = {gx, gy}, *ge[2] = {geqx, geqy};
    for (int i = 0; i < 2; ++i) {
      const double he = 0.5 * (g[i][q] + g[i][r]), ho = 0.5 * (g[i][q] - g[i][r]);
      const double ee = 0.5 * (ge[i][q] + ge[i][r]), eo = 0.5 * (ge[i][q] - ge[i][r]);
      out[9 + 5 * i + q] = g[i][q] - (he - ee) / tme - (ho - eo) / tmo;
    }
  }
}

static void step_rows(const orc_params *p, const double *in, double *out,
                      int y0, int y1) {
  for (int y = y0; y < y1; ++y) {
    for (int x = 0; x < p->nx; ++x) {
      node_t n;
      gather_node(p, in, x, y, &n);
      double o[NPLANES];
      if (p->nsolid > 0 && orc_is_solid(p, x, y)) {
        /* a solid node keeps the rest state */
        for (int q = 0; q < NQ9; ++q) o[q] = n.f[q];
        for (int q = 0; q < NQ5; ++q) o[9 + q] = n.gx[q], o[14 + q] = n.gy[q];
      } else {
        orc_collide(p, n.f, n.gx, n.gy, n.rho, n.ux, n.uy, n.bx, n.by, n.Fx, n.Fy, o);
      }
      for (int q = 0; q < NPLANES; ++q) out[idx(p, q, y, x)] = o[q];
    }
  }
}

/* Initial state: equilibrium at rest with density rho0 and B = (0, B0),
 * i.e. zero induced field (solid nodes: rho = 1); stored as post-collision
 * populations. */
void orc_init(const orc_params *p, double rho0, double *state) {
  double feq[NQ9], feq1[NQ9], gex[NQ5], gey[NQ5];
  orc_feq(rho0, 0.0, 0.0, feq);
  orc_feq(1.0, 0.0, 0.0, feq1);
  orc_geq(0.0, p->b0, 0.0, 0.0, gex, gey);
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      const int solid = p->nsolid > 0 && orc_is_solid(p, x, y);
      for (int q = 0; q < NQ9; ++q) state[idx(p, q, y, x)] = solid ? feq1[q] : feq[q];
      for (int q = 0; q < NQ5; ++q) {
        state[idx(p, 9 + q, y, x)] = gex[q];
        state[idx(p, 14 + q, y, x)] = gey[q];
      }
    }
}

/* One time step in -> out (distinct buffers). */
void orc_step(const orc_params *p, const double *in, double *out,
              int nthreads) {
#if defined(_OPENMP)
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
#endif
  for (int y = 0; y < p->ny; ++y) step_rows(p, in, out, y, y + 1);
  (void)nthreads;
}

/* nsteps time steps in place on `state`, using `scratch` (same size). */
void orc_run(const orc_params *p, double *state, double *scratch,
             int64_t nsteps, int nthreads) {
  const size_t n = (size_t)NPLANES * (size_t)p->nx * (size_t)p->ny;
  double *a = state, *b = scratch;
  for (int64_t s = 0; s < nsteps; ++s) {
    orc_step(p, a, b, nthreads);
    double *t = a;
    a = b;
    b = t;
  }
  if (a != state) memcpy(state, a, n * sizeof(double));
}

/* Observables of a stored state: S1-S4 without the collision, i.e. the
 * fields the next step collides with.  Any output may be NULL. */
void orc_observe(const orc_params *p, const double *state, double *rho,
                 double *ux, double *uy, double *bx, double *by, double *jz) {
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      node_t n;
      gather_node(p, state, x, y, &n);
      const size_t k = (size_t)y * p->nx + x;
      if (rho) rho[k] = n.rho;
      if (ux) ux[k] = n.ux;
      if (uy) uy[k] = n.uy;
      if (bx) bx[k] = n.bx;
      if (by) by[k] = n.by;
      if (jz) jz[k] = n.jz;
    }
}

/* Post-streaming, post-closure populations of one node (for closure tests). */
void orc_gather(const orc_params *p, const double *state, int x, int y,
                double *pops19) {
  node_t n;
  gather_node(p, state, x, y, &n);
  for (int q = 0; q < NQ9; ++q) pops19[q] = n.f[q];
  for (int q = 0; q < NQ5; ++q) {
    pops19[9 + q] = n.gx[q];
    pops19[14 + q] = n.gy[q];
  }
}

int orc_abi_version(void) { return 4; }
