/*
 * FP64 CPU oracle for the three-dimensional extension of the lattice-kinetic
 * MHD channel step (Yahia & Premnath, arXiv 2112.13930): a D3Q19 flow
 * distribution with the Lorentz force and a three-component vector magnetic
 * distribution on a D3Q7 lattice, closed at the Hartmann walls y = 0 and
 * y = ny-1 by the paper's two Shercliff schemes; x is periodic, z periodic
 * (a channel) or bounded by stationary link-closed Shercliff side walls (a
 * rectangular duct).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite and the benchmark's CPU-baseline leg
 * use it.  It shares no code, header or table with the HIP library, nor with
 * the two-dimensional oracle.
 *
 * The paper writes its schemes in two dimensions and notes (Sec. IX) that
 * both extend readily to three.  The extension taken here (its readings are
 * listed at each function) keeps every relation of Secs. IV-VII and App. A/B
 * component by component:
 *   - D3Q19 with weights 1/3, 1/18 (6 axis links) and 1/36 (12 diagonals),
 *     c_s^2 = 1/3.  Under z-invariance its populations summed over e_z are
 *     exactly D2Q9 (weights 4/9, 1/9, 1/36) with the same equilibrium.
 *   - D3Q7 for g with W_0 = 0 and W = 1/6 on the six axis links, c_sm^2 =
 *     1/3: the only D3Q7 weights whose sum over e_z gives the paper's D2Q5
 *     (W_0 = 1/3, W = 1/6).  The rest population then stays zero.
 * A z-invariant three-dimensional run therefore reproduces the
 * two-dimensional scheme exactly, which the tests check against the
 * independent two-dimensional oracle.
 *
 * State layout: post-collision populations, 40 planes, plane-major, each
 * plane [nz][ny][nx] with x fastest:
 *   planes  0..18  f_alpha           (D3Q19)
 *   planes 19..25  g_{alpha x}       (D3Q7, alpha = 0..6)
 *   planes 26..32  g_{alpha y}
 *   planes 33..39  g_{alpha z}
 * Row y = 0 is the lower wall side (y = -a), y = ny-1 the upper (y = +a).
 * Wall velocities are along x; the imposed field B0 is along +y.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NQF 19
#define NQG 7
#define NPL3 40

/* D3Q19: 0 rest; 1..4 the in-plane axis links (+x, +y, -x, -y); 5..8 the
 * in-plane diagonals (1,1), (-1,1), (-1,-1), (1,-1) -- both as in D2Q9 --;
 * 9, 10 = +z, -z; 11..14 the xz diagonals; 15..18 the yz diagonals. */
static const int E3X[NQF] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0};
static const int E3Y[NQF] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1};
static const int E3Z[NQF] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1, -1, 1};
static const double W3[NQF] = {
    1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* D3Q7: 0 rest (weight 0), then +x, +y, -x, -y (as in D2Q5), +z, -z. */
static const int G3X[NQG] = {0, 1, 0, -1, 0, 0, 0};
static const int G3Y[NQG] = {0, 0, 1, 0, -1, 0, 0};
static const int G3Z[NQG] = {0, 0, 0, 0, 0, 1, -1};
static const double WG3[NQG] = {0.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};

static const double CS2 = 1.0 / 3.0;
static const double CSM2 = 1.0 / 3.0;

enum { O3_LINK = 0, O3_MOMENT = 1 };
enum { O3_LOWER = 0, O3_UPPER = 1 };
/* Collision: BGK, or two relaxation times with tau_f on the even part of f
 * (viscosity) and tau_m on the odd part of g (magnetic diffusivity); tau_fm
 * and tau_mp are the free times of the other parts. */
enum { O3_BGK = 0, O3_TRT = 1, O3_MRT = 2 };

typedef struct {
  int32_t nx, ny, nz, bc;
  double tau_f, tau_m;
  double b0;         /* imposed field along +y */
  double fx, fy, fz; /* external body force */
  double c_lo, c_hi; /* wall conductance ratios c_w (0 .. INFINITY) */
  double u_lo, u_hi; /* wall velocities along x */
  double a;          /* half-width */
  int32_t collision, pad_;
  double tau_fm;     /* TRT: odd part of f */
  double tau_mp;     /* TRT: even part of g */
  int32_t side_walls, pad2_; /* 1: stationary Shercliff walls at z = -1/2 and nz - 1/2 */
  double cs_lo, cs_hi;       /* their wall conductance ratios (0 .. INFINITY) */
  double s_fe, s_feps, s_fq; /* MRT rates of f's e, epsilon (and pi), q (and m) moments */
  double s_md;               /* MRT rate of g's two traceless second moments */
} orc3_params;

static int opp3(int q) {
  for (int r = 0; r < NQF; ++r)
    if (E3X[r] == -E3X[q] && E3Y[r] == -E3Y[q] && E3Z[r] == -E3Z[q]) return r;
  return -1;
}

static int oppg(int q) {
  for (int r = 0; r < NQG; ++r)
    if (G3X[r] == -G3X[q] && G3Y[r] == -G3Y[q] && G3Z[r] == -G3Z[q]) return r;
  return -1;
}

/* f^eq: w rho [1 + e.u/cs2 + (e.u)^2/(2 cs2^2) - u.u/(2 cs2)] (Sec. V). */
void orc3_feq(double rho, const double *u, double *feq) {
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int q = 0; q < NQF; ++q) {
    const double eu = E3X[q] * u[0] + E3Y[q] * u[1] + E3Z[q] * u[2];
    feq[q] = W3[q] * rho * (1.0 + eu / CS2 + (eu * eu) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
  }
}

/* g^eq_{alpha i} = W_alpha { B_i + e_{alpha j} (u_j B_i - B_j u_i) / cs2m }
 * (Sec. IV), j summed over the three axes; geq[alpha*3 + i]. */
void orc3_geq(const double *b, const double *u, double *geq) {
  for (int q = 0; q < NQG; ++q) {
    const int e[3] = {G3X[q], G3Y[q], G3Z[q]};
    for (int i = 0; i < 3; ++i) {
      double flux = 0.0;
      for (int j = 0; j < 3; ++j) flux += e[j] * (u[j] * b[i] - b[j] * u[i]);
      geq[q * 3 + i] = WG3[q] * (b[i] + flux / CSM2);
    }
  }
}

/* S_alpha = (e_alpha - u).F f^eq_alpha / (rho cs2) (Sec. V). */
void orc3_source(double rho, const double *u, const double *F, const double *feq, double *S) {
  for (int q = 0; q < NQF; ++q) {
    const double dot = (E3X[q] - u[0]) * F[0] + (E3Y[q] - u[1]) * F[1] + (E3Z[q] - u[2]) * F[2];
    S[q] = dot * feq[q] / (rho * CS2);
  }
}

/*
 * Coupled local solve for u and J (the three-dimensional form of the
 * two-dimensional reading): rho u = m + F/2 with F = F_ext + J x B (Secs. II,
 * V), and each component of J = curl B from the antisymmetric
 * non-equilibrium part of Lambda (Sec. IV):
 *   J_x = -k [(L_yz - L0_yz) - (L_zy - L0_zy)]
 *   J_y = -k [(L_zx - L0_zx) - (L_xz - L0_xz)]
 *   J_z = -k [(L_xy - L0_xy) - (L_yx - L0_yx)],   L0_ji = u_j B_i - B_j u_i,
 * k = 1/(tau_m cs2m).  Six linear equations in (u_x, u_y, u_z, J_x, J_y, J_z),
 * solved by Gaussian elimination with partial pivoting.  lam[j*3+i] =
 * Lambda_ji = sum_alpha e_{alpha j} g_{alpha i}.
 */
void orc3_local_solve(double rho, const double *m, const double *b, const double *lam,
                      double tau_m, const double *fext, double *out /* u[3], J[3] */) {
  const double k = 1.0 / (tau_m * CSM2);
  const double bx = b[0], by = b[1], bz = b[2];
  /* D_k = Lambda_ij - Lambda_ji for (i, j, k) cyclic */
  const double dyz = lam[1 * 3 + 2] - lam[2 * 3 + 1];
  const double dzx = lam[2 * 3 + 0] - lam[0 * 3 + 2];
  const double dxy = lam[0 * 3 + 1] - lam[1 * 3 + 0];
  double M[6][7] = {
      /* rho u - (J x B)/2 = m + F_ext/2 */
      {rho, 0, 0, 0, -bz / 2.0, by / 2.0, m[0] + fext[0] / 2.0},
      {0, rho, 0, bz / 2.0, 0, -bx / 2.0, m[1] + fext[1] / 2.0},
      {0, 0, rho, -by / 2.0, bx / 2.0, 0, m[2] + fext[2] / 2.0},
      /* J - 2k (u x B) = -k D */
      {0, -2.0 * k * bz, 2.0 * k * by, 1, 0, 0, -k * dyz},
      {2.0 * k * bz, 0, -2.0 * k * bx, 0, 1, 0, -k * dzx},
      {-2.0 * k * by, 2.0 * k * bx, 0, 0, 0, 1, -k * dxy},
  };
  for (int c = 0; c < 6; ++c) {
    int piv = c;
    for (int r = c + 1; r < 6; ++r)
      if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
    if (piv != c)
      for (int j = 0; j < 7; ++j) {
        const double t = M[c][j];
        M[c][j] = M[piv][j];
        M[piv][j] = t;
      }
    for (int r = c + 1; r < 6; ++r) {
      const double fac = M[r][c] / M[c][c];
      for (int j = c; j < 7; ++j) M[r][j] -= fac * M[c][j];
    }
  }
  for (int r = 5; r >= 0; --r) {
    double s = M[r][6];
    for (int j = r + 1; j < 6; ++j) s -= M[r][j] * out[j];
    out[r] = s / M[r][r];
  }
}

/*
 * Link-based closures at a wall (Sec. VI, App. B.1), applied per link:
 *   f: half-way bounce-back with Ladd's term 2 w e_x U_w / cs2 for every
 *      incoming link (the five with e_y pointing into the fluid);
 *   g, tangential components i = x, z: the theta-weighted Shercliff closure
 *      g_in = ((theta-1)/(theta+1)) g~_out - (2 theta/(theta+1)) W (e_y/cs2m)
 *      B0 U_w delta_ix (the wall moves along x, so only B_x carries the
 *      moving-wall term); theta = c_w a / (tau_m - 1/2); c_w = INFINITY
 *      takes the perfectly conducting limit;
 *   g, normal component: anti-bounce-back to B_y = B0, g_in = -g~_out + 2 W B0.
 * own: the node's post-collision populations of the previous step (40).
 */
void orc3_link_closure(const orc3_params *p, int wall, const double *own, double *f, double *g) {
  const int ey_in = (wall == O3_LOWER) ? +1 : -1;
  const double cw = (wall == O3_LOWER) ? p->c_lo : p->c_hi;
  const double uw = (wall == O3_LOWER) ? p->u_lo : p->u_hi;
  for (int q = 0; q < NQF; ++q) {
    if (E3Y[q] != ey_in) continue;
    f[q] = own[opp3(q)] + 2.0 * W3[q] * E3X[q] * uw / CS2;
  }
  for (int q = 0; q < NQG; ++q) {
    if (G3Y[q] != ey_in) continue;
    const int o = oppg(q);
    for (int i = 0; i < 3; ++i) {
      const double gbar = own[19 + i * 7 + o];
      if (i == 1) {
        g[q * 3 + i] = -gbar + 2.0 * WG3[q] * p->b0;
        continue;
      }
      const double moving = (i == 0) ? WG3[q] * (G3Y[q] / CSM2) * p->b0 * uw : 0.0;
      if (isinf(cw)) {
        g[q * 3 + i] = gbar - 2.0 * moving;
      } else {
        const double theta = cw * p->a / (p->tau_m - 0.5);
        g[q * 3 + i] = ((theta - 1.0) / (theta + 1.0)) * gbar - (2.0 * theta / (theta + 1.0)) * moving;
      }
    }
  }
}

/*
 * Side walls of a duct (link-based only), stationary, half-way between the
 * layers z = 0 and z = -1 (lower) or nz-1 and nz (upper), applied to every
 * link whose source lies behind the wall:
 *   f: half-way bounce-back;
 *   g, tangential components x and y: the theta-weighted Shercliff closure of
 *      Sec. VI on the induced field b = B - (0, B0, 0), i.e.
 *        g_in,x = r g~_out,x,   g_in,y - W B0 = r (g~_out,y - W B0),
 *      r = (theta-1)/(theta+1), theta = c_s a / (tau_m - 1/2) (the same
 *      length a as at the Hartmann walls); c_s = INFINITY gives r = 1;
 *   g, normal component z: anti-bounce-back to B_z = 0, g_in,z = -g~_out,z.
 * A link crossing a Hartmann wall and a side wall at an edge is closed by
 * both; for f the results coincide (bounce-back, no moving-wall term since
 * such links have e_x = 0).
 */
void orc3_side_closure(const orc3_params *p, int wall, const double *own, double *f, double *g) {
  const int ez_in = (wall == O3_LOWER) ? +1 : -1;
  const double cw = (wall == O3_LOWER) ? p->cs_lo : p->cs_hi;
  const double r = isinf(cw) ? 1.0 : (cw * p->a / (p->tau_m - 0.5) - 1.0) /
                                         (cw * p->a / (p->tau_m - 0.5) + 1.0);
  for (int q = 0; q < NQF; ++q)
    if (E3Z[q] == ez_in) f[q] = own[opp3(q)];
  for (int q = 0; q < NQG; ++q) {
    if (G3Z[q] != ez_in) continue;
    const int o = oppg(q);
    const double wb0 = WG3[q] * p->b0;
    g[q * 3 + 0] = r * own[19 + 0 * 7 + o];
    g[q * 3 + 1] = r * (own[19 + 1 * 7 + o] - wb0) + wb0;
    g[q * 3 + 2] = -own[19 + 2 * 7 + o];
  }
}

/*
 * On-node moment-based closures (Sec. VII, App. A, App. B.2) extended to the
 * five unknown D3Q19 populations of a wall node (e_y into the fluid).  The
 * paper's constraint set is taken per tangential direction: with rho from
 * the normal-momentum constraint Pi_y = 0,
 *   Pi_x = rho U_w,  Pi_xx = rho (cs2 + U_w^2),  Pi_z = 0,  Pi_zz = rho cs2,
 * each pair fixing the two unknowns that carry e_x (resp. e_z), and the
 * normal unknown closing Pi_y.  Under z-invariance this reduces to the
 * paper's closure (Pi_10, Pi_01, Pi_20) for the e_z-summed populations.
 * g: tangential components x and z from the discrete Shercliff constraint
 *   +-A (Lambda_yi + B0 U_w delta_ix) + C B_i = 0 (A = 1/(tau_m cs2m),
 * C = 1/(c_w a)), limits c_w = 0 and INFINITY as printed; normal component
 * from sum_alpha g_{alpha y} = B0.
 * f, g: post-streaming populations of the node; unknowns overwritten.
 */
void orc3_moment_closure(const orc3_params *p, int wall, double *f, double *g) {
  const double cw = (wall == O3_LOWER) ? p->c_lo : p->c_hi;
  const double U = (wall == O3_LOWER) ? p->u_lo : p->u_hi;
  const int ey_in = (wall == O3_LOWER) ? +1 : -1;
  /* known sums */
  double k0 = 0.0, kout = 0.0, px = 0.0, pxx = 0.0, pz = 0.0, pzz = 0.0;
  for (int q = 0; q < NQF; ++q) {
    if (E3Y[q] == ey_in) continue; /* unknown */
    if (E3Y[q] == 0) k0 += f[q];
    else kout += f[q];
    px += E3X[q] * f[q];
    pxx += E3X[q] * E3X[q] * f[q];
    pz += E3Z[q] * f[q];
    pzz += E3Z[q] * E3Z[q] * f[q];
  }
  /* Pi_y = 0: the unknowns carry as much normal momentum as the knowns */
  const double rho = k0 + 2.0 * kout;
  /* unknowns: the normal link, the two with e_x = +-1, the two with e_z = +-1 */
  int qn = -1, qxp = -1, qxm = -1, qzp = -1, qzm = -1;
  for (int q = 0; q < NQF; ++q) {
    if (E3Y[q] != ey_in) continue;
    if (E3X[q] == 0 && E3Z[q] == 0) qn = q;
    if (E3X[q] == 1) qxp = q;
    if (E3X[q] == -1) qxm = q;
    if (E3Z[q] == 1) qzp = q;
    if (E3Z[q] == -1) qzm = q;
  }
  const double sx = rho * U - px;                /* f_xp - f_xm */
  const double sxx = rho * (CS2 + U * U) - pxx;  /* f_xp + f_xm */
  const double sz = -pz;                         /* f_zp - f_zm */
  const double szz = rho * CS2 - pzz;            /* f_zp + f_zm */
  f[qxp] = 0.5 * (sxx + sx);
  f[qxm] = 0.5 * (sxx - sx);
  f[qzp] = 0.5 * (szz + sz);
  f[qzm] = 0.5 * (szz - sz);
  f[qn] = kout - (f[qxp] + f[qxm] + f[qzp] + f[qzm]);

  /* g: the unknown link is the one with e_y into the fluid */
  int gin = -1;
  for (int q = 0; q < NQG; ++q)
    if (G3Y[q] == ey_in) gin = q;
  const int gout = oppg(gin);
  const double A = 1.0 / (p->tau_m * CSM2);
  for (int i = 0; i < 3; ++i) {
    double others = 0.0; /* every population of component i but the two y links */
    for (int q = 0; q < NQG; ++q)
      if (q != gin && q != gout) others += g[q * 3 + i];
    if (i == 1) {
      g[gin * 3 + 1] = p->b0 - (others + g[gout * 3 + 1]);
      continue;
    }
    /* lower: A (g_in - g_out + B0 U) + C (others + g_in + g_out) = 0
     * upper: -A (g_out - g_in + B0 U) + C (...) = 0, i.e. the same with U -> -U
     * (Lambda_yi = g_2i - g_4i; at the upper wall g_in = g_4i). */
    const double bu = (i == 0) ? p->b0 * U : 0.0;
    const double s = (wall == O3_LOWER) ? bu : -bu;
    if (cw == 0.0) {
      g[gin * 3 + i] = -(others + g[gout * 3 + i]);
    } else if (isinf(cw)) {
      g[gin * 3 + i] = g[gout * 3 + i] - s;
    } else {
      const double C = 1.0 / (cw * p->a);
      g[gin * 3 + i] = ((A - C) * g[gout * 3 + i] - C * others - A * s) / (A + C);
    }
  }
}

static inline size_t idx3(const orc3_params *p, int plane, int z, int y, int x) {
  return (((size_t)plane * (size_t)p->nz + (size_t)z) * (size_t)p->ny + (size_t)y) * (size_t)p->nx +
         (size_t)x;
}

typedef struct {
  double f[NQF], g[NQG * 3];
  double rho, u[3], b[3], j[3], F[3];
} node3_t;

static int wrap(int v, int n) { return ((v % n) + n) % n; }

/* source layer of a pull along e_z: periodic, or -1 behind a side wall */
static int src_z(const orc3_params *p, int z, int ez) {
  const int sz = z - ez;
  if (p->side_walls) return (sz >= 0 && sz < p->nz) ? sz : -1;
  return wrap(sz, p->nz);
}

static void gather3(const orc3_params *p, const double *in, int x, int y, int z, node3_t *n) {
  /* pull streaming; x periodic, z periodic or bounded by side walls */
  for (int q = 0; q < NQF; ++q) {
    const int sy = y - E3Y[q], sz = src_z(p, z, E3Z[q]);
    n->f[q] = (sy >= 0 && sy < p->ny && sz >= 0)
                  ? in[idx3(p, q, sz, sy, wrap(x - E3X[q], p->nx))]
                  : NAN;
  }
  for (int q = 0; q < NQG; ++q) {
    const int sy = y - G3Y[q], sz = src_z(p, z, G3Z[q]);
    for (int i = 0; i < 3; ++i)
      n->g[q * 3 + i] = (sy >= 0 && sy < p->ny && sz >= 0)
                            ? in[idx3(p, 19 + i * 7 + q, sz, sy, wrap(x - G3X[q], p->nx))]
                            : NAN;
  }
  const int wall = (y == 0) || (y == p->ny - 1);
  const int side = p->side_walls && ((z == 0) || (z == p->nz - 1));
  if (wall || side) {
    double own[NPL3];
    for (int k = 0; k < NPL3; ++k) own[k] = in[idx3(p, k, z, y, x)];
    for (int w = 0; w < 2 && wall; ++w) {
      const int at = (w == O3_LOWER) ? (y == 0) : (y == p->ny - 1);
      if (!at) continue;
      if (p->bc == O3_LINK) orc3_link_closure(p, w, own, n->f, n->g);
      else orc3_moment_closure(p, w, n->f, n->g);
    }
    for (int w = 0; w < 2 && side; ++w) {
      const int at = (w == O3_LOWER) ? (z == 0) : (z == p->nz - 1);
      if (at) orc3_side_closure(p, w, own, n->f, n->g);
    }
  }
  double rho = 0.0, m[3] = {0, 0, 0}, b[3] = {0, 0, 0}, lam[9] = {0};
  for (int q = 0; q < NQF; ++q) {
    rho += n->f[q];
    m[0] += E3X[q] * n->f[q];
    m[1] += E3Y[q] * n->f[q];
    m[2] += E3Z[q] * n->f[q];
  }
  for (int q = 0; q < NQG; ++q) {
    const int e[3] = {G3X[q], G3Y[q], G3Z[q]};
    for (int i = 0; i < 3; ++i) {
      b[i] += n->g[q * 3 + i];
      for (int jj = 0; jj < 3; ++jj) lam[jj * 3 + i] += e[jj] * n->g[q * 3 + i];
    }
  }
  n->rho = rho;
  for (int i = 0; i < 3; ++i) n->b[i] = b[i];
  if (wall && p->bc == O3_MOMENT) {
    /* wet wall node: Dirichlet velocity from the closure, no force; J from
     * the non-equilibrium Lambda with that velocity (as in two dimensions) */
    const double k = 1.0 / (p->tau_m * CSM2);
    for (int i = 0; i < 3; ++i) n->u[i] = m[i] / rho;
    const double *u = n->u;
    const double uxb[3] = {u[1] * b[2] - u[2] * b[1], u[2] * b[0] - u[0] * b[2],
                           u[0] * b[1] - u[1] * b[0]};
    n->j[0] = -k * ((lam[1 * 3 + 2] - lam[2 * 3 + 1]) - 2.0 * uxb[0]);
    n->j[1] = -k * ((lam[2 * 3 + 0] - lam[0 * 3 + 2]) - 2.0 * uxb[1]);
    n->j[2] = -k * ((lam[0 * 3 + 1] - lam[1 * 3 + 0]) - 2.0 * uxb[2]);
    n->F[0] = n->F[1] = n->F[2] = 0.0;
    return;
  }
  const double fext[3] = {p->fx, p->fy, p->fz};
  double sol[6];
  orc3_local_solve(rho, m, b, lam, p->tau_m, fext, sol);
  for (int i = 0; i < 3; ++i) {
    n->u[i] = sol[i];
    n->j[i] = sol[3 + i];
  }
  const double *J = n->j;
  n->F[0] = p->fx + (J[1] * b[2] - J[2] * b[1]);
  n->F[1] = p->fy + (J[2] * b[0] - J[0] * b[2]);
  n->F[2] = p->fz + (J[0] * b[1] - J[1] * b[0]);
}

/* Collision of one node: f[19] and g[7*3] (g[q*3+i]) post-streaming and
 * post-closure, with the fields of the solve; out receives the 40 planes
 * (f, then g per component).  BGK as in Sec. V; TRT relaxes the parts even
 * and odd under e -> -e at their own rates, the source's parts with the
 * matching weights 1 - 1/(2 tau); MRT relaxes the moments of the bases above
 * at their own rates. */
/* MRT rows.  f (D3Q19, d'Humieres, Ginzburg, Krafczyk, Lallemand and Luo,
 * Phil. Trans. R. Soc. A 360 (2002) 437), as functions of e: rho = 1,
 * e = 19|e|^2 - 30, epsilon = (21|e|^4 - 53|e|^2 + 24)/2, j_i = e_i,
 * q_i = (5|e|^2 - 9) e_i, 3p_xx = 3e_x^2 - |e|^2, 3pi_xx = (3|e|^2 - 5)(3e_x^2 -
 * |e|^2), p_ww = e_y^2 - e_z^2, pi_ww = (3|e|^2 - 5)(e_y^2 - e_z^2), p_xy =
 * e_x e_y, p_yz, p_xz, m_x = (e_y^2 - e_z^2) e_x, m_y = (e_z^2 - e_x^2) e_y,
 * m_z = (e_x^2 - e_y^2) e_z.  Rates: the five stresses at 1/tau_f; e at
 * s_fe; epsilon and the fourth-order pi at s_feps; q and the third-order m
 * at s_fq; rho and j (which do not matter) at 1/tau_f and s_fq.
 * g (D3Q7 per component): B = 1, Lambda_i = e_i, epsilon = 7|e|^2 - 6 (over
 * rest and axis links), and the traceless 2e_x^2 - e_y^2 - e_z^2 and
 * e_y^2 - e_z^2; Lambda at 1/tau_m, the traceless pair at s_md, B and
 * epsilon at s_md too (the rest weight is zero, so epsilon has no
 * non-equilibrium part). */
static void mrt3_rows(double M[NQF][NQF], double s[NQF], const orc3_params *p) {
  const double snu = 1.0 / p->tau_f;
  for (int a = 0; a < NQF; ++a) {
    const double ex = E3X[a], ey = E3Y[a], ez = E3Z[a];
    const double e2 = ex * ex + ey * ey + ez * ez;
    const double r[NQF] = {1.0,
                           19.0 * e2 - 30.0,
                           (21.0 * e2 * e2 - 53.0 * e2 + 24.0) / 2.0,
                           ex, (5.0 * e2 - 9.0) * ex,
                           ey, (5.0 * e2 - 9.0) * ey,
                           ez, (5.0 * e2 - 9.0) * ez,
                           3.0 * ex * ex - e2, (3.0 * e2 - 5.0) * (3.0 * ex * ex - e2),
                           ey * ey - ez * ez, (3.0 * e2 - 5.0) * (ey * ey - ez * ez),
                           ex * ey, ey * ez, ex * ez,
                           (ey * ey - ez * ez) * ex, (ez * ez - ex * ex) * ey,
                           (ex * ex - ey * ey) * ez};
    for (int k = 0; k < NQF; ++k) M[k][a] = r[k];
  }
  const double rates[NQF] = {snu, p->s_fe, p->s_feps, p->s_fq, p->s_fq, p->s_fq, p->s_fq,
                             p->s_fq, p->s_fq, snu, p->s_feps, snu, p->s_feps, snu, snu, snu,
                             p->s_fq, p->s_fq, p->s_fq};
  for (int k = 0; k < NQF; ++k) s[k] = rates[k];
}

static void mrt3g_rows(double M[NQG][NQG], double s[NQG], const orc3_params *p) {
  for (int a = 0; a < NQG; ++a) {
    const double ex = G3X[a], ey = G3Y[a], ez = G3Z[a];
    const double e2 = ex * ex + ey * ey + ez * ez;
    const double r[NQG] = {1.0, ex, ey, ez, 7.0 * e2 - 6.0, 2.0 * ex * ex - ey * ey - ez * ez,
                           ey * ey - ez * ez};
    for (int k = 0; k < NQG; ++k) M[k][a] = r[k];
  }
  const double sl = 1.0 / p->tau_m;
  const double rates[NQG] = {p->s_md, sl, sl, sl, p->s_md, p->s_md, p->s_md};
  for (int k = 0; k < NQG; ++k) s[k] = rates[k];
}

/* One MRT update of n populations h (stride hs) with basis rows M (n x n,
 * row-major): the non-equilibrium part of moment k relaxes at s[k], the
 * source's moment k (src may be NULL) enters with 1 - s[k]/2, and the
 * moments map back through M^T diag(1/|row|^2) (the rows are orthogonal). */
static void mrt3_update(int n, const double *M, const double *s, const double *h, int hs,
                        const double *heq, const double *src, double *out, int os) {
  double c[NQF];
  for (int k = 0; k < n; ++k) {
    double neq = 0.0, ms = 0.0, norm = 0.0;
    for (int a = 0; a < n; ++a) {
      neq += M[k * n + a] * (h[a * hs] - heq[a * hs]);
      if (src) ms += M[k * n + a] * src[a];
      norm += M[k * n + a] * M[k * n + a];
    }
    c[k] = (-s[k] * neq + (1.0 - 0.5 * s[k]) * ms) / norm;
  }
  for (int a = 0; a < n; ++a) {
    double d = 0.0;
    for (int k = 0; k < n; ++k) d += M[k * n + a] * c[k];
    out[a * os] = h[a * hs] + d;
  }
}

void orc3_collide(const orc3_params *p, const double *f, const double *g, double rho,
                  const double *u, const double *b, const double *F, double *out) {
  double feq[NQF], S[NQF], geq[NQG * 3];
  orc3_feq(rho, u, feq);
  orc3_source(rho, u, F, feq, S);
  orc3_geq(b, u, geq);
  if (p->collision == O3_MRT) {
    double M[NQF][NQF], sf[NQF], Mg[NQG][NQG], sg[NQG];
    mrt3_rows(M, sf, p);
    mrt3_update(NQF, &M[0][0], sf, f, 1, feq, S, out, 1);
    mrt3g_rows(Mg, sg, p);
    for (int i = 0; i < 3; ++i)
      mrt3_update(NQG, &Mg[0][0], sg, g + i, 3, geq + i, NULL, out + 19 + i * 7, 1);
    return;
  }
  if (p->collision != O3_TRT) {
    for (int q = 0; q < NQF; ++q)
      out[q] = f[q] - (f[q] - feq[q]) / p->tau_f + (1.0 - 1.0 / (2.0 * p->tau_f)) * S[q];
    for (int q = 0; q < NQG; ++q)
      for (int i = 0; i < 3; ++i)
        out[19 + i * 7 + q] = g[q * 3 + i] - (g[q * 3 + i] - geq[q * 3 + i]) / p->tau_m;
    return;
  }
  const double tfe = p->tau_f, tfo = p->tau_fm;
  for (int q = 0; q < NQF; ++q) {
    const int r = opp3(q);
    const double fe = 0.5 * (f[q] + f[r]), fo = 0.5 * (f[q] - f[r]);
    const double ee = 0.5 * (feq[q] + feq[r]), eo = 0.5 * (feq[q] - feq[r]);
    const double se = 0.5 * (S[q] + S[r]), so = 0.5 * (S[q] - S[r]);
    out[q] = f[q] - (fe - ee) / tfe - (fo - eo) / tfo + (1.0 - 1.0 / (2.0 * tfe)) * se +
             (1.0 - 1.0 / (2.0 * tfo)) * so;
  }
  const double tme = p->tau_mp, tmo = p->tau_m;
  for (int q = 0; q < NQG; ++q) {
    const int r = oppg(q);
    for (int i = 0; i < 3; ++i) {
      const double he = 0.5 * (g[q * 3 + i] + g[r * 3 + i]);
      const double ho = 0.5 * (g[q * 3 + i] - g[r * 3 + i]);
      const double ee = 0.5 * (geq[q * 3 + i] + geq[r * 3 + i]);
      const double eo = 0.5 * (geq[q * 3 + i] - geq[r * 3 + i]);
      out[19 + i * 7 + q] = g[q * 3 + i] - (he - ee) / tme - (ho - eo) / tmo;
    }
  }
}

static void step_line(const orc3_params *p, const double *in, double *out, int z, int y) {
  for (int x = 0; x < p->nx; ++x) {
    node3_t n;
    gather3(p, in, x, y, z, &n);
    double o[NPL3];
    orc3_collide(p, n.f, n.g, n.rho, n.u, n.b, n.F, o);
    for (int q = 0; q < NPL3; ++q) out[idx3(p, q, z, y, x)] = o[q];
  }
}

void orc3_init(const orc3_params *p, double rho0, double *state) {
  double feq[NQF], geq[NQG * 3];
  const double u0[3] = {0, 0, 0}, b0[3] = {0, p->b0, 0};
  orc3_feq(rho0, u0, feq);
  orc3_geq(b0, u0, geq);
  for (int z = 0; z < p->nz; ++z)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        for (int q = 0; q < NQF; ++q) state[idx3(p, q, z, y, x)] = feq[q];
        for (int q = 0; q < NQG; ++q)
          for (int i = 0; i < 3; ++i) state[idx3(p, 19 + i * 7 + q, z, y, x)] = geq[q * 3 + i];
      }
}

void orc3_step(const orc3_params *p, const double *in, double *out, int nthreads) {
  const int lines = p->nz * p->ny;
#if defined(_OPENMP)
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
#endif
  for (int l = 0; l < lines; ++l) step_line(p, in, out, l / p->ny, l % p->ny);
  (void)nthreads;
}

void orc3_run(const orc3_params *p, double *state, double *scratch, int64_t nsteps, int nthreads) {
  const size_t n = (size_t)NPL3 * (size_t)p->nx * (size_t)p->ny * (size_t)p->nz;
  double *a = state, *b = scratch;
  for (int64_t s = 0; s < nsteps; ++s) {
    orc3_step(p, a, b, nthreads);
    double *t = a;
    a = b;
    b = t;
  }
  if (a != state) memcpy(state, a, n * sizeof(double));
}

/* Observables of the state (streaming, closure, moments and solve, no
 * collision): rho, u[3], B[3], J[3] per node; out[k * N + node], k = 0..9. */
void orc3_observe(const orc3_params *p, const double *state, double *out) {
  const size_t N = (size_t)p->nx * p->ny * p->nz;
  for (int z = 0; z < p->nz; ++z)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        node3_t n;
        gather3(p, state, x, y, z, &n);
        const size_t i = ((size_t)z * p->ny + y) * p->nx + x;
        const double v[10] = {n.rho, n.u[0], n.u[1], n.u[2], n.b[0], n.b[1], n.b[2], n.j[0], n.j[1], n.j[2]};
        for (int k = 0; k < 10; ++k) out[k * N + i] = v[k];
      }
}

/* Post-closure populations of one node (40 values), for closure tests. */
void orc3_gather(const orc3_params *p, const double *state, int x, int y, int z, double *out) {
  node3_t n;
  gather3(p, state, x, y, z, &n);
  for (int q = 0; q < NQF; ++q) out[q] = n.f[q];
  for (int q = 0; q < NQG; ++q)
    for (int i = 0; i < 3; ++i) out[19 + i * 7 + q] = n.g[q * 3 + i];
}
