// Per-node fused update of the lattice-kinetic MHD step for gfx950.
//
// One call updates one lattice node: pull the 19 post-collision populations
// of the previous step from the node's neighbours (structure-of-arrays
// planes, x contiguous), close the populations that would come from behind a
// wall (link-based or on-node moment-based Shercliff closures), take the
// moments, solve the local u <-> J_z coupling in closed form, collide f and g
// (BGK) and store the 19 new populations.  Every stored value of the previous
// step is read exactly once per step, so the step streams 19 reads and 19
// writes per node through HBM.
//
// Storage: S is the stored type (double, float or _Float16), C the compute
// type.  Every population is stored as its deviation from the rest state at
// unit density and B = (0, B0) -- f_alpha - w_alpha, g_alpha,x and
// g_alpha,y - W_alpha B0.  Binary16 storage further subtracts a per-row
// reference D[y][plane] kept in the compute type (zero until a rebase moves
// each row's x-mean into it) and scales by 2^12, so the stored values carry
// only what the flow, the induced field and their x-variation put into
// them.  A pulled value is decoded with the reference of the row it comes
// from; a stored value is encoded with its own row's.
//
// Method references (Yahia & Premnath, arXiv 2112.13930):
//   equilibria, source, moments: Secs. IV, V;  J_z: Sec. IV;  F = J x B: Sec. II
//   link-based closures: Sec. VI (Eq. linkbasedBCschemefinal), App. B.1
//   moment-based closures: Sec. VII, App. A, App. B.2
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lks_sr.hpp"

// Arithmetic of the reduced-precision modes (compile-time; the defaults are
// the product configuration):
//   LKS_FP32_COMPUTE_DOUBLE  FP32-stored populations are computed in FP64.
//                            The step is HBM-bound, so this costs no time,
//                            and FP32 arithmetic leaves a rounding residual
//                            that slow modes of a steady channel amplify.
//   LKS_SR_FP32, LKS_SR_FP16 stored values are rounded stochastically (needs a
//                            compute type wider than the storage type).
#ifndef LKS_FP32_COMPUTE_DOUBLE
#define LKS_FP32_COMPUTE_DOUBLE 1
#endif
#ifndef LKS_SR_FP32
#define LKS_SR_FP32 1
#endif
#ifndef LKS_SR_FP16
#define LKS_SR_FP16 1
#endif

namespace lks {

enum { BC_LINK = 0, BC_MOMENT = 1 };
// The kernels' scheme parameter is the wall scheme, optionally combined with
// COLL_TRT for the two-relaxation-time collision (BGK otherwise).
constexpr int COLL_TRT = 4;
// ... and with WALLS_X for an enclosure (link-closed walls bounding x)
constexpr int WALLS_X = 8;
// ... and with WALLS_Q for link-based Hartmann walls at a cut distance
// q != 1/2 from their wall rows
constexpr int WALLS_Q = 16;
// ... and with IN_BATCH inside the batched kernel: its rows follow each
// other without padding, so cache lines straddle rows, and it inlines every
// scheme, so code length and divergent branches cost more than elsewhere
constexpr int IN_BATCH = 32;
// ... and with COLL_MRT for the multiple-relaxation-time collision
constexpr int COLL_MRT = 64;
// ... and, with COLL_TRT, MRT_RT where the MRT corrections are applied when
// the coefficients ask for them (Coef::mrt_on): the batched kernel runs TRT
// and MRT channels through one inlined scheme
constexpr int MRT_RT = 128;
constexpr int wall_of(int scheme) { return scheme & 3; }
constexpr bool trt_of(int scheme) { return (scheme & COLL_TRT) != 0; }
constexpr bool xwalls_of(int scheme) { return (scheme & WALLS_X) != 0; }
constexpr bool cut_of(int scheme) { return (scheme & WALLS_Q) != 0; }
constexpr bool in_batch(int scheme) { return (scheme & IN_BATCH) != 0; }
constexpr bool mrt_of(int scheme) { return (scheme & COLL_MRT) != 0; }
constexpr bool mrt_rt_of(int scheme) { return (scheme & MRT_RT) != 0; }
enum { MODE_STEP = 0, MODE_RECORD = 1, MODE_RESIDUAL = 2, MODE_MOMENTS = 3 };

// Closure coefficients of one wall (computed on the host in FP64).
//   link:   g_in,x = r * g~_out,x + t                 (Eq. movingwalllinkbasedclosure)
//           r = (theta-1)/(theta+1), t = -/+ theta/(theta+1) B0 U_w (lower/upper)
//   moment: g_in,x = r * g_opp,x - s * (g_0x+g_1x+g_3x) + t
//           r = (phi-1)/(phi+1), s = 1/(phi+1), t = -/+ phi/(phi+1) B0 U_w,
//           phi = c_w a / (tau_m cs2m)   (Sec. VII, App. B.2, both limits exact)
//   uw6 = U_w/6 is Ladd's moving-wall term 2 w e_x U_w / cs2 of the diagonals.
template <typename C>
struct Wall {
  C r, s, t, u, uw6;
};

// Two-relaxation-time coefficients.  With n = f^eq - f, the update of a
// population whose opposite is abar (e_abar = -e_a),
//   f~_a = f_a + pa n_a + pb n_abar + sa S_a + sb S_abar,
// relaxes the even part (f_a + f_abar)/2 at w+ and the odd part at w-, and
// adds the even and odd parts of the source with 1 - w+/2 and 1 - w-/2:
//   pa = (w+ + w-)/2, pb = (w+ - w-)/2, sa = 1 - pa/2, sb = -pb/2.
// f: w+ = 1/tau_f (viscosity), w- from the magic parameter Lambda_f;
// g: w- = 1/tau_m (magnetic diffusivity), w+ = gp from Lambda_m; g has no
// source.  Rest populations are even: f at omega_f/kappa_f, g at gp.
template <typename C>
struct Trt {
  C fa, fb, fsa, fsb;
  C ga, gb, gp;
};

// Multiple-relaxation-time coefficients (host FP64).  MRT differs from the
// TRT step whose even rates are 1/tau_f (f) and s_me (g) and whose odd
// rates are s_fq (f) and 1/tau_m (g) only in the rates of f's moments e and
// epsilon and of g's moment d; with M_k the basis row, n = feq - f and S the
// source, the difference is
//   f: M_k (s_k - 1/tau_f) (M_k.n - M_k.S / 2) / |M_k|^2   for k = e, epsilon,
//   g: M_d (s_md - s_me) M_d.n / |M_d|^2,
// rows e = (-4, -1 x4, 2 x4), epsilon = (4, -2 x4, 1 x4) over rest, axis and
// diagonal populations, and d = (0, 1, -1, 1, -1) over D2Q5.
// In three dimensions (D3Q19, d'Humieres et al. 2002) the corrected even
// rows are e = 19|e|^2 - 30 (s_fe), epsilon = (21|e|^4 - 53|e|^2 + 24)/2,
// 3pi_xx = (3|e|^2 - 5)(3e_x^2 - |e|^2) and pi_ww = (3|e|^2 - 5)(e_y^2 - e_z^2)
// (all at s_feps), with |M|^2 = 2394, 252, 72, 24; the odd rows q and m keep
// TRT's odd rate, and g (D3Q7, zero rest weight) is the TRT step with even
// rate s_md.
template <typename C>
struct Mrt {
  C ke, keps; // (s - 1/tau_f) / 36
  C kd;       // (s_md - s_me) / 4
  C ke3, keps3, kpx3, kpw3; // (s - 1/tau_f) / |M|^2, three dimensions
};

// A link-based Hartmann wall at a cut distance q (0 < q <= 1) from its
// wall row (host FP64 coefficients).  With o the outgoing post-collision
// population at the wall row and X the same direction's population at the
// next node into the fluid (near, q < 1/2) or the wall row's own incoming
// post-collision population (q >= 1/2):
//   f:   f_in = fa o + fb X + lscale * (moving-wall term), then the mass the
//        wall would let through returns to the incoming populations
//        (weights 4/6, 1/6, 1/6);
//   g with wall value zero (normal component; tangential at c = 0):
//        g_in = za o + zb X   (stored deviations);
//   g_x at a conducting wall: g_in = r o0 + kappa (o2 - 2 o1 + o0) + tmove
//        + tshear (u - U), with o1, o2 one and two nodes further in and u
//        the wall row's velocity from its post-collision momentum.
template <typename C>
struct Cut {
  int near, conducting;
  C fa, fb, lscale, za, zb, r, kappa, tmove, tshear, u;
};

template <typename C>
struct Coef {
  C omega_f;  // 1/tau_f
  C kappa_f;  // 1 - 1/(2 tau_f)
  C omega_m;  // 1/tau_m
  C k_m;      // 1/(tau_m cs2m)
  C b0;       // imposed field (along +y)
  C fex, fey; // external body force
  Wall<C> lo, hi;
  Trt<C> trt; // used by schemes with COLL_TRT
  Mrt<C> mrt; // used by schemes with COLL_MRT, or MRT_RT when mrt_on
  int mrt_on; // 1 for an MRT channel
  C xr_lo, xr_hi; // enclosure walls (WALLS_X): (theta-1)/(theta+1) at x = 0, nx-1
  Cut<C> clo, chi; // Hartmann walls at cut distances (WALLS_Q)
};

// Geometry of one channel's planes (element units).
struct Geom {
  int nx, ny;
  int pitch;          // elements between rows
  long long plane;    // elements between planes
};

// Observables a mode may need.
template <typename C>
struct NodeObs {
  C rho, rhop, ux, uy, bx, by, jz; // rhop = rho - 1 as accumulated from the deviations
};

// Every stored population is read once per step (pull).  A pull along x
// shifts a block's row segment by one node, so one cache line at each end of
// the segment is shared with the neighbouring block: those pulls (ldx) go
// through the caches, where the neighbour finds the line.  The others (ld)
// stream past them, as the stores do, unless rows are packed (NT false,
// the batched kernel): then a line at a row's end also holds the next
// row's start.
template <typename S, typename C, bool NT = true>
__device__ __forceinline__ C ld(const S *__restrict__ p) {
  if constexpr (NT) return static_cast<C>(__builtin_nontemporal_load(p));
  else return static_cast<C>(*p);
}
template <typename S, typename C>
__device__ __forceinline__ C ldx(const S *__restrict__ p) {
  return static_cast<C>(*p);
}

template <typename S, typename C>
__device__ __forceinline__ void st(S *__restrict__ p, C v) {
  __builtin_nontemporal_store(static_cast<S>(v), p);
}

// ---- stochastic rounding of the stored populations ----
// Round-to-nearest storage leaves the same rounding residual in every step
// once the flow is steady, and slow modes integrate it; rounding to one of
// the two neighbouring representable values with probabilities given by the
// distances makes the residual change from step to step (lks_sr.hpp).
template <typename S, typename C, bool SR, bool SEL = false>
__device__ __forceinline__ S to_store(C v, uint32_t r) {
  if constexpr (SR) {
    return round_sr<S, C, SEL>(v, r);
  } else {
    (void)r;
    return static_cast<S>(v);
  }
}

// Stochastic rounding applies when the compute type is wider than storage.
template <typename S, typename C>
constexpr bool kUseSR = (sizeof(C) > sizeof(S)) &&
                        ((sizeof(S) == 4 && LKS_SR_FP32) || (sizeof(S) == 2 && LKS_SR_FP16));

// Binary16 storage keeps a per-row reference D[y][plane] (compute type) that
// a rebase fills with each row's x-mean; wider storage keeps none.  It also
// stores its values multiplied by 2^12 (exact): once rebased, a steady row's
// stored values are far below binary16's normal range (2^-14), where the
// grid would be a fixed 2^-24 and set the noise floor of stochastic
// rounding; scaled, they keep 11 significant bits down to 2^-26.  Stored
// magnitudes stay below 16 (deviations of order one), far from the binary16
// limit 65504.
template <typename S> constexpr bool kRowRef = sizeof(S) == 2;
constexpr double kStoreUp16 = 4096.0, kStoreDown16 = 1.0 / 4096.0;

// Decode a stored value with the reference row it belongs to.
template <typename S, typename C>
__device__ __forceinline__ C dec(C v, const C *__restrict__ row, int plane) {
  if constexpr (kRowRef<S>) return v * C(kStoreDown16) + row[plane];
  else return v;
}

template <bool D> struct ComputeSel { using type = float; };
template <> struct ComputeSel<true> { using type = double; };
using Fp32Compute = ComputeSel<(LKS_FP32_COMPUTE_DOUBLE != 0)>::type;

// Weights (Secs. IV and V).
template <typename C> struct W {
  static constexpr C w0 = C(4) / C(9), w1 = C(1) / C(9), w5 = C(1) / C(36);
  static constexpr C W0 = C(1) / C(3), W1 = C(1) / C(6);
};

// Post-collision update of f_alpha in deviation form (Sec. V):
//   f~' = f' + omega (feq' - f') + kappa S,
//   feq' = w (rho' + rho poly),  S = 3 w (e.F - u.F) (1 + poly),
//   poly = 3 e.u + 4.5 (e.u)^2 - 1.5 u.u.
template <typename C>
__device__ __forceinline__ C collide_f(C f, C w, C ex, C ey, C rhop, C rho,
                                       C ux, C uy, C usq15, C Fx, C Fy, C uF,
                                       C omega, C kappa) {
  const C eu = ex * ux + ey * uy;
  const C poly = C(3) * eu + C(4.5) * eu * eu - usq15;
  const C feq = w * (rhop + rho * poly);
  const C S = C(3) * w * (ex * Fx + ey * Fy - uF) * (C(1) + poly);
  return f + omega * (feq - f) + kappa * S;
}

// Two-relaxation-time update of the pair (a, abar) of opposite f
// populations in deviation form (see Trt); eu = e_a.u and eF = e_a.F.
template <typename C>
__device__ __forceinline__ void collide_f_pair(C &fa, C &fb, C w, C eu, C eF, C rhop, C rho,
                                               C usq15, C uF, const Trt<C> &t) {
  const C even = C(4.5) * eu * eu - usq15;
  const C odd = C(3) * eu;
  const C pa = even + odd, pb = even - odd; // poly of a and of abar
  const C na = w * (rhop + rho * pa) - fa;
  const C nb = w * (rhop + rho * pb) - fb;
  const C Sa = C(3) * w * (eF - uF) * (C(1) + pa);
  const C Sb = C(3) * w * (-eF - uF) * (C(1) + pb);
  const C ra = fa + t.fa * na + t.fb * nb + t.fsa * Sa + t.fsb * Sb;
  const C rb = fb + t.fa * nb + t.fb * na + t.fsa * Sb + t.fsb * Sa;
  fa = ra;
  fb = rb;
}

// The same, also returning (n_a + n_abar) - (S_a + S_abar)/2, the pair's
// part of what the MRT corrections of the even moments e and epsilon act on.
template <typename C>
__device__ __forceinline__ void collide_f_pair(C &fa, C &fb, C w, C eu, C eF, C rhop, C rho,
                                               C usq15, C uF, const Trt<C> &t, C &tsum) {
  const C even = C(4.5) * eu * eu - usq15;
  const C odd = C(3) * eu;
  const C pa = even + odd, pb = even - odd;
  const C na = w * (rhop + rho * pa) - fa;
  const C nb = w * (rhop + rho * pb) - fb;
  const C Sa = C(3) * w * (eF - uF) * (C(1) + pa);
  const C Sb = C(3) * w * (-eF - uF) * (C(1) + pb);
  const C ra = fa + t.fa * na + t.fb * nb + t.fsa * Sa + t.fsb * Sb;
  const C rb = fb + t.fa * nb + t.fb * na + t.fsa * Sb + t.fsb * Sa;
  fa = ra;
  fb = rb;
  tsum = (na + nb) - C(0.5) * (Sa + Sb);
}

// Two-relaxation-time update of a pair of opposite g populations with
// equilibria ea, eb.
template <typename C>
__device__ __forceinline__ void collide_g_pair(C &ga, C &gb, C ea, C eb, const Trt<C> &t) {
  const C na = ea - ga, nb = eb - gb;
  const C ra = ga + t.ga * na + t.gb * nb;
  const C rb = gb + t.ga * nb + t.gb * na;
  ga = ra;
  gb = rb;
}

// Everything after streaming for one node: wall closure, moments, coupled
// solve, collision.  f, gx, gy hold the pulled (post-streaming) populations;
// those that would come from behind a wall are set by the closure (the
// link-based closure reads the node's own previous values from src).  The
// 19 new stored values (rounded to S) are returned in out (not for
// MODE_MOMENTS).
template <typename S, typename C, int BC, int MODE, bool SR>
__device__ __forceinline__ void node_finish(const Geom &g, const Coef<C> &k,
                                            const S *__restrict__ src,
                                            const C *__restrict__ ref, int x, int y,
                                            C (&f)[9], C (&gx)[5], C (&gy)[5],
                                            NodeObs<C> &obs, uint32_t sseed, S (&out)[19]) {
  const long long P = g.plane;
  const bool lo = (y == 0);
  const bool hi = (y == g.ny - 1);
  const long long r0 = (long long)y * g.pitch;
  const C *__restrict__ Dy = ref + (long long)y * 19; // reference of this row
  // ---- wall closures for the populations entering from a wall ----
  if constexpr (xwalls_of(BC)) {
    // Enclosure walls at x = -1/2 and nx - 1/2 (parallel to the imposed
    // field, stationary): bounce-back of f, theta closure of the induced
    // tangential b_y (stored as g_y - W B0), anti-bounce-back of B_x.  The
    // values pulled across the wall (periodic addresses) are replaced; the
    // Hartmann closure below then takes the corner links that cross it.
    if (x == 0) {
      f[1] = dec<S>(ld<S, C>(src + 3 * P + r0 + x), Dy, 3);
      f[5] = dec<S>(ld<S, C>(src + 7 * P + r0 + x), Dy, 7);
      f[8] = dec<S>(ld<S, C>(src + 6 * P + r0 + x), Dy, 6);
      gx[1] = -dec<S>(ld<S, C>(src + 12 * P + r0 + x), Dy, 12);
      gy[1] = k.xr_lo * dec<S>(ld<S, C>(src + 17 * P + r0 + x), Dy, 17);
    }
    if (x == g.nx - 1) {
      f[3] = dec<S>(ld<S, C>(src + 1 * P + r0 + x), Dy, 1);
      f[6] = dec<S>(ld<S, C>(src + 8 * P + r0 + x), Dy, 8);
      f[7] = dec<S>(ld<S, C>(src + 5 * P + r0 + x), Dy, 5);
      gx[3] = -dec<S>(ld<S, C>(src + 10 * P + r0 + x), Dy, 10);
      gy[3] = k.xr_hi * dec<S>(ld<S, C>(src + 15 * P + r0 + x), Dy, 15);
    }
  }
  if constexpr (wall_of(BC) == BC_LINK && cut_of(BC)) {
    // Hartmann walls at cut distances (Cut<C>); s = +1 at the lower wall,
    // -1 at the upper (the e_y of the incoming populations)
    auto at = [&](int plane, int yy, int xx) -> C {
      return dec<S>(ld<S, C>(src + plane * P + (long long)yy * g.pitch + xx),
                    ref + (long long)yy * 19, plane);
    };
    const int xm = (x == 0) ? g.nx - 1 : x - 1, xp = (x == g.nx - 1) ? 0 : x + 1;
    auto close = [&](const Cut<C> &c, int s, C uw6) {
      // incoming f: normal a0, diagonals a1 (e_x = +1), a2 (e_x = -1), each
      // with its opposite (outgoing) plane
      const int a0 = s > 0 ? 2 : 4, a1 = s > 0 ? 5 : 8, a2 = s > 0 ? 6 : 7;
      const int o0 = s > 0 ? 4 : 2, o1 = s > 0 ? 7 : 6, o2 = s > 0 ? 8 : 5;
      const int yn = y + s;
      const C out0 = at(o0, y, x), out1 = at(o1, y, x), out2 = at(o2, y, x);
      const C X0 = c.near ? at(o0, yn, x) : at(a0, y, x);
      const C X1 = c.near ? at(o1, yn, xp) : at(a1, y, x);
      const C X2 = c.near ? at(o2, yn, xm) : at(a2, y, x);
      const C n0 = c.fa * out0 + c.fb * X0;
      const C n1 = c.fa * out1 + c.fb * X1 + c.lscale * uw6;
      const C n2 = c.fa * out2 + c.fb * X2 - c.lscale * uw6;
      const C defect = (out0 + out1 + out2) - (n0 + n1 + n2);
      f[a0] = n0 + defect * (C(2) / C(3));
      f[a1] = n1 + defect * (C(1) / C(6));
      f[a2] = n2 + defect * (C(1) / C(6));
      // field: the D2Q5 link entering from the wall and its outgoing one
      const int gi = s > 0 ? 2 : 4, go = s > 0 ? 4 : 2;
      const C yo = at(14 + go, y, x);
      const C yX = c.near ? at(14 + go, yn, x) : at(14 + gi, y, x);
      gy[gi] = c.za * yo + c.zb * yX;
      const C xo = at(9 + go, y, x);
      if (!c.conducting) {
        const C xX = c.near ? at(9 + go, yn, x) : at(9 + gi, y, x);
        gx[gi] = c.za * xo + c.zb * xX;
      } else {
        const C x1 = at(9 + go, yn, x), x2 = at(9 + go, yn + s, x);
        C rhop = C(0), mx = C(0);
#pragma unroll
        for (int b = 0; b < 9; ++b) {
          const C v = at(b, y, x);
          rhop += v;
          mx += C(b == 1 || b == 5 || b == 8 ? 1 : (b == 3 || b == 6 || b == 7 ? -1 : 0)) * v;
        }
        const C un = mx / (C(1) + rhop);
        gx[gi] = c.r * xo + c.kappa * (x2 - C(2) * x1 + xo) + c.tmove + c.tshear * (un - c.u);
      }
    };
    // upper wall: the diagonal a1 = 8 has e_x = +1, a2 = 7 has e_x = -1;
    // Ladd's term is -U/6 on 7 and +U/6 on 8
    if (lo) close(k.clo, +1, k.lo.uw6);
    if (hi) close(k.chi, -1, k.hi.uw6);
  } else if (wall_of(BC) == BC_LINK) {
    // Half-way bounce-back of f with Ladd's moving-wall term; theta-weighted
    // bounce-back/anti-bounce-back of g_x; anti-bounce-back to B_y = B0 for
    // g_y, which for the deviations g_y - W B0 is g'_in = -g~'_out.  All from
    // the node's own post-collision values.
    if (lo) {
      f[2] = dec<S>(ld<S, C>(src + 4 * P + r0 + x), Dy, 4);
      f[5] = dec<S>(ld<S, C>(src + 7 * P + r0 + x), Dy, 7) + k.lo.uw6;
      f[6] = dec<S>(ld<S, C>(src + 8 * P + r0 + x), Dy, 8) - k.lo.uw6;
      gx[2] = k.lo.r * dec<S>(ld<S, C>(src + 13 * P + r0 + x), Dy, 13) + k.lo.t;
      gy[2] = -dec<S>(ld<S, C>(src + 18 * P + r0 + x), Dy, 18);
    }
    if (hi) {
      f[4] = dec<S>(ld<S, C>(src + 2 * P + r0 + x), Dy, 2);
      f[7] = dec<S>(ld<S, C>(src + 5 * P + r0 + x), Dy, 5) - k.hi.uw6;
      f[8] = dec<S>(ld<S, C>(src + 6 * P + r0 + x), Dy, 6) + k.hi.uw6;
      gx[4] = k.hi.r * dec<S>(ld<S, C>(src + 11 * P + r0 + x), Dy, 11) + k.hi.t;
      gy[4] = -dec<S>(ld<S, C>(src + 16 * P + r0 + x), Dy, 16);
    }
  } else {
    // On-node closures from the moment constraints, written for the
    // deviations f' = f - w (the weights of each relation sum out).
    if (lo) {
      const C U = k.lo.u;
      const C rhop = f[0] + f[1] + f[3] + C(2) * (f[4] + f[7] + f[8]);
      const C rho = C(1) + rhop;
      f[2] = -rhop * (C(1) / C(3)) - rho * U * U +
             (f[1] + f[3] + f[4] + C(2) * (f[7] + f[8]));
      f[5] = rhop * (C(1) / C(6)) + C(0.5) * rho * (U * U + U) - (f[1] + f[8]);
      f[6] = rhop * (C(1) / C(6)) + C(0.5) * rho * (U * U - U) - (f[3] + f[7]);
      gx[2] = k.lo.r * gx[4] - k.lo.s * (gx[0] + gx[1] + gx[3]) + k.lo.t;
      gy[2] = -(gy[0] + gy[1] + gy[3] + gy[4]); // sum g_y = B0
    }
    if (hi) {
      const C U = k.hi.u;
      const C rhop = f[0] + f[1] + f[3] + C(2) * (f[2] + f[5] + f[6]);
      const C rho = C(1) + rhop;
      f[4] = -rhop * (C(1) / C(3)) - rho * U * U +
             (f[1] + f[2] + f[3] + C(2) * (f[5] + f[6]));
      f[7] = rhop * (C(1) / C(6)) + C(0.5) * rho * (U * U - U) - (f[3] + f[6]);
      f[8] = rhop * (C(1) / C(6)) + C(0.5) * rho * (U * U + U) - (f[1] + f[5]);
      gx[4] = k.hi.r * gx[2] - k.hi.s * (gx[0] + gx[1] + gx[3]) + k.hi.t;
      gy[4] = -(gy[0] + gy[1] + gy[2] + gy[3]); // sum g_y = B0
    }
  }

  // ---- moments ----
  const C rhop = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const C rho = C(1) + rhop;
  const C mx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  const C my = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
  const C bx = (gx[0] + gx[1]) + (gx[2] + gx[3]) + gx[4];
  const C byp = (gy[0] + gy[1]) + (gy[2] + gy[3]) + gy[4]; // B_y - B0
  const C by = k.b0 + byp;
  const C D = (gy[1] - gy[3]) - (gx[2] - gx[4]); // Lambda_xy - Lambda_yx

  // ---- coupled local solve ----
  C ux, uy, jz, Fx, Fy;
  const C inv_rho = C(1) / rho;
  if (wall_of(BC) == BC_MOMENT && (lo || hi)) {
    // wet wall node: velocity fixed by the closure, no force
    ux = mx * inv_rho;
    uy = my * inv_rho;
    jz = -k.k_m * (D - C(2) * (ux * by - uy * bx));
    Fx = C(0);
    Fy = C(0);
  } else {
    // rho u = m + F/2, F = F_ext + J_z (-B_y, B_x),
    // J_z = -k [(L_xy - L0_xy) - (L_yx - L0_yx)], L0_xy = -L0_yx = u_x B_y - u_y B_x
    //  => J_z = k (2P - rho D) / (rho + k |B|^2),
    //     P = (m_x + Fe_x/2) B_y - (m_y + Fe_y/2) B_x.
    const C px = mx + C(0.5) * k.fex;
    const C py = my + C(0.5) * k.fey;
    const C Pm = px * by - py * bx;
    jz = k.k_m * (C(2) * Pm - rho * D) / (rho + k.k_m * (bx * bx + by * by));
    Fx = k.fex - jz * by;
    Fy = k.fey + jz * bx;
    ux = (mx + C(0.5) * Fx) * inv_rho;
    uy = (my + C(0.5) * Fy) * inv_rho;
  }
  obs.rho = rho;
  obs.rhop = rhop;
  obs.ux = ux;
  obs.uy = uy;
  obs.bx = bx;
  obs.by = by;
  obs.jz = jz;
  if (MODE == MODE_MOMENTS) return;

  // ---- collide and store ----
  // random words for the stochastic rounding of this node's 19 stores,
  // drawn in plane order
  Rng rng(SR ? node_seed(sseed, (uint32_t)(y * g.nx + x)) : 0u);
  // encode a post-collision value against this row's reference
  auto put = [&](C v, int plane) -> S {
    (void)plane;
    if constexpr (kRowRef<S>) v = (v - Dy[plane]) * C(kStoreUp16);
    return to_store<S, C, SR, in_batch(BC)>(v, SR ? rng.next() : 0u);
  };
  const C om = k.omega_f, ka = k.kappa_f;
  const C usq15 = C(1.5) * (ux * ux + uy * uy);
  const C uF = ux * Fx + uy * Fy;
  const C w0 = W<C>::w0, w1 = W<C>::w1, w5 = W<C>::w5;
  // g^eq_{a i} = W_a [B_i + e_aj (u_j B_i - B_j u_i) / cs2m]  (Sec. IV):
  // with E = u_x B_y - u_y B_x only g_2x, g_4x (-/+ 3E) and g_1y, g_3y (+/- 3E)
  // carry the flux term.
  const C E3 = C(3) * (ux * by - uy * bx);
  const C W0 = W<C>::W0, W1 = W<C>::W1;
  if constexpr (trt_of(BC) || mrt_of(BC)) {
    // pairs (1,3), (2,4), (5,7), (6,8) of D2Q9 and (1,3), (2,4) of D2Q5;
    // stores stay in plane order, so every plane keeps its random word.
    // MRT: the TRT step, then the corrections of e, epsilon and d (Mrt).
    const Trt<C> &t = k.trt;
    // MRT: te, tp = the e and epsilon moments of n - S/2 (rows (-4, -1 x4,
    // 2 x4) and (4, -2 x4, 1 x4)), accumulated pair by pair
    constexpr bool kMrt = mrt_of(BC) || mrt_rt_of(BC);
    const bool mrt_now = mrt_of(BC) || (mrt_rt_of(BC) && k.mrt_on != 0);
    const C t0 = (w0 * (rhop - rho * usq15) - f[0]) - C(0.5) * (C(3) * w0 * (-uF) * (C(1) - usq15));
    C te = C(-4) * t0, tp = C(4) * t0, tq;
    f[0] = collide_f(f[0], w0, C(0), C(0), rhop, rho, ux, uy, usq15, Fx, Fy, uF, om, ka);
    collide_f_pair(f[1], f[3], w1, ux, Fx, rhop, rho, usq15, uF, t, tq);
    te -= tq, tp -= C(2) * tq;
    collide_f_pair(f[2], f[4], w1, uy, Fy, rhop, rho, usq15, uF, t, tq);
    te -= tq, tp -= C(2) * tq;
    collide_f_pair(f[5], f[7], w5, ux + uy, Fx + Fy, rhop, rho, usq15, uF, t, tq);
    te += C(2) * tq, tp += tq;
    collide_f_pair(f[6], f[8], w5, uy - ux, Fy - Fx, rhop, rho, usq15, uF, t, tq);
    te += C(2) * tq, tp += tq;
    // (selects rather than a branch where the flag is a run-time value: the
    // branch cost the batched kernel 20 registers)
    C gdx = C(0), gdy = C(0);
    if constexpr (kMrt) {
      const Mrt<C> &m = k.mrt;
      const C de = m.ke * te, dp = m.keps * tp;
      const C d0 = C(4) * (dp - de), dax = -de - C(2) * dp, ddg = C(2) * de + dp;
      f[0] = mrt_now ? f[0] + d0 : f[0];
#pragma unroll
      for (int q = 1; q < 5; ++q) f[q] = mrt_now ? f[q] + dax : f[q];
#pragma unroll
      for (int q = 5; q < 9; ++q) f[q] = mrt_now ? f[q] + ddg : f[q];
      // d = (g1 + g3) - (g2 + g4) of n = geq - g, before the update
      gdx = m.kd * ((C(2) * W1 * bx - gx[1] - gx[3]) - (C(2) * W1 * bx - gx[2] - gx[4]));
      gdy = m.kd * ((C(2) * W1 * byp - gy[1] - gy[3]) - (C(2) * W1 * byp - gy[2] - gy[4]));
    }
    gx[0] += t.gp * (W0 * bx - gx[0]);
    collide_g_pair(gx[1], gx[3], W1 * bx, W1 * bx, t);
    collide_g_pair(gx[2], gx[4], W1 * (bx - E3), W1 * (bx + E3), t);
    gy[0] += t.gp * (W0 * byp - gy[0]);
    collide_g_pair(gy[1], gy[3], W1 * (byp + E3), W1 * (byp - E3), t);
    collide_g_pair(gy[2], gy[4], W1 * byp, W1 * byp, t);
    if constexpr (kMrt) {
      gx[1] = mrt_now ? gx[1] + gdx : gx[1], gx[3] = mrt_now ? gx[3] + gdx : gx[3];
      gx[2] = mrt_now ? gx[2] - gdx : gx[2], gx[4] = mrt_now ? gx[4] - gdx : gx[4];
      gy[1] = mrt_now ? gy[1] + gdy : gy[1], gy[3] = mrt_now ? gy[3] + gdy : gy[3];
      gy[2] = mrt_now ? gy[2] - gdy : gy[2], gy[4] = mrt_now ? gy[4] - gdy : gy[4];
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) out[q] = put(f[q], q);
#pragma unroll
    for (int q = 0; q < 5; ++q) out[9 + q] = put(gx[q], 9 + q);
#pragma unroll
    for (int q = 0; q < 5; ++q) out[14 + q] = put(gy[q], 14 + q);
    return;
  }
  out[0] = put(collide_f(f[0], w0, C(0), C(0), rhop, rho, ux, uy, usq15, Fx, Fy, uF, om, ka), 0);
  out[1] = put(collide_f(f[1], w1, C(1), C(0), rhop, rho, ux, uy, usq15, Fx, Fy, uF, om, ka), 1);
  out[2] = put(collide_f(f[2], w1, C(0), C(1), rhop, rho, ux, uy, usq15, Fx, Fy, uF, om, ka), 2);
  out[3] = put(collide_f(f[3], w1, C(-1), C(0), rhop, rho, ux, uy, usq15, Fx, Fy, uF, om, ka), 3);
  out[4] = put(collide_f(f[4], w1, C(0), C(-1), rhop, rho, ux, uy, usq15, Fx, Fy, uF, om, ka), 4);
  out[5] = put(collide_f(f[5], w5, C(1), C(1), rhop, rho, ux, uy, usq15, Fx, Fy, uF, om, ka), 5);
  out[6] = put(collide_f(f[6], w5, C(-1), C(1), rhop, rho, ux, uy, usq15, Fx, Fy, uF, om, ka), 6);
  out[7] = put(collide_f(f[7], w5, C(-1), C(-1), rhop, rho, ux, uy, usq15, Fx, Fy, uF, om, ka), 7);
  out[8] = put(collide_f(f[8], w5, C(1), C(-1), rhop, rho, ux, uy, usq15, Fx, Fy, uF, om, ka), 8);

  const C wm = k.omega_m;
  out[9] = put(gx[0] + wm * (W0 * bx - gx[0]), 9);
  out[10] = put(gx[1] + wm * (W1 * bx - gx[1]), 10);
  out[11] = put(gx[2] + wm * (W1 * (bx - E3) - gx[2]), 11);
  out[12] = put(gx[3] + wm * (W1 * bx - gx[3]), 12);
  out[13] = put(gx[4] + wm * (W1 * (bx + E3) - gx[4]), 13);
  out[14] = put(gy[0] + wm * (W0 * byp - gy[0]), 14);
  out[15] = put(gy[1] + wm * (W1 * (byp + E3) - gy[1]), 15);
  out[16] = put(gy[2] + wm * (W1 * byp - gy[2]), 16);
  out[17] = put(gy[3] + wm * (W1 * (byp - E3) - gy[3]), 17);
  out[18] = put(gy[4] + wm * (W1 * byp - gy[4]), 18);
}


template <typename S, typename C, int BC, int MODE, bool SR>
__device__ __forceinline__ void node_update(const Geom &g, const Coef<C> &k,
                                            const S *__restrict__ src,
                                            const C *__restrict__ ref,
                                            S *__restrict__ dst, int x, int y,
                                            NodeObs<C> &obs, uint32_t sseed) {
  const int nx = g.nx;
  const long long P = g.plane;
  const int xm = (x == 0) ? nx - 1 : x - 1;
  const int xp = (x == nx - 1) ? 0 : x + 1;
  const bool lo = (y == 0);
  const bool hi = (y == g.ny - 1);
  const long long r0 = (long long)y * g.pitch;
  const long long rm = r0 - g.pitch;
  const long long rp = r0 + g.pitch;

  // ---- pull streaming: f_a(x) = f~_a(x - e_a) ----
  // stored values are decoded with the reference of the row they come from
  const C *__restrict__ Dy = ref + (long long)y * 19;
  const C *__restrict__ Dm = lo ? Dy : Dy - 19; // row y - 1 (used only off the lower wall)
  const C *__restrict__ Dp = hi ? Dy : Dy + 19; // row y + 1 (used only off the upper wall)
  constexpr bool NT = !in_batch(BC);
  C f[9], gx[5], gy[5];
  f[0] = dec<S>(ld<S, C, NT>(src + r0 + x), Dy, 0);
  f[1] = dec<S>(ldx<S, C>(src + 1 * P + r0 + xm), Dy, 1);
  f[3] = dec<S>(ldx<S, C>(src + 3 * P + r0 + xp), Dy, 3);
  gx[0] = dec<S>(ld<S, C, NT>(src + 9 * P + r0 + x), Dy, 9);
  gx[1] = dec<S>(ldx<S, C>(src + 10 * P + r0 + xm), Dy, 10);
  gx[3] = dec<S>(ldx<S, C>(src + 12 * P + r0 + xp), Dy, 12);
  gy[0] = dec<S>(ld<S, C, NT>(src + 14 * P + r0 + x), Dy, 14);
  gy[1] = dec<S>(ldx<S, C>(src + 15 * P + r0 + xm), Dy, 15);
  gy[3] = dec<S>(ldx<S, C>(src + 17 * P + r0 + xp), Dy, 17);
  if (!lo) {
    f[2] = dec<S>(ld<S, C, NT>(src + 2 * P + rm + x), Dm, 2);
    f[5] = dec<S>(ldx<S, C>(src + 5 * P + rm + xm), Dm, 5);
    f[6] = dec<S>(ldx<S, C>(src + 6 * P + rm + xp), Dm, 6);
    gx[2] = dec<S>(ld<S, C, NT>(src + 11 * P + rm + x), Dm, 11);
    gy[2] = dec<S>(ld<S, C, NT>(src + 16 * P + rm + x), Dm, 16);
  }
  if (!hi) {
    f[4] = dec<S>(ld<S, C, NT>(src + 4 * P + rp + x), Dp, 4);
    f[7] = dec<S>(ldx<S, C>(src + 7 * P + rp + xp), Dp, 7);
    f[8] = dec<S>(ldx<S, C>(src + 8 * P + rp + xm), Dp, 8);
    gx[4] = dec<S>(ld<S, C, NT>(src + 13 * P + rp + x), Dp, 13);
    gy[4] = dec<S>(ld<S, C, NT>(src + 18 * P + rp + x), Dp, 18);
  }

  NodeObs<C> &o_ = obs;
  S out[19];
  node_finish<S, C, BC, MODE, SR>(g, k, src, ref, x, y, f, gx, gy, o_, sseed, out);
  if constexpr (MODE != MODE_MOMENTS) {
    const long long o = r0 + x;
#pragma unroll
    for (int q = 0; q < 19; ++q) __builtin_nontemporal_store(out[q], dst + q * P + o);
  } else {
    (void)dst;
  }
}

// ---- FP64 block reduction (deterministic: fixed shuffle and LDS order) ----
template <int NV>
__device__ __forceinline__ void wave_sum(double (&v)[NV]) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] += __shfl_xor(v[i], off, 64);
  }
}

// Sums v over the block; thread 0 of the block returns the totals in v.
template <int NV, int NTHREADS>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds) {
  constexpr int NW = NTHREADS / 64;
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  wave_sum<NV>(v);
  if constexpr (NW > 1) {
    const int lane = tid & 63, wid = tid >> 6;
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < NV; ++i) lds[wid * NV + i] = v[i];
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        double s = 0.0;
        for (int w = 0; w < NW; ++w) s += lds[w * NV + i];
        v[i] = s;
      }
    }
  }
}

} // namespace lks
