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

#include <type_traits>

#include "lks_geometry.hpp"
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
// ... and with SOLIDS where solid bodies (curved walls) lie in the channel
constexpr int SOLIDS = 256;
constexpr int wall_of(int scheme) { return scheme & 3; }
constexpr bool trt_of(int scheme) { return (scheme & COLL_TRT) != 0; }
constexpr bool xwalls_of(int scheme) { return (scheme & WALLS_X) != 0; }
constexpr bool cut_of(int scheme) { return (scheme & WALLS_Q) != 0; }
constexpr bool in_batch(int scheme) { return (scheme & IN_BATCH) != 0; }
constexpr bool mrt_of(int scheme) { return (scheme & COLL_MRT) != 0; }
constexpr bool mrt_rt_of(int scheme) { return (scheme & MRT_RT) != 0; }
constexpr bool solids_of(int scheme) { return (scheme & SOLIDS) != 0; }
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
  const int32_t *sidx;     // solid bodies (SOLIDS): per node kSolidFluid, kSolidNode or
  const CurvedNode *snode; // an index into snode (device arrays, lks_geometry.hpp)
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
  C fx, fy;                        // total force the collision adds to the momentum
};

// Every stored population is read once per step (pull).  A pull along x
// shifts a block's row segment by one node, so one cache line at each end of
// the segment is shared with the neighbouring block: those pulls (ldx) go
// through the caches, where the neighbour finds the line.  The others (ld)
// stream past them, as the stores do, unless rows are packed (NT false,
// the batched kernel in FP32 and FP64 storage): then a line at a row's end
// also holds the next row's start.  (Binary16 storage in the batched
// kernel streams them all the same: measured faster there.)
// Populations live in global memory.  Loads and stores go through pointers
// of that address space, so that the compiler emits global (not flat)
// instructions also where the base pointer was read from memory (the batched
// kernel's channel descriptors) rather than passed as a kernel argument.
template <typename T> using gptr = __attribute__((address_space(1))) T *;

// A plane's base address pinned in scalar registers.  Where every plane is
// accessed at one common per-thread offset (the stores), the compiler would
// otherwise add that offset to the kernel's base once and then each plane's
// stride to the result, in 64-bit vector arithmetic per plane; an opaque
// scalar base keeps the scalar-base + 32-bit vector-offset form instead.
// p must be the same in every active lane of the wavefront (a kernel
// argument, or a channel's buffer where a block works on one channel).
template <typename T> __device__ __forceinline__ T *sbase(T *p) {
  // (reading it from the first lane tells the compiler that it is uniform
  // where its analysis cannot)
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  asm("" : "+s"(lo), "+s"(hi));
  return reinterpret_cast<T *>(((uint64_t)hi << 32) | lo);
}

template <typename S, typename C, bool NT = true>
__device__ __forceinline__ C ld(const S *__restrict__ p) {
  if constexpr (NT) return static_cast<C>(__builtin_nontemporal_load((gptr<const S>)p));
  else return static_cast<C>(*(gptr<const S>)p);
}
template <typename S, typename C>
__device__ __forceinline__ C ldx(const S *__restrict__ p) {
  return static_cast<C>(*(gptr<const S>)p);
}

template <typename S, typename C>
__device__ __forceinline__ void st(S *__restrict__ p, C v) {
  __builtin_nontemporal_store(static_cast<S>(v), (gptr<S>)p);
}

// ---- stochastic rounding of the stored populations ----
// Round-to-nearest storage leaves the same rounding residual in every step
// once the flow is steady, and slow modes integrate it; rounding to one of
// the two neighbouring representable values with probabilities given by the
// distances makes the residual change from step to step (lks_sr.hpp).
template <typename S, typename C, bool SR>
__device__ __forceinline__ S to_store(C v, uint32_t r) {
  if constexpr (SR) {
    return round_sr<S, C>(v, r);
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
// Elements per row of the reference tables (19 planes, padded for aligned
// vector loads).
constexpr int kRefRow = 20;

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
// INC: the increment f~' - f' instead of the new value.
template <typename C, bool INC = false>
__device__ __forceinline__ C collide_f(C f, C w, C ex, C ey, C rhop, C rho,
                                       C ux, C uy, C usq15, C Fx, C Fy, C uF,
                                       C omega, C kappa) {
  const C eu = ex * ux + ey * uy;
  const C poly = C(3) * eu + C(4.5) * eu * eu - usq15;
  const C feq = w * (rhop + rho * poly);
  const C S = C(3) * w * (ex * Fx + ey * Fy - uF) * (C(1) + poly);
  if constexpr (INC) return omega * (feq - f) + kappa * S;
  else return f + omega * (feq - f) + kappa * S;
}

// Two-relaxation-time update of the pair (a, abar) of opposite f
// populations in deviation form (see Trt); eu = e_a.u and eF = e_a.F.
template <typename C, bool INC = false>
__device__ __forceinline__ void collide_f_pair(C &fa, C &fb, C w, C eu, C eF, C rhop, C rho,
                                               C usq15, C uF, const Trt<C> &t) {
  const C even = C(4.5) * eu * eu - usq15;
  const C odd = C(3) * eu;
  const C pa = even + odd, pb = even - odd; // poly of a and of abar
  const C na = w * (rhop + rho * pa) - fa;
  const C nb = w * (rhop + rho * pb) - fb;
  const C Sa = C(3) * w * (eF - uF) * (C(1) + pa);
  const C Sb = C(3) * w * (-eF - uF) * (C(1) + pb);
  if constexpr (INC) {
    const C ra = t.fa * na + t.fb * nb + t.fsa * Sa + t.fsb * Sb;
    const C rb = t.fa * nb + t.fb * na + t.fsa * Sb + t.fsb * Sa;
    fa = ra;
    fb = rb;
  } else {
    const C ra = fa + t.fa * na + t.fb * nb + t.fsa * Sa + t.fsb * Sb;
    const C rb = fb + t.fa * nb + t.fb * na + t.fsa * Sb + t.fsb * Sa;
    fa = ra;
    fb = rb;
  }
}

// The same, also returning (n_a + n_abar) - (S_a + S_abar)/2, the pair's
// part of what the MRT corrections of the even moments e and epsilon act on.
template <typename C, bool INC = false>
__device__ __forceinline__ void collide_f_pair(C &fa, C &fb, C w, C eu, C eF, C rhop, C rho,
                                               C usq15, C uF, const Trt<C> &t, C &tsum) {
  const C even = C(4.5) * eu * eu - usq15;
  const C odd = C(3) * eu;
  const C pa = even + odd, pb = even - odd;
  const C na = w * (rhop + rho * pa) - fa;
  const C nb = w * (rhop + rho * pb) - fb;
  const C Sa = C(3) * w * (eF - uF) * (C(1) + pa);
  const C Sb = C(3) * w * (-eF - uF) * (C(1) + pb);
  if constexpr (INC) {
    const C ra = t.fa * na + t.fb * nb + t.fsa * Sa + t.fsb * Sb;
    const C rb = t.fa * nb + t.fb * na + t.fsa * Sb + t.fsb * Sa;
    fa = ra;
    fb = rb;
  } else {
    const C ra = fa + t.fa * na + t.fb * nb + t.fsa * Sa + t.fsb * Sb;
    const C rb = fb + t.fa * nb + t.fb * na + t.fsa * Sb + t.fsb * Sa;
    fa = ra;
    fb = rb;
  }
  tsum = (na + nb) - C(0.5) * (Sa + Sb);
}

// BGK increments of the pair (a, abar) of opposite f populations
// (f~ - f = omega (feq - f) + kappa S for each), written with the parts of
// the equilibrium and the source even and odd under e -> -e.
template <typename C>
__device__ __forceinline__ void collide_f_pair_bgk(C &fa, C &fb, C w, C eu, C eF, C rhop, C rho,
                                                   C usq15, C uF, C omega, C kappa) {
  const C even = C(4.5) * eu * eu - usq15;
  const C odd = C(3) * eu;
  const C pa = even + odd, pb = even - odd;
  const C na = w * (rhop + rho * pa) - fa;
  const C nb = w * (rhop + rho * pb) - fb;
  const C ks = C(3) * w * kappa;
  fa = omega * na + ks * ((eF - uF) * (C(1) + pa));
  fb = omega * nb + ks * ((-eF - uF) * (C(1) + pb));
}

// Two-relaxation-time update of a pair of opposite g populations with
// equilibria ea, eb.
template <typename C, bool INC = false>
__device__ __forceinline__ void collide_g_pair(C &ga, C &gb, C ea, C eb, const Trt<C> &t) {
  const C na = ea - ga, nb = eb - gb;
  if constexpr (INC) {
    const C ra = t.ga * na + t.gb * nb;
    const C rb = t.ga * nb + t.gb * na;
    ga = ra;
    gb = rb;
  } else {
    const C ra = ga + t.ga * na + t.gb * nb;
    const C rb = gb + t.ga * nb + t.gb * na;
    ga = ra;
    gb = rb;
  }
}

// ---- wall closures of the populations entering from a wall ----

// Links of a fluid node that come from a solid body (curved walls, the
// coefficients of lks_geometry.hpp): f_a = ca o + cb X + mw and, for the
// D2Q5 links, g_a = za o + zb X per component, o the node's own population
// leaving towards the surface and X the next node's (near) or the node's own
// h_a.  Populations are in the stored deviation form, in which these maps
// hold unchanged (ca + cb = 1; the surface holds g at its rest value).
template <typename S, typename C>
__device__ __forceinline__ void solid_closure(const Geom &g, const CurvedNode &cn,
                                              const S *__restrict__ src,
                                              const C *__restrict__ ref, int x, int y,
                                              C (&f)[9], C (&gx)[5], C (&gy)[5]) {
  constexpr int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  constexpr int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
  const long long P = g.plane;
  auto at = [&](int plane, int yy, int xx) -> C {
    xx = xx < 0 ? xx + g.nx : (xx >= g.nx ? xx - g.nx : xx);
    return dec<S>(ld<S, C>(src + plane * P + (long long)yy * g.pitch + xx),
                  ref + (long long)yy * kRefRow, plane);
  };
  const uint32_t cut = cn.cut, near = cn.near;
#pragma unroll
  for (int a = 1; a < 9; ++a) {
    if (!((cut >> a) & 1u)) continue;
    const int b = opp[a];
    const bool nr = (near >> a) & 1u;
    const int xs = nr ? x + ex[a] : x, ys = nr ? y + ey[a] : y; // X's node
    const int px = nr ? b : a;                                  // and plane
    f[a] = C(cn.ca[a - 1]) * at(b, y, x) + C(cn.cb[a - 1]) * at(px, ys, xs) + C(cn.mw[a - 1]);
    if (a <= 4) {
      const C za = C(cn.za[a - 1]), zb = C(cn.zb[a - 1]);
      gx[a] = za * at(9 + b, y, x) + zb * at(9 + px, ys, xs);
      gy[a] = za * at(14 + b, y, x) + zb * at(14 + px, ys, xs);
    }
  }
}

// Enclosure walls at x = -1/2 and nx - 1/2 (parallel to the imposed field,
// stationary): bounce-back of f, theta closure of the induced tangential
// b_y (stored as g_y - W B0), anti-bounce-back of B_x.  The values pulled
// across the wall (periodic addresses) are replaced from the node's own
// previous values; a Hartmann closure applied afterwards takes the corner
// links that cross it.
template <typename S, typename C>
__device__ __forceinline__ void xwall_closure(const Geom &g, const Coef<C> &k,
                                              const S *__restrict__ src,
                                              const C *__restrict__ Dy, int x, int y,
                                              C (&f)[9], C (&gx)[5], C (&gy)[5]) {
  const long long P = g.plane;
  const long long r0 = (long long)y * g.pitch;
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

// Link-based Hartmann walls at cut distances (Cut<C>).
template <typename S, typename C>
__device__ __forceinline__ void cut_closure(const Geom &g, const Coef<C> &k,
                                            const S *__restrict__ src,
                                            const C *__restrict__ ref, int x, int y,
                                            C (&f)[9], C (&gx)[5], C (&gy)[5]) {
  const long long P = g.plane;
  const bool lo = (y == 0);
  const bool hi = (y == g.ny - 1);
  // s = +1 at the lower wall, -1 at the upper (the e_y of the incoming
  // populations)
  auto at = [&](int plane, int yy, int xx) -> C {
    return dec<S>(ld<S, C>(src + plane * P + (long long)yy * g.pitch + xx),
                  ref + (long long)yy * kRefRow, plane);
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
}

// The paper's two Hartmann-wall closures (walls half-way between rows for
// the link-based scheme, on the wall rows for the moment-based one) as
// affine maps of the node's values: closed = A(values) + b.  For the link
// scheme the values are the node's own post-collision populations leaving
// through the wall, own[] = (f_4, f_7, f_8, g_4x, g_4y) at the lower wall and
// (f_2, f_5, f_6, g_2x, g_2y) at the upper one; for the moment scheme they are
// the node's known post-streaming populations in f, gx, gy.  AFF false
// applies A alone, to deviations from a reference state whose closed values
// carry b.
//   link:   half-way bounce-back of f with Ladd's moving-wall term; the
//           theta-weighted bounce-back/anti-bounce-back of g_x; anti-bounce-
//           back to B_y = B0 of g_y, which for the deviations g_y - W B0 is
//           g'_in = -g~'_out (Sec. VI Eq. linkbasedBCschemefinal, App. B.1).
//   moment: f from the moment constraints Pi_10 = rho U, Pi_01 = 0,
//           Pi_20 = rho (cs2 + U^2) written for the deviations f' = f - w;
//           g_x from the discrete Shercliff relation; g_y from sum g_y = B0
//           (Sec. VII, App. A, App. B.2).
template <typename T, int WALL, bool AFF>
__device__ __forceinline__ void hartmann_closure(bool lo, bool hi, T (&f)[9], T (&gx)[5],
                                                 T (&gy)[5], const T (&own)[5],
                                                 const Wall<T> &wl, const Wall<T> &wh) {
  const T one = AFF ? T(1) : T(0);
  if constexpr (WALL == BC_LINK) {
    if (lo) {
      f[2] = own[0];
      f[5] = AFF ? own[1] + wl.uw6 : own[1];
      f[6] = AFF ? own[2] - wl.uw6 : own[2];
      gx[2] = AFF ? wl.r * own[3] + wl.t : wl.r * own[3];
      gy[2] = -own[4];
    }
    if (hi) {
      f[4] = own[0];
      f[7] = AFF ? own[1] - wh.uw6 : own[1];
      f[8] = AFF ? own[2] + wh.uw6 : own[2];
      gx[4] = AFF ? wh.r * own[3] + wh.t : wh.r * own[3];
      gy[4] = -own[4];
    }
  } else {
    if (lo) {
      const T U = wl.u;
      const T rhop = f[0] + f[1] + f[3] + T(2) * (f[4] + f[7] + f[8]);
      const T rho = one + rhop;
      f[2] = -rhop * (T(1) / T(3)) - rho * U * U + (f[1] + f[3] + f[4] + T(2) * (f[7] + f[8]));
      f[5] = rhop * (T(1) / T(6)) + T(0.5) * rho * (U * U + U) - (f[1] + f[8]);
      f[6] = rhop * (T(1) / T(6)) + T(0.5) * rho * (U * U - U) - (f[3] + f[7]);
      gx[2] = AFF ? wl.r * gx[4] - wl.s * (gx[0] + gx[1] + gx[3]) + wl.t
                  : wl.r * gx[4] - wl.s * (gx[0] + gx[1] + gx[3]);
      gy[2] = -(gy[0] + gy[1] + gy[3] + gy[4]); // sum g_y = B0
    }
    if (hi) {
      const T U = wh.u;
      const T rhop = f[0] + f[1] + f[3] + T(2) * (f[2] + f[5] + f[6]);
      const T rho = one + rhop;
      f[4] = -rhop * (T(1) / T(3)) - rho * U * U + (f[1] + f[2] + f[3] + T(2) * (f[5] + f[6]));
      f[7] = rhop * (T(1) / T(6)) + T(0.5) * rho * (U * U - U) - (f[3] + f[6]);
      f[8] = rhop * (T(1) / T(6)) + T(0.5) * rho * (U * U + U) - (f[1] + f[5]);
      gx[4] = AFF ? wh.r * gx[2] - wh.s * (gx[0] + gx[1] + gx[3]) + wh.t
                  : wh.r * gx[2] - wh.s * (gx[0] + gx[1] + gx[3]);
      gy[4] = -(gy[0] + gy[1] + gy[2] + gy[3]); // sum g_y = B0
    }
  }
}

// Everything after streaming for one node: wall closure, moments, coupled
// solve, collision.  f, gx, gy hold the pulled (post-streaming) populations;
// those that would come from behind a wall are set by the closure (the
// link-based closure reads the node's own previous values from src).  The
// 19 new stored values (rounded to S) are returned in out (not for
// MODE_MOMENTS).
// XA: the caller has applied every closure already, and the collision's
// increments (new minus old value) are returned in f, gx, gy instead; the
// caller accumulates and stores them (node_finish_x).
template <typename S, typename C, int BC, int MODE, bool SR, bool XA = false>
__device__ __forceinline__ void node_finish(const Geom &g, const Coef<C> &k,
                                            const S *__restrict__ src,
                                            const C *__restrict__ ref, int x, int y,
                                            C (&f)[9], C (&gx)[5], C (&gy)[5],
                                            NodeObs<C> &obs, uint32_t sseed, S (&out)[19]) {
  const bool lo = (y == 0);
  const bool hi = (y == g.ny - 1);
  const C *__restrict__ Dy = ref + (long long)y * kRefRow; // reference of this row
  // ---- wall closures for the populations entering from a wall ----
  if constexpr (!XA) {
    if constexpr (xwalls_of(BC)) xwall_closure<S, C>(g, k, src, Dy, x, y, f, gx, gy);
    if constexpr (wall_of(BC) == BC_LINK && cut_of(BC)) {
      cut_closure<S, C>(g, k, src, ref, x, y, f, gx, gy);
    } else if constexpr (wall_of(BC) == BC_LINK) {
      if (lo || hi) {
        const long long P = g.plane;
        const long long r0 = (long long)y * g.pitch;
        // the node's own post-collision values leaving through the wall
        const int p0 = lo ? 4 : 2, p1 = lo ? 7 : 5, p2 = lo ? 8 : 6;
        const C own[5] = {dec<S>(ld<S, C>(src + p0 * P + r0 + x), Dy, p0),
                          dec<S>(ld<S, C>(src + p1 * P + r0 + x), Dy, p1),
                          dec<S>(ld<S, C>(src + p2 * P + r0 + x), Dy, p2),
                          dec<S>(ld<S, C>(src + (9 + p0) * P + r0 + x), Dy, 9 + p0),
                          dec<S>(ld<S, C>(src + (14 + p0) * P + r0 + x), Dy, 14 + p0)};
        hartmann_closure<C, BC_LINK, true>(lo, hi, f, gx, gy, own, k.lo, k.hi);
      }
    } else {
      const C none[5] = {C(0), C(0), C(0), C(0), C(0)};
      hartmann_closure<C, BC_MOMENT, true>(lo, hi, f, gx, gy, none, k.lo, k.hi);
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
  // (the exact-accumulation mode takes the hardware reciprocal, 1 ulp: its
  // error stays out of the conserved moments, which are restored in FP64)
  auto recip = [](C v) -> C {
    if constexpr (XA && sizeof(C) == 4) return __builtin_amdgcn_rcpf(v);
    else return C(1) / v;
  };
  const C inv_rho = recip(rho);
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
    if constexpr (XA) jz = k.k_m * (C(2) * Pm - rho * D) * recip(rho + k.k_m * (bx * bx + by * by));
    else jz = k.k_m * (C(2) * Pm - rho * D) / (rho + k.k_m * (bx * bx + by * by));
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
  obs.fx = Fx;
  obs.fy = Fy;
  if (MODE == MODE_MOMENTS) return;

  // ---- collide and store ----
  // random words for the stochastic rounding of this node's 19 stores,
  // drawn in plane order
  Rng rng(SR && !XA ? node_seed(sseed, (uint32_t)(y * g.nx + x)) : 0u);
  // encode a post-collision value against this row's reference
  auto put = [&](C v, int plane) -> S {
    (void)plane;
    if constexpr (kRowRef<S>) v = (v - Dy[plane]) * C(kStoreUp16);
    return to_store<S, C, SR>(v, SR ? rng.next() : 0u);
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
    f[0] = collide_f<C, XA>(f[0], w0, C(0), C(0), rhop, rho, ux, uy, usq15, Fx, Fy, uF, om, ka);
    collide_f_pair<C, XA>(f[1], f[3], w1, ux, Fx, rhop, rho, usq15, uF, t, tq);
    te -= tq, tp -= C(2) * tq;
    collide_f_pair<C, XA>(f[2], f[4], w1, uy, Fy, rhop, rho, usq15, uF, t, tq);
    te -= tq, tp -= C(2) * tq;
    collide_f_pair<C, XA>(f[5], f[7], w5, ux + uy, Fx + Fy, rhop, rho, usq15, uF, t, tq);
    te += C(2) * tq, tp += tq;
    collide_f_pair<C, XA>(f[6], f[8], w5, uy - ux, Fy - Fx, rhop, rho, usq15, uF, t, tq);
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
    if constexpr (XA) gx[0] = t.gp * (W0 * bx - gx[0]);
    else gx[0] += t.gp * (W0 * bx - gx[0]);
    collide_g_pair<C, XA>(gx[1], gx[3], W1 * bx, W1 * bx, t);
    collide_g_pair<C, XA>(gx[2], gx[4], W1 * (bx - E3), W1 * (bx + E3), t);
    if constexpr (XA) gy[0] = t.gp * (W0 * byp - gy[0]);
    else gy[0] += t.gp * (W0 * byp - gy[0]);
    collide_g_pair<C, XA>(gy[1], gy[3], W1 * (byp + E3), W1 * (byp - E3), t);
    collide_g_pair<C, XA>(gy[2], gy[4], W1 * byp, W1 * byp, t);
    if constexpr (kMrt) {
      gx[1] = mrt_now ? gx[1] + gdx : gx[1], gx[3] = mrt_now ? gx[3] + gdx : gx[3];
      gx[2] = mrt_now ? gx[2] - gdx : gx[2], gx[4] = mrt_now ? gx[4] - gdx : gx[4];
      gy[1] = mrt_now ? gy[1] + gdy : gy[1], gy[3] = mrt_now ? gy[3] + gdy : gy[3];
      gy[2] = mrt_now ? gy[2] - gdy : gy[2], gy[4] = mrt_now ? gy[4] - gdy : gy[4];
    }
    if constexpr (!XA) {
#pragma unroll
      for (int q = 0; q < 9; ++q) out[q] = put(f[q], q);
#pragma unroll
      for (int q = 0; q < 5; ++q) out[9 + q] = put(gx[q], 9 + q);
#pragma unroll
      for (int q = 0; q < 5; ++q) out[14 + q] = put(gy[q], 14 + q);
    }
    return;
  }
  const C wm = k.omega_m;
  if constexpr (XA) {
    // the opposite pairs share e.u and the even part of the equilibrium
    f[0] = collide_f<C, true>(f[0], w0, C(0), C(0), rhop, rho, ux, uy, usq15, Fx, Fy, uF, om, ka);
    collide_f_pair_bgk(f[1], f[3], w1, ux, Fx, rhop, rho, usq15, uF, om, ka);
    collide_f_pair_bgk(f[2], f[4], w1, uy, Fy, rhop, rho, usq15, uF, om, ka);
    collide_f_pair_bgk(f[5], f[7], w5, ux + uy, Fx + Fy, rhop, rho, usq15, uF, om, ka);
    collide_f_pair_bgk(f[6], f[8], w5, uy - ux, Fy - Fx, rhop, rho, usq15, uF, om, ka);
    gx[0] = wm * (W0 * bx - gx[0]);
    gx[1] = wm * (W1 * bx - gx[1]);
    gx[2] = wm * (W1 * (bx - E3) - gx[2]);
    gx[3] = wm * (W1 * bx - gx[3]);
    gx[4] = wm * (W1 * (bx + E3) - gx[4]);
    gy[0] = wm * (W0 * byp - gy[0]);
    gy[1] = wm * (W1 * (byp + E3) - gy[1]);
    gy[2] = wm * (W1 * byp - gy[2]);
    gy[3] = wm * (W1 * (byp - E3) - gy[3]);
    gy[4] = wm * (W1 * byp - gy[4]);
    return;
  } else {
    out[0] = put(collide_f(f[0], w0, C(0), C(0), rhop, rho, ux, uy, usq15, Fx, Fy, uF, om, ka), 0);
    out[1] = put(collide_f(f[1], w1, C(1), C(0), rhop, rho, ux, uy, usq15, Fx, Fy, uF, om, ka), 1);
    out[2] = put(collide_f(f[2], w1, C(0), C(1), rhop, rho, ux, uy, usq15, Fx, Fy, uF, om, ka), 2);
    out[3] = put(collide_f(f[3], w1, C(-1), C(0), rhop, rho, ux, uy, usq15, Fx, Fy, uF, om, ka), 3);
    out[4] = put(collide_f(f[4], w1, C(0), C(-1), rhop, rho, ux, uy, usq15, Fx, Fy, uF, om, ka), 4);
    out[5] = put(collide_f(f[5], w5, C(1), C(1), rhop, rho, ux, uy, usq15, Fx, Fy, uF, om, ka), 5);
    out[6] = put(collide_f(f[6], w5, C(-1), C(1), rhop, rho, ux, uy, usq15, Fx, Fy, uF, om, ka), 6);
    out[7] = put(collide_f(f[7], w5, C(-1), C(-1), rhop, rho, ux, uy, usq15, Fx, Fy, uF, om, ka), 7);
    out[8] = put(collide_f(f[8], w5, C(1), C(-1), rhop, rho, ux, uy, usq15, Fx, Fy, uF, om, ka), 8);

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
}

// ---- binary16 storage with FP32 arithmetic and exact accumulation ----
//
// The stored value of plane q at row y is s = (v - D[y][q]) * 2^12, v the
// post-collision deviation and D the row reference (FP32 values).  Per row
// two more tables describe the pre-collision values a node of that row
// collides with: v_pre[q] = V[y][q] + e[q] 2^-12, where e is the small part
// that varies along the row -- a pulled stored value, or a linear map of
// such values where a Hartmann-wall closure sets the population -- and V
// holds the rest: the reference of the row the population comes from, or
// the closure applied to the references with its constant terms.
// K[y][q] = (V[y][q] - D[y][q]) 2^12 in FP64, so that the new stored value
// of a population with collision increment d is K + e + d 2^12, exactly.
// The collision works in FP32 on V + e 2^-12.  Its increments then have
// their conserved moments restored in FP64 -- zero for mass and for B, the
// total force F for momentum -- and the new stored value is formed in FP64
// before the stochastic rounding.  FP32 rounding then leaves no residual in
// the moments the collision conserves, which the slow modes of a steady
// channel would otherwise integrate step after step; what it leaves in the
// other moments relaxes within a few steps.
struct XTabs {
  float *D;    // row references [ny][kRefRow] (FP32 values)
  double *D64; // the same as doubles (FP64 decoding)
  float *V;    // pre-collision references, FP32
  double *K;   // (V - D) 2^12, FP64
};

__host__ __device__ inline long long xtab_bytes(int ny, int elem) {
  return ((long long)ny * kRefRow * elem + 255) / 256 * 256;
}

__host__ __device__ inline XTabs xtabs_of(void *base, int ny) {
  char *p = static_cast<char *>(base);
  const long long b4 = xtab_bytes(ny, 4), b8 = xtab_bytes(ny, 8);
  return XTabs{reinterpret_cast<float *>(p), reinterpret_cast<double *>(p + b4),
               reinterpret_cast<float *>(p + b4 + b8), reinterpret_cast<double *>(p + 2 * b4 + b8)};
}

__host__ __device__ inline long long xtabs_total_bytes(int ny) {
  return 2 * xtab_bytes(ny, 4) + 2 * xtab_bytes(ny, 8);
}

// The precision mode that works this way: binary16 storage, FP32 compute.
template <typename S, typename C>
constexpr bool kXA = sizeof(S) == 2 && sizeof(C) == 4;

// Pre-collision tables of one row y (FP64 arithmetic on the references).
// Pulled planes take the reference of their source row; planes a Hartmann
// closure sets take the closure of the references (moment scheme) or of the
// row's own references (link scheme), with the constant terms.  Planes set by
// the closures that stay in FP32 (cut-distance walls) take the row's own
// reference, K = 0.
template <int BC>
__device__ __forceinline__ void xtab_row(const Geom &g, const Coef<double> &k, XTabs t, int y) {
  const bool lo = (y == 0), hi = (y == g.ny - 1);
  const float *Dy = t.D + (long long)y * kRefRow;
  const float *Dm = lo ? Dy : Dy - kRefRow;
  const float *Dp = hi ? Dy : Dy + kRefRow;
  double v[19];
  // source row of each plane: planes 2, 5, 6, 11, 16 move up (from y - 1),
  // 4, 7, 8, 13, 18 down (from y + 1), the others along the row
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    const bool up = q == 2 || q == 5 || q == 6 || q == 11 || q == 16;
    const bool dn = q == 4 || q == 7 || q == 8 || q == 13 || q == 18;
    v[q] = (double)(up ? Dm[q] : (dn ? Dp[q] : Dy[q]));
  }
  if constexpr (wall_of(BC) == BC_LINK && cut_of(BC)) {
    // set in FP32 by the cut-distance closure: e = (v - V) 2^12 with V = D
    if (lo) {
      const int cl[5] = {2, 5, 6, 11, 16};
#pragma unroll
      for (int j = 0; j < 5; ++j) v[cl[j]] = (double)Dy[cl[j]];
    }
    if (hi) {
      const int cl[5] = {4, 7, 8, 13, 18};
#pragma unroll
      for (int j = 0; j < 5; ++j) v[cl[j]] = (double)Dy[cl[j]];
    }
  } else if (lo || hi) {
    double f[9], gx[5], gy[5];
#pragma unroll
    for (int q = 0; q < 9; ++q) f[q] = v[q];
#pragma unroll
    for (int q = 0; q < 5; ++q) gx[q] = v[9 + q], gy[q] = v[14 + q];
    const int p0 = lo ? 4 : 2, p1 = lo ? 7 : 5, p2 = lo ? 8 : 6;
    const double own[5] = {(double)Dy[p0], (double)Dy[p1], (double)Dy[p2], (double)Dy[9 + p0],
                           (double)Dy[14 + p0]};
    hartmann_closure<double, wall_of(BC), true>(lo, hi, f, gx, gy, own, k.lo, k.hi);
#pragma unroll
    for (int q = 0; q < 9; ++q) v[q] = f[q];
#pragma unroll
    for (int q = 0; q < 5; ++q) v[9 + q] = gx[q], v[14 + q] = gy[q];
  }
  const long long r = (long long)y * kRefRow;
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    t.V[r + q] = (float)v[q];
    t.D64[r + q] = (double)Dy[q];
    // pulled planes (and FP32-closed ones) have V = a reference, exact in
    // FP32; a Hartmann closure's V keeps its FP64 value in K
    t.K[r + q] = (v[q] - (double)Dy[q]) * kStoreUp16;
  }
  t.V[r + 19] = 0.0f;
  t.D64[r + 19] = 0.0;
  t.K[r + 19] = 0.0;
}

// Collide one node of a binary16 state in FP32 with exact accumulation.
// raw[] holds the 19 pulled stored values (unused where a wall closes the
// population); not for MODE_MOMENTS, which this path does not serve.
// Vy and Ky are row y's entries of t.V and t.K, or a copy of them (the
// batched kernel stages the rows of a tile in LDS).
// The new values before their rounding to binary16 go to emit(q, z_q), in
// plane order; the caller rounds and stores them (stochastically, with the
// node's F16Words in that order).
template <typename S, int BC, int MODE, typename Emit>
__device__ __forceinline__ void node_finish_x(const Geom &g, const Coef<float> &k,
                                              const S *__restrict__ src, XTabs t,
                                              const float *__restrict__ Vy,
                                              const double *__restrict__ Ky, int x, int y,
                                              const S (&raw)[19], NodeObs<float> &obs,
                                              Emit &&emit) {
  static_assert(MODE != MODE_MOMENTS, "observables decode in FP64");
  const bool lo = (y == 0), hi = (y == g.ny - 1);
  const float *__restrict__ Dy = t.D + (long long)y * kRefRow;
  constexpr float up = float(kStoreUp16);
  // the scales as vector registers: a VALU instruction reads at most one
  // scalar register or literal, and the row tables are scalar where the row
  // is uniform
  float down = float(kStoreDown16);
  asm volatile("" : "+v"(down));
  // small parts in stored units (x 2^12)
  float e[19];
#pragma unroll
  for (int q = 0; q < 19; ++q) e[q] = (float)raw[q];
  float f[9], gx[5], gy[5];
#pragma unroll
  for (int q = 0; q < 9; ++q) f[q] = __builtin_fmaf(e[q], down, Vy[q]);
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    gx[q] = __builtin_fmaf(e[9 + q], down, Vy[9 + q]);
    gy[q] = __builtin_fmaf(e[14 + q], down, Vy[14 + q]);
  }
  // closures kept in FP32 (enclosure walls, cut-distance walls): e = (v - V)
  // 2^12 for the populations they set (exact: v and V are close)
  if constexpr (xwalls_of(BC)) {
    if (x == 0 || x == g.nx - 1) {
      xwall_closure<S, float>(g, k, src, Dy, x, y, f, gx, gy);
      if (x == 0) {
        e[1] = (f[1] - Vy[1]) * up, e[5] = (f[5] - Vy[5]) * up, e[8] = (f[8] - Vy[8]) * up;
        e[10] = (gx[1] - Vy[10]) * up, e[15] = (gy[1] - Vy[15]) * up;
      }
      if (x == g.nx - 1) {
        e[3] = (f[3] - Vy[3]) * up, e[6] = (f[6] - Vy[6]) * up, e[7] = (f[7] - Vy[7]) * up;
        e[12] = (gx[3] - Vy[12]) * up, e[17] = (gy[3] - Vy[17]) * up;
      }
    }
  }
  // (each wall written out with its own constant plane numbers, so that
  // the arrays stay in registers)
  auto wall_rows = [&](auto low) {
    constexpr bool L = decltype(low)::value;
    constexpr int a0 = L ? 2 : 4, a1 = L ? 5 : 8, a2 = L ? 6 : 7; // entering planes
    if constexpr (wall_of(BC) == BC_LINK && cut_of(BC)) {
      cut_closure<S, float>(g, k, src, t.D, x, y, f, gx, gy);
      e[a0] = (f[a0] - Vy[a0]) * up, e[a1] = (f[a1] - Vy[a1]) * up, e[a2] = (f[a2] - Vy[a2]) * up;
      e[9 + a0] = (gx[a0] - Vy[9 + a0]) * up, e[14 + a0] = (gy[a0] - Vy[14 + a0]) * up;
    } else {
      // Hartmann walls: the closure's linear part on the small parts e; V
      // holds the closure of the references with its constants
      float ef[9], egx[5], egy[5], own[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < 9; ++q) ef[q] = e[q];
#pragma unroll
      for (int q = 0; q < 5; ++q) egx[q] = e[9 + q], egy[q] = e[14 + q];
      if constexpr (wall_of(BC) == BC_LINK) {
        const long long P = g.plane, r0 = (long long)y * g.pitch;
        constexpr int p0 = L ? 4 : 2, p1 = L ? 7 : 5, p2 = L ? 8 : 6; // leaving planes
        own[0] = ld<S, float>(src + p0 * P + r0 + x);
        own[1] = ld<S, float>(src + p1 * P + r0 + x);
        own[2] = ld<S, float>(src + p2 * P + r0 + x);
        own[3] = ld<S, float>(src + (9 + p0) * P + r0 + x);
        own[4] = ld<S, float>(src + (14 + p0) * P + r0 + x);
      }
      hartmann_closure<float, wall_of(BC), false>(L, !L, ef, egx, egy, own, k.lo, k.hi);
      e[a0] = ef[a0], e[a1] = ef[a1], e[a2] = ef[a2];
      e[9 + a0] = egx[a0], e[14 + a0] = egy[a0];
      f[a0] = __builtin_fmaf(e[a0], down, Vy[a0]);
      f[a1] = __builtin_fmaf(e[a1], down, Vy[a1]);
      f[a2] = __builtin_fmaf(e[a2], down, Vy[a2]);
      gx[a0] = __builtin_fmaf(e[9 + a0], down, Vy[9 + a0]);
      gy[a0] = __builtin_fmaf(e[14 + a0], down, Vy[14 + a0]);
    }
  };
  if (lo) wall_rows(std::true_type{});
  else if (hi) wall_rows(std::false_type{});
  S unused[19];
  // (k's relaxation coefficients carry the factor 2^12 of the stored units,
  // so the increments come back in stored units)
  node_finish<S, float, BC, MODE, false, true>(g, k, src, t.D, x, y, f, gx, gy, obs, 0u, unused);
  // conserved moments of the increments, in FP64: mass and B are unchanged
  // by the collision and momentum gains the force
  double d[19];
#pragma unroll
  for (int q = 0; q < 9; ++q) d[q] = (double)f[q];
#pragma unroll
  for (int q = 0; q < 5; ++q) d[9 + q] = (double)gx[q], d[14 + q] = (double)gy[q];
  const double m0 = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
  const double mx = ((d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7])) - (double)(obs.fx * up);
  const double my = ((d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8])) - (double)(obs.fy * up);
  const double sx = (d[9] + d[10]) + (d[11] + d[12]) + d[13];
  const double sy = (d[14] + d[15]) + (d[16] + d[17]) + d[18];
  // removed on the rest population (mass), on the opposite axis pairs
  // (momentum; their mass and second moments cancel) and on the rest
  // populations of g (B)
  d[0] -= m0;
  d[1] -= 0.5 * mx, d[3] += 0.5 * mx;
  d[2] -= 0.5 * my, d[4] += 0.5 * my;
  d[9] -= sx;
  d[14] -= sy;
  // new stored values (K + d) + e: K and d cancel to about the size of the
  // stored values, exactly in FP64; that difference and then its sum with e
  // round in binary32 at the stored values' own magnitude, before the
  // stochastic rounding to binary16, two at a time
  // Planes pulled along the row (no y component: 0, 1, 3 of f, 0, 1, 3 of
  // g_x and g_y) have K = 0 in every scheme: their source row is the node's
  // own and no wall closure sets them.
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    const bool along_row = q == 0 || q == 1 || q == 3 || q == 9 || q == 10 || q == 12 ||
                           q == 14 || q == 15 || q == 17;
    emit(q, (along_row ? (float)d[q] : (float)(d[q] + Ky[q])) + e[q]);
  }
}

// STAGED, xV, xK: for binary16 storage with FP32 arithmetic, row y's
// pre-collision tables come from the caller's copy xV, xK (else from ref).
template <typename S, typename C, int BC, int MODE, bool SR, bool STAGED = false>
__device__ __forceinline__ void node_update(const Geom &g, const Coef<C> &k,
                                            const S *__restrict__ src,
                                            const C *__restrict__ ref,
                                            S *__restrict__ dst, int x, int y,
                                            NodeObs<C> &obs, uint32_t sseed,
                                            const float *xV = nullptr,
                                            const double *xK = nullptr) {
  const int nx = g.nx;
  const long long P = g.plane;
  const int xm = (x == 0) ? nx - 1 : x - 1;
  const int xp = (x == nx - 1) ? 0 : x + 1;
  const bool lo = (y == 0);
  const bool hi = (y == g.ny - 1);
  const long long r0 = (long long)y * g.pitch;
  const long long rm = r0 - g.pitch;
  const long long rp = r0 + g.pitch;
  constexpr bool NT = !in_batch(BC) || sizeof(S) == 2;
  // the node's byte offset in a plane for the stores, formed in 32 bits so
  // that it stays their 32-bit vector offset (against a scalar plane base)
  uint32_t so = ((uint32_t)y * (uint32_t)g.pitch + (uint32_t)x) * (uint32_t)sizeof(S);
  asm("" : "+v"(so)); // (kept as one 32-bit value: not re-widened into the address)

  if constexpr (kXA<S, C> && MODE != MODE_MOMENTS) {
    // binary16 with FP32 arithmetic: pull the stored values undecoded.
    // Addresses are a plane's base (uniform) plus a 32-bit offset within the
    // plane, shared by every plane pulled from the same neighbour, so that
    // each load and store takes a scalar base and one vector offset.
    auto pl = [&](int q) -> const char * {
      return reinterpret_cast<const char *>(src + (long long)q * P);
    };
    // element i of a plane, the byte offset kept in 32 bits (planes hold
    // fewer than 2^31 elements)
    auto el = [](const char *plane, uint32_t i) -> gptr<const S> {
      return (gptr<const S>)(plane + (uint32_t)(i * (uint32_t)sizeof(S)));
    };
    auto lu = [&](const char *plane, uint32_t i) -> S {
      if constexpr (NT) return __builtin_nontemporal_load(el(plane, i));
      else return *el(plane, i);
    };
    auto lc = [&](const char *plane, uint32_t i) -> S { return *el(plane, i); };
    const uint32_t c0 = (uint32_t)(r0 + x), cm = (uint32_t)(r0 + xm), cp = (uint32_t)(r0 + xp);
    const uint32_t d0 = (uint32_t)(rm + x), dm = (uint32_t)(rm + xm), dp = (uint32_t)(rm + xp);
    const uint32_t u0 = (uint32_t)(rp + x), um = (uint32_t)(rp + xm), up = (uint32_t)(rp + xp);
    S raw[19];
#pragma unroll
    for (int q = 0; q < 19; ++q) raw[q] = S(0);
    raw[0] = lu(pl(0), c0);
    raw[1] = lc(pl(1), cm);
    raw[3] = lc(pl(3), cp);
    raw[9] = lu(pl(9), c0);
    raw[10] = lc(pl(10), cm);
    raw[12] = lc(pl(12), cp);
    raw[14] = lu(pl(14), c0);
    raw[15] = lc(pl(15), cm);
    raw[17] = lc(pl(17), cp);
    if (!lo) {
      raw[2] = lu(pl(2), d0);
      raw[5] = lc(pl(5), dm);
      raw[6] = lc(pl(6), dp);
      raw[11] = lu(pl(11), d0);
      raw[16] = lu(pl(16), d0);
    }
    if (!hi) {
      raw[4] = lu(pl(4), u0);
      raw[7] = lc(pl(7), up);
      raw[8] = lc(pl(8), um);
      raw[13] = lu(pl(13), u0);
      raw[18] = lu(pl(18), u0);
    }
    S out[19];
    NodeObs<float> &o_ = obs;
    const XTabs t = xtabs_of(const_cast<C *>(ref), g.ny);
    const long long row = (long long)y * kRefRow;
    F16Words ew(SR ? node_seed(sseed, (uint32_t)(y * g.nx + x)) : 0u);
    node_finish_x<S, BC, MODE>(g, k, src, t, STAGED ? xV : t.V + row, STAGED ? xK : t.K + row, x,
                               y, raw, o_, [&](int q, float zq) {
                                 if constexpr (SR) out[q] = sr_f16(zq, ew.word(q));
                                 else out[q] = (S)zq;
                               });
#pragma unroll
    for (int q = 0; q < 19; ++q)
      __builtin_nontemporal_store(out[q],
                                  (gptr<S>)(reinterpret_cast<char *>(sbase(dst + (long long)q * P)) + so));
    return;
  } else {
    // solid bodies: a solid node keeps the rest state (stored deviations
    // zero) and reports rho = 1, u = 0, B = (0, B0), J = 0
    int32_t sid = kSolidFluid;
    if constexpr (solids_of(BC)) {
      sid = k.sidx[(long long)y * g.nx + x];
      if (sid == kSolidNode) {
        obs.rho = C(1);
        obs.rhop = C(0);
        obs.ux = obs.uy = obs.bx = obs.jz = obs.fx = obs.fy = C(0);
        obs.by = k.b0;
        if constexpr (MODE != MODE_MOMENTS) {
          const long long o = r0 + x;
#pragma unroll
          for (int q = 0; q < 19; ++q) st<S, S>(dst + q * P + o, S(0));
        }
        return;
      }
    }
    // ---- pull streaming: f_a(x) = f~_a(x - e_a) ----
    // stored values are decoded with the reference of the row they come from
    const C *__restrict__ Dy = ref + (long long)y * kRefRow;
    const C *__restrict__ Dm = lo ? Dy : Dy - kRefRow; // row y - 1 (used only off the lower wall)
    const C *__restrict__ Dp = hi ? Dy : Dy + kRefRow; // row y + 1 (used only off the upper wall)
    // a plane's (uniform) base and a 32-bit element offset within it, as in
    // the branch above (planes hold fewer than 2^31 / 19 elements of at most
    // 8 bytes)
    auto at = [&](int q, uint32_t i) -> const S * {
      return reinterpret_cast<const S *>(reinterpret_cast<const char *>(src + (long long)q * P) +
                                         (uint32_t)(i * (uint32_t)sizeof(S)));
    };
    const uint32_t c0 = (uint32_t)(r0 + x), cm = (uint32_t)(r0 + xm), cp = (uint32_t)(r0 + xp);
    const uint32_t d0 = (uint32_t)(rm + x), dm = (uint32_t)(rm + xm), dp = (uint32_t)(rm + xp);
    const uint32_t u0 = (uint32_t)(rp + x), um = (uint32_t)(rp + xm), up = (uint32_t)(rp + xp);
    C f[9], gx[5], gy[5];
    f[0] = dec<S>(ld<S, C, NT>(at(0, c0)), Dy, 0);
    f[1] = dec<S>(ldx<S, C>(at(1, cm)), Dy, 1);
    f[3] = dec<S>(ldx<S, C>(at(3, cp)), Dy, 3);
    gx[0] = dec<S>(ld<S, C, NT>(at(9, c0)), Dy, 9);
    gx[1] = dec<S>(ldx<S, C>(at(10, cm)), Dy, 10);
    gx[3] = dec<S>(ldx<S, C>(at(12, cp)), Dy, 12);
    gy[0] = dec<S>(ld<S, C, NT>(at(14, c0)), Dy, 14);
    gy[1] = dec<S>(ldx<S, C>(at(15, cm)), Dy, 15);
    gy[3] = dec<S>(ldx<S, C>(at(17, cp)), Dy, 17);
    if (!lo) {
      f[2] = dec<S>(ld<S, C, NT>(at(2, d0)), Dm, 2);
      f[5] = dec<S>(ldx<S, C>(at(5, dm)), Dm, 5);
      f[6] = dec<S>(ldx<S, C>(at(6, dp)), Dm, 6);
      gx[2] = dec<S>(ld<S, C, NT>(at(11, d0)), Dm, 11);
      gy[2] = dec<S>(ld<S, C, NT>(at(16, d0)), Dm, 16);
    }
    if (!hi) {
      f[4] = dec<S>(ld<S, C, NT>(at(4, u0)), Dp, 4);
      f[7] = dec<S>(ldx<S, C>(at(7, up)), Dp, 7);
      f[8] = dec<S>(ldx<S, C>(at(8, um)), Dp, 8);
      gx[4] = dec<S>(ld<S, C, NT>(at(13, u0)), Dp, 13);
      gy[4] = dec<S>(ld<S, C, NT>(at(18, u0)), Dp, 18);
    }

    if constexpr (solids_of(BC))
      if (sid >= 0) solid_closure<S, C>(g, k.snode[sid], src, ref, x, y, f, gx, gy);
    NodeObs<C> &o_ = obs;
    S out[19];
    node_finish<S, C, BC, MODE, SR>(g, k, src, ref, x, y, f, gx, gy, o_, sseed, out);
    if constexpr (MODE != MODE_MOMENTS) {
#pragma unroll
      for (int q = 0; q < 19; ++q)
        st<S, S>(reinterpret_cast<S *>(reinterpret_cast<char *>(sbase(dst + (long long)q * P)) + so),
                 out[q]);
    } else {
      (void)dst;
    }
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
