// Per-node update of the three-dimensional channel or duct: pull streaming
// of the D3Q19 flow and the three-component D3Q7 field populations,
// Shercliff closures at the Hartmann walls y = 0 and y = ny - 1 (x periodic;
// z periodic, or bounded by side walls in a duct),
// moments, the coupled u/J solve, collision and stochastically rounded store.
//
// Lattices (the three-dimensional extension of Secs. IV and V): D3Q19 with
// weights 1/3, 1/18, 1/36 for f; D3Q7 for each field component with rest
// weight 0 and 1/6 on the six axis links, so that c_sm^2 = 1/3 as in the
// paper's D2Q5 and the e_z sums of a z-invariant state are exactly the
// two-dimensional scheme.  The rest population of g is then identically zero
// and is not stored.
//
// Stored planes (deviations from rest at unit density, B = (0, B0, 0)):
//   0..18   f_q - w_q            D3Q19 (q as in the velocity table below)
//   19..24  g_{a x}               a = +x, +y, -x, -y, +z, -z
//   25..30  g_{a y} - B0/6
//   31..36  g_{a z}
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lks_node.hpp"

namespace lks {

constexpr int kPlanes3 = 37;

// D3Q19: 0 rest; 1..4 = +x, +y, -x, -y; 5..8 = (1,1,0), (-1,1,0), (-1,-1,0),
// (1,-1,0); 9, 10 = +z, -z; 11..14 = (1,0,1), (-1,0,-1), (1,0,-1), (-1,0,1);
// 15..18 = (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1).
struct D3Q19 {
  static constexpr int ex[19] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int ey[19] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int ez[19] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr int opp[19] = {0, 3, 4, 1, 2, 7, 8, 5, 6, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
};
// D3Q7 links without the rest: 0 = +x, 1 = +y, 2 = -x, 3 = -y, 4 = +z, 5 = -z.
struct D3Q6 {
  static constexpr int ex[6] = {1, 0, -1, 0, 0, 0};
  static constexpr int ey[6] = {0, 1, 0, -1, 0, 0};
  static constexpr int ez[6] = {0, 0, 0, 0, 1, -1};
};

template <typename C> struct W3 {
  static constexpr C w(int q) {
    return q == 0 ? C(1) / C(3) : ((q <= 4 || q == 9 || q == 10) ? C(1) / C(18) : C(1) / C(36));
  }
};

// State layout in z slabs: layer z holds its 37 planes of ny * nx values
// one after the other, each starting on a 256-byte boundary (slab
// elements apart), so value (q, z, y, x) sits at
//   (z * 37 + q) * slab + y * nx + x.
// A block's 37 streams then fall into three neighbouring layers rather than
// across 37 planes of the whole volume.
struct Geom3 {
  int nx, ny, nz;
  long long slab; // elements from one (layer, plane) to the next
  int side;       // 1: side walls bound z (a duct), 0: z periodic
};

__host__ __device__ inline long long at3(const Geom3 &g, int q, long long node) {
  const long long layer = (long long)g.nx * g.ny;
  const long long z = node / layer;
  return (z * kPlanes3 + q) * g.slab + (node - z * layer);
}

// Side-wall closure coefficients of a duct: g_in,i = r g~_out,i for the
// tangential induced components (x, and y as stored minus W B0), for the
// z = 0 side (lo) and the z = nz-1 side (hi); r = (theta-1)/(theta+1).
template <typename C> struct Side3 {
  C r_lo, r_hi;
};

struct NodeObs3 {
  double rhop, ux, uy, uz, bx, by, bz, jx, jy, jz;
};

// Even rows of the D3Q19 MRT basis (three-dimensional Mrt corrections).
constexpr int mrt3_e2(int q) { return D3Q19::ex[q] * D3Q19::ex[q] + D3Q19::ey[q] * D3Q19::ey[q] + D3Q19::ez[q] * D3Q19::ez[q]; }
constexpr int mrt3_e(int q) { return 19 * mrt3_e2(q) - 30; }
constexpr int mrt3_eps(int q) { return (21 * mrt3_e2(q) * mrt3_e2(q) - 53 * mrt3_e2(q) + 24) / 2; }
constexpr int mrt3_pixx(int q) {
  return (3 * mrt3_e2(q) - 5) * (3 * D3Q19::ex[q] * D3Q19::ex[q] - mrt3_e2(q));
}
constexpr int mrt3_piww(int q) {
  return (3 * mrt3_e2(q) - 5) * (D3Q19::ey[q] * D3Q19::ey[q] - D3Q19::ez[q] * D3Q19::ez[q]);
}

// Interior rows (no wall closure): the kernel for the rows 1..ny-2 keeps the
// pulled values in the storage type and widens them at use, which halves the
// registers they take in FP32 storage (the step is occupancy-bound).
constexpr int BC_NONE = 2;

template <typename S, typename C, int BC, int MODE, bool SR>
__device__ __forceinline__ void node3_update(const Geom3 &g, const Coef<C> &k, C fez,
                                             const Side3<C> &sw, const S *__restrict__ src,
                                             S *__restrict__ dst, int x, int y, int z,
                                             NodeObs3 &obs, uint32_t sseed) {
  // BC: the wall scheme (BC_NONE for interior rows), optionally | COLL_TRT
  constexpr int WB = wall_of(BC);
  // register type of the pulled values
  using R = typename ComputeSel<(WB != BC_NONE && sizeof(C) == 8) || sizeof(S) == 8>::type;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const bool lo = (WB != BC_NONE) && (y == 0), hi = (WB != BC_NONE) && (y == ny - 1);
  const int xs[3] = {x == 0 ? nx - 1 : x - 1, x, x == nx - 1 ? 0 : x + 1}; // x - e for e = 1, 0, -1
  const int zs[3] = {z == 0 ? nz - 1 : z - 1, z, z == nz - 1 ? 0 : z + 1};
  const uint32_t own = ((uint32_t)z * (uint32_t)ny + (uint32_t)y) * (uint32_t)nx + (uint32_t)x;
  // Addresses: the base of a (layer, plane), uniform over the block and
  // pinned in scalar registers, plus a 32-bit byte offset in it (a layer's
  // plane holds fewer than 2^32 bytes), so that every access takes the
  // scalar-base + 32-bit vector-offset form instead of a 64-bit vector
  // address per plane.  The store offset, shared by every plane, is kept as
  // one 32-bit value (the empty register constraint).
  auto base = [&](auto *p, int zz, int q) {
    return sbase(p + ((long long)zz * kPlanes3 + q) * g.slab);
  };
  // population q arriving along e from layer zs[1 - ez] (pull: from x - e)
  auto in_ = [&](int q, int ez_, uint32_t b) {
    return reinterpret_cast<const S *>(reinterpret_cast<const char *>(base(src, zs[1 - ez_], q)) +
                                       b);
  };
  uint32_t own_b = ((uint32_t)y * (uint32_t)nx + (uint32_t)x) * (uint32_t)sizeof(S);
  asm("" : "+v"(own_b));
  // in-layer byte offset of the source of a population moving along e
  auto srcoff = [&](int ex_, int ey_) -> uint32_t {
    return ((uint32_t)(y - ey_) * (uint32_t)nx + (uint32_t)xs[1 - ex_]) * (uint32_t)sizeof(S);
  };

  // ---- pull streaming; populations entering from a wall are closed below ----
  R f[19], gx[6], gy[6], gz[6];
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    const int ey_ = D3Q19::ey[q];
    if ((ey_ == 1 && lo) || (ey_ == -1 && hi)) {
      f[q] = R(0);
      continue;
    }
    const S *p = in_(q, D3Q19::ez[q], srcoff(D3Q19::ex[q], ey_));
    f[q] = D3Q19::ex[q] != 0 ? ldx<S, R>(p) : ld<S, R>(p);
  }
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    const int ey_ = D3Q6::ey[a];
    if ((ey_ == 1 && lo) || (ey_ == -1 && hi)) {
      gx[a] = gy[a] = gz[a] = R(0);
      continue;
    }
    const uint32_t o = srcoff(D3Q6::ex[a], ey_);
    const int ez_ = D3Q6::ez[a];
    if (D3Q6::ex[a] != 0) {
      gx[a] = ldx<S, R>(in_(19 + a, ez_, o));
      gy[a] = ldx<S, R>(in_(25 + a, ez_, o));
      gz[a] = ldx<S, R>(in_(31 + a, ez_, o));
    } else {
      gx[a] = ld<S, R>(in_(19 + a, ez_, o));
      gy[a] = ld<S, R>(in_(25 + a, ez_, o));
      gz[a] = ld<S, R>(in_(31 + a, ez_, o));
    }
  }

  // ---- wall closures ----
  if constexpr (WB == BC_LINK) {
    // Half-way bounce-back with Ladd's term (+-U/6 on the in-plane diagonals);
    // tangential field components by the theta-weighted Shercliff closure
    // (moving-wall term on B_x only), the normal one by anti-bounce-back,
    // all from the node's own post-collision values.
    auto own_ = [&](int plane) { return ld<S, C>(in_(plane, 0, own_b)); };
    if (lo) {
      f[2] = own_(4);
      f[5] = own_(7) + k.lo.uw6;
      f[6] = own_(8) - k.lo.uw6;
      f[15] = own_(16);
      f[17] = own_(18);
      gx[1] = k.lo.r * own_(19 + 3) + k.lo.t;
      gz[1] = k.lo.r * own_(31 + 3);
      gy[1] = -own_(25 + 3);
    }
    if (hi) {
      f[4] = own_(2);
      f[7] = own_(5) - k.hi.uw6;
      f[8] = own_(6) + k.hi.uw6;
      f[16] = own_(15);
      f[18] = own_(17);
      gx[3] = k.hi.r * own_(19 + 1) + k.hi.t;
      gz[3] = k.hi.r * own_(31 + 1);
      gy[3] = -own_(25 + 1);
    }
    // Side walls of a duct (stationary): bounce-back of f, theta closure of
    // the induced tangential components b_x and b_y, anti-bounce-back of
    // B_z.  The values pulled across the wall (periodic addresses) are
    // replaced here; at an edge the links crossing both walls get the same
    // bounce-back value from either closure.
    if (g.side && z == 0) {
      f[9] = own_(10);
      f[11] = own_(12);
      f[14] = own_(13);
      f[15] = own_(16);
      f[18] = own_(17);
      gx[4] = sw.r_lo * own_(19 + 5);
      gy[4] = sw.r_lo * own_(25 + 5);
      gz[4] = -own_(31 + 5);
    }
    if (g.side && z == nz - 1) {
      f[10] = own_(9);
      f[12] = own_(11);
      f[13] = own_(14);
      f[16] = own_(15);
      f[17] = own_(18);
      gx[5] = sw.r_hi * own_(19 + 4);
      gy[5] = sw.r_hi * own_(25 + 4);
      gz[5] = -own_(31 + 4);
    }
  } else if constexpr (WB == BC_MOMENT) {
    // On-node closures from the paper's constraint set taken per tangential
    // direction (Pi_y = 0 fixes rho; Pi_x = rho U, Pi_xx = rho (cs2 + U^2),
    // Pi_z = 0, Pi_zz = rho cs2), written for the deviations f' = f - w.
    if (lo || hi) {
      const int s = lo ? 1 : -1; // e_y of the unknowns
      const C U = lo ? k.lo.u : k.hi.u;
      // known sums (unknowns hold zero)
      C k0 = C(0), kout = C(0), px = C(0), pxx = C(0), pz = C(0), pzz = C(0);
#pragma unroll
      for (int q = 0; q < 19; ++q) {
        if (D3Q19::ey[q] == s) continue;
        if (D3Q19::ey[q] == 0) k0 += f[q];
        else kout += f[q];
        px += C(D3Q19::ex[q]) * f[q];
        pxx += C(D3Q19::ex[q] * D3Q19::ex[q]) * f[q];
        pz += C(D3Q19::ez[q]) * f[q];
        pzz += C(D3Q19::ez[q] * D3Q19::ez[q]) * f[q];
      }
      const C rhop = k0 + C(2) * kout;
      const C sx = (C(1) + rhop) * U - px;
      const C sxx = rhop * (C(1) / C(3)) + (C(1) + rhop) * U * U - pxx;
      const C sz = -pz;
      const C szz = rhop * (C(1) / C(3)) - pzz;
      // lower: +x (1,1,0) = 5, -x (-1,1,0) = 6, +z (0,1,1) = 15, -z (0,1,-1) = 17, n = 2
      // upper: +x (1,-1,0) = 8, -x (-1,-1,0) = 7, +z (0,-1,1) = 18, -z (0,-1,-1) = 16, n = 4
      const C fxp = C(0.5) * (sxx + sx), fxm = C(0.5) * (sxx - sx);
      const C fzp = C(0.5) * (szz + sz), fzm = C(0.5) * (szz - sz);
      const C fn = kout - (fxp + fxm + fzp + fzm);
      // field: tangential from the discrete Shercliff constraint, normal from
      // sum g_y = B0 (for the deviations: sum g'_y = 0); in = +y link at the
      // lower wall, -y at the upper
      const C ox = gx[0] + gx[2] + gx[4] + gx[5];
      const C oy = gy[0] + gy[2] + gy[4] + gy[5];
      const C oz = gz[0] + gz[2] + gz[4] + gz[5];
      if (lo) {
        f[5] = fxp;
        f[6] = fxm;
        f[15] = fzp;
        f[17] = fzm;
        f[2] = fn;
        gx[1] = k.lo.r * gx[3] - k.lo.s * ox + k.lo.t;
        gz[1] = k.lo.r * gz[3] - k.lo.s * oz;
        gy[1] = -(oy + gy[3]);
      } else {
        f[8] = fxp;
        f[7] = fxm;
        f[18] = fzp;
        f[16] = fzm;
        f[4] = fn;
        gx[3] = k.hi.r * gx[1] - k.hi.s * ox + k.hi.t;
        gz[3] = k.hi.r * gz[1] - k.hi.s * oz;
        gy[3] = -(oy + gy[1]);
      }
    }
  }

  // ---- moments ----
  C rhop = C(0), mx = C(0), my = C(0), mz = C(0);
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    const C v = C(f[q]);
    rhop += v;
    mx += C(D3Q19::ex[q]) * v;
    my += C(D3Q19::ey[q]) * v;
    mz += C(D3Q19::ez[q]) * v;
  }
  const C rho = C(1) + rhop;
  auto G = [](R v) { return C(v); };
  const C bx = ((G(gx[0]) + G(gx[1])) + (G(gx[2]) + G(gx[3]))) + (G(gx[4]) + G(gx[5]));
  const C byp = ((G(gy[0]) + G(gy[1])) + (G(gy[2]) + G(gy[3]))) + (G(gy[4]) + G(gy[5]));
  const C by = k.b0 + byp;
  const C bz = ((G(gz[0]) + G(gz[1])) + (G(gz[2]) + G(gz[3]))) + (G(gz[4]) + G(gz[5]));
  // D = (L_yz - L_zy, L_zx - L_xz, L_xy - L_yx), L_ji = g_{+j,i} - g_{-j,i}
  const C dyz = (G(gz[1]) - G(gz[3])) - (G(gy[4]) - G(gy[5]));
  const C dzx = (G(gx[4]) - G(gx[5])) - (G(gz[0]) - G(gz[2]));
  const C dxy = (G(gy[0]) - G(gy[2])) - (G(gx[1]) - G(gx[3]));

  // ---- coupled local solve ----
  const C kk = k.k_m;
  C ux, uy, uz, jx, jy, jz, Fx, Fy, Fz;
  const C inv_rho = C(1) / rho;
  if (WB == BC_MOMENT && (lo || hi)) {
    // wet wall node: velocity fixed by the closure, no force
    ux = mx * inv_rho;
    uy = my * inv_rho;
    uz = mz * inv_rho;
    jx = -kk * (dyz - C(2) * (uy * bz - uz * by));
    jy = -kk * (dzx - C(2) * (uz * bx - ux * bz));
    jz = -kk * (dxy - C(2) * (ux * by - uy * bx));
    Fx = Fy = Fz = C(0);
  } else {
    // (rho + k|B|^2) J - k B (B.J) = R = k (2 p x B - rho D), p = m + F_ext/2,
    // inverted exactly: J = (R + (k/rho) B (B.R)) / (rho + k|B|^2)
    const C px = mx + C(0.5) * k.fex, py = my + C(0.5) * k.fey, pz = mz + C(0.5) * fez;
    const C Rx = kk * (C(2) * (py * bz - pz * by) - rho * dyz);
    const C Ry = kk * (C(2) * (pz * bx - px * bz) - rho * dzx);
    const C Rz = kk * (C(2) * (px * by - py * bx) - rho * dxy);
    const C bR = (bx * Rx + by * Ry + bz * Rz) * kk * inv_rho;
    const C inv_a = C(1) / (rho + kk * (bx * bx + by * by + bz * bz));
    jx = (Rx + bx * bR) * inv_a;
    jy = (Ry + by * bR) * inv_a;
    jz = (Rz + bz * bR) * inv_a;
    Fx = k.fex + (jy * bz - jz * by);
    Fy = k.fey + (jz * bx - jx * bz);
    Fz = fez + (jx * by - jy * bx);
    ux = (mx + C(0.5) * Fx) * inv_rho;
    uy = (my + C(0.5) * Fy) * inv_rho;
    uz = (mz + C(0.5) * Fz) * inv_rho;
  }
  obs.rhop = (double)rhop;
  obs.ux = (double)ux;
  obs.uy = (double)uy;
  obs.uz = (double)uz;
  obs.bx = (double)bx;
  obs.by = (double)by;
  obs.bz = (double)bz;
  obs.jx = (double)jx;
  obs.jy = (double)jy;
  obs.jz = (double)jz;
  if (MODE == MODE_MOMENTS) return;

  // ---- collide and store ----
  // Widen a pulled value again for its collision: the empty register
  // constraint hides the earlier widening from common-subexpression
  // elimination, so only the narrow value stays live across the solve.
  auto rewiden = [](R v) -> C {
    if constexpr (sizeof(R) < sizeof(C)) asm volatile("" : "+v"(v));
    return C(v);
  };
  Rng rng(SR ? node_seed(sseed, (uint32_t)own) : 0u);
  auto put = [&](int plane, C v) {
    __builtin_nontemporal_store(to_store<S, C, SR>(v, SR ? rng.next() : 0u),
                                (gptr<S>)(reinterpret_cast<char *>(base(dst, z, plane)) + own_b));
  };
  const C om = k.omega_f, ka = k.kappa_f;
  const C usq15 = C(1.5) * (ux * ux + uy * uy + uz * uz);
  const C uF = ux * Fx + uy * Fy + uz * Fz;
  // g^eq_{a i} = W [B_i + 3 e_a (u_a B_i - B_a u_i)] along the link's axis a;
  // the component along the axis keeps W B_a.  Deviations: the y component
  // is stored minus W B0.  (Formed after the f collisions, which keeps them
  // out of the registers live there.)
  struct GEq3 {
    C x[6], y[6], z[6];
  };
  auto geq3 = [&]() -> GEq3 {
    const C W = C(1) / C(6);
    const C exy = C(3) * (ux * by - uy * bx); // u_x B_y - B_x u_y
    const C exz = C(3) * (ux * bz - uz * bx);
    const C eyz = C(3) * (uy * bz - uz * by);
    return GEq3{{W * bx, W * (bx - exy), W * bx, W * (bx + exy), W * (bx - exz), W * (bx + exz)},
                {W * (byp + exy), W * byp, W * (byp - exy), W * byp, W * (byp - eyz), W * (byp + eyz)},
                {W * (bz + exz), W * (bz + eyz), W * (bz - exz), W * (bz - eyz), W * bz, W * bz}};
  };
  if constexpr (trt_of(BC) || mrt_of(BC)) {
    // opposite pairs: D3Q19 (1,3) (2,4) (5,7) (6,8) (9,10) (11,12) (13,14)
    // (15,16) (17,18); D3Q7 links (+x,-x) (+y,-y) (+z,-z)
    const Trt<C> &t = k.trt;
    const C rhop_ = rhop, rho_ = rho, usq15_ = usq15, uF_ = uF;
    const C ux_ = ux, uy_ = uy, uz_ = uz, Fx_ = Fx, Fy_ = Fy, Fz_ = Fz;
    (void)rhop_, (void)rho_, (void)usq15_, (void)uF_, (void)ux_, (void)uy_, (void)uz_;
    (void)Fx_, (void)Fy_, (void)Fz_;
    constexpr int first[9] = {1, 2, 5, 6, 9, 11, 13, 15, 17};
    // MRT: corrections along the even rows e, epsilon, 3pi_xx, pi_ww (Mrt),
    // from the moments of n - S/2 taken in a first pass over the pairs (the
    // two populations of a pair share their even row values); the TRT step
    // then adds them as it stores
    C ce = C(0), cp = C(0), cpx = C(0), cpw = C(0);
    if constexpr (mrt_of(BC)) {
      // opaque copies of the fields: the equilibria and sources of this pass
      // must not be shared with the collision's (kept live in between, they
      // spilled)
      auto opaque = [](C v) -> C {
        asm volatile("" : "+v"(v));
        return v;
      };
      const C rhop = opaque(rhop_), rho = opaque(rho_), usq15 = opaque(usq15_), uF = opaque(uF_);
      const C ux = opaque(ux_), uy = opaque(uy_), uz = opaque(uz_);
      const C Fx = opaque(Fx_), Fy = opaque(Fy_), Fz = opaque(Fz_);
      const C t0 = (W3<C>::w(0) * (rhop - rho * usq15) - rewiden(f[0])) -
                   C(0.5) * (C(3) * W3<C>::w(0) * (-uF) * (C(1) - usq15));
      C te = C(-30) * t0, tp = C(12) * t0, tpx = C(0), tpw = C(0);
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const int q = first[i], r = D3Q19::opp[q];
        const C ex_ = C(D3Q19::ex[q]), ey_ = C(D3Q19::ey[q]), ez_ = C(D3Q19::ez[q]);
        const C w = W3<C>::w(q), eu = ex_ * ux + ey_ * uy + ez_ * uz;
        const C eF = ex_ * Fx + ey_ * Fy + ez_ * Fz;
        const C even = C(4.5) * eu * eu - usq15, odd = C(3) * eu;
        const C pa = even + odd, pb = even - odd;
        const C ts = (w * (rhop + rho * pa) - rewiden(f[q])) + (w * (rhop + rho * pb) - rewiden(f[r])) -
                     C(0.5) * (C(3) * w * (eF - uF) * (C(1) + pa) + C(3) * w * (-eF - uF) * (C(1) + pb));
        te += C(mrt3_e(q)) * ts, tp += C(mrt3_eps(q)) * ts;
        tpx += C(mrt3_pixx(q)) * ts, tpw += C(mrt3_piww(q)) * ts;
      }
      const Mrt<C> &m = k.mrt;
      ce = m.ke3 * te, cp = m.keps3 * tp, cpx = m.kpx3 * tpx, cpw = m.kpw3 * tpw;
      __builtin_amdgcn_sched_barrier(0); // keep the two passes apart
    }
    auto corr = [&](int q) -> C {
      return C(mrt3_e(q)) * ce + C(mrt3_eps(q)) * cp + C(mrt3_pixx(q)) * cpx + C(mrt3_piww(q)) * cpw;
    };
    {
      const C fq = rewiden(f[0]);
      const C feq = W3<C>::w(0) * (rhop - rho * usq15);
      const C src_q = C(3) * W3<C>::w(0) * (-uF) * (C(1) - usq15);
      C v = fq + om * (feq - fq) + ka * src_q;
      if constexpr (mrt_of(BC)) v += corr(0);
      put(0, v);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int q = first[i], r = D3Q19::opp[q];
      const C ex_ = C(D3Q19::ex[q]), ey_ = C(D3Q19::ey[q]), ez_ = C(D3Q19::ez[q]);
      C fa = rewiden(f[q]), fb = rewiden(f[r]);
      collide_f_pair(fa, fb, W3<C>::w(q), ex_ * ux + ey_ * uy + ez_ * uz,
                     ex_ * Fx + ey_ * Fy + ez_ * Fz, rhop, rho, usq15, uF, t);
      if constexpr (mrt_of(BC)) {
        const C cq = corr(q);
        fa += cq, fb += cq;
      }
      put(q, fa);
      put(r, fb);
    }
    const GEq3 ge = geq3();
    constexpr int ga_[3] = {0, 1, 4}, gb_[3] = {2, 3, 5};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int a = ga_[i], b = gb_[i];
      C xa = rewiden(gx[a]), xb = rewiden(gx[b]);
      C ya = rewiden(gy[a]), yb = rewiden(gy[b]);
      C za = rewiden(gz[a]), zb = rewiden(gz[b]);
      collide_g_pair(xa, xb, ge.x[a], ge.x[b], t);
      collide_g_pair(ya, yb, ge.y[a], ge.y[b], t);
      collide_g_pair(za, zb, ge.z[a], ge.z[b], t);
      put(19 + a, xa);
      put(19 + b, xb);
      put(25 + a, ya);
      put(25 + b, yb);
      put(31 + a, za);
      put(31 + b, zb);
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    const C ex_ = C(D3Q19::ex[q]), ey_ = C(D3Q19::ey[q]), ez_ = C(D3Q19::ez[q]);
    const C w = W3<C>::w(q);
    const C eu = ex_ * ux + ey_ * uy + ez_ * uz;
    const C poly = C(3) * eu + C(4.5) * eu * eu - usq15;
    const C feq = w * (rhop + rho * poly);
    const C src_q = C(3) * w * ((ex_ * Fx + ey_ * Fy + ez_ * Fz) - uF) * (C(1) + poly);
    const C fq = rewiden(f[q]);
    put(q, fq + om * (feq - fq) + ka * src_q);
  }
  const C wm = k.omega_m;
  const GEq3 ge = geq3();
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    const C vx = rewiden(gx[a]), vy = rewiden(gy[a]), vz = rewiden(gz[a]);
    put(19 + a, vx + wm * (ge.x[a] - vx));
    put(25 + a, vy + wm * (ge.y[a] - vy));
    put(31 + a, vz + wm * (ge.z[a] - vz));
  }
}

} // namespace lks
