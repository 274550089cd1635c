// Solid bodies in a channel (curved walls): host-side classification of the
// nodes and the per-link closure coefficients the step kernel reads.
//
// A node is solid if it lies strictly inside a body (lks_solid).  A fluid
// node whose population f_a is pulled from a solid node x - e_a has that link
// cut by the body's surface at the fraction q of the link from the node; the
// closure (interpolated bounce-back of f, interpolated anti-bounce-back of g
// with the induced field zero on the surface) is a linear map of the node's
// own post-collision populations and of one neighbour's, with coefficients
// that depend on q only:
//   near (q < 1/2, x + e_a fluid):  h_a = ca o + cb X,  X = h~_abar(x + e_a)
//   far  (q >= 1/2):                h_a = ca o + cb X,  X = h~_a(x)
//   q < 1/2 with x + e_a solid:     half-way bounce-back (ca = 1, cb = 0)
// o = h~_abar(x) the node's own population leaving towards the surface; f
// adds the moving-wall term mw = 2 w_a e_a.u_w / cs2 (scaled by 1/(2q) on the
// far branch), u_w the surface velocity where the link crosses it.
#pragma once

#include <cmath>
#include <cstdint>
#include <vector>

#include "lks_mhd.h"

namespace lks {

// Per-node entry of the solid-body table: kSolidFluid (no link from a solid
// node), kSolidNode (solid), or the index of the node's CurvedNode.
constexpr int32_t kSolidFluid = -1;
constexpr int32_t kSolidNode = -2;

struct CurvedNode {
  uint32_t cut;  // bit a (1..8): f_a (and, for a <= 4, g_a) is pulled from a solid node
  uint32_t near; // bit a: X is the next node into the fluid, else the node's own h_a
  double ca[8], cb[8], mw[8]; // f, link a at index a - 1
  double za[4], zb[4];        // g (both components), link a at index a - 1
};

namespace geom {

constexpr int kEx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kEy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr double kW[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                          1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

// x distance of X from a body's centre, to the nearest periodic image.
inline double wrap_dx(double X, double cx, int nx) {
  const double L = (double)nx, d = X - cx;
  return d - L * std::floor(d / L + 0.5);
}

inline bool in_body(const lks_solid &b, int nx, double X, double Y) {
  if (b.kind == LKS_SOLID_BELOW) return Y < b.cy;
  if (b.kind == LKS_SOLID_ABOVE) return Y > b.cy;
  const double dx = wrap_dx(X, b.cx, nx), dy = Y - b.cy;
  const double d2 = dx * dx + dy * dy;
  return b.kind == LKS_SOLID_DISC ? d2 < b.r * b.r : d2 > b.r * b.r;
}

inline bool solid_at(const lks_mhd_params &p, double X, double Y) {
  for (int k = 0; k < p.nsolids; ++k)
    if (in_body(p.solids[k], p.nx, X, Y)) return true;
  return false;
}

// Surface crossing on the link from node (x, y) towards (x, y) - e_a, which
// body b contains: the fraction t of the link and the surface velocity there.
inline void crossing(const lks_solid &b, int nx, int x, int y, int a, double *t, double *ux,
                     double *uy) {
  const double ex = kEx[a], ey = kEy[a];
  if (b.kind == LKS_SOLID_BELOW || b.kind == LKS_SOLID_ABOVE) {
    *t = ((double)y - b.cy) / ey; // ey != 0: a half-plane is only reached across rows
    *ux = b.u;
    *uy = 0.0;
    return;
  }
  // node at P (relative to the centre), point P - t e on the circle
  const double px = wrap_dx((double)x, b.cx, nx), py = (double)y - b.cy;
  const double ee = ex * ex + ey * ey, pe = px * ex + py * ey;
  const double h = pe * pe - ee * (px * px + py * py - b.r * b.r);
  const double root = std::sqrt(h > 0.0 ? h : 0.0);
  // into a disc the first crossing, out of a bore the second
  *t = (b.kind == LKS_SOLID_DISC ? pe - root : pe + root) / ee;
  const double wx = px - *t * ex, wy = py - *t * ey;
  *ux = -b.omega * wy;
  *uy = b.omega * wx;
}

} // namespace geom

// Classify every node and build the link tables.  idx gets nx * ny entries
// (kSolidFluid, kSolidNode or an index into nodes).  Returns false with a
// message in *why if a node next to a body lies on a Hartmann wall row.
inline bool build_solid_tables(const lks_mhd_params &p, std::vector<int32_t> *idx,
                               std::vector<CurvedNode> *nodes, const char **why) {
  using namespace geom;
  const int nx = p.nx, ny = p.ny;
  idx->assign((size_t)nx * ny, kSolidFluid);
  nodes->clear();
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x)
      if (solid_at(p, x, y)) (*idx)[(size_t)y * nx + x] = kSolidNode;
  auto solid_node = [&](int x, int y) {
    return (*idx)[(size_t)y * nx + (((x % nx) + nx) % nx)] == kSolidNode;
  };
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      if ((*idx)[(size_t)y * nx + x] == kSolidNode) continue;
      CurvedNode cn{};
      for (int a = 1; a < 9; ++a) {
        // upstream point x - e_a (rows beyond the grid count if a body
        // covers them)
        const int uyi = y - kEy[a];
        const bool up_solid = (uyi >= 0 && uyi < ny) ? solid_node(x - kEx[a], uyi)
                                                     : solid_at(p, x - kEx[a], uyi);
        if (!up_solid) continue;
        const double ux = (double)(x - kEx[a]), uy = (double)uyi;
        double q = 2.0, wux = 0.0, wuy = 0.0;
        for (int k = 0; k < p.nsolids; ++k) {
          const lks_solid &b = p.solids[k];
          if (!in_body(b, nx, ux, uy)) continue;
          double t, vx, vy;
          crossing(b, nx, x, y, a, &t, &vx, &vy);
          if (!(t > 0.0)) t = 1e-12; // a node on the surface itself
          if (t > 1.0) t = 1.0;
          if (t < q) q = t, wux = vx, wuy = vy;
        }
        if (q > 1.0) continue;
        cn.cut |= 1u << a;
        const int yn = y + kEy[a];
        const bool near = q < 0.5 && yn >= 0 && yn < ny && !solid_node(x + kEx[a], yn);
        const bool far = q >= 0.5;
        const double m = 6.0 * kW[a] * (kEx[a] * wux + kEy[a] * wuy); // 2 w e.u / cs2
        const int i = a - 1;
        if (near) {
          cn.near |= 1u << a;
          cn.ca[i] = 2.0 * q, cn.cb[i] = 1.0 - 2.0 * q, cn.mw[i] = m;
        } else if (far) {
          cn.ca[i] = 0.5 / q, cn.cb[i] = 1.0 - 0.5 / q, cn.mw[i] = m * 0.5 / q;
        } else {
          cn.ca[i] = 1.0, cn.cb[i] = 0.0, cn.mw[i] = m;
        }
        if (a <= 4) {
          if (near) cn.za[i] = -2.0 * q, cn.zb[i] = 2.0 * q - 1.0;
          else if (far) cn.za[i] = -0.5 / q, cn.zb[i] = 1.0 - 0.5 / q;
          else cn.za[i] = -1.0, cn.zb[i] = 0.0;
        }
      }
      if (!cn.cut) continue;
      if (y == 0 || y == ny - 1) {
        *why = "a node next to a solid body lies on a Hartmann wall row (0 or ny - 1)";
        return false;
      }
      (*idx)[(size_t)y * nx + x] = (int32_t)nodes->size();
      nodes->push_back(cn);
    }
  return true;
}

} // namespace lks
