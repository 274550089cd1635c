// Host-side helpers shared by the single-channel and batched entry points:
// thread-local error reporting, HIP error checks, parameter validation and
// derivation, and the FP64 wall-closure coefficients.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "lks_mhd.h"
#include "lks_node.hpp"

namespace lks {

void set_error(const char *fmt, ...);
void clear_error();

#define LKS_HIP_CHECK(call)                                                   \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) {                                                   \
      ::lks::set_error("%s failed: %s", #call, hipGetErrorString(e_));        \
      return LKS_EDEVICE;                                                     \
    }                                                                         \
  } while (0)

// Validated parameter set with the derived lattice quantities.
struct Channel {
  lks_mhd_params p;
  lks_mhd_derived d;
};

// Validate and derive; LKS_OK or LKS_EINVAL with a message.
int derive_channel(const lks_mhd_params *p, Channel *out);

// FP64 closure coefficients of both walls (see Wall<C> in lks_node.hpp).
struct WallD {
  double r, s, t, u, uw6;
};
void wall_coefficients(const Channel &c, WallD *lo, WallD *hi);

// inc_scale multiplies the coefficients that only ever scale collision
// increments (relaxation rates and source weights): the FP32-arithmetic
// binary16 mode takes its increments in stored units (x 2^12); a power of
// two changes no rounding.
template <typename C>
Coef<C> make_coef(const Channel &c, double inc_scale = 1.0) {
  WallD lo, hi;
  wall_coefficients(c, &lo, &hi);
  Coef<C> k;
  k.sidx = nullptr; // solid-body tables: set where a channel's memory is laid out
  k.snode = nullptr;
  const double sc = inc_scale;
  k.omega_f = C(sc * (1.0 / c.p.tau_f));
  k.kappa_f = C(sc * (1.0 - 0.5 / c.p.tau_f));
  k.omega_m = C(sc * (1.0 / c.p.tau_m));
  k.k_m = C(3.0 / c.p.tau_m);
  k.b0 = C(c.d.b0);
  k.fex = C(c.d.fx);
  k.fey = C(c.d.fy);
  k.lo = Wall<C>{C(lo.r), C(lo.s), C(lo.t), C(lo.u), C(lo.uw6)};
  k.hi = Wall<C>{C(hi.r), C(hi.s), C(hi.t), C(hi.u), C(hi.uw6)};
  // TRT pair coefficients (Trt<C>); under BGK they describe the same
  // operator (pb = sb = 0) and go unused
  // (MRT: the TRT step its corrections start from, odd rate s_fq for f and
  // even rate s_me for g; under BGK and TRT these are 1/tau_f_odd, 1/tau_m_even)
  const double fp = 1.0 / c.p.tau_f, fm = c.d.s_fq;
  const double gp = c.d.s_me, gm = 1.0 / c.p.tau_m;
  const double fa = 0.5 * (fp + fm), fb = 0.5 * (fp - fm);
  k.trt = Trt<C>{C(sc * fa), C(sc * fb), C(sc * (1.0 - 0.5 * fa)), C(sc * (-0.5 * fb)),
                 C(sc * (0.5 * (gp + gm))), C(sc * (0.5 * (gp - gm))), C(sc * gp)};
  // MRT corrections on top of that TRT step (Mrt<C>)
  k.mrt = Mrt<C>{C(sc * ((c.d.s_fe - fp) / 36.0)),    C(sc * ((c.d.s_feps - fp) / 36.0)),
                 C(sc * ((c.d.s_md - c.d.s_me) / 4.0)), C(sc * ((c.d.s_fe - fp) / 2394.0)),
                 C(sc * ((c.d.s_feps - fp) / 252.0)),  C(sc * ((c.d.s_feps - fp) / 72.0)),
                 C(sc * ((c.d.s_feps - fp) / 24.0))};
  k.mrt_on = c.p.collision == LKS_MRT ? 1 : 0;
  // enclosure walls: r = (theta-1)/(theta+1), theta = c a / (tau_m - 1/2)
  auto xr = [&](double cw) {
    if (std::isinf(cw)) return 1.0;
    const double th = cw * c.d.a / (c.p.tau_m - 0.5);
    return (th - 1.0) / (th + 1.0);
  };
  k.xr_lo = C(c.p.x_walls ? xr(c.p.c_x_lower) : 1.0);
  k.xr_hi = C(c.p.x_walls ? xr(c.p.c_x_upper) : 1.0);
  // Hartmann walls at cut distances (Cut<C>)
  auto cut = [&](double q, double cw, double U, int s) {
    const bool near = q < 0.5;
    const double tau = c.p.tau_m;
    const double r = std::isinf(cw) ? 1.0 : (cw * c.d.a + q - tau) / (cw * c.d.a + q + tau - 1.0);
    const double b0c = 0.5 * q * q + (tau - 1.0) * q;
    const double btc = 0.5 * (1.0 - q) * (1.0 - q) + (tau - 1.0) * (1.0 - q);
    const double kk = 0.125 + 0.5 * (tau - 1.0);
    Cut<C> o;
    o.near = near ? 1 : 0;
    o.conducting = cw > 0.0 ? 1 : 0;
    o.fa = C(near ? 2.0 * q : 0.5 / q);
    o.fb = C(near ? 1.0 - 2.0 * q : 1.0 - 0.5 / q);
    o.lscale = C(near ? 1.0 : 0.5 / q);
    o.za = C(near ? -2.0 * q : -0.5 / q);
    o.zb = C(near ? 2.0 * q - 1.0 : 1.0 - 0.5 / q);
    o.r = C(r);
    o.kappa = C(btc - r * b0c - (1.0 - r) * kk);
    // W (e_y / cs2m) B0 = s B0 / 2 for the incoming D2Q5 link
    o.tmove = C(-(1.0 + r) * 0.5 * s * c.d.b0 * U);
    o.tshear = C((0.5 - q) * (1.0 + r) * 0.5 * s * c.d.b0 / q);
    o.u = C(U);
    return o;
  };
  k.clo = cut(c.p.q_lower, c.p.c_lower, c.p.u_lower, +1);
  k.chi = cut(c.p.q_upper, c.p.c_upper, c.p.u_upper, -1);
  return k;
}

// The kernels' scheme parameter of a channel: wall scheme | collision.
inline int scheme_of(const lks_mhd_params &p) {
  return (p.bc == LKS_BC_LINK ? BC_LINK : BC_MOMENT) | (p.collision == LKS_TRT ? COLL_TRT : 0) |
         (p.collision == LKS_MRT ? COLL_MRT : 0) |
         (p.x_walls ? WALLS_X : 0) | ((p.q_lower != 0.5 || p.q_upper != 0.5) ? WALLS_Q : 0) |
         (p.nsolids > 0 ? SOLIDS : 0);
}

inline bool valid_precision(int precision) {
  return precision >= LKS_FP64 && precision <= LKS_FP16_STORE_F64;
}

inline bool is_binary16(int precision) {
  return precision == LKS_FP16_STORE || precision == LKS_FP16_STORE_F64;
}

inline size_t elem_bytes(int precision) {
  return precision == LKS_FP64 ? 8 : (precision == LKS_FP32 ? 4 : 2);
}

// Storage type S and compute type C of a precision mode.
template <typename S_, typename C_> struct Types {
  using S = S_;
  using C = C_;
};

// Calls f(Types<S, C>{}) for the precision's types.
template <typename F>
decltype(auto) dispatch_precision(int precision, F &&f) {
  switch (precision) {
  case LKS_FP64: return f(Types<double, double>{});
  case LKS_FP32: return f(Types<float, Fp32Compute>{});
  case LKS_FP16_STORE: return f(Types<_Float16, float>{});
  default: return f(Types<_Float16, double>{});
  }
}

// Elements per plane, rounded up so that every plane starts 256-byte aligned.
inline long long plane_elems(int nx, int ny, int precision) {
  const long long n = (long long)nx * ny;
  const long long per256 = 256 / (long long)elem_bytes(precision);
  return (n + per256 - 1) / per256 * per256;
}

inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Bytes added between the planes of a single channel's state.  Planes of a
// power-of-two size (a 4096^2 plane of binary32 is 64 MiB) put the 19
// streams of a block at addresses equal in every low bit; 8448 bytes
// (33 x 256) apart they run 1-2% faster on the 4096^2 step in each storage
// precision (measured; presumably the streams then spread over cache sets
// and memory banks).  Batched channels keep their packed planes.
constexpr long long kPlanePadBytes = 8448;

inline long long single_plane_elems(int nx, int ny, int precision) {
  return plane_elems(nx, ny, precision) + kPlanePadBytes / (long long)elem_bytes(precision);
}

// Device bytes of a channel's row-reference area: the FP32-arithmetic
// binary16 mode keeps its four tables (XTabs), the others one row reference
// of doubles (used by binary16 storage only).
inline size_t ref_area_bytes(int ny, int precision) {
  return precision == LKS_FP16_STORE ? (size_t)xtabs_total_bytes(ny)
                                     : align256((size_t)ny * kRefRow * sizeof(double));
}

} // namespace lks
