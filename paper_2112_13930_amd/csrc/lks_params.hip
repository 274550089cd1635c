// Parameter validation and derivation of the lattice quantities (host, FP64).
//
//   nu = cs2 (tau_f - 1/2), eta = cs2m (tau_m - 1/2)           (Secs. IV, V)
//   Ha = B0 a sqrt(sigma / (rho nu)), sigma = 1/(eta mu_m), mu_m = 1  (Sec. VIII)
//   U_ref = a^2 F_x / (rho nu) and the Chang-Lundgren centreline velocity
//   u*(0) = (K/Ha)(1 - 1/cosh Ha), K = (c+1)/(Ha c + tanh Ha)          (Sec. VIII)
//   theta = c_w a / (tau_m - 1/2)                         (Eq. weightingfactor)
//   phi = c_w a / (tau_m cs2m)     (ratio of the two coefficients of Sec. VII)
//   TRT free rates: tau- = 1/2 + Lambda / (tau+ - 1/2) and conversely
//   link walls at cut distances q: a = (ny - 1 + q_lower + q_upper)/2
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "lks_common.hpp"
#include "lks_geometry.hpp"

namespace lks {

static thread_local std::string g_error;

void set_error(const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
}

void clear_error() { g_error.clear(); }

static int bad(const char *msg) {
  set_error("invalid parameters: %s", msg);
  return LKS_EINVAL;
}

static bool finite(double v) { return std::isfinite(v); }

// Centreline velocity of the Chang-Lundgren profile in units of U_ref.
static double cl_centre(double ha, double c) {
  if (ha < 1e-6) return 0.5; // plane Poiseuille limit
  const double K = std::isinf(c) ? 1.0 / ha : (c + 1.0) / (ha * c + std::tanh(ha));
  return (K / ha) * (1.0 - 1.0 / std::cosh(ha));
}

int derive_channel(const lks_mhd_params *p, Channel *out) {
  if (!p) return bad("null parameter pointer");
  if (p->nx < 1) return bad("nx must be >= 1");
  if (p->bc != LKS_BC_LINK && p->bc != LKS_BC_MOMENT) return bad("bc must be LKS_BC_LINK or LKS_BC_MOMENT");
  if (p->ny < (p->bc == LKS_BC_LINK ? 2 : 3)) return bad("ny must be >= 2 (link) or >= 3 (moment)");
  // (19 planes, each padded by up to 8192 values, index in 32 bits)
  if ((long long)p->nx * (long long)p->ny > (long long)(((1LL << 31) - 1) / 19) - 8192)
    return bad("nx * ny too large (19 planes must index in 32 bits)");
  if (!lks::valid_precision(p->precision)) return bad("unknown precision");
  if (!finite(p->tau_f) || p->tau_f <= 0.5) return bad("tau_f must be finite and > 1/2");
  if (!finite(p->tau_m) || p->tau_m <= 0.5) return bad("tau_m must be finite and > 1/2");
  if (std::isnan(p->c_lower) || p->c_lower < 0.0) return bad("c_lower must be in [0, inf]");
  if (std::isnan(p->c_upper) || p->c_upper < 0.0) return bad("c_upper must be in [0, inf]");
  if (!finite(p->u_lower) || !finite(p->u_upper)) return bad("wall velocities must be finite");
  if (!finite(p->rho0) || p->rho0 <= 0.0) return bad("rho0 must be finite and > 0");
  if (!finite(p->fy)) return bad("fy must be finite");
  if (p->collision != LKS_BGK && p->collision != LKS_TRT && p->collision != LKS_MRT)
    return bad("collision must be LKS_BGK, LKS_TRT or LKS_MRT");
  if (p->x_walls != 0 && p->x_walls != 1) return bad("x_walls must be 0 or 1");
  if (p->x_walls) {
    if (p->bc != LKS_BC_LINK) return bad("enclosure walls need link-based closures");
    if (p->nx < 2) return bad("an enclosure needs nx >= 2");
    if (std::isnan(p->c_x_lower) || p->c_x_lower < 0.0 || std::isnan(p->c_x_upper) ||
        p->c_x_upper < 0.0)
      return bad("c_x_lower and c_x_upper must be in [0, inf]");
  }
  if (!(p->q_lower > 0.0 && p->q_lower <= 1.0) || !(p->q_upper > 0.0 && p->q_upper <= 1.0))
    return bad("q_lower and q_upper must be in (0, 1]");
  const bool cut = p->q_lower != 0.5 || p->q_upper != 0.5;
  if (cut) {
    if (p->bc != LKS_BC_LINK) return bad("walls at cut distances need link-based closures");
    if (p->x_walls) return bad("walls at cut distances are not available in enclosures");
    if (p->ny < 3) return bad("walls at cut distances need ny >= 3");
  }
  if (p->nsolids < 0 || p->nsolids > LKS_MAX_SOLIDS) return bad("nsolids must be in [0, 4]");
  if (p->nsolids > 0) {
    for (int k = 0; k < p->nsolids; ++k) {
      const lks_solid &b = p->solids[k];
      if (b.kind < LKS_SOLID_DISC || b.kind > LKS_SOLID_ABOVE) return bad("unknown solid kind");
      if (!finite(b.cx) || !finite(b.cy) || !finite(b.omega) || !finite(b.u))
        return bad("solid body parameters must be finite");
      if ((b.kind == LKS_SOLID_DISC || b.kind == LKS_SOLID_BORE) && !(finite(b.r) && b.r > 0.0))
        return bad("a circle needs a finite radius > 0");
    }
    if (p->precision != LKS_FP64 && p->precision != LKS_FP32)
      return bad("solid bodies need FP64 or FP32 storage");
    if (p->x_walls || cut)
      return bad("solid bodies need an x-periodic channel with half-way Hartmann walls");
    std::vector<int32_t> idx;
    std::vector<CurvedNode> nodes;
    const char *why = nullptr;
    if (!build_solid_tables(*p, &idx, &nodes, &why)) return bad(why);
  }
  if (p->collision != LKS_BGK &&
      (!finite(p->lambda_f) || p->lambda_f <= 0.0 || !finite(p->lambda_m) || p->lambda_m <= 0.0))
    return bad("TRT and MRT need finite lambda_f > 0 and lambda_m > 0");
  if (p->collision == LKS_MRT) {
    auto rate_ok = [](double s, bool nan_ok) { return (nan_ok && std::isnan(s)) || (s > 0.0 && s < 2.0); };
    if (!rate_ok(p->s_fe, false) || !rate_ok(p->s_feps, false) || !rate_ok(p->s_fq, true) ||
        !rate_ok(p->s_me, true) || !rate_ok(p->s_md, true))
      return bad("MRT rates must be in (0, 2) (s_fq, s_me, s_md may be NaN)");
  }

  Channel c;
  c.p = *p;
  lks_mhd_derived &d = c.d;
  d.nu = (p->tau_f - 0.5) / 3.0;
  d.eta = (p->tau_m - 0.5) / 3.0;
  d.a = (p->bc == LKS_BC_LINK) ? 0.5 * (p->ny - 1 + p->q_lower + p->q_upper) : 0.5 * (p->ny - 1);
  if (std::isnan(p->ha)) {
    if (!finite(p->b0)) return bad("b0 must be finite when ha is NaN");
    d.b0 = p->b0;
  } else {
    if (!finite(p->ha) || p->ha < 0.0) return bad("ha must be NaN or finite and >= 0");
    d.b0 = p->ha * std::sqrt(p->rho0 * d.nu * d.eta) / d.a;
    if (!std::isnan(p->b0) && std::fabs(p->b0 - d.b0) > 1e-12 * std::fmax(1.0, std::fabs(d.b0)))
      return bad("ha and b0 are both set and inconsistent");
  }
  if (std::isnan(p->fx)) {
    if (!finite(p->u_max)) return bad("u_max must be finite when fx is NaN");
    if (p->c_lower != p->c_upper)
      return bad("deriving fx from u_max needs equal wall conductance ratios");
    const double ha = std::isnan(p->ha) ? d.b0 * d.a / std::sqrt(p->rho0 * d.nu * d.eta) : p->ha;
    d.fx = p->u_max * p->rho0 * d.nu / (d.a * d.a * cl_centre(ha, p->c_lower));
  } else {
    if (!finite(p->fx)) return bad("fx must be finite or NaN");
    d.fx = p->fx;
  }
  d.fy = p->fy;
  d.theta_lower = std::isinf(p->c_lower) ? INFINITY : p->c_lower * d.a / (p->tau_m - 0.5);
  d.theta_upper = std::isinf(p->c_upper) ? INFINITY : p->c_upper * d.a / (p->tau_m - 0.5);
  d.phi_lower = std::isinf(p->c_lower) ? INFINITY : p->c_lower * d.a * 3.0 / p->tau_m;
  d.phi_upper = std::isinf(p->c_upper) ? INFINITY : p->c_upper * d.a * 3.0 / p->tau_m;
  // a conducting wall at a cut distance: the single-node coefficient
  // (c a + q - tau_m)/(c a + q + tau_m - 1) needs a denominator away from 0
  for (int w = 0; w < 2 && cut; ++w) {
    const double c = w ? p->c_upper : p->c_lower, q = w ? p->q_upper : p->q_lower;
    if (c > 0.0 && std::isfinite(c) && c * d.a + q + p->tau_m - 1.0 < 0.25)
      return bad("a conducting wall at cut distance q needs c a + q + tau_m - 1 >= 1/4");
  }
  // TRT: the free rate of each distribution from its magic parameter
  // Lambda = (tau+ - 1/2)(tau- - 1/2)
  if (p->collision != LKS_BGK) {
    d.tau_f_odd = 0.5 + p->lambda_f / (p->tau_f - 0.5);
    d.tau_m_even = 0.5 + p->lambda_m / (p->tau_m - 0.5);
  } else {
    d.tau_f_odd = p->tau_f;
    d.tau_m_even = p->tau_m;
  }
  // MRT rates in use; under BGK and TRT the ones those operators amount to
  if (p->collision == LKS_MRT) {
    d.s_fe = p->s_fe;
    d.s_feps = p->s_feps;
    d.s_fq = std::isnan(p->s_fq) ? 1.0 / d.tau_f_odd : p->s_fq;
    d.s_me = std::isnan(p->s_me) ? 1.0 / d.tau_m_even : p->s_me;
    d.s_md = std::isnan(p->s_md) ? 1.0 / d.tau_m_even : p->s_md;
  } else {
    d.s_fe = d.s_feps = 1.0 / p->tau_f;
    d.s_fq = 1.0 / d.tau_f_odd;
    d.s_me = d.s_md = 1.0 / d.tau_m_even;
  }
  if (out) *out = c;
  return LKS_OK;
}

// (x - 1)/(x + 1), 1/(x + 1), x/(x + 1) for x in [0, inf].
static void ratio3(double x, double *rm, double *inv, double *frac) {
  if (std::isinf(x)) {
    *rm = 1.0;
    *inv = 0.0;
    *frac = 1.0;
  } else {
    *rm = (x - 1.0) / (x + 1.0);
    *inv = 1.0 / (x + 1.0);
    *frac = x / (x + 1.0);
  }
}

void wall_coefficients(const Channel &c, WallD *lo, WallD *hi) {
  const bool link = c.p.bc == LKS_BC_LINK;
  const double xl = link ? c.d.theta_lower : c.d.phi_lower;
  const double xu = link ? c.d.theta_upper : c.d.phi_upper;
  double rm, inv, frac;
  ratio3(xl, &rm, &inv, &frac);
  // lower wall: incoming direction e_y = +1 -> moving term -frac B0 U
  lo->r = rm;
  lo->s = inv;
  lo->t = -frac * c.d.b0 * c.p.u_lower;
  lo->u = c.p.u_lower;
  lo->uw6 = c.p.u_lower / 6.0;
  ratio3(xu, &rm, &inv, &frac);
  // upper wall: incoming direction e_y = -1 -> moving term +frac B0 U
  hi->r = rm;
  hi->s = inv;
  hi->t = frac * c.d.b0 * c.p.u_upper;
  hi->u = c.p.u_upper;
  hi->uw6 = c.p.u_upper / 6.0;
}

} // namespace lks

extern "C" {

int lks_mhd_abi_version(void) { return LKS_MHD_ABI_VERSION; }

const char *lks_mhd_last_error(void) { return lks::g_error.c_str(); }

void lks_mhd_default_params(lks_mhd_params *p, int32_t nx, int32_t ny) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->nx = nx;
  p->ny = ny;
  p->bc = LKS_BC_LINK;
  p->precision = LKS_FP32;
  p->tau_f = 0.8;
  p->tau_m = 0.8;
  p->ha = NAN;
  p->b0 = 0.0;
  p->c_lower = 0.0;
  p->c_upper = 0.0;
  p->u_lower = 0.0;
  p->u_upper = 0.0;
  p->fx = 0.0;
  p->fy = 0.0;
  p->u_max = 0.0;
  p->rho0 = 1.0;
  p->collision = LKS_BGK;
  p->lambda_f = 3.0 / 16.0;
  p->lambda_m = 0.25;
  p->q_lower = 0.5;
  p->q_upper = 0.5;
  p->s_fe = 1.64;  // Lallemand & Luo (2000)
  p->s_feps = 1.54;
  p->s_fq = NAN;
  p->s_me = NAN;
  p->s_md = NAN;
}

int lks_mhd_validate(const lks_mhd_params *p) {
  lks::clear_error();
  return lks::derive_channel(p, nullptr);
}

int lks_mhd_derive(const lks_mhd_params *p, lks_mhd_derived *out) {
  lks::clear_error();
  lks::Channel c;
  const int rc = lks::derive_channel(p, &c);
  if (rc == LKS_OK && out) *out = c.d;
  return rc;
}

int lks_mhd_bytes_per_node(int32_t precision) {
  if (!lks::valid_precision(precision)) return 0;
  return (int)(2 * 19 * lks::elem_bytes(precision));
}

} // extern "C"
