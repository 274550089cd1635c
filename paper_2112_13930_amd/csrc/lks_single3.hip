// Three-dimensional channel: the fused step kernel over one z-periodic channel
// with Shercliff walls at y = 0 and y = ny - 1, its record/residual/moments
// variants, state exchange and hipGraph replay (see lks_node3.hpp for the
// lattices and the stored planes).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>

#include "lks_common.hpp"
#include "lks_node3.hpp"

namespace lks {

struct ObsOut3 {
  double *rho, *ux, *uy, *uz, *bx, *by, *bz, *jx, *jy, *jz;
};

constexpr int NRED3 = 6; // du2, u2, db2, b2, sum_u, nonfinite

// One block of 256 threads per tile of 256 consecutive x of one (y, z) line.
// A step is two launches over disjoint rows, both reading the same state:
// BC_NONE covers the interior rows 1..ny-2, BC_LINK / BC_MOMENT the two wall
// rows.  Tiles are numbered interior first (tile_base offsets the wall
// launch), so residual partial sums keep one fixed order.  ctr[2]: step
// counters as in the two-dimensional kernel; only the launch with owner set
// advances them.
// Waves per SIMD: 4 (at most 128 registers), except the MRT kernels in FP64,
// which spill at 4 and run as fast as TRT at 3 (154 registers).  The
// binary32 interior kernel also fits 5 (at most 96 registers) with two
// registers spilled, which ran 1% slower than 4 (20.6 against 20.8 G
// node-updates/s at 256^3, one box, alternating builds).
#ifndef LKS_STEP3_WAVES_FP32_INTERIOR
#define LKS_STEP3_WAVES_FP32_INTERIOR 4
#endif
template <typename S, int BC>
constexpr int kWaves3 =
    (wall_of(BC) == BC_NONE && sizeof(S) == 4 && !mrt_of(BC)) ? LKS_STEP3_WAVES_FP32_INTERIOR
    : (mrt_of(BC) && sizeof(S) == 8)                           ? 3
                                                               : 4;

// Rows of a launch.  Interior: (y, z) with 1 <= y <= ny-2 and every z, or
// 1 <= z <= nz-2 in a duct, numbered z-major.  Walls: the two Hartmann rows
// y = 0, ny-1 of every z, then in a duct the side rows z = 0, nz-1 of every
// interior y.
template <typename S, typename C, int BC, int MODE>
__global__ __launch_bounds__(256, (kWaves3<S, BC>)) void k_step3(
    Geom3 g, Coef<C> k, C fez, Side3<C> sw, const S *__restrict__ src, S *__restrict__ dst,
    int tiles_x, int tile_base, double *__restrict__ rec, double *__restrict__ partials,
    ObsOut3 oo, uint32_t *__restrict__ ctr, int parity, int owner) {
  constexpr bool SR = kUseSR<S, C> && MODE != MODE_MOMENTS;
  uint32_t sseed = 0;
  if constexpr (MODE != MODE_MOMENTS) {
    const uint32_t step = ctr[parity];
    if (owner && blockIdx.x == 0 && threadIdx.x == 0) ctr[parity ^ 1] = step + 1u;
    if constexpr (SR) sseed = step_seed(step);
  }
  const int line = (int)blockIdx.x / tiles_x;
  const int tx = (int)blockIdx.x - line * tiles_x;
  int y, z;
  if constexpr (wall_of(BC) == BC_NONE) {
    const int nrows = g.ny - 2;
    z = line / nrows + g.side;
    y = 1 + (line - (z - g.side) * nrows);
  } else if (line < 2 * g.nz) {
    z = line >> 1;
    y = (line & 1) ? g.ny - 1 : 0;
  } else {
    const int s = line - 2 * g.nz;
    z = (s & 1) ? g.nz - 1 : 0;
    y = 1 + (s >> 1);
  }
  const int tile = tile_base + (int)blockIdx.x;
  const int x = tx * 256 + (int)threadIdx.x;
  const bool act = x < g.nx;
  NodeObs3 o{};
  if (act) node3_update<S, C, BC, MODE, SR>(g, k, fez, sw, src, dst, x, y, z, o, sseed);
  const long long n = (long long)g.nx * g.ny * g.nz;
  const long long i = ((long long)z * g.ny + y) * g.nx + x;
  if constexpr (MODE == MODE_RECORD) {
    if (act) {
      rec[i] = o.ux;
      rec[n + i] = o.bx;
    }
  }
  if constexpr (MODE == MODE_MOMENTS) {
    if (act) {
      if (oo.rho) oo.rho[i] = 1.0 + o.rhop;
      if (oo.ux) oo.ux[i] = o.ux;
      if (oo.uy) oo.uy[i] = o.uy;
      if (oo.uz) oo.uz[i] = o.uz;
      if (oo.bx) oo.bx[i] = o.bx;
      if (oo.by) oo.by[i] = o.by;
      if (oo.bz) oo.bz[i] = o.bz;
      if (oo.jx) oo.jx[i] = o.jx;
      if (oo.jy) oo.jy[i] = o.jy;
      if (oo.jz) oo.jz[i] = o.jz;
    }
  }
  if constexpr (MODE == MODE_RESIDUAL) {
    __shared__ double lds[4 * NRED3];
    double v[NRED3] = {0, 0, 0, 0, 0, 0};
    if (act) {
      const double du = o.ux - rec[i], db = o.bx - rec[n + i];
      v[0] = du * du;
      v[1] = o.ux * o.ux;
      v[2] = db * db;
      v[3] = o.bx * o.bx;
      v[4] = o.ux;
      const bool ok = isfinite(o.rhop) && isfinite(o.ux) && isfinite(o.uy) && isfinite(o.uz) &&
                      isfinite(o.bx) && isfinite(o.by) && isfinite(o.bz) && 1.0 + o.rhop > 0.0;
      v[5] = ok ? 0.0 : 1.0;
    }
    block_sum<NRED3, 256>(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int j = 0; j < NRED3; ++j) partials[(long long)tile * 8 + j] = v[j];
    }
  }
}

__global__ __launch_bounds__(256) void k_finalize3(const double *__restrict__ partials, int ntiles,
                                                   double *__restrict__ out) {
  __shared__ double lds[4 * NRED3];
  double v[NRED3] = {0, 0, 0, 0, 0, 0};
  for (int t = threadIdx.x; t < ntiles; t += 256)
#pragma unroll
    for (int j = 0; j < NRED3; ++j) v[j] += partials[(long long)t * 8 + j];
  block_sum<NRED3, 256>(v, lds);
  if (threadIdx.x == 0)
    for (int j = 0; j < NRED3; ++j) out[j] = v[j];
}

// State <-> raw FP64 populations [40][nz][ny][nx] (the rest population of g
// is written as zero and must be zero on input).
template <typename S>
__global__ void k_init3(Geom3 g, double rho0, S *__restrict__ dst) {
  const long long n = (long long)g.nx * g.ny * g.nz;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int q = 0; q < 19; ++q) dst[at3(g, q, i)] = (S)(W3<double>::w(q) * (rho0 - 1.0));
  for (int q = 19; q < kPlanes3; ++q) dst[at3(g, q, i)] = (S)0.0;
}

template <typename S>
__global__ void k_save3(Geom3 g, double b0, const S *__restrict__ src, double *__restrict__ out) {
  const long long n = (long long)g.nx * g.ny * g.nz;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int q = 0; q < 19; ++q) out[q * n + i] = (double)src[at3(g, q, i)] + W3<double>::w(q);
  for (int c = 0; c < 3; ++c) {
    out[(19 + 7 * c) * n + i] = 0.0;
    const double off = c == 1 ? b0 / 6.0 : 0.0;
    for (int a = 0; a < 6; ++a)
      out[(20 + 7 * c + a) * n + i] = (double)src[at3(g, 19 + 6 * c + a, i)] + off;
  }
}

template <typename S>
__global__ void k_load3(Geom3 g, double b0, const double *__restrict__ in, S *__restrict__ dst) {
  const long long n = (long long)g.nx * g.ny * g.nz;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int q = 0; q < 19; ++q) dst[at3(g, q, i)] = (S)(in[q * n + i] - W3<double>::w(q));
  for (int c = 0; c < 3; ++c) {
    const double off = c == 1 ? b0 / 6.0 : 0.0;
    for (int a = 0; a < 6; ++a)
      dst[at3(g, 19 + 6 * c + a, i)] = (S)(in[(20 + 7 * c + a) * n + i] - off);
  }
}

} // namespace lks

using namespace lks;

struct lks_mhd3 {
  Channel ch;
  double fz = 0.0;
  int device = 0;
  hipStream_t stream = nullptr;
  Geom3 geom{};
  void *buf[2] = {nullptr, nullptr};
  double *rec = nullptr, *partials = nullptr, *result = nullptr;
  uint32_t *ctr = nullptr;
  int cur = 0;
  int64_t steps = 0;
  int tiles_x = 0, ntiles = 0;
  Coef<double> kd{};
  Coef<float> kf{};
  Side3<double> sd{};
  Side3<float> sf{};
  int graph_steps = 0;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
};

namespace {

template <typename C> const Coef<C> &coef3(const lks_mhd3 *h);
template <> const Coef<double> &coef3<double>(const lks_mhd3 *h) { return h->kd; }
template <> const Coef<float> &coef3<float>(const lks_mhd3 *h) { return h->kf; }
template <typename C> Side3<C> side3(const lks_mhd3 *h);
template <> Side3<double> side3<double>(const lks_mhd3 *h) { return h->sd; }
template <> Side3<float> side3<float>(const lks_mhd3 *h) { return h->sf; }

struct Layout3 {
  long long slab; // elements per (layer, plane), see Geom3
  size_t state_bytes, rec_bytes, part_bytes, total;
  int tiles_x, ntiles;
};

int validate3(const lks_mhd3_params *p, Channel *c) {
  if (!p) {
    set_error("invalid parameters: null pointer");
    return LKS_EINVAL;
  }
  const int rc = derive_channel(&p->base, c);
  if (rc != LKS_OK) return rc;
  if (p->nz < 1) {
    set_error("invalid parameters: nz must be >= 1");
    return LKS_EINVAL;
  }
  if ((long long)p->base.nx * p->base.ny * p->nz > (long long)((1LL << 31) - 1)) {
    set_error("invalid parameters: nx * ny * nz must be below 2^31");
    return LKS_EINVAL;
  }
  if (p->base.precision != LKS_FP64 && p->base.precision != LKS_FP32) {
    set_error("invalid parameters: the three-dimensional channel stores FP64 or FP32 populations");
    return LKS_EINVAL;
  }
  // the kernels address a layer's plane with 32-bit byte offsets (a
  // state of 74 such planes would exceed any device's memory long before)
  if ((long long)p->base.nx * p->base.ny * (long long)elem_bytes(p->base.precision) >
      (long long)((1LL << 32) - 256)) {
    set_error("invalid parameters: one layer's population plane (nx * ny values) must hold "
              "fewer than 2^32 bytes");
    return LKS_EINVAL;
  }
  if (!std::isfinite(p->fz)) {
    set_error("invalid parameters: fz must be finite");
    return LKS_EINVAL;
  }
  if (p->base.nsolids > 0) {
    set_error("invalid parameters: solid bodies are two-dimensional (base.nsolids = 0)");
    return LKS_EINVAL;
  }
  if (p->base.x_walls) {
    set_error("invalid parameters: x is periodic in three dimensions (base.x_walls = 0)");
    return LKS_EINVAL;
  }
  if (p->base.q_lower != 0.5 || p->base.q_upper != 0.5) {
    set_error("invalid parameters: the three-dimensional walls are half-way (q = 1/2)");
    return LKS_EINVAL;
  }

  if (p->side_walls != 0 && p->side_walls != 1) {
    set_error("invalid parameters: side_walls must be 0 or 1");
    return LKS_EINVAL;
  }
  if (p->side_walls) {
    if (p->base.bc != LKS_BC_LINK) {
      set_error("invalid parameters: side walls need link-based closures");
      return LKS_EINVAL;
    }
    if (p->nz < 2) {
      set_error("invalid parameters: a duct needs nz >= 2");
      return LKS_EINVAL;
    }
    if (std::isnan(p->c_side_lower) || p->c_side_lower < 0.0 || std::isnan(p->c_side_upper) ||
        p->c_side_upper < 0.0) {
      set_error("invalid parameters: side-wall conductance ratios must be in [0, inf]");
      return LKS_EINVAL;
    }
  }
  return LKS_OK;
}

// (theta-1)/(theta+1) of a side wall, theta = c a / (tau_m - 1/2).
double side_r(double c, const Channel &ch) {
  if (std::isinf(c)) return 1.0;
  const double th = c * ch.d.a / (ch.p.tau_m - 0.5);
  return (th - 1.0) / (th + 1.0);
}

Layout3 layout3(const lks_mhd3_params *p) {
  Layout3 L;
  const long long n = (long long)p->base.nx * p->base.ny * p->nz;
  const size_t eb = elem_bytes(p->base.precision);
  const long long per256 = 256 / (long long)eb;
  const long long layer = (long long)p->base.nx * p->base.ny;
  L.slab = (layer + per256 - 1) / per256 * per256;
  L.state_bytes = align256((size_t)kPlanes3 * p->nz * L.slab * eb);
  L.rec_bytes = align256((size_t)2 * n * sizeof(double));
  L.tiles_x = (p->base.nx + 255) / 256;
  L.ntiles = L.tiles_x * p->base.ny * p->nz;
  L.part_bytes = align256((size_t)L.ntiles * 8 * sizeof(double));
  L.total = 2 * L.state_bytes + L.rec_bytes + L.part_bytes + 256 + 256;
  return L;
}

template <typename S, typename C, int BC, int MODE>
hipError_t launch3_t(lks_mhd3 *h, const void *src, void *dst, ObsOut3 oo) {
  const Geom3 &g = h->geom;
  const int interior = h->tiles_x * (g.ny - 2) * (g.nz - 2 * g.side);
  const int walls = h->tiles_x * (2 * g.nz + 2 * g.side * (g.ny - 2));
  if (interior > 0) {
    constexpr int kInterior = BC_NONE | (BC & (COLL_TRT | COLL_MRT));
    hipLaunchKernelGGL((k_step3<S, C, kInterior, MODE>), dim3(interior), dim3(256), 0, h->stream,
                       h->geom, coef3<C>(h), (C)h->fz, side3<C>(h), static_cast<const S *>(src),
                       static_cast<S *>(dst), h->tiles_x, 0, h->rec, h->partials, oo, h->ctr,
                       h->cur, 1);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_step3<S, C, BC, MODE>), dim3(walls), dim3(256), 0, h->stream, h->geom,
                     coef3<C>(h), (C)h->fz, side3<C>(h), static_cast<const S *>(src),
                     static_cast<S *>(dst),
                     h->tiles_x, interior, h->rec, h->partials, oo, h->ctr, h->cur,
                     interior > 0 ? 0 : 1);
  return hipGetLastError();
}

template <typename S, typename C, int MODE>
hipError_t launch3_s(lks_mhd3 *h, const void *src, void *dst, ObsOut3 oo) {
  // observables do not depend on the collision operator
  const int sch = MODE == MODE_MOMENTS ? wall_of(scheme_of(h->ch.p)) : scheme_of(h->ch.p);
  switch (sch) {
  case BC_LINK: return launch3_t<S, C, BC_LINK, MODE>(h, src, dst, oo);
  case BC_MOMENT: return launch3_t<S, C, BC_MOMENT, MODE>(h, src, dst, oo);
  case BC_LINK | COLL_TRT:
    if constexpr (MODE != MODE_MOMENTS) return launch3_t<S, C, BC_LINK | COLL_TRT, MODE>(h, src, dst, oo);
    break;
  case BC_MOMENT | COLL_TRT:
    if constexpr (MODE != MODE_MOMENTS) return launch3_t<S, C, BC_MOMENT | COLL_TRT, MODE>(h, src, dst, oo);
    break;
  case BC_LINK | COLL_MRT:
    if constexpr (MODE != MODE_MOMENTS) return launch3_t<S, C, BC_LINK | COLL_MRT, MODE>(h, src, dst, oo);
    break;
  case BC_MOMENT | COLL_MRT:
    if constexpr (MODE != MODE_MOMENTS) return launch3_t<S, C, BC_MOMENT | COLL_MRT, MODE>(h, src, dst, oo);
    break;
  default: break;
  }
  return hipErrorInvalidValue;
}

template <int MODE>
hipError_t launch3(lks_mhd3 *h, const void *src, void *dst, ObsOut3 oo) {
  if (h->ch.p.precision == LKS_FP64) return launch3_s<double, double, MODE>(h, src, dst, oo);
  return launch3_s<float, Fp32Compute, MODE>(h, src, dst, oo);
}

int one_step3(lks_mhd3 *h, int mode) {
  const void *src = h->buf[h->cur];
  void *dst = h->buf[h->cur ^ 1];
  ObsOut3 oo{};
  hipError_t e;
  switch (mode) {
  case MODE_STEP: e = launch3<MODE_STEP>(h, src, dst, oo); break;
  case MODE_RECORD: e = launch3<MODE_RECORD>(h, src, dst, oo); break;
  default: e = launch3<MODE_RESIDUAL>(h, src, dst, oo); break;
  }
  if (e != hipSuccess) {
    set_error("3D step kernel launch failed: %s", hipGetErrorString(e));
    return LKS_EDEVICE;
  }
  h->cur ^= 1;
  h->steps += 1;
  return LKS_OK;
}

void drop_graphs3(lks_mhd3 *h) {
  for (auto &g : h->gexec)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

int capture3(lks_mhd3 *h, int parity) {
  hipGraph_t graph = nullptr;
  const int saved_cur = h->cur;
  const int64_t saved_steps = h->steps;
  h->cur = parity;
  LKS_HIP_CHECK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  int rc = LKS_OK;
  for (int i = 0; i < h->graph_steps && rc == LKS_OK; ++i) rc = one_step3(h, MODE_STEP);
  hipError_t e = hipStreamEndCapture(h->stream, &graph);
  h->cur = saved_cur;
  h->steps = saved_steps;
  if (rc != LKS_OK) return rc;
  if (e != hipSuccess) {
    set_error("hipStreamEndCapture failed: %s", hipGetErrorString(e));
    return LKS_EDEVICE;
  }
  e = hipGraphInstantiate(&h->gexec[parity], graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    set_error("hipGraphInstantiate failed: %s", hipGetErrorString(e));
    return LKS_EDEVICE;
  }
  return LKS_OK;
}

template <typename F>
int with_device3(lks_mhd3 *h, F &&fn) {
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) prev = h->device;
  if (prev != h->device) LKS_HIP_CHECK(hipSetDevice(h->device));
  const int rc = fn();
  if (prev != h->device) (void)hipSetDevice(prev);
  return rc;
}

int set_counter3(lks_mhd3 *h, int64_t steps) {
  const uint32_t v[2] = {(uint32_t)steps, (uint32_t)steps};
  LKS_HIP_CHECK(hipMemcpyAsync(h->ctr, v, sizeof v, hipMemcpyHostToDevice, h->stream));
  LKS_HIP_CHECK(hipStreamSynchronize(h->stream));
  return LKS_OK;
}

unsigned elementwise_grid3(const lks_mhd3 *h) {
  const long long n = (long long)h->geom.nx * h->geom.ny * h->geom.nz;
  return (unsigned)((n + 255) / 256);
}

} // namespace

extern "C" {

size_t lks_mhd3_state_bytes(const lks_mhd3_params *p) {
  clear_error();
  Channel c;
  if (validate3(p, &c) != LKS_OK) return 0;
  return layout3(p).total;
}

int lks_mhd3_bytes_per_node(int32_t precision) {
  if (precision != LKS_FP64 && precision != LKS_FP32) return 0;
  return (int)(2 * kPlanes3 * elem_bytes(precision));
}

int lks_mhd3_create(const lks_mhd3_params *p, void *dev_buf, size_t bytes, void *hip_stream,
                    lks_mhd3_t **out) {
  clear_error();
  if (!out) {
    set_error("out must not be NULL");
    return LKS_EINVAL;
  }
  *out = nullptr;
  Channel c;
  int rc = validate3(p, &c);
  if (rc != LKS_OK) return rc;
  const Layout3 L = layout3(p);
  if (!dev_buf || (reinterpret_cast<uintptr_t>(dev_buf) & 255u)) {
    set_error("dev_buf must be a non-NULL 256-byte aligned device pointer");
    return LKS_EINVAL;
  }
  if (bytes < L.total) {
    set_error("dev_buf holds %zu bytes, %zu needed", bytes, L.total);
    return LKS_ENOMEM;
  }
  lks_mhd3 *h = new (std::nothrow) lks_mhd3();
  if (!h) {
    set_error("host allocation failed");
    return LKS_ENOMEM;
  }
  h->ch = c;
  h->fz = p->fz;
  if (hipGetDevice(&h->device) != hipSuccess) h->device = 0;
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->geom = Geom3{c.p.nx, c.p.ny, p->nz, L.slab, p->side_walls};
  h->sd = Side3<double>{side_r(p->c_side_lower, c), side_r(p->c_side_upper, c)};
  h->sf = Side3<float>{(float)h->sd.r_lo, (float)h->sd.r_hi};
  char *base = static_cast<char *>(dev_buf);
  h->buf[0] = base;
  h->buf[1] = base + L.state_bytes;
  h->rec = reinterpret_cast<double *>(base + 2 * L.state_bytes);
  h->partials = reinterpret_cast<double *>(base + 2 * L.state_bytes + L.rec_bytes);
  h->result = reinterpret_cast<double *>(base + 2 * L.state_bytes + L.rec_bytes + L.part_bytes);
  h->ctr = reinterpret_cast<uint32_t *>(base + 2 * L.state_bytes + L.rec_bytes + L.part_bytes + 256);
  h->tiles_x = L.tiles_x;
  h->ntiles = L.ntiles;
  h->kd = make_coef<double>(c);
  h->kf = make_coef<float>(c);
  if (c.p.collision == LKS_MRT) {
    // D3Q7 has no rest weight, so g's isotropic second moment carries no
    // non-equilibrium part and its TRT step takes the even rate s_md
    const double gp = c.d.s_md, gm = 1.0 / c.p.tau_m;
    h->kd.trt.ga = 0.5 * (gp + gm), h->kd.trt.gb = 0.5 * (gp - gm), h->kd.trt.gp = gp;
    h->kf.trt.ga = (float)(0.5 * (gp + gm)), h->kf.trt.gb = (float)(0.5 * (gp - gm));
    h->kf.trt.gp = (float)gp;
  }
  rc = with_device3(h, [&]() -> int {
    if (c.p.precision == LKS_FP64)
      hipLaunchKernelGGL(k_init3<double>, dim3(elementwise_grid3(h)), dim3(256), 0, h->stream, h->geom,
                         c.p.rho0, static_cast<double *>(h->buf[0]));
    else
      hipLaunchKernelGGL(k_init3<float>, dim3(elementwise_grid3(h)), dim3(256), 0, h->stream, h->geom,
                         c.p.rho0, static_cast<float *>(h->buf[0]));
    LKS_HIP_CHECK(hipGetLastError());
    return set_counter3(h, 0);
  });
  if (rc != LKS_OK) {
    delete h;
    return rc;
  }
  *out = h;
  return LKS_OK;
}

int lks_mhd3_destroy(lks_mhd3_t *h) {
  clear_error();
  if (!h) return LKS_OK;
  drop_graphs3(h);
  delete h;
  return LKS_OK;
}

int lks_mhd3_set_graph(lks_mhd3_t *h, int32_t steps_per_graph) {
  clear_error();
  if (!h || steps_per_graph < 0 || (steps_per_graph % 2) != 0) {
    set_error("steps_per_graph must be an even number >= 0");
    return LKS_EINVAL;
  }
  if (steps_per_graph != 0 && h->stream == nullptr) {
    set_error("graph capture needs a non-default stream");
    return LKS_EINVAL;
  }
  drop_graphs3(h);
  h->graph_steps = steps_per_graph;
  return LKS_OK;
}

int64_t lks_mhd3_steps_done(const lks_mhd3_t *h) { return h ? h->steps : -1; }

int lks_mhd3_step(lks_mhd3_t *h, int64_t nsteps) {
  clear_error();
  if (!h || nsteps < 0) {
    set_error("invalid handle or negative step count");
    return LKS_EINVAL;
  }
  return with_device3(h, [&]() -> int {
    int64_t n = nsteps;
    while (n > 0) {
      if (h->graph_steps >= 2 && n >= h->graph_steps) {
        if (!h->gexec[h->cur]) {
          const int rc = capture3(h, h->cur);
          if (rc != LKS_OK) return rc;
        }
        LKS_HIP_CHECK(hipGraphLaunch(h->gexec[h->cur], h->stream));
        h->steps += h->graph_steps;
        n -= h->graph_steps;
      } else {
        const int rc = one_step3(h, MODE_STEP);
        if (rc != LKS_OK) return rc;
        n -= 1;
      }
    }
    return LKS_OK;
  });
}

int lks_mhd3_run_to_steady(lks_mhd3_t *h, double tol, int64_t check_every, int64_t max_steps,
                           int64_t *steps_done, double *residual, double *flow_rate) {
  clear_error();
  if (!h || check_every < 2 || max_steps < 0 || !(tol >= 0.0)) {
    set_error("invalid handle, check_every < 2, max_steps < 0 or tol < 0");
    return LKS_EINVAL;
  }
  double res = NAN, q = NAN;
  int status = LKS_ENOTCONV;
  const int rc = with_device3(h, [&]() -> int {
    int64_t done = 0;
    while (done + check_every <= max_steps) {
      int rc2 = one_step3(h, MODE_RECORD);
      if (rc2 != LKS_OK) return rc2;
      if ((rc2 = lks_mhd3_step(h, check_every - 2)) != LKS_OK) return rc2;
      if ((rc2 = one_step3(h, MODE_RESIDUAL)) != LKS_OK) return rc2;
      hipLaunchKernelGGL(k_finalize3, dim3(1), dim3(256), 0, h->stream, h->partials, h->ntiles,
                         h->result);
      LKS_HIP_CHECK(hipGetLastError());
      double sums[NRED3];
      LKS_HIP_CHECK(hipMemcpyAsync(sums, h->result, sizeof sums, hipMemcpyDeviceToHost, h->stream));
      LKS_HIP_CHECK(hipStreamSynchronize(h->stream));
      done += check_every;
      const double win = (double)(check_every - 1);
      const double ru = std::sqrt(sums[0]) / std::fmax(std::sqrt(sums[1]), 1e-300) / win;
      const double rb = std::sqrt(sums[2]) / std::fmax(std::sqrt(sums[3]), 1e-300) / win;
      res = std::fmax(ru, rb);
      q = sums[4] / ((double)h->geom.nx * h->geom.nz);
      if (sums[5] != 0.0 || !std::isfinite(res)) {
        status = LKS_EUNSTABLE;
        set_error("non-finite or non-positive density/velocity/field after %lld steps",
                  (long long)h->steps);
        return LKS_OK;
      }
      if (res < tol) {
        status = LKS_OK;
        return LKS_OK;
      }
    }
    status = LKS_ENOTCONV;
    set_error("residual %.3e above tolerance %.3e after %lld steps", res, tol, (long long)h->steps);
    return LKS_OK;
  });
  if (steps_done) *steps_done = h->steps;
  if (residual) *residual = res;
  if (flow_rate) *flow_rate = q;
  return rc != LKS_OK ? rc : status;
}

int lks_mhd3_moments(lks_mhd3_t *h, double *rho, double *ux, double *uy, double *uz, double *bx,
                     double *by, double *bz, double *jx, double *jy, double *jz) {
  clear_error();
  if (!h) {
    set_error("invalid handle");
    return LKS_EINVAL;
  }
  return with_device3(h, [&]() -> int {
    ObsOut3 oo{rho, ux, uy, uz, bx, by, bz, jx, jy, jz};
    const hipError_t e = launch3<MODE_MOMENTS>(h, h->buf[h->cur], nullptr, oo);
    if (e != hipSuccess) {
      set_error("3D moments kernel launch failed: %s", hipGetErrorString(e));
      return LKS_EDEVICE;
    }
    return LKS_OK;
  });
}

int lks_mhd3_save_state(lks_mhd3_t *h, double *dev_pops) {
  clear_error();
  if (!h || !dev_pops) {
    set_error("invalid handle or NULL destination");
    return LKS_EINVAL;
  }
  return with_device3(h, [&]() -> int {
    if (h->ch.p.precision == LKS_FP64)
      hipLaunchKernelGGL(k_save3<double>, dim3(elementwise_grid3(h)), dim3(256), 0, h->stream, h->geom,
                         h->ch.d.b0, static_cast<const double *>(h->buf[h->cur]), dev_pops);
    else
      hipLaunchKernelGGL(k_save3<float>, dim3(elementwise_grid3(h)), dim3(256), 0, h->stream, h->geom,
                         h->ch.d.b0, static_cast<const float *>(h->buf[h->cur]), dev_pops);
    LKS_HIP_CHECK(hipGetLastError());
    return LKS_OK;
  });
}

int lks_mhd3_load_state(lks_mhd3_t *h, const double *dev_pops, int64_t steps) {
  clear_error();
  if (!h || !dev_pops || steps < 0) {
    set_error("invalid handle, NULL source or negative step count");
    return LKS_EINVAL;
  }
  return with_device3(h, [&]() -> int {
    if (h->ch.p.precision == LKS_FP64)
      hipLaunchKernelGGL(k_load3<double>, dim3(elementwise_grid3(h)), dim3(256), 0, h->stream, h->geom,
                         h->ch.d.b0, dev_pops, static_cast<double *>(h->buf[h->cur]));
    else
      hipLaunchKernelGGL(k_load3<float>, dim3(elementwise_grid3(h)), dim3(256), 0, h->stream, h->geom,
                         h->ch.d.b0, dev_pops, static_cast<float *>(h->buf[h->cur]));
    LKS_HIP_CHECK(hipGetLastError());
    h->steps = steps;
    return set_counter3(h, steps);
  });
}

} // extern "C"
