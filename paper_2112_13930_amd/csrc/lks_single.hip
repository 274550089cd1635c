// Single-channel entry points: the fused step kernel over one channel, the
// record/residual/moments variants of it, init/save/load, FP64 residual
// reduction and hipGraph replay of step sequences.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "lks_aux.hpp"
#include "lks_common.hpp"

namespace lks {

struct ObsOut {
  double *rho, *ux, *uy, *bx, *by, *jz;
};

constexpr int NRED = 6; // du2, u2, db2, b2, sum_u, nonfinite

// Launch shapes of the step kernel: BX x BY threads per block cover a tile
// of BX x BY nodes; REMAP maps consecutive tiles onto the same XCD (the
// hardware deals workgroups round-robin to the 8 XCDs).
// vx > 1: each thread updates vx consecutive nodes of a row with vector loads
// and stores (needs nx % vx == 0; only the plain step uses these shapes).
struct Shape {
  int bx, by;
  bool remap;
  int vx;
};
constexpr Shape kShapes[] = {{256, 1, false, 1}, {64, 4, true, 1}, {128, 2, true, 1},
                             {256, 1, true, 1},  {64, 4, false, 1}, {256, 1, false, 2},
                             {256, 1, false, 4}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);
constexpr int kRedShape = 1; // shape used by record/residual/moments kernels

__device__ __forceinline__ int map_tile(bool remap) {
  const int id = blockIdx.x;
  if (!remap) return id;
  const int per = gridDim.x >> 3; // grid is a multiple of 8 when remapping
  return (id & 7) * per + (id >> 3);
}

// ctr[2]: the channel-local index of the step in flight is ctr[parity]; the
// first block of a step writes ctr[parity ^ 1] = ctr[parity] + 1 for the next
// step, which reads the other slot, so no launch reads what it writes.
template <typename S, typename C, int BC, int MODE, int BX, int BY, bool REMAP>
__global__ __launch_bounds__(BX *BY) void k_step(Geom g, Coef<C> k,
                                                 const S *__restrict__ src,
                                                 S *__restrict__ dst,
                                                 const C *__restrict__ ref,
                                                 int tiles_x, int ntiles,
                                                 double *__restrict__ rec,
                                                 double *__restrict__ partials,
                                                 ObsOut oo, uint32_t *__restrict__ ctr,
                                                 int parity) {
  constexpr bool SR = kUseSR<S, C> && MODE != MODE_MOMENTS;
  uint32_t sseed = 0;
  if constexpr (MODE != MODE_MOMENTS) {
    const uint32_t step = ctr[parity];
    if (blockIdx.x == 0 && threadIdx.x == 0 && threadIdx.y == 0) ctr[parity ^ 1] = step + 1u;
    if constexpr (SR) sseed = step_seed(step);
  }
  const int tile = map_tile(REMAP);
  if (tile >= ntiles) return; // uniform per block
  const int ty = tile / tiles_x;
  const int tx = tile - ty * tiles_x;
  const int x = tx * BX + (int)threadIdx.x;
  // (one row per block when BY == 1: the row is then uniform, and the
  // binary16 row tables are read as scalars)
  const int y = BY == 1 ? ty : ty * BY + (int)threadIdx.y;
  const bool act = (x < g.nx) && (y < g.ny);
  NodeObs<C> o{};
  if (act) node_update<S, C, BC, MODE, SR>(g, k, src, ref, dst, x, y, o, sseed);
  const long long n = (long long)g.nx * g.ny;
  const long long i = (long long)y * g.nx + x;
  if constexpr (MODE == MODE_RECORD) {
    if (act) {
      rec[i] = (double)o.ux;
      rec[n + i] = (double)o.bx;
    }
  }
  if constexpr (MODE == MODE_MOMENTS) {
    if (act) {
      if (oo.rho) oo.rho[i] = 1.0 + (double)o.rhop;
      if (oo.ux) oo.ux[i] = (double)o.ux;
      if (oo.uy) oo.uy[i] = (double)o.uy;
      if (oo.bx) oo.bx[i] = (double)o.bx;
      if (oo.by) oo.by[i] = (double)o.by;
      if (oo.jz) oo.jz[i] = (double)o.jz;
    }
  }
  if constexpr (MODE == MODE_RESIDUAL) {
    __shared__ double lds[(BX * BY / 64) * NRED];
    double v[NRED] = {0, 0, 0, 0, 0, 0};
    if (act) {
      const double u = (double)o.ux, b = (double)o.bx;
      const double du = u - rec[i], db = b - rec[n + i];
      v[0] = du * du;
      v[1] = u * u;
      v[2] = db * db;
      v[3] = b * b;
      v[4] = u;
      const bool ok = isfinite((double)o.rho) && isfinite(u) && isfinite((double)o.uy) &&
                      isfinite(b) && isfinite((double)o.by) && (double)o.rho > 0.0 &&
                        fabs(u) < 1.0 && fabs((double)o.uy) < 1.0;
      v[5] = ok ? 0.0 : 1.0;
    }
    block_sum<NRED, BX * BY>(v, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
#pragma unroll
      for (int j = 0; j < NRED; ++j) partials[(long long)tile * 8 + j] = v[j];
    }
  }
}

// Plain step with VX consecutive nodes per thread: the unshifted planes are
// read and all planes written as VX-wide vectors; an x-shifted plane needs
// one more element beyond the vector (x0 - 1 or x0 + VX, wrapped), read as a
// scalar.  Per node the arithmetic is node_finish, as in k_step, so the
// results are bitwise those of the scalar kernel.
template <typename S, typename C, int BC, int VX>
__global__ __launch_bounds__(256) void k_step_vec(Geom g, Coef<C> k, const S *__restrict__ src,
                                                  S *__restrict__ dst, const C *__restrict__ ref,
                                                  int tiles_x, int ntiles,
                                                  uint32_t *__restrict__ ctr, int parity) {
  using V = S __attribute__((ext_vector_type(VX)));
  constexpr bool SR = kUseSR<S, C>;
  const uint32_t step = ctr[parity];
  if (blockIdx.x == 0 && threadIdx.x == 0) ctr[parity ^ 1] = step + 1u;
  const uint32_t sseed = SR ? step_seed(step) : 0u;
  const int tile = blockIdx.x;
  if (tile >= ntiles) return;
  const int y = tile / tiles_x;
  const int tx = tile - y * tiles_x;
  const int x0 = (tx * 256 + (int)threadIdx.x) * VX;
  if (x0 >= g.nx) return;
  const int nx = g.nx;
  const long long P = g.plane;
  const bool lo = (y == 0), hi = (y == g.ny - 1);
  const long long r0 = (long long)y * g.pitch, rm = r0 - g.pitch, rp = r0 + g.pitch;
  const int xm0 = (x0 == 0) ? nx - 1 : x0 - 1;     // x - 1 of the first node
  const int xpe = (x0 + VX == nx) ? 0 : x0 + VX;    // x + 1 of the last node
  // a plane's base (uniform) plus a 32-bit byte offset within the plane
  // (planes hold fewer than 2^31 / 19 elements of at most 8 bytes), so that
  // each access takes a scalar base and one vector offset
  auto at = [&](int q, long long e) -> const char * {
    return reinterpret_cast<const char *>(src + (long long)q * P) + (uint32_t)(e * (long long)sizeof(S));
  };
  auto vld = [&](int q, long long e) { return *(gptr<const V>)at(q, e); };
  auto sld = [&](int q, long long e) { return *(gptr<const S>)at(q, e); };
  const V a0 = vld(0, r0 + x0), a1 = vld(1, r0 + x0), a3 = vld(3, r0 + x0);
  const S e1 = sld(1, r0 + xm0), e3 = sld(3, r0 + xpe);
  const V b0 = vld(9, r0 + x0), b1 = vld(10, r0 + x0), b3 = vld(12, r0 + x0);
  const S eb1 = sld(10, r0 + xm0), eb3 = sld(12, r0 + xpe);
  const V c0 = vld(14, r0 + x0), c1 = vld(15, r0 + x0), c3 = vld(17, r0 + x0);
  const S ec1 = sld(15, r0 + xm0), ec3 = sld(17, r0 + xpe);
  V a2{}, a5{}, a6{}, b2{}, c2{}, a4{}, a7{}, a8{}, b4{}, c4{};
  S e5{}, e6{}, e7{}, e8{};
  if (!lo) {
    a2 = vld(2, rm + x0);
    a5 = vld(5, rm + x0);
    a6 = vld(6, rm + x0);
    e5 = sld(5, rm + xm0);
    e6 = sld(6, rm + xpe);
    b2 = vld(11, rm + x0);
    c2 = vld(16, rm + x0);
  }
  if (!hi) {
    a4 = vld(4, rp + x0);
    a7 = vld(7, rp + x0);
    a8 = vld(8, rp + x0);
    e7 = sld(7, rp + xpe);
    e8 = sld(8, rp + xm0);
    b4 = vld(13, rp + x0);
    c4 = vld(18, rp + x0);
  }
  const C *__restrict__ Dy = ref + (long long)y * kRefRow; // row references (binary16 only)
  const C *__restrict__ Dm = lo ? Dy : Dy - kRefRow;
  const C *__restrict__ Dp = hi ? Dy : Dy + kRefRow;
  V outv[19];
#pragma unroll
  for (int v = 0; v < VX; ++v) {
    // pulled populations of node x0 + v: x - 1 planes take element v - 1
    // (or the extra scalar for v = 0), x + 1 planes element v + 1
    if constexpr (kXA<S, C>) {
      // binary16 computed in FP32: the undecoded values in plane order
      const S raw[19] = {a0[v],
                         v == 0 ? e1 : a1[v > 0 ? v - 1 : 0],
                         a2[v],
                         v == VX - 1 ? e3 : a3[v < VX - 1 ? v + 1 : 0],
                         a4[v],
                         v == 0 ? e5 : a5[v > 0 ? v - 1 : 0],
                         v == VX - 1 ? e6 : a6[v < VX - 1 ? v + 1 : 0],
                         v == VX - 1 ? e7 : a7[v < VX - 1 ? v + 1 : 0],
                         v == 0 ? e8 : a8[v > 0 ? v - 1 : 0],
                         b0[v],
                         v == 0 ? eb1 : b1[v > 0 ? v - 1 : 0],
                         b2[v],
                         v == VX - 1 ? eb3 : b3[v < VX - 1 ? v + 1 : 0],
                         b4[v],
                         c0[v],
                         v == 0 ? ec1 : c1[v > 0 ? v - 1 : 0],
                         c2[v],
                         v == VX - 1 ? ec3 : c3[v < VX - 1 ? v + 1 : 0],
                         c4[v]};
      NodeObs<C> o{};
      const XTabs t = xtabs_of(const_cast<C *>(ref), g.ny);
      const long long row = (long long)y * kRefRow;
      // the node's random words (F16Words), each rounding written straight
      // into node v's half of the plane's vector
      F16Words ew(SR ? node_seed(sseed, (uint32_t)(y * nx + x0 + v)) : 0u);
      const int v0 = v & ~1; // (the loop is unrolled: v is a constant)
      node_finish_x<S, BC, MODE_STEP>(g, k, src, t, t.V + row, t.K + row, x0 + v, y, raw, o,
                                      [&](int q, float zq) {
                                        if constexpr (SR) {
                                          S lo = outv[q][v0], hi = outv[q][v0 + 1];
                                          if (v & 1) sr_f16_half<true>(lo, hi, zq, ew.word(q));
                                          else sr_f16_half<false>(lo, hi, zq, ew.word(q));
                                          outv[q][v0] = lo, outv[q][v0 + 1] = hi;
                                        } else {
                                          outv[q][v] = (S)zq;
                                        }
                                      });
    } else {
    C f[9], gx[5], gy[5];
    f[0] = dec<S>((C)a0[v], Dy, 0);
    f[1] = dec<S>((C)(v == 0 ? e1 : a1[v > 0 ? v - 1 : 0]), Dy, 1);
    f[3] = dec<S>((C)(v == VX - 1 ? e3 : a3[v < VX - 1 ? v + 1 : 0]), Dy, 3);
    f[2] = dec<S>((C)a2[v], Dm, 2);
    f[5] = dec<S>((C)(v == 0 ? e5 : a5[v > 0 ? v - 1 : 0]), Dm, 5);
    f[6] = dec<S>((C)(v == VX - 1 ? e6 : a6[v < VX - 1 ? v + 1 : 0]), Dm, 6);
    f[4] = dec<S>((C)a4[v], Dp, 4);
    f[7] = dec<S>((C)(v == VX - 1 ? e7 : a7[v < VX - 1 ? v + 1 : 0]), Dp, 7);
    f[8] = dec<S>((C)(v == 0 ? e8 : a8[v > 0 ? v - 1 : 0]), Dp, 8);
    gx[0] = dec<S>((C)b0[v], Dy, 9);
    gx[1] = dec<S>((C)(v == 0 ? eb1 : b1[v > 0 ? v - 1 : 0]), Dy, 10);
    gx[3] = dec<S>((C)(v == VX - 1 ? eb3 : b3[v < VX - 1 ? v + 1 : 0]), Dy, 12);
    gx[2] = dec<S>((C)b2[v], Dm, 11);
    gx[4] = dec<S>((C)b4[v], Dp, 13);
    gy[0] = dec<S>((C)c0[v], Dy, 14);
    gy[1] = dec<S>((C)(v == 0 ? ec1 : c1[v > 0 ? v - 1 : 0]), Dy, 15);
    gy[3] = dec<S>((C)(v == VX - 1 ? ec3 : c3[v < VX - 1 ? v + 1 : 0]), Dy, 17);
    gy[2] = dec<S>((C)c2[v], Dm, 16);
    gy[4] = dec<S>((C)c4[v], Dp, 18);
    NodeObs<C> o{};
    S out[19];
    node_finish<S, C, BC, MODE_STEP, SR>(g, k, src, ref, x0 + v, y, f, gx, gy, o, sseed, out);
#pragma unroll
    for (int q = 0; q < 19; ++q) outv[q][v] = out[q];
    }
  }
  // byte offset in a plane, formed in 32 bits (so that it stays the store's
  // 32-bit vector offset)
  uint32_t so = ((uint32_t)y * (uint32_t)g.pitch + (uint32_t)x0) * (uint32_t)sizeof(S);
  asm("" : "+v"(so));
#pragma unroll
  for (int q = 0; q < 19; ++q)
    __builtin_nontemporal_store(outv[q],
                                (gptr<V>)(reinterpret_cast<char *>(sbase(dst + (long long)q * P)) + so));
}

// Step counters of a channel set on the device (no host copy).
__global__ void k_set_counter(uint32_t *__restrict__ ctr, uint32_t v) {
  if (threadIdx.x < 2) ctr[threadIdx.x] = v;
}

// Fixed-order sum of per-tile partials (one block of 256 threads).
__global__ __launch_bounds__(256) void k_finalize(const double *__restrict__ partials,
                                                  int ntiles, double *__restrict__ out) {
  __shared__ double lds[4 * NRED];
  double v[NRED] = {0, 0, 0, 0, 0, 0};
  for (int t = threadIdx.x; t < ntiles; t += 256)
#pragma unroll
    for (int j = 0; j < NRED; ++j) v[j] += partials[(long long)t * 8 + j];
  block_sum<NRED, 256>(v, lds);
  if (threadIdx.x == 0)
    for (int j = 0; j < NRED; ++j) out[j] = v[j];
}

} // namespace lks

using namespace lks;

struct lks_mhd {
  Channel ch;
  int device = 0;
  hipStream_t stream = nullptr;
  Geom geom{};
  void *buf[2] = {nullptr, nullptr};
  double *rec = nullptr;
  double *partials = nullptr;
  double *result = nullptr;
  uint32_t *ctr = nullptr; // step counters [2] (device)
  void *ref = nullptr;      // row references [ny][19] of the compute type (device)
  int cur = 0;
  int64_t steps = 0;
  int shape = 0;
  int red_tiles_x = 0, red_ntiles = 0, red_grid = 0;
  Coef<double> kd{};
  Coef<float> kf{};
  int graph_steps = 0;
  int64_t rebase_every = 0; // plain stepping: rebase before steps at multiples of this
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
};

namespace {

struct Layout {
  long long plane;
  size_t state_bytes, rec_bytes, part_bytes, ref_bytes, total;
  int red_tiles_x, red_ntiles;
  size_t sidx_bytes, snode_bytes; // solid bodies: per-node index, link table
};

Layout layout_of(const Channel &c) {
  Layout L;
  const int prec = c.p.precision;
  L.plane = single_plane_elems(c.p.nx, c.p.ny, prec);
  L.state_bytes = align256((size_t)19 * L.plane * elem_bytes(prec));
  L.rec_bytes = align256((size_t)2 * c.p.nx * c.p.ny * sizeof(double));
  const Shape s = kShapes[kRedShape];
  L.red_tiles_x = (c.p.nx + s.bx - 1) / s.bx;
  L.red_ntiles = L.red_tiles_x * ((c.p.ny + s.by - 1) / s.by);
  L.part_bytes = align256((size_t)L.red_ntiles * 8 * sizeof(double));
  L.ref_bytes = ref_area_bytes(c.p.ny, prec);
  L.sidx_bytes = L.snode_bytes = 0;
  if (c.p.nsolids > 0) {
    std::vector<int32_t> idx;
    std::vector<CurvedNode> nodes;
    const char *why = nullptr;
    (void)build_solid_tables(c.p, &idx, &nodes, &why); // validated by derive_channel
    L.sidx_bytes = align256((size_t)c.p.nx * c.p.ny * sizeof(int32_t));
    L.snode_bytes = align256(std::max<size_t>(nodes.size(), 1) * sizeof(CurvedNode));
  }
  L.total = 2 * L.state_bytes + L.rec_bytes + L.part_bytes + 256 + 256 + L.ref_bytes +
            L.sidx_bytes + L.snode_bytes;
  return L;
}

int grid_for(int ntiles, bool remap) { return remap ? (ntiles + 7) / 8 * 8 : ntiles; }

// Default rebase interval of plain stepping for binary16 states.
constexpr int64_t kDefaultRebase = 1000;

template <typename C> const Coef<C> &coef_of(const lks_mhd *h);
template <> const Coef<double> &coef_of<double>(const lks_mhd *h) { return h->kd; }
template <> const Coef<float> &coef_of<float>(const lks_mhd *h) { return h->kf; }

// Row references a kernel of (S, C) reads: the observables of the
// FP32-arithmetic binary16 mode decode its FP32 references in FP64.
template <typename S, typename C>
const C *ref_of(const lks_mhd *h) {
  if constexpr (kRowRef<S> && sizeof(C) == 8)
    if (h->ch.p.precision == LKS_FP16_STORE) return xtabs_of(h->ref, h->geom.ny).D64;
  return static_cast<const C *>(h->ref);
}

template <typename S, typename C, int BC, int MODE, int SH>
hipError_t launch_shape(lks_mhd *h, const void *src, void *dst, ObsOut oo) {
  constexpr Shape s = kShapes[SH];
  const Coef<C> &k = coef_of<C>(h);
  if constexpr (s.vx > 1 && MODE == MODE_STEP) {
    const int tiles_x = (h->geom.nx + s.bx * s.vx - 1) / (s.bx * s.vx);
    const int ntiles = tiles_x * h->geom.ny;
    hipLaunchKernelGGL((k_step_vec<S, C, BC, s.vx>), dim3(ntiles), dim3(s.bx), 0, h->stream,
                       h->geom, k, static_cast<const S *>(src), static_cast<S *>(dst),
                       ref_of<S, C>(h), tiles_x, ntiles, h->ctr, h->cur);
    return hipGetLastError();
  }
  const int tiles_x = (h->geom.nx + s.bx - 1) / s.bx;
  const int ntiles = tiles_x * ((h->geom.ny + s.by - 1) / s.by);
  const int grid = grid_for(ntiles, s.remap);
  hipLaunchKernelGGL((k_step<S, C, BC, MODE, s.bx, s.by, s.remap>), dim3(grid),
                     dim3(s.bx, s.by), 0, h->stream, h->geom, k,
                     static_cast<const S *>(src), static_cast<S *>(dst),
                     ref_of<S, C>(h), tiles_x, ntiles, h->rec, h->partials, oo,
                     h->ctr, h->cur);
  return hipGetLastError();
}

template <typename S, typename C, int BC, int MODE>
hipError_t launch_bc(lks_mhd *h, int shape, const void *src, void *dst, ObsOut oo) {
  switch (shape) {
  case 0: return launch_shape<S, C, BC, MODE, 0>(h, src, dst, oo);
  case 1: return launch_shape<S, C, BC, MODE, 1>(h, src, dst, oo);
  case 2: return launch_shape<S, C, BC, MODE, 2>(h, src, dst, oo);
  case 3: return launch_shape<S, C, BC, MODE, 3>(h, src, dst, oo);
  case 4: return launch_shape<S, C, BC, MODE, 4>(h, src, dst, oo);
  case 5: return launch_shape<S, C, BC, MODE, 5>(h, src, dst, oo);
  default: return launch_shape<S, C, BC, MODE, 6>(h, src, dst, oo);
  }
}

template <int MODE>
hipError_t launch_mode(lks_mhd *h, int shape, const void *src, void *dst, ObsOut oo) {
  // observables do not depend on the collision operator (the walls they do)
  const int sch =
      MODE == MODE_MOMENTS ? scheme_of(h->ch.p) & ~(COLL_TRT | COLL_MRT) : scheme_of(h->ch.p);
  constexpr bool kCollide = MODE != MODE_MOMENTS;
  return dispatch_precision(h->ch.p.precision, [&](auto t) -> hipError_t {
    using S = typename decltype(t)::S;
    // observables of binary16 computed in FP32 are taken in FP64
    using C0 = typename decltype(t)::C;
    using C = std::conditional_t<MODE == MODE_MOMENTS && kXA<S, C0>, double, C0>;
    switch (sch) {
    case BC_LINK: return launch_bc<S, C, BC_LINK, MODE>(h, shape, src, dst, oo);
    case BC_MOMENT: return launch_bc<S, C, BC_MOMENT, MODE>(h, shape, src, dst, oo);
    case BC_LINK | WALLS_X: return launch_bc<S, C, BC_LINK | WALLS_X, MODE>(h, shape, src, dst, oo);
    case BC_LINK | COLL_TRT:
      if constexpr (kCollide) return launch_bc<S, C, BC_LINK | COLL_TRT, MODE>(h, shape, src, dst, oo);
      break;
    case BC_MOMENT | COLL_TRT:
      if constexpr (kCollide) return launch_bc<S, C, BC_MOMENT | COLL_TRT, MODE>(h, shape, src, dst, oo);
      break;
    case BC_LINK | COLL_TRT | WALLS_X:
      if constexpr (kCollide)
        return launch_bc<S, C, BC_LINK | COLL_TRT | WALLS_X, MODE>(h, shape, src, dst, oo);
      break;
    case BC_LINK | WALLS_Q: return launch_bc<S, C, BC_LINK | WALLS_Q, MODE>(h, shape, src, dst, oo);
    case BC_LINK | COLL_TRT | WALLS_Q:
      if constexpr (kCollide)
        return launch_bc<S, C, BC_LINK | COLL_TRT | WALLS_Q, MODE>(h, shape, src, dst, oo);
      break;
    case BC_LINK | COLL_MRT:
      if constexpr (kCollide) return launch_bc<S, C, BC_LINK | COLL_MRT, MODE>(h, shape, src, dst, oo);
      break;
    case BC_MOMENT | COLL_MRT:
      if constexpr (kCollide) return launch_bc<S, C, BC_MOMENT | COLL_MRT, MODE>(h, shape, src, dst, oo);
      break;
    case BC_LINK | COLL_MRT | WALLS_X:
      if constexpr (kCollide)
        return launch_bc<S, C, BC_LINK | COLL_MRT | WALLS_X, MODE>(h, shape, src, dst, oo);
      break;
    case BC_LINK | COLL_MRT | WALLS_Q:
      if constexpr (kCollide)
        return launch_bc<S, C, BC_LINK | COLL_MRT | WALLS_Q, MODE>(h, shape, src, dst, oo);
      break;
    default: break;
    }
    // solid bodies: FP64 and FP32 storage, plain launches (shape 0)
    if constexpr (!kRowRef<S>) {
      switch (sch) {
      case BC_LINK | SOLIDS: return launch_shape<S, C, BC_LINK | SOLIDS, MODE, 0>(h, src, dst, oo);
      case BC_MOMENT | SOLIDS:
        return launch_shape<S, C, BC_MOMENT | SOLIDS, MODE, 0>(h, src, dst, oo);
      case BC_LINK | COLL_TRT | SOLIDS:
        if constexpr (kCollide)
          return launch_shape<S, C, BC_LINK | COLL_TRT | SOLIDS, MODE, 0>(h, src, dst, oo);
        break;
      case BC_MOMENT | COLL_TRT | SOLIDS:
        if constexpr (kCollide)
          return launch_shape<S, C, BC_MOMENT | COLL_TRT | SOLIDS, MODE, 0>(h, src, dst, oo);
        break;
      case BC_LINK | COLL_MRT | SOLIDS:
        if constexpr (kCollide)
          return launch_shape<S, C, BC_LINK | COLL_MRT | SOLIDS, MODE, 0>(h, src, dst, oo);
        break;
      case BC_MOMENT | COLL_MRT | SOLIDS:
        if constexpr (kCollide)
          return launch_shape<S, C, BC_MOMENT | COLL_MRT | SOLIDS, MODE, 0>(h, src, dst, oo);
        break;
      default: break;
      }
    }
    return hipErrorInvalidValue;
  });
}

// One step from buf[cur] into buf[cur^1].
int one_step(lks_mhd *h, int mode) {
  const void *src = h->buf[h->cur];
  void *dst = h->buf[h->cur ^ 1];
  ObsOut oo{};
  hipError_t e;
  switch (mode) {
  case MODE_STEP: e = launch_mode<MODE_STEP>(h, h->shape, src, dst, oo); break;
  case MODE_RECORD: e = launch_mode<MODE_RECORD>(h, kRedShape, src, dst, oo); break;
  default: e = launch_mode<MODE_RESIDUAL>(h, kRedShape, src, dst, oo); break;
  }
  if (e != hipSuccess) {
    set_error("step kernel launch failed: %s", hipGetErrorString(e));
    return LKS_EDEVICE;
  }
  h->cur ^= 1;
  h->steps += 1;
  return LKS_OK;
}

int capture_graph(lks_mhd *h, int parity) {
  hipGraph_t graph = nullptr;
  const int saved_cur = h->cur;
  const int64_t saved_steps = h->steps;
  h->cur = parity;
  LKS_HIP_CHECK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  int rc = LKS_OK;
  for (int i = 0; i < h->graph_steps && rc == LKS_OK; ++i) rc = one_step(h, MODE_STEP);
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

void drop_graphs(lks_mhd *h) {
  for (auto &g : h->gexec)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

template <typename F>
int with_device(lks_mhd *h, F &&fn) {
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) prev = h->device;
  if (prev != h->device) LKS_HIP_CHECK(hipSetDevice(h->device));
  const int rc = fn();
  if (prev != h->device) (void)hipSetDevice(prev);
  return rc;
}

// Set the step counter of the current buffer (outside any graph capture).
int set_counter(lks_mhd *h, int64_t steps) {
  const uint32_t v[2] = {(uint32_t)steps, (uint32_t)steps};
  LKS_HIP_CHECK(hipMemcpyAsync(h->ctr, v, sizeof v, hipMemcpyHostToDevice, h->stream));
  LKS_HIP_CHECK(hipStreamSynchronize(h->stream));
  return LKS_OK;
}

int elementwise_grid(const lks_mhd *h) {
  const long long n = (long long)h->geom.nx * h->geom.ny;
  return (int)((n + 255) / 256);
}

// Pre-collision tables of the FP32-arithmetic binary16 mode, after every
// change of its row references.
int refresh_tables(lks_mhd *h) {
  if (h->ch.p.precision != LKS_FP16_STORE) return LKS_OK;
  const dim3 grid((unsigned)((h->geom.ny + 255) / 256));
  const int sch = scheme_of(h->ch.p);
  if (cut_of(sch))
    hipLaunchKernelGGL(k_xtables<BC_LINK | WALLS_Q>, grid, dim3(256), 0, h->stream, h->geom, h->kd, h->ref);
  else if (wall_of(sch) == BC_LINK)
    hipLaunchKernelGGL(k_xtables<BC_LINK>, grid, dim3(256), 0, h->stream, h->geom, h->kd, h->ref);
  else
    hipLaunchKernelGGL(k_xtables<BC_MOMENT>, grid, dim3(256), 0, h->stream, h->geom, h->kd, h->ref);
  LKS_HIP_CHECK(hipGetLastError());
  return LKS_OK;
}

// Clear the row references (the stored values then hold the deviations).
int zero_ref(lks_mhd *h) {
  const long long n = (long long)(ref_area_bytes(h->geom.ny, h->ch.p.precision) / sizeof(double));
  hipLaunchKernelGGL(k_zero<double>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->stream,
                     static_cast<double *>(h->ref), n);
  LKS_HIP_CHECK(hipGetLastError());
  return refresh_tables(h);
}

// Row rebase of a binary16 state (other storage keeps no row reference).
int rebase_now(lks_mhd *h) {
  return dispatch_precision(h->ch.p.precision, [&](auto t) -> int {
    using S = typename decltype(t)::S;
    using C = typename decltype(t)::C;
    if constexpr (kRowRef<S>) {
      hipLaunchKernelGGL((k_rebase_rows<S, C>), dim3(h->geom.ny), dim3(256), 0, h->stream, h->geom,
                         static_cast<S *>(h->buf[h->cur]), static_cast<C *>(h->ref),
                         (uint32_t)h->steps);
      LKS_HIP_CHECK(hipGetLastError());
      return refresh_tables(h);
    }
    return LKS_OK;
  });
}

bool rebase_due(const lks_mhd *h) {
  return h->rebase_every > 0 && h->steps % h->rebase_every == 0;
}

// Device memory of lks_mhd_advance_noalloc: one static array per device the
// library runs on, held until the process ends.  In host code its name is
// only a stand-in; kernels take the address hipGetSymbolAddress returns for
// the current device.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// The scratch array's address on the current device (looked up once per
// device); LKS_EDEVICE if the lookup fails.
int scratch_address(void **out) {
  int dev = 0;
  LKS_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d beyond the %d the scratch table holds", dev, kMaxDevices);
    return LKS_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_error("hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
      return LKS_EDEVICE;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return LKS_OK;
}

} // namespace

// The binary16 storage rounding, element by element (lks_round_binary16).
__global__ __launch_bounds__(256) void k_round_binary16(const float *__restrict__ v,
                                                        const uint32_t *__restrict__ r,
                                                        uint16_t *__restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = __builtin_bit_cast(uint16_t, sr_f16(v[i], r[i]));
}

extern "C" {

size_t lks_mhd_state_bytes(const lks_mhd_params *p) {
  clear_error();
  Channel c;
  if (derive_channel(p, &c) != LKS_OK) return 0;
  return layout_of(c).total;
}

int lks_mhd_create(const lks_mhd_params *p, void *dev_buf, size_t bytes,
                   void *hip_stream, lks_mhd_t **out) {
  clear_error();
  if (!out) {
    set_error("out must not be NULL");
    return LKS_EINVAL;
  }
  *out = nullptr;
  Channel c;
  int rc = derive_channel(p, &c);
  if (rc != LKS_OK) return rc;
  const Layout L = layout_of(c);
  if (!dev_buf || (reinterpret_cast<uintptr_t>(dev_buf) & 255u)) {
    set_error("dev_buf must be a non-NULL 256-byte aligned device pointer");
    return LKS_EINVAL;
  }
  if (bytes < L.total) {
    set_error("dev_buf holds %zu bytes, %zu needed", bytes, L.total);
    return LKS_ENOMEM;
  }
  lks_mhd *h = new (std::nothrow) lks_mhd();
  if (!h) {
    set_error("host allocation failed");
    return LKS_ENOMEM;
  }
  h->ch = c;
  if (hipGetDevice(&h->device) != hipSuccess) h->device = 0;
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->geom = Geom{c.p.nx, c.p.ny, c.p.nx, L.plane};
  char *base = static_cast<char *>(dev_buf);
  h->buf[0] = base;
  h->buf[1] = base + L.state_bytes;
  h->rec = reinterpret_cast<double *>(base + 2 * L.state_bytes);
  h->partials = reinterpret_cast<double *>(base + 2 * L.state_bytes + L.rec_bytes);
  h->result = reinterpret_cast<double *>(base + 2 * L.state_bytes + L.rec_bytes + L.part_bytes);
  h->ctr = reinterpret_cast<uint32_t *>(base + 2 * L.state_bytes + L.rec_bytes + L.part_bytes + 256);
  h->ref = base + 2 * L.state_bytes + L.rec_bytes + L.part_bytes + 512;
  h->red_tiles_x = L.red_tiles_x;
  h->red_ntiles = L.red_ntiles;
  h->kd = make_coef<double>(c);
  // binary16 computed in FP32 takes its increments in stored units
  h->kf = make_coef<float>(c, c.p.precision == LKS_FP16_STORE ? kStoreUp16 : 1.0);
  // binary16 planes: two nodes per thread (4-byte accesses) measured fastest
  h->shape = (is_binary16(c.p.precision) && c.p.nx % 2 == 0) ? 5 : 0;
  h->rebase_every = is_binary16(c.p.precision) ? kDefaultRebase : 0;
  // solid bodies: the per-node index and the link table after the rest
  std::vector<int32_t> sidx;
  std::vector<CurvedNode> snode;
  if (c.p.nsolids > 0) {
    const char *why = nullptr;
    (void)build_solid_tables(c.p, &sidx, &snode, &why); // validated by derive_channel
    char *sb = base + L.total - L.sidx_bytes - L.snode_bytes;
    h->kd.sidx = h->kf.sidx = reinterpret_cast<const int32_t *>(sb);
    h->kd.snode = h->kf.snode = reinterpret_cast<const CurvedNode *>(sb + L.sidx_bytes);
  }
  rc = with_device(h, [&]() -> int {
    if (!sidx.empty()) {
      LKS_HIP_CHECK(hipMemcpyAsync(const_cast<int32_t *>(h->kd.sidx), sidx.data(),
                                   sidx.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                   h->stream));
      if (!snode.empty())
        LKS_HIP_CHECK(hipMemcpyAsync(const_cast<CurvedNode *>(h->kd.snode), snode.data(),
                                     snode.size() * sizeof(CurvedNode), hipMemcpyHostToDevice,
                                     h->stream));
      LKS_HIP_CHECK(hipStreamSynchronize(h->stream)); // the host vectors go out of scope
    }
    const int grid = elementwise_grid(h);
    dispatch_precision(c.p.precision, [&](auto t) {
      using S = typename decltype(t)::S;
      hipLaunchKernelGGL(k_init<S>, dim3(grid), dim3(256), 0, h->stream, h->geom, c.p.rho0,
                         static_cast<S *>(h->buf[0]), h->kd.sidx);
    });
    LKS_HIP_CHECK(hipGetLastError());
    const int r = zero_ref(h);
    return r != LKS_OK ? r : set_counter(h, 0);
  });
  if (rc != LKS_OK) {
    delete h;
    return rc;
  }
  *out = h;
  return LKS_OK;
}

int lks_mhd_destroy(lks_mhd_t *h) {
  clear_error();
  if (!h) return LKS_OK;
  drop_graphs(h);
  delete h;
  return LKS_OK;
}

int lks_mhd_set_launch_shape(lks_mhd_t *h, int32_t shape) {
  clear_error();
  if (!h || shape < 0 || shape >= kNumShapes) {
    set_error("shape must be in [0, %d)", kNumShapes);
    return LKS_EINVAL;
  }
  if (h->ch.p.nsolids > 0 && shape != 0) {
    set_error("channels with solid bodies run launch shape 0 only");
    return LKS_EINVAL;
  }
  if (h->ch.p.nx % kShapes[shape].vx != 0) {
    set_error("shape %d updates %d nodes per thread and needs nx %% %d == 0", shape,
              kShapes[shape].vx, kShapes[shape].vx);
    return LKS_EINVAL;
  }
  if (h->shape != shape) drop_graphs(h);
  h->shape = shape;
  return LKS_OK;
}

int lks_mhd_set_graph(lks_mhd_t *h, int32_t steps_per_graph) {
  clear_error();
  if (!h || steps_per_graph < 0 || (steps_per_graph % 2) != 0) {
    set_error("steps_per_graph must be an even number >= 0");
    return LKS_EINVAL;
  }
  if (steps_per_graph != 0 && h->stream == nullptr) {
    set_error("graph capture needs a non-default stream");
    return LKS_EINVAL;
  }
  drop_graphs(h);
  h->graph_steps = steps_per_graph;
  return LKS_OK;
}

int64_t lks_mhd_steps_done(const lks_mhd_t *h) { return h ? h->steps : -1; }

int lks_mhd_step(lks_mhd_t *h, int64_t nsteps) {
  clear_error();
  if (!h || nsteps < 0) {
    set_error("invalid handle or negative step count");
    return LKS_EINVAL;
  }
  return with_device(h, [&]() -> int {
    int64_t n = nsteps;
    while (n > 0) {
      if (rebase_due(h)) {
        const int rc = rebase_now(h);
        if (rc != LKS_OK) return rc;
      }
      // a graph replay must not step over a rebase point
      const int64_t to_rebase =
          h->rebase_every > 0 ? h->rebase_every - h->steps % h->rebase_every : INT64_MAX;
      if (h->graph_steps >= 2 && n >= h->graph_steps && to_rebase >= h->graph_steps) {
        if (!h->gexec[h->cur]) {
          const int rc = capture_graph(h, h->cur);
          if (rc != LKS_OK) return rc;
        }
        LKS_HIP_CHECK(hipGraphLaunch(h->gexec[h->cur], h->stream));
        h->steps += h->graph_steps;
        n -= h->graph_steps;
      } else {
        const int rc = one_step(h, MODE_STEP);
        if (rc != LKS_OK) return rc;
        n -= 1;
      }
    }
    return LKS_OK;
  });
}

int lks_mhd_run_to_steady(lks_mhd_t *h, double tol, int64_t check_every,
                          int64_t max_steps, int64_t *steps_done,
                          double *residual, double *flow_rate) {
  clear_error();
  if (!h || check_every < 2 || max_steps < 0 || !(tol >= 0.0)) {
    set_error("invalid handle, check_every < 2, max_steps < 0 or tol < 0");
    return LKS_EINVAL;
  }
  double res = NAN, q = NAN;
  int status = LKS_ENOTCONV;
  // windows rebase at their start; the plain-stepping interval is off inside
  const int64_t saved_rebase = h->rebase_every;
  h->rebase_every = 0;
  const int rc = with_device(h, [&]() -> int {
    int64_t done = 0;
    while (done + check_every <= max_steps) {
      // window of check_every steps: the first records phi, the last
      // compares phi with the record check_every - 1 steps later; binary16
      // states are rebased at the start of every window
      int rc2 = rebase_now(h);
      if (rc2 != LKS_OK) return rc2;
      if ((rc2 = one_step(h, MODE_RECORD)) != LKS_OK) return rc2;
      if (rc2 != LKS_OK) return rc2;
      if ((rc2 = lks_mhd_step(h, check_every - 2)) != LKS_OK) return rc2;
      if ((rc2 = one_step(h, MODE_RESIDUAL)) != LKS_OK) return rc2;
      hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, h->stream, h->partials, h->red_ntiles, h->result);
      LKS_HIP_CHECK(hipGetLastError());
      double sums[NRED];
      LKS_HIP_CHECK(hipMemcpyAsync(sums, h->result, sizeof sums, hipMemcpyDeviceToHost, h->stream));
      LKS_HIP_CHECK(hipStreamSynchronize(h->stream));
      done += check_every;
      const double win = (double)(check_every - 1);
      const double ru = std::sqrt(sums[0]) / std::fmax(std::sqrt(sums[1]), 1e-300) / win;
      const double rb = std::sqrt(sums[2]) / std::fmax(std::sqrt(sums[3]), 1e-300) / win;
      res = std::fmax(ru, rb);
      q = sums[4] / h->geom.nx;
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
  h->rebase_every = saved_rebase;
  if (steps_done) *steps_done = h->steps;
  if (residual) *residual = res;
  if (flow_rate) *flow_rate = q;
  return rc != LKS_OK ? rc : status;
}

int lks_mhd_moments_device(lks_mhd_t *h, double *rho, double *ux, double *uy,
                           double *bx, double *by, double *jz) {
  clear_error();
  if (!h) {
    set_error("invalid handle");
    return LKS_EINVAL;
  }
  return with_device(h, [&]() -> int {
    ObsOut oo{rho, ux, uy, bx, by, jz};
    hipError_t e = launch_mode<MODE_MOMENTS>(h, kRedShape, h->buf[h->cur], nullptr, oo);
    if (e != hipSuccess) {
      set_error("moments kernel launch failed: %s", hipGetErrorString(e));
      return LKS_EDEVICE;
    }
    return LKS_OK;
  });
}

int lks_mhd_moments(lks_mhd_t *h, double *rho, double *ux, double *uy, double *bx,
                    double *by, double *jz) {
  clear_error();
  if (!h) {
    set_error("invalid handle");
    return LKS_EINVAL;
  }
  return with_device(h, [&]() -> int {
    // two fields at a time through the record buffer (2 nx ny doubles),
    // which no step in flight uses between calls
    const long long n = (long long)h->geom.nx * h->geom.ny;
    double *host[6] = {rho, ux, uy, bx, by, jz};
    for (int pair = 0; pair < 3; ++pair) {
      double *a = host[2 * pair], *b = host[2 * pair + 1];
      if (!a && !b) continue;
      double *dev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
      if (a) dev[2 * pair] = h->rec;
      if (b) dev[2 * pair + 1] = h->rec + n;
      ObsOut oo{dev[0], dev[1], dev[2], dev[3], dev[4], dev[5]};
      hipError_t e = launch_mode<MODE_MOMENTS>(h, kRedShape, h->buf[h->cur], nullptr, oo);
      if (e != hipSuccess) {
        set_error("moments kernel launch failed: %s", hipGetErrorString(e));
        return LKS_EDEVICE;
      }
      if (a)
        LKS_HIP_CHECK(hipMemcpyAsync(a, h->rec, n * sizeof(double), hipMemcpyDeviceToHost,
                                     h->stream));
      if (b)
        LKS_HIP_CHECK(hipMemcpyAsync(b, h->rec + n, n * sizeof(double), hipMemcpyDeviceToHost,
                                     h->stream));
      LKS_HIP_CHECK(hipStreamSynchronize(h->stream));
    }
    return LKS_OK;
  });
}

int lks_mhd_save_state(lks_mhd_t *h, double *dev_pops) {
  clear_error();
  if (!h || !dev_pops) {
    set_error("invalid handle or NULL destination");
    return LKS_EINVAL;
  }
  return with_device(h, [&]() -> int {
    const int grid = elementwise_grid(h);
    dispatch_precision(h->ch.p.precision, [&](auto t) {
      using S = typename decltype(t)::S;
      // binary16 computed in FP32 decodes its FP32 references in FP64
      using C0 = typename decltype(t)::C;
      using C = std::conditional_t<kXA<S, C0>, double, C0>;
      hipLaunchKernelGGL((k_save<S, C>), dim3(grid), dim3(256), 0, h->stream, h->geom, h->ch.d.b0,
                         static_cast<const S *>(h->buf[h->cur]), ref_of<S, C>(h), dev_pops);
    });
    LKS_HIP_CHECK(hipGetLastError());
    return LKS_OK;
  });
}

int lks_mhd_load_state(lks_mhd_t *h, const double *dev_pops, int64_t steps) {
  clear_error();
  if (!h || !dev_pops || steps < 0) {
    set_error("invalid handle, NULL source or negative step count");
    return LKS_EINVAL;
  }
  return with_device(h, [&]() -> int {
    const int grid = elementwise_grid(h);
    dispatch_precision(h->ch.p.precision, [&](auto t) {
      using S = typename decltype(t)::S;
      hipLaunchKernelGGL(k_load<S>, dim3(grid), dim3(256), 0, h->stream, h->geom, h->ch.d.b0,
                         dev_pops, static_cast<S *>(h->buf[h->cur]));
    });
    LKS_HIP_CHECK(hipGetLastError());
    const int r = zero_ref(h);
    if (r != LKS_OK) return r;
    h->steps = steps;
    return set_counter(h, steps);
  });
}

int lks_mhd_rebase(lks_mhd_t *h) {
  clear_error();
  if (!h) {
    set_error("invalid handle");
    return LKS_EINVAL;
  }
  return with_device(h, [&]() -> int { return rebase_now(h); });
}

int lks_mhd_advance_noalloc(const lks_mhd_params *p, double *dev_pops, int64_t step0,
                            int64_t nsteps, void *hip_stream) {
  clear_error();
  if (!dev_pops || step0 < 0 || nsteps < 0) {
    set_error("NULL populations or negative step count");
    return LKS_EINVAL;
  }
  Channel c;
  int rc = derive_channel(p, &c);
  if (rc != LKS_OK) return rc;
  if (c.p.nsolids > 0) {
    set_error("channels with solid bodies need lks_mhd_create (their tables are uploaded)");
    return LKS_EINVAL;
  }
  const Layout L = layout_of(c);
  if (L.total > kScratchBytes) {
    set_error("channel needs %zu bytes of working memory, the scratch array holds %zu", L.total,
              kScratchBytes);
    return LKS_ENOMEM;
  }
  void *base_ptr = nullptr;
  if ((rc = scratch_address(&base_ptr)) != LKS_OK) return rc;
  // a handle on the stack over the scratch array, carved as lks_mhd_create
  // carves the caller's buffer (no graphs: plain launches)
  lks_mhd h;
  h.ch = c;
  if (hipGetDevice(&h.device) != hipSuccess) h.device = 0;
  h.stream = static_cast<hipStream_t>(hip_stream);
  h.geom = Geom{c.p.nx, c.p.ny, c.p.nx, L.plane};
  char *base = static_cast<char *>(base_ptr);
  h.buf[0] = base;
  h.buf[1] = base + L.state_bytes;
  h.rec = reinterpret_cast<double *>(base + 2 * L.state_bytes);
  h.partials = reinterpret_cast<double *>(base + 2 * L.state_bytes + L.rec_bytes);
  h.result = reinterpret_cast<double *>(base + 2 * L.state_bytes + L.rec_bytes + L.part_bytes);
  h.ctr = reinterpret_cast<uint32_t *>(base + 2 * L.state_bytes + L.rec_bytes + L.part_bytes + 256);
  h.ref = base + 2 * L.state_bytes + L.rec_bytes + L.part_bytes + 512;
  h.red_tiles_x = L.red_tiles_x;
  h.red_ntiles = L.red_ntiles;
  h.kd = make_coef<double>(c);
  h.kf = make_coef<float>(c, c.p.precision == LKS_FP16_STORE ? kStoreUp16 : 1.0);
  h.shape = (is_binary16(c.p.precision) && c.p.nx % 2 == 0) ? 5 : 0;
  h.rebase_every = is_binary16(c.p.precision) ? kDefaultRebase : 0;
  // load (as lks_mhd_load_state), step (as lks_mhd_step), save
  const int grid = elementwise_grid(&h);
  dispatch_precision(c.p.precision, [&](auto t) {
    using S = typename decltype(t)::S;
    hipLaunchKernelGGL(k_load<S>, dim3(grid), dim3(256), 0, h.stream, h.geom, c.d.b0, dev_pops,
                       static_cast<S *>(h.buf[0]));
  });
  LKS_HIP_CHECK(hipGetLastError());
  if ((rc = zero_ref(&h)) != LKS_OK) return rc;
  hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(64), 0, h.stream, h.ctr, (uint32_t)step0);
  LKS_HIP_CHECK(hipGetLastError());
  h.steps = step0;
  if ((rc = lks_mhd_step(&h, nsteps)) != LKS_OK) return rc;
  rc = lks_mhd_save_state(&h, dev_pops);
  drop_graphs(&h);
  return rc;
}

int lks_round_binary16(const float *v, const uint32_t *r, uint16_t *out, int64_t n,
                       void *hip_stream) {
  clear_error();
  if (n < 0 || n > INT32_MAX || (n > 0 && (!v || !r || !out))) {
    set_error("invalid arrays or element count");
    return LKS_EINVAL;
  }
  if (n == 0) return LKS_OK;
  hipLaunchKernelGGL(k_round_binary16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(hip_stream), v, r, out, n);
  LKS_HIP_CHECK(hipGetLastError());
  return LKS_OK;
}

int lks_mhd_set_rebase(lks_mhd_t *h, int64_t every) {
  clear_error();
  if (!h || every < 0) {
    set_error("invalid handle or negative rebase interval");
    return LKS_EINVAL;
  }
  h->rebase_every = is_binary16(h->ch.p.precision) ? every : 0;
  return LKS_OK;
}

} // extern "C"
