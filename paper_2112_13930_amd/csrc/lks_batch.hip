// Batched channels: many independent channels of uneven size advanced by one
// persistent launch per step over a packed device tile list.
//
// Pool layout (caller-owned device memory):
//   [channel descriptors][tile list][tile count][per-tile partials]
//   [per-slot sums][channel states ...]
// A channel's region holds its two population buffers, its record buffer and
// its row references.
// The step kernel reads the tile count and the descriptors from device
// memory, so admitting or retiring channels rewrites that memory and never
// needs a new launch configuration: a captured two-step graph stays valid.
//
// Every node is updated by the same node_update() as the single-channel
// kernel, so a channel's populations are bitwise those of a solo run with the
// same precision and step count.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <type_traits>
#include <vector>

#include "lks_aux.hpp"
#include "lks_common.hpp"

namespace lks {

struct ChanDesc {
  void *buf[2];
  double *rec;
  void *ref; // row references [ny][19] of the compute type
  Geom g;
  int bc;         // scheme: wall scheme | COLL_TRT for the TRT or MRT collision
  int phase;      // buffer holding the state when the global parity is 0
  int tile_first; // first tile of this channel in the list
  int tile_count;
  uint32_t step_base; // global step count at admission
  // node index -> row without a hardware divide: y = (umulhi(i, m) + i) >> s
  // with s = ceil(log2 nx), m = floor(2^32 (2^s - nx) / nx) + 1 (exact for
  // every i < 2^31)
  uint32_t nx_magic;
  int nx_shift;
  Coef<float> kf;
  Coef<double> kd;
};

// A tile is the work of one 256-thread block: either a w x h rectangle of a
// channel (w * h == 256, x0/y0 its corner) or, with w == 0, a run of n <=
// 256 * h consecutive nodes of the channel's [ny][nx] planes starting at node
// x0 (thread t takes the nodes t, t + 256, ... below n).  Linear tiles keep
// every wavefront on 64 consecutive addresses whatever the channel width.
struct Tile {
  int chan;
  int x0, y0;
  int w, h;
  int n;
  int pad[2];
};

// Binary16 storage with FP32 arithmetic reads 19 FP32 and 19 FP64 table
// entries per node from its row (XTabs V and K).  The batched kernel copies
// the rows a tile touches into LDS first: rows differ between the lanes of a
// wavefront, and per-lane reads of the tables from memory would cost the
// vector memory path more than the populations themselves.  A tile spans at
// most kStageRows rows (linear tiles are cut to (kStageRows - 1) nx nodes).
constexpr int kStageRows = 64;

// Grid of the step launch: the next power of two above the tile count, at
// most batch_blocks_per_cu blocks per CU (power-of-two buckets keep a
// captured graph valid while channels come and go).  Measured on the
// 256-channel mix: FP32 storage runs fastest with a block per tile (38.4
// against 35.9 G node updates/s at 64 blocks per CU), binary16 with FP32
// arithmetic, which stages row tables per tile, at 64 blocks per CU (46.5
// against 45.4 at 32 and 45.2 at 256).
int batch_blocks_per_cu(int precision) { return precision == LKS_FP16_STORE ? 64 : 1024; }

constexpr int kTileThreads = 256;
// Steps in the long captured graph (even: a graph starts and ends at parity 0).
constexpr int kLongGraphSteps = 16;
constexpr int kWidthClasses = 7;
constexpr int NREDB = 6;

// MRT channels run through the TRT scheme with their corrections switched on
// per channel (MRT_RT).

template <typename C> __device__ __forceinline__ const Coef<C> &coef_of(const ChanDesc &c);
template <> __device__ __forceinline__ const Coef<float> &coef_of<float>(const ChanDesc &c) { return c.kf; }
template <> __device__ __forceinline__ const Coef<double> &coef_of<double>(const ChanDesc &c) { return c.kd; }

// Waves per SIMD the step asks the compiler for (1: no constraint).  Every
// variant runs unconstrained: FP32 storage takes 82 registers (5 waves) with
// the BGK schemes alone and 112 (4) with the TRT/MRT ones; binary16 with
// FP32 arithmetic 93 (5), with FP64 arithmetic 104 (4).  Asking the FP32
// BGK step for 6 waves spills.
template <typename S, typename C, int MODE, bool TRT>
constexpr int kBatchWaves = 1;

// gctr[2]: global step counters as in the single-channel kernel; a channel's
// own step index is gctr[parity] - step_base.
// TRT: the pool holds TRT or MRT channels (else only BGK ones, and the
// kernel is built for those two schemes alone, with fewer registers).
template <typename S, typename C, int MODE, bool TRT>
__global__ __launch_bounds__(kTileThreads, (kBatchWaves<S, C, MODE, TRT>)) void k_batch_step(
    const ChanDesc *__restrict__ chans, const Tile *__restrict__ tiles,
    const int *__restrict__ ntiles_dev, int parity, double *__restrict__ partials,
    uint32_t *__restrict__ gctr) {
  constexpr bool SR = kUseSR<S, C>;
  constexpr bool XA = kXA<S, C>;
  const uint32_t gstep = gctr[parity];
  if (blockIdx.x == 0 && threadIdx.x == 0) gctr[parity ^ 1] = gstep + 1u;
  const int nt = *ntiles_dev;
  __shared__ double lds[(kTileThreads / 64) * NREDB];
  __shared__ __align__(16) float sV[XA ? kStageRows * kRefRow : 4];
  __shared__ __align__(16) double sK[XA ? kStageRows * kRefRow : 2];
  // Tiles of consecutive nodes share the cache lines at their boundaries.
  // The hardware deals workgroups round-robin to the 8 XCDs, each with its
  // own L2: within every group of 64 blocks, XCD j's 8 blocks take 8
  // consecutive tiles, so that 7 of 8 tile boundaries stay within one L2
  // while the whole grid still sweeps the tile list in order.
  int t_first = blockIdx.x;
  if ((gridDim.x & 63) == 0) {
    const int b = blockIdx.x;
    t_first = (b & ~63) | ((b & 7) << 3) | ((b >> 3) & 7);
  }
  for (int t = t_first; t < nt; t += gridDim.x) { // uniform per block
    const Tile tl = tiles[t];
    const ChanDesc &c = chans[tl.chan];
    const int cur = parity ^ c.phase;
    const S *src = static_cast<const S *>(c.buf[cur]);
    S *dst = static_cast<S *>(c.buf[cur ^ 1]);
    const uint32_t sseed = SR ? step_seed(gstep - c.step_base) : 0u;
    double v[NREDB] = {0, 0, 0, 0, 0, 0};
    auto row_of = [&](uint32_t i) -> int {
      return (int)(((uint64_t)__umulhi(i, c.nx_magic) + i) >> c.nx_shift);
    };
    // first row of the tile's rows staged in LDS
    int ya = 0;
    if constexpr (XA) {
      int yb;
      if (tl.w == 0) {
        ya = row_of((uint32_t)tl.x0);
        yb = row_of((uint32_t)(tl.x0 + tl.n - 1));
      } else {
        ya = tl.y0;
        yb = min(c.g.ny - 1, tl.y0 + tl.h - 1);
      }
      const int cnt = min(yb - ya + 1, kStageRows) * kRefRow;
      const XTabs xt = xtabs_of(c.ref, c.g.ny);
      const float *gV = xt.V + (long long)ya * kRefRow;
      const double *gK = xt.K + (long long)ya * kRefRow;
      __syncthreads(); // the previous tile's nodes have read their rows
      for (int j = threadIdx.x; j < cnt; j += kTileThreads) {
        sV[j] = gV[j];
        sK[j] = gK[j];
      }
      __syncthreads();
    }
    auto one = [&](int x, int y) {
      NodeObs<C> o{};
      const C *ref = static_cast<const C *>(c.ref);
      const float *xV = XA ? sV + (y - ya) * kRefRow : nullptr;
      const double *xK = XA ? sK + (y - ya) * kRefRow : nullptr;
      if constexpr (TRT) {
        switch (c.bc) { // uniform per block
        case BC_LINK:
          node_update<S, C, BC_LINK | IN_BATCH, MODE, SR, XA>(c.g, coef_of<C>(c), src, ref, dst,
                                                              x, y, o, sseed, xV, xK);
          break;
        case BC_MOMENT:
          node_update<S, C, BC_MOMENT | IN_BATCH, MODE, SR, XA>(c.g, coef_of<C>(c), src, ref,
                                                                dst, x, y, o, sseed, xV, xK);
          break;
        case BC_LINK | COLL_TRT:
          node_update<S, C, BC_LINK | COLL_TRT | MRT_RT | IN_BATCH, MODE, SR, XA>(
              c.g, coef_of<C>(c), src, ref, dst, x, y, o, sseed, xV, xK);
          break;
        default:
          node_update<S, C, BC_MOMENT | COLL_TRT | MRT_RT | IN_BATCH, MODE, SR, XA>(
              c.g, coef_of<C>(c), src, ref, dst, x, y, o, sseed, xV, xK);
          break;
        }
      } else if (c.bc == BC_LINK) { // uniform per block
        node_update<S, C, BC_LINK | IN_BATCH, MODE, SR, XA>(c.g, coef_of<C>(c), src, ref, dst, x,
                                                            y, o, sseed, xV, xK);
      } else {
        node_update<S, C, BC_MOMENT | IN_BATCH, MODE, SR, XA>(c.g, coef_of<C>(c), src, ref, dst,
                                                              x, y, o, sseed, xV, xK);
      }
      const long long i = (long long)y * c.g.nx + x;
      const long long n = (long long)c.g.nx * c.g.ny;
      if constexpr (MODE == MODE_RECORD) {
        c.rec[i] = (double)o.ux;
        c.rec[n + i] = (double)o.bx;
      }
      if constexpr (MODE == MODE_RESIDUAL) {
        const double u = (double)o.ux, b = (double)o.bx;
        const double du = u - c.rec[i], db = b - c.rec[n + i];
        v[0] += du * du;
        v[1] += u * u;
        v[2] += db * db;
        v[3] += b * b;
        v[4] += u;
        const bool ok = isfinite((double)o.rho) && isfinite(u) && isfinite((double)o.uy) &&
                        isfinite(b) && isfinite((double)o.by) && (double)o.rho > 0.0 &&
                        fabs(u) < 1.0 && fabs((double)o.uy) < 1.0;
        v[5] += ok ? 0.0 : 1.0;
      }
    };
    // one call site of the node update for both tile kinds (a rectangle is
    // one pass), so that each scheme's code is inlined once
    const int passes = tl.w == 0 ? tl.h : 1;
    for (int j = 0; j < passes; ++j) {
      int x, y;
      bool in;
      if (tl.w == 0) {
        const int li = (int)threadIdx.x + j * kTileThreads;
        const int i = tl.x0 + li;
        y = row_of((uint32_t)i);
        x = i - y * c.g.nx;
        in = li < tl.n;
      } else {
        const int lx = (int)threadIdx.x % tl.w;
        const int ly = (int)threadIdx.x / tl.w;
        x = tl.x0 + lx;
        y = tl.y0 + ly;
        in = (ly < tl.h) && (x < c.g.nx) && (y < c.g.ny);
      }
      if (in) one(x, y);
    }
    if constexpr (MODE == MODE_RESIDUAL) {
      block_sum<NREDB, kTileThreads>(v, lds);
      if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NREDB; ++j) partials[(long long)t * 8 + j] = v[j];
      }
      __syncthreads(); // lds is reused by the next tile
    }
  }
}

// Per-slot fixed-order sums of the slot's tile partials (one block per slot).
__global__ __launch_bounds__(64) void k_batch_finalize(const ChanDesc *__restrict__ chans,
                                                       const int *__restrict__ active,
                                                       const double *__restrict__ partials,
                                                       double *__restrict__ sums) {
  const int slot = blockIdx.x;
  if (!active[slot]) return;
  const ChanDesc &c = chans[slot];
  double v[NREDB] = {0, 0, 0, 0, 0, 0};
  for (int t = threadIdx.x; t < c.tile_count; t += 64)
#pragma unroll
    for (int j = 0; j < NREDB; ++j) v[j] += partials[(long long)(c.tile_first + t) * 8 + j];
  wave_sum<NREDB>(v);
  if (threadIdx.x == 0)
    for (int j = 0; j < NREDB; ++j) sums[(long long)slot * 8 + j] = v[j];
}

// Observables of one channel (no collision), FP64 outputs.
struct ObsOutB {
  double *rho, *ux, *uy, *bx, *by, *jz;
};

template <typename S, typename C, int BC>
__global__ __launch_bounds__(256) void k_chan_moments(Geom g, Coef<C> k, const S *__restrict__ src,
                                                      const C *__restrict__ ref, ObsOutB oo) {
  const long long n = (long long)g.nx * g.ny;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int y = (int)(i / g.nx), x = (int)(i - (long long)y * g.nx);
  NodeObs<C> o{};
  node_update<S, C, BC, MODE_MOMENTS, false>(g, k, src, ref, nullptr, x, y, o, 0u);
  if (oo.rho) oo.rho[i] = 1.0 + (double)o.rhop;
  if (oo.ux) oo.ux[i] = (double)o.ux;
  if (oo.uy) oo.uy[i] = (double)o.uy;
  if (oo.bx) oo.bx[i] = (double)o.bx;
  if (oo.by) oo.by[i] = (double)o.by;
  if (oo.jz) oo.jz[i] = (double)o.jz;
}

// Row rebase of every active binary16 channel: block (row, slot).
template <typename S, typename C>
__global__ __launch_bounds__(256) void k_batch_rebase(const ChanDesc *__restrict__ chans,
                                                      const int *__restrict__ active, int parity,
                                                      const uint32_t *__restrict__ gctr) {
  __shared__ double lds[5 * 19];
  const int slot = blockIdx.y, y = blockIdx.x;
  if (!active[slot]) return;
  const ChanDesc &c = chans[slot];
  if (y >= c.g.ny) return;
  const int cur = parity ^ c.phase;
  rebase_row<S, C, kUseSR<S, C>>(static_cast<S *>(c.buf[cur]),
                                 static_cast<C *>(c.ref) + (long long)y * kRefRow, c.g, y,
                                 rebase_seed(gctr[parity] - c.step_base), lds);
}

// Pre-collision tables of every active channel after a rebase (binary16
// computed in FP32): block (row group, slot).
__global__ __launch_bounds__(256) void k_batch_xtables(const ChanDesc *__restrict__ chans,
                                                       const int *__restrict__ active) {
  const int slot = blockIdx.y;
  if (!active[slot]) return;
  const ChanDesc &c = chans[slot];
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= c.g.ny) return;
  if (wall_of(c.bc) == BC_LINK) xtab_row<BC_LINK>(c.g, c.kd, xtabs_of(c.ref, c.g.ny), y);
  else xtab_row<BC_MOMENT>(c.g, c.kd, xtabs_of(c.ref, c.g.ny), y);
}

} // namespace lks

using namespace lks;

namespace {

struct Slot {
  bool used = false;
  Channel ch;
  size_t offset = 0, bytes = 0; // region in the pool
  int64_t admit_step = 0;        // global step count at admission
  int width_class = 0;
};

struct Region {
  size_t offset, bytes;
};

} // namespace

struct lks_mhd_batch {
  int precision = LKS_FP32;
  int device = 0;
  hipStream_t stream = nullptr;
  int max_channels = 0;
  int64_t max_nodes = 0;
  int max_tiles = 0;
  char *pool = nullptr;
  size_t pool_bytes = 0;
  // carved device arrays
  ChanDesc *d_chans = nullptr;
  Tile *d_tiles = nullptr;
  int *d_ntiles = nullptr;
  int *d_active = nullptr;
  double *d_partials = nullptr;
  double *d_sums = nullptr;
  uint32_t *d_gctr = nullptr;
  size_t heap_begin = 0;
  std::vector<Region> free_list; // sorted by offset
  std::vector<Slot> slots;
  std::vector<ChanDesc> h_chans;
  std::vector<Tile> h_tiles;
  std::vector<int> h_active;
  // tile shape per width class: (w, h) as in Tile; default linear, 256 nodes
  int tile_w[kWidthClasses] = {0, 0, 0, 0, 0, 0, 0};
  int tile_h[kWidthClasses] = {1, 1, 1, 1, 1, 1, 1};
  int64_t global_steps = 0;
  int parity = 0;
  int64_t nodes = 0;
  int nactive = 0;
  int grid = 0, grid_cap = 0;
  bool dirty = false;
  bool any_trt = false; // an active channel runs the TRT or MRT collision
  hipGraphExec_t gexec = nullptr;      // two steps
  hipGraphExec_t gexec_long = nullptr; // kLongGraphSteps steps
};

namespace {

size_t overhead(int max_channels, int max_tiles) {
  size_t b = 0;
  b += align256((size_t)max_channels * sizeof(ChanDesc));
  b += align256((size_t)max_tiles * sizeof(Tile));
  b += 256;                                            // tile count
  b += align256((size_t)max_channels * sizeof(int));   // active flags
  b += align256((size_t)max_tiles * 8 * sizeof(double));
  b += align256((size_t)max_channels * 8 * sizeof(double));
  b += 256; // global step counters
  return b;
}

int tiles_for(int64_t max_nodes, int max_channels) {
  // Every tile of a channel except its last column / row of tiles is full;
  // 32 nodes per tile on average is a safe lower bound for any shape table.
  const int64_t t = max_nodes / 32 + 8LL * max_channels + 64;
  return (int)std::min<int64_t>(t, (1LL << 30));
}

int width_class_of(int nx) {
  int k = 0;
  int lim = 8;
  while (k < kWidthClasses - 1 && nx > lim) {
    lim *= 2;
    ++k;
  }
  return k;
}

size_t channel_region_bytes(const Channel &c, int precision) {
  const long long plane = plane_elems(c.p.nx, c.p.ny, precision);
  const size_t state = align256((size_t)19 * plane * elem_bytes(precision));
  const size_t rec = align256((size_t)2 * c.p.nx * c.p.ny * sizeof(double));
  const size_t ref = ref_area_bytes(c.p.ny, precision);
  return 2 * state + rec + ref;
}

template <typename C> const Coef<C> &coef_host(const ChanDesc &d);
template <> const Coef<float> &coef_host<float>(const ChanDesc &d) { return d.kf; }
template <> const Coef<double> &coef_host<double>(const ChanDesc &d) { return d.kd; }

template <typename F>
int with_device(lks_mhd_batch *b, F &&fn) {
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) prev = b->device;
  if (prev != b->device) LKS_HIP_CHECK(hipSetDevice(b->device));
  const int rc = fn();
  if (prev != b->device) (void)hipSetDevice(prev);
  return rc;
}

bool pool_alloc(lks_mhd_batch *b, size_t bytes, size_t *off) {
  for (size_t i = 0; i < b->free_list.size(); ++i) {
    Region &r = b->free_list[i];
    if (r.bytes >= bytes) {
      *off = r.offset;
      r.offset += bytes;
      r.bytes -= bytes;
      if (r.bytes == 0) b->free_list.erase(b->free_list.begin() + i);
      return true;
    }
  }
  return false;
}

void pool_free(lks_mhd_batch *b, size_t off, size_t bytes) {
  auto it = std::lower_bound(b->free_list.begin(), b->free_list.end(), off,
                             [](const Region &r, size_t o) { return r.offset < o; });
  it = b->free_list.insert(it, Region{off, bytes});
  // merge with neighbours
  const size_t i = it - b->free_list.begin();
  if (i + 1 < b->free_list.size() &&
      b->free_list[i].offset + b->free_list[i].bytes == b->free_list[i + 1].offset) {
    b->free_list[i].bytes += b->free_list[i + 1].bytes;
    b->free_list.erase(b->free_list.begin() + i + 1);
  }
  if (i > 0 && b->free_list[i - 1].offset + b->free_list[i - 1].bytes == b->free_list[i].offset) {
    b->free_list[i - 1].bytes += b->free_list[i].bytes;
    b->free_list.erase(b->free_list.begin() + i);
  }
}

// Nodes of a full linear tile of h nodes per thread.
long long linear_tile_nodes(int precision, int nx, int h) {
  const long long per = (long long)kTileThreads * h;
  if (precision == LKS_FP16_STORE) return std::min(per, (long long)(kStageRows - 1) * nx);
  return per;
}

// Tiles of one channel for a tile shape (w, h) (w == 0: linear).
int count_tiles(int precision, int nx, int ny, int w, int h) {
  if (w == 0) {
    const long long per = linear_tile_nodes(precision, nx, h);
    return (int)(((long long)nx * ny + per - 1) / per);
  }
  return ((nx + w - 1) / w) * ((ny + h - 1) / h);
}

int total_tiles(const lks_mhd_batch *b, const int *tile_w, const int *tile_h) {
  long long t = 0;
  for (const Slot &s : b->slots)
    if (s.used)
      t += count_tiles(b->precision, s.ch.p.nx, s.ch.p.ny, tile_w[s.width_class],
                       tile_h[s.width_class]);
  return t > (1LL << 30) ? (1 << 30) : (int)t;
}

// Rebuild descriptors' tile ranges and the tile list; upload both.
int rebuild(lks_mhd_batch *b) {
  b->h_tiles.clear();
  for (int s = 0; s < b->max_channels; ++s) {
    Slot &sl = b->slots[s];
    ChanDesc &d = b->h_chans[s];
    if (!sl.used) {
      d.tile_first = 0;
      d.tile_count = 0;
      continue;
    }
    const int w = b->tile_w[sl.width_class];
    const int h = b->tile_h[sl.width_class];
    d.tile_first = (int)b->h_tiles.size();
    if (w == 0) {
      const long long nn = (long long)sl.ch.p.nx * sl.ch.p.ny;
      const long long per = linear_tile_nodes(b->precision, sl.ch.p.nx, h);
      for (long long i0 = 0; i0 < nn; i0 += per)
        b->h_tiles.push_back(Tile{s, (int)i0, 0, 0, h, (int)std::min(per, nn - i0), {0, 0}});
    } else {
      for (int y0 = 0; y0 < sl.ch.p.ny; y0 += h)
        for (int x0 = 0; x0 < sl.ch.p.nx; x0 += w)
          b->h_tiles.push_back(Tile{s, x0, y0, w, h, w * h, {0, 0}});
    }
    d.tile_count = (int)b->h_tiles.size() - d.tile_first;
  }
  if ((int)b->h_tiles.size() > b->max_tiles) {
    set_error("tile list of %zu tiles exceeds the capacity %d", b->h_tiles.size(), b->max_tiles);
    return LKS_ENOMEM;
  }
  const int nt = (int)b->h_tiles.size();
  LKS_HIP_CHECK(hipMemcpyAsync(b->d_chans, b->h_chans.data(), b->max_channels * sizeof(ChanDesc),
                               hipMemcpyHostToDevice, b->stream));
  if (nt > 0)
    LKS_HIP_CHECK(hipMemcpyAsync(b->d_tiles, b->h_tiles.data(), nt * sizeof(Tile),
                                 hipMemcpyHostToDevice, b->stream));
  LKS_HIP_CHECK(hipMemcpyAsync(b->d_ntiles, &nt, sizeof(int), hipMemcpyHostToDevice, b->stream));
  LKS_HIP_CHECK(hipMemcpyAsync(b->d_active, b->h_active.data(), b->max_channels * sizeof(int),
                               hipMemcpyHostToDevice, b->stream));
  LKS_HIP_CHECK(hipStreamSynchronize(b->stream)); // host vectors may change next
  b->dirty = false;
  int grid = 1;
  while (grid < nt && grid < b->grid_cap) grid *= 2;
  if (grid > b->grid_cap) grid = b->grid_cap;
  bool any_trt = false;
  for (int s = 0; s < b->max_channels; ++s)
    if (b->slots[s].used && (b->h_chans[s].bc & COLL_TRT)) any_trt = true;
  if (grid != b->grid || any_trt != b->any_trt) {
    // the captured graphs hold the old launch size and kernel
    b->grid = grid;
    b->any_trt = any_trt;
    if (b->gexec) {
      (void)hipGraphExecDestroy(b->gexec);
      b->gexec = nullptr;
    }
    if (b->gexec_long) {
      (void)hipGraphExecDestroy(b->gexec_long);
      b->gexec_long = nullptr;
    }
  }
  return LKS_OK;
}

template <int MODE>
hipError_t launch_batch(lks_mhd_batch *b, int parity) {
  dispatch_precision(b->precision, [&](auto t) {
    using S = typename decltype(t)::S;
    using C = typename decltype(t)::C;
    if (b->any_trt)
      hipLaunchKernelGGL((k_batch_step<S, C, MODE, true>), dim3(b->grid), dim3(kTileThreads), 0,
                         b->stream, b->d_chans, b->d_tiles, b->d_ntiles, parity, b->d_partials,
                         b->d_gctr);
    else
      hipLaunchKernelGGL((k_batch_step<S, C, MODE, false>), dim3(b->grid), dim3(kTileThreads), 0,
                         b->stream, b->d_chans, b->d_tiles, b->d_ntiles, parity, b->d_partials,
                         b->d_gctr);
  });
  return hipGetLastError();
}

int batch_one(lks_mhd_batch *b, int mode) {
  hipError_t e;
  switch (mode) {
  case MODE_STEP: e = launch_batch<MODE_STEP>(b, b->parity); break;
  case MODE_RECORD: e = launch_batch<MODE_RECORD>(b, b->parity); break;
  default: e = launch_batch<MODE_RESIDUAL>(b, b->parity); break;
  }
  if (e != hipSuccess) {
    set_error("batched step launch failed: %s", hipGetErrorString(e));
    return LKS_EDEVICE;
  }
  b->parity ^= 1;
  b->global_steps += 1;
  return LKS_OK;
}

int capture(lks_mhd_batch *b, int nsteps, hipGraphExec_t *out) {
  hipGraph_t graph = nullptr;
  LKS_HIP_CHECK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  const int p0 = b->parity;
  const int64_t s0 = b->global_steps;
  b->parity = 0;
  int rc = LKS_OK;
  for (int i = 0; i < nsteps && rc == LKS_OK; ++i) rc = batch_one(b, MODE_STEP);
  b->parity = p0;
  b->global_steps = s0;
  hipError_t e = hipStreamEndCapture(b->stream, &graph);
  if (rc != LKS_OK) return rc;
  if (e != hipSuccess) {
    set_error("hipStreamEndCapture failed: %s", hipGetErrorString(e));
    return LKS_EDEVICE;
  }
  e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    set_error("hipGraphInstantiate failed: %s", hipGetErrorString(e));
    return LKS_EDEVICE;
  }
  return LKS_OK;
}

// Write the global step count into the device counter the next launch reads
// (used when steps are counted without a launch).
int sync_counter(lks_mhd_batch *b) {
  const uint32_t v[2] = {(uint32_t)b->global_steps, (uint32_t)b->global_steps};
  LKS_HIP_CHECK(hipMemcpyAsync(b->d_gctr, v, sizeof v, hipMemcpyHostToDevice, b->stream));
  LKS_HIP_CHECK(hipStreamSynchronize(b->stream));
  return LKS_OK;
}

// Row rebase of every active channel (binary16 storage only).
int batch_rebase(lks_mhd_batch *b) {
  if (!is_binary16(b->precision) || b->nactive == 0) return LKS_OK;
  if (b->dirty) {
    const int rc = rebuild(b);
    if (rc != LKS_OK) return rc;
  }
  int max_ny = 1, top = 0;
  for (int s = 0; s < b->max_channels; ++s)
    if (b->slots[s].used) {
      max_ny = std::max(max_ny, b->slots[s].ch.p.ny);
      top = s + 1;
    }
  dispatch_precision(b->precision, [&](auto t) {
    using S = typename decltype(t)::S;
    using C = typename decltype(t)::C;
    if constexpr (kRowRef<S>)
      hipLaunchKernelGGL((k_batch_rebase<S, C>), dim3(max_ny, top), dim3(256), 0, b->stream,
                         b->d_chans, b->d_active, b->parity, b->d_gctr);
  });
  LKS_HIP_CHECK(hipGetLastError());
  if (b->precision == LKS_FP16_STORE) {
    hipLaunchKernelGGL(k_batch_xtables, dim3((max_ny + 255) / 256, top), dim3(256), 0, b->stream,
                       b->d_chans, b->d_active);
    LKS_HIP_CHECK(hipGetLastError());
  }
  return LKS_OK;
}

int batch_steps(lks_mhd_batch *b, int64_t n, bool use_graph) {
  if (b->dirty) {
    const int rc = rebuild(b);
    if (rc != LKS_OK) return rc;
  }
  if (b->nactive == 0) {
    b->global_steps += n; // nothing to advance; keep parity bookkeeping
    b->parity ^= (int)(n & 1);
    return sync_counter(b);
  }
  if (use_graph && b->stream == nullptr) {
    set_error("graph capture needs a non-default stream");
    return LKS_EINVAL;
  }
  while (n > 0) {
    if (use_graph && n >= kLongGraphSteps && b->parity == 0) {
      if (!b->gexec_long) {
        const int rc = capture(b, kLongGraphSteps, &b->gexec_long);
        if (rc != LKS_OK) return rc;
      }
      LKS_HIP_CHECK(hipGraphLaunch(b->gexec_long, b->stream));
      b->global_steps += kLongGraphSteps;
      n -= kLongGraphSteps;
    } else if (use_graph && n >= 2 && b->parity == 0) {
      if (!b->gexec) {
        const int rc = capture(b, 2, &b->gexec);
        if (rc != LKS_OK) return rc;
      }
      LKS_HIP_CHECK(hipGraphLaunch(b->gexec, b->stream));
      b->global_steps += 2;
      n -= 2;
    } else {
      const int rc = batch_one(b, MODE_STEP);
      if (rc != LKS_OK) return rc;
      n -= 1;
    }
  }
  return LKS_OK;
}

template <typename S>
void launch_init(lks_mhd_batch *b, const Slot &s, void *buf) {
  const long long n = (long long)s.ch.p.nx * s.ch.p.ny;
  const Geom g{s.ch.p.nx, s.ch.p.ny, s.ch.p.nx, plane_elems(s.ch.p.nx, s.ch.p.ny, b->precision)};
  hipLaunchKernelGGL(k_init<S>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, b->stream, g,
                     s.ch.p.rho0, static_cast<S *>(buf));
}

} // namespace

extern "C" {

size_t lks_mhd_batch_overhead_bytes(int32_t max_channels, int64_t max_nodes) {
  if (max_channels <= 0 || max_nodes <= 0) return 0;
  return overhead(max_channels, tiles_for(max_nodes, max_channels));
}

size_t lks_mhd_batch_channel_bytes(const lks_mhd_params *p, int32_t precision) {
  clear_error();
  Channel c;
  if (derive_channel(p, &c) != LKS_OK) return 0;
  if (!valid_precision(precision)) return 0;
  return channel_region_bytes(c, precision);
}

int lks_mhd_batch_create(int32_t precision, int32_t max_channels, int64_t max_nodes,
                         void *dev_pool, size_t pool_bytes, void *hip_stream,
                         lks_mhd_batch_t **out) {
  clear_error();
  if (!out || max_channels <= 0 || max_channels > 65535 || max_nodes <= 0 ||
      !valid_precision(precision)) {
    set_error("invalid batch arguments");
    return LKS_EINVAL;
  }
  *out = nullptr;
  if (!dev_pool || (reinterpret_cast<uintptr_t>(dev_pool) & 255u)) {
    set_error("dev_pool must be a non-NULL 256-byte aligned device pointer");
    return LKS_EINVAL;
  }
  const int max_tiles = tiles_for(max_nodes, max_channels);
  const size_t ov = overhead(max_channels, max_tiles);
  if (pool_bytes < ov) {
    set_error("pool holds %zu bytes, the batch tables alone need %zu", pool_bytes, ov);
    return LKS_ENOMEM;
  }
  lks_mhd_batch *b = new (std::nothrow) lks_mhd_batch();
  if (!b) {
    set_error("host allocation failed");
    return LKS_ENOMEM;
  }
  b->precision = precision;
  if (hipGetDevice(&b->device) != hipSuccess) b->device = 0;
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->max_channels = max_channels;
  b->max_nodes = max_nodes;
  b->max_tiles = max_tiles;
  b->pool = static_cast<char *>(dev_pool);
  b->pool_bytes = pool_bytes;
  char *p = b->pool;
  b->d_chans = reinterpret_cast<ChanDesc *>(p);
  p += align256((size_t)max_channels * sizeof(ChanDesc));
  b->d_tiles = reinterpret_cast<Tile *>(p);
  p += align256((size_t)max_tiles * sizeof(Tile));
  b->d_ntiles = reinterpret_cast<int *>(p);
  p += 256;
  b->d_active = reinterpret_cast<int *>(p);
  p += align256((size_t)max_channels * sizeof(int));
  b->d_partials = reinterpret_cast<double *>(p);
  p += align256((size_t)max_tiles * 8 * sizeof(double));
  b->d_sums = reinterpret_cast<double *>(p);
  p += align256((size_t)max_channels * 8 * sizeof(double));
  b->d_gctr = reinterpret_cast<uint32_t *>(p);
  p += 256;
  b->heap_begin = (size_t)(p - b->pool);
  if (pool_bytes > b->heap_begin) b->free_list.push_back(Region{b->heap_begin, pool_bytes - b->heap_begin});
  b->slots.resize(max_channels);
  b->h_chans.resize(max_channels);
  std::memset(b->h_chans.data(), 0, b->h_chans.size() * sizeof(ChanDesc));
  b->h_active.assign(max_channels, 0);
  int cus = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, b->device) == hipSuccess && prop.multiProcessorCount > 0)
    cus = prop.multiProcessorCount;
  b->grid_cap = cus * batch_blocks_per_cu(precision); // blocks of 256 threads
  b->grid = 1;
  const int rc = with_device(b, [&]() -> int {
    const uint32_t z[2] = {0u, 0u};
    LKS_HIP_CHECK(hipMemcpyAsync(b->d_gctr, z, sizeof z, hipMemcpyHostToDevice, b->stream));
    return rebuild(b);
  });
  if (rc != LKS_OK) {
    delete b;
    return rc;
  }
  *out = b;
  return LKS_OK;
}

int lks_mhd_batch_destroy(lks_mhd_batch_t *b) {
  clear_error();
  if (!b) return LKS_OK;
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->gexec_long) (void)hipGraphExecDestroy(b->gexec_long);
  delete b;
  return LKS_OK;
}

int lks_mhd_batch_admit(lks_mhd_batch_t *b, const lks_mhd_params *p, int32_t *slot) {
  clear_error();
  if (!b || !p || !slot) {
    set_error("invalid batch, parameters or slot pointer");
    return LKS_EINVAL;
  }
  lks_mhd_params q = *p;
  q.precision = b->precision;
  Channel c;
  int rc = derive_channel(&q, &c);
  if (rc != LKS_OK) return rc;
  if (q.x_walls) {
    set_error("invalid parameters: batches hold x-periodic channels only (x_walls = 0)");
    return LKS_EINVAL;
  }
  if (q.q_lower != 0.5 || q.q_upper != 0.5) {
    set_error("invalid parameters: batches hold half-way walls only (q = 1/2)");
    return LKS_EINVAL;
  }
  if (q.nsolids > 0) {
    set_error("invalid parameters: batches hold channels without solid bodies");
    return LKS_EINVAL;
  }

  const int64_t n = (int64_t)q.nx * q.ny;
  if (b->nodes + n > b->max_nodes) {
    set_error("batch node capacity %lld exceeded", (long long)b->max_nodes);
    return LKS_ENOMEM;
  }
  int s = -1;
  for (int i = 0; i < b->max_channels; ++i)
    if (!b->slots[i].used) {
      s = i;
      break;
    }
  if (s < 0) {
    set_error("all %d slots are in use", b->max_channels);
    return LKS_ENOMEM;
  }
  Slot sl;
  sl.used = true;
  sl.ch = c;
  sl.width_class = width_class_of(q.nx);
  // tile capacity check for the current shape table
  {
    if ((long long)total_tiles(b, b->tile_w, b->tile_h) +
            count_tiles(b->precision, q.nx, q.ny, b->tile_w[sl.width_class],
                        b->tile_h[sl.width_class]) >
        b->max_tiles) {
      set_error("tile list capacity exceeded");
      return LKS_ENOMEM;
    }
  }
  sl.bytes = channel_region_bytes(c, b->precision);
  if (!pool_alloc(b, sl.bytes, &sl.offset)) {
    set_error("pool has no free region of %zu bytes", sl.bytes);
    return LKS_ENOMEM;
  }
  const long long plane = plane_elems(q.nx, q.ny, b->precision);
  const size_t state = align256((size_t)19 * plane * elem_bytes(b->precision));
  char *base = b->pool + sl.offset;
  ChanDesc d{};
  d.buf[0] = base;
  d.buf[1] = base + state;
  d.rec = reinterpret_cast<double *>(base + 2 * state);
  d.ref = base + 2 * state + align256((size_t)2 * q.nx * q.ny * sizeof(double));
  d.g = Geom{q.nx, q.ny, q.nx, plane};
  {
    int sh = 0;
    while ((1LL << sh) < (long long)q.nx) ++sh;
    d.nx_shift = sh;
    d.nx_magic = (uint32_t)((((1ULL << 32) * ((1ULL << sh) - (uint64_t)q.nx)) / (uint64_t)q.nx) + 1ULL);
  }
  // an MRT channel runs the TRT scheme with its corrections switched on
  d.bc = (scheme_of(q) & ~COLL_MRT) | (q.collision == LKS_MRT ? COLL_TRT : 0);
  // the initial state goes to buf[0]; at the next step the global parity is
  // b->parity, and the channel must read buf[0] then: phase = parity.
  d.phase = b->parity;
  d.step_base = (uint32_t)b->global_steps;
  // binary16 computed in FP32 takes its increments in stored units
  d.kf = make_coef<float>(c, b->precision == LKS_FP16_STORE ? kStoreUp16 : 1.0);
  d.kd = make_coef<double>(c);
  sl.admit_step = b->global_steps;
  rc = with_device(b, [&]() -> int {
    dispatch_precision(b->precision, [&](auto t) {
      launch_init<typename decltype(t)::S>(b, sl, d.buf[0]);
    });
    LKS_HIP_CHECK(hipGetLastError());
    const long long nr = (long long)(ref_area_bytes(q.ny, b->precision) / sizeof(double));
    hipLaunchKernelGGL(k_zero<double>, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, b->stream,
                       static_cast<double *>(d.ref), nr);
    LKS_HIP_CHECK(hipGetLastError());
    if (b->precision == LKS_FP16_STORE) {
      // pre-collision tables of the FP32-arithmetic binary16 mode
      const dim3 tg((unsigned)((q.ny + 255) / 256));
      if (wall_of(d.bc) == BC_LINK)
        hipLaunchKernelGGL(k_xtables<BC_LINK>, tg, dim3(256), 0, b->stream, d.g, d.kd, d.ref);
      else
        hipLaunchKernelGGL(k_xtables<BC_MOMENT>, tg, dim3(256), 0, b->stream, d.g, d.kd, d.ref);
      LKS_HIP_CHECK(hipGetLastError());
    }
    return LKS_OK;
  });
  if (rc != LKS_OK) {
    pool_free(b, sl.offset, sl.bytes);
    return rc;
  }
  b->slots[s] = sl;
  b->h_chans[s] = d;
  b->h_active[s] = 1;
  b->nodes += n;
  b->nactive += 1;
  b->dirty = true;
  *slot = s;
  return LKS_OK;
}

int lks_mhd_batch_retire(lks_mhd_batch_t *b, int32_t slot) {
  clear_error();
  if (!b || slot < 0 || slot >= b->max_channels || !b->slots[slot].used) {
    set_error("invalid batch or slot");
    return LKS_EINVAL;
  }
  Slot &sl = b->slots[slot];
  // the pool region may be reused by the next admission: finish pending work
  const int rc = with_device(b, [&]() -> int {
    LKS_HIP_CHECK(hipStreamSynchronize(b->stream));
    return LKS_OK;
  });
  if (rc != LKS_OK) return rc;
  pool_free(b, sl.offset, sl.bytes);
  b->nodes -= (int64_t)sl.ch.p.nx * sl.ch.p.ny;
  b->nactive -= 1;
  sl = Slot();
  std::memset(&b->h_chans[slot], 0, sizeof(ChanDesc));
  b->h_active[slot] = 0;
  b->dirty = true;
  return LKS_OK;
}

int32_t lks_mhd_batch_active(const lks_mhd_batch_t *b) { return b ? b->nactive : -1; }
int64_t lks_mhd_batch_nodes(const lks_mhd_batch_t *b) { return b ? b->nodes : -1; }

static bool valid_shape(int w, int h) {
  if (w == 0) return h == 1 || h == 2 || h == 4;
  const bool ok_w = w == 8 || w == 16 || w == 32 || w == 64 || w == 128 || w == 256;
  return ok_w && w * h == kTileThreads;
}

int lks_mhd_batch_set_tile(lks_mhd_batch_t *b, int32_t width_class, int32_t tile_w, int32_t tile_h) {
  clear_error();
  if (!b || width_class < 0 || width_class >= kWidthClasses || !valid_shape(tile_w, tile_h)) {
    set_error("invalid width class or tile shape (w in {8..256} with w*h = 256, or w = 0 with h in {1, 2, 4})");
    return LKS_EINVAL;
  }
  int tw[kWidthClasses], th[kWidthClasses];
  std::memcpy(tw, b->tile_w, sizeof tw);
  std::memcpy(th, b->tile_h, sizeof th);
  tw[width_class] = tile_w;
  th[width_class] = tile_h;
  if (total_tiles(b, tw, th) > b->max_tiles) {
    set_error("tile list capacity exceeded by this shape");
    return LKS_ENOMEM;
  }
  b->tile_w[width_class] = tile_w;
  b->tile_h[width_class] = tile_h;
  b->dirty = true;
  return LKS_OK;
}

int lks_mhd_batch_step(lks_mhd_batch_t *b, int64_t nsteps, int32_t use_graph) {
  clear_error();
  if (!b || nsteps < 0) {
    set_error("invalid batch or negative step count");
    return LKS_EINVAL;
  }
  return with_device(b, [&]() -> int { return batch_steps(b, nsteps, use_graph != 0); });
}

int lks_mhd_batch_step_check(lks_mhd_batch_t *b, int64_t nsteps, int32_t use_graph,
                             double *residuals, int32_t *unstable) {
  clear_error();
  if (!b || nsteps < 2) {
    set_error("invalid batch or nsteps < 2");
    return LKS_EINVAL;
  }
  std::vector<double> sums((size_t)b->max_channels * 8, 0.0);
  const int rc = with_device(b, [&]() -> int {
    int r = LKS_OK;
    if (b->dirty && (r = rebuild(b)) != LKS_OK) return r;
    if (b->nactive > 0) {
      // the first step of the window records phi, the last compares;
      // binary16 states are rebased at the start of every window
      if ((r = batch_rebase(b)) != LKS_OK) return r;
      if ((r = batch_one(b, MODE_RECORD)) != LKS_OK) return r;
      if ((r = batch_steps(b, nsteps - 2, use_graph != 0)) != LKS_OK) return r;
      if ((r = batch_one(b, MODE_RESIDUAL)) != LKS_OK) return r;
      hipLaunchKernelGGL(k_batch_finalize, dim3(b->max_channels), dim3(64), 0, b->stream,
                         b->d_chans, b->d_active, b->d_partials, b->d_sums);
      LKS_HIP_CHECK(hipGetLastError());
      LKS_HIP_CHECK(hipMemcpyAsync(sums.data(), b->d_sums, sums.size() * sizeof(double),
                                   hipMemcpyDeviceToHost, b->stream));
    } else {
      b->global_steps += nsteps;
      b->parity ^= (int)(nsteps & 1);
      if ((r = sync_counter(b)) != LKS_OK) return r;
    }
    LKS_HIP_CHECK(hipStreamSynchronize(b->stream));
    return LKS_OK;
  });
  if (rc != LKS_OK) return rc;
  for (int s = 0; s < b->max_channels; ++s) {
    double r = NAN;
    int bad = 0;
    if (b->slots[s].used) {
      const double *v = &sums[(size_t)s * 8];
      const double win = (double)(nsteps - 1);
      const double ru = std::sqrt(v[0]) / std::fmax(std::sqrt(v[1]), 1e-300) / win;
      const double rb = std::sqrt(v[2]) / std::fmax(std::sqrt(v[3]), 1e-300) / win;
      r = std::fmax(ru, rb);
      bad = (v[5] != 0.0 || !std::isfinite(r)) ? 1 : 0;
    }
    if (residuals) residuals[s] = r;
    if (unstable) unstable[s] = bad;
  }
  return LKS_OK;
}

int lks_mhd_batch_rebase(lks_mhd_batch_t *b) {
  clear_error();
  if (!b) {
    set_error("invalid batch");
    return LKS_EINVAL;
  }
  return with_device(b, [&]() -> int { return batch_rebase(b); });
}

int64_t lks_mhd_batch_steps_done(const lks_mhd_batch_t *b, int32_t slot) {
  if (!b || slot < 0 || slot >= b->max_channels || !b->slots[slot].used) return -1;
  return b->global_steps - b->slots[slot].admit_step;
}

int lks_mhd_batch_moments(lks_mhd_batch_t *b, int32_t slot, double *rho, double *ux,
                          double *uy, double *bx, double *by, double *jz) {
  clear_error();
  if (!b || slot < 0 || slot >= b->max_channels || !b->slots[slot].used) {
    set_error("invalid batch or slot");
    return LKS_EINVAL;
  }
  const ChanDesc &d = b->h_chans[slot];
  const int cur = b->parity ^ d.phase;
  const ObsOutB oo{rho, ux, uy, bx, by, jz};
  const long long n = (long long)d.g.nx * d.g.ny;
  const dim3 grid((unsigned)((n + 255) / 256));
  return with_device(b, [&]() -> int {
    const bool link = wall_of(d.bc) == BC_LINK;
    dispatch_precision(b->precision, [&](auto t) {
      using S = typename decltype(t)::S;
      // binary16 computed in FP32: observables decode in FP64
      using C0 = typename decltype(t)::C;
      using C = std::conditional_t<kXA<S, C0>, double, C0>;
      const S *src = static_cast<const S *>(d.buf[cur]);
      const C *ref = kXA<S, C0> ? reinterpret_cast<const C *>(xtabs_of(d.ref, d.g.ny).D64)
                                : static_cast<const C *>(d.ref);
      if (link)
        hipLaunchKernelGGL((k_chan_moments<S, C, BC_LINK>), grid, dim3(256), 0, b->stream, d.g,
                           coef_host<C>(d), src, ref, oo);
      else
        hipLaunchKernelGGL((k_chan_moments<S, C, BC_MOMENT>), grid, dim3(256), 0, b->stream, d.g,
                           coef_host<C>(d), src, ref, oo);
    });
    LKS_HIP_CHECK(hipGetLastError());
    return LKS_OK;
  });
}

int lks_mhd_batch_save_state(lks_mhd_batch_t *b, int32_t slot, double *dev_pops) {
  clear_error();
  if (!b || !dev_pops || slot < 0 || slot >= b->max_channels || !b->slots[slot].used) {
    set_error("invalid batch, slot or destination");
    return LKS_EINVAL;
  }
  const ChanDesc &d = b->h_chans[slot];
  const int cur = b->parity ^ d.phase;
  const long long n = (long long)d.g.nx * d.g.ny;
  const dim3 grid((unsigned)((n + 255) / 256));
  return with_device(b, [&]() -> int {
    dispatch_precision(b->precision, [&](auto t) {
      using S = typename decltype(t)::S;
      using C0 = typename decltype(t)::C;
      using C = std::conditional_t<kXA<S, C0>, double, C0>;
      const C *ref = kXA<S, C0> ? reinterpret_cast<const C *>(xtabs_of(d.ref, d.g.ny).D64)
                                : static_cast<const C *>(d.ref);
      hipLaunchKernelGGL((k_save<S, C>), grid, dim3(256), 0, b->stream, d.g,
                         b->slots[slot].ch.d.b0, static_cast<const S *>(d.buf[cur]), ref,
                         dev_pops);
    });
    LKS_HIP_CHECK(hipGetLastError());
    return LKS_OK;
  });
}

int lks_mhd_batch_autotune(lks_mhd_batch_t *b, int32_t trial_steps, int32_t *tiles_out) {
  clear_error();
  if (!b || trial_steps < 1) {
    set_error("invalid batch or trial_steps < 1");
    return LKS_EINVAL;
  }
  const int cand_w[9] = {0, 0, 0, 8, 16, 32, 64, 128, 256};
  const int cand_h[9] = {1, 2, 4, 32, 16, 8, 4, 2, 1};
  const int rc = with_device(b, [&]() -> int {
    bool present[kWidthClasses] = {false};
    for (const Slot &s : b->slots)
      if (s.used) present[s.width_class] = true;
    hipEvent_t e0, e1;
    LKS_HIP_CHECK(hipEventCreate(&e0));
    LKS_HIP_CHECK(hipEventCreate(&e1));
    int result = LKS_OK;
    for (int k = 0; k < kWidthClasses && result == LKS_OK; ++k) {
      if (!present[k]) continue;
      // rectangles no wider than twice the class's upper width bound
      const int upper = (k == kWidthClasses - 1) ? 1 << 30 : (8 << k);
      // the incumbent shape is timed first; a candidate replaces the best so
      // far only if it is at least 3% faster (trial timings are noisy)
      float best = 1e30f;
      int best_w = b->tile_w[k], best_h = b->tile_h[k];
      for (int ci = -1; ci < 9; ++ci) {
        const int w = ci < 0 ? best_w : cand_w[ci], h = ci < 0 ? best_h : cand_h[ci];
        if (ci >= 0 && w == best_w && h == best_h) continue;
        if (w > 2 * upper && w != 8) continue;
        int tw[kWidthClasses], th[kWidthClasses];
        std::memcpy(tw, b->tile_w, sizeof tw);
        std::memcpy(th, b->tile_h, sizeof th);
        tw[k] = w;
        th[k] = h;
        if (total_tiles(b, tw, th) > b->max_tiles) continue;
        b->tile_w[k] = w;
        b->tile_h[k] = h;
        b->dirty = true;
        // the trial steps advance every channel; an even count keeps the
        // parity, and the steps are counted like any other
        int r = batch_steps(b, 2, false); // warm-up
        if (r == LKS_OK) r = (hipEventRecord(e0, b->stream) == hipSuccess) ? LKS_OK : LKS_EDEVICE;
        if (r == LKS_OK) r = batch_steps(b, 2 * ((trial_steps + 1) / 2), false);
        if (r == LKS_OK) r = (hipEventRecord(e1, b->stream) == hipSuccess) ? LKS_OK : LKS_EDEVICE;
        if (r == LKS_OK) r = (hipEventSynchronize(e1) == hipSuccess) ? LKS_OK : LKS_EDEVICE;
        float ms = 0.f;
        if (r == LKS_OK) r = (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) ? LKS_OK : LKS_EDEVICE;
        if (r != LKS_OK) {
          if (r == LKS_EDEVICE) set_error("autotune timing failed");
          result = r;
          break;
        }
        if (ms < 0.97f * best) {
          best = ms;
          best_w = w;
          best_h = h;
        }
      }
      b->tile_w[k] = best_w;
      b->tile_h[k] = best_h;
      b->dirty = true;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return result;
  });
  if (tiles_out)
    for (int k = 0; k < kWidthClasses; ++k) {
      tiles_out[2 * k] = b->tile_w[k];
      tiles_out[2 * k + 1] = b->tile_h[k];
    }
  return rc;
}

} // extern "C"
