// Helper kernels shared by the single-channel and batched paths: rest-state
// initialisation, conversion between the stored state and raw FP64
// populations [19][ny][nx], and the row rebase of binary16 states.
#pragma once

#include <hip/hip_runtime.h>

#include "lks_node.hpp"

namespace lks {

// Rest state at density rho0 with B = (0, B0).  Stored deviations:
// f' = w (rho0 - 1), g_x = 0, g'_y = 0 (binary16: times its scale 2^12).
template <typename S>
__global__ void k_init(Geom g, double rho0, S *__restrict__ dst,
                       const int32_t *__restrict__ sidx = nullptr) {
  const long long n = (long long)g.nx * g.ny;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int y = (int)(i / g.nx), x = (int)(i - (long long)y * g.nx);
  const long long o = (long long)y * g.pitch + x;
  const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  const double up = kRowRef<S> ? kStoreUp16 : 1.0;
  // solid nodes (sidx, when given) rest at unit density
  const double r0 = (sidx && sidx[i] == kSolidNode) ? 1.0 : rho0;
  for (int q = 0; q < 9; ++q) dst[q * g.plane + o] = (S)(w[q] * (r0 - 1.0) * up);
  for (int q = 0; q < 5; ++q) {
    dst[(9 + q) * g.plane + o] = (S)0.0;
    dst[(14 + q) * g.plane + o] = (S)0.0;
  }
}

// Stored state <-> raw FP64 populations [19][ny][nx].
template <typename S, typename C>
__global__ void k_save(Geom g, double b0, const S *__restrict__ src, const C *__restrict__ D,
                       double *__restrict__ out) {
  const long long n = (long long)g.nx * g.ny;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int y = (int)(i / g.nx), x = (int)(i - (long long)y * g.nx);
  const long long o = (long long)y * g.pitch + x;
  const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  const double Wm[5] = {1.0 / 3, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
  for (int q = 0; q < 19; ++q) {
    const double v = (double)dec<S, C>((C)src[q * g.plane + o], D + (long long)y * kRefRow, q);
    out[q * n + i] = q < 9 ? v + w[q] : (q < 14 ? v : v + Wm[q - 14] * b0);
  }
}

template <typename S>
__global__ void k_load(Geom g, double b0, const double *__restrict__ in, S *__restrict__ dst) {
  const long long n = (long long)g.nx * g.ny;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int y = (int)(i / g.nx), x = (int)(i - (long long)y * g.nx);
  const long long o = (long long)y * g.pitch + x;
  const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  const double Wm[5] = {1.0 / 3, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
  const double up = kRowRef<S> ? kStoreUp16 : 1.0;
  for (int q = 0; q < 19; ++q) {
    const double v = in[q * n + i];
    dst[q * g.plane + o] = (S)((q < 9 ? v - w[q] : (q < 14 ? v : v - Wm[q - 14] * b0)) * up);
  }
}

template <typename T>
__global__ void k_zero(T *__restrict__ p, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = T(0);
}

// Rebase one row of a binary16 state: move the x-mean of every plane's
// decoded-minus-reference values into the row's reference (compute type) and
// re-encode the row against it.  Decoded populations keep their values up
// to one rounding of stored values that no longer carry the row's mean, so
// the storage precision is spent on the x-variation alone.  One 256-thread
// block; lds holds 4 * 19 + 19 doubles.
template <typename S, typename C, bool SR>
__device__ __forceinline__ void rebase_row(S *__restrict__ buf, C *__restrict__ Drow,
                                           const Geom &g, int y, uint32_t seed, double *lds) {
  const int tid = threadIdx.x;
  const long long r0 = (long long)y * g.pitch;
  double acc[19];
#pragma unroll
  for (int q = 0; q < 19; ++q) acc[q] = 0.0;
  for (int x = tid; x < g.nx; x += 256)
#pragma unroll
    for (int q = 0; q < 19; ++q) acc[q] += (double)buf[q * g.plane + r0 + x];
  wave_sum<19>(acc);
  if ((tid & 63) == 0)
#pragma unroll
    for (int q = 0; q < 19; ++q) lds[(tid >> 6) * 19 + q] = acc[q];
  __syncthreads();
  if (tid < 19) {
    // new reference and the shift it represents, both in the compute type
    const double mean = ((lds[tid] + lds[19 + tid]) + (lds[38 + tid] + lds[57 + tid])) / g.nx;
    const C m = (C)(mean * kStoreDown16);
    const C Dn = Drow[tid] + m;
    const double shift = (double)Dn - (double)Drow[tid]; // exact
    Drow[tid] = Dn;
    lds[76 + tid] = shift;
  }
  __syncthreads();
  double sh[19];
#pragma unroll
  for (int q = 0; q < 19; ++q) sh[q] = lds[76 + q];
  for (int x = tid; x < g.nx; x += 256) {
    Rng rng(SR ? node_seed(seed, (uint32_t)(y * g.nx + x)) : 0u);
#pragma unroll
    for (int q = 0; q < 19; ++q) {
      S *p = buf + q * g.plane + r0 + x;
      // re-encoded in FP64 (exact for these magnitudes), then rounded once
      *p = to_store<S, double, SR>(((double)*p * kStoreDown16 - sh[q]) * kStoreUp16,
                                   SR ? rng.next() : 0u);
    }
  }
  __syncthreads(); // lds is reused by the next row
}

// Single channel: one block per row.
template <typename S, typename C>
__global__ __launch_bounds__(256) void k_rebase_rows(Geom g, S *__restrict__ buf,
                                                     C *__restrict__ D, uint32_t step) {
  __shared__ double lds[5 * 19];
  rebase_row<S, C, kUseSR<S, C>>(buf, D + (long long)blockIdx.x * kRefRow, g, (int)blockIdx.x,
                                 rebase_seed(step), lds);
}

// Pre-collision tables (XTabs) of every row of one channel whose binary16
// state is computed in FP32; run after every change of the row references.
template <int BC>
__global__ __launch_bounds__(256) void k_xtables(Geom g, Coef<double> k, void *base) {
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  if (y < g.ny) xtab_row<BC>(g, k, xtabs_of(base, g.ny), y);
}

} // namespace lks
