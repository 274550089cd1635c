// Element-wise helper kernels shared by the single-channel and batched
// paths: rest-state initialisation and conversion between the stored state
// and raw FP64 populations [19][ny][nx].
#pragma once

#include <hip/hip_runtime.h>

#include "lks_node.hpp"

namespace lks {

// Rest state at density rho0 with B = (0, B0).  Stored deviations:
// f' = w (rho0 - 1), g_x = 0, g'_y = 0.
template <typename S>
__global__ void k_init(Geom g, double rho0, S *__restrict__ dst) {
  const long long n = (long long)g.nx * g.ny;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int y = (int)(i / g.nx), x = (int)(i - (long long)y * g.nx);
  const long long o = (long long)y * g.pitch + x;
  const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  for (int q = 0; q < 9; ++q) dst[q * g.plane + o] = (S)(w[q] * (rho0 - 1.0));
  for (int q = 0; q < 5; ++q) {
    dst[(9 + q) * g.plane + o] = (S)0.0;
    dst[(14 + q) * g.plane + o] = (S)0.0;
  }
}

// Stored state <-> raw FP64 populations [19][ny][nx].
template <typename S>
__global__ void k_save(Geom g, double b0, const S *__restrict__ src, double *__restrict__ out) {
  const long long n = (long long)g.nx * g.ny;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int y = (int)(i / g.nx), x = (int)(i - (long long)y * g.nx);
  const long long o = (long long)y * g.pitch + x;
  const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  const double Wm[5] = {1.0 / 3, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
  for (int q = 0; q < 19; ++q) {
    const double v = (double)src[q * g.plane + o];
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
  for (int q = 0; q < 19; ++q) {
    const double v = in[q * n + i];
    dst[q * g.plane + o] = (S)(q < 9 ? v - w[q] : (q < 14 ? v : v - Wm[q - 14] * b0));
  }
}

} // namespace lks
