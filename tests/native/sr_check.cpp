// Host check of the stochastic rounding used for stored populations
// (paper_2112_13930_amd/csrc/lks_sr.hpp): for each test value v the result
// must be one of the two neighbours of v in the target format, and over a
// stratified sweep of the random word the share of results on the larger
// magnitude side must equal the exact probability
//   (|v| - |lo|) / (|hi| - |lo|)
// to within the sweep's resolution (and, binary16 taking 13 random bits, to
// within 2^-13 where binary16's subnormal spacing leaves bits of v below the
// random ones).  Exactly representable values must come back unchanged.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>

#include "lks_sr.hpp"

using lks::sr_f16;
using lks::sr_f32;

static int fails = 0;
static long checks = 0;

template <typename T> static uint32_t tbits(T x) {
  if constexpr (sizeof(T) == 4) return __builtin_bit_cast(uint32_t, x);
  else return __builtin_bit_cast(uint16_t, x);
}
template <typename T> static T from_bits(uint32_t b) {
  if constexpr (sizeof(T) == 4) return __builtin_bit_cast(float, b);
  else return __builtin_bit_cast(_Float16, (uint16_t)b);
}

// Neighbours lo (smaller magnitude) and hi (larger magnitude) of |v| in T,
// found by stepping the bit pattern of the nearest value.
template <typename T> static void neighbours(long double av, T &lo, T &hi) {
  T h = (T)av;  // nearest (or the largest finite if av overflows: not tested)
  if ((long double)h > av) {
    hi = h;
    lo = from_bits<T>(tbits(h) - 1);
    if (tbits(h) == 0) lo = h;
  } else {
    lo = h;
    hi = from_bits<T>(tbits(h) + 1);
  }
}

// Random words as the kernels draw them (lks::Rng): 16 random bits on top,
// bit 15 set.  With bits16 the sweep covers the 2^16 possible words exactly.
static bool g_bits16 = false;

template <typename T, typename W, typename F>
static void check(W v, F round, int nsweep) {
  const long double av = std::fabs((long double)v);
  T lo, hi;
  neighbours<T>(av, lo, hi);
  const bool exact = (long double)lo == av;
  int up = 0;
  for (int i = 0; i < nsweep; ++i) {
    const uint32_t r = g_bits16 ? (((uint32_t)(((uint64_t)i << 16) / (uint64_t)nsweep) << 16) | 0x8000u)
                                : (uint32_t)(((uint64_t)i << 32) / (uint64_t)nsweep) + 977u;
    const T res = round(v, r);
    const long double ar = std::fabs((long double)res);
    const bool neg_ok = std::signbit((double)v) ? (std::signbit((double)res) || ar == 0) : !std::signbit((double)res);
    ++checks;
    if (!neg_ok || (ar != (long double)lo && ar != (long double)hi) || (exact && ar != av)) {
      if (fails++ < 10)
        printf("bad result: v=%.17Lg res=%.17Lg lo=%.17Lg hi=%.17Lg\n", (long double)v, (long double)res,
               (long double)lo, (long double)hi);
      return;
    }
    up += (ar == (long double)hi && !exact) ? 1 : 0;
  }
  if (!exact) {
    const long double p = (av - (long double)lo) / ((long double)hi - (long double)lo);
    const long double want = p * nsweep;
    // binary16 below 2^-14: the probability is resolved to 2^-13
    const long double slack = sizeof(T) == 2 && av < 0x1p-14L ? nsweep * 0x1p-13L : 0.0L;
    if (std::fabs((long double)up - want) > 1.5L + slack) {
      if (fails++ < 10)
        printf("bad probability: v=%.17Lg p=%.9Lf got %d of %d (want %.2Lf)\n", (long double)v, p, up,
               nsweep, want);
    }
  }
}

int main() {
  std::mt19937_64 g(12345);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  const int N = 4096;
  auto f32 = [](double v, uint32_t r) { return sr_f32(v, r); };
  auto f16f = [](float v, uint32_t r) { return sr_f16(v, r); };
  for (int t = 0; t < 4000; ++t) {
    // magnitudes spread over many binades, both signs
    const double mag = std::exp2(-40.0 + 56.0 * U(g)) * (1.0 + U(g));
    const double v = (t & 1) ? -mag : mag;
    if (std::fabs(v) < 65504.0) {
      check<_Float16>((float)v, f16f, N);
    }
    if (std::fabs(v) > 1e-30) check<float>(v, f32, N);
  }
  // beyond binary16's range the result is infinite
  for (double v : {65536.0, -70000.0, 1e6}) {
    ++checks;
    if (!std::isinf((double)sr_f16((float)v, 12345u))) {
      ++fails;
      printf("no overflow to inf for %g\n", v);
    }
  }
  // binary16 subnormal range, the boundaries and exact values
  const double special[] = {0.0, 0x1p-24, 0x1p-25, 0x1.8p-25, 0x1.fffp-25, 0x1.8p-24, 0x1p-14,
                            0x1.ffcp-15, 0x1.ffdp-15, 0x1p-15 * 3, 1.0, 1.0 + 0x1p-11, 65504.0,
                            0.1, 1.0 / 3, 0x1.0000001p0, -0x1p-20, -0.0};
  for (double v : special) {
    check<_Float16>((float)v, f16f, N);
    if (v == 0 || std::fabs(v) > 1e-30) check<float>(v, f32, N);
  }
  // the kernels' 16-bit words: every word of the 2^16, probability to +-1.5/65536
  g_bits16 = true;
  std::mt19937_64 g2(777);
  for (int t = 0; t < 300; ++t) {
    const double mag = std::exp2(-40.0 + 56.0 * U(g2)) * (1.0 + U(g2));
    const double v = (t & 1) ? -mag : mag;
    if (std::fabs(v) < 65504.0) {
      check<_Float16>((float)v, f16f, 65536);
    }
    if (std::fabs(v) > 1e-30) check<float>(v, f32, 65536);
  }
  // binary16's subnormal range in full: over all 2^13 values of the 13 bits
  // used, the number of results rounded up is trunc(|v| 2^37) mod 2^13
  // (|v| 2^24 has that many 2^-13 parts above its integer part), and the
  // smaller neighbour is trunc(|v| 2^24) 2^-24
  {
    std::mt19937_64 g5(31);
    for (int t = 0; t < 20000; ++t) {
      const float v = (float)(std::exp2(-44.0 + 30.0 * U(g5)) * ((t & 1) ? -1.0 : 1.0));
      const long double s = std::fabs((long double)v) * 0x1p24L;
      const long double lo = std::floor(s);
      const long long want = (long long)std::floor(std::fabs((long double)v) * 0x1p37L) % 8192;
      long long up = 0;
      for (uint32_t k = 0; k < 8192; ++k) {
        const long double res = std::fabs((long double)sr_f16(v, k << 19)) * 0x1p24L;
        ++checks;
        if (res != lo && res != lo + 1) {
          if (fails++ < 10) printf("subnormal: v=%a k=%u res=%Lg\n", (double)v, k, res);
          break;
        }
        up += res == lo + 1 ? 1 : 0;
      }
      if (up != want && fails++ < 10) printf("subnormal count: v=%a %lld != %lld\n", (double)v, up, want);
    }
  }
  // the generator's words: top 16 bits spread over all values, bit 15 set
  lks::Rng rng(12345u);
  int hist[16] = {0};
  for (int i = 0; i < 1 << 20; ++i) {
    const uint32_t w = rng.next();
    ++checks;
    if ((w & 0xFFFFu) != 0x8000u) ++fails;
    ++hist[w >> 28];
  }
  for (int b = 0; b < 16; ++b)
    if (std::abs(hist[b] - (1 << 16)) > 2000) {
      ++fails;
      printf("random word histogram bin %d: %d\n", b, hist[b]);
    }
  printf("%s: %ld results checked, %d failures\n", fails ? "FAIL" : "OK", checks, fails);
  return fails ? 1 : 0;
}
