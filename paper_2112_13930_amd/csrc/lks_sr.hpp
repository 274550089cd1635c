// Stochastic rounding of computed populations to their storage type, and the
// random bits it uses.  Host-compilable (the unit test checks it on the CPU).
//
// Rounding: the result is one of the two neighbours of v in the target
// format, the farther one with probability |v - nearest lower-magnitude
// neighbour| / spacing, resolved to the random word's resolution (2^-32 of
// the spacing for a full word; the kernels pass 16 random bits, 2^-16).  It is computed by
// adding uniform random bits below the target's last place to the magnitude
// bits of v and truncating there (a carry out of the kept bits rounds up,
// across a binade too); binary64 reaches binary16 through the nearest
// binary32.  Values beyond the target's range become infinite (and are
// reported as non-finite by the residual check).
//
// Random bits: one hashed seed per node and step (counter-based, so a run is
// reproducible bit for bit and independent of launch shape or batch mix),
// then one xorshift32 step (Marsaglia 2003) per two stored values.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__) || defined(__HIP__)
#define LKS_HD __host__ __device__
#else
#define LKS_HD
#endif

namespace lks {

// 32-bit integer finalizer with the xorshift-multiply constants of the
// "lowbias32" hash found by C. Wellons' hash-prospector search (2018).
LKS_HD inline uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

// Per-node stream of random words for stochastic rounding.  next() gives a
// 32-bit word whose top 16 bits are random and whose bit 15 is set (the
// middle of the 2^-16 bin the 16 bits select); two consecutive calls share
// one xorshift32 step.  16 bits resolve the rounding probability to 2^-16
// of the target spacing, far below any other error of the stored values.
struct Rng {
  uint32_t s, w = 0;
  bool half = false;
  LKS_HD explicit Rng(uint32_t seed) : s(seed | 1u) {} // xorshift needs s != 0
  LKS_HD uint32_t next() {
    if (half) {
      half = false;
      return (w << 16) | 0x8000u;
    }
    s ^= s << 13;
    s ^= s >> 17;
    s ^= s << 5;
    w = s;
    half = true;
    return (w & 0xFFFF0000u) | 0x8000u;
  }
};

LKS_HD inline uint32_t step_seed(uint32_t step) { return mix32(step * 0x9E3779B1U + 0x632BE5ABU); }

// Seed of the re-encoding done by a rebase after `step` steps (a stream
// distinct from the steps').
LKS_HD inline uint32_t rebase_seed(uint32_t step) { return mix32(step * 0x27D4EB2FU + 0x165667B1U); }

LKS_HD inline uint32_t node_seed(uint32_t sseed, uint32_t idx) {
  return mix32(idx * 0x85EBCA77U ^ sseed);
}

LKS_HD inline uint64_t bits64(double v) { return __builtin_bit_cast(uint64_t, v); }
LKS_HD inline double dbl(uint64_t b) { return __builtin_bit_cast(double, b); }
LKS_HD inline uint32_t bits32(float v) { return __builtin_bit_cast(uint32_t, v); }
LKS_HD inline float flt(uint32_t b) { return __builtin_bit_cast(float, b); }

// binary64 -> binary32: 29 bits below binary32's last place.  (Inputs below
// binary32's normal range, |v| < 2^-126, are rounded once more to nearest.)
LKS_HD inline float sr_f32(double v, uint32_t r) {
  const uint64_t b = (bits64(v) + (uint64_t)(r >> 3)) & ~(uint64_t)0x1FFFFFFFu;
  return (float)dbl(b); // exact: 24 significant bits left
}

// binary32 -> binary16.  Below 2^-24 the result is 0 or 2^-24 (binary16's
// smallest subnormal) with probability |v| / 2^-24; above, random bits are
// added below binary16's last place and truncated.
LKS_HD inline _Float16 sr_f16(float v, uint32_t r) {
  const uint32_t b = bits32(v);
  // |v| >= 2^-14 (binary16's normal range and above): binary16's last place
  // is 13 bits above binary32's; adding to the magnitude bits of b leaves its
  // sign alone.  Zeros come out unchanged the same way.
  const uint32_t m = b & 0x7FFFFFFFu;
  if (m >= 0x38800000u || m == 0u) return (_Float16)flt((b + (r >> 19)) & ~0x1FFFu);
  const uint32_t sign = b & 0x80000000u;
  const uint32_t mag = b ^ sign;
  const int e = (int)(mag >> 23) - 127;
  if (e < -24) {
    const float p = (float)(r >> 8) * 0x1p-48f; // uniform in [0, 2^-24)
    return (_Float16)flt(sign | (p < flt(mag) ? 0x33800000u : 0u));
  }
  const int k = e >= -14 ? 13 : -1 - e;
  const uint32_t t = (mag + (r >> (32 - k))) & ~((1u << k) - 1u);
  return (_Float16)flt(sign | t); // exact
}

// The same result with both cases computed and one selected (no branch).
// The branch suits kernels of one scheme, whose wavefronts mostly agree on
// it and which lose occupancy to the registers of the select form; the
// select suits the batched kernel, whose small channels mix both cases in a
// wavefront and which inlines every scheme's stores.
LKS_HD inline _Float16 sr_f16_sel(float v, uint32_t r) {
  const uint32_t b = bits32(v);
  const uint32_t sign = b & 0x80000000u;
  const uint32_t mag = b ^ sign;
  const int e = (int)(mag >> 23) - 127;
  const float p = (float)(r >> 8) * 0x1p-48f;
  const uint32_t tiny = p < flt(mag) ? 0x33800000u : 0u;
  const int k = e >= -14 ? 13 : (e >= -24 ? -1 - e : 23);
  const uint32_t t = (mag + (r >> (32 - k))) & ~((1u << k) - 1u);
  return (_Float16)flt(sign | (e < -24 ? tiny : t));
}

// binary32 -> binary16 for a conversion that truncates (round toward zero):
// zeros and binary16's normal range get the random bits of sr_f16's fast
// path added below binary16's last place and leave the masking to the
// truncation; the rest is sr_f16's exact binary16 result, which truncation
// keeps.  Truncating the returned value gives sr_f16's bits, except that
// magnitudes beyond binary16's range saturate at 65504 instead of becoming
// infinite (and infinities may come back as NaN).  The kernels convert two
// such values at once.
LKS_HD inline float sr16_pre(float v, uint32_t r) {
  const uint32_t b = bits32(v), m = b & 0x7FFFFFFFu;
  if (m >= 0x38800000u || m == 0u) return flt(b + (r >> 19));
  return (float)sr_f16(v, r);
}

// Round toward zero to binary16 (host model of the device conversion).
LKS_HD inline _Float16 f16_rtz(float t) {
  const uint32_t b = bits32(t);
  const uint32_t mag = b & 0x7FFFFFFFu, sign = b & 0x80000000u;
  if (mag >= 0x7F800000u) return (_Float16)t;                           // inf, NaN
  if (mag >= 0x477FE000u) return (_Float16)flt(sign | 0x477FE000u);      // 65504
  if (mag >= 0x38800000u) return (_Float16)flt(sign | (mag & ~0x1FFFu)); // exact
  const float q = __builtin_truncf(flt(mag) * 0x1p24f) * 0x1p-24f;     // subnormal grid
  return (_Float16)flt(sign | bits32(q));
}

// Stochastic rounding of v (compute type C) to storage type S; identity for
// equal types.  SEL picks the select form of the binary16 rounding (same
// result).
template <typename S, typename C, bool SEL = false>
LKS_HD inline S round_sr(C v, uint32_t r) {
  if constexpr (sizeof(S) == sizeof(C)) {
    (void)r;
    return (S)v;
  } else {
    if constexpr (sizeof(S) == 4) return sr_f32(v, r);
    // binary64 goes to the nearest binary32 first: that moves v by at most
    // 2^-25 |v|, 2^-14 of a binary16 spacing, and costs a few integer
    // instructions where rounding at v's binary16 spacing in FP64 took ten
    // FP64 ones (the binary16 step is arithmetic-bound)
    else if constexpr (SEL) return sr_f16_sel((float)v, r);
    else return sr_f16((float)v, r);
  }
}

} // namespace lks
