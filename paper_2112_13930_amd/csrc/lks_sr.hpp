// Stochastic rounding of computed populations to their storage type, and the
// random bits it uses.  Host-compilable (the unit test checks it on the CPU).
//
// Rounding: the result is one of the two neighbours of v in the target
// format, the farther one with probability |v - nearest lower-magnitude
// neighbour| / spacing, resolved to the random bits used: 29 below binary32's
// last place (binary64 -> binary32), 13 below binary16's (binary32 ->
// binary16, also in binary16's subnormal range, whose spacing is 2^-24).
// It is computed by adding uniform random bits below the target's last place
// to the magnitude of v and truncating there (a carry out of the kept bits
// rounds up, across a binade too); binary64 reaches binary16 through the
// nearest binary32.  Values beyond the target's range become infinite (and
// are reported as non-finite by the residual check).  On the GPU the
// binary32 -> binary16 rounding is the hardware's stochastic conversion
// (v_cvt_sr_f16_f32), which takes the top 13 bits of its random word; the
// host form below gives the same bits.
//
// Random bits: one hashed seed per node and step (counter-based, so a run is
// reproducible bit for bit and independent of launch shape or batch mix),
// then xorshift32 steps (Marsaglia 2003) from it: one per two stored values
// in binary32/binary64 storage (Rng); in binary16 storage four, whose XOR
// combinations give the node's ten words (F16Words).
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

// One step of Marsaglia's xorshift32 (shifts 13, 17, 5) on a nonzero state;
// returns the new state.
LKS_HD inline uint32_t xorshift32(uint32_t &s) {
  s ^= s << 13;
  s ^= s >> 17;
  s ^= s << 5;
  return s;
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
  // One xorshift32 step: the word two calls of next() are cut from (their top
  // 13 bits are those of the word and of the word shifted left by 16, which
  // is all the binary16 rounding takes).  Not to be mixed with next().
  LKS_HD uint32_t draw() { return xorshift32(s); }
  LKS_HD uint32_t next() {
    if (half) {
      half = false;
      return (w << 16) | 0x8000u;
    }
    w = xorshift32(s);
    half = true;
    return (w & 0xFFFF0000u) | 0x8000u;
  }
};

// Random words of the binary16 stores of one node: 19 values, each rounded
// with 13 bits (sr_f16).  Four xorshift32 steps from the node's seed give
// W1..W4; planes 2j and 2j + 1 take the top 13 bits of word j and of word j
// shifted left by 16, the words j = 0..9 being
//   W1, W3, W4, W1^W2, W1^W3, W1^W4, W3^W4, W1^W2^W4, W1^W3^W4, W2
// (plane 18 takes word 9's top bits only).  Each 13-bit field is a linear
// map over GF(2) of the 32-bit seed, and any two of the 19 fields are
// jointly uniform over the seed (their stacked 26 x 32 map has full rank, as
// it has for ten consecutive xorshift words): the rounding errors of a
// node's values are pairwise independent, so a moment summed from them has
// the variance it would have with independent errors.  That takes 32
// integer instructions per node where ten xorshift steps took 60.  (The
// seed keeps all 32 bits: only zero, which xorshift cannot take, is
// replaced; forcing the low bit to one instead would leave 31 bits and
// linear relations between some pairs of fields.)  word(q) must be called
// for q = 0, 1, ..., 18 in turn.
struct F16Words {
  uint32_t w1, w2, w3, w4, w = 0;
  LKS_HD explicit F16Words(uint32_t seed) {
    uint32_t s = seed ? seed : 0x9E3779B9u;
    w1 = xorshift32(s);
    w2 = xorshift32(s);
    w3 = xorshift32(s);
    w4 = xorshift32(s);
  }
  LKS_HD uint32_t word(int q) {
    if (!(q & 1)) {
      switch (q >> 1) {
      case 0: w = w1; break;
      case 1: w = w3; break;
      case 2: w = w4; break;
      case 3: w = w1 ^ w2; break;
      case 4: w = w1 ^ w3; break;
      case 5: w = w1 ^ w4; break;
      case 6: w = w3 ^ w4; break;
      case 7: w = (w1 ^ w2) ^ w4; break;
      case 8: w = (w1 ^ w3) ^ w4; break;
      default: w = w2; break;
      }
    }
    return (q & 1) ? w << 16 : w;
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

// binary32 -> binary16 with the top 13 bits of r.  From binary16's normal
// range up (|v| >= 2^-14, and zeros and non-finite values) the 13 bits are
// added below binary16's last place, which lies 13 bits above binary32's,
// and truncated there; a carry past 65504 gives infinity.  Below, binary16's
// spacing is 2^-24: the result is sign(v) trunc(|v| 2^24 + r13 2^-13) 2^-24,
// computed here in units of 2^-37 as trunc((trunc(|v| 2^37) + r13) 2^-13)
// (equal, as r13 is an integer).
LKS_HD inline _Float16 sr_f16(float v, uint32_t r) {
#if defined(__HIP_DEVICE_COMPILE__)
  typedef _Float16 h2 __attribute__((ext_vector_type(2)));
  return __builtin_amdgcn_cvt_sr_f16_f32(h2{}, v, r, false)[0];
#else
  const uint32_t b = bits32(v), m = b & 0x7FFFFFFFu;
  if (m >= 0x38800000u || m == 0u) return (_Float16)flt((b + (r >> 19)) & ~0x1FFFu);
  const uint32_t e8 = m >> 23; // biased exponent; 0 for binary32 subnormals
  const uint32_t sig = e8 ? (m & 0x7FFFFFu) | 0x800000u : m;
  // |v| = sig 2^(E - 23), E = e8 - 127 (or -126): in units of 2^-37 that is
  // sig 2^(e8 - 113), a right shift of at least 1 here
  const int rs = 113 - (int)(e8 ? e8 : 1);
  const uint32_t u = rs < 32 ? sig >> rs : 0u;
  const uint32_t t = (u + (r >> 19)) >> 13; // result in units of 2^-24, <= 2^10
  const float mag = (float)t * 0x1p-24f;   // exact
  return (_Float16)flt((b & 0x80000000u) | bits32(mag));
#endif
}

// v rounded stochastically to binary16 (sr_f16) into the low (HIGH false)
// or high half of the pair (lo, hi); the other half is kept.
template <bool HIGH>
LKS_HD inline void sr_f16_half(_Float16 &lo, _Float16 &hi, float v, uint32_t r) {
#if defined(__HIP_DEVICE_COMPILE__)
  typedef _Float16 h2 __attribute__((ext_vector_type(2)));
  h2 p = {lo, hi};
  p = __builtin_amdgcn_cvt_sr_f16_f32(p, v, r, HIGH);
  lo = p[0];
  hi = p[1];
#else
  (HIGH ? hi : lo) = sr_f16(v, r);
#endif
}

// Two values rounded stochastically to binary16 (sr_f16 each), returned as
// the low and high halves of one register's pair.
LKS_HD inline void sr_f16_pair(float a, float b, uint32_t ra, uint32_t rb, _Float16 &oa,
                               _Float16 &ob) {
#if defined(__HIP_DEVICE_COMPILE__)
  typedef _Float16 h2 __attribute__((ext_vector_type(2)));
  h2 p = __builtin_amdgcn_cvt_sr_f16_f32(h2{}, a, ra, false);
  p = __builtin_amdgcn_cvt_sr_f16_f32(p, b, rb, true);
  oa = p[0];
  ob = p[1];
#else
  oa = sr_f16(a, ra);
  ob = sr_f16(b, rb);
#endif
}

// Stochastic rounding of v (compute type C) to storage type S; identity for
// equal types.
template <typename S, typename C>
LKS_HD inline S round_sr(C v, uint32_t r) {
  if constexpr (sizeof(S) == sizeof(C)) {
    (void)r;
    return (S)v;
  } else {
    if constexpr (sizeof(S) == 4) return sr_f32(v, r);
    // binary64 goes to the nearest binary32 first: that moves v by at most
    // 2^-25 |v|, 2^-14 of a binary16 spacing, and leaves the rest to one
    // hardware conversion where rounding at v's binary16 spacing in FP64 took
    // ten FP64 instructions (the binary16 step is arithmetic-bound)
    else return sr_f16((float)v, r);
  }
}

} // namespace lks
