// FP64 -> FP16 conversion with a single round-to-nearest-even step, done on
// the bit pattern (IEEE 754-2008 binary64 -> binary16).  Converting through
// FP32 rounds twice and can land one FP16 ulp away: 1 + 2^-11 + 2^-30 rounds
// up to 1 + 2^-10 here, but to 1 through FP32 (the FP32 step leaves a tie,
// which the FP16 step breaks to even).  The reduced-precision link stores are
// defined with the single rounding.  Plain C++, usable in host and device code.
#pragma once
#include <stdint.h>
#include <string.h>

#if defined(__HIPCC__)
#define QIRAL_HD __host__ __device__
#else
#define QIRAL_HD
#endif

namespace qiral {

QIRAL_HD inline uint16_t d2h_rne(double d) {
  uint64_t b;
  memcpy(&b, &d, sizeof b);
  const uint16_t sign = (uint16_t)((b >> 48) & 0x8000u);
  const int e = (int)((b >> 52) & 0x7ff);
  const uint64_t m = b & 0xfffffffffffffull;
  if (e == 0x7ff) return (uint16_t)(sign | 0x7c00u | (m ? 0x200u : 0u));   // Inf, NaN (quiet)
  const int E = e - 1023;                                                   // unbiased exponent
  if (E > 15) return (uint16_t)(sign | 0x7c00u);                            // beyond the FP16 range
  if (E < -25) return sign;   // below half the smallest FP16 subnormal (2^-25): rounds to 0
  const uint64_t sig = e ? (m | (1ull << 52)) : m;                          // 53-bit significand
  // keep 11 significant bits for a normal result (E >= -14); fewer for a
  // subnormal one, whose unit is 2^-24
  const int shift = E >= -14 ? 42 : 42 + (-14 - E);                         // 42 .. 53
  uint64_t q = sig >> shift;
  const uint64_t rem = sig & ((1ull << shift) - 1), half = 1ull << (shift - 1);
  if (rem > half || (rem == half && (q & 1))) ++q;
  // normal: q in [2^10, 2^11] (2^11 carries into the exponent); subnormal: q in [0, 2^10]
  const uint32_t bits = E >= -14 ? ((uint32_t)(E + 15) << 10) + (uint32_t)(q - 1024) : (uint32_t)q;
  if (bits >= 0x7c00u) return (uint16_t)(sign | 0x7c00u);                  // rounded past 65504
  return (uint16_t)(sign | bits);
}

}  // namespace qiral
