// alp_keys.h -- FP32 values as unsigned integer keys that order like the
// values, for reductions with integer LDS atomics (min / max).  No HIP header
// here, so a host compiler can include it with ALP_HD defined empty and test
// the ordering.
#pragma once
#include <stdint.h>

#ifndef ALP_HD
#define ALP_HD __host__ __device__ __forceinline__
#endif

namespace alp {

ALP_HD uint32_t f32_bits(float x) { return __builtin_bit_cast(uint32_t, x); }
ALP_HD float f32_from_bits(uint32_t b) { return __builtin_bit_cast(float, b); }

// Finite x: the sign bit set for x with a clear sign bit, every bit flipped
// for x with a set one, so that x < y gives key(x) < key(y).  (-0 keys just
// below +0; both decode to themselves.)  Non-negative values also order like
// their plain bits, which the max reductions of squared lengths use.
ALP_HD uint32_t f32_key(float x) {
  const uint32_t b = f32_bits(x);
  return (b & 0x80000000u) ? ~b : b | 0x80000000u;
}
ALP_HD float f32_of_key(uint32_t k) { return f32_from_bits((k & 0x80000000u) ? k & 0x7fffffffu : ~k); }

}  // namespace alp
