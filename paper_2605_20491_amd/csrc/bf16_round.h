// Rounding to BF16 (1 sign, 8 exponent, 7 fraction bits), the same code on the
// host and the device.
//
// Two routes are used by the library:
//  * factor copies: FP64 -> BF16 rounded once to nearest, ties to even
//    (bf16_from_f64), in integer arithmetic on the FP64 bit pattern, so the
//    result does not depend on the FP32 conversion or denormal mode;
//  * data: values are taken to FP32 first (round to nearest even, as the
//    FP32-input paths hold them) and then rounded to BF16 (bf16_from_f32).
//    For FP64 data this rounds twice; it differs from bf16_from_f64 exactly
//    when the FP32 rounding lands on a BF16 midpoint, about 2^-17 of values.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ts {

// FP32 -> BF16, nearest even.  Inf stays Inf; NaN stays NaN (quiet bit set).
__host__ __device__ inline uint16_t bf16_from_f32(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Shift a significand right by s >= 1 bits, rounding to nearest even.
__host__ __device__ inline uint64_t shr_rne(uint64_t m, int s) {
  if (s >= 64) return 0;
  const uint64_t q = m >> s;
  const uint64_t rem = m & ((1ull << s) - 1ull);
  const uint64_t half = 1ull << (s - 1);
  return q + ((rem > half || (rem == half && (q & 1ull))) ? 1ull : 0ull);
}

// FP64 -> BF16, rounded once to nearest even (subnormal BF16 results kept).
__host__ __device__ inline uint16_t bf16_from_f64(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint16_t sign = (uint16_t)((u >> 63) << 15);
  const int ex = (int)((u >> 52) & 0x7ff);
  const uint64_t frac = u & ((1ull << 52) - 1ull);
  if (ex == 0x7ff) return (uint16_t)(sign | 0x7f80u | (frac ? 0x40u : 0u));
  if (ex == 0) return sign;  // FP64 subnormals are far below the BF16 range
  const uint64_t m = (1ull << 52) | frac;  // value = m * 2^(e - 52)
  const int e = ex - 1023;
  if (e >= -126) {
    uint64_t r = shr_rne(m, 45);  // 8-bit significand, may carry to 2^8
    int eb = e + 127;
    if (r == (1ull << 8)) { r >>= 1; eb += 1; }
    if (eb >= 255) return (uint16_t)(sign | 0x7f80u);
    return (uint16_t)(sign | ((uint16_t)eb << 7) | (uint16_t)(r & 0x7fu));
  }
  // subnormal BF16: units of 2^-133; r == 128 is the smallest normal, same encoding
  const uint64_t r = shr_rne(m, -(e + 81));
  return (uint16_t)(sign | (uint16_t)r);
}

}  // namespace ts
