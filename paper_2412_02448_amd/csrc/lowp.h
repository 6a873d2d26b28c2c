// Low-precision vector stores: BF16 and OCP FP8 E4M3 with one FP32 scale per
// vector.  The graph searches may rank objects by distances to such a copy and
// re-score their best results with the FP32 vectors.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace unify {

// BF16 = the upper half of an FP32 pattern.
__device__ __forceinline__ float bf16_to_f32(uint32_t b) { return __uint_as_float(b << 16); }

// Nearest BF16 (ties to the even significand); NaN stays a quiet NaN.
__device__ __forceinline__ uint32_t f32_to_bf16(float x) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (u >> 16) | 0x40u;
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// OCP FP8 E4M3 (no infinities; 0x7F/0xFF are NaN): value = (-1)^s 2^(e-7) (1 + m/8),
// subnormals 2^-6 m/8.  Placing the 7 magnitude bits at FP32 bits 20..26 gives
// 2^(e-127) (1 + m/8), or the FP32 subnormal m 2^-129 when e = 0; scaling by
// 2^120 is exact and yields the E4M3 value in both cases.  The NaN codes are
// never written by the encoder below (finite inputs) and decode to +-480.
__device__ __forceinline__ float e4m3_to_f32(uint32_t c) {
  const uint32_t bits = ((c & 0x80u) << 24) | ((c & 0x7Fu) << 20);
  return __uint_as_float(bits) * 0x1p120f;
}

// Nearest E4M3 code (ties to the even significand); magnitudes of 448 and above
// clamp to 448; NaN -> 0x7F.
__device__ __forceinline__ uint32_t f32_to_e4m3(float y) {
  const uint32_t u = __float_as_uint(y);
  const uint32_t sign = (u >> 24) & 0x80u;
  const uint32_t a = u & 0x7FFFFFFFu;
  if (a > 0x7F800000u) return 0x7Fu;
  if (a >= 0x43E00000u) return sign | 0x7Eu;  // 448 = 1.75 * 2^8
  if (a < 0x3C800000u) {                      // below 2^-6: the subnormal grid m * 2^-9
    const float t = __uint_as_float(a) * 512.0f;  // exact
    return sign | (uint32_t)__builtin_rintf(t);   // 0..8; 8 is the smallest normal's code
  }
  // keep 3 significand bits; round the dropped 20 to nearest, ties to even
  const uint32_t r = a + 0x7FFFFu + ((a >> 20) & 1u);
  return sign | ((((r >> 23) - 120u) << 3) | ((r >> 20) & 7u));
}

// Value of an FP8 component: code value times the vector's scale, rounded once
// to FP32.  Written as an fma with +0 so that the product can never be fused
// into a later subtraction (the rounded product is the stored value).
__device__ __forceinline__ float fp8_value(uint32_t c, float scale) {
  return __builtin_fmaf(e4m3_to_f32(c), scale, 0.0f);
}

}  // namespace unify
