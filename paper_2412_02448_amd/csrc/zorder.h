// The z-order composite attribute of two attributes (the paper's multi-attribute
// discussion in Sec. 5.9, approach 2): each attribute maps to an order-preserving
// coordinate on a 2^31-cell axis, and the key interleaves the two coordinates' bits.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace unify {

constexpr uint64_t ZTOP = (1ull << 31) - 1;  // last cell of an axis

// Coordinate of x on an axis with smallest value base: 0 at or below base, else
// (x - base) taken modulo 2^64 and shifted right by shift (left by -shift when
// negative), capped at ZTOP.  Non-decreasing in x.
__host__ __device__ __forceinline__ uint64_t zcoord(int64_t x, int64_t base, int32_t shift) {
  if (x <= base) return 0;
  const uint64_t t = static_cast<uint64_t>(x) - static_cast<uint64_t>(base);
  if (shift >= 0) {
    const uint64_t u = t >> shift;
    return u < ZTOP ? u : ZTOP;
  }
  return t > (ZTOP >> -shift) ? ZTOP : t << -shift;
}

// The 31 low bits of x moved to the even bit positions (bit j to bit 2j), by the
// usual halving mask sequence.
__host__ __device__ __forceinline__ uint64_t zspread(uint64_t x) {
  x &= ZTOP;
  x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
  x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
  x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
  x = (x | (x << 2)) & 0x3333333333333333ull;
  x = (x | (x << 1)) & 0x5555555555555555ull;
  return x;
}

// Key of the cell (u1, u2): u1's bits in the odd positions, u2's in the even ones.
__host__ __device__ __forceinline__ int64_t zkey(uint64_t u1, uint64_t u2) {
  return static_cast<int64_t>((zspread(u1) << 1) | zspread(u2));
}

}  // namespace unify
