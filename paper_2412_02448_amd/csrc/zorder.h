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

// The bits at the even positions of x gathered into the low 31 bits (the inverse of zspread).
__host__ __device__ __forceinline__ uint64_t zcompact(uint64_t x) {
  x &= 0x5555555555555555ull;
  x = (x | (x >> 1)) & 0x3333333333333333ull;
  x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
  x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
  x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
  x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
  return x;
}

// The smallest key above z whose cell lies in the box of cells spanned by the keys lo
// (its lower corner) and hi (its upper corner), for a key z below hi outside the box;
// -1 when there is none (the search for the next box key of Tropf and Herzog's range
// search on z-ordered data).  From the top bit down, the box is split at each bit where
// its corners differ: when z lies below the split, the upper part's first key is the
// answer should nothing of the lower part follow z; when z lies above it, only the upper
// part can hold the answer.
__host__ __device__ __forceinline__ int64_t znext(uint64_t z, uint64_t lo, uint64_t hi) {
  int64_t best = -1;
  for (int b = 61; b >= 0; --b) {
    const uint64_t m = 1ull << b;
    // the bits of this bit's coordinate below it
    const uint64_t below = (m - 1) & ((b & 1) ? 0xAAAAAAAAAAAAAAAAull : 0x5555555555555555ull);
    const bool zb = z & m, lb = lo & m, hb = hi & m;
    if (lb == hb) {
      if (zb == lb) continue;
      // z leaves the box's span at this bit: below it, the box's first key follows z;
      // above it, nothing of the box (or of the part kept) does
      return zb ? best : static_cast<int64_t>(lo);
    }
    // the corners differ (lo 0, hi 1): the lower part ends with hi's coordinate at
    // 0111..., the upper part starts with lo's at 1000...
    const uint64_t up = (lo & ~below) | m;
    if (!zb) {
      best = static_cast<int64_t>(up);
      hi = (hi & ~m) | below;
    } else {
      lo = up;
    }
  }
  return best;
}

}  // namespace unify
