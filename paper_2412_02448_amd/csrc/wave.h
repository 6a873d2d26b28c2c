// Wavefront-level building blocks for gfx950 (64 lanes): 64-bit key shuffles,
// bitonic sort / merge across lanes, ballot-based compaction, and the
// canonical FP32 squared distance evaluated by 16 lanes per vector.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace unify {

typedef unsigned long long u64;
constexpr u64 KEY_MAX = ~0ull;
constexpr int WAVE = 64;

// Key = (FP32 distance bits, id).  Distances are >= +0, so comparing the keys
// as unsigned 64-bit integers orders by (distance, id).
__device__ __forceinline__ u64 make_key(float d, int32_t id) {
  return ((u64)__float_as_uint(d) << 32) | (uint32_t)id;
}
__device__ __forceinline__ float key_dist(u64 k) { return __uint_as_float((uint32_t)(k >> 32)); }
__device__ __forceinline__ int32_t key_id(u64 k) { return (int32_t)(uint32_t)k; }

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ u64 shfl64(u64 v, int src) {
  uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, WAVE);
  uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, WAVE);
  return ((u64)hi << 32) | lo;
}
__device__ __forceinline__ u64 shfl_xor64(u64 v, int m) {
  uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, WAVE);
  uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, WAVE);
  return ((u64)hi << 32) | lo;
}

// Value of lane (lane ^ M), by DPP for M <= 8 (no LDS round trip):
//   xor 1, 2: quad permutations; xor 4: quad [3,2,1,0] then half-row mirror
//   (lane i reads i ^ 7, which holds the value of (i ^ 7) ^ 3 = i ^ 4);
//   xor 8: row rotation by 8 (i +- 8 mod 16 = i ^ 8).
template <int M>
__device__ __forceinline__ uint32_t xor_lane32(uint32_t x) {
  if constexpr (M == 1) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false);
  } else if constexpr (M == 2) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false);
  } else if constexpr (M == 4) {
    const int y = __builtin_amdgcn_update_dpp(0, (int)x, 0x1B, 0xF, 0xF, false);
    return (uint32_t)__builtin_amdgcn_update_dpp(0, y, 0x141, 0xF, 0xF, false);
  } else if constexpr (M == 8) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x128, 0xF, 0xF, false);
  } else {
    return (uint32_t)__shfl_xor((int)x, M, WAVE);
  }
}
template <int M>
__device__ __forceinline__ u64 xor_lane64(u64 v) {
  return ((u64)xor_lane32<M>((uint32_t)(v >> 32)) << 32) | xor_lane32<M>((uint32_t)v);
}
// Value of lane (i - n) mod 16 within each 16-lane row (DPP row rotate right).
template <int N>
__device__ __forceinline__ float row_ror(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x120 + N, 0xF, 0xF, false));
}
template <int N>
__device__ __forceinline__ uint32_t row_ror_u(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x120 + N, 0xF, 0xF, false);
}

__device__ __forceinline__ u64 umin64(u64 a, u64 b) { return a < b ? a : b; }
__device__ __forceinline__ u64 umax64(u64 a, u64 b) { return a < b ? b : a; }

// Lanes below this one whose bit is set in mask.
__device__ __forceinline__ int rank_in(u64 mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}
__device__ __forceinline__ u64 ballot(bool p) { return __ballot(p); }

// Wave-wide minimum of a 64-bit key (rows by DPP rotation, then across rows).
__device__ __forceinline__ u64 wave_min64(u64 v) {
  u64 o;
  o = ((u64)row_ror_u<8>((uint32_t)(v >> 32)) << 32) | row_ror_u<8>((uint32_t)v);
  v = umin64(v, o);
  o = ((u64)row_ror_u<4>((uint32_t)(v >> 32)) << 32) | row_ror_u<4>((uint32_t)v);
  v = umin64(v, o);
  o = ((u64)row_ror_u<2>((uint32_t)(v >> 32)) << 32) | row_ror_u<2>((uint32_t)v);
  v = umin64(v, o);
  o = ((u64)row_ror_u<1>((uint32_t)(v >> 32)) << 32) | row_ror_u<1>((uint32_t)v);
  v = umin64(v, o);
  v = umin64(v, shfl_xor64(v, 16));
  v = umin64(v, shfl_xor64(v, 32));
  return v;
}

// One compare-exchange step of a bitonic network: partner lane ^ J; the lower
// lane keeps the minimum when `asc`, else the maximum.
template <int J>
__device__ __forceinline__ u64 cmpx(u64 x, bool asc, int lane) {
  const u64 y = xor_lane64<J>(x);
  const bool low = (lane & J) == 0;
  return (low == asc) ? umin64(x, y) : umax64(x, y);
}

// Bitonic sort of one key per lane, ascending by lane index.
__device__ __forceinline__ u64 sort64(u64 x) {
  const int lane = lane_id();
  x = cmpx<1>(x, (lane & 2) == 0, lane);
  x = cmpx<2>(x, (lane & 4) == 0, lane);
  x = cmpx<1>(x, (lane & 4) == 0, lane);
  x = cmpx<4>(x, (lane & 8) == 0, lane);
  x = cmpx<2>(x, (lane & 8) == 0, lane);
  x = cmpx<1>(x, (lane & 8) == 0, lane);
  x = cmpx<8>(x, (lane & 16) == 0, lane);
  x = cmpx<4>(x, (lane & 16) == 0, lane);
  x = cmpx<2>(x, (lane & 16) == 0, lane);
  x = cmpx<1>(x, (lane & 16) == 0, lane);
  x = cmpx<16>(x, (lane & 32) == 0, lane);
  x = cmpx<8>(x, (lane & 32) == 0, lane);
  x = cmpx<4>(x, (lane & 32) == 0, lane);
  x = cmpx<2>(x, (lane & 32) == 0, lane);
  x = cmpx<1>(x, (lane & 32) == 0, lane);
  x = cmpx<32>(x, true, lane);
  x = cmpx<16>(x, true, lane);
  x = cmpx<8>(x, true, lane);
  x = cmpx<4>(x, true, lane);
  x = cmpx<2>(x, true, lane);
  x = cmpx<1>(x, true, lane);
  return x;
}

// a, b ascending across lanes -> a = 64 smallest of both (ascending),
// b = 64 largest (ascending).
__device__ __forceinline__ void merge64(u64& a, u64& b) {
  const int lane = lane_id();
  u64 br = shfl64(b, WAVE - 1 - lane);
  u64 lo = umin64(a, br), hi = umax64(a, br);
  lo = cmpx<32>(lo, true, lane);
  hi = cmpx<32>(hi, true, lane);
  lo = cmpx<16>(lo, true, lane);
  hi = cmpx<16>(hi, true, lane);
  lo = cmpx<8>(lo, true, lane);
  hi = cmpx<8>(hi, true, lane);
  lo = cmpx<4>(lo, true, lane);
  hi = cmpx<4>(hi, true, lane);
  lo = cmpx<2>(lo, true, lane);
  hi = cmpx<2>(hi, true, lane);
  lo = cmpx<1>(lo, true, lane);
  hi = cmpx<1>(hi, true, lane);
  a = lo;
  b = hi;
}

// Sorted list of keys in LDS, `cap` entries used at most, `len` valid.
// Inserts a batch (one key per lane, KEY_MAX = none; need not be sorted);
// keeps the `cap` smallest.  len is wave-uniform.
__device__ __forceinline__ void list_insert(u64* lst, int& len, int cap, u64 key) {
  const int lane = lane_id();
  const int add = __popcll(ballot(key != KEY_MAX));
  if (add == 0) return;
  u64 carry = sort64(key);
  const int total = min(len + add, cap);
  const int used_blocks = (len + WAVE - 1) / WAVE;
  const int new_blocks = (total + WAVE - 1) / WAVE;
  for (int blk = 0; blk < new_blocks; ++blk) {
    u64 a = blk < used_blocks ? lst[blk * WAVE + lane] : KEY_MAX;
    merge64(a, carry);
    const int pos = blk * WAVE + lane;
    lst[pos] = pos < total ? a : KEY_MAX;
  }
  len = total;
}

// Canonical FP32 squared distance of 4 vectors per wave (16 lanes each).
// Lane s = lane & 15 owns the 4-element groups g = s, s + 16, ... (< d / 4) and
// accumulates them in increasing order with fused multiply-adds; the 16
// partials are then combined by the butterfly P[s] + P[s ^ 8], then ^ 4, ^ 2,
// ^ 1.  Rotating by 8, 4, 2, 1 within the row computes exactly that tree: after
// the step for t, every partial is unchanged by xor-ing bits >= log2(t) of its
// lane, and (s - t) mod 16 differs from s ^ t only in those bits.  Every lane of
// the row ends with the same value.
__device__ __forceinline__ float group_reduce16(float p) {
  p = p + row_ror<8>(p);
  p = p + row_ror<4>(p);
  p = p + row_ror<2>(p);
  p = p + row_ror<1>(p);
  return p;
}

__device__ __forceinline__ float fma_sq4(float4 x, float4 q, float acc) {
#pragma clang fp contract(off)
  float e0 = x.x - q.x;
  acc = __builtin_fmaf(e0, e0, acc);
  float e1 = x.y - q.y;
  acc = __builtin_fmaf(e1, e1, acc);
  float e2 = x.z - q.z;
  acc = __builtin_fmaf(e2, e2, acc);
  float e3 = x.w - q.w;
  acc = __builtin_fmaf(e3, e3, acc);
  return acc;
}

// Keys of cnt vectors, four per round (16 lanes each), RB rounds of loads in
// flight: id_of(i) names the i-th vector, load(v, g) returns its 4-element group
// g as FP32; the key of the i-th lands in keys[i] (LDS).
template <int NG, class IdOf, class Load4>
__device__ __forceinline__ void eval_keys_generic(int G, const float4 (&qv)[NG], int cnt, IdOf id_of,
                                                  Load4 load, u64* keys) {
  constexpr int RB = NG <= 2 ? 4 : (NG <= 4 ? 2 : 1);
  const int lane = lane_id();
  const int s = lane & 15, g4 = lane >> 4;
  for (int base = 0; base < cnt; base += 4 * RB) {
    float4 x[RB][NG];
    int32_t vid[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int idx = base + 4 * r + g4;
      vid[r] = idx < cnt ? id_of(idx) : -1;
#pragma unroll
      for (int i = 0; i < NG; ++i) {
        const int g = s + 16 * i;
        x[r][i] = (vid[r] >= 0 && g < G) ? load((int64_t)vid[r], g) : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      float acc = 0.0f;
#pragma unroll
      for (int i = 0; i < NG; ++i) {
        if (s + 16 * i < G) acc = fma_sq4(x[r][i], qv[i], acc);
      }
      acc = group_reduce16(acc);
      const int idx = base + 4 * r + g4;
      if (s == 0 && idx < cnt) keys[idx] = make_key(acc, vid[r]);
    }
  }
}

}  // namespace unify
