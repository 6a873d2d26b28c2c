// Builds the BF16 or FP8 copy of the resident FP32 vectors on the device, with
// the per-vector error bound eps_v >= ||copy_v - x_v|| that lets the pre-filter
// scan rank by the copy and still return the exact FP32 result.
#include <hip/hip_runtime.h>

#include <cmath>

#include "lowp.h"
#include "unify_internal.h"

namespace unify {
namespace {

constexpr int QW = 4;  // rows (one wavefront each) per 256-thread block

// FP8 scale of a row: max_t |x_t| / 448, 1 for a zero row, by correctly rounded
// FP32 division (the device default for `/`), as are the quotients x_t / s.
// eps_v bounds ||copy_v - x_v||: each difference e_t = back_t - x_t is exact in
// FP32 (the two values lie within a factor of two of each other, or one is
// zero), and the sum of the e_t^2 passes through at most d / 64 + 7 roundings
// to nearest (products, a lane's sum, six shuffle additions), so widening the
// root of the computed sum by 2^-18 relative covers them for d <= 2048; 1e-21
// covers squares that underflow.  An exact copy gets 0.
template <int PREC>
__global__ void __launch_bounds__(256) k_quant(const float* __restrict__ vec, int64_t n, int d,
                                               uint16_t* __restrict__ bf, uint8_t* __restrict__ f8,
                                               float* __restrict__ scale, float* __restrict__ eps) {
  const int lane = threadIdx.x & 63;
  const int64_t v = (int64_t)blockIdx.x * QW + (threadIdx.x >> 6);
  if (v >= n) return;  // uniform per wavefront
  const float* x = vec + v * d;
  float s = 1.0f;
  if constexpr (PREC == UNIFY_FP8E4M3) {
    float mx = 0.0f;
    for (int t = lane; t < d; t += 64) mx = fmaxf(mx, fabsf(x[t]));
    for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    if (mx > 0.0f) s = mx / 448.0f;
  }
  float e2 = 0.0f;
  bool nz = false;  // some difference is not zero (its square may underflow)
  for (int t = lane; t < d; t += 64) {
    const float xt = x[t];
    float back;
    if constexpr (PREC == UNIFY_BF16) {
      const uint32_t c = f32_to_bf16(xt);
      bf[v * d + t] = (uint16_t)c;
      back = bf16_to_f32(c);
    } else {
      const uint32_t c = f32_to_e4m3(xt / s);
      f8[v * d + t] = (uint8_t)c;
      back = fp8_value(c, s);
    }
    const float e = back - xt;  // exact
    e2 = __builtin_fmaf(e, e, e2);
    nz = nz || e != 0.0f;
  }
  for (int o = 32; o >= 1; o >>= 1) e2 += __shfl_xor(e2, o, 64);
  nz = __ballot(nz) != 0;
  if (lane == 0) {
    if constexpr (PREC == UNIFY_FP8E4M3) scale[v] = s;
    eps[v] = nz ? __builtin_sqrtf(e2) * (1.0f + 0x1p-18f) + 1e-21f : 0.0f;  // 0 exactly for an exact copy
  }
}

// Squared norm of every row of the store PREC (as the searches decode it),
// in FP32 by fused multiply-adds: the norm-expansion scan bounds its error by
// (d + 8) u times the exact value.
template <int PREC>
__global__ void __launch_bounds__(256) k_rownorm(DevIndex ix, float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t v = (int64_t)blockIdx.x * QW + (threadIdx.x >> 6);
  if (v >= ix.n) return;  // uniform per wavefront
  const int d = ix.d;
  float acc = 0.0f;
  for (int t = lane; t < d; t += 64) {
    float x;
    if constexpr (PREC == UNIFY_FP32) x = ix.vec[v * d + t];
    else if constexpr (PREC == UNIFY_BF16) x = bf16_to_f32(ix.vec_bf16[v * d + t]);
    else x = fp8_value(ix.vec_fp8[v * d + t], ix.vec_scale[v]);
    acc = __builtin_fmaf(x, x, acc);
  }
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) out[v] = acc;
}

// The squared row norms of the store `precision` (built the first time), made
// the ones later searches read.  Synchronous.
int store_norms(unify_index_t ix, int precision) {
  DevIndex& dv = ix->dv;
  if (!ix->nrm_of[precision] && dv.n > 0) {
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(float) * dv.n) != hipSuccess) {
      set_error("device allocation failed (row norms)");
      return UNIFY_ENOMEM;
    }
    ix->allocs.push_back(p);
    const dim3 grid((unsigned)((dv.n + QW - 1) / QW));
    if (precision == UNIFY_BF16) hipLaunchKernelGGL(k_rownorm<UNIFY_BF16>, grid, dim3(256), 0, 0, dv, (float*)p);
    else if (precision == UNIFY_FP8E4M3)
      hipLaunchKernelGGL(k_rownorm<UNIFY_FP8E4M3>, grid, dim3(256), 0, 0, dv, (float*)p);
    else hipLaunchKernelGGL(k_rownorm<UNIFY_FP32>, grid, dim3(256), 0, 0, dv, (float*)p);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
      set_error("row-norm kernel failed");
      return UNIFY_EDEVICE;
    }
    ix->nrm_of[precision] = (const float*)p;
  }
  dv.vec_nrm = ix->nrm_of[precision];
  return UNIFY_OK;
}

}  // namespace

// Makes `precision` the store the searches read, first building the copy of
// dv.vec and its error bounds when the index does not hold it yet (the
// allocations join ix->allocs).  Synchronous.
int quantize_store(unify_index_t ix, int precision) {
  DevIndex& dv = ix->dv;
  const bool have = precision == UNIFY_FP32 || (precision == UNIFY_BF16 && dv.vec_bf16) ||
                    (precision == UNIFY_FP8E4M3 && dv.vec_fp8) || dv.n == 0;
  if (have) {
    dv.precision = precision;
    dv.vec_eps = ix->eps_of[precision];
    return store_norms(ix, precision);
  }
  const size_t cells = (size_t)dv.n * dv.d;
  auto alloc = [&](size_t bytes, void** p) {
    if (hipMalloc(p, bytes) != hipSuccess) {
      set_error("device allocation failed (low-precision store)");
      return false;
    }
    ix->allocs.push_back(*p);
    return true;
  };
  void *codes = nullptr, *sc = nullptr, *ep = nullptr;
  const size_t esz = precision == UNIFY_BF16 ? 2 : 1;
  if (!alloc(cells * esz, &codes) || !alloc(sizeof(float) * dv.n, &ep)) return UNIFY_ENOMEM;
  if (precision == UNIFY_FP8E4M3 && !alloc(sizeof(float) * dv.n, &sc)) return UNIFY_ENOMEM;
  const dim3 grid((unsigned)((dv.n + QW - 1) / QW));
  if (precision == UNIFY_BF16)
    hipLaunchKernelGGL(k_quant<UNIFY_BF16>, grid, dim3(256), 0, 0, dv.vec, dv.n, dv.d, (uint16_t*)codes,
                       (uint8_t*)nullptr, (float*)nullptr, (float*)ep);
  else
    hipLaunchKernelGGL(k_quant<UNIFY_FP8E4M3>, grid, dim3(256), 0, 0, dv.vec, dv.n, dv.d, (uint16_t*)nullptr,
                       (uint8_t*)codes, (float*)sc, (float*)ep);
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    set_error("quantisation kernel failed");
    return UNIFY_EDEVICE;
  }
  if (precision == UNIFY_BF16) {
    dv.vec_bf16 = (const uint16_t*)codes;
  } else {
    dv.vec_fp8 = (const uint8_t*)codes;
    dv.vec_scale = (const float*)sc;
  }
  ix->eps_of[precision] = (const float*)ep;
  dv.precision = precision;
  dv.vec_eps = (const float*)ep;
  return store_norms(ix, precision);
}

}  // namespace unify
