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

// FP8 scale of a row: max_t |x_t| / 448, 1 for a zero row.  The division is
// done in FP64 and rounded to FP32, which gives the correctly rounded FP32
// quotient (FP64 carries more than twice FP32's significand plus two bits).
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
    if (mx > 0.0f) s = (float)((double)mx / 448.0);
  }
  double e2 = 0.0;
  for (int t = lane; t < d; t += 64) {
    const float xt = x[t];
    float back;
    if constexpr (PREC == UNIFY_BF16) {
      const uint32_t c = f32_to_bf16(xt);
      bf[v * d + t] = (uint16_t)c;
      back = bf16_to_f32(c);
    } else {
      const float y = (float)((double)xt / (double)s);
      const uint32_t c = f32_to_e4m3(y);
      f8[v * d + t] = (uint8_t)c;
      back = fp8_value(c, s);
    }
    const double e = (double)back - (double)xt;  // exact in FP64
    e2 += e * e;
  }
  for (int o = 32; o >= 1; o >>= 1) e2 += __shfl_xor(e2, o, 64);
  if (lane == 0) {
    if constexpr (PREC == UNIFY_FP8E4M3) scale[v] = s;
    // FP64 rounding of the sum and the root is far below 2^-30 relative
    eps[v] = __double2float_ru(sqrt(e2) * (1.0 + 0x1p-30));
  }
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
    return UNIFY_OK;
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
  return UNIFY_OK;
}

}  // namespace unify
