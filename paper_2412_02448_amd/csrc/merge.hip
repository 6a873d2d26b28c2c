// Disjunctive two-attribute queries (the paper's multi-attribute extension,
// approach 1): one HSIG per attribute, each searched with its own range, and
// the two result lists of every query merged.  Over the same objects (same
// external ids and vectors) an object found by both searches carries the same
// canonical FP32 distance in both lists, so merging by (distance, id) and
// dropping repeated keys leaves the k nearest distinct objects; with exact
// per-index answers this is the exact answer of the OR query.
#include <hip/hip_runtime.h>

#include "unify_internal.h"

namespace unify {
namespace {

// One thread per query: a two-way merge of two ascending lists (-1 / +inf
// padded), distinct keys only.
__global__ void __launch_bounds__(256) k_merge_or(const int64_t* __restrict__ ia, const float* __restrict__ da,
                                                  const int64_t* __restrict__ ib, const float* __restrict__ db,
                                                  int64_t nq, int k, int64_t* __restrict__ oi,
                                                  float* __restrict__ od) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  const int64_t* A = ia + q * k;
  const int64_t* B = ib + q * k;
  const float* DA = da + q * k;
  const float* DB = db + q * k;
  int a = 0, b = 0, w = 0;
  int run = 0;  // first output of the current run of equal distances
  while (w < k) {
    const bool ha = a < k && A[a] >= 0, hb = b < k && B[b] >= 0;
    if (!ha && !hb) break;
    bool take_a;
    if (ha && hb) take_a = DA[a] < DB[b] || (DA[a] == DB[b] && A[a] <= B[b]);
    else take_a = ha;
    const int64_t id = take_a ? A[a] : B[b];
    const float d = take_a ? DA[a] : DB[b];
    if (take_a) ++a;
    else ++b;
    // the same object from the other list has the same distance: it is already in this run
    if (w > 0 && d == od[q * k + w - 1]) {
      bool seen = false;
      for (int t = run; t < w; ++t) seen |= oi[q * k + t] == id;
      if (seen) continue;
    } else {
      run = w;
    }
    oi[q * k + w] = id;
    od[q * k + w] = d;
    ++w;
  }
  for (; w < k; ++w) {
    oi[q * k + w] = -1;
    od[q * k + w] = __builtin_inff();
  }
}

}  // namespace
}  // namespace unify

using namespace unify;

extern "C" int unify_merge_or(const int64_t* ids_a, const float* dist_a, const int64_t* ids_b, const float* dist_b,
                              int64_t nq, int32_t k, int64_t* out_ids, float* out_dist, void* hip_stream) {
  if (nq < 0 || k < 1 || (nq > 0 && (!ids_a || !dist_a || !ids_b || !dist_b || !out_ids || !out_dist))) {
    set_error("unify_merge_or: bad arguments");
    return UNIFY_EINVAL;
  }
  if (nq == 0) return UNIFY_OK;
  hipLaunchKernelGGL(k_merge_or, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, (hipStream_t)hip_stream, ids_a,
                     dist_a, ids_b, dist_b, nq, k, out_ids, out_dist);
  if (hipGetLastError() != hipSuccess) {
    set_error("unify_merge_or: launch failed");
    return UNIFY_EDEVICE;
  }
  return UNIFY_OK;
}
