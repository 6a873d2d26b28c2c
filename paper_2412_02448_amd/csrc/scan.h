// Device-wide exclusive prefix sum of int32 counts into int64 offsets
// (off[n] = total), three launches on one stream.  Each translation unit that
// includes this header gets its own copy of the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace unify {
namespace {

__global__ void scan_blocks(const int32_t* __restrict__ cnt, int64_t n, int64_t* __restrict__ off,
                            int64_t* __restrict__ bsum) {
  __shared__ int64_t s[1024];
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  const int64_t v = i < n ? cnt[i] : 0;
  s[threadIdx.x] = v;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    int64_t t = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  if (i < n) off[i] = s[threadIdx.x] - v;
  if (threadIdx.x == 1023) bsum[blockIdx.x] = s[1023];
}

__global__ void scan_top(int64_t* bsum, int64_t nb) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int64_t run = 0;
    for (int64_t b = 0; b < nb; ++b) {
      const int64_t v = bsum[b];
      bsum[b] = run;
      run += v;
    }
    bsum[nb] = run;
  }
}

__global__ void scan_add(int64_t* off, int64_t n, const int64_t* bsum, int64_t nb) {
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  if (i < n) off[i] += bsum[blockIdx.x];
  if (i == 0) off[n] = bsum[nb];
}

__global__ void fill_i32(int32_t* a, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// bsum needs (n + 1023) / 1024 + 1 entries.
inline void exclusive_scan(const int32_t* cnt, int64_t n, int64_t* off, int64_t* bsum, hipStream_t st) {
  const int64_t nb = (n + 1023) / 1024;
  if (nb == 0) {
    hipLaunchKernelGGL(scan_top, dim3(1), dim3(1), 0, st, bsum, (int64_t)0);
    hipLaunchKernelGGL(scan_add, dim3(1), dim3(1024), 0, st, off, (int64_t)0, bsum, (int64_t)0);
    return;
  }
  hipLaunchKernelGGL(scan_blocks, dim3((unsigned)nb), dim3(1024), 0, st, cnt, n, off, bsum);
  hipLaunchKernelGGL(scan_top, dim3(1), dim3(1), 0, st, bsum, nb);
  hipLaunchKernelGGL(scan_add, dim3((unsigned)nb), dim3(1024), 0, st, off, n, bsum, nb);
}

}  // namespace
}  // namespace unify
