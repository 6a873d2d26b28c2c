// Strategy A (pre-filter, Sec. 4.2) for a batch: the exact k nearest objects of
// each query's id slice [lo, hi), with the canonical FP32 distance.
//
// Slices of different queries overlap, so the id space is cut into tiles of
// PT_V objects and every tile is read once per group of up to PT_QG queries
// whose slices meet it: a 256-thread block stages PT_CV vectors at a time in
// LDS and each wavefront scores them for its queries, keeping one sorted
// partial top-k per (query, tile).  A second kernel merges each query's
// partial lists.  Queries whose slice spans more than span_cap tiles (only a
// forced pre-filter on a wide range) stay with the per-query scan of the
// search kernel.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "scan.h"
#include "unify_internal.h"
#include "wave.h"

namespace unify {

constexpr int PT_V = 2048;  // objects per tile
constexpr int PT_QG = 16;   // queries per work item

struct PreArgs {
  DevIndex ix;
  const float* Q;
  int64_t nq;
  int32_t k, kcap, cv, span_cap;
  int64_t ntiles;
  QPlan* plan;
  int32_t* qspan;   // [nq] tiles of each tiled query (0 otherwise)
  int64_t* qoff;    // [nq + 1] first partial-list slot of each query
  int32_t* tcount;  // [ntiles] queries meeting each tile
  int64_t* toff;    // [ntiles + 1]
  int32_t* tfill;   // [ntiles]
  int32_t* wcnt;    // [ntiles] work items of each tile
  int64_t* woff;    // [ntiles + 1]
  int32_t* tq;      // [pairs] queries of each tile
  u64* part;        // [pairs][k] partial top-k lists
  int32_t* counter; // work-item counter
  int64_t* out_ids;
  float* out_dist;
  int32_t* out_stats;
};

__device__ __forceinline__ int64_t first_tile(const QPlan& P) { return P.lo / PT_V; }
__device__ __forceinline__ int64_t last_tile(const QPlan& P) { return (P.hi - 1) / PT_V; }

// Marks the pre-filter queries the tiles will answer and counts queries per tile.
__global__ void k_pre_span(PreArgs A) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= A.nq) return;
  QPlan P = A.plan[q];
  int32_t span = 0;
  if (P.strat == UNIFY_PRE) {
    const int64_t t0 = first_tile(P), t1 = last_tile(P);
    if (t1 - t0 + 1 <= A.span_cap) {
      span = (int32_t)(t1 - t0 + 1);
      for (int64_t t = t0; t <= t1; ++t) atomicAdd(&A.tcount[t], 1);
      A.plan[q].tiled = 1;
    }
  }
  A.qspan[q] = span;
}

__global__ void k_pre_fill(PreArgs A) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= A.nq || A.qspan[q] == 0) return;
  const QPlan P = A.plan[q];
  for (int64_t t = first_tile(P); t <= last_tile(P); ++t) {
    const int32_t slot = atomicAdd(&A.tfill[t], 1);
    A.tq[A.toff[t] + slot] = (int32_t)q;
  }
}

__global__ void k_pre_work(PreArgs A) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < A.ntiles) A.wcnt[t] = (A.tcount[t] + PT_QG - 1) / PT_QG;
}

// Keys of the staged vectors [v0, v0 + cnt) (cnt <= 64) for the four queries of
// this wave: 16-lane group g holds query g's vector in qv and every group reads
// the same staged vector (an LDS broadcast), so one round scores one vector for
// four queries with the canonical summation order.  The key of (query g,
// vector v0 + i) lands in kb[g * 64 + i].
template <int NG>
__device__ __forceinline__ void eval_bcast(int G, const float4 (&qv)[NG], int64_t v0, int cnt, const float* xs,
                                           int ld, int64_t c0, u64* kb) {
  constexpr int RB = NG <= 2 ? 4 : (NG <= 4 ? 2 : 1);
  const int lane = lane_id(), s = lane & 15, g4 = lane >> 4;
  for (int base = 0; base < cnt; base += RB) {
    float4 x[RB][NG];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int v = base + r;
#pragma unroll
      for (int i = 0; i < NG; ++i) {
        const int gg = s + 16 * i;
        x[r][i] = (v < cnt && gg < G) ? *reinterpret_cast<const float4*>(xs + (size_t)(v0 + v - c0) * ld + 4 * gg)
                                      : make_float4(0.f, 0.f, 0.f, 0.f);
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
      if (s == 0 && base + r < cnt) kb[g4 * WAVE + base + r] = make_key(acc, (int32_t)(v0 + base + r));
    }
  }
}

template <int NG>
__global__ void __launch_bounds__(256) k_pre_tile(PreArgs A) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int d = A.ix.d, G = d >> 2, ld = d + 4;
  float* xs = reinterpret_cast<float*>(smem);                    // [cv][d + 4]
  u64* lists = reinterpret_cast<u64*>(xs + (size_t)A.cv * ld);  // [PT_QG][kcap]
  u64* kbuf = lists + (size_t)PT_QG * A.kcap;                    // [4 waves][4][64]
  __shared__ int32_t qid[PT_QG], qlo[PT_QG], qhi[PT_QG], llen[PT_QG];
  __shared__ int64_t sh_w;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, g4 = lane >> 4, s = lane & 15;
  const int64_t W = A.woff[A.ntiles];
  while (true) {
    __syncthreads();
    if (tid == 0) sh_w = atomicAdd(A.counter, 1);
    __syncthreads();
    const int64_t w = sh_w;
    if (w >= W) break;
    // tile of work item w: the last t with woff[t] <= w
    int64_t lo_t = 0, hi_t = A.ntiles;
    while (hi_t - lo_t > 1) {
      const int64_t mid = (lo_t + hi_t) >> 1;
      if (A.woff[mid] <= w) lo_t = mid;
      else hi_t = mid;
    }
    const int64_t t = lo_t;
    const int64_t g = w - A.woff[t];
    const int64_t qbase = A.toff[t] + g * PT_QG;
    const int nqg = (int)min<int64_t>(PT_QG, A.tcount[t] - g * PT_QG);
    const int64_t t0 = t * PT_V, t1 = min<int64_t>(A.ix.n, t0 + PT_V);
    if (tid < PT_QG) {
      if (tid < nqg) {
        const int32_t q = A.tq[qbase + tid];
        const QPlan P = A.plan[q];
        qid[tid] = q;
        qlo[tid] = P.lo;
        qhi[tid] = P.hi;
      } else {
        qid[tid] = -1;
        qlo[tid] = 0;
        qhi[tid] = 0;  // empty slice
      }
      llen[tid] = 0;
    }
    for (int i = tid; i < nqg * A.kcap; i += 256) lists[i] = KEY_MAX;
    __syncthreads();
    // this wave's four queries (one per 16-lane group) and their union within the tile
    const int myq = 4 * wv + g4;
    float4 qv[NG];
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      const int gq = s + 16 * i;
      qv[i] = (myq < nqg && gq < G) ? *reinterpret_cast<const float4*>(A.Q + (int64_t)qid[myq] * d + 4 * gq)
                                    : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    int64_t wlo = t1, whi = t0;
    for (int j = 0; j < 4; ++j) {
      const int qj = 4 * wv + j;
      if (qj < nqg) {
        wlo = min<int64_t>(wlo, max<int64_t>(t0, qlo[qj]));
        whi = max<int64_t>(whi, min<int64_t>(t1, qhi[qj]));
      }
    }
    int64_t ulo = t1, uhi = t0;
    for (int i = 0; i < nqg; ++i) {
      ulo = min<int64_t>(ulo, max<int64_t>(t0, qlo[i]));
      uhi = max<int64_t>(uhi, min<int64_t>(t1, qhi[i]));
    }
    u64* kb = kbuf + (size_t)wv * 4 * WAVE;
    for (int64_t c0 = ulo; c0 < uhi; c0 += A.cv) {
      const int cn = (int)min<int64_t>(A.cv, uhi - c0);
      __syncthreads();
      for (int i = tid; i < cn * G; i += 256) {
        const int v = i / G, gg = i % G;
        *reinterpret_cast<float4*>(xs + (size_t)v * ld + 4 * gg) =
            *reinterpret_cast<const float4*>(A.ix.vec + (c0 + v) * d + 4 * gg);
      }
      __syncthreads();
      const int64_t a = max<int64_t>(c0, wlo), b = min<int64_t>(c0 + cn, whi);
      for (int64_t b0 = a; b0 < b; b0 += WAVE) {
        const int cnt = (int)min<int64_t>(WAVE, b - b0);
        eval_bcast<NG>(G, qv, b0, cnt, xs, ld, c0, kb);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int j = 0; j < 4; ++j) {
          const int qj = 4 * wv + j;
          if (qj >= nqg) break;
          int len = llen[qj];
          u64* lst = lists + (size_t)qj * A.kcap;
          const u64 T = len == A.k ? lst[A.k - 1] : KEY_MAX;
          const int64_t id = b0 + lane;
          u64 key = lane < cnt ? kb[j * WAVE + lane] : KEY_MAX;
          if (id < qlo[qj] || id >= qhi[qj] || !(key < T)) key = KEY_MAX;
          list_insert(lst, len, A.k, key);
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          if (lane == 0) llen[qj] = len;
        }
      }
    }
    __syncthreads();
    // partial lists to their slots
    for (int i = tid; i < nqg * A.k; i += 256) {
      const int qi = i / A.k, r = i % A.k;
      const QPlan P = A.plan[qid[qi]];
      const int64_t slot = A.qoff[qid[qi]] + (t - first_tile(P));
      A.part[slot * A.k + r] = lists[(size_t)qi * A.kcap + r];
    }
  }
}

// One wavefront per tiled query: merge its partial lists, write the answer.
__global__ void __launch_bounds__(64) k_pre_merge(PreArgs A) {
  extern __shared__ __align__(16) unsigned char smem[];
  u64* lst = reinterpret_cast<u64*>(smem);  // [kcap]
  const int lane = lane_id();
  for (int64_t q = blockIdx.x; q < A.nq; q += gridDim.x) {
    const int32_t span = A.qspan[q];
    if (span == 0) continue;
    for (int i = lane; i < A.kcap; i += WAVE) lst[i] = KEY_MAX;
    __syncthreads();
    int len = 0;
    const int64_t base = A.qoff[q];
    for (int j = 0; j < span; ++j) {
      for (int r0 = 0; r0 < A.k; r0 += WAVE) {
        const u64 key = r0 + lane < A.k ? A.part[(base + j) * A.k + r0 + lane] : KEY_MAX;
        list_insert(lst, len, A.k, key);
        __syncthreads();
      }
    }
    for (int r = lane; r < A.k; r += WAVE) {
      const u64 key = r < len ? lst[r] : KEY_MAX;
      A.out_ids[q * A.k + r] = key == KEY_MAX ? -1 : A.ix.ext[key_id(key)];
      A.out_dist[q * A.k + r] = key == KEY_MAX ? __builtin_inff() : key_dist(key);
    }
    if (A.out_stats && lane == 0) {
      const QPlan P = A.plan[q];
      int32_t* st = A.out_stats + q * 8;
      st[0] = P.hi - P.lo;
      st[1] = 0;
      st[2] = 0;
      st[3] = 3;
      st[4] = 0;
      st[5] = UNIFY_PRE;
      st[6] = P.hi - P.lo;
      st[7] = 0;
    }
    __syncthreads();
  }
}

namespace {
typedef void (*TileFn)(PreArgs);
TileFn tile_kernel(int d) {
  const int ng = (d + 63) / 64;
  if (ng <= 2) return k_pre_tile<2>;
  if (ng <= 4) return k_pre_tile<4>;
  if (ng <= 8) return k_pre_tile<8>;
  if (ng <= 15) return k_pre_tile<15>;
  if (ng <= 32) return k_pre_tile<32>;
  return nullptr;
}
}  // namespace

// Bytes of scratch launch_prescan needs for nq queries.
size_t prescan_scratch_bytes(const DevIndex& dv, int64_t nq, int k, int span_cap) {
  const int64_t ntiles = (dv.n + PT_V - 1) / PT_V;
  const int64_t pairs = nq * (int64_t)span_cap;
  const int64_t nbq = (nq + 1023) / 1024 + 1, nbt = (ntiles + 1023) / 1024 + 1;
  size_t b = 0;
  b += 4 * nq + 8 * (nq + 1);                 // qspan, qoff
  b += 4 * ntiles * 3 + 8 * (ntiles + 1) * 2;  // tcount, tfill, wcnt, toff, woff
  b += 4 * pairs + 8 * pairs * k;             // tq, part
  b += 8 * (nbq + nbt) + 64;                  // scan block sums, counter
  return b + 16 * 64;                         // alignment slack
}

int span_cap_for(const DevIndex& dv, int64_t tauA) { return (int)std::min<int64_t>(64, tauA / PT_V + 2); }

// Enqueues the tiled pre-filter scan for the queries of `plan` marked UNIFY_PRE
// whose slices span at most span_cap tiles; marks them tiled in the plan.
int launch_prescan(const DevIndex& dv, const float* Q, int64_t nq, int k, int span_cap, QPlan* plan, void* scratch,
                   int64_t* out_ids, float* out_dist, int32_t* out_stats, int device, hipStream_t st) {
  PreArgs A{};
  A.ix = dv;
  A.Q = Q;
  A.nq = nq;
  A.k = k;
  A.kcap = (k + WAVE - 1) / WAVE * WAVE;
  A.span_cap = span_cap;
  A.ntiles = (dv.n + PT_V - 1) / PT_V;
  const int64_t pairs = nq * (int64_t)span_cap;
  char* p = static_cast<char*>(scratch);
  auto take = [&](size_t bytes) {
    char* r = p;
    p += (bytes + 15) / 16 * 16;
    return r;
  };
  A.plan = plan;
  A.qspan = reinterpret_cast<int32_t*>(take(4 * nq));
  A.qoff = reinterpret_cast<int64_t*>(take(8 * (nq + 1)));
  A.tcount = reinterpret_cast<int32_t*>(take(4 * A.ntiles));
  A.tfill = reinterpret_cast<int32_t*>(take(4 * A.ntiles));
  A.wcnt = reinterpret_cast<int32_t*>(take(4 * A.ntiles));
  A.toff = reinterpret_cast<int64_t*>(take(8 * (A.ntiles + 1)));
  A.woff = reinterpret_cast<int64_t*>(take(8 * (A.ntiles + 1)));
  A.tq = reinterpret_cast<int32_t*>(take(4 * pairs));
  A.part = reinterpret_cast<u64*>(take(8 * pairs * k));
  int64_t* bsum = reinterpret_cast<int64_t*>(take(8 * ((std::max(nq, A.ntiles) + 1023) / 1024 + 1)));
  A.counter = reinterpret_cast<int32_t*>(take(64));
  A.out_ids = out_ids;
  A.out_dist = out_dist;
  A.out_stats = out_stats;
  // per-dimension staging: up to 64 vectors, at most 64 KiB of LDS
  const int ld = dv.d + 4;
  A.cv = (int)std::max(4, std::min(64, (int)(65536 / (ld * 4)) & ~3));
  TileFn fn = tile_kernel(dv.d);
  if (!fn) return UNIFY_EINVAL;
  const size_t lds = (size_t)A.cv * ld * 4 + (size_t)PT_QG * A.kcap * 8 + 4 * 4 * WAVE * 8;

  // counters zeroed by kernels (no memset nodes, so the sequence can be captured)
  auto zero = [&](int32_t* a, int64_t n) {
    hipLaunchKernelGGL(fill_i32, dim3((unsigned)std::max<int64_t>(1, (n + 255) / 256)), dim3(256), 0, st, a, n, 0);
  };
  zero(A.tcount, A.ntiles);
  zero(A.tfill, A.ntiles);
  zero(A.counter, 1);
  const unsigned gq = (unsigned)((nq + 255) / 256);
  hipLaunchKernelGGL(k_pre_span, dim3(gq), dim3(256), 0, st, A);
  exclusive_scan(A.qspan, nq, A.qoff, bsum, st);
  exclusive_scan(A.tcount, A.ntiles, A.toff, bsum, st);
  hipLaunchKernelGGL(k_pre_fill, dim3(gq), dim3(256), 0, st, A);
  hipLaunchKernelGGL(k_pre_work, dim3((unsigned)((A.ntiles + 255) / 256)), dim3(256), 0, st, A);
  exclusive_scan(A.wcnt, A.ntiles, A.woff, bsum, st);
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds) != hipSuccess)
    return UNIFY_EDEVICE;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(fn), 256, lds) !=
          hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || per_cu < 1)
    return UNIFY_EDEVICE;
  hipLaunchKernelGGL(fn, dim3((unsigned)(per_cu * cus)), dim3(256), lds, st, A);
  hipLaunchKernelGGL(k_pre_merge, dim3((unsigned)std::min<int64_t>(nq, 65536)), dim3(64), (size_t)A.kcap * 8, st,
                     A);
  return hipGetLastError() == hipSuccess ? UNIFY_OK : UNIFY_EDEVICE;
}

}  // namespace unify
