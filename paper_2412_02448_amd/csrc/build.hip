// Batched HSIG construction on the GPU.
//
// The paper builds HSIG by inserting objects one at a time (Alg. 6): for every
// segment j, ANNSearch finds the new object's efCons nearest objects of segment
// j, Prune keeps at most M of them as chunk j, and each kept neighbour o gets
// the reverse edge in its chunk for the new object's segment, re-pruned when
// that chunk overflows (Alg. 4); GlobalEdgeMasking (Alg. 5) then marks at most
// M of the node's chunk edges as the global HNSW edges used by post-filtering.
//
// This builder produces the same structure for all objects at once, layer by
// layer:
//   1. candidates: the exact K nearest objects of segment j for every object
//      (one tiled distance pass per segment, K = min(efCons, 256));
//   2. forward chunks: Prune(v, candidates, M);
//   3. reverse edges: every forward edge v -> o (v in segment i) offers v to
//      chunk i of o; a chunk that then holds more than M objects is re-pruned;
//   4. global edges: Prune(v, all chunks of v, M) per object, then each object
//      o receives the marks of the objects v that marked o while o links back
//      to v, in insertion (external id) order, falling back to its own pruned
//      set whenever the marks exceed M -- Alg. 5 applied to the final graph.
// Chunks are sorted by (distance to owner, id), as the hybrid search expects.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <numeric>
#include <shared_mutex>

#include "lowp.h"
#include "unify_internal.h"
#include "wave.h"

namespace unify {

int make_resident(HostIndex&& H, int device, int precision, unify_index_t* out);

namespace {

constexpr int KT_R = 128;  // rows per candidate block
constexpr int KT_C = 64;   // candidate columns per tile
constexpr int KT_D = 64;   // dimensions per staged slice
constexpr int KC = 256;    // candidate list capacity per (object, segment): efCons up to 256
constexpr int CAPR = 256;  // nearest candidates kept before a prune

__global__ void b_gather(const float* __restrict__ X, int d, const int32_t* __restrict__ nodes, int64_t nl,
                         float* __restrict__ out) {
  const int64_t G = (int64_t)d / 4;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nl * G; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / G, g = i % G;
    reinterpret_cast<float4*>(out)[i] = reinterpret_cast<const float4*>(X + (int64_t)nodes[r] * d)[g];
  }
}

__global__ void b_norms(const float* __restrict__ X, int d, int64_t nl, float* __restrict__ xn) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nl; r += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int t = 0; t < d; ++t) {
      const float x = X[r * d + t];
      s = __builtin_fmaf(x, x, s);
    }
    xn[r] = s;
  }
}

// Inserts a batch into a sorted list held in global memory; returns the worst
// kept key when the list is full (KEY_MAX otherwise).
__device__ u64 glist_insert(u64* lst, int& len, int cap, u64 key) {
  const int lane = lane_id();
  const int add = __popcll(ballot(key != KEY_MAX));
  if (add == 0) return len == cap ? lst[cap - 1] : KEY_MAX;
  u64 carry = sort64(key);
  const int total = min(len + add, cap);
  const int used = (len + WAVE - 1) / WAVE, nb = (total + WAVE - 1) / WAVE;
  u64 worst = KEY_MAX;
  for (int blk = 0; blk < nb; ++blk) {
    u64 a = blk < used ? lst[blk * WAVE + lane] : KEY_MAX;
    merge64(a, carry);
    const int pos = blk * WAVE + lane;
    lst[pos] = pos < total ? a : KEY_MAX;
    if (blk == (cap - 1) / WAVE) {
      uint32_t lo = (uint32_t)__shfl((int)(uint32_t)a, (cap - 1) % WAVE, WAVE);
      uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(a >> 32), (cap - 1) % WAVE, WAVE);
      worst = ((u64)hi << 32) | lo;
    }
  }
  len = total;
  return total == cap ? worst : KEY_MAX;
}

// Exact K nearest candidates of segment j for rows [row0, row0 + nrows) of a layer
// (or for rows[row0 .. row0 + nrows) when a row list is given).
struct KnnArgs {
  const float* X;
  const float* xn;
  int d, S, K;
  int64_t row0, nrows;
  const int64_t* sstart;  // [S+1] compact id ranges of the segments
  u64* lists;             // [nrows][S][KC]
  int32_t* lens;          // [nrows][S]
  u64* pend;              // [nrows][S][KT_C]
  const int32_t* rows;    // optional: the layer rows to process
};

__global__ void __launch_bounds__(256) b_knn(KnnArgs A) {
  __shared__ float qT[KT_D][KT_R];
  __shared__ float xT[KT_D][KT_C + 4];
  __shared__ u64 tau[KT_R];
  __shared__ int pcnt[KT_R];
  __shared__ int lenr[KT_R];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int j = blockIdx.y;
  const int64_t lr0 = (int64_t)blockIdx.x * KT_R;  // first local row
  const int64_t c_begin = A.sstart[j], c_end = A.sstart[j + 1];
  const int d = A.d, S = A.S;
  if (tid < KT_R) {
    tau[tid] = KEY_MAX;
    pcnt[tid] = 0;
    lenr[tid] = 0;
  }
  const int rg = tid >> 4, cg = tid & 15;
  for (int64_t c0 = c_begin; c0 < c_end; c0 += KT_C) {
    float acc[8][4];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[i][t] = 0.f;
    for (int k0 = 0; k0 < d; k0 += KT_D) {
      __syncthreads();
      // rows: lanes take consecutive rows so that the transposed stores do not conflict
      for (int it = 0; it < (KT_R * KT_D / 4) / 256; ++it) {
        const int idx = tid + 256 * it;
        const int r = idx % KT_R, g = idx / KT_R;
        const int64_t lr = lr0 + r;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (lr < A.nrows && k0 + 4 * g < d) {
          const int64_t row = A.rows ? (int64_t)A.rows[A.row0 + lr] : A.row0 + lr;
          v = *reinterpret_cast<const float4*>(A.X + row * d + k0 + 4 * g);
        }
        qT[4 * g + 0][r] = v.x;
        qT[4 * g + 1][r] = v.y;
        qT[4 * g + 2][r] = v.z;
        qT[4 * g + 3][r] = v.w;
      }
      for (int it = 0; it < (KT_C * KT_D / 4) / 256; ++it) {
        const int idx = tid + 256 * it;
        const int c = idx / (KT_D / 4), g = idx % (KT_D / 4);
        const int64_t col = c0 + c;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (col < c_end && k0 + 4 * g < d) v = *reinterpret_cast<const float4*>(A.X + col * d + k0 + 4 * g);
        xT[4 * g + 0][c] = v.x;
        xT[4 * g + 1][c] = v.y;
        xT[4 * g + 2][c] = v.z;
        xT[4 * g + 3][c] = v.w;
      }
      __syncthreads();
#pragma unroll 4
      for (int kk = 0; kk < KT_D; ++kk) {
        const float4 qa = *reinterpret_cast<const float4*>(&qT[kk][rg * 8]);
        const float4 qb = *reinterpret_cast<const float4*>(&qT[kk][rg * 8 + 4]);
        const float4 xa = *reinterpret_cast<const float4*>(&xT[kk][cg * 4]);
        const float q[8] = {qa.x, qa.y, qa.z, qa.w, qb.x, qb.y, qb.z, qb.w};
        const float x[4] = {xa.x, xa.y, xa.z, xa.w};
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
          for (int t = 0; t < 4; ++t) acc[i][t] = __builtin_fmaf(q[i], x[t], acc[i][t]);
      }
    }
    // distances, filtered against each row's current K-th key
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int r = rg * 8 + i;
      const int64_t lr = lr0 + r;
      if (lr >= A.nrows) continue;
      const int64_t row = A.rows ? (int64_t)A.rows[A.row0 + lr] : A.row0 + lr;
      const float qn = A.xn[row];
      const u64 tr = tau[r];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t col = c0 + cg * 4 + t;
        if (col >= c_end || col == row) continue;
        float dist = qn + A.xn[col] - 2.0f * acc[i][t];
        dist = dist > 0.f ? dist : 0.f;
        const u64 key = make_key(dist, (int32_t)col);
        if (key < tr) {
          const int slot = atomicAdd(&pcnt[r], 1);
          A.pend[(lr * S + j) * KT_C + slot] = key;
        }
      }
    }
    __syncthreads();
    // merge the pending candidates of each row into its list (wave w owns 32 rows)
    for (int rr = 0; rr < KT_R / 4; ++rr) {
      const int r = wv * (KT_R / 4) + rr;
      const int cnt = pcnt[r];
      if (cnt == 0) continue;
      const int64_t lr = lr0 + r;
      const int64_t base = lr * S + j;
      const u64 key = lane < cnt ? A.pend[base * KT_C + lane] : KEY_MAX;
      int len = lenr[r];
      const u64 worst = glist_insert(A.lists + base * KC, len, A.K, key);
      if (lane == 0) {
        lenr[r] = len;
        tau[r] = worst;
        pcnt[r] = 0;
      }
    }
    __syncthreads();
  }
  if (tid < KT_R && lr0 + tid < A.nrows) A.lens[(lr0 + tid) * S + j] = lenr[tid];
}

// ---------------------------------------------------------------------------
// Candidates on the matrix cores (rows of at most 256 elements).  The distance
// of a row to a column is the norm expansion |x|^2 + |y|^2 - 2 x.y over BF16
// copies of both vectors (the dot product on v_mfma_f32_16x16x32_bf16, FP32
// accumulation): the squared distance of the rounded points, which only ranks
// the candidates; Prune recomputes every distance it uses from the FP32
// vectors.  A workgroup takes 256 rows and one segment: wavefront w holds rows
// 64 w .. 64 w + 63 as MFMA A operands in registers and streams the segment's
// columns through LDS, 64 per step (double-buffered).  A candidate enters a
// row's pending buffer when it is not farther than the row's current K-th
// candidate; a row with 64 or more pending is merged into its sorted list at
// the end of the step, the rest at the end, so the threshold tightens as the
// segment is scanned.  Rows are private to their wavefront: merges need no
// workgroup barrier.
// ---------------------------------------------------------------------------
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_b;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_b;
constexpr int MK_RT = 4;                   // 16-row tiles per wavefront
constexpr int MK_ROWS = 4 * 16 * MK_RT;    // rows per workgroup
constexpr int MK_CT = 4;                   // 16-column tiles per step
constexpr int MK_PC = 128;                 // pending candidates per (row, segment)
constexpr int MK_DMAX = 256;               // widest rows on this path

// Orders a wavefront's memory operations before its later ones (LDS and global).
__device__ __forceinline__ void wave_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// BF16 copies of rows [0, nl) of X, zero-padded to dp elements, and their squared norms.
__global__ void b_bf16_rows(const float* __restrict__ X, int d, int dp, int64_t nl, uint16_t* __restrict__ Xb,
                            float* __restrict__ xnb) {
  const int lane = lane_id();
  const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t r = w0; r < nl; r += nw) {
    float s = 0.f;
    for (int t = lane; t < dp; t += WAVE) {
      const uint32_t b = t < d ? f32_to_bf16(X[r * d + t]) : 0u;
      Xb[r * dp + t] = (uint16_t)b;
      const float xb = bf16_to_f32(b);
      s = __builtin_fmaf(xb, xb, s);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, WAVE);
    if (lane == 0) xnb[r] = s;
  }
}

struct KnnMArgs {
  const uint16_t* Xb;  // [nl][dp] BF16 rows
  const float* xnb;    // [nl] their squared norms
  int dp, S, K;
  int64_t row0, nrows;
  const int64_t* sstart;  // [S+1] compact id ranges of the segments
  u64* lists;             // [nrows][S][KC]
  int32_t* lens;          // [nrows][S]
  u64* pend;              // [nrows][S][MK_PC]
  const int32_t* rows;    // optional: the layer rows to process (rows[row0 + lr]; else row0 + lr)
};

__host__ __device__ constexpr size_t knn_mfma_lds(int ks) {
  return sizeof(uint16_t) * 2 * 64 * (size_t)(32 * ks + 8) + sizeof(float) * MK_ROWS + 2 * sizeof(int32_t) * MK_ROWS;
}

template <int KS>
__global__ void __launch_bounds__(256, KS <= 3 ? 2 : 1) b_knn_mfma(KnnMArgs A) {
  extern __shared__ __align__(16) unsigned char knn_lds[];
  constexpr int stride = 32 * KS + 8;  // staged column (elements), padded against bank conflicts
  uint16_t* buf0 = reinterpret_cast<uint16_t*>(knn_lds);
  uint16_t* buf1 = buf0 + 64 * stride;
  float* tau = reinterpret_cast<float*>(buf1 + 64 * stride);  // per row: its K-th candidate's distance
  int32_t* pcnt = reinterpret_cast<int32_t*>(tau + MK_ROWS);  // per row: pending candidates
  int32_t* lenr = pcnt + MK_ROWS;                              // per row: list length
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int j = blockIdx.y, S = A.S, dp = A.dp;
  const int64_t lr0 = (int64_t)blockIdx.x * MK_ROWS;  // first local row of the workgroup
  const int64_t c_begin = A.sstart[j], c_end = A.sstart[j + 1];
  tau[tid] = __builtin_inff();
  pcnt[tid] = 0;
  lenr[tid] = 0;
  const int mrow = lane & 15, kq = lane >> 4;  // MFMA lane roles: row / column, k quarter
  // layer row of local row lr
  auto row_of = [&](int64_t lr) { return A.rows ? (int64_t)A.rows[A.row0 + lr] : A.row0 + lr; };
  // A operands: rows 16 rt + mrow of this wavefront, elements 32 s + 8 kq .. + 7
  bf16x8_b a[MK_RT][KS];
#pragma unroll
  for (int rt = 0; rt < MK_RT; ++rt) {
    const int64_t lr = lr0 + wv * 64 + 16 * rt + mrow;
    const int64_t row = lr < A.nrows ? row_of(lr) : 0;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const uint4 w = lr < A.nrows ? *reinterpret_cast<const uint4*>(A.Xb + row * dp + 32 * s + 8 * kq)
                                   : make_uint4(0u, 0u, 0u, 0u);
      a[rt][s] = __builtin_bit_cast(bf16x8_b, w);
    }
  }
  // the lane's output rows: 16 rt + 4 kq + i
  float xr[MK_RT][4];
#pragma unroll
  for (int rt = 0; rt < MK_RT; ++rt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t lr = lr0 + wv * 64 + 16 * rt + 4 * kq + i;
      xr[rt][i] = lr < A.nrows ? A.xnb[row_of(lr)] : 0.f;
    }
  const int64_t ncol = c_end - c_begin;
  const int nsteps = (int)((ncol + 63) / 64);
  // staging: KS chunks of 8 elements per thread and step
  uint4 st[KS];
  auto gload = [&](int step) {
#pragma unroll
    for (int c = 0; c < KS; ++c) {
      const int idx = tid + 256 * c, col = idx / (4 * KS), ch = idx - col * (4 * KS);
      const int64_t gc = c_begin + (int64_t)step * 64 + col;
      st[c] = gc < c_end ? *reinterpret_cast<const uint4*>(A.Xb + gc * dp + 8 * ch) : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto lstore = [&](uint16_t* b) {
#pragma unroll
    for (int c = 0; c < KS; ++c) {
      const int idx = tid + 256 * c, col = idx / (4 * KS), ch = idx - col * (4 * KS);
      *reinterpret_cast<uint4*>(b + col * stride + 8 * ch) = st[c];
    }
  };
  if (nsteps > 0) {
    gload(0);
    lstore(buf0);
  }
  __syncthreads();
  int32_t* const wp = pcnt + wv * 64;
  // merges the pending candidates of local row r (of this wavefront) into its list
  auto merge = [&](int r) {
    const int64_t lr = lr0 + wv * 64 + r;
    const int64_t base = lr * S + j;
    const int cnt = wp[r];
    int len = lenr[wv * 64 + r];
    u64 worst = KEY_MAX;
    for (int b0 = 0; b0 < cnt; b0 += WAVE) {
      const u64 key = b0 + lane < cnt ? A.pend[base * MK_PC + b0 + lane] : KEY_MAX;
      worst = glist_insert(A.lists + base * KC, len, A.K, key);
      wave_order();  // the list's stores before the next batch reads it
    }
    if (lane == 0) {
      lenr[wv * 64 + r] = len;
      tau[wv * 64 + r] = worst == KEY_MAX ? __builtin_inff() : key_dist(worst);
      wp[r] = 0;
    }
  };
  for (int step = 0; step < nsteps; ++step) {
    const uint16_t* cur = (step & 1) ? buf1 : buf0;
    uint16_t* nxt = (step & 1) ? buf0 : buf1;
    if (step + 1 < nsteps) gload(step + 1);
    f32x4_b acc[MK_RT][MK_CT];
#pragma unroll
    for (int rt = 0; rt < MK_RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < MK_CT; ++ct) acc[rt][ct] = f32x4_b{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int ct = 0; ct < MK_CT; ++ct) {
        const bf16x8_b b = *reinterpret_cast<const bf16x8_b*>(cur + (16 * ct + mrow) * stride + 32 * s + 8 * kq);
#pragma unroll
        for (int rt = 0; rt < MK_RT; ++rt)
          acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rt][s], b, acc[rt][ct], 0, 0, 0);
      }
    // filter: lane holds rows 16 rt + 4 kq + i against column 16 ct + mrow of the step.
    // dist <= threshold  <=>  2 acc >= (xr - threshold) + xc: one add and one compare per
    // product.  Rows past the end get hr = +inf and columns past the end xc = +inf (never
    // pass: the sum is +inf or NaN); a row without K candidates yet has hr = -inf.
    const int64_t cb = c_begin + (int64_t)step * 64;
    float hr[MK_RT][4];
#pragma unroll
    for (int rt = 0; rt < MK_RT; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 16 * rt + 4 * kq + i;
        hr[rt][i] = lr0 + wv * 64 + r < A.nrows ? xr[rt][i] - tau[wv * 64 + r] : __builtin_inff();
      }
#pragma unroll
    for (int ct = 0; ct < MK_CT; ++ct) {
      const int64_t col = cb + 16 * ct + mrow;
      const float xc = col < c_end ? A.xnb[col] : __builtin_inff();  // past the end: never passes
#pragma unroll
      for (int rt = 0; rt < MK_RT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (2.0f * acc[rt][ct][i] >= hr[rt][i] + xc) {
            const int r = 16 * rt + 4 * kq + i;  // local row of the wavefront
            const int64_t lr = lr0 + wv * 64 + r;
            if (col != row_of(lr)) {
              float dist = __builtin_fmaf(-2.0f, acc[rt][ct][i], xr[rt][i] + xc);
              dist = dist > 0.f ? dist : 0.f;
              const int slot = atomicAdd(&wp[r], 1);
              A.pend[((lr * S + j) * MK_PC) + slot] = make_key(dist, (int32_t)col);
            }
          }
        }
    }
    wave_order();  // this wavefront's pending stores and counts before the merges read them
    const bool last = step + 1 == nsteps;
    u64 need = ballot(wp[lane] >= (last ? 1 : 64));
    while (need) {
      const int r = __ffsll((unsigned long long)need) - 1;
      need &= need - 1;
      merge(r);
      wave_order();
    }
    if (step + 1 < nsteps) lstore(nxt);
    __syncthreads();
  }
  if (lr0 + tid < A.nrows) A.lens[(lr0 + tid) * S + j] = lenr[tid];
}

// Generic Prune (Sec. 2.2) of one owner per task, one wavefront per task.
// Candidates: a_cnt[t] (or a_stride) keys at a + t * a_stride, then b_cnt[t]
// keys at b + b_off[t]; only the id half of a key is used.  Distances are
// recomputed from the vectors, duplicates removed, the nearest CAPR kept; if
// more than Mcap remain (or always, when !only_if_over), the greedy rule keeps
// a candidate unless an already kept one is nearer to it than the owner is.
struct PruneArgs {
  const float* X;
  int d;
  int64_t ntask;
  int64_t owner0;
  int32_t owner_div;
  const u64* a;
  int32_t a_stride;
  const int32_t* a_cnt;
  const u64* b;
  const int64_t* b_off;    // b_off[t] - b_base: first key of task t in b
  int64_t b_base;
  const int32_t* b_cnt;
  int32_t Mcap;
  int32_t only_if_over;
  u64* out;                // [ntask][Mcap]
  const int32_t* owners;   // optional: owner = owners[owner0 + task / owner_div]
  const int64_t* task_of;  // optional: the tasks to run (all ntask of them otherwise)
};

template <int NG>
__device__ __forceinline__ void load_row(const float* X, int d, int64_t v, float4 (&x)[NG]) {
  const int s = lane_id() & 15, G = d >> 2;
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    const int g = s + 16 * i;
    x[i] = g < G ? *reinterpret_cast<const float4*>(X + v * d + 4 * g) : make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

template <int NG>
__device__ __forceinline__ float group_dist(const float4 (&a)[NG], const float4 (&b)[NG]) {
  float acc = 0.f;
#pragma unroll
  for (int i = 0; i < NG; ++i) acc = fma_sq4(a[i], b[i], acc);
  return group_reduce16(acc);
}

// SG > 0: kept vectors stay in registers (4 per group of 16 lanes, SG groups);
// SG == 0 (wide vectors): kept ids stay in LDS and their distances to each
// candidate are evaluated from memory.
template <int NG, int SG>
__global__ void __launch_bounds__(64) b_prune(PruneArgs A) {
  __shared__ u64 lst[CAPR];
  __shared__ u64 bk[WAVE];
  __shared__ int32_t ids[WAVE];
  __shared__ int32_t selid[WAVE];
  const int lane = lane_id(), g4 = lane >> 4;
  for (int64_t it = blockIdx.x; it < A.ntask; it += gridDim.x) {
    const int64_t t = A.task_of ? A.task_of[it] : it;
    const int64_t oi = A.owner0 + t / A.owner_div;
    const int64_t owner = A.owners ? (int64_t)A.owners[oi] : oi;
    float4 qv[NG];
    load_row<NG>(A.X, A.d, owner, qv);
    int len = 0;
    for (int i = lane; i < CAPR; i += WAVE) lst[i] = KEY_MAX;
    __syncthreads();
    const int na = A.a_cnt ? A.a_cnt[t] : A.a_stride;
    const int nb = A.b ? A.b_cnt[t] : 0;
    const int64_t boff = A.b ? A.b_off[t] - A.b_base : 0;
    for (int base = 0; base < na + nb; base += WAVE) {
      const int i = base + lane;
      int32_t v = -1;
      if (i < na) {
        const u64 kk = A.a[t * A.a_stride + i];
        if (kk != KEY_MAX) v = key_id(kk);
      } else if (i < na + nb) {
        const u64 kk = A.b[boff + (i - na)];
        if (kk != KEY_MAX) v = key_id(kk);
      }
      if (v == (int32_t)owner) v = -1;
      const u64 m = ballot(v >= 0);
      if (v >= 0) ids[rank_in(m)] = v;
      const int cnt = __popcll(m);
      __syncthreads();
      eval_keys_generic<NG>(
          A.d >> 2, qv, cnt, [&](int i) { return ids[i]; },
          [&](int64_t v, int g) { return *reinterpret_cast<const float4*>(A.X + v * A.d + 4 * g); }, bk);
      __syncthreads();
      list_insert(lst, len, CAPR, lane < cnt ? bk[lane] : KEY_MAX);
      __syncthreads();
    }
    // drop duplicates (equal keys are adjacent)
    {
      u64 prev_last = KEY_MAX;
      int w = 0;
      for (int b0 = 0; b0 < len; b0 += WAVE) {
        const int i = b0 + lane;
        const u64 kk = i < len ? lst[i] : KEY_MAX;
        u64 prev = shfl64(kk, lane > 0 ? lane - 1 : 0);
        if (lane == 0) prev = prev_last;
        prev_last = shfl64(kk, WAVE - 1);
        const bool keep = i < len && kk != prev;
        const u64 km = ballot(keep);
        __syncthreads();
        if (keep) lst[w + rank_in(km)] = kk;
        w += __popcll(km);
        __syncthreads();
      }
      len = w;
    }
    u64* out = A.out + t * A.Mcap;
    if (A.only_if_over && len <= A.Mcap) {
      for (int i = lane; i < A.Mcap; i += WAVE) out[i] = i < len ? lst[i] : KEY_MAX;
      __syncthreads();
      continue;
    }
    if constexpr (SG == 0) {
      int nsel = 0;
      for (int pos = 0; pos < len && nsel < A.Mcap; ++pos) {
        const u64 key = lst[pos];
        const int32_t r = key_id(key);
        const float dvr = key_dist(key);
        bool bad = false;
        if (nsel > 0) {
          float4 xr[NG];
          load_row<NG>(A.X, A.d, r, xr);
          eval_keys_generic<NG>(
              A.d >> 2, xr, nsel, [&](int i) { return selid[i]; },
              [&](int64_t v, int g) { return *reinterpret_cast<const float4*>(A.X + v * A.d + 4 * g); }, bk);
          __syncthreads();
          bad = lane < nsel && key_dist(bk[lane]) < dvr;
          __syncthreads();
        }
        if (__any(bad)) continue;
        if (lane == 0) {
          selid[nsel] = r;
          out[nsel] = key;
        }
        ++nsel;
        __syncthreads();
      }
      for (int i = nsel + lane; i < A.Mcap; i += WAVE) out[i] = KEY_MAX;
      __syncthreads();
      continue;
    }
    // greedy selection; kept vectors stay in registers (group g keeps numbers 4s+g)
    float4 sel[SG > 0 ? SG : 1][NG];
#pragma unroll
    for (int s = 0; s < SG; ++s)
#pragma unroll
      for (int i = 0; i < NG; ++i) sel[s][i] = make_float4(0.f, 0.f, 0.f, 0.f);
    int nsel = 0;
    for (int pos = 0; pos < len && nsel < A.Mcap; ++pos) {
      const u64 key = lst[pos];
      const int32_t r = key_id(key);
      const float dvr = key_dist(key);
      float4 xr[NG];
      load_row<NG>(A.X, A.d, r, xr);
      bool bad = false;
#pragma unroll
      for (int s = 0; s < SG; ++s) {
        if (4 * s < nsel) {
          const float de = group_dist<NG>(sel[s], xr);
          if (4 * s + g4 < nsel && de < dvr) bad = true;
        }
      }
      if (__any(bad)) continue;
#pragma unroll
      for (int s = 0; s < SG; ++s)
        if (s == nsel / 4 && g4 == nsel % 4) {
#pragma unroll
          for (int i = 0; i < NG; ++i) sel[s][i] = xr[i];
        }
      if (lane == 0) out[nsel] = key;
      ++nsel;
    }
    for (int i = nsel + lane; i < A.Mcap; i += WAVE) out[i] = KEY_MAX;
    __syncthreads();
  }
}

// Reverse edges: every forward edge row -> o (row in segment si) is offered to chunk si of o.
// Row r of fwd belongs to layer row rows[r] when a row list is given.  Only the slots
// (o * S + si) in [slot_lo, slot_hi) are counted and, with rev, written at off[slot] - base.
__global__ void b_rev(const u64* __restrict__ fwd, int64_t nrows, int S, int M, const int32_t* __restrict__ segc,
                      int32_t* __restrict__ cnt, const int64_t* __restrict__ off, u64* __restrict__ rev,
                      const int32_t* __restrict__ rows, int64_t slot_lo = 0, int64_t slot_hi = INT64_MAX,
                      int64_t base = 0) {
  const int64_t total = nrows * S * M;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const u64 kk = fwd[e];
    if (kk == KEY_MAX) continue;
    const int64_t r = e / ((int64_t)S * M);
    const int64_t row = rows ? (int64_t)rows[r] : r;
    const int32_t o = key_id(kk);
    const int64_t slot = (int64_t)o * S + segc[row];
    if (slot < slot_lo || slot >= slot_hi) continue;
    const int32_t p = atomicAdd(&cnt[slot], 1);
    if (rev) rev[off[slot] - base + p] = make_key(0.f, (int32_t)row);
  }
}

// Global-edge bits of rows [r0, r0 + nr): bit pos of row r is set when entry pos of
// its chunks is one of its marks (an id occurs at most once in a row: chunks hold
// distinct objects of distinct segments).  One wavefront per row.
__global__ void b_gbits(const u64* __restrict__ fwd, const int32_t* __restrict__ glist, int64_t r0, int64_t nr,
                        int S, int M, int W, uint32_t* __restrict__ bits) {
  const int lane = lane_id();
  const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = w0; i < nr; i += nw) {
    const int64_t r = r0 + i;
    const int32_t* mk = glist + r * M;
    for (int p0 = 0; p0 < W * 32; p0 += WAVE) {
      const int pos = p0 + lane;
      bool hit = false;
      if (pos < S * M) {
        const u64 kk = fwd[r * S * M + pos];
        if (kk != KEY_MAX) {
          const int32_t id = key_id(kk);
          for (int t = 0; t < M; ++t) hit |= mk[t] == id;
        }
      }
      const u64 m = ballot(hit);
      if (lane == 0) bits[i * W + p0 / 32] = (uint32_t)m;
      if (lane == 0 && p0 / 32 + 1 < W) bits[i * W + p0 / 32 + 1] = (uint32_t)(m >> 32);
    }
  }
}

// Exclusive prefix sum of n int32 counts into int64 offsets (off[n] = total).
__global__ void b_scan_blocks(const int32_t* __restrict__ cnt, int64_t n, int64_t* __restrict__ off,
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
__global__ void b_scan_top(int64_t* bsum, int64_t nb) {
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
__global__ void b_scan_add(int64_t* off, int64_t n, const int64_t* bsum, int64_t nb) {
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  if (i < n) off[i] += bsum[blockIdx.x];
  if (i == 0) off[n] = bsum[nb];
}

// Global-edge marks, reverse part: v marked o (o in P(v)) and o links back to v.
__global__ void b_mask_rev(const u64* __restrict__ P, const u64* __restrict__ chunks, int64_t nrows, int S, int M,
                           const int32_t* __restrict__ segc, int32_t* __restrict__ cnt,
                           const int64_t* __restrict__ off, int32_t* __restrict__ rev) {
  const int64_t total = nrows * M;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const u64 kk = P[e];
    if (kk == KEY_MAX) continue;
    const int64_t v = e / M;
    const int32_t o = key_id(kk);
    const u64* ch = chunks + ((int64_t)o * S + segc[v]) * M;
    bool back = false;
    for (int t = 0; t < M; ++t)
      if (ch[t] != KEY_MAX && key_id(ch[t]) == (int32_t)v) back = true;
    if (!back) continue;
    const int32_t p = atomicAdd(&cnt[o], 1);
    if (rev) rev[off[o] + p] = (int32_t)v;
  }
}

// Final marks of each object: its own pruned set P(o), then the reverse marks in
// ascending external id, restarting from P(o) whenever more than M are marked.
__global__ void b_mask_final(const u64* __restrict__ P, int64_t nrows, int M, const int64_t* __restrict__ off,
                             const int32_t* __restrict__ rev, const int64_t* __restrict__ ext_of,
                             int32_t* __restrict__ glist) {
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < nrows; o += (int64_t)gridDim.x * blockDim.x) {
    int32_t marks[65];
    int np = 0;
    for (int t = 0; t < M; ++t)
      if (P[o * M + t] != KEY_MAX) marks[np++] = key_id(P[o * M + t]);
    int nm = np;
    const int64_t b = off[o], e = off[o + 1];
    int64_t last = -1;
    for (int64_t step = b; step < e; ++step) {
      // next reverse mark in ascending external id
      int32_t best = -1;
      int64_t bx = INT64_MAX;
      for (int64_t q = b; q < e; ++q) {
        const int64_t x = ext_of[rev[q]];
        if (x > last && x < bx) {
          bx = x;
          best = rev[q];
        }
      }
      last = bx;
      bool have = false;
      for (int t = 0; t < nm; ++t) have |= marks[t] == best;
      if (have) continue;
      marks[nm++] = best;
      if (nm > M) {
        nm = np;
        for (int t = 0; t < M; ++t)
          if (P[o * M + t] != KEY_MAX) marks[t] = key_id(P[o * M + t]);
      }
    }
    for (int t = 0; t < M; ++t) glist[o * M + t] = t < nm ? marks[t] : -1;
  }
}

#define BHIP(x)                                                       \
  do {                                                                \
    hipError_t e_ = (x);                                              \
    if (e_ != hipSuccess) {                                           \
      set_error(std::string("build: ") + #x + ": " + hipGetErrorString(e_)); \
      return UNIFY_EDEVICE;                                           \
    }                                                                 \
  } while (0)

struct DevBuf {
  std::vector<void*> ptrs;
  ~DevBuf() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <class T>
  T* alloc(size_t count) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return static_cast<T*>(p);
  }
  void release(void* p) {
    for (auto& q : ptrs)
      if (q == p) {
        (void)hipFree(q);
        q = nullptr;
      }
  }
};

int scan(DevBuf& buf, const int32_t* cnt, int64_t n, int64_t* off) {
  const int64_t nb = (n + 1023) / 1024;
  int64_t* bsum = buf.alloc<int64_t>(nb + 1);
  if (!bsum) {
    set_error("build: out of device memory");
    return UNIFY_ENOMEM;
  }
  hipLaunchKernelGGL(b_scan_blocks, dim3((unsigned)nb), dim3(1024), 0, 0, cnt, n, off, bsum);
  hipLaunchKernelGGL(b_scan_top, dim3(1), dim3(1), 0, 0, bsum, nb);
  hipLaunchKernelGGL(b_scan_add, dim3((unsigned)nb), dim3(1024), 0, 0, off, n, bsum, nb);
  BHIP(hipGetLastError());
  buf.release(bsum);
  return UNIFY_OK;
}

typedef void (*PruneFn)(PruneArgs);
PruneFn prune_kernel(int d, int Mcap) {
  const int ng = (d + 63) / 64;
  if (Mcap > 64) return nullptr;
  if (Mcap <= 32) {
    if (ng <= 2) return b_prune<2, 8>;
    if (ng <= 4) return b_prune<4, 8>;
  } else {
    if (ng <= 2) return b_prune<2, 16>;
  }
  if (ng <= 4) return b_prune<4, 0>;
  if (ng <= 8) return b_prune<8, 0>;
  if (ng <= 15) return b_prune<15, 0>;
  if (ng <= 32) return b_prune<32, 0>;
  return nullptr;
}

int run_prune(PruneArgs A, hipStream_t st = nullptr) {
  PruneFn fn = prune_kernel(A.d, A.Mcap);
  if (!fn) {
    set_error("build: unsupported (d, M) for the GPU builder (d <= 2048, M <= 64)");
    return UNIFY_EINVAL;
  }
  const int64_t grid = std::min<int64_t>(A.ntask, 1 << 20);
  hipLaunchKernelGGL(fn, dim3((unsigned)std::max<int64_t>(grid, 1)), dim3(64), 0, st, A);
  BHIP(hipGetLastError());
  return UNIFY_OK;
}

// Candidate ids (-1: none) to keys; kept keys back to ids.
__global__ void b_ids_to_keys(const int32_t* __restrict__ ids, int64_t cnt, u64* __restrict__ keys) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
    keys[i] = ids[i] >= 0 ? make_key(0.f, ids[i]) : KEY_MAX;
}
__global__ void b_keys_to_ids(const u64* __restrict__ keys, int64_t cnt, int32_t* __restrict__ ids) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
    ids[i] = keys[i] == KEY_MAX ? -1 : key_id(keys[i]);
}

// Launches b_knn_mfma for rows [row0, row0 + nrows) against every segment.
int run_knn_mfma(const KnnMArgs& km) {
  const dim3 grid((unsigned)((km.nrows + MK_ROWS - 1) / MK_ROWS), (unsigned)km.S);
  switch (km.dp / 32) {
#define KNN_CASE(KS)                                                                                              \
  case KS:                                                                                                        \
    BHIP(hipFuncSetAttribute(reinterpret_cast<const void*>(b_knn_mfma<KS>),                                       \
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)knn_mfma_lds(KS)));                 \
    hipLaunchKernelGGL(b_knn_mfma<KS>, grid, dim3(256), knn_mfma_lds(KS), 0, km);                                 \
    break;
    KNN_CASE(1) KNN_CASE(2) KNN_CASE(3) KNN_CASE(4) KNN_CASE(5) KNN_CASE(6) KNN_CASE(7) KNN_CASE(8)
#undef KNN_CASE
    default:
      set_error("build: rows too wide for the matrix-core candidate pass");
      return UNIFY_EINVAL;
  }
  BHIP(hipGetLastError());
  return UNIFY_OK;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Builds one layer over `nodes` (internal ids, ascending).  Outputs, on the
// host: chunks [nl][S][M] and marks [nl][M] as internal ids (-1 padded).
// emit(c0, cnt, chunks, bits) receives layer rows c0 .. c0 + cnt - 1 (positions in
// `nodes`) in order: chunks [cnt][S][M] as internal ids (-1 padded) and their
// global-edge bits [cnt][ceil(S M / 32)].
using EmitRows = std::function<void(int64_t, int64_t, const int32_t*, const uint32_t*)>;
int build_layer(const float* dX, int d, int S, int M, int K, const std::vector<int32_t>& nodes,
                const std::vector<int64_t>& seg_start, const std::vector<int64_t>& ext, const EmitRows& emit,
                bool verbose) {
  const int64_t nl = (int64_t)nodes.size();
  DevBuf buf;
  // compact vectors of this layer
  const float* X = dX;
  std::vector<int64_t> sst(S + 1, 0);
  std::vector<int32_t> segc(nl);
  {
    int j = 0;
    for (int64_t c = 0; c < nl; ++c) {
      while (j + 1 <= S && nodes[c] >= seg_start[j + 1]) ++j;
      segc[c] = j;
    }
    for (int jj = 0; jj <= S; ++jj)
      sst[jj] = std::lower_bound(nodes.begin(), nodes.end(), (int32_t)std::min<int64_t>(seg_start[jj], INT32_MAX)) -
                nodes.begin();
    sst[S] = nl;
  }
  const bool identity = nl > 0 && nodes.back() == nl - 1;
  if (!identity) {
    int32_t* dnodes = buf.alloc<int32_t>(nl);
    float* Xl = buf.alloc<float>((size_t)nl * d);
    if (!dnodes || !Xl) {
      set_error("build: out of device memory");
      return UNIFY_ENOMEM;
    }
    BHIP(hipMemcpy(dnodes, nodes.data(), 4 * nl, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(b_gather, dim3(1024), dim3(256), 0, 0, dX, d, dnodes, nl, Xl);
    X = Xl;
  }
  float* xn = buf.alloc<float>(nl);
  int64_t* dsst = buf.alloc<int64_t>(S + 1);
  int32_t* dsegc = buf.alloc<int32_t>(nl);
  int64_t* dext = buf.alloc<int64_t>(nl);
  u64* fwd = buf.alloc<u64>((size_t)nl * S * M);
  if (!xn || !dsst || !dsegc || !dext || !fwd) {
    set_error("build: out of device memory");
    return UNIFY_ENOMEM;
  }
  {
    std::vector<int64_t> ext_c(nl);
    for (int64_t c = 0; c < nl; ++c) ext_c[c] = ext[nodes[c]];
    BHIP(hipMemcpy(dext, ext_c.data(), 8 * nl, hipMemcpyHostToDevice));
  }
  BHIP(hipMemcpy(dsst, sst.data(), 8 * (S + 1), hipMemcpyHostToDevice));
  BHIP(hipMemcpy(dsegc, segc.data(), 4 * nl, hipMemcpyHostToDevice));
  hipLaunchKernelGGL(b_norms, dim3(1024), dim3(256), 0, 0, X, d, nl, xn);
  BHIP(hipGetLastError());

  // 1-2: candidates and forward chunks, in row chunks
  const int64_t rows_per = std::min<int64_t>(nl, 131072);
  // rows of at most MK_DMAX elements: candidates on the matrix cores (BF16 copies)
  const int dp = (d + 31) / 32 * 32;
  const bool mfma = dp <= MK_DMAX;
  u64* lists = buf.alloc<u64>((size_t)rows_per * S * KC);
  int32_t* lens = buf.alloc<int32_t>((size_t)rows_per * S);
  u64* pend = mfma ? nullptr : buf.alloc<u64>((size_t)rows_per * S * KT_C);
  if (!lists || !lens || (!mfma && !pend)) {
    set_error("build: out of device memory");
    return UNIFY_ENOMEM;
  }
  uint16_t* Xb = nullptr;
  float* xnb = nullptr;
  u64* pendm = nullptr;
  if (mfma) {
    Xb = buf.alloc<uint16_t>((size_t)nl * dp);
    xnb = buf.alloc<float>(nl);
    pendm = buf.alloc<u64>((size_t)rows_per * S * MK_PC);
    if (!Xb || !xnb || !pendm) {
      set_error("build: out of device memory");
      return UNIFY_ENOMEM;
    }
    hipLaunchKernelGGL(b_bf16_rows, dim3(2048), dim3(256), 0, 0, X, d, dp, nl, Xb, xnb);
    BHIP(hipGetLastError());
  }
  double t0 = now_s();
  for (int64_t r0 = 0; r0 < nl; r0 += rows_per) {
    const int64_t nr = std::min(rows_per, nl - r0);
    if (mfma) {
      const int rc = run_knn_mfma(KnnMArgs{Xb, xnb, dp, S, K, r0, nr, dsst, lists, lens, pendm, nullptr});
      if (rc) return rc;
    } else {
      KnnArgs ka{X, xn, d, S, K, r0, nr, dsst, lists, lens, pend};
      hipLaunchKernelGGL(b_knn, dim3((unsigned)((nr + KT_R - 1) / KT_R), (unsigned)S), dim3(256), 0, 0, ka);
    }
    BHIP(hipGetLastError());
    PruneArgs pa{};
    pa.X = X;
    pa.d = d;
    pa.ntask = nr * S;
    pa.owner0 = r0;
    pa.owner_div = S;
    pa.a = lists;
    pa.a_stride = KC;
    pa.a_cnt = lens;
    pa.Mcap = M;
    pa.only_if_over = 0;
    pa.out = fwd + (size_t)r0 * S * M;
    int rc = run_prune(pa);
    if (rc) return rc;
    BHIP(hipDeviceSynchronize());
    if (verbose)
      std::fprintf(stderr, "[build] layer n=%lld: candidates+prune rows %lld/%lld (%.1fs)\n", (long long)nl,
                   (long long)(r0 + nr), (long long)nl, now_s() - t0);
  }
  buf.release(lists);
  buf.release(lens);
  if (pend) buf.release(pend);
  if (mfma) {
    buf.release(pendm);
    buf.release(Xb);
    buf.release(xnb);
  }

  // 3: reverse edges and re-prune, over ranges of owners whose reverse edges fit the
  // device memory left (at 10M objects and 64 segments they outgrow one buffer)
  int32_t* rcnt = buf.alloc<int32_t>((size_t)nl * S);
  int64_t* roff = buf.alloc<int64_t>((size_t)nl * S + 1);
  if (!rcnt || !roff) {
    set_error("build: out of device memory");
    return UNIFY_ENOMEM;
  }
  BHIP(hipMemset(rcnt, 0, 4 * (size_t)nl * S));
  hipLaunchKernelGGL(b_rev, dim3(4096), dim3(256), 0, 0, fwd, nl, S, M, dsegc, rcnt, nullptr, nullptr, nullptr,
                     (int64_t)0, INT64_MAX, (int64_t)0);
  int rc = scan(buf, rcnt, nl * S, roff);
  if (rc) return rc;
  int64_t total = 0;
  BHIP(hipMemcpy(&total, roff + (size_t)nl * S, 8, hipMemcpyDeviceToHost));
  size_t free_b = 0, total_b = 0;
  BHIP(hipMemGetInfo(&free_b, &total_b));
  const int64_t cap = std::max<int64_t>(std::min<int64_t>(std::max<int64_t>(total, 1),
                                                           (int64_t)(free_b / 2 / sizeof(u64))),
                                        (int64_t)S * M * 1024);
  u64* rev = buf.alloc<u64>((size_t)cap);
  if (!rev) {
    set_error("build: out of device memory");
    return UNIFY_ENOMEM;
  }
  int64_t nranges = 0;
  for (int64_t o0 = 0; o0 < nl;) {
    // the longest run of owners from o0 whose reverse edges fit, by halving
    int64_t o1 = nl, lo = 0, hi = 0;
    BHIP(hipMemcpy(&lo, roff + (size_t)o0 * S, 8, hipMemcpyDeviceToHost));
    while (true) {
      BHIP(hipMemcpy(&hi, roff + (size_t)o1 * S, 8, hipMemcpyDeviceToHost));
      if (hi - lo <= cap || o1 == o0 + 1) break;
      o1 = o0 + (o1 - o0 + 1) / 2;
    }
    if (hi - lo > cap) {
      set_error("build: the reverse edges of one object exceed the device memory");
      return UNIFY_ENOMEM;
    }
    BHIP(hipMemset(rcnt + (size_t)o0 * S, 0, 4 * (size_t)(o1 - o0) * S));
    hipLaunchKernelGGL(b_rev, dim3(4096), dim3(256), 0, 0, fwd, nl, S, M, dsegc, rcnt, roff, rev, nullptr, o0 * S,
                       o1 * S, lo);
    PruneArgs pa{};
    pa.X = X;
    pa.d = d;
    pa.ntask = (o1 - o0) * S;
    pa.owner0 = o0;
    pa.owner_div = S;
    pa.a = fwd + (size_t)o0 * S * M;
    pa.a_stride = M;
    pa.b = rev;
    pa.b_off = roff + (size_t)o0 * S;
    pa.b_base = lo;
    pa.b_cnt = rcnt + (size_t)o0 * S;
    pa.Mcap = M;
    pa.only_if_over = 1;
    pa.out = fwd + (size_t)o0 * S * M;  // each task reads its own row before writing it
    rc = run_prune(pa);
    if (rc) return rc;
    BHIP(hipDeviceSynchronize());
    ++nranges;
    o0 = o1;
  }
  buf.release(rev);
  if (verbose)
    std::fprintf(stderr, "[build] layer n=%lld: reverse edges %lld in %lld owner ranges (%.1fs)\n", (long long)nl,
                 (long long)total, (long long)nranges, now_s() - t0);

  // 4: global-edge marks
  u64* P = buf.alloc<u64>((size_t)nl * M);
  int32_t* mcnt = buf.alloc<int32_t>(nl);
  int64_t* moff = buf.alloc<int64_t>(nl + 1);
  int32_t* glist = buf.alloc<int32_t>((size_t)nl * M);
  if (!P || !mcnt || !moff || !glist) {
    set_error("build: out of device memory");
    return UNIFY_ENOMEM;
  }
  {
    PruneArgs pa{};
    pa.X = X;
    pa.d = d;
    pa.ntask = nl;
    pa.owner0 = 0;
    pa.owner_div = 1;
    pa.a = fwd;
    pa.a_stride = S * M;
    pa.Mcap = M;
    pa.only_if_over = 1;
    pa.out = P;
    rc = run_prune(pa);
    if (rc) return rc;
  }
  BHIP(hipMemset(mcnt, 0, 4 * nl));
  hipLaunchKernelGGL(b_mask_rev, dim3(4096), dim3(256), 0, 0, P, fwd, nl, S, M, dsegc, mcnt, nullptr, nullptr);
  rc = scan(buf, mcnt, nl, moff);
  if (rc) return rc;
  int64_t mtotal = 0;
  BHIP(hipMemcpy(&mtotal, moff + nl, 8, hipMemcpyDeviceToHost));
  int32_t* mrev = buf.alloc<int32_t>((size_t)std::max<int64_t>(mtotal, 1));
  if (!mrev) {
    set_error("build: out of device memory");
    return UNIFY_ENOMEM;
  }
  BHIP(hipMemset(mcnt, 0, 4 * nl));
  hipLaunchKernelGGL(b_mask_rev, dim3(4096), dim3(256), 0, 0, P, fwd, nl, S, M, dsegc, mcnt, moff, mrev);
  hipLaunchKernelGGL(b_mask_final, dim3((unsigned)((nl + 255) / 256)), dim3(256), 0, 0, P, nl, M, moff, mrev, dext,
                     glist);
  BHIP(hipGetLastError());
  BHIP(hipDeviceSynchronize());
  if (verbose)
    std::fprintf(stderr, "[build] layer n=%lld: global marks (%.1fs)\n", (long long)nl, now_s() - t0);

  // 5: to the host in slices of rows, as internal ids, with the global-edge bits
  const int W = (S * M + 31) / 32;
  const int64_t rows_out = std::max<int64_t>(1, std::min<int64_t>(nl, (int64_t)(64 << 20) / ((int64_t)S * M)));
  uint32_t* dbits = buf.alloc<uint32_t>((size_t)rows_out * W);
  if (!dbits) {
    set_error("build: out of device memory");
    return UNIFY_ENOMEM;
  }
  std::vector<u64> hk((size_t)rows_out * S * M);
  std::vector<int32_t> ch((size_t)rows_out * S * M);
  std::vector<uint32_t> hb((size_t)rows_out * W);
  for (int64_t r0 = 0; r0 < nl; r0 += rows_out) {
    const int64_t nr = std::min(rows_out, nl - r0);
    hipLaunchKernelGGL(b_gbits, dim3(2048), dim3(256), 0, 0, fwd, glist, r0, nr, S, M, W, dbits);
    BHIP(hipGetLastError());
    BHIP(hipMemcpy(hk.data(), fwd + (size_t)r0 * S * M, 8 * (size_t)nr * S * M, hipMemcpyDeviceToHost));
    BHIP(hipMemcpy(hb.data(), dbits, 4 * (size_t)nr * W, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < (size_t)nr * S * M; ++i) ch[i] = hk[i] == KEY_MAX ? -1 : nodes[(int32_t)(uint32_t)hk[i]];
    emit(r0, nr, ch.data(), hb.data());
  }
  return UNIFY_OK;
}

}  // namespace

// The builder's Prune on caller-given candidate lists (device memory throughout).
int prune_impl(const float* X, int64_t n, int32_t d, const int32_t* owners, const int32_t* cand, int64_t t,
               int32_t c, int32_t M, int32_t* out, void* stream) {
  if (t < 0 || n < 1 || d < 4 || d % 4 || d > 2048 || c < 1 || c > CAPR || M < 1 || M > 64 ||
      (t > 0 && (!X || !owners || !cand || !out))) {
    set_error("unify_prune: t >= 0, n >= 1, d % 4 == 0, 4 <= d <= 2048, 1 <= c <= 256, 1 <= M <= 64, "
              "non-null buffers");
    return UNIFY_EINVAL;
  }
  if (t == 0) return UNIFY_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  void* mem = nullptr;
  const size_t nin = (size_t)t * c, nout = (size_t)t * M;
  BHIP(hipMallocAsync(&mem, sizeof(u64) * (nin + nout), st));
  u64* keys = static_cast<u64*>(mem);
  u64* okeys = keys + nin;
  hipLaunchKernelGGL(b_ids_to_keys, dim3(1024), dim3(256), 0, st, cand, (int64_t)nin, keys);
  PruneArgs pa{};
  pa.X = X;
  pa.d = d;
  pa.ntask = t;
  pa.owner0 = 0;
  pa.owner_div = 1;
  pa.owners = owners;
  pa.a = keys;
  pa.a_stride = c;
  pa.Mcap = M;
  pa.only_if_over = 0;
  pa.out = okeys;
  int rc = run_prune(pa, st);
  if (rc == UNIFY_OK) hipLaunchKernelGGL(b_keys_to_ids, dim3(1024), dim3(256), 0, st, okeys, (int64_t)nout, out);
  if (hipFreeAsync(mem, st) != hipSuccess && rc == UNIFY_OK) rc = UNIFY_EDEVICE;
  return rc;
}

int build_impl(const float* vectors, const int64_t* attr, const double* level_u, int64_t n, int32_t d, int32_t S,
               int32_t M, int32_t ef_cons, int device, int precision, unify_index_t* out) {
  if (!vectors || !attr || !level_u || !out) {
    set_error("build: null argument");
    return UNIFY_EINVAL;
  }
  if (n < 2 || n >= (int64_t(1) << 31) || d < 4 || d % 4 || d > 2048 || S < 1 || S > 64 || M < 2 || M > 64 ||
      ef_cons < 1) {
    set_error("build: arguments out of range (2 <= n < 2^31, d % 4 == 0, d <= 2048, 1 <= S <= 64, 2 <= M <= 64)");
    return UNIFY_EINVAL;
  }
  for (int64_t i = 0; i < n; ++i)
    if (!(level_u[i] > 0.0 && level_u[i] <= 1.0)) {
      set_error("build: level variates must lie in (0, 1]");
      return UNIFY_EINVAL;
    }
  if (hipSetDevice(device) != hipSuccess) {
    set_error("build: hipSetDevice failed");
    return UNIFY_EDEVICE;
  }
  const bool verbose = std::getenv("UNIFY_BUILD_VERBOSE") != nullptr;
  const int K = std::min(ef_cons, KC);
  HostIndex H;
  H.n = n;
  H.d = d;
  H.S = S;
  H.M0 = M;
  H.MU = M;
  H.ef_cons = ef_cons;
  H.mL = 1.0 / std::log((double)M);
  // attribute order: internal id = rank by (attribute, external id)
  std::vector<int64_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(),
            [&](int64_t a, int64_t b) { return attr[a] < attr[b] || (attr[a] == attr[b] && a < b); });
  H.attr.resize(n);
  H.ext.resize(n);
  H.level.resize(n);
  H.uprow.resize(n);
  H.vec.resize((size_t)n * d);
  for (int64_t r = 0; r < n; ++r) {
    const int64_t v = order[r];
    H.attr[r] = attr[v];
    H.ext[r] = v;
    const double lv = std::floor(-std::log(level_u[v]) * H.mL);
    H.level[r] = (uint8_t)std::min(lv, 30.0);
    std::memcpy(&H.vec[(size_t)r * d], vectors + (size_t)v * d, 4 * (size_t)d);
  }
  // segments: equi-depth boundaries over all objects; a boundary value opens its segment
  H.seg_start.assign(S + 1, 0);
  for (int j = 1; j < S; ++j) {
    const int64_t b = H.attr[(size_t)((int64_t)j * n / S)];
    H.seg_start[j] = std::lower_bound(H.attr.begin(), H.attr.end(), b) - H.attr.begin();
  }
  H.seg_start[S] = n;
  int L = 0;
  int64_t R = 0;
  for (int64_t r = 0; r < n; ++r) {
    L = std::max<int>(L, H.level[r]);
    H.uprow[r] = H.level[r] > 0 ? (int32_t)R : -1;
    R += H.level[r];
  }
  H.L = L;
  H.R = R;
  // entries: the first object (smallest external id) at each segment's top level
  H.seg_entry.assign(S, -1);
  H.seg_maxlevel.assign(S, -1);
  for (int j = 0; j < S; ++j) {
    for (int64_t r = H.seg_start[j]; r < H.seg_start[j + 1]; ++r) {
      const int lv = H.level[r];
      if (lv > H.seg_maxlevel[j] || (lv == H.seg_maxlevel[j] && H.ext[r] < H.ext[H.seg_entry[j]])) {
        H.seg_maxlevel[j] = lv;
        H.seg_entry[j] = (int32_t)r;
      }
    }
  }
  H.gentry = -1;
  for (int64_t r = 0; r < n; ++r)
    if (H.level[r] == L && (H.gentry < 0 || H.ext[r] < H.ext[H.gentry])) H.gentry = (int32_t)r;
  H.W0 = (S * M + 31) / 32;
  H.WU = H.W0;
  H.adj0.assign((size_t)n * S * M, -1);
  H.gbits0.assign((size_t)n * H.W0, 0u);
  H.adjU.assign((size_t)R * S * M, -1);
  H.gbitsU.assign((size_t)R * H.WU, 0u);

  float* dX = nullptr;
  if (hipMalloc(&dX, H.vec.size() * 4) != hipSuccess) {
    set_error("build: out of device memory");
    return UNIFY_ENOMEM;
  }
  struct Free {
    float* p;
    ~Free() { (void)hipFree(p); }
  } free_dx{dX};
  BHIP(hipMemcpy(dX, H.vec.data(), H.vec.size() * 4, hipMemcpyHostToDevice));

  for (int l = L; l >= 0; --l) {
    std::vector<int32_t> nodes;
    for (int64_t r = 0; r < n; ++r)
      if (H.level[r] >= l) nodes.push_back((int32_t)r);
    if (nodes.size() < 2) continue;
    auto emit = [&](int64_t c0, int64_t cnt, const int32_t* ch, const uint32_t* bits) {
      for (int64_t c = c0; c < c0 + cnt; ++c) {
        const int64_t v = nodes[c];
        const size_t ur = l == 0 ? (size_t)v : (size_t)(H.uprow[v] + l - 1);
        int32_t* row = l == 0 ? &H.adj0[ur * S * M] : &H.adjU[ur * S * M];
        uint32_t* bw = l == 0 ? &H.gbits0[ur * H.W0] : &H.gbitsU[ur * H.WU];
        std::memcpy(row, ch + (size_t)(c - c0) * S * M, 4 * (size_t)S * M);
        std::memcpy(bw, bits + (size_t)(c - c0) * H.W0, 4 * (size_t)H.W0);
      }
    };
    int rc = build_layer(dX, d, S, M, K, nodes, H.seg_start, H.ext, emit, verbose);
    if (rc) return rc;
  }
  std::string err;
  int rc = validate_index(H, err);
  if (rc) {
    set_error("build produced an invalid index: " + err);
    return rc;
  }
  return make_resident(std::move(H), device, precision, out);
}

// ---------------------------------------------------------------------------
// Incremental insertion (Alg. 6, HSIGInsert, applied to a batch of new objects).
//
// The new objects take the next external ids.  Internal ids stay attribute
// ranks, so the resident tables are rebuilt in the merged order (a remap pass
// over every row, bandwidth-bound) into a new version of the index; segment
// boundaries do not move.  Then, on every layer that gains objects, the new
// objects get their chunks from exact candidates among the layer's objects of
// each segment (old and new) and Prune, each kept neighbour is offered the
// reverse edge (chunks that overflow are re-pruned; untouched chunks keep their
// order), and the layer's global-edge marks are recomputed from its final chunks
// by the builder's rule.  The new version replaces the old one between searches.
// ---------------------------------------------------------------------------
namespace {

// dst[rowmap[r]][c] = idmap[src[r][c]] (-1 stays -1) for c < ws; dst rows are wd wide.
__global__ void i_remap(const int32_t* __restrict__ src, int64_t rows, int ws, int32_t* __restrict__ dst, int wd,
                        const int32_t* __restrict__ rowmap, const int32_t* __restrict__ idmap) {
  const int64_t total = rows * ws;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / ws;
    const int c = (int)(e - r * ws);
    const int32_t v = src[e];
    dst[(int64_t)rowmap[r] * wd + c] = v >= 0 ? idmap[v] : -1;
  }
}

// Row r of src (d floats) to row rowmap[r] of dst.
__global__ void i_scatter_vec(const float* __restrict__ src, int64_t rows, int d, float* __restrict__ dst,
                              const int32_t* __restrict__ rowmap) {
  const int64_t G = d / 4, total = rows * G;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / G, g = e - r * G;
    reinterpret_cast<float4*>(dst + (int64_t)rowmap[r] * d)[g] = reinterpret_cast<const float4*>(src + r * d)[g];
  }
}

// The layer's chunks as keys over layer positions; position p reads adjacency row rowsrc[p].
__global__ void i_load_chunks(const int32_t* __restrict__ adj, const int64_t* __restrict__ rowsrc, int64_t nl,
                              int width, const int32_t* __restrict__ pos_of, u64* __restrict__ out) {
  const int64_t total = nl * width;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / width;
    const int c = (int)(e - p * width);
    const int32_t v = adj[rowsrc[p] * width + c];
    const int32_t q = v >= 0 ? pos_of[v] : -1;
    out[e] = q >= 0 ? make_key(0.f, q) : KEY_MAX;
  }
}

// Row r of fwd (the r-th new object) into the chunk table at position newpos[r].
__global__ void i_scatter_keys(const u64* __restrict__ fwd, int64_t nnew, int width, const int32_t* __restrict__ newpos,
                               u64* __restrict__ chunks) {
  const int64_t total = nnew * width;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / width;
    const int c = (int)(e - r * width);
    chunks[(int64_t)newpos[r] * width + c] = fwd[e];
  }
}

// The (position, segment) chunks that receive reverse edges, in any order.
__global__ void i_tasks(const int32_t* __restrict__ cnt, int64_t n, int64_t* __restrict__ tasks,
                        unsigned long long* __restrict__ ntask) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (cnt[i] > 0) tasks[atomicAdd(ntask, 1ull)] = i;
}

// Chunks back into the adjacency rows, as internal ids.
__global__ void i_store_chunks(const u64* __restrict__ chunks, int64_t nl, int width,
                               const int64_t* __restrict__ rowsrc, const int32_t* __restrict__ nodes,
                               int32_t* __restrict__ adj) {
  const int64_t total = nl * width;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / width;
    const int c = (int)(e - p * width);
    const u64 kk = chunks[e];
    adj[rowsrc[p] * width + c] = kk == KEY_MAX ? -1 : nodes[key_id(kk)];
  }
}

// Marks (layer positions, M per row) into the global-edge lists (GC per row).
__global__ void i_store_glist(const int32_t* __restrict__ marks, int64_t nl, int M,
                              const int64_t* __restrict__ rowsrc, const int32_t* __restrict__ nodes,
                              int32_t* __restrict__ glist, int GC) {
  const int64_t total = nl * GC;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / GC;
    const int c = (int)(e - p * GC);
    const int32_t v = c < M ? marks[p * M + c] : -1;
    glist[rowsrc[p] * GC + c] = v >= 0 ? nodes[v] : -1;
  }
}

unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 16384)); }

// One layer of an insertion.  nodes: the layer's objects (new internal ids,
// ascending); rowsrc[p]: adjacency/global-list row of nodes[p]; newpos: the
// positions of the new objects.  Reads and rewrites adj (width S * mc) and glist.
int insert_layer(const float* dX, int d, int S, int mc, int K, const std::vector<int32_t>& nodes,
                 const std::vector<int64_t>& rowsrc, const std::vector<int32_t>& newpos,
                 const std::vector<int64_t>& seg_start, const std::vector<int64_t>& ext, int64_t nall, int32_t* adj,
                 int32_t* glist, int GC, bool verbose) {
  const int64_t nl = (int64_t)nodes.size(), nnew = (int64_t)newpos.size();
  const int W = S * mc;
  DevBuf buf;
  std::vector<int64_t> sst(S + 1, 0);
  std::vector<int32_t> segc(nl);
  {
    int j = 0;
    for (int64_t c = 0; c < nl; ++c) {
      while (j + 1 <= S && nodes[c] >= seg_start[j + 1]) ++j;
      segc[c] = j;
    }
    for (int jj = 0; jj <= S; ++jj)
      sst[jj] = std::lower_bound(nodes.begin(), nodes.end(), (int32_t)std::min<int64_t>(seg_start[jj], INT32_MAX)) -
                nodes.begin();
    sst[S] = nl;
  }
  std::vector<int32_t> pos_of((size_t)nall, -1);
  std::vector<int64_t> ext_c(nl);
  for (int64_t p = 0; p < nl; ++p) {
    pos_of[nodes[p]] = (int32_t)p;
    ext_c[p] = ext[nodes[p]];
  }
  int32_t* dnodes = buf.alloc<int32_t>(nl);
  float* X = buf.alloc<float>((size_t)nl * d);
  float* xn = buf.alloc<float>(nl);
  int64_t* dsst = buf.alloc<int64_t>(S + 1);
  int32_t* dsegc = buf.alloc<int32_t>(nl);
  int64_t* dext = buf.alloc<int64_t>(nl);
  int64_t* drow = buf.alloc<int64_t>(nl);
  int32_t* dnew = buf.alloc<int32_t>(nnew);
  int32_t* dpos = buf.alloc<int32_t>(nall);
  u64* chunks = buf.alloc<u64>((size_t)nl * W);
  u64* fwd = buf.alloc<u64>((size_t)nnew * W);
  if (!dnodes || !X || !xn || !dsst || !dsegc || !dext || !drow || !dnew || !dpos || !chunks || !fwd) {
    set_error("insert: out of device memory");
    return UNIFY_ENOMEM;
  }
  BHIP(hipMemcpy(dnodes, nodes.data(), 4 * nl, hipMemcpyHostToDevice));
  BHIP(hipMemcpy(dsst, sst.data(), 8 * (S + 1), hipMemcpyHostToDevice));
  BHIP(hipMemcpy(dsegc, segc.data(), 4 * nl, hipMemcpyHostToDevice));
  BHIP(hipMemcpy(dext, ext_c.data(), 8 * nl, hipMemcpyHostToDevice));
  BHIP(hipMemcpy(drow, rowsrc.data(), 8 * nl, hipMemcpyHostToDevice));
  BHIP(hipMemcpy(dnew, newpos.data(), 4 * nnew, hipMemcpyHostToDevice));
  BHIP(hipMemcpy(dpos, pos_of.data(), 4 * nall, hipMemcpyHostToDevice));
  hipLaunchKernelGGL(b_gather, dim3(1024), dim3(256), 0, 0, dX, d, dnodes, nl, X);
  hipLaunchKernelGGL(b_norms, dim3(1024), dim3(256), 0, 0, X, d, nl, xn);
  hipLaunchKernelGGL(i_load_chunks, dim3(grid_for(nl * W)), dim3(256), 0, 0, adj, drow, nl, W, dpos, chunks);
  BHIP(hipGetLastError());

  // 1-2: candidates of the new objects in every segment of the layer, forward chunks
  double t0 = now_s();
  const int64_t rows_per = std::min<int64_t>(nnew, 131072);
  // rows of at most MK_DMAX elements: candidates on the matrix cores (BF16 copies)
  const int dp = (d + 31) / 32 * 32;
  const bool mfma = dp <= MK_DMAX;
  u64* lists = buf.alloc<u64>((size_t)rows_per * S * KC);
  int32_t* lens = buf.alloc<int32_t>((size_t)rows_per * S);
  u64* pend = buf.alloc<u64>((size_t)rows_per * S * (mfma ? MK_PC : KT_C));
  uint16_t* Xb = mfma ? buf.alloc<uint16_t>((size_t)nl * dp) : nullptr;
  float* xnb = mfma ? buf.alloc<float>(nl) : nullptr;
  if (!lists || !lens || !pend || (mfma && (!Xb || !xnb))) {
    set_error("insert: out of device memory");
    return UNIFY_ENOMEM;
  }
  if (mfma) hipLaunchKernelGGL(b_bf16_rows, dim3(2048), dim3(256), 0, 0, X, d, dp, nl, Xb, xnb);
  for (int64_t r0 = 0; r0 < nnew; r0 += rows_per) {
    const int64_t nr = std::min(rows_per, nnew - r0);
    if (mfma) {
      const int rc = run_knn_mfma(KnnMArgs{Xb, xnb, dp, S, K, r0, nr, dsst, lists, lens, pend, dnew});
      if (rc) return rc;
    } else {
      KnnArgs ka{X, xn, d, S, K, r0, nr, dsst, lists, lens, pend, dnew};
      hipLaunchKernelGGL(b_knn, dim3((unsigned)((nr + KT_R - 1) / KT_R), (unsigned)S), dim3(256), 0, 0, ka);
    }
    BHIP(hipGetLastError());
    PruneArgs pa{};
    pa.X = X;
    pa.d = d;
    pa.ntask = nr * S;
    pa.owner0 = r0;
    pa.owner_div = S;
    pa.owners = dnew;
    pa.a = lists;
    pa.a_stride = KC;
    pa.a_cnt = lens;
    pa.Mcap = mc;
    pa.only_if_over = 0;
    pa.out = fwd + (size_t)r0 * W;
    int rc = run_prune(pa);
    if (rc) return rc;
  }
  BHIP(hipDeviceSynchronize());
  buf.release(lists);
  buf.release(lens);
  buf.release(pend);
  if (mfma) {
    buf.release(Xb);
    buf.release(xnb);
  }
  hipLaunchKernelGGL(i_scatter_keys, dim3(grid_for(nnew * W)), dim3(256), 0, 0, fwd, nnew, W, dnew, chunks);
  BHIP(hipGetLastError());
  if (verbose)
    std::fprintf(stderr, "[insert] layer n=%lld new=%lld: candidates+prune (%.2fs)\n", (long long)nl, (long long)nnew,
                 now_s() - t0);

  // 3: reverse edges of the new objects; chunks that receive some are merged and re-pruned
  int32_t* rcnt = buf.alloc<int32_t>((size_t)nl * S);
  int64_t* roff = buf.alloc<int64_t>((size_t)nl * S + 1);
  unsigned long long* dnt = buf.alloc<unsigned long long>(1);
  if (!rcnt || !roff || !dnt) {
    set_error("insert: out of device memory");
    return UNIFY_ENOMEM;
  }
  BHIP(hipMemset(rcnt, 0, 4 * (size_t)nl * S));
  hipLaunchKernelGGL(b_rev, dim3(4096), dim3(256), 0, 0, fwd, nnew, S, mc, dsegc, rcnt, nullptr, nullptr, dnew);
  int rc = scan(buf, rcnt, nl * S, roff);
  if (rc) return rc;
  int64_t total = 0;
  BHIP(hipMemcpy(&total, roff + (size_t)nl * S, 8, hipMemcpyDeviceToHost));
  u64* rev = buf.alloc<u64>((size_t)std::max<int64_t>(total, 1));
  int64_t* tasks = buf.alloc<int64_t>((size_t)std::max<int64_t>(std::min<int64_t>(total, nl * S), 1));
  if (!rev || !tasks) {
    set_error("insert: out of device memory");
    return UNIFY_ENOMEM;
  }
  BHIP(hipMemset(rcnt, 0, 4 * (size_t)nl * S));
  hipLaunchKernelGGL(b_rev, dim3(4096), dim3(256), 0, 0, fwd, nnew, S, mc, dsegc, rcnt, roff, rev, dnew);
  BHIP(hipMemset(dnt, 0, sizeof(unsigned long long)));
  hipLaunchKernelGGL(i_tasks, dim3(grid_for(nl * S)), dim3(256), 0, 0, rcnt, nl * S, tasks, dnt);
  BHIP(hipGetLastError());
  unsigned long long ntask = 0;
  BHIP(hipMemcpy(&ntask, dnt, sizeof(ntask), hipMemcpyDeviceToHost));
  if ((int64_t)ntask > std::min<int64_t>(total, nl * S)) {
    set_error("insert: reverse-edge task count out of range");
    return UNIFY_EDEVICE;
  }
  if (ntask > 0) {
    PruneArgs pa{};
    pa.X = X;
    pa.d = d;
    pa.ntask = (int64_t)ntask;
    pa.owner0 = 0;
    pa.owner_div = S;
    pa.a = chunks;
    pa.a_stride = mc;
    pa.b = rev;
    pa.b_off = roff;
    pa.b_cnt = rcnt;
    pa.Mcap = mc;
    pa.only_if_over = 1;
    pa.out = chunks;  // each task reads its own row before writing it
    pa.task_of = tasks;
    rc = run_prune(pa);
    if (rc) return rc;
  }
  BHIP(hipDeviceSynchronize());
  buf.release(rev);
  buf.release(tasks);
  if (verbose)
    std::fprintf(stderr, "[insert] layer n=%lld: reverse edges %lld into %llu chunks (%.2fs)\n", (long long)nl,
                 (long long)total, ntask, now_s() - t0);

  // 4: global-edge marks of the layer from its final chunks
  u64* P = buf.alloc<u64>((size_t)nl * mc);
  int32_t* mcnt = buf.alloc<int32_t>(nl);
  int64_t* moff = buf.alloc<int64_t>(nl + 1);
  int32_t* marks = buf.alloc<int32_t>((size_t)nl * mc);
  if (!P || !mcnt || !moff || !marks) {
    set_error("insert: out of device memory");
    return UNIFY_ENOMEM;
  }
  {
    PruneArgs pa{};
    pa.X = X;
    pa.d = d;
    pa.ntask = nl;
    pa.owner0 = 0;
    pa.owner_div = 1;
    pa.a = chunks;
    pa.a_stride = W;
    pa.Mcap = mc;
    pa.only_if_over = 1;
    pa.out = P;
    rc = run_prune(pa);
    if (rc) return rc;
  }
  BHIP(hipMemset(mcnt, 0, 4 * nl));
  hipLaunchKernelGGL(b_mask_rev, dim3(4096), dim3(256), 0, 0, P, chunks, nl, S, mc, dsegc, mcnt, nullptr, nullptr);
  rc = scan(buf, mcnt, nl, moff);
  if (rc) return rc;
  int64_t mtotal = 0;
  BHIP(hipMemcpy(&mtotal, moff + nl, 8, hipMemcpyDeviceToHost));
  int32_t* mrev = buf.alloc<int32_t>((size_t)std::max<int64_t>(mtotal, 1));
  if (!mrev) {
    set_error("insert: out of device memory");
    return UNIFY_ENOMEM;
  }
  BHIP(hipMemset(mcnt, 0, 4 * nl));
  hipLaunchKernelGGL(b_mask_rev, dim3(4096), dim3(256), 0, 0, P, chunks, nl, S, mc, dsegc, mcnt, moff, mrev);
  hipLaunchKernelGGL(b_mask_final, dim3((unsigned)((nl + 255) / 256)), dim3(256), 0, 0, P, nl, mc, moff, mrev, dext,
                     marks);
  // 5: back into the index
  hipLaunchKernelGGL(i_store_chunks, dim3(grid_for(nl * W)), dim3(256), 0, 0, chunks, nl, W, drow, dnodes, adj);
  hipLaunchKernelGGL(i_store_glist, dim3(grid_for(nl * GC)), dim3(256), 0, 0, marks, nl, mc, drow, dnodes, glist, GC);
  BHIP(hipGetLastError());
  BHIP(hipDeviceSynchronize());
  if (verbose) std::fprintf(stderr, "[insert] layer n=%lld: global marks (%.2fs)\n", (long long)nl, now_s() - t0);
  return UNIFY_OK;
}

// Device allocations of a new index version; freed unless kept.
struct Version {
  std::vector<void*> ptrs;
  bool keep = false;
  ~Version() {
    if (!keep)
      for (void* p : ptrs) (void)hipFree(p);
  }
  template <class T>
  T* alloc(size_t count) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return static_cast<T*>(p);
  }
};

}  // namespace

int insert_impl(unify_index_t ix, const float* vectors, const int64_t* attr, const double* level_u, int64_t m) {
  if (!ix || m < 0 || (m > 0 && (!vectors || !attr || !level_u))) {
    set_error("insert: null argument or negative count");
    return UNIFY_EINVAL;
  }
  if (m == 0) return UNIFY_OK;
  std::lock_guard<std::mutex> serial(ix->insert_mu);
  if (hipSetDevice(ix->device) != hipSuccess) {
    set_error("insert: hipSetDevice failed");
    return UNIFY_EDEVICE;
  }
  const bool verbose = std::getenv("UNIFY_BUILD_VERBOSE") != nullptr;
  std::shared_lock<std::shared_mutex> rl(ix->version_mu);
  const DevIndex dv = ix->dv;
  const HostIndex& O = ix->host;
  const int64_t n = dv.n, n2 = n + m;
  const int S = dv.S, d = dv.d;
  if (n2 >= (int64_t(1) << 31)) {
    set_error("insert: the index would exceed 2^31 - 1 objects");
    return UNIFY_EINVAL;
  }
  if (!prune_kernel(d, dv.M0) || !prune_kernel(d, dv.MU) || O.ef_cons < 1) {
    set_error("insert: unsupported index shape (d <= 2048, M <= 64, efCons >= 1)");
    return UNIFY_EINVAL;
  }
  for (int64_t t = 0; t < m; ++t)
    if (!(level_u[t] > 0.0 && level_u[t] <= 1.0)) {
      set_error("insert: level variates must lie in (0, 1]");
      return UNIFY_EINVAL;
    }
  const double mL = O.mL > 0 ? O.mL : 1.0 / std::log((double)dv.M0);
  const int K = std::min(O.ef_cons, KC);
  int64_t xb = 0;
  for (int64_t i = 0; i < n; ++i) xb = std::max(xb, O.ext[i] + 1);
  std::vector<int> lev_new(m);
  for (int64_t t = 0; t < m; ++t) lev_new[t] = (int)std::min(std::floor(-std::log(level_u[t]) * mL), 30.0);
  // merged attribute order; an old object precedes a new one with the same attribute (smaller external id)
  std::vector<int64_t> ordn(m);
  std::iota(ordn.begin(), ordn.end(), 0);
  std::stable_sort(ordn.begin(), ordn.end(), [&](int64_t a, int64_t b) { return attr[a] < attr[b]; });
  std::vector<int32_t> nid_old(n), nid_new(m);
  HostIndex H;
  H.n = n2;
  H.d = d;
  H.S = S;
  H.M0 = O.M0;
  H.MU = O.MU;
  H.ef_cons = O.ef_cons;
  H.mL = O.mL;
  H.seed = O.seed;
  H.W0 = O.W0;
  H.WU = O.WU;
  H.attr.resize(n2);
  H.ext.resize(n2);
  H.level.resize(n2);
  std::vector<uint8_t> isnew(n2, 0);
  {
    int64_t i = 0, t = 0;
    for (int64_t r = 0; r < n2; ++r) {
      if (t >= m || (i < n && O.attr[i] <= attr[ordn[t]])) {
        nid_old[i] = (int32_t)r;
        H.attr[r] = O.attr[i];
        H.ext[r] = O.ext[i];
        H.level[r] = O.level[i];
        ++i;
      } else {
        const int64_t u = ordn[t++];
        nid_new[u] = (int32_t)r;
        H.attr[r] = attr[u];
        H.ext[r] = xb + u;
        H.level[r] = (uint8_t)lev_new[u];
        isnew[r] = 1;
      }
    }
  }
  H.uprow.resize(n2);
  int64_t R2 = 0;
  for (int64_t r = 0; r < n2; ++r) {
    H.uprow[r] = H.level[r] > 0 ? (int32_t)R2 : -1;
    R2 += H.level[r];
  }
  H.R = R2;
  std::vector<int32_t> rowmap_up((size_t)std::max<int64_t>(dv.R, 1));
  for (int64_t i = 0; i < n; ++i)
    for (int l = 1; l <= O.level[i]; ++l) rowmap_up[O.uprow[i] + l - 1] = H.uprow[nid_old[i]] + l - 1;
  // fixed boundaries: segment j starts at the first attribute >= b_j
  std::vector<int64_t> bval(S > 1 ? S - 1 : 0);
  for (int j = 1; j < S; ++j) bval[j - 1] = O.seg_start[j] < n ? O.attr[O.seg_start[j]] : INT64_MAX;
  H.seg_start.assign(S + 1, 0);
  for (int j = 1; j < S; ++j)
    H.seg_start[j] = std::lower_bound(H.attr.begin(), H.attr.end(), bval[j - 1]) - H.attr.begin();
  H.seg_start[S] = n2;
  // entries (Alg. 6): a segment's entry changes only when an object of that
  // segment exceeds its top level; the first such object wins
  H.seg_entry.resize(S);
  H.seg_maxlevel = O.seg_maxlevel;
  for (int j = 0; j < S; ++j) H.seg_entry[j] = O.seg_entry[j] >= 0 ? nid_old[O.seg_entry[j]] : -1;
  H.L = O.L;
  H.gentry = O.gentry >= 0 ? nid_old[O.gentry] : -1;
  for (int64_t t = 0; t < m; ++t) {
    const int j = (int)(std::upper_bound(bval.begin(), bval.end(), attr[t]) - bval.begin());
    if (lev_new[t] > H.seg_maxlevel[j]) {
      H.seg_maxlevel[j] = lev_new[t];
      H.seg_entry[j] = nid_new[t];
    }
    if (lev_new[t] > H.L) {
      H.L = lev_new[t];
      H.gentry = nid_new[t];
    }
  }

  // the new version: remapped copies of the resident tables
  Version V;
  const int GC2 = std::max(dv.GC, std::max(dv.M0, dv.MU));
  const int W0 = S * dv.M0, WU = S * dv.MU;
  int64_t* d_attr = V.alloc<int64_t>(n2);
  int64_t* d_ext = V.alloc<int64_t>(n2);
  int64_t* d_ss = V.alloc<int64_t>(S + 1);
  int32_t* d_se = V.alloc<int32_t>(S);
  int32_t* d_sm = V.alloc<int32_t>(S);
  int32_t* d_up = V.alloc<int32_t>(n2);
  float* d_vec = V.alloc<float>((size_t)n2 * d);
  int32_t* d_adj0 = V.alloc<int32_t>((size_t)n2 * W0);
  int32_t* d_gl0 = V.alloc<int32_t>((size_t)n2 * GC2);
  int32_t* d_adjU = V.alloc<int32_t>((size_t)R2 * WU);
  int32_t* d_glU = V.alloc<int32_t>((size_t)R2 * GC2);
  DevBuf tmp;
  float* d_new = tmp.alloc<float>((size_t)m * d);
  int32_t* d_nold = tmp.alloc<int32_t>(n);
  int32_t* d_nnew = tmp.alloc<int32_t>(m);
  int32_t* d_rmap = tmp.alloc<int32_t>(rowmap_up.size());
  if (!d_attr || !d_ext || !d_ss || !d_se || !d_sm || !d_up || !d_vec || !d_adj0 || !d_gl0 || !d_adjU || !d_glU ||
      !d_new || !d_nold || !d_nnew || !d_rmap) {
    set_error("insert: out of device memory");
    return UNIFY_ENOMEM;
  }
  BHIP(hipMemcpy(d_attr, H.attr.data(), 8 * n2, hipMemcpyHostToDevice));
  BHIP(hipMemcpy(d_ext, H.ext.data(), 8 * n2, hipMemcpyHostToDevice));
  BHIP(hipMemcpy(d_ss, H.seg_start.data(), 8 * (S + 1), hipMemcpyHostToDevice));
  BHIP(hipMemcpy(d_se, H.seg_entry.data(), 4 * S, hipMemcpyHostToDevice));
  BHIP(hipMemcpy(d_sm, H.seg_maxlevel.data(), 4 * S, hipMemcpyHostToDevice));
  BHIP(hipMemcpy(d_up, H.uprow.data(), 4 * n2, hipMemcpyHostToDevice));
  BHIP(hipMemcpy(d_new, vectors, 4 * (size_t)m * d, hipMemcpyHostToDevice));
  BHIP(hipMemcpy(d_nold, nid_old.data(), 4 * n, hipMemcpyHostToDevice));
  BHIP(hipMemcpy(d_nnew, nid_new.data(), 4 * m, hipMemcpyHostToDevice));
  BHIP(hipMemcpy(d_rmap, rowmap_up.data(), 4 * rowmap_up.size(), hipMemcpyHostToDevice));
  BHIP(hipMemset(d_adj0, 0xFF, 4 * (size_t)n2 * W0));
  BHIP(hipMemset(d_gl0, 0xFF, 4 * (size_t)n2 * GC2));
  if (R2 > 0) {
    BHIP(hipMemset(d_adjU, 0xFF, 4 * (size_t)R2 * WU));
    BHIP(hipMemset(d_glU, 0xFF, 4 * (size_t)R2 * GC2));
  }
  const double t0 = now_s();
  hipLaunchKernelGGL(i_scatter_vec, dim3(grid_for(n * d / 4)), dim3(256), 0, 0, dv.vec, n, d, d_vec, d_nold);
  hipLaunchKernelGGL(i_scatter_vec, dim3(grid_for(m * d / 4)), dim3(256), 0, 0, d_new, m, d, d_vec, d_nnew);
  hipLaunchKernelGGL(i_remap, dim3(grid_for(n * W0)), dim3(256), 0, 0, dv.adj0, n, W0, d_adj0, W0, d_nold, d_nold);
  hipLaunchKernelGGL(i_remap, dim3(grid_for(n * dv.GC)), dim3(256), 0, 0, dv.glist0, n, dv.GC, d_gl0, GC2, d_nold,
                     d_nold);
  if (dv.R > 0) {
    hipLaunchKernelGGL(i_remap, dim3(grid_for(dv.R * WU)), dim3(256), 0, 0, dv.adjU, dv.R, WU, d_adjU, WU, d_rmap,
                       d_nold);
    hipLaunchKernelGGL(i_remap, dim3(grid_for(dv.R * dv.GC)), dim3(256), 0, 0, dv.glistU, dv.R, dv.GC, d_glU, GC2,
                       d_rmap, d_nold);
  }
  BHIP(hipGetLastError());
  BHIP(hipDeviceSynchronize());
  if (verbose) std::fprintf(stderr, "[insert] remapped %lld + %lld objects (%.2fs)\n", (long long)n, (long long)m,
                            now_s() - t0);

  // every layer that gains objects, top down
  for (int l = H.L; l >= 0; --l) {
    std::vector<int32_t> nodes, newpos;
    std::vector<int64_t> rowsrc;
    for (int64_t r = 0; r < n2; ++r) {
      if (H.level[r] < l) continue;
      if (isnew[r]) newpos.push_back((int32_t)nodes.size());
      nodes.push_back((int32_t)r);
      rowsrc.push_back(l == 0 ? r : (int64_t)H.uprow[r] + l - 1);
    }
    if (newpos.empty() || nodes.size() < 2) continue;
    int rc = insert_layer(d_vec, d, S, l == 0 ? dv.M0 : dv.MU, K, nodes, rowsrc, newpos, H.seg_start, H.ext, n2,
                          l == 0 ? d_adj0 : d_adjU, l == 0 ? d_gl0 : d_glU, GC2, verbose);
    if (rc) return rc;
  }
  if (verbose) std::fprintf(stderr, "[insert] done (%.2fs)\n", now_s() - t0);

  DevIndex nv = dv;
  nv.n = n2;
  nv.L = H.L;
  nv.gentry = H.gentry;
  nv.R = R2;
  nv.GC = GC2;
  nv.attr = d_attr;
  nv.ext = d_ext;
  nv.seg_start = d_ss;
  nv.seg_entry = d_se;
  nv.seg_maxlevel = d_sm;
  nv.uprow = d_up;
  nv.vec = d_vec;
  nv.adj0 = d_adj0;
  nv.glist0 = d_gl0;
  nv.adjU = R2 > 0 ? d_adjU : nullptr;
  nv.glistU = R2 > 0 ? d_glU : nullptr;
  nv.vec_bf16 = nullptr;
  nv.vec_fp8 = nullptr;
  nv.vec_scale = nullptr;
  nv.vec_eps = nullptr;
  nv.attr2 = nullptr;  // a second attribute is set again for the grown index
  nv.attr2_sample = nullptr;
  nv.n2s = 0;
  nv.precision = UNIFY_FP32;
  rl.unlock();

  // swap between searches: wait for every search enqueued on the old version
  std::unique_lock<std::shared_mutex> wl(ix->version_mu);
  const int precision = ix->dv.precision;  // as the caller last set it
  BHIP(hipDeviceSynchronize());  // every search, on any visited pool
  for (void* p : ix->allocs)
    if (p) (void)hipFree(p);
  ix->allocs = V.ptrs;
  V.keep = true;
  for (auto& e : ix->eps_of) e = nullptr;
  for (auto& e : ix->nrm_of) e = nullptr;
  ix->dv = nv;
  ix->z = ZOrder{};  // the z-order attributes are set again for the grown index
  ix->host = std::move(H);
  ++ix->version;
  const int rc = quantize_store(ix, precision);
  return rc == UNIFY_OK ? ensure_pool(ix) : rc;  // rows for the new size
}

}  // namespace unify
