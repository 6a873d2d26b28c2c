// Range-filtered k-NN search over a resident HSIG on gfx950.
//
// One 64-lane wavefront runs one work item (persistent waves pull items from a
// work list): a graph search, or one chunk of a pre-filter scan.  The
// strategies follow Sec. 4.2 of the paper:
//   pre    (strategy A): exact scan of the contiguous id slice [lo, hi), split
//          into chunks on several wavefronts and merged by k_pre_merge;
//   hybrid (strategy C): the scheme of Alg. 2 with Alg. 7 on each layer, over the
//          first ceil(m / S') entries of each active chunk;
//   post   (strategy B): Alg. 2 with Alg. 1 over the global (marked) edges, then
//          the range filter.
// The choice between them is the range-aware rule of Sec. 4.2.
//
// A layer search keeps three structures in LDS:
//   visited  an 8-way set-associative cache of ids; an id whose set is full
//            is decided by its bit in the wave's HBM bitmap row instead (each
//            id lives in exactly one of the two), and a layer search that used
//            the row clears the words it set before it returns;
//   cand     an unsorted array of keys with tombstones; pop = wave argmin;
//   ann      a sorted key list kept by bitonic block merges.
// One step pops up to p candidates (p = 1 is the sequential loop), gathers
// their unvisited neighbours, evaluates all distances at once, and admits each
// neighbour against the threshold taken before the step.  With a strict total
// order on keys this gives the same ann and the same stopping point as
// evaluating the neighbours one at a time: an entry a batch admits that the
// sequential loop would reject has a key at or above the final threshold).  If a query's candidate array outgrows its LDS capacity,
// the query is abandoned and re-run by a second launch with a larger array.
// With a BF16 / FP8 store, graph results are re-scored in FP32 and the
// pre-filter scan proves its result with error bounds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "lowp.h"
#include "unify_internal.h"
#include "wave.h"
#include "zorder.h"

// Scratch of the allocation-free entry point (plans, work list and partial
// lists of one call): one array in every GPU's memory from the moment the code
// object is loaded until the process ends.  Host code never passes this name to
// a kernel (on the host it is only a stand-in); it uses the device address
// hipGetSymbolAddress returns for the current device.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace unify {

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[MAX_DEVICES] = {};  // device address of `scratch` on each device

// The address of `scratch` on `device` (the current device), looked up once.
int noalloc_scratch(int device, void** out) {
  if (device < 0 || device >= MAX_DEVICES) {
    set_error("device ordinal out of range");
    return UNIFY_EINVAL;
  }
  std::lock_guard<std::mutex> g(g_noalloc_mu);
  if (!g_noalloc_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return UNIFY_EDEVICE;
    }
    g_noalloc_ptr[device] = p;
  }
  *out = g_noalloc_ptr[device];
  return UNIFY_OK;
}
}  // namespace

struct SearchArgs {
  DevIndex ix;
  const float* Q;
  int64_t nq;
  int32_t k, ef, m, p, rerank;
  int32_t ccap, hcap, ef_blocks, nbr_cap, sel_cap;
  int32_t pass;  // 0: first pass, 1: larger-capacity re-run
  float bA, bB, bC, bD;  // constants of root_bounds
  int64_t* out_ids;
  float* out_dist;
  int32_t* out_stats;
  const QPlan* plan;
  const int32_t* work;    // query indices to run
  const int32_t* wchunk;  // chunk of each work entry (pre-filter scans), or null for 0
  const int32_t* nwork;   // number of entries in work
  u64* part;              // partial top-k lists of split pre-filter scans, k keys per chunk
  int32_t* qacc;          // [nq][4] per query: chunks finished, FP32 re-scores, objects scanned,
                          // chunks that fell back to the FP32 scan
  int32_t* next;          // work counter
  int32_t* fb_list;       // queries abandoned by the first pass
  int32_t* fb_count;
  uint32_t* vrows;        // [nslots][vstride] visited rows, one per persistent wave
  int64_t vstride;        // words of a row: the bitmap (bwords) then the log (VLOG_CAP)
  int64_t bwords;         // words of a row's bitmap (ceil(n / 32), padded)
  int64_t nslots;
  const struct ConjArgs* conj;  // conjunctive queries (written by the plan kernel), or null
  // cooperative searches: heavy queries work[0, *nheavy), the graph searches work[0, *nbeam)
  // (the rest of the work list holds pre-filter chunks), the heavy counter, first visited row
  const int32_t* nheavy;
  const int32_t* nbeam;
  int32_t* mw_next;
  int64_t mw_row0;
};

// Second attribute and per-query inclusive ranges of a conjunctive search; for a
// box search on a z-order index, both attributes and both ranges (attr1 is null
// otherwise).  The search kernel reaches them through one pointer, read where a
// test is made, so single-attribute searches hold no extra registers.
struct ConjArgs {
  const int64_t* attr2;
  const int64_t* l2;
  const int64_t* h2;
  const int64_t* attr1;
  const int64_t* l1;
  const int64_t* h1;
  int64_t zb1, zb2;  // box searches: the key map
  int32_t zs1, zs2;
};

// The attribute test of a conjunctive or box query (always true for others).
struct Sec {
  int32_t q;
};
__device__ __forceinline__ bool sec_ok(const SearchArgs& A, Sec s, int32_t v) {
  if (!A.conj) return true;
  const ConjArgs c = *A.conj;
  const bool in2 = c.attr2[v] >= c.l2[s.q] && c.attr2[v] <= c.h2[s.q];
  return c.attr1 ? in2 && c.attr1[v] >= c.l1[s.q] && c.attr1[v] <= c.h1[s.q] : in2;
}

constexpr uint32_t HASH_EMPTY = 0xFFFFFFFFu;
// Register budgets of the search kernels (measured on the 1M workload): the
// BF16 and FP8 kernels are held to 128 VGPRs for 4 wavefronts per SIMD (BF16
// with 4 rounds of raw loads in flight instead of 8, which would spill), the
// FP32 kernel to 168 for 3; a wavefront's LDS then decides (about 8.5 KB with
// a 512-entry visited cache for 4 per SIMD).  Rows wider than 256 elements
// hold the query in NG * 4 registers and keep the compiler's own budget.
constexpr int WAVES_PER_SIMD_FP32 = 3, WAVES_PER_SIMD_LOW = 4, BF16_ROUNDS = 4;
constexpr int PRE_NCH_MAX = 8;      // chunks per pre-filter scan at most
constexpr int PLAN_SAMPLES = 2048;  // sorted attributes staged in LDS by the plan kernel
constexpr int PRE_SPLIT_KMAX = 128;  // larger k scans its slice in one wavefront
// Matrix-core pre-filter scan (see k_tile_scan).
constexpr int TILE_ROWS = 256;  // objects per super-block
constexpr int TILE_Q = 16;      // queries per matrix tile (the MFMA M dimension)
constexpr int TILE_KMAX = 32;   // larger k scans per wavefront
constexpr int TILE_DMAX = 512;  // wider rows scan per wavefront (the tile's queries stay in LDS)
constexpr int TILE_PAIRS_PER_QUERY = 6;  // record budget per query of a batch (beyond it: per-wave scans)
constexpr int STRAT_INVALID = -2;    // out_strategy of a row whose requested strategy is unknown
constexpr int STATUS_INVALID = 3;    // its status counter

// ---------------------------------------------------------------------------
// Plan: the range becomes an id interval [lo, hi) (the skip-list walk of
// strategy A reduces to two binary searches over the sorted attributes), Y =
// hi - lo, the active segments are those of lo and hi - 1, and the strategy
// follows the range-aware rule unless the caller forces one.
// ---------------------------------------------------------------------------
__device__ int64_t lower_bound_i64(const int64_t* a, int64_t n, int64_t x) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}
__device__ int64_t upper_bound_i64(const int64_t* a, int64_t n, int64_t x) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] <= x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Plans every query: its in-range id interval, strategy, active segments and the
// pre-filter's chunks.  A box search (box != 0, z-order index z) takes l, h as the
// first attribute's ranges and l2, h2 as the second's, and searches the key range
// between the keys of the box's lower and upper corners, which holds every object
// of the box (the coordinates and the key are non-decreasing).
__global__ void k_plan(DevIndex ix, const int64_t* __restrict__ l, const int64_t* __restrict__ h,
                       const int64_t* __restrict__ l2, const int64_t* __restrict__ h2, ZOrder z, int32_t box,
                       ConjArgs* __restrict__ conj, const int8_t* __restrict__ strat_in, int64_t nq, int64_t tauA, int64_t tauB,
                       int32_t k, int32_t chunk, int32_t tile_on, QPlan* __restrict__ plan,
                       int8_t* __restrict__ out_strat, int64_t* __restrict__ out_ids, float* __restrict__ out_dist,
                       int32_t* __restrict__ out_stats) {
  // every stride-th sorted attribute in LDS: the binary searches then touch HBM
  // only inside one stride-long window
  __shared__ int64_t samp[PLAN_SAMPLES];
  const int64_t stride = (ix.n + PLAN_SAMPLES - 1) / PLAN_SAMPLES;
  const int64_t ns = (ix.n + stride - 1) / stride;
  for (int64_t j = threadIdx.x; j < ns; j += blockDim.x) samp[j] = ix.attr[j * stride];
  __syncthreads();
  if (conj && blockIdx.x == 0 && threadIdx.x == 0)
    *conj = box ? ConjArgs{z.a2, l2, h2, z.a1, l, h, z.base1, z.base2, z.shift1, z.shift2}
                : ConjArgs{ix.attr2, l2, h2, nullptr, nullptr, nullptr, 0, 0, 0, 0};
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  int64_t lq = l[q], hq = h[q];
  if (box) {
    if (lq <= hq && l2[q] <= h2[q]) {
      const int64_t zl = zkey(zcoord(lq, z.base1, z.shift1), zcoord(l2[q], z.base2, z.shift2));
      hq = zkey(zcoord(hq, z.base1, z.shift1), zcoord(h2[q], z.base2, z.shift2));
      lq = zl;
    } else {
      lq = 1;
      hq = 0;
    }
  }
  int64_t lo = 0, hi = 0;
  if (lq <= hq) {
    // samp[a - 1] < lq <= samp[a] bounds the first attr >= lq to ((a-1) stride, a stride];
    // likewise the first attr > hq
    const int64_t a = lower_bound_i64(samp, ns, lq), b = upper_bound_i64(samp, ns, hq);
    const int64_t a0 = a > 0 ? (a - 1) * stride + 1 : 0, a1 = a < ns ? a * stride : ix.n;
    const int64_t b0 = b > 0 ? (b - 1) * stride + 1 : 0, b1 = b < ns ? b * stride : ix.n;
    lo = a0 + lower_bound_i64(ix.attr + a0, a1 - a0, lq);
    hi = b0 + upper_bound_i64(ix.attr + b0, b1 - b0, hq);
    if (hi < lo) hi = lo;
  }
  int64_t Y = hi - lo;
  int s = strat_in ? (int)strat_in[q] : UNIFY_AUTO;
  // a strategy outside AUTO..POST is not run: the row is padded and reported as
  // strategy STRAT_INVALID with status 3
  const bool bad = s < UNIFY_AUTO || s > UNIFY_POST;
  if (bad) Y = 0;
  if (s == UNIFY_AUTO) {
    if (box) {
      // box query: c of the ns sampled pairs lie in the box, an estimate of c n / ns
      // objects.  Box objects lie in [lo, hi), so only the pairs at ids
      // floor(j n / ns) in [lo, hi) -- j0 <= j < j1 -- can count.
      int64_t c = 0;
      if (Y > 0) {
        const int64_t j0 = (lo * z.ns + ix.n - 1) / ix.n, j1 = (hi * z.ns + ix.n - 1) / ix.n;
        const int64_t a1 = l[q], b1 = h[q], a2 = l2[q], b2 = h2[q];
        for (int64_t j = j0; j < j1; ++j) {
          const int64_t x = z.s1[j], y = z.s2[j];
          c += x >= a1 && x <= b1 && y >= a2 && y <= b2;
        }
      }
      const int64_t cn = c * ix.n;
      s = (Y <= tauA || cn <= tauA * z.ns) ? UNIFY_PRE : (cn >= tauB * z.ns ? UNIFY_POST : UNIFY_HYBRID);
    } else if (l2 && ix.n2s > 0) {
      // conjunctive query: the objects passing both ranges are estimated as Y times the
      // fraction c2 / n2s of the second attribute's sample inside its range
      const int64_t a2 = l2[q], b2 = h2[q];
      const int64_t c2 = a2 <= b2 ? upper_bound_i64(ix.attr2_sample, ix.n2s, b2) -
                                        lower_bound_i64(ix.attr2_sample, ix.n2s, a2)
                                  : 0;
      const int64_t yj = Y * c2;
      s = (Y <= tauA || yj <= tauA * ix.n2s) ? UNIFY_PRE : (yj >= tauB * ix.n2s ? UNIFY_POST : UNIFY_HYBRID);
    } else {
      s = Y <= tauA ? UNIFY_PRE : (Y >= tauB ? UNIFY_POST : UNIFY_HYBRID);
    }
  }
  QPlan P;
  P.lo = (int32_t)lo;
  P.hi = (int32_t)hi;
  P.a = P.b = 0;
  P.nch = 1;
  P.clen = (int32_t)Y;
  P.pbase = 0;
  P.tsb = 0;
  P.tbase = 0;
  if (Y > 0) {
    P.a = (int32_t)(upper_bound_i64(ix.seg_start, ix.S + 1, lo) - 1);
    P.b = (int32_t)(upper_bound_i64(ix.seg_start, ix.S + 1, hi - 1) - 1);
    P.strat = s;
    if (s == UNIFY_PRE && k <= PRE_SPLIT_KMAX) {
      P.nch = (int32_t)std::min<int64_t>(PRE_NCH_MAX, (Y + chunk - 1) / chunk);
      P.clen = (int32_t)((Y + P.nch - 1) / P.nch);
    }
    // a candidate for the matrix-core scan (the work list decides within its record budget)
    if (s == UNIFY_PRE && tile_on && !l2) P.tsb = (int32_t)((hi - 1) / TILE_ROWS - lo / TILE_ROWS + 1);
  } else {
    P.strat = -1;
    for (int t = 0; t < k; ++t) {
      out_ids[q * k + t] = -1;
      out_dist[q * k + t] = __builtin_inff();
    }
    if (out_stats) {
      for (int t = 0; t < 8; ++t) out_stats[q * 8 + t] = 0;
      if (bad) {
        out_stats[q * 8 + 3] = STATUS_INVALID;
        out_stats[q * 8 + 5] = STRAT_INVALID;
      }
    }
  }
  plan[q] = P;
  if (out_strat) out_strat[q] = (int8_t)(bad ? STRAT_INVALID : s);
}

// Work list, longest work first so that the persistent waves finish together:
// the hybrid searches from the smallest range up (a narrow range leaves more
// out-of-range objects to walk through), then the post-filter searches, then
// the chunks of the pre-filter scans (short and uniform) bucketed by where they
// start, so that waves scanning at the same time read nearby rows.  Also
// numbers the partial-list slots of split scans (QPlan.pbase) and resets the
// counters.  One block.
__device__ __forceinline__ int graph_bucket(const QPlan& P) {
  const int lg = 31 - __clz(max(P.hi - P.lo, 1));  // floor(log2 Y)
  return P.strat == UNIFY_HYBRID ? lg : 32 + lg;
}

__global__ void k_worklist(QPlan* __restrict__ plan, int64_t nq, int64_t n, int64_t pcap, int32_t heavy_cap,
                           int32_t* __restrict__ work, int32_t* __restrict__ wchunk,
                           int32_t* __restrict__ counters /* nwork, next, fb_count, fb_next, graph searches,
                                                             tile items, heavy, heavy next */) {
  constexpr int NB = 1024, NG = 64;
  __shared__ int32_t spart[1024];
  __shared__ int64_t tpart[1024];
  __shared__ int32_t bucket[NB];
  __shared__ int32_t gbucket[NG];
  const int t = threadIdx.x, T = blockDim.x;
  for (int b = t; b < NB; b += T) bucket[b] = 0;
  if (t < NG) gbucket[t] = 0;
  // records of the matrix-core scan: each thread's candidates in its own query order,
  // threads in order (a deterministic assignment); a query whose records would pass
  // pcap is scanned per wavefront instead
  int64_t tc = 0;
  for (int64_t q = t; q < nq; q += T) {
    const QPlan P = plan[q];
    if (P.strat == UNIFY_PRE && P.tsb > 0) tc += P.tsb;
  }
  tpart[t] = tc;
  __syncthreads();
  for (int off = 1; off < T; off <<= 1) {
    const int64_t v = t >= off ? tpart[t - off] : 0;
    __syncthreads();
    tpart[t] += v;
    __syncthreads();
  }
  int64_t tcur = tpart[t] - tc;
  int32_t sc = 0;
  for (int64_t q = t; q < nq; q += T) {  // interleaved, so that plan reads coalesce
    QPlan P = plan[q];
    if (P.strat == UNIFY_PRE && P.tsb > 0) {
      if (tcur + P.tsb <= pcap) {
        plan[q].tbase = (int32_t)tcur;
        tcur += P.tsb;
        continue;
      }
      plan[q].tsb = 0;
      P.tsb = 0;
    }
    if (P.strat == UNIFY_HYBRID || P.strat == UNIFY_POST) {
      atomicAdd(&gbucket[graph_bucket(P)], 1);
    } else if (P.strat == UNIFY_PRE) {
      for (int j = 0; j < P.nch; ++j)
        atomicAdd(&bucket[(int)((int64_t)(P.lo + j * P.clen) * NB / n)], 1);
      if (P.nch > 1) sc += P.nch;
    }
  }
  spart[t] = sc;
  __syncthreads();
  for (int off = 1; off < T; off <<= 1) {
    const int32_t sv = t >= off ? spart[t - off] : 0;
    const int32_t bv = (t >= off && t < NB) ? bucket[t - off] : 0;
    const int32_t gv = (t >= off && t < NG) ? gbucket[t - off] : 0;
    __syncthreads();
    spart[t] += sv;
    if (t < NB) bucket[t] += bv;
    if (t < NG) gbucket[t] += gv;
    __syncthreads();
  }
  const int32_t nbeam = gbucket[NG - 1];
  const int32_t nchunks = bucket[NB - 1];
  const int32_t my_end = t < NB ? bucket[t] : 0;  // inclusive prefix count of chunks
  __syncthreads();
  if (t < NB) bucket[t] = nbeam + my_end;  // one past the last slot of bucket t
  __syncthreads();
  int32_t spos = spart[t] - sc;
  for (int64_t q = t; q < nq; q += T) {
    QPlan P = plan[q];
    if (P.strat == UNIFY_HYBRID || P.strat == UNIFY_POST) {
      const int32_t w = atomicSub(&gbucket[graph_bucket(P)], 1) - 1;
      work[w] = (int32_t)q;
      wchunk[w] = 0;
    } else if (P.strat == UNIFY_PRE && P.tsb == 0) {
      for (int j = 0; j < P.nch; ++j) {
        const int b = (int)((int64_t)(P.lo + j * P.clen) * NB / n);
        const int32_t w = atomicSub(&bucket[b], 1) - 1;
        work[w] = (int32_t)q;
        wchunk[w] = j;
      }
      if (P.nch > 1) {
        plan[q].pbase = spos;
        spos += P.nch;
      }
    }
  }
  if (t == 0) {
    // the first heavy_cap graph searches (the narrowest hybrid ranges first) go to the
    // cooperative kernel; the one-wavefront kernel starts after them
    const int32_t nheavy = min(nbeam, heavy_cap);
    counters[0] = nbeam + nchunks;
    counters[1] = nheavy;
    counters[2] = 0;
    counters[3] = 0;
    counters[4] = nbeam;
    counters[6] = nheavy;
    counters[7] = 0;
  }
}

__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// ---------------------------------------------------------------------------
// Vector loads: 4 consecutive elements of row v, group g, as FP32.
// ---------------------------------------------------------------------------
// Raw rows of each store: the words a lane loads for one 4-element group, kept
// packed in registers until the distance is computed, so a wave can hold more
// rows in flight the narrower the store is.
template <int PREC>
struct Store;

template <>
struct Store<UNIFY_FP32> {
  typedef float4 Raw;
  static constexpr int WORDS = 4;
  __device__ static Raw load(const DevIndex& ix, int64_t v, int g) {
    return *reinterpret_cast<const float4*>(ix.vec + v * ix.d + 4 * g);
  }
  __device__ static float scale(const DevIndex&, int64_t) { return 1.0f; }
  __device__ static float4 decode(Raw r, float) { return r; }
};

template <>
struct Store<UNIFY_BF16> {
  typedef uint2 Raw;
  static constexpr int WORDS = 2;
  __device__ static Raw load(const DevIndex& ix, int64_t v, int g) {
    return *reinterpret_cast<const uint2*>(ix.vec_bf16 + v * ix.d + 4 * g);
  }
  __device__ static float scale(const DevIndex&, int64_t) { return 1.0f; }
  __device__ static float4 decode(Raw w, float) {
    return make_float4(bf16_to_f32(w.x & 0xFFFFu), __uint_as_float(w.x & 0xFFFF0000u), bf16_to_f32(w.y & 0xFFFFu),
                       __uint_as_float(w.y & 0xFFFF0000u));
  }
};

template <>
struct Store<UNIFY_FP8E4M3> {
  typedef uint32_t Raw;
  static constexpr int WORDS = 1;
  __device__ static Raw load(const DevIndex& ix, int64_t v, int g) {
    return *reinterpret_cast<const uint32_t*>(ix.vec_fp8 + v * ix.d + 4 * g);
  }
  __device__ static float scale(const DevIndex& ix, int64_t v) { return ix.vec_scale[v]; }
  // gfx950's packed conversion decodes OCP E4M3 exactly (the same values as
  // e4m3_to_f32); each value is then scaled as fp8_value does.
  __device__ static float4 decode(Raw w, float sc) {
    const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, false);
    const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, true);
    return make_float4(__builtin_fmaf(lo[0], sc, 0.0f), __builtin_fmaf(lo[1], sc, 0.0f),
                       __builtin_fmaf(hi[0], sc, 0.0f), __builtin_fmaf(hi[1], sc, 0.0f));
  }
};

// Keys (canonical FP32 distance, id) of cnt vectors of the store PREC: four
// vectors per round (16 lanes each, lane s takes groups s, s + 16, ...), RB
// rounds of raw loads in flight; the i-th vector is id_of(i) and its key lands
// in keys[i] (LDS).  Depth: GRAPH evaluations use RB = 16 / NG rounds (at most
// 8: 32 rows in flight at d <= 128; wider rows keep fewer, since the query
// itself then holds NG * 4 registers; BF16 at most BF16_ROUNDS, for its
// register budget); STREAM (the pre-filter scans, whose loop holds little else)
// keeps 16 / NG for every store; SHALLOW (2 rounds at most) serves the FP32
// re-scores inside low-precision kernels, whose registers would otherwise add
// to the hot path's and spill.
enum EvalDepth { GRAPH = 0, SHALLOW = 1, STREAM = 2 };

template <int NG, int PREC, int DEPTH = GRAPH, class IdOf>
__device__ __forceinline__ void eval_keys(const DevIndex& ix, const float4 (&qv)[NG], int cnt, IdOf id_of,
                                          u64* keys) {
  typedef Store<PREC> St;
  constexpr int RB0 = (DEPTH == SHALLOW ? 2 : 16) / NG;
  constexpr int RBMAX = (PREC == UNIFY_BF16 && DEPTH == GRAPH) ? BF16_ROUNDS : 8;
  constexpr int RB = RB0 < 1 ? 1 : (RB0 > RBMAX ? RBMAX : RB0);
  const int G = ix.d >> 2;
  const int lane = lane_id();
  const int s = lane & 15, g4 = lane >> 4;
  for (int base = 0; base < cnt; base += 4 * RB) {
    typename St::Raw x[RB][NG];
    float sc[RB];
    int32_t vid[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int idx = base + 4 * r + g4;
      vid[r] = idx < cnt ? id_of(idx) : -1;
      sc[r] = vid[r] >= 0 ? St::scale(ix, vid[r]) : 1.0f;
#pragma unroll
      for (int i = 0; i < NG; ++i) {
        const int g = s + 16 * i;
        x[r][i] = (vid[r] >= 0 && g < G) ? St::load(ix, (int64_t)vid[r], g) : typename St::Raw{};
      }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      float acc = 0.0f;
#pragma unroll
      for (int i = 0; i < NG; ++i) {
        if (s + 16 * i < G) acc = fma_sq4(St::decode(x[r][i], sc[r]), qv[i], acc);
      }
      acc = group_reduce16(acc);
      const int idx = base + 4 * r + g4;
      if (s == 0 && idx < cnt) keys[idx] = make_key(acc, vid[r]);
    }
  }
}

// ---------------------------------------------------------------------------
// Per-wave LDS state
// ---------------------------------------------------------------------------
struct Lds {
  u64* ann;
  u64* cand;
  uint32_t* hash;
  u64* bkeys;  // neighbour ids (low 32 bits) before evaluation, their keys after
  u64* sel;    // selection S1: the ranked list (sel_cap - 64 entries), then 64 scratch keys
};

// Visited set of one layer search, decided per id.  An 8-way set-associative
// cache of ids in LDS holds an id while its set has room (a set never loses an
// entry within a layer search, so a miss in a set with room proves the id new);
// an id whose set is full is decided by its bit in the wave's (workgroup's) HBM
// visited row: an atomic OR sets it, and the bit's old value says whether the id
// was visited.  Each id thus lives in exactly one of the two, and concurrent
// lanes (or wavefronts) claim it exactly once through the LDS compare-and-swap
// or the OR.  A row is a bitmap of n bits, all clear between layer searches,
// followed by a log of the bitmap words the layer search made non-zero, which it
// clears at its end (the whole bitmap if the log overflowed).  Only this wave
// (workgroup) uses its row; workgroup-scope fences order its own stores and loads.
constexpr int VWAYS = 8;
constexpr int VLOG_CAP = 8192;  // logged words per row

struct VRow {
  uint32_t* bits;  // [bwords]
  uint32_t* log;   // [VLOG_CAP]
};
__device__ __forceinline__ VRow vrow_of(const SearchArgs& A, int64_t slot) {
  uint32_t* r = A.vrows + slot * A.vstride;
  return VRow{r, r + A.bwords};
}

__device__ __forceinline__ uint32_t* cache_set(uint32_t* cache, int setbits, int32_t v) {
  const uint32_t set = ((uint32_t)v * 2654435761u) >> (32 - setbits);
  return cache + set * VWAYS;
}

__device__ __forceinline__ bool cache_hit(const uint32_t* base, int32_t v) {
  const uint4 a = *reinterpret_cast<const uint4*>(base);
  const uint4 b = *reinterpret_cast<const uint4*>(base + 4);
  const uint32_t u = (uint32_t)v;
  return a.x == u || a.y == u || a.z == u || a.w == u || b.x == u || b.y == u || b.z == u || b.w == u;
}

// Local mode: true when v is new; `full` when it could not be recorded.  Lanes
// holding the same id in one batch race through the same ways: one inserts it,
// the others find it in the way they tried and report it visited.
__device__ __forceinline__ bool visit_local(uint32_t* cache, int setbits, int32_t v, bool& full) {
  uint32_t* base = cache_set(cache, setbits, v);
  if (cache_hit(base, v)) return false;
#pragma unroll
  for (int w = 0; w < VWAYS; ++w) {
    const uint32_t old = atomicCAS(base + w, HASH_EMPTY, (uint32_t)v);
    if (old == HASH_EMPTY) return true;
    if (old == (uint32_t)v) return false;
  }
  full = true;
  return true;
}

// Sets v's bit in the bitmap: true when it was clear.  `fresh`: the word was
// zero before (exactly one lane of those that set bits in it sees that), so its
// index belongs in the log.
__device__ __forceinline__ bool mark_bit(uint32_t* bits, int32_t v, bool& fresh) {
  const uint32_t m = 1u << ((uint32_t)v & 31u);
  const uint32_t old =
      __hip_atomic_fetch_or(bits + ((uint32_t)v >> 5), m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  fresh = old == 0u;
  return (old & m) == 0u;
}

// True when v is new.  `spill`: v's set was full and the row decided; `fresh`: the
// row's word was zero before (its index belongs in the log).
__device__ __forceinline__ bool visit(uint32_t* cache, int setbits, uint32_t* bits, int32_t v, bool& spill,
                                      bool& fresh) {
  bool full = false;
  fresh = false;
  const bool isnew = visit_local(cache, setbits, v, full);
  spill = full;
  return full ? mark_bit(bits, v, fresh) : isnew;
}

// Appends the words that `fresh` lanes made non-zero to the log (one wavefront;
// nlog counts past VLOG_CAP once it overflows).
__device__ __forceinline__ void log_words(const VRow& R, int& nlog, bool fresh, int32_t v) {
  const u64 fm = ballot(fresh);
  if (fresh) {
    const int i = nlog + rank_in(fm);
    if (i < VLOG_CAP) R.log[i] = (uint32_t)v >> 5;
  }
  nlog += __popcll(fm);
}

// Leaves the bitmap all clear again: the logged words, or every word when the
// log overflowed.  Thread t of nt; the caller orders these stores before the
// row's next use.
__device__ __forceinline__ void clear_row(const VRow& R, int nlog, int64_t bwords, int t, int nt) {
  if (nlog <= VLOG_CAP) {
    for (int i = t; i < nlog; i += nt) R.bits[R.log[i]] = 0u;
  } else {
    for (int64_t i = t; i < bwords; i += nt) R.bits[i] = 0u;
  }
}

__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Orders one wavefront's LDS writes before its later reads by other lanes, in a
// block of several independent wavefronts (no block barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The LDS sync of code one wavefront runs: a block barrier where the block is that
// wavefront (WS = false), a wavefront-level one where other wavefronts of the block
// run other code (WS = true).
template <bool WS>
__device__ __forceinline__ void lsync() {
  if constexpr (WS) wave_lds_sync();
  else __syncthreads();
}

struct Counters {
  int32_t ndist = 0, nexp = 0, nrerank = 0, nadj = 0;
  int32_t spill = 0;  // a layer search decided some ids in its HBM bitmap row (a cache set was full)
  int32_t coop = 0;   // the query ran as a cooperative (several-wavefront) search
};
constexpr int32_t STAT_SPILL_BIT = 0x100;  // status counter flag: the visited set spilled to HBM
constexpr int32_t STAT_COOP_BIT = 0x200;   // status counter flag: a cooperative search

// One layer of the search (Alg. 1 / Alg. 7 with beam width p).  On return, the
// ann list holds `al` keys ascending.  Returns false on capacity overflow.
template <int NG, int PREC, bool S1 = false>
__device__ bool layer_search(const SearchArgs& A, const Lds& L, const float4 (&qv)[NG], const QPlan& P,
                             Sec sec, bool hybrid, bool filter, int c, int32_t ep, u64 ep_key, int layer, int efl,
                             int p, int& al, Counters& cnt, const VRow& R) {
  const DevIndex& ix = A.ix;
  const int lane = lane_id();
  int hbits = 0;
  while ((1 << hbits) < A.hcap) ++hbits;
  int nlog = 0;  // words logged in R
  for (int i = lane; i < A.hcap; i += WAVE) L.hash[i] = HASH_EMPTY;
  __syncthreads();
  const int setbits = hbits - 3;  // hcap / VWAYS sets
  bool spilled = false;  // some id was decided by the HBM row
  bool overflow = false;
  if (lane == 0) L.hash[(cache_set(L.hash, setbits, ep) - L.hash)] = (uint32_t)ep;
  // cand = {ep}; ann = {ep} unless filtered out
  if (lane == 0) L.cand[0] = ep_key;
  int cl = 1;
  const bool ep_in = !filter || (ep >= P.lo && ep < P.hi && sec_ok(A, sec, ep));
  L.ann[lane] = (ep_in && lane == 0) ? ep_key : KEY_MAX;
  al = ep_in ? 1 : 0;
  __syncthreads();

  const int mc = layer == 0 ? ix.M0 : ix.MU;
  const int Sa = P.b - P.a + 1;
  const int per_node = hybrid ? Sa * min(c, mc) : ix.GC;
  const int64_t max_steps = ix.n + 2;
  int64_t steps = 0;
  int32_t popped[8];

  while (true) {
    if (++steps > max_steps) {
      overflow = true;
      break;
    }
    const bool full = al == efl;
    const u64 T = full ? L.ann[efl - 1] : KEY_MAX;
    // pop up to p candidates that pass the stopping test
    int npop = 0;
    for (int t = 0; t < p; ++t) {
      u64 best = KEY_MAX;
      int bidx = -1;
      for (int i = lane; i < cl; i += WAVE) {
        u64 kk = L.cand[i];
        if (kk < best) {
          best = kk;
          bidx = i;
        }
      }
      const u64 mn = wave_min64(best);
      if (mn == KEY_MAX || (full && mn > T)) break;
      const u64 who = ballot(best == mn);
      const int src = __ffsll((unsigned long long)who) - 1;
      const int idx = __shfl(bidx, src, WAVE);
      if (lane == src) L.cand[idx] = KEY_MAX;
      popped[t] = key_id(mn);
      ++npop;
      __syncthreads();
    }
    if (npop == 0) break;
    cnt.nexp += npop;
    cnt.nadj += npop * ((S1 && hybrid) ? Sa * mc : per_node);
    // unvisited neighbours of the popped candidates.  The adjacency entries of
    // all popped objects are loaded first (GB loads of 64 entries in flight per
    // wave) into the neighbour buffer, densely, so a step waits for one round
    // trip; the visited checks then compact the buffer in place.
    int nn = 0;
    int64_t rowbase = 0;  // lane t < npop: first entry of popped[t]'s row
    if (lane < npop) {
      int32_t o = popped[0];
      for (int t = 1; t < npop; ++t)
        if (lane == t) o = popped[t];
      const int64_t r = layer == 0 ? (int64_t)o : (int64_t)ix.uprow[o] + layer - 1;
      rowbase = r * (hybrid ? (int64_t)ix.S * mc : (int64_t)ix.GC);
    }
    const int32_t* table = hybrid ? (layer == 0 ? ix.adj0 : ix.adjU) : (layer == 0 ? ix.glist0 : ix.glistU);
    const int cc = min(c, mc);
    int ntot = npop * per_node;
    constexpr int GB = 8;
    if constexpr (S1) {
      if (hybrid) {
        // selection S1: each popped object's entries in the active chunks, ranked by
        // the distance to that object (its row stands in for the query); the m nearest
        ntot = 0;
        const int etot = Sa * mc, mk = A.m;
        u64* slist = L.sel;
        u64* stmp = L.sel + A.sel_cap - WAVE;
        for (int t = 0; t < npop; ++t) {
          const int32_t o = popped[t];
          const int64_t rb = (int64_t)shfl64((u64)rowbase, t);
          float4 qo[NG];
          {
            const int s = lane & 15, G = ix.d >> 2;
            const float sc = Store<PREC>::scale(ix, o);
#pragma unroll
            for (int i = 0; i < NG; ++i) {
              const int g = s + 16 * i;
              qo[i] = g < G ? Store<PREC>::decode(Store<PREC>::load(ix, o, g), sc) : make_float4(0.f, 0.f, 0.f, 0.f);
            }
          }
          int sl = 0;
          for (int i = lane; i < A.sel_cap - WAVE; i += WAVE) slist[i] = KEY_MAX;
          __syncthreads();
          for (int e0 = 0; e0 < etot; e0 += WAVE) {
            const int e = e0 + lane;
            const int32_t u = e < etot ? table[rb + (int64_t)(P.a + e / mc) * mc + e % mc] : -1;
            const u64 um = ballot(u >= 0);
            const int cu = __popcll(um);
            if (cu == 0) continue;
            if (u >= 0) stmp[rank_in(um)] = (uint32_t)u;
            __syncthreads();
            eval_keys<NG, PREC>(ix, qo, cu, [&](int i) { return key_id(stmp[i]); }, stmp);
            __syncthreads();
            const u64 key = lane < cu ? stmp[lane] : KEY_MAX;
            const u64 Tm = sl == mk ? slist[mk - 1] : KEY_MAX;
            list_insert(slist, sl, mk, key < Tm ? key : KEY_MAX);
            __syncthreads();
          }
          for (int i = lane; i < sl; i += WAVE) L.bkeys[ntot + i] = (u64)(uint32_t)key_id(slist[i]);
          ntot += sl;
          __syncthreads();
        }
      }
    }
    for (int e0 = 0; e0 < ntot && !(S1 && hybrid); e0 += GB * WAVE) {
      int32_t vv[GB];
#pragma unroll
      for (int u = 0; u < GB; ++u) {
        const int e = e0 + u * WAVE + lane;
        const int t = e / per_node, tt = e - t * per_node;
        const int64_t rb = (int64_t)shfl64((u64)rowbase, min(t, WAVE - 1));
        vv[u] = e < ntot ? (hybrid ? table[rb + (int64_t)(P.a + tt / cc) * mc + tt % cc] : table[rb + tt]) : -1;
      }
#pragma unroll
      for (int u = 0; u < GB; ++u) {
        const int e = e0 + u * WAVE + lane;
        if (e < ntot) L.bkeys[e] = (u64)(uint32_t)vv[u];
      }
    }
    __syncthreads();
    // the visited checks of up to TB blocks of entries are issued together, so a step waits
    // for one round of atomics on the visited row instead of one per block (which lane of
    // a batch claims a repeated id does not matter: the evaluated keys are admitted against
    // the pre-step threshold and kept in key order).  4 blocks in the BF16 kernel, 2 in the
    // FP32 one; the FP8 kernel, and every kernel for rows wider than 256 elements (whose
    // query alone holds 4 NG registers), have none to spare and take one at a time.
    constexpr int TB = NG > 4 ? 1 : (PREC == UNIFY_BF16 ? 4 : (PREC == UNIFY_FP32 ? 2 : 1));
    for (int b0 = 0; b0 < ntot; b0 += TB * WAVE) {
      int32_t vv[TB];
      bool isn[TB];
#pragma unroll
      for (int u = 0; u < TB; ++u) {
        const int e = b0 + u * WAVE + lane;
        vv[u] = e < ntot ? (int32_t)(uint32_t)L.bkeys[e] : -1;
      }
      __syncthreads();  // these blocks are read before new ids are written over them
#pragma unroll
      for (int u = 0; u < TB; ++u) {
        bool sp = false, fresh = false;
        isn[u] = vv[u] >= 0 && visit(L.hash, setbits, R.bits, vv[u], sp, fresh);
        spilled |= __any(sp);
        log_words(R, nlog, fresh, vv[u]);
      }
#pragma unroll
      for (int u = 0; u < TB; ++u) {
        const u64 nm = ballot(isn[u]);
        if (isn[u]) L.bkeys[nn + rank_in(nm)] = (uint32_t)vv[u];
        nn += __popcll(nm);
      }
    }
    if (nn == 0) continue;
    __syncthreads();
    cnt.ndist += nn;
    eval_keys<NG, PREC>(ix, qv, nn, [&](int i) { return key_id(L.bkeys[i]); }, L.bkeys);
    __syncthreads();
    // admission against the threshold from before this step
    for (int base = 0; base < nn; base += WAVE) {
      const int tt = base + lane;
      const u64 key = tt < nn ? L.bkeys[tt] : KEY_MAX;
      const bool adm = key != KEY_MAX && key < T;
      const u64 am = ballot(adm);
      const int na = __popcll(am);
      if (na == 0) continue;
      if (cl + na > A.ccap) {
        // compact: drop tombstones and keys that can no longer be expanded
        const u64 W = al == efl ? L.ann[efl - 1] : KEY_MAX;
        int ncl = 0;
        for (int i0 = 0; i0 < cl; i0 += WAVE) {
          const int i = i0 + lane;
          const u64 kk = i < cl ? L.cand[i] : KEY_MAX;
          const bool keep = kk != KEY_MAX && kk <= W;
          const u64 km = ballot(keep);
          __syncthreads();
          if (keep) L.cand[ncl + rank_in(km)] = kk;
          ncl += __popcll(km);
          __syncthreads();
        }
        cl = ncl;
        if (cl + na > A.ccap) {
          overflow = true;
          break;
        }
      }
      if (adm) L.cand[cl + rank_in(am)] = key;
      cl += na;
      const int32_t id = key_id(key);
      const bool in_r = adm && (!filter || (id >= P.lo && id < P.hi && sec_ok(A, sec, id)));
      list_insert(L.ann, al, efl, in_r ? key : KEY_MAX);
      __syncthreads();
    }
    if (overflow) break;
  }
  if (spilled) {
    cnt.spill = 1;
    wave_fence();  // the log's stores before their loads
    clear_row(R, nlog, A.bwords, lane, WAVE);
    wave_fence();  // the clears before the row's next atomics
  }
  return !__any(overflow);
}

// The pre-filter scan of a box query steps over the runs of its key range that lie
// outside the box: from id i (inside the slice, below hi), the first id not before i
// whose key can lie in the box -- i itself when its cell is in the box's cells, else
// the first key at or above the next box key after i's (hi when there is none).  Cells
// in the box hold every box object; wave-uniform.  Not inlined: its registers stay out
// of the search kernels' budgets.
__device__ __attribute__((noinline)) int32_t box_next(const SearchArgs& A, Sec s, int32_t i, int32_t hi) {
  const ConjArgs c = *A.conj;
  const uint64_t z = static_cast<uint64_t>(A.ix.attr[i]);
  const uint64_t x = zcompact(z >> 1), y = zcompact(z);
  const uint64_t x0 = zcoord(c.l1[s.q], c.zb1, c.zs1), x1 = zcoord(c.h1[s.q], c.zb1, c.zs1);
  const uint64_t y0 = zcoord(c.l2[s.q], c.zb2, c.zs2), y1 = zcoord(c.h2[s.q], c.zb2, c.zs2);
  if (x >= x0 && x <= x1 && y >= y0 && y <= y1) return i;
  const int64_t nz = znext(z, static_cast<uint64_t>(zkey(x0, y0)), static_cast<uint64_t>(zkey(x1, y1)));
  if (nz < 0) return hi;
  return i + 1 + (int32_t)lower_bound_i64(A.ix.attr + i + 1, hi - i - 1, nz);
}

// Strategy A: exact top-k over the id slice [lo, hi) (FP32 store; PREC names
// the kernel's ranking store, for which this is the fallback when it is not FP32).
template <int NG, int PREC>
__device__ void pre_scan(const SearchArgs& A, const Lds& L, const float4 (&qv)[NG], const QPlan& P,
                         Sec sec, int& al, Counters& cnt) {
  const int lane = lane_id();
  const int k = A.k;
  al = 0;
  for (int blk = 0; blk * WAVE < k; ++blk) L.ann[blk * WAVE + lane] = KEY_MAX;
  __syncthreads();
  for (int base = P.lo; base < P.hi; base += WAVE) {
    const int cntv = min(WAVE, P.hi - base);
    eval_keys<NG, UNIFY_FP32, (PREC != UNIFY_FP32 ? SHALLOW : STREAM)>(A.ix, qv, cntv,
                                                                      [&](int i) { return base + i; }, L.bkeys);
    __syncthreads();
    const u64 key = lane < cntv && sec_ok(A, sec, base + lane) ? L.bkeys[lane] : KEY_MAX;
    const u64 T = al == k ? L.ann[k - 1] : KEY_MAX;
    list_insert(L.ann, al, k, key < T ? key : KEY_MAX);
    __syncthreads();
  }
  cnt.ndist += P.hi - P.lo;
}

// Strategy A for a conjunctive query: the slice's second attributes are tested
// first, and the objects that pass are gathered (up to a wavefront's worth) and
// scored with the FP32 distance.
template <int NG, int PREC, bool SKIP>
__device__ void pre_scan_multi(const SearchArgs& A, const Lds& L, const float4 (&qv)[NG], const QPlan& P, Sec sec,
                               int& al, Counters& cnt) {
  const int lane = lane_id();
  const int k = A.k;
  al = 0;
  for (int blk = 0; blk * WAVE < k; ++blk) L.ann[blk * WAVE + lane] = KEY_MAX;
  __syncthreads();
  const bool box = SKIP && A.conj->attr1 != nullptr;
  int base = box && P.lo < P.hi ? box_next(A, sec, P.lo, P.hi) : P.lo;
  while (true) {
    // gather up to a wavefront's worth of passing ids into L.bkeys
    int nb = 0;
    while (base < P.hi) {
      const int32_t v = base + lane;
      const bool pass = v < P.hi && sec_ok(A, sec, v);
      const u64 pm = ballot(pass);
      const int c = __popcll(pm);
      if (nb + c > WAVE) break;  // this block starts the next batch
      if (pass) L.bkeys[nb + rank_in(pm)] = (uint32_t)v;
      nb += c;
      base += WAVE;
      if (box && base < P.hi) base = box_next(A, sec, base, P.hi);
    }
    if (nb == 0) break;
    __syncthreads();
    eval_keys<NG, UNIFY_FP32, (PREC != UNIFY_FP32 ? SHALLOW : STREAM)>(
        A.ix, qv, nb, [&](int i) { return key_id(L.bkeys[i]); }, L.bkeys);
    __syncthreads();
    const u64 key = lane < nb ? L.bkeys[lane] : KEY_MAX;
    const u64 T = al == k ? L.ann[k - 1] : KEY_MAX;
    list_insert(L.ann, al, k, key < T ? key : KEY_MAX);
    __syncthreads();
    cnt.ndist += nb;
  }
}

// Bounds on sqrt(s), s = the canonical FP32 distance of an object, from st =
// the same distance to its low-precision copy c, with ||c - x|| <= eps.  Both
// distances carry a relative error of at most g (all terms are non-negative),
// so with rho = ||x - q|| and rho~ = ||c - q||:
//   sqrt(s) in rho [sqrt(1-g), sqrt(1+g)],  rho in [rho~ - eps, rho~ + eps],
//   rho~ in sqrt(st) [1/sqrt(1+g), 1/sqrt(1-g)],
// hence sqrt(s) >= sqrt(st) A - eps B and sqrt(s) <= sqrt(st) C + eps D with
// A = sqrt((1-g)/(1+g)), B = sqrt(1-g), C = sqrt((1+g)/(1-g)), D = sqrt(1+g).
// The host widens A, B, C, D by 2^-20 relative, far more than the few FP32
// roundings below (each <= 2^-24; sqrtf within 2^-23), and 1e-18 covers
// underflow; a negative lower bound is clamped to 0.
__device__ __forceinline__ void root_bounds(float st, float eps, const SearchArgs& A, float& lb, float& ub) {
  const float r = __builtin_sqrtf(st);
  const float l = __builtin_fmaf(r, A.bA, -__builtin_fmaf(eps, A.bB, 1e-18f));
  lb = l > 0.0f ? l : 0.0f;  // never -0: keys order non-negative floats by their bits
  ub = __builtin_fmaf(r, A.bC, __builtin_fmaf(eps, A.bD, 1e-18f));
}

// Strategy A over a BF16 / FP8 copy, with the exact FP32 result.  Every object
// of the slice gets bounds [lb, ub] on the root of its FP32 distance from the
// copy's distance.  The k smallest ub are kept (ann); any object in the exact
// top k has lb <= sqrt(s) <= sqrt(k-th smallest s) <= (k-th smallest ub), so
// the objects whose lb is at most the current k-th smallest ub contain the
// exact top k.  They are appended to cand (unsorted; when it fills, entries
// above the current threshold are dropped), and the survivors of the final
// threshold are re-scored in FP32.  Returns false when cand cannot hold the
// qualifying objects (the caller then runs the FP32 scan).
template <int NG, int PREC>
__device__ bool pre_scan_lowp(const SearchArgs& A, const Lds& L, const float4 (&qv)[NG], const QPlan& P, int& al,
                              Counters& cnt) {
  const DevIndex& ix = A.ix;
  const int lane = lane_id();
  const int k = A.k;
  int ul = 0, cl = 0;
  for (int blk = 0; blk * WAVE < k; ++blk) L.ann[blk * WAVE + lane] = KEY_MAX;
  __syncthreads();
  for (int base = P.lo; base < P.hi; base += WAVE) {
    const int cntv = min(WAVE, P.hi - base);
    eval_keys<NG, PREC, STREAM>(ix, qv, cntv, [&](int i) { return base + i; }, L.bkeys);
    __syncthreads();
    cnt.ndist += cntv;
    float lb = 0.f, ub = 0.f;
    const bool have = lane < cntv;
    if (have) root_bounds(key_dist(L.bkeys[lane]), ix.vec_eps[base + lane], A, lb, ub);
    const int32_t v = base + lane;
    const u64 uk = have ? make_key(ub, v) : KEY_MAX;
    const u64 TU0 = ul == k ? L.ann[k - 1] : KEY_MAX;
    list_insert(L.ann, ul, k, uk < TU0 ? uk : KEY_MAX);
    __syncthreads();
    const float TU = ul == k ? key_dist(L.ann[k - 1]) : __builtin_inff();
    const bool adm = have && lb <= TU;
    const u64 am = ballot(adm);
    const int add = __popcll(am);
    if (cl + add > A.ccap) {
      // drop the entries the threshold has passed since they were appended
      int wpos = 0;
      for (int b0 = 0; b0 < cl; b0 += WAVE) {
        const int t = b0 + lane;
        const u64 e = t < cl ? L.cand[t] : KEY_MAX;
        const bool keep = t < cl && key_dist(e) <= TU;
        const u64 km = ballot(keep);
        __syncthreads();  // this block is read before any lane overwrites it
        if (keep) L.cand[wpos + rank_in(km)] = e;
        wpos += __popcll(km);
      }
      cl = wpos;
      __syncthreads();
      if (cl + add > A.ccap) return false;
    }
    if (adm) L.cand[cl + rank_in(am)] = make_key(lb, v);
    cl += add;
    __syncthreads();
  }
  const float TU = ul == k ? key_dist(L.ann[k - 1]) : __builtin_inff();
  // re-score the qualifying entries of cand in FP32
  al = 0;
  for (int blk = 0; blk * WAVE < k; ++blk) L.ann[blk * WAVE + lane] = KEY_MAX;
  __syncthreads();
  for (int base = 0; base < cl; base += WAVE) {
    const int t = base + lane;
    const bool use = t < cl && key_dist(L.cand[t]) <= TU;
    const u64 um = ballot(use);
    const int nb = __popcll(um);
    if (nb == 0) continue;
    const int32_t v = use ? key_id(L.cand[t]) : 0;
    __syncthreads();
    if (use) L.bkeys[rank_in(um)] = (uint32_t)v;
    __syncthreads();
    eval_keys<NG, UNIFY_FP32, SHALLOW>(ix, qv, nb, [&](int i) { return key_id(L.bkeys[i]); }, L.bkeys);
    __syncthreads();
    const u64 key = lane < nb ? L.bkeys[lane] : KEY_MAX;
    const u64 T = al == k ? L.ann[k - 1] : KEY_MAX;
    list_insert(L.ann, al, k, key < T ? key : KEY_MAX);
    __syncthreads();
    cnt.nrerank += nb;
  }
  return true;
}

// Graph search results over a BF16 / FP8 copy: the first rerank * k in-range
// entries of ann (ascending by the copy's distance) are re-scored with the FP32
// distance into a sorted list of k in L.cand.  Returns that list's length.
template <int NG, bool WS = false>
__device__ int rerank_graph(const SearchArgs& A, const Lds& L, const float4 (&qv)[NG], const QPlan& P,
                            Sec sec, int al, bool post, Counters& cnt) {
  const int lane = lane_id();
  const int k = A.k;
  const int R = A.rerank * k;
  int rl = 0, taken = 0;
  for (int blk = 0; blk * WAVE < k; ++blk) L.cand[blk * WAVE + lane] = KEY_MAX;
  lsync<WS>();
  for (int base = 0; base < al && taken < R; base += WAVE) {
    const int t = base + lane;
    const u64 key = t < al ? L.ann[t] : KEY_MAX;
    const int32_t id = key_id(key);
    bool keep = key != KEY_MAX && (!post || (id >= P.lo && id < P.hi && sec_ok(A, sec, id)));
    const u64 km = ballot(keep);
    keep = keep && taken + rank_in(km) < R;
    const u64 um = ballot(keep);
    const int nb = __popcll(um);
    if (nb == 0) continue;
    lsync<WS>();
    if (keep) L.bkeys[rank_in(um)] = (uint32_t)id;
    lsync<WS>();
    eval_keys<NG, UNIFY_FP32, SHALLOW>(A.ix, qv, nb, [&](int i) { return key_id(L.bkeys[i]); }, L.bkeys);
    lsync<WS>();
    const u64 nk = lane < nb ? L.bkeys[lane] : KEY_MAX;
    const u64 T = rl == k ? L.cand[k - 1] : KEY_MAX;
    list_insert(L.cand, rl, k, nk < T ? nk : KEY_MAX);
    lsync<WS>();
    taken += nb;
    cnt.nrerank += nb;
  }
  return rl;
}

// A pre-filter scan split into chunks: each chunk's wavefront stores its exact
// top-k list (ascending, KEY_MAX padded) and adds its counters; k_pre_merge,
// launched after the search kernel, merges the lists (the union of the chunks'
// top-k lists holds the slice's top k).
__device__ void pre_store_chunk(const SearchArgs& A, const Lds& L, int32_t q, const QPlan& P, int chunk, int al,
                                const Counters& cnt, bool fell) {
  const int lane = lane_id();
  const int k = A.k;
  u64* mine = A.part + ((int64_t)P.pbase + chunk) * k;
  for (int t = lane; t < k; t += WAVE) mine[t] = t < al ? L.ann[t] : KEY_MAX;
  if (lane == 0) {
    int32_t* acc = A.qacc + (int64_t)q * 4;
    atomicAdd(acc + 1, cnt.nrerank);
    atomicAdd(acc + 2, cnt.ndist);
    if (fell) atomicAdd(acc + 3, 1);
  }
}

// Outputs of one query (one wavefront): hybrid / pre take the first k; post keeps
// in-range entries in order.  Graph results over a low-precision copy come
// re-scored and filtered.
template <int NG, int PREC, bool WS = false>
__device__ void write_result(const SearchArgs& A, const Lds& L, const float4 (&qv)[NG], const QPlan& P, Sec sec,
                             int32_t q, int al, bool ok, int status, bool hybrid, Counters& cnt) {
  const DevIndex& ix = A.ix;
  const int lane = lane_id();
  const int kout = A.k;
  const u64* res = L.ann;
  bool post_filter = P.strat == UNIFY_POST;
  if (PREC != UNIFY_FP32 && P.strat != UNIFY_PRE && ok && al > 0) {
    al = rerank_graph<NG, WS>(A, L, qv, P, sec, al, post_filter, cnt);
    res = L.cand;
    post_filter = false;
  }
  int written = 0;
  for (int base = 0; base < al && written < kout; base += WAVE) {
    const int t = base + lane;
    const u64 key = t < al ? res[t] : KEY_MAX;
    const int32_t id = key_id(key);
    const bool keep = key != KEY_MAX && (!post_filter || (id >= P.lo && id < P.hi && sec_ok(A, sec, id)));
    const u64 km = ballot(keep);
    const int pos = written + rank_in(km);
    if (keep && pos < kout) {
      A.out_ids[(int64_t)q * kout + pos] = ix.ext[id];
      A.out_dist[(int64_t)q * kout + pos] = key_dist(key);
    }
    written += __popcll(km);
  }
  written = min(written, kout);
  if (!ok) written = 0;
  for (int t = written + lane; t < kout; t += WAVE) {
    A.out_ids[(int64_t)q * kout + t] = -1;
    A.out_dist[(int64_t)q * kout + t] = __builtin_inff();
  }
  if (A.out_stats && lane == 0) {
    int32_t* st = A.out_stats + (int64_t)q * 8;
    st[0] = cnt.ndist;
    st[1] = cnt.nexp;
    st[2] = cnt.nrerank;
    st[3] = (ok ? status : 2) | (cnt.spill ? STAT_SPILL_BIT : 0) | (cnt.coop ? STAT_COOP_BIT : 0);
    st[4] = cnt.nadj;
    st[5] = P.strat;
    st[6] = P.hi - P.lo;
    st[7] = hybrid ? P.b - P.a + 1 : 0;
  }
}


__device__ __forceinline__ bool ne_missing(int top) { return top < 0; }

template <int NG, int PREC, bool S1 = false>
__device__ void run_query(const SearchArgs& A, const Lds& L, int32_t q, int chunk, const VRow& R) {
  const DevIndex& ix = A.ix;
  const int lane = lane_id();
  const QPlan P = A.plan[q];
  const Sec sec{q};
  float4 qv[NG];
  {
    const int s = lane & 15, G = ix.d >> 2;
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      const int g = s + 16 * i;
      qv[i] = g < G ? *reinterpret_cast<const float4*>(A.Q + (int64_t)q * ix.d + 4 * g)
                    : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  Counters cnt;
  int al = 0;
  bool ok = true;
  const bool hybrid = P.strat == UNIFY_HYBRID;
  int status = A.pass;
  if (P.strat == UNIFY_PRE) {
    QPlan Pc = P;  // this chunk of the slice
    Pc.lo = P.lo + chunk * P.clen;
    Pc.hi = min(P.hi, Pc.lo + P.clen);
    // a low-precision scan whose bounds cannot settle its top k is redone in FP32
    // conjunctive queries: the gathering scan where the kernel's registers absorb a
    // second scan loop; elsewhere the plain scan (one call site) scores every object
    // and drops those failing the second test
    constexpr bool GATHER = NG <= 4 && PREC != UNIFY_FP8E4M3;
    bool fell = false;
    if (GATHER && A.conj) {
      // (the S1 kernels, at the edge of their register budget, scan box slices whole)
      pre_scan_multi<NG, PREC, !S1>(A, L, qv, Pc, sec, al, cnt);
    } else if (PREC == UNIFY_FP32 || A.conj || !pre_scan_lowp<NG, PREC>(A, L, qv, Pc, al, cnt)) {
      fell = PREC != UNIFY_FP32 && !A.conj;
      pre_scan<NG, PREC>(A, L, qv, Pc, sec, al, cnt);
    }
    if (P.nch > 1) {
      pre_store_chunk(A, L, q, P, chunk, al, cnt, fell);
      return;
    }
    if (fell) status = 1;
  } else {
    const int Sa = P.b - P.a + 1;
    const int c = (A.m + Sa - 1) / Sa;
    int32_t ep;
    int top;
    u64 ep_key;
    if (hybrid) {
      // entry of the active segment with the highest top level; ties: nearer, then smaller id
      top = -1;
      for (int j = P.a; j <= P.b; ++j)
        if (ix.seg_entry[j] >= 0) top = max(top, ix.seg_maxlevel[j]);
      int ne = 0;
      for (int j0 = P.a; j0 <= P.b; j0 += WAVE) {
        const int j = j0 + lane;
        const bool is = j <= P.b && ix.seg_entry[j] >= 0 && ix.seg_maxlevel[j] == top;
        const u64 mk = ballot(is);
        if (is) L.bkeys[ne + rank_in(mk)] = (uint32_t)ix.seg_entry[j];
        ne += __popcll(mk);
      }
      __syncthreads();
      eval_keys<NG, PREC>(ix, qv, ne, [&](int i) { return key_id(L.bkeys[i]); }, L.bkeys);
      __syncthreads();
      cnt.ndist += ne;
      const u64 kk = lane < ne ? L.bkeys[lane] : KEY_MAX;
      ep_key = wave_min64(kk);
      ep = key_id(ep_key);
      __syncthreads();
      if (ne == 0) {  // no entry among the active segments: nothing to search
        top = -1;
        ok = false;
      }
    } else {
      top = ix.L;
      ep = ix.gentry;
      L.bkeys[0] = (uint32_t)ep;
      __syncthreads();
      eval_keys<NG, PREC>(ix, qv, 1, [&](int i) { return key_id(L.bkeys[i]); }, L.bkeys);
      __syncthreads();
      ep_key = L.bkeys[0];
      cnt.ndist += 1;
      __syncthreads();
    }
    for (int layer = top; layer >= 1 && ok; --layer) {
      ok = layer_search<NG, PREC, S1>(A, L, qv, P, sec, hybrid, false, c, ep, ep_key, layer, 1, 1, al, cnt, R);
      ep_key = L.ann[0];
      ep = key_id(ep_key);
      __syncthreads();
    }
    if (ok)
      ok = layer_search<NG, PREC, S1>(A, L, qv, P, sec, hybrid, hybrid, c, ep, ep_key, 0, A.ef, A.p, al, cnt, R);
    if (ne_missing(top)) {
      al = 0;
      ok = true;
    }
  }
  if (!ok) {
    if (A.pass == 0) {
      if (lane == 0) {
        const int32_t slot = atomicAdd(A.fb_count, 1);
        A.fb_list[slot] = q;
      }
      return;
    }
  }
  write_result<NG, PREC>(A, L, qv, P, sec, q, al, ok, status, hybrid, cnt);
}

// ---------------------------------------------------------------------------
// Cooperative graph search: MW wavefronts of one workgroup run one query.  The
// longest searches of a batch (the hybrid searches of the narrowest ranges, at
// the head of the work list) bound a step; spreading each step's adjacency
// gather, visited checks and distance evaluations over MW wavefronts shortens
// them.  Wavefront 0 pops the candidates and admits the evaluated keys by the
// rule of the one-wavefront search (so the same ann list results); the visited
// set is the workgroup's LDS cache, shared by its wavefronts, with the HBM row for
// ids whose cache set is full, so whichever wavefront meets an id first claims it
// by one compare-and-swap in LDS (or one atomic OR on the row).  Three workgroup
// barriers per step.
// ---------------------------------------------------------------------------
struct LdsMW {
  u64* ann;
  u64* cand;
  uint32_t* hash;
  u64* bkeys;   // entry and result stages (wavefront 0)
  u64* nbuf;    // per wavefront: its new ids, then their keys
  int32_t* sh;  // broadcast slots
};
enum { SH_NPOP = 8, SH_POPPED = 9 /* 8 slots */, SH_CL = 17, SH_AL = 18, SH_OVER = 19, SH_EP = 20, SH_TOP = 21,
       SH_W = 22, SH_EPKEY = 24 /* 2 slots */, SH_NLOG = 26, SH_SPILL = 27, SH_SLOTS = 28 };

// LDS bytes of a cooperative search's workgroup (besides the broadcast slots).
__host__ __device__ inline size_t lds_bytes_mw(int ef_blocks, int ccap, int hcap, int nbr_cap, int mw) {
  return sizeof(u64) * ((size_t)ef_blocks * WAVE + ccap + nbr_cap + nbr_cap + (size_t)mw * WAVE) +
         sizeof(uint32_t) * hcap;
}

template <int NG, int PREC, int MW>
__device__ bool layer_search_mw(const SearchArgs& A, const LdsMW& L, const float4 (&qv)[NG], const QPlan& P,
                                Sec sec, bool hybrid, bool filter, int c, int32_t ep, u64 ep_key, int layer,
                                int efl, int p, int& al, Counters& cnt, const VRow& R) {
  const DevIndex& ix = A.ix;
  const int lane = lane_id();
  const int wv = threadIdx.x >> 6, tid = threadIdx.x;
  constexpr int NT = 64 * MW;
  int hbits = 0;
  while ((1 << hbits) < A.hcap) ++hbits;
  const int setbits = hbits - 3;
  for (int i = tid; i < A.hcap; i += NT) L.hash[i] = HASH_EMPTY;
  __syncthreads();
  if (tid == 0) {
    L.sh[SH_NLOG] = 0;
    L.sh[SH_SPILL] = 0;
    L.hash[cache_set(L.hash, setbits, ep) - L.hash] = (uint32_t)ep;
    L.cand[0] = ep_key;
  }
  int cl = 1;
  const bool ep_in = !filter || (ep >= P.lo && ep < P.hi && sec_ok(A, sec, ep));
  if (wv == 0) L.ann[lane] = (ep_in && lane == 0) ? ep_key : KEY_MAX;
  al = ep_in ? 1 : 0;
  bool overflow = false;
  __syncthreads();

  const int mc = layer == 0 ? ix.M0 : ix.MU;
  const int Sa = P.b - P.a + 1;
  const int per_node = hybrid ? Sa * min(c, mc) : ix.GC;
  const int cc = min(c, mc);
  const int32_t* table = hybrid ? (layer == 0 ? ix.adj0 : ix.adjU) : (layer == 0 ? ix.glist0 : ix.glistU);
  const int64_t max_steps = ix.n + 2;
  int64_t steps = 0;
  while (true) {
    if (++steps > max_steps) {
      overflow = true;
      break;
    }
    const bool full = al == efl;
    const u64 T = full ? L.ann[efl - 1] : KEY_MAX;
    // wavefront 0 pops up to p candidates that pass the stopping test
    if (wv == 0) {
      int npop = 0;
      for (int t = 0; t < p; ++t) {
        u64 best = KEY_MAX;
        int bidx = -1;
        for (int i = lane; i < cl; i += WAVE) {
          const u64 kk = L.cand[i];
          if (kk < best) {
            best = kk;
            bidx = i;
          }
        }
        const u64 mn = wave_min64(best);
        if (mn == KEY_MAX || (full && mn > T)) break;
        const u64 who = ballot(best == mn);
        const int src = __ffsll((unsigned long long)who) - 1;
        const int idx = __shfl(bidx, src, WAVE);
        if (lane == src) L.cand[idx] = KEY_MAX;
        if (lane == 0) L.sh[SH_POPPED + t] = key_id(mn);
        ++npop;
        wave_lds_sync();
      }
      if (lane == 0) L.sh[SH_NPOP] = npop;
    }
    __syncthreads();
    const int npop = L.sh[SH_NPOP];
    if (npop == 0) break;
    cnt.nexp += npop;
    cnt.nadj += npop * per_node;
    // this wavefront's share of the entries, [e0, e1); its new ids go to nbuf[e0 ..]
    const int ntot = npop * per_node;
    const int share = (ntot + MW * WAVE - 1) / (MW * WAVE) * WAVE;
    const int e0 = wv * share, e1 = min(ntot, e0 + share);
    int64_t rowbase = 0;  // lane t < npop: first entry of popped[t]'s row
    if (lane < npop) {
      const int32_t o = L.sh[SH_POPPED + lane];
      const int64_t r = layer == 0 ? (int64_t)o : (int64_t)ix.uprow[o] + layer - 1;
      rowbase = r * (hybrid ? (int64_t)ix.S * mc : (int64_t)ix.GC);
    }
    u64* mine = L.nbuf + e0;
    int nnw = 0;
    constexpr int GB = 8;
    for (int b0 = e0; b0 < e1; b0 += GB * WAVE) {
      int32_t vv[GB];
#pragma unroll
      for (int u = 0; u < GB; ++u) {
        const int e = b0 + u * WAVE + lane;
        const int t = e / per_node, tt = e - t * per_node;
        const int64_t rb = (int64_t)shfl64((u64)rowbase, min(t, WAVE - 1));
        vv[u] = e < e1 ? (hybrid ? table[rb + (int64_t)(P.a + tt / cc) * mc + tt % cc] : table[rb + tt]) : -1;
      }
#pragma unroll
      for (int u = 0; u < GB; ++u) {
        const int32_t v = vv[u];
        bool sp = false, fresh = false;
        const bool isnew = v >= 0 && visit(L.hash, setbits, R.bits, v, sp, fresh);
        const bool anysp = __any(sp);
        if (lane == 0 && anysp) L.sh[SH_SPILL] = 1;
        // the words this wavefront made non-zero go to the shared log
        const u64 fm = ballot(fresh);
        if (fm) {
          int b = 0;
          if (lane == 0) b = atomicAdd(&L.sh[SH_NLOG], __popcll(fm));
          b = __shfl(b, 0, WAVE);
          const int i = b + rank_in(fm);
          if (fresh && i < VLOG_CAP) R.log[i] = (uint32_t)v >> 5;
        }
        const u64 nm = ballot(isnew);
        if (isnew) mine[nnw + rank_in(nm)] = (uint32_t)v;
        nnw += __popcll(nm);
      }
    }
    wave_lds_sync();
    if (nnw > 0) eval_keys<NG, PREC>(ix, qv, nnw, [&](int i) { return key_id(mine[i]); }, mine);
    if (lane == 0) L.sh[wv] = nnw;
    __syncthreads();
    // wavefront 0 admits every wavefront's keys against the threshold from before this step
    if (wv == 0) {
      for (int w2 = 0; w2 < MW && !overflow; ++w2) {
        const int nn = L.sh[w2];
        cnt.ndist += nn;
        const u64* theirs = L.nbuf + w2 * share;
        for (int base = 0; base < nn; base += WAVE) {
          const int tt = base + lane;
          const u64 key = tt < nn ? theirs[tt] : KEY_MAX;
          const bool adm = key != KEY_MAX && key < T;
          const u64 am = ballot(adm);
          const int na = __popcll(am);
          if (na == 0) continue;
          if (cl + na > A.ccap) {
            // compact: drop tombstones and keys that can no longer be expanded
            const u64 W = al == efl ? L.ann[efl - 1] : KEY_MAX;
            int ncl = 0;
            for (int i0 = 0; i0 < cl; i0 += WAVE) {
              const int i = i0 + lane;
              const u64 kk = i < cl ? L.cand[i] : KEY_MAX;
              const bool keep = kk != KEY_MAX && kk <= W;
              const u64 km = ballot(keep);
              wave_lds_sync();
              if (keep) L.cand[ncl + rank_in(km)] = kk;
              ncl += __popcll(km);
              wave_lds_sync();
            }
            cl = ncl;
            if (cl + na > A.ccap) {
              overflow = true;
              break;
            }
          }
          if (adm) L.cand[cl + rank_in(am)] = key;
          cl += na;
          const int32_t id = key_id(key);
          const bool in_r = adm && (!filter || (id >= P.lo && id < P.hi && sec_ok(A, sec, id)));
          list_insert(L.ann, al, efl, in_r ? key : KEY_MAX);
          wave_lds_sync();
        }
      }
      if (lane == 0) {
        L.sh[SH_CL] = cl;
        L.sh[SH_AL] = al;
        L.sh[SH_OVER] = overflow ? 1 : 0;
      }
    }
    __syncthreads();
    if (wv != 0) {
      cl = L.sh[SH_CL];
      al = L.sh[SH_AL];
      overflow = L.sh[SH_OVER] != 0;
    }
    if (overflow) break;
  }
  __syncthreads();  // every wavefront's bits and log entries before the clear
  if (L.sh[SH_SPILL]) {
    cnt.spill = 1;
    clear_row(R, L.sh[SH_NLOG], A.bwords, tid, NT);
  }
  __syncthreads();  // the clears before the row's next use
  return !overflow;
}

template <int NG, int PREC, int MW>
__device__ void run_query_mw(const SearchArgs& A, const LdsMW& L, int32_t q, const VRow& R) {
  const DevIndex& ix = A.ix;
  const int lane = lane_id(), wv = threadIdx.x >> 6;
  const QPlan P = A.plan[q];
  const Sec sec{q};
  float4 qv[NG];
  {
    const int s = lane & 15, G = ix.d >> 2;
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      const int g = s + 16 * i;
      qv[i] = g < G ? *reinterpret_cast<const float4*>(A.Q + (int64_t)q * ix.d + 4 * g)
                    : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  Counters cnt;
  cnt.coop = 1;
  int al = 0;
  const bool hybrid = P.strat == UNIFY_HYBRID;
  const int Sa = P.b - P.a + 1;
  const int c = (A.m + Sa - 1) / Sa;
  // entry (wavefront 0): for the hybrid search the entry of the active segment with the
  // highest top level (ties: nearer, then smaller id), else the global entry
  if (wv == 0) {
    int32_t ep = -1;
    int top = -1;
    u64 ep_key = KEY_MAX;
    if (hybrid) {
      for (int j = P.a; j <= P.b; ++j)
        if (ix.seg_entry[j] >= 0) top = max(top, ix.seg_maxlevel[j]);
      int ne = 0;
      for (int j0 = P.a; j0 <= P.b; j0 += WAVE) {
        const int j = j0 + lane;
        const bool is = j <= P.b && ix.seg_entry[j] >= 0 && ix.seg_maxlevel[j] == top;
        const u64 mk = ballot(is);
        if (is) L.bkeys[ne + rank_in(mk)] = (uint32_t)ix.seg_entry[j];
        ne += __popcll(mk);
      }
      wave_lds_sync();
      eval_keys<NG, PREC>(ix, qv, ne, [&](int i) { return key_id(L.bkeys[i]); }, L.bkeys);
      wave_lds_sync();
      cnt.ndist += ne;
      const u64 kk = lane < ne ? L.bkeys[lane] : KEY_MAX;
      ep_key = wave_min64(kk);
      ep = key_id(ep_key);
      if (ne == 0) top = -1;
    } else {
      top = ix.L;
      ep = ix.gentry;
      L.bkeys[0] = (uint32_t)ep;
      wave_lds_sync();
      eval_keys<NG, PREC>(ix, qv, 1, [&](int i) { return key_id(L.bkeys[i]); }, L.bkeys);
      wave_lds_sync();
      ep_key = L.bkeys[0];
      cnt.ndist += 1;
    }
    if (lane == 0) {
      L.sh[SH_EP] = ep;
      L.sh[SH_TOP] = top;
      L.sh[SH_EPKEY] = (int32_t)(uint32_t)ep_key;
      L.sh[SH_EPKEY + 1] = (int32_t)(uint32_t)(ep_key >> 32);
    }
  }
  __syncthreads();
  int32_t ep = L.sh[SH_EP];
  const int top = L.sh[SH_TOP];
  u64 ep_key = ((u64)(uint32_t)L.sh[SH_EPKEY + 1] << 32) | (uint32_t)L.sh[SH_EPKEY];
  __syncthreads();
  bool ok = true;
  for (int layer = top; layer >= 1 && ok; --layer) {
    ok = layer_search_mw<NG, PREC, MW>(A, L, qv, P, sec, hybrid, false, c, ep, ep_key, layer, 1, 1, al, cnt, R);
    ep_key = L.ann[0];
    ep = key_id(ep_key);
    __syncthreads();
  }
  if (ok && top >= 0)
    ok = layer_search_mw<NG, PREC, MW>(A, L, qv, P, sec, hybrid, hybrid, c, ep, ep_key, 0, A.ef, A.p, al, cnt, R);
  if (top < 0) {  // no entry among the active segments: nothing to search
    al = 0;
    ok = true;
  }
  if (!ok && A.pass == 0) {
    if (threadIdx.x == 0) {
      const int32_t slot = atomicAdd(A.fb_count, 1);
      A.fb_list[slot] = q;
    }
    return;
  }
  if (wv == 0) {
    Lds Lw;
    Lw.ann = L.ann;
    Lw.cand = L.cand;
    Lw.hash = L.hash;
    Lw.bkeys = L.bkeys;
    Lw.sel = nullptr;
    write_result<NG, PREC, true>(A, Lw, qv, P, sec, q, al, ok, A.pass, hybrid, cnt);
  }
}

// Persistent cooperative searches: first the heavy queries (the head of the work
// list, work[0, nheavy)), then queries of the shared remainder, with the
// one-wavefront kernel.  Workgroup g owns visited row mw_row0 + g.
template <int NG, int PREC, int MW>
__global__ void __launch_bounds__(64 * MW) k_search_mw(SearchArgs A) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ int32_t sh[SH_SLOTS];
  LdsMW L;
  unsigned char* p = lds_raw;
  L.ann = reinterpret_cast<u64*>(p);
  p += sizeof(u64) * A.ef_blocks * WAVE;
  L.cand = reinterpret_cast<u64*>(p);
  p += sizeof(u64) * A.ccap;
  L.bkeys = reinterpret_cast<u64*>(p);
  p += sizeof(u64) * A.nbr_cap;
  L.nbuf = reinterpret_cast<u64*>(p);
  p += sizeof(u64) * (A.nbr_cap + MW * WAVE);
  L.hash = reinterpret_cast<uint32_t*>(p);
  L.sh = sh;
  const int32_t nwork = *A.nwork, nheavy = *A.nheavy, nbeam = *A.nbeam;
  const VRow R = vrow_of(A, A.mw_row0 + blockIdx.x);  // the workgroup's visited row
  bool heavy = true;  // thread 0's view
  while (true) {
    if (threadIdx.x == 0) {
      int32_t w = nwork;
      if (heavy) {
        w = atomicAdd(A.mw_next, 1);
        if (w >= nheavy) heavy = false;
      }
      if (!heavy) {
        // a graph search of the shared remainder, never a pre-filter chunk (those follow the
        // graph searches in the work list and are the one-wavefront kernel's)
        w = nwork;
        int32_t cur = __hip_atomic_load(A.next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        while (cur < nbeam) {
          const int32_t seen = atomicCAS(A.next, cur, cur + 1);
          if (seen == cur) {
            w = cur;
            break;
          }
          cur = seen;
        }
      }
      sh[SH_W] = w;
    }
    __syncthreads();
    const int32_t w = sh[SH_W];
    __syncthreads();
    if (w >= nwork) break;
    run_query_mw<NG, PREC, MW>(A, L, A.work[w], R);
    __syncthreads();
  }
}

template <int NG, int PREC, int PASS, bool S1 = false>
__global__ void __launch_bounds__(64, NG > 4 ? 1 : (PREC == UNIFY_FP32 ? WAVES_PER_SIMD_FP32 : WAVES_PER_SIMD_LOW)) k_search(SearchArgs A) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  Lds L;
  unsigned char* p = lds_raw;
  L.ann = reinterpret_cast<u64*>(p);
  p += sizeof(u64) * A.ef_blocks * WAVE;
  L.cand = reinterpret_cast<u64*>(p);
  p += sizeof(u64) * A.ccap;
  L.bkeys = reinterpret_cast<u64*>(p);
  p += sizeof(u64) * A.nbr_cap;
  L.sel = reinterpret_cast<u64*>(p);  // S1 only (sel_cap = 0 otherwise)
  p += sizeof(u64) * A.sel_cap;
  L.hash = reinterpret_cast<uint32_t*>(p);
  const int32_t nwork = *A.nwork;
  const VRow R = vrow_of(A, blockIdx.x);  // this wave's visited row
  while (true) {
    int32_t w = 0;
    if (lane_id() == 0) w = atomicAdd(A.next, 1);
    w = __shfl(w, 0, WAVE);
    if (w >= nwork) break;
    run_query<NG, PREC, S1>(A, L, A.work[w], A.wchunk ? A.wchunk[w] : 0, R);
    __syncthreads();
  }
}

// Outputs of the split pre-filter scans: one wavefront per query merges its
// chunks' top-k lists (k <= PRE_SPLIT_KMAX) and writes the k results and the counters.
__global__ void __launch_bounds__(256) k_pre_merge(DevIndex ix, const QPlan* __restrict__ plan, int64_t nq, int k,
                                                   const u64* __restrict__ part, const int32_t* __restrict__ qacc,
                                                   int64_t* __restrict__ out_ids, float* __restrict__ out_dist,
                                                   int32_t* __restrict__ out_stats) {
  __shared__ u64 lists[4][PRE_SPLIT_KMAX];
  const int lane = lane_id();
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= nq) return;  // uniform per wavefront
  const QPlan P = plan[q];
  if (P.strat != UNIFY_PRE || P.nch <= 1 || P.tsb > 0) return;  // tsb > 0: the matrix-core scan answers it
  u64* lst = lists[threadIdx.x >> 6];
  for (int t = lane; t < PRE_SPLIT_KMAX; t += WAVE) lst[t] = KEY_MAX;
  int al = 0;
  const u64* all = part + (int64_t)P.pbase * k;
  const int tot = P.nch * k;
  for (int base = 0; base < tot; base += WAVE) {
    const int t = base + lane;
    const u64 key = t < tot ? all[t] : KEY_MAX;
    const u64 T = al == k ? lst[k - 1] : KEY_MAX;
    list_insert(lst, al, k, key < T ? key : KEY_MAX);
  }
  for (int t = lane; t < k; t += WAVE) {
    const u64 key = t < al ? lst[t] : KEY_MAX;
    out_ids[q * k + t] = key != KEY_MAX ? ix.ext[key_id(key)] : -1;
    out_dist[q * k + t] = key != KEY_MAX ? key_dist(key) : __builtin_inff();
  }
  if (out_stats && lane == 0) {
    int32_t* st = out_stats + q * 8;
    st[0] = qacc[q * 4 + 2];
    st[1] = 0;
    st[2] = qacc[q * 4 + 1];
    st[3] = qacc[q * 4 + 3] > 0 ? 1 : 0;
    st[4] = 0;
    st[5] = UNIFY_PRE;
    st[6] = P.hi - P.lo;
    st[7] = 0;
  }
}

// ---------------------------------------------------------------------------
// Strategy A on the matrix cores.  The pre-filter queries of a batch share the
// attribute-sorted store: a super-block of TILE_ROWS consecutive objects is read
// once for up to 16 of the queries whose slices touch it, and the distance of
// every (query, object) pair is formed by the norm expansion
//   s~ = ||x~||^2 - 2 q . x~ + ||q||^2
// with the products q . x~ on MFMA (BF16 inputs for the BF16 and FP8 stores, the
// query split into two BF16 parts; FP32 inputs for the FP32 store), accumulated
// in FP32.  s~ only selects: with a bound E on its error, eps_v on the copy's
// error and the relative error g of the canonical FP32 distance, every object
// gets [lb, ub] around the root of its canonical distance.  Within a
// super-block the objects with lb <= min(k-th smallest ub of the block, the
// smallest such value any block of the query has published) are recorded; the
// k-th smallest ub over a query's records is the k-th smallest over its slice
// (each of those k objects is recorded by its block), and every object of the
// exact top k has lb <= that value.  k_tile_final re-scores the recorded
// objects below it with the canonical FP32 distance, so the result is exactly
// the FP32 scan's.  A query whose records overflow is scanned in FP32 instead.
// ---------------------------------------------------------------------------

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

struct TileArgs {
  DevIndex ix;
  const QPlan* plan;
  const float* Q;
  int64_t nq;
  int32_t k, kcq;
  uint32_t* qhl;        // [nq][d] BF16 split of each query: high part | low part << 16
  float4* qinfo;        // [nq] (||q||^2, ||q||, bound on ||q - (hi + lo)||, 0)
  uint32_t* tglob;      // [nq] smallest published block threshold (FP32 bits)
  int32_t* cnt_sb;      // [nsb] queries per super-block, then the fill cursor
  int32_t* fill_sb;     // [nsb]
  int32_t* off_sb;      // [nsb + 1] first list entry of each super-block
  int32_t* ioff;        // [nsb + 1] first work item of each super-block
  int32_t* list;        // [pcap] queries of each super-block
  int32_t* item_sb;     // [pcap] super-block of each work item
  int32_t* rec_cnt;     // [pcap] objects recorded per (query, super-block), kcq + 1 = overflow
  u64* rec_key;         // [pcap][kcq] (lb bits << 32) | id
  float* rec_ub;        // [pcap][kcq] ub of the same object
  int32_t* counters;    // [6]: work items of the scan
  int64_t nsb;
  float cE, bA, bB, bC, bD;
};

// Queries of the matrix-core scan: the BF16 split, norms and error bound of each
// query, its threshold, and the count of queries per super-block.
__global__ void __launch_bounds__(256) k_tile_prep(TileArgs T) {
  const int lane = threadIdx.x & 63;
  const int64_t q = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (q >= T.nq) return;  // uniform per wavefront
  const QPlan P = T.plan[q];
  if (P.strat != UNIFY_PRE || P.tsb == 0) return;
  const int sb0 = P.lo / TILE_ROWS;
  for (int j = lane; j < P.tsb; j += WAVE) atomicAdd(&T.cnt_sb[sb0 + j], 1);
  const int d = T.ix.d;
  const float* qq = T.Q + q * d;
  float n2 = 0.0f, e2 = 0.0f;
  for (int t = lane; t < d; t += WAVE) {
    const float x = qq[t];
    n2 = __builtin_fmaf(x, x, n2);
    if (T.ix.precision != UNIFY_FP32) {
      // q = hi + lo + res, each step exact: a value minus its nearest BF16 is exact in FP32
      const uint32_t hi = f32_to_bf16(x);
      const float r = x - bf16_to_f32(hi);
      const uint32_t lo = f32_to_bf16(r);
      const float res = r - bf16_to_f32(lo);
      T.qhl[q * d + t] = hi | (lo << 16);
      e2 = __builtin_fmaf(res, res, e2);
    }
  }
  for (int o = 32; o >= 1; o >>= 1) {
    n2 += __shfl_xor(n2, o, WAVE);
    e2 += __shfl_xor(e2, o, WAVE);
  }
  if (lane == 0) {
    // the sum of squares passes through at most d / 64 + 7 roundings: 2^-18 covers them
    const float eq = T.ix.precision == UNIFY_FP32 ? 0.0f : __builtin_sqrtf(e2) * (1.0f + 0x1p-18f) + 1e-21f;
    T.qinfo[q] = make_float4(n2, __builtin_sqrtf(n2), eq, 0.0f);
    T.tglob[q] = 0x7F800000u;  // +inf
  }
}

// Offsets of the super-blocks' query lists and of their work items (one item =
// one super-block and up to TILE_Q of its queries).  One workgroup of NW wavefronts
// (beside the graph search, one for indexes up to a million objects, where a single
// wavefront starts soonest, up to 16 for larger ones; 16 when it runs alone): wavefront w takes a
// contiguous range of super-blocks, finds the list entries and items before it from
// the other wavefronts' totals, and walks its range 64 super-blocks per round, their
// counts scanned across the lanes, 8 rounds' counts loaded ahead.
__global__ void __launch_bounds__(1024) k_tile_index(TileArgs T) {
  __shared__ int32_t wa[16], wi[16];
  const int lane = lane_id(), w = threadIdx.x >> 6, NW = blockDim.x >> 6;
  const int64_t per = ((T.nsb + NW - 1) / NW + WAVE - 1) / WAVE * WAVE;
  const int64_t b0 = std::min<int64_t>(T.nsb, w * per), b1 = std::min<int64_t>(T.nsb, b0 + per);
  int32_t pa = 0, pi = 0;  // list entries and work items before the current round (wave-uniform)
  if (NW > 1) {
    int32_t ta = 0, ti = 0;
    for (int64_t b = b0 + lane; b < b1; b += WAVE) {
      const int32_t c = T.cnt_sb[b];
      ta += c;
      ti += (c + TILE_Q - 1) / TILE_Q;
    }
    for (int o = 32; o >= 1; o >>= 1) {
      ta += __shfl_xor(ta, o, WAVE);
      ti += __shfl_xor(ti, o, WAVE);
    }
    if (lane == 0) {
      wa[w] = ta;
      wi[w] = ti;
    }
    __syncthreads();
    for (int j = 0; j < w; ++j) {
      pa += wa[j];
      pi += wi[j];
    }
  }
  constexpr int R = 8;
  for (int64_t base = b0; base < b1; base += R * WAVE) {
    int32_t c[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t b = base + r * WAVE + lane;
      c[r] = b < b1 ? T.cnt_sb[b] : 0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t b = base + r * WAVE + lane;
      const int32_t ni = (c[r] + TILE_Q - 1) / TILE_Q;
      int32_t sa = c[r], si = ni;  // inclusive prefix sums over the lanes
      for (int o = 1; o < WAVE; o <<= 1) {
        const int32_t va = __shfl_up(sa, o, WAVE), vi = __shfl_up(si, o, WAVE);
        if (lane >= o) {
          sa += va;
          si += vi;
        }
      }
      if (b < b1) {
        const int32_t oi = pi + si - ni;
        T.off_sb[b] = pa + sa - c[r];
        T.ioff[b] = oi;
        T.fill_sb[b] = 0;
        for (int j = 0; j < ni; ++j) T.item_sb[oi + j] = (int32_t)b;
      }
      pa += __shfl(sa, WAVE - 1, WAVE);
      pi += __shfl(si, WAVE - 1, WAVE);
    }
  }
  // the last wavefront's range ends at nsb: its running totals are the grand totals
  if (w == NW - 1 && lane == 0) {
    T.off_sb[T.nsb] = pa;
    T.ioff[T.nsb] = pi;
    T.counters[5] = pi;
  }
}

// Every query of the matrix-core scan joins the list of each super-block it touches.
__global__ void __launch_bounds__(256) k_tile_fill(TileArgs T) {
  const int lane = threadIdx.x & 63;
  const int64_t q = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (q >= T.nq) return;
  const QPlan P = T.plan[q];
  if (P.strat != UNIFY_PRE || P.tsb == 0) return;
  const int sb0 = P.lo / TILE_ROWS;
  for (int j = lane; j < P.tsb; j += WAVE) {
    const int b = sb0 + j;
    T.list[T.off_sb[b] + atomicAdd(&T.fill_sb[b], 1)] = (int32_t)q;
  }
}

// k-th smallest (1-based, k <= count of values below +inf) of the 4 values per
// lane, as FP32 bits (non-negative values order as their bits): the largest x
// with fewer than k values below it, built from the top bit down.
__device__ __forceinline__ uint32_t kth_smallest4(const uint32_t (&u)[4], int k) {
  uint32_t pre = 0;
  for (int bit = 30; bit >= 0; --bit) {
    const uint32_t c = pre | (1u << bit);
    int below = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) below += __popcll(ballot(u[i] < c));
    if (below < k) pre = c;
  }
  return pre;
}

// One workgroup of 4 wavefronts per work item; PREC = the store in use.
// Wavefront w contracts the item's queries with rows 64 w .. 64 w + 63 of the
// super-block and selects for queries w, w + 4, ...  LDS: the queries as MFMA
// A operands, then lb / ub of every (query, object) of the super-block.
constexpr int TILE_WAVES = 4;
template <int PREC, bool ALONE>
__global__ void __launch_bounds__(64 * TILE_WAVES, ALONE ? 1 : 4) k_tile_scan(TileArgs T) {
  // k-steps of loads in flight: beside the graph search 1 (BF16) or 2 keep a wavefront
  // within 128 registers, so it fits where one search wavefront has left a SIMD; run
  // alone (before the graph search), 4 hide more latency
  constexpr int KPF = ALONE ? 4 : (PREC == UNIFY_BF16 ? 1 : 2);
  extern __shared__ __align__(16) unsigned char tile_lds[];
  const int lane = lane_id(), wv = threadIdx.x >> 6, tid = threadIdx.x;
  constexpr int NT = 64 * TILE_WAVES;
  const int d = T.ix.d;
  const int stride = d + 8;  // padded row (elements) of the staged queries
  // A operands: BF16 stores: hi and lo parts, u16 [TILE_Q][stride] each; FP32: f32 [TILE_Q][stride]
  uint16_t* ahi = reinterpret_cast<uint16_t*>(tile_lds);
  uint16_t* alo = ahi + TILE_Q * stride;
  float* af = reinterpret_cast<float*>(tile_lds);
  float* LB = reinterpret_cast<float*>(tile_lds + (size_t)TILE_Q * stride * 4);
  float* UB = LB + TILE_Q * TILE_ROWS;
  __shared__ int32_t s_q[TILE_Q], s_lo[TILE_Q], s_hi[TILE_Q], s_pair[TILE_Q];
  __shared__ float4 s_info[TILE_Q];
  const int nitems = T.counters[5];
  const int n = (int)T.ix.n;
  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
    const int sb = T.item_sb[item];
    const int g = item - T.ioff[sb];
    const int qb = T.off_sb[sb] + g * TILE_Q;
    const int nqg = min(TILE_Q, T.off_sb[sb + 1] - qb);
    if (tid < TILE_Q) {
      if (tid < nqg) {
        const int32_t q = T.list[qb + tid];
        const QPlan P = T.plan[q];
        s_q[tid] = q;
        s_lo[tid] = P.lo;
        s_hi[tid] = P.hi;
        s_pair[tid] = P.tbase + (sb - P.lo / TILE_ROWS);
        s_info[tid] = T.qinfo[q];
      } else {
        s_q[tid] = -1;
        s_lo[tid] = s_hi[tid] = 0;
      }
    }
    for (int idx = tid; idx < TILE_Q * TILE_ROWS; idx += NT) {
      LB[idx] = __builtin_inff();
      UB[idx] = __builtin_inff();
    }
    __syncthreads();
    // stage the queries, 4 elements per load (zero rows beyond nqg)
    {
      constexpr int MAXV = TILE_Q * TILE_DMAX / 4 / NT;  // loads per thread at most
      const int nvec = TILE_Q * d / 4;
      uint4 wv4[MAXV];
#pragma unroll
      for (int j = 0; j < MAXV; ++j) {
        const int v = tid + j * NT;
        const int m = v / (d / 4), t4 = v - m * (d / 4);
        const int q = v < nvec ? s_q[m] : -1;
        if constexpr (PREC == UNIFY_FP32)
          wv4[j] = q >= 0 ? *reinterpret_cast<const uint4*>(T.Q + (int64_t)q * d + 4 * t4) : make_uint4(0, 0, 0, 0);
        else
          wv4[j] = q >= 0 ? *reinterpret_cast<const uint4*>(T.qhl + (int64_t)q * d + 4 * t4) : make_uint4(0, 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < MAXV; ++j) {
        const int v = tid + j * NT;
        if (v >= nvec) break;
        const int m = v / (d / 4), t = 4 * (v - m * (d / 4));
        if constexpr (PREC == UNIFY_FP32) {
          *reinterpret_cast<uint4*>(af + m * stride + t) = wv4[j];
        } else {
          const uint4 w = wv4[j];
          *reinterpret_cast<uint2*>(ahi + m * stride + t) =
              make_uint2((w.x & 0xFFFFu) | (w.y << 16), (w.z & 0xFFFFu) | (w.w << 16));
          *reinterpret_cast<uint2*>(alo + m * stride + t) =
              make_uint2((w.x >> 16) | (w.y & 0xFFFF0000u), (w.z >> 16) | (w.w & 0xFFFF0000u));
        }
      }
    }
    __syncthreads();
    const int mrow = lane & 15, kq = lane >> 4;  // MFMA lane roles: row / column, k quarter
    {
      const int r0 = sb * TILE_ROWS + wv * 64;
      bool cover = false;
      if (lane < nqg) cover = s_lo[lane] < r0 + 64 && s_hi[lane] > r0;
      if (r0 < n && __any(cover)) {
        f32x4_t acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        if constexpr (PREC == UNIFY_FP32) {
          // 16x16x4 FP32 MFMA: a k-step of 16 elements = 4 instructions; lane (n, kq) holds
          // elements 16 s + 4 kq .. + 3 of object n and of query n (as the A row).  Loads of
          // KPF k-steps are issued before their products.
          for (int s0 = 0; s0 < d / 16; s0 += KPF) {
            float4 x[KPF][4];
#pragma unroll
            for (int ss = 0; ss < KPF; ++ss)
#pragma unroll
              for (int t = 0; t < 4; ++t) {
                const int row = r0 + 16 * t + mrow, s = s0 + ss;
                x[ss][t] = (row < n && s < d / 16)
                               ? *reinterpret_cast<const float4*>(T.ix.vec + (int64_t)row * d + 16 * s + 4 * kq)
                               : make_float4(0.f, 0.f, 0.f, 0.f);
              }
#pragma unroll
            for (int ss = 0; ss < KPF; ++ss) {
              if (s0 + ss >= d / 16) break;
              const float4 qa = *reinterpret_cast<const float4*>(af + mrow * stride + 16 * (s0 + ss) + 4 * kq);
#pragma unroll
              for (int t = 0; t < 4; ++t) {
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa.x, x[ss][t].x, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa.y, x[ss][t].y, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa.z, x[ss][t].z, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa.w, x[ss][t].w, acc[t], 0, 0, 0);
              }
            }
          }
        } else {
          // 16x16x32 BF16 MFMA: a k-step of 32 elements; lane (n, kq) holds elements
          // 32 s + 8 kq .. + 7 of object n and of query n (A); the query in two parts.
          // Loads of KPF k-steps are issued before their products.
          for (int s0 = 0; s0 < d / 32; s0 += KPF) {
            uint4 x[KPF][4];
#pragma unroll
            for (int ss = 0; ss < KPF; ++ss)
#pragma unroll
              for (int t = 0; t < 4; ++t) {
                const int row = r0 + 16 * t + mrow, s = s0 + ss;
                const bool in = row < n && s < d / 32;
                if constexpr (PREC == UNIFY_BF16) {
                  x[ss][t] = in ? *reinterpret_cast<const uint4*>(T.ix.vec_bf16 + (int64_t)row * d + 32 * s + 8 * kq)
                                : make_uint4(0u, 0u, 0u, 0u);
                } else {
                  const uint2 w = in ? *reinterpret_cast<const uint2*>(T.ix.vec_fp8 + (int64_t)row * d + 32 * s + 8 * kq)
                                     : make_uint2(0u, 0u);
                  x[ss][t] = make_uint4(w.x, w.y, 0u, 0u);
                }
              }
#pragma unroll
            for (int ss = 0; ss < KPF; ++ss) {
              if (s0 + ss >= d / 32) break;
              const int s = s0 + ss;
              const bf16x8_t qh = *reinterpret_cast<const bf16x8_t*>(ahi + mrow * stride + 32 * s + 8 * kq);
              const bf16x8_t ql = *reinterpret_cast<const bf16x8_t*>(alo + mrow * stride + 32 * s + 8 * kq);
#pragma unroll
              for (int t = 0; t < 4; ++t) {
                bf16x8_t xb;
                if constexpr (PREC == UNIFY_BF16) {
                  xb = __builtin_bit_cast(bf16x8_t, x[ss][t]);
                } else {
                  // E4M3 codes decode exactly to BF16 (3 significand bits, exponents 2^-9 .. 2^8)
                  uint32_t h[4];
#pragma unroll
                  for (int c = 0; c < 2; ++c) {
                    const uint32_t word = c == 0 ? x[ss][t].x : x[ss][t].y;
                    const auto f0 = __builtin_amdgcn_cvt_pk_f32_fp8((int)word, false);
                    const auto f1 = __builtin_amdgcn_cvt_pk_f32_fp8((int)word, true);
                    h[2 * c] = (__float_as_uint(f0[0]) >> 16) | (__float_as_uint(f0[1]) & 0xFFFF0000u);
                    h[2 * c + 1] = (__float_as_uint(f1[0]) >> 16) | (__float_as_uint(f1[1]) & 0xFFFF0000u);
                  }
                  xb = __builtin_bit_cast(bf16x8_t, make_uint4(h[0], h[1], h[2], h[3]));
                }
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(qh, xb, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ql, xb, acc[t], 0, 0, 0);
              }
            }
          }
        }
        // lane holds, for tile t, the products of queries 4 kq + i with object r0 + 16 t + mrow
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int row = r0 + 16 * t + mrow;
          float nrm = 0.f, eps = 0.f, sc = 1.f;
          if (row < n) {
            nrm = T.ix.vec_nrm[row];
            if (PREC != UNIFY_FP32) eps = T.ix.vec_eps[row];
            if (PREC == UNIFY_FP8E4M3) sc = T.ix.vec_scale[row];
          }
          const float xn = __builtin_sqrtf(nrm);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int m = 4 * kq + i;
            if (m >= nqg || row < s_lo[m] || row >= s_hi[m]) continue;
            const float4 qi = s_info[m];
            const float dot = PREC == UNIFY_FP8E4M3 ? acc[t][i] * sc : acc[t][i];
            const float st = __builtin_fmaf(-2.0f, dot, nrm) + qi.x;
            const float xs = xn + qi.y;
            const float E = __builtin_fmaf(T.cE * xs, xs, __builtin_fmaf(2.0000019f * xn, qi.z, 1e-30f));
            const float rl = __builtin_sqrtf(fmaxf(st - E, 0.0f));
            const float rh = __builtin_sqrtf(st + E);
            const float l = __builtin_fmaf(rl, T.bA, -__builtin_fmaf(eps, T.bB, 1e-18f));
            const int col = wv * 64 + 16 * t + mrow;
            LB[m * TILE_ROWS + col] = l > 0.0f ? l : 0.0f;
            UB[m * TILE_ROWS + col] = __builtin_fmaf(rh, T.bC, __builtin_fmaf(eps, T.bD, 1e-18f));
          }
        }
      }
    }
    __syncthreads();
    // per query (wavefront w takes queries w, w + 4, ...): block threshold, records,
    // published threshold
    for (int m = wv; m < nqg; m += TILE_WAVES) {
      uint32_t u[4];
      float lb[4];
      int valid = 0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float ub = UB[m * TILE_ROWS + 64 * c + lane];
        u[c] = __float_as_uint(ub);
        lb[c] = LB[m * TILE_ROWS + 64 * c + lane];
        valid += __popcll(ballot(ub != __builtin_inff()));
      }
      const int32_t q = s_q[m];
      const uint32_t tloc = valid >= T.k ? kth_smallest4(u, T.k) : 0x7F800000u;
      const uint32_t tg = __hip_atomic_load(&T.tglob[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const float thr = __uint_as_float(min(tloc, tg));
      const int64_t pair = s_pair[m];
      int cnt = 0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const bool e = u[c] != 0x7F800000u && lb[c] <= thr;
        const u64 em = ballot(e);
        const int pos = cnt + rank_in(em);
        if (e && pos < T.kcq) {
          const int32_t id = sb * TILE_ROWS + 64 * c + lane;
          T.rec_key[pair * T.kcq + pos] = make_key(lb[c], id);
          T.rec_ub[pair * T.kcq + pos] = __uint_as_float(u[c]);
        }
        cnt += __popcll(em);
      }
      if (lane == 0) {
        T.rec_cnt[pair] = min(cnt, T.kcq + 1);
        if (tloc < tg) atomicMin(&T.tglob[q], tloc);
      }
    }
    __syncthreads();
  }
}

// Results of the matrix-core scan: one wavefront per query.  The k-th smallest ub
// over the query's records, then the canonical FP32 distance of every recorded
// object whose lb is not above it; the plain FP32 scan when a record overflowed.
// The records of a query are contiguous; they are read 4 entries per lane per
// round (all loads of a round issued together).
template <int NG>
__global__ void __launch_bounds__(64) k_tile_final(TileArgs T, int64_t* __restrict__ out_ids,
                                                   float* __restrict__ out_dist, int32_t* __restrict__ out_stats) {
  __shared__ u64 lst[WAVE];  // list_insert works on whole 64-entry blocks
  __shared__ u64 keys[WAVE];
  const int lane = lane_id();
  const int64_t q = blockIdx.x;  // one wavefront per workgroup and query
  if (q >= T.nq) return;
  const QPlan P = T.plan[q];
  if (P.strat != UNIFY_PRE || P.tsb == 0) return;
  const DevIndex& ix = T.ix;
  const int k = T.k, kcq = T.kcq;
  float4 qv[NG];
  {
    const int s = lane & 15, G = ix.d >> 2;
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      const int g = s + 16 * i;
      qv[i] = g < G ? *reinterpret_cast<const float4*>(T.Q + q * ix.d + 4 * g) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  constexpr int U = 4;
  const int64_t first = (int64_t)P.tbase * kcq;
  const int total = P.tsb * kcq;
  lst[lane] = KEY_MAX;
  int al = 0;
  bool over = false;
  // pass 1: the k smallest ub
  for (int b0 = 0; b0 < total && !over; b0 += U * WAVE) {
    u64 rk[U];
    float ru[U];
    int rc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = b0 + u * WAVE + lane;
      rc[u] = e < total ? T.rec_cnt[P.tbase + e / kcq] : 0;
      rk[u] = e < total ? T.rec_key[first + e] : KEY_MAX;
      ru[u] = e < total ? T.rec_ub[first + e] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = b0 + u * WAVE + lane;
      over = over || __any(rc[u] > kcq);
      const bool valid = e < total && (e % kcq) < rc[u];
      const u64 key = valid ? make_key(ru[u], key_id(rk[u])) : KEY_MAX;
      const u64 Tk = al == k ? lst[k - 1] : KEY_MAX;
      if (__any(key < Tk)) {  // once the list is full most blocks hold nothing below its end
        list_insert(lst, al, k, key < Tk ? key : KEY_MAX);
        wave_lds_sync();
      }
    }
  }
  const float thr = al == k ? key_dist(lst[k - 1]) : __builtin_inff();
  int32_t nres = 0;
  wave_lds_sync();
  lst[lane] = KEY_MAX;
  al = 0;
  if (!over) {
    // pass 2: canonical FP32 distances of the objects whose lb is not above thr, gathered
    // across the records into batches of up to a wavefront's worth before each evaluation
    int acc = 0;  // gathered ids in keys[0, acc)
    auto flush = [&]() {
      wave_lds_sync();
      eval_keys<NG, UNIFY_FP32, STREAM>(ix, qv, acc, [&](int x) { return key_id(keys[x]); }, keys);
      wave_lds_sync();
      const u64 key = lane < acc ? keys[lane] : KEY_MAX;
      const u64 Tk = al == k ? lst[k - 1] : KEY_MAX;
      if (__any(key < Tk)) list_insert(lst, al, k, key < Tk ? key : KEY_MAX);
      wave_lds_sync();
      nres += acc;
      acc = 0;
    };
    for (int b0 = 0; b0 < total; b0 += U * WAVE) {
      u64 rk[U];
      int rc[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = b0 + u * WAVE + lane;
        rc[u] = e < total ? T.rec_cnt[P.tbase + e / kcq] : 0;
        rk[u] = e < total ? T.rec_key[first + e] : KEY_MAX;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = b0 + u * WAVE + lane;
        const bool use = e < total && (e % kcq) < rc[u] && key_dist(rk[u]) <= thr;
        const u64 um = ballot(use);
        const int nb = __popcll(um);
        if (nb == 0) continue;
        if (acc + nb > WAVE) flush();
        if (use) keys[acc + rank_in(um)] = (uint32_t)key_id(rk[u]);
        acc += nb;
      }
    }
    if (acc > 0) flush();
  } else {
    for (int base = P.lo; base < P.hi; base += WAVE) {
      const int cntv = min(WAVE, P.hi - base);
      eval_keys<NG, UNIFY_FP32, STREAM>(ix, qv, cntv, [&](int x) { return base + x; }, keys);
      wave_lds_sync();
      const u64 key = lane < cntv ? keys[lane] : KEY_MAX;
      const u64 Tk = al == k ? lst[k - 1] : KEY_MAX;
      list_insert(lst, al, k, key < Tk ? key : KEY_MAX);
      wave_lds_sync();
    }
    nres = P.hi - P.lo;
  }
  for (int t = lane; t < k; t += WAVE) {
    const u64 key = t < al ? lst[t] : KEY_MAX;
    out_ids[q * k + t] = key != KEY_MAX ? ix.ext[key_id(key)] : -1;
    out_dist[q * k + t] = key != KEY_MAX ? key_dist(key) : __builtin_inff();
  }
  if (out_stats && lane == 0) {
    int32_t* st = out_stats + q * 8;
    st[0] = P.hi - P.lo;
    st[1] = 0;
    st[2] = nres;
    st[3] = over ? 1 : 0;
    st[4] = P.tsb;  // records of the matrix-core scan (adjacency entries for graph searches)
    st[5] = UNIFY_PRE;
    st[6] = P.hi - P.lo;
    st[7] = 0;
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

namespace {

size_t lds_bytes(int ef_blocks, int ccap, int hcap, int nbr_cap, int sel_cap = 0) {
  return sizeof(u64) * ((size_t)ef_blocks * WAVE + ccap + nbr_cap + sel_cap) + sizeof(uint32_t) * hcap;
}

typedef void (*KernelFn)(SearchArgs);
typedef void (*KernelFnT)(TileArgs);
typedef void (*FinalFn)(TileArgs, int64_t*, float*, int32_t*);

template <int PREC, int PASS, bool S1>
KernelFn pick_kernel(int d) {
  const int ng = (d + 63) / 64;
  if (ng <= 2) return k_search<2, PREC, PASS, S1>;
  if (ng <= 4) return k_search<4, PREC, PASS, S1>;
  if (ng <= 8) return k_search<8, PREC, PASS, S1>;
  if (ng <= 15) return k_search<15, PREC, PASS, S1>;
  if (ng <= 32) return k_search<32, PREC, PASS, S1>;
  return nullptr;
}

template <int PASS, bool S1>
KernelFn kernel_for_sel(int d, int prec) {
  if (prec == UNIFY_BF16) return pick_kernel<UNIFY_BF16, PASS, S1>(d);
  if (prec == UNIFY_FP8E4M3) return pick_kernel<UNIFY_FP8E4M3, PASS, S1>(d);
  return pick_kernel<UNIFY_FP32, PASS, S1>(d);
}

template <int PASS>
KernelFn kernel_for(int d, int prec, bool s1 = false) {
  return s1 ? kernel_for_sel<PASS, true>(d, prec) : kernel_for_sel<PASS, false>(d, prec);
}

template <int PREC, int MW>
KernelFn pick_mw(int d) {
  const int ng = (d + 63) / 64;
  if (ng <= 2) return k_search_mw<2, PREC, MW>;
  if (ng <= 4) return k_search_mw<4, PREC, MW>;
  if (ng <= 8) return k_search_mw<8, PREC, MW>;
  if (ng <= 15) return k_search_mw<15, PREC, MW>;
  if (ng <= 32) return k_search_mw<32, PREC, MW>;
  return nullptr;
}

template <int MW>
KernelFn mw_for_prec(int d, int prec) {
  if (prec == UNIFY_BF16) return pick_mw<UNIFY_BF16, MW>(d);
  if (prec == UNIFY_FP8E4M3) return pick_mw<UNIFY_FP8E4M3, MW>(d);
  return pick_mw<UNIFY_FP32, MW>(d);
}

KernelFn kernel_mw(int d, int prec, int mw) { return mw == 4 ? mw_for_prec<4>(d, prec) : mw_for_prec<2>(d, prec); }

#define HIP_OK(x)                                                            \
  do {                                                                       \
    hipError_t e_ = (x);                                                     \
    if (e_ != hipSuccess) {                                                  \
      set_error(std::string(#x) + ": " + hipGetErrorString(e_));             \
      return UNIFY_EDEVICE;                                                  \
    }                                                                        \
  } while (0)

// Validated parameters of one search configuration.
struct Resolved {
  int32_t k, ef, m, p, ccap, hcap, rerank, pre_chunk;
  int64_t tauA, tauB;
  uint32_t flags;
  bool tile;    // pre-filter scans may run on the matrix cores
  int32_t kcq;  // objects one (query, super-block) record holds
  int32_t wpq;    // wavefronts per heavy graph search (1: no cooperative kernel)
  int32_t heavy;  // heavy graph searches per batch at most
};

int resolve(unify_index_t ix, int64_t nq, int32_t k, int32_t ef, const unify_params* prm, Resolved& R) {
  if (!ix) {
    set_error("null index");
    return UNIFY_EINVAL;
  }
  if (nq < 0 || nq >= (int64_t(1) << 28)) {
    set_error("nq out of range");
    return UNIFY_EINVAL;
  }
  if (k < 1 || k > 256) {
    set_error("k must be in [1, 256]");
    return UNIFY_EINVAL;
  }
  if (ef < k || ef > 256) {
    set_error("ef must be in [k, 256]");
    return UNIFY_EINVAL;
  }
  unify_params P{};
  if (prm) P = *prm;
  const DevIndex& dv = ix->dv;
  R.k = k;
  R.ef = ef;
  R.m = P.m > 0 ? P.m : dv.M0;
  R.p = P.beam_p > 0 ? P.beam_p : 1;
  const double ta = P.tau_a_frac > 0 ? P.tau_a_frac : 0.01;
  const double tb = P.tau_b_frac > 0 ? P.tau_b_frac : 0.5;
  // candidate array: 512 entries, or 8 ef rounded up to a power of two for longer lists (a
  // hybrid search keeps out-of-range objects in it; at ef = 128, 512 entries sent 1.5% of the
  // serving workload's queries to the larger-capacity re-run, which then ended the batch)
  R.ccap = 512;
  while (R.ccap < 8 * ef) R.ccap *= 2;
  if (P.cand_cap > 0) R.ccap = P.cand_cap;
  R.hcap = P.visit_cap > 0 ? P.visit_cap : (dv.precision == UNIFY_FP32 ? 1024 : 512);
  R.rerank = P.rerank_mult > 0 ? P.rerank_mult : 4;
  R.wpq = P.waves_per_query > 0 ? P.waves_per_query : 1;
  R.heavy = P.heavy_queries > 0 ? P.heavy_queries : ix->cus;
  R.pre_chunk = P.pre_chunk > 0 ? P.pre_chunk : 2048;
  R.flags = P.flags;
  if (R.m > dv.S * dv.M0 || R.p > 8 || ta > 1.0 || tb > 1.0 || R.ccap < 64 || R.ccap > 4096 ||
      (R.ccap & (R.ccap - 1)) || R.hcap < 256 || R.hcap > 16384 || (R.hcap & (R.hcap - 1)) || R.rerank > 256 ||
      R.pre_chunk < 64 || (R.wpq != 1 && R.wpq != 2 && R.wpq != 4) || P.heavy_queries < 0 ||
      ((R.flags & UNIFY_FLAG_SELECT_S1) && R.wpq > 1)) {
    set_error("params out of range (m <= S*M0, beam_p <= 8, tau fractions <= 1, cand_cap and visit_cap powers "
              "of two in [64, 4096] and [256, 16384], rerank_mult <= 256, pre_chunk >= 64, waves_per_query 1, 2 "
              "or 4 and not with selection S1, heavy_queries >= 0)");
    return UNIFY_EINVAL;
  }
  // the FP32 rerank of a low-precision search builds its k results in the candidate array
  if (dv.precision != UNIFY_FP32)
    while (R.ccap < k) R.ccap *= 2;
  R.tauA = (int64_t)std::floor(ta * (double)dv.n);
  R.tauB = (int64_t)std::ceil(tb * (double)dv.n);
  // the matrix-core scan: k <= TILE_KMAX, d <= TILE_DMAX, whole MFMA k-steps (16 elements
  // for FP32, 32 for BF16 / FP8 rows), the store's row norms resident
  R.tile = !(R.flags & UNIFY_FLAG_PRE_WAVE_SCAN) && k <= TILE_KMAX && dv.d <= TILE_DMAX && dv.vec_nrm &&
           dv.d % (dv.precision == UNIFY_FP32 ? 16 : 32) == 0 && dv.n < (int64_t(1) << 31);
  // records hold the block's k smallest upper bounds and the few objects whose bounds
  // overlap them; FP8 bounds are wider
  R.kcq = (2 * k + 12 + 7) / 8 * 8 * (dv.precision == UNIFY_FP8E4M3 ? 2 : 1);
  if (!kernel_for<0>(dv.d, dv.precision)) {
    set_error("unsupported dimension");
    return UNIFY_EINVAL;
  }
  return UNIFY_OK;
}

}  // namespace

// The side stream of the cooperative kernel, the visited rows and the event
// that orders the search kernels using them.  The index's pool is made when the
// index becomes resident (load, build, insertion), so that searches need no
// allocation of their own.
int make_side(SideStream& s, bool coop, bool tile) {
  if (coop) {
    if (!s.stream) HIP_OK(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
    for (hipEvent_t* e : {&s.fork, &s.join})
      if (!*e) HIP_OK(hipEventCreateWithFlags(e, hipEventDisableTiming));
  }
  if (tile) {
    if (!s.tstream) HIP_OK(hipStreamCreateWithFlags(&s.tstream, hipStreamNonBlocking));
    for (hipEvent_t* e : {&s.tfork, &s.tjoin})
      if (!*e) HIP_OK(hipEventCreateWithFlags(e, hipEventDisableTiming));
  }
  return UNIFY_OK;
}

void free_side(SideStream& s) {
  for (hipEvent_t e : {s.fork, s.join, s.tfork, s.tjoin})
    if (e) (void)hipEventDestroy(e);
  for (hipStream_t t : {s.stream, s.tstream})
    if (t) (void)hipStreamDestroy(t);
  s = SideStream{};
}

namespace {
int64_t bitmap_words(int64_t n) { return ((n + 31) / 32 + 63) / 64 * 64; }
}  // namespace

size_t pool_row_bytes(int64_t n) { return sizeof(uint32_t) * (size_t)(bitmap_words(n) + VLOG_CAP); }

int pool_ensure(VisitPool& p, int64_t n) {
  if (!p.last) HIP_OK(hipEventCreateWithFlags(&p.last, hipEventDisableTiming));
  if (p.rows && p.n == n) return UNIFY_OK;
  if (p.rows) {
    HIP_OK(hipEventSynchronize(p.last));
    HIP_OK(hipFree(p.rows));
    p.rows = nullptr;
    p.nrows = 0;
  }
  size_t free_b = 0, total_b = 0;
  HIP_OK(hipMemGetInfo(&free_b, &total_b));
  const size_t rb = pool_row_bytes(n);
  const int64_t fit = (int64_t)(free_b / 4 / rb);
  const int64_t rows = std::min<int64_t>(std::max<int64_t>(p.max_rows, 1), fit);
  void* r = nullptr;
  if (rows < 1 || hipMalloc(&r, rb * (size_t)rows) != hipSuccess) {
    set_error("no device memory for the visited rows");
    return UNIFY_ENOMEM;
  }
  HIP_OK(hipMemset(r, 0, rb * (size_t)rows));
  HIP_OK(hipDeviceSynchronize());
  p.rows = static_cast<uint32_t*>(r);
  p.nrows = rows;
  p.bwords = bitmap_words(n);
  p.stride = p.bwords + VLOG_CAP;
  p.n = n;
  return UNIFY_OK;
}

void pool_free(VisitPool& p) {
  if (p.last) {
    (void)hipEventSynchronize(p.last);
    (void)hipEventDestroy(p.last);
  }
  if (p.rows) (void)hipFree(p.rows);
  free_side(p.side);
  p.rows = nullptr;
  p.last = nullptr;
  p.nrows = 0;
  p.n = -1;
}

int ensure_pool(unify_index_t ix) {
  if (!ix->cus) HIP_OK(hipDeviceGetAttribute(&ix->cus, hipDeviceAttributeMultiprocessorCount, ix->device));
  if (!ix->pool.max_rows) ix->pool.max_rows = (int64_t)ix->cus * 16;
  // the index's side streams exist from the start: the allocation-free call creates nothing
  if (make_side(ix->pool.side, true, true) != UNIFY_OK) return UNIFY_EDEVICE;
  return pool_ensure(ix->pool, ix->dv.n);
}

namespace {

// Per-call device scratch: plans, work list (graph queries and pre-filter
// chunks), chunk of each entry, fallback list, counters, per-query merge
// counters, partial top-k lists of split pre-filter scans.
struct Scratch {
  QPlan* plan;
  int32_t *work, *wchunk, *fb, *counters, *qacc;
  u64* part;
  // matrix-core pre-filter scan (pcap = 0: none)
  int64_t pcap, nsb;
  uint32_t *qhl, *tglob;
  float4* qinfo;
  int32_t *cnt_sb, *fill_sb, *off_sb, *ioff, *list, *item_sb, *rec_cnt;
  u64* rec_key;
  float* rec_ub;
};

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// Device scratch of one search of nq queries; pcap records for the matrix-core
// scan (0: none), each of kcq objects.  Returns the bytes; fills S when given.
size_t scratch_layout(const DevIndex& dv, int64_t nq, int k, int64_t pcap, int kcq, void* base, Scratch* S) {
  const int64_t wcap = nq * PRE_NCH_MAX;
  const size_t plan_b = up256(sizeof(QPlan) * nq), work_b = up256(sizeof(int32_t) * wcap),
               fb_b = up256(sizeof(int32_t) * nq), acc_b = up256(sizeof(int32_t) * 4 * nq),
               part_b = k <= PRE_SPLIT_KMAX ? up256(sizeof(u64) * (size_t)wcap * k) : 0;
  const int64_t nsb = (dv.n + TILE_ROWS - 1) / TILE_ROWS;
  size_t qhl_b = 0, info_b = 0, tg_b = 0, sb_b = 0, sb1_b = 0, list_b = 0, rc_b = 0, rk_b = 0, ru_b = 0;
  if (pcap > 0) {
    qhl_b = dv.precision != UNIFY_FP32 ? up256(sizeof(uint32_t) * (size_t)nq * dv.d) : 0;
    info_b = up256(sizeof(float4) * nq);
    tg_b = up256(sizeof(uint32_t) * nq);
    sb_b = up256(sizeof(int32_t) * nsb);
    sb1_b = up256(sizeof(int32_t) * (nsb + 1));
    list_b = up256(sizeof(int32_t) * pcap);
    rc_b = list_b;
    rk_b = up256(sizeof(u64) * (size_t)pcap * kcq);
    ru_b = up256(sizeof(float) * (size_t)pcap * kcq);
  }
  if (S) {
    char* sp = static_cast<char*>(base);
    S->plan = reinterpret_cast<QPlan*>(sp);
    S->work = reinterpret_cast<int32_t*>(sp += plan_b);
    S->wchunk = reinterpret_cast<int32_t*>(sp += work_b);
    S->fb = reinterpret_cast<int32_t*>(sp += work_b);
    S->counters = reinterpret_cast<int32_t*>(sp += fb_b);  // nwork, next, fb_count, fb_next, -, tile items
    S->qacc = reinterpret_cast<int32_t*>(sp += 256);
    sp += acc_b;
    S->part = part_b ? reinterpret_cast<u64*>(sp) : nullptr;
    sp += part_b;
    S->pcap = pcap;
    S->nsb = nsb;
    S->qhl = qhl_b ? reinterpret_cast<uint32_t*>(sp) : nullptr;
    sp += qhl_b;
    S->qinfo = reinterpret_cast<float4*>(sp);
    sp += info_b;
    S->tglob = reinterpret_cast<uint32_t*>(sp);
    sp += tg_b;
    S->cnt_sb = reinterpret_cast<int32_t*>(sp);
    sp += sb_b;
    S->fill_sb = reinterpret_cast<int32_t*>(sp);
    sp += sb_b;
    S->off_sb = reinterpret_cast<int32_t*>(sp);
    sp += sb1_b;
    S->ioff = reinterpret_cast<int32_t*>(sp);
    sp += sb1_b;
    S->list = reinterpret_cast<int32_t*>(sp);
    sp += list_b;
    S->item_sb = reinterpret_cast<int32_t*>(sp);
    sp += list_b;
    S->rec_cnt = reinterpret_cast<int32_t*>(sp);
    sp += rc_b;
    S->rec_key = reinterpret_cast<u64*>(sp);
    sp += rk_b;
    S->rec_ub = reinterpret_cast<float*>(sp);
  }
  return plan_b + 2 * work_b + fb_b + 256 + acc_b + part_b + qhl_b + info_b + tg_b + 2 * sb_b + 2 * sb1_b +
         2 * list_b + rc_b + rk_b + ru_b;
}

// Records of the matrix-core scan for a batch of nq queries.
int64_t tile_pcap(const Resolved& R, int64_t nq) { return R.tile ? TILE_PAIRS_PER_QUERY * nq + 64 : 0; }

// A launch configuration of the persistent search kernel, prepared outside any
// stream capture: dynamic LDS size set on the function, grid from occupancy.
struct Pass {
  KernelFn fn;
  size_t lds;
  unsigned grid;
};

// cache = false: the occupancy found is not added to the index's table (the
// allocation-free entry point keeps host memory unchanged too).
int prepare_pass(unify_index_t ix, KernelFn fn, size_t lds, int64_t nq, int64_t row_cap, Pass& out,
                 bool cache = true, int reserve = 0, int block = 64) {
  const auto key = std::make_pair(reinterpret_cast<const void*>(fn), lds);
  auto it = ix->occupancy.find(key);
  int per_cu = 0;
  if (it != ix->occupancy.end()) {
    per_cu = it->second;
  } else {
    HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(fn), block, lds));
    if (cache) ix->occupancy[key] = per_cu;
  }
  if (per_cu < 1) {
    set_error("search kernel does not fit on a compute unit");
    return UNIFY_EDEVICE;
  }
  // reserve: wavefronts per compute unit left for a kernel running beside this one
  int64_t grid = (int64_t)std::max(1, per_cu - reserve) * ix->cus;
  grid = std::min<int64_t>(grid, row_cap);
  grid = std::min<int64_t>(grid, nq);
  out.fn = fn;
  out.lds = lds;
  out.grid = (unsigned)std::max<int64_t>(grid, 1);
  return UNIFY_OK;
}

// Everything one search launches, with its arguments fixed.
struct Launch {
  DevIndex dv;
  const float* queries;
  int64_t nq;
  const int64_t *l, *h;
  const int64_t *l2 = nullptr, *h2 = nullptr;  // conjunctive and box searches
  bool box = false;                             // box search on the z-order index z
  ZOrder z;
  const int8_t* strategy;
  int64_t* out_ids;
  float* out_dist;
  int8_t* out_strategy;
  int32_t* out_stats;
  Resolved R;
  Scratch S;
  SearchArgs A, B, C;  // first pass, re-run pass, cooperative searches
  Pass p0, p1, pc;
  bool mw = false;
  // matrix-core pre-filter scan
  bool tile = false;
  TileArgs T;
  KernelFnT scan_fn = nullptr;
  FinalFn final_fn = nullptr;
  size_t scan_lds = 0;
  unsigned scan_grid = 0;
};

int prepare_launch(unify_index_t ix, const Resolved& R, const float* queries, int64_t nq, const int64_t* l,
                   const int64_t* h, const int8_t* strategy, int64_t* out_ids, float* out_dist,
                   int8_t* out_strategy, int32_t* out_stats, void* scratch, int64_t pcap, const VisitPool& pool,
                   Launch& X, const int64_t* l2 = nullptr, const int64_t* h2 = nullptr, bool cache = true) {
  const DevIndex& dv = ix->dv;
  X.dv = dv;
  X.queries = queries;
  X.nq = nq;
  X.l = l;
  X.h = h;
  X.strategy = strategy;
  X.out_ids = out_ids;
  X.out_dist = out_dist;
  X.out_strategy = out_strategy;
  X.out_stats = out_stats;
  X.R = R;
  if (l2) pcap = 0;  // conjunctive scans test the second attribute: per wavefront
  scratch_layout(dv, nq, R.k, pcap, R.kcq, scratch, &X.S);
  const int S = dv.S;
  const int per_node = std::max(std::min(R.m + S - 1, S * std::max(dv.M0, dv.MU)), dv.GC);
  SearchArgs A{};
  A.ix = dv;
  A.Q = queries;
  A.nq = nq;
  A.k = R.k;
  A.ef = R.ef;
  A.m = R.m;
  A.p = R.p;
  A.rerank = R.rerank;
  {
    // canonical FP32 distance: each term passes through at most e + 6 roundings
    // (the subtraction, squared; e fused multiply-adds; 4 butterfly additions),
    // e = elements per partial sum, so its relative error is at most
    // g = n u / (1 - n u), n = e + 6, u = 2^-24
    const int G = dv.d / 4;
    const double nr = 4.0 * ((G + 15) / 16) + 6.0, u = std::ldexp(1.0, -24);
    const double g = nr * u / (1.0 - nr * u), w = std::ldexp(1.0, -20);
    A.bA = (float)(std::sqrt((1.0 - g) / (1.0 + g)) * (1.0 - w));
    A.bB = (float)(std::sqrt(1.0 - g) * (1.0 + w));
    A.bC = (float)(std::sqrt((1.0 + g) / (1.0 - g)) * (1.0 + w));
    A.bD = (float)(std::sqrt(1.0 + g) * (1.0 + w));
  }
  A.ef_blocks = (std::max(R.ef, R.k) + WAVE - 1) / WAVE;
  A.nbr_cap = std::max((R.p * per_node + WAVE - 1) / WAVE * WAVE, WAVE);
  // selection S1 ranks a popped object's entries: a list of m plus 64 scratch keys
  A.sel_cap = (R.flags & UNIFY_FLAG_SELECT_S1) ? (R.m + WAVE - 1) / WAVE * WAVE + WAVE : 0;
  A.out_ids = out_ids;
  A.out_dist = out_dist;
  A.out_stats = out_stats;
  // the counters block holds 4 counters, then (conjunctive searches) the ConjArgs
  A.conj = l2 ? reinterpret_cast<const ConjArgs*>(X.S.counters + 16) : nullptr;
  X.l2 = l2;
  X.h2 = h2;
  A.plan = X.S.plan;
  A.vrows = pool.rows;
  A.vstride = pool.stride;
  A.bwords = pool.bwords;
  A.nslots = pool.nrows;
  // first pass: modest LDS per wave for occupancy
  A.ccap = R.ccap;
  A.hcap = R.hcap;
  A.pass = 0;
  A.work = X.S.work;
  A.wchunk = X.S.wchunk;
  A.part = X.S.part;
  A.qacc = X.S.qacc;
  A.nwork = X.S.counters + 0;
  A.next = X.S.counters + 1;
  A.fb_list = X.S.fb;
  A.fb_count = X.S.counters + 2;
  A.nheavy = X.S.counters + 6;
  A.nbeam = X.S.counters + 4;
  A.mw_next = X.S.counters + 7;
  A.mw_row0 = 0;
  // second pass over the abandoned queries with the largest LDS that fits
  int maxlds = 0;
  if (hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, ix->device) != hipSuccess)
    maxlds = 65536;
  int cc = 16384, hc = std::max(R.hcap, 2048);
  while (lds_bytes(A.ef_blocks, cc, hc, A.nbr_cap, A.sel_cap) > (size_t)maxlds && cc > 2 * R.ccap) cc /= 2;
  SearchArgs B = A;
  B.ccap = cc;
  B.hcap = hc;
  B.pass = 1;
  B.work = X.S.fb;
  B.wchunk = nullptr;  // only graph searches are re-run
  B.nwork = X.S.counters + 2;
  B.next = X.S.counters + 3;
  X.A = A;
  X.B = B;
  const bool s1 = (R.flags & UNIFY_FLAG_SELECT_S1) != 0;
  X.tile = pcap > 0;
  if (X.tile) {
    TileArgs T{};
    T.ix = dv;
    T.plan = X.S.plan;
    T.Q = queries;
    T.nq = nq;
    T.k = R.k;
    T.kcq = R.kcq;
    T.qhl = X.S.qhl;
    T.qinfo = X.S.qinfo;
    T.tglob = X.S.tglob;
    T.cnt_sb = X.S.cnt_sb;
    T.fill_sb = X.S.fill_sb;
    T.off_sb = X.S.off_sb;
    T.ioff = X.S.ioff;
    T.list = X.S.list;
    T.item_sb = X.S.item_sb;
    T.rec_cnt = X.S.rec_cnt;
    T.rec_key = X.S.rec_key;
    T.rec_ub = X.S.rec_ub;
    T.counters = X.S.counters;
    T.nsb = X.S.nsb;
    // bounds of the norm expansion: |s~ - ||x~ - q||^2| <= cE (||x~|| + ||q||)^2 + 2 ||x~|| eq,
    // cE = 3 (d + 8) u covering the products' accumulation (two parts of the query), both
    // norms and the two additions; g and the constants as for the low-precision scan
    const int G = dv.d / 4;
    const double u = std::ldexp(1.0, -24), w = std::ldexp(1.0, -20);
    const double nr = 4.0 * ((G + 15) / 16) + 6.0, g = nr * u / (1.0 - nr * u);
    T.cE = (float)(3.0 * (dv.d + 8) * u * (1.0 + w));
    T.bA = (float)(std::sqrt(1.0 - g) * (1.0 - w));
    T.bB = (float)(std::sqrt(1.0 - g) * (1.0 + w));
    T.bC = (float)(std::sqrt(1.0 + g) * (1.0 + w));
    T.bD = T.bC;
    X.T = T;
    // the scan runs alone when the phases run one after another, else beside the search
    if (R.flags & UNIFY_FLAG_SERIAL_PHASES)
      X.scan_fn = dv.precision == UNIFY_BF16 ? k_tile_scan<UNIFY_BF16, true>
                  : dv.precision == UNIFY_FP8E4M3 ? k_tile_scan<UNIFY_FP8E4M3, true> : k_tile_scan<UNIFY_FP32, true>;
    else
      X.scan_fn = dv.precision == UNIFY_BF16 ? k_tile_scan<UNIFY_BF16, false>
                  : dv.precision == UNIFY_FP8E4M3 ? k_tile_scan<UNIFY_FP8E4M3, false> : k_tile_scan<UNIFY_FP32, false>;
    const int ng = (dv.d + 63) / 64;
    X.final_fn = ng <= 2 ? k_tile_final<2> : (ng <= 4 ? k_tile_final<4> : k_tile_final<8>);
    X.scan_lds = (size_t)TILE_Q * (dv.d + 8) * 4 + 2 * (size_t)TILE_Q * TILE_ROWS * sizeof(float);
    HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void*>(X.scan_fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)X.scan_lds));
    int per_cu = 0;
    HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(X.scan_fn),
                                                        64 * TILE_WAVES, X.scan_lds));
    X.scan_grid = (unsigned)std::max(1, std::max(1, per_cu) * ix->cus);
  }
  // cooperative searches of the heavy queries: one workgroup of wpq wavefronts per compute
  // unit, beside the one-wavefront kernel, whose grid leaves them room
  X.mw = R.wpq > 1 && R.heavy > 0;
  int reserve = 0;
  int64_t row_cap = pool.nrows;
  if (X.mw) {
    SearchArgs C = A;
    C.ccap = std::max(A.ccap, 1024);
    C.hcap = std::max(A.hcap, 2048);
    KernelFn fc = kernel_mw(dv.d, dv.precision, R.wpq);
    if (!fc) {
      set_error("unsupported dimension");
      return UNIFY_EINVAL;
    }
    const size_t lc = lds_bytes_mw(C.ef_blocks, C.ccap, C.hcap, C.nbr_cap, R.wpq);
    const int64_t gc = std::min<int64_t>(ix->cus, std::max<int64_t>(1, pool.nrows / 8));
    C.mw_row0 = pool.nrows - gc;  // the last gc visited rows
    HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void*>(fc), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lc));
    X.pc = Pass{fc, lc, (unsigned)gc};
    X.C = C;
    reserve = R.wpq;
    row_cap = C.mw_row0;
  }
  int rc = prepare_pass(ix, kernel_for<0>(dv.d, dv.precision, s1),
                        lds_bytes(A.ef_blocks, A.ccap, A.hcap, A.nbr_cap, A.sel_cap), nq, row_cap, X.p0, cache,
                        reserve);
  // the re-run pass holds the few queries that overflowed: a small grid launches faster
  if (rc == UNIFY_OK)
    rc = prepare_pass(ix, kernel_for<1>(dv.d, dv.precision, s1),
                      lds_bytes(B.ef_blocks, B.ccap, B.hcap, B.nbr_cap, B.sel_cap), std::min<int64_t>(nq, 512),
                      pool.nrows, X.p1, cache);
  return rc;
}

// The matrix-core scan runs on the side stream, beside the graph search.
bool tile_beside(const Launch& X) { return X.tile && !(X.R.flags & UNIFY_FLAG_SERIAL_PHASES); }

// The side streams a launch uses, made before it is enqueued (or captured).
int make_side_for(SideStream& s, const Launch& X) { return make_side(s, X.mw, tile_beside(X)); }

// Kernel launches only (no allocation, no memset, no synchronisation), so the
// sequence can be captured into a HIP graph.  ev: 8 events to record, or null.
// order: the visited pool whose previous search kernels the search kernels must
// follow (null inside a graph capture, where the caller orders the replay
// instead).  whole = true: the plan and work-list kernels wait too (their
// scratch is shared with the previous call's search kernels).
int enqueue_launch(const Launch& X, hipStream_t st, hipEvent_t* ev, const SideStream& side,
                   VisitPool* order = nullptr, bool whole = false) {
  const unsigned pb = 256;
  const int64_t nq = X.nq;
  std::unique_lock<std::mutex> g;
  if (order) {
    g = std::unique_lock<std::mutex>(order->mu);
    if (whole) HIP_OK(hipStreamWaitEvent(st, order->last, 0));
  }
  const unsigned qb4 = (unsigned)((nq + 3) / 4);
  if (ev) HIP_OK(hipEventRecord(ev[0], st));
  hipLaunchKernelGGL(k_plan, dim3((unsigned)((nq + pb - 1) / pb)), dim3(pb), 0, st, X.dv, X.l, X.h, X.l2, X.h2, X.z,
                     (int32_t)X.box,
                     const_cast<ConjArgs*>(X.A.conj), X.strategy, nq,
                     X.R.tauA, X.R.tauB, X.R.k, X.R.pre_chunk, (int32_t)X.tile, X.S.plan, X.out_strategy,
                     X.out_ids, X.out_dist, X.out_stats);
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((4 * nq + pb - 1) / pb)), dim3(pb), 0, st, X.S.qacc, 4 * nq, 0);
  if (X.tile)
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((X.S.nsb + pb - 1) / pb)), dim3(pb), 0, st, X.S.cnt_sb,
                       X.S.nsb, 0);
  hipLaunchKernelGGL(k_worklist, dim3(1), dim3(1024), 0, st, X.S.plan, nq, X.dv.n, X.S.pcap,
                     (int32_t)(X.mw ? X.R.heavy : 0), X.S.work, X.S.wchunk, X.S.counters);
  HIP_OK(hipGetLastError());
  if (ev) HIP_OK(hipEventRecord(ev[1], st));
  // the matrix-core scan: its own queries and scratch, beside the graph search
  // (on the side stream) unless the phases run one after another
  const bool tside = tile_beside(X);
  hipStream_t ts = st;
  if (tside) {
    HIP_OK(hipEventRecord(side.tfork, st));
    HIP_OK(hipStreamWaitEvent(side.tstream, side.tfork, 0));
    ts = side.tstream;
  }
  if (X.tile) {
    // one-wavefront workgroups: beside the graph search they start as soon as any of its
    // wavefronts leaves a SIMD, rather than waiting for several to leave one compute unit
    hipLaunchKernelGGL(k_tile_prep, dim3((unsigned)nq), dim3(64), 0, ts, X.T);
    const int nw = tside ? (int)std::min<int64_t>(16, std::max<int64_t>(1, X.S.nsb / 4096)) : 16;
    hipLaunchKernelGGL(k_tile_index, dim3(1), dim3(64 * nw), 0, ts, X.T);
    hipLaunchKernelGGL(k_tile_fill, dim3((unsigned)nq), dim3(64), 0, ts, X.T);
    if (ev) HIP_OK(hipEventRecord(ev[2], ts));
    hipLaunchKernelGGL(X.scan_fn, dim3(X.scan_grid), dim3(64 * TILE_WAVES), X.scan_lds, ts, X.T);
    if (ev) HIP_OK(hipEventRecord(ev[3], ts));
    hipLaunchKernelGGL(X.final_fn, dim3((unsigned)nq), dim3(64), 0, ts, X.T, X.out_ids, X.out_dist, X.out_stats);
    HIP_OK(hipGetLastError());
    if (ev) HIP_OK(hipEventRecord(ev[4], ts));
    if (tside) HIP_OK(hipEventRecord(side.tjoin, ts));
  } else if (ev) {
    for (int i = 2; i <= 4; ++i) HIP_OK(hipEventRecord(ev[i], st));
  }
  if (order && !whole) HIP_OK(hipStreamWaitEvent(st, order->last, 0));
  if (X.mw) {
    // the cooperative kernel on the side stream, concurrently with the one-wavefront kernel
    HIP_OK(hipEventRecord(side.fork, st));
    HIP_OK(hipStreamWaitEvent(side.stream, side.fork, 0));
    hipLaunchKernelGGL(X.pc.fn, dim3(X.pc.grid), dim3(64 * X.R.wpq), X.pc.lds, side.stream, X.C);
    HIP_OK(hipGetLastError());
    HIP_OK(hipEventRecord(side.join, side.stream));
  }
  hipLaunchKernelGGL(X.p0.fn, dim3(X.p0.grid), dim3(64), X.p0.lds, st, X.A);
  HIP_OK(hipGetLastError());
  if (X.mw) HIP_OK(hipStreamWaitEvent(st, side.join, 0));
  if (ev) HIP_OK(hipEventRecord(ev[5], st));
  // the merge and the re-run follow the matrix-core scan (its FP32 fallbacks join the re-run)
  if (tside) HIP_OK(hipStreamWaitEvent(st, side.tjoin, 0));
  if (X.S.part) {
    hipLaunchKernelGGL(k_pre_merge, dim3(qb4), dim3(256), 0, st, X.dv, X.S.plan, nq, X.R.k,
                       X.S.part, X.S.qacc, X.out_ids, X.out_dist, X.out_stats);
    HIP_OK(hipGetLastError());
  }
  if (ev) HIP_OK(hipEventRecord(ev[6], st));
  hipLaunchKernelGGL(X.p1.fn, dim3(X.p1.grid), dim3(64), X.p1.lds, st, X.B);
  HIP_OK(hipGetLastError());
  if (order) HIP_OK(hipEventRecord(order->last, st));
  if (ev) HIP_OK(hipEventRecord(ev[7], st));
  return UNIFY_OK;
}

}  // namespace

namespace {
int search_common(unify_index_t ix, const float* queries, int64_t nq, const int64_t* l, const int64_t* h,
                  const int64_t* l2, const int64_t* h2, int32_t k, int32_t ef, const int8_t* strategy,
                  const unify_params* prm, int64_t* out_ids, float* out_dist, int8_t* out_strategy,
                  int32_t* out_stats, void* stream, bool box = false) {
  if (!ix) {
    set_error("null index");
    return UNIFY_EINVAL;
  }
  std::shared_lock<std::shared_mutex> version(ix->version_mu);
  if ((!l2) != (!h2)) {
    set_error("l2 and h2 are given together");
    return UNIFY_EINVAL;
  }
  if (box ? !ix->z.a1 : (l2 && !ix->dv.attr2)) {
    set_error(box ? "the index has no z-order attributes (unify_set_zorder)"
                  : "the index has no second attribute (unify_set_attr2)");
    return UNIFY_EINVAL;
  }
  Resolved R;
  int rc = resolve(ix, nq, k, ef, prm, R);
  if (rc != UNIFY_OK) return rc;
  if (!queries || !l || !h || !out_ids || !out_dist) {
    if (nq == 0) return UNIFY_OK;
    set_error("null buffer");
    return UNIFY_EINVAL;
  }
  if (nq == 0) return UNIFY_OK;
  HIP_OK(hipSetDevice(ix->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  rc = ensure_pool(ix);
  if (rc != UNIFY_OK) return rc;
  const bool timing = (R.flags & UNIFY_FLAG_TIMING) != 0;
  if (timing) {
    for (hipEvent_t& e : ix->ev)
      if (!e) HIP_OK(hipEventCreate(&e));
    ix->timed = true;
  }
  void* scratch = nullptr;
  const int64_t pcap = l2 ? 0 : tile_pcap(R, nq);
  HIP_OK(hipMallocAsync(&scratch, scratch_layout(ix->dv, nq, k, pcap, R.kcq, nullptr, nullptr), st));
  Launch X;
  rc = prepare_launch(ix, R, queries, nq, l, h, strategy, out_ids, out_dist, out_strategy, out_stats, scratch, pcap,
                      ix->pool, X, l2, h2);
  X.box = box;
  X.z = ix->z;
  if (timing) ix->timed_side = tile_beside(X);
  if (rc == UNIFY_OK) rc = make_side_for(ix->pool.side, X);
  if (rc == UNIFY_OK) rc = enqueue_launch(X, st, timing ? ix->ev : nullptr, ix->pool.side, &ix->pool);
  if (hipFreeAsync(scratch, st) != hipSuccess && rc == UNIFY_OK) rc = UNIFY_EDEVICE;
  return rc;
}
}  // namespace

int search_impl(unify_index_t ix, const float* queries, int64_t nq, const int64_t* l, const int64_t* h,
                int32_t k, int32_t ef, const int8_t* strategy, const unify_params* prm, int64_t* out_ids,
                float* out_dist, int8_t* out_strategy, int32_t* out_stats, void* stream) {
  return search_common(ix, queries, nq, l, h, nullptr, nullptr, k, ef, strategy, prm, out_ids, out_dist,
                       out_strategy, out_stats, stream);
}

int search_multi_impl(unify_index_t ix, const float* queries, int64_t nq, const int64_t* l, const int64_t* h,
                      const int64_t* l2, const int64_t* h2, int32_t k, int32_t ef, const int8_t* strategy,
                      const unify_params* prm, int64_t* out_ids, float* out_dist, int8_t* out_strategy,
                      int32_t* out_stats, void* stream) {
  if (nq > 0 && (!l2 || !h2)) {
    set_error("null second range");
    return UNIFY_EINVAL;
  }
  return search_common(ix, queries, nq, l, h, l2, h2, k, ef, strategy, prm, out_ids, out_dist, out_strategy,
                       out_stats, stream);
}

int search_box_impl(unify_index_t ix, const float* queries, int64_t nq, const int64_t* l1, const int64_t* h1,
                    const int64_t* l2, const int64_t* h2, int32_t k, int32_t ef, const int8_t* strategy,
                    const unify_params* prm, int64_t* out_ids, float* out_dist, int8_t* out_strategy,
                    int32_t* out_stats, void* stream) {
  if (nq > 0 && (!l2 || !h2)) {
    set_error("null second range");
    return UNIFY_EINVAL;
  }
  return search_common(ix, queries, nq, l1, h1, l2, h2, k, ef, strategy, prm, out_ids, out_dist, out_strategy,
                       out_stats, stream, true);
}


// Scratch of a search of nq queries with parameters prm on index ix (0 when they are invalid).
size_t search_scratch_bytes(unify_index_t ix, int64_t nq, int32_t k, int32_t ef, const unify_params* prm) {
  Resolved R;
  if (resolve(ix, nq, k, ef, prm, R) != UNIFY_OK) return 0;
  return scratch_layout(ix->dv, nq, k, tile_pcap(R, nq), R.kcq, nullptr, nullptr);
}

// unify_search with caller-provided scratch (at least search_scratch_bytes(nq, k)
// bytes of device memory) and visited pool (null: the index's), for loops that
// must not allocate per call.  A caller's pool is (re)made here for the current
// index size.
int search_impl_scratch(unify_index_t ix, const float* queries, int64_t nq, const int64_t* l, const int64_t* h,
                        int32_t k, int32_t ef, const int8_t* strategy, const unify_params* prm, int64_t* out_ids,
                        float* out_dist, int8_t* out_strategy, int32_t* out_stats, void* scratch,
                        size_t scratch_bytes, VisitPool* pool, void* stream) {
  if (!ix) {
    set_error("null index");
    return UNIFY_EINVAL;
  }
  std::shared_lock<std::shared_mutex> version(ix->version_mu);
  Resolved R;
  int rc = resolve(ix, nq, k, ef, prm, R);
  if (rc != UNIFY_OK) return rc;
  if (nq == 0) return UNIFY_OK;
  // the record budget of the matrix-core scan shrinks to what the scratch holds
  int64_t pcap = tile_pcap(R, nq);
  while (pcap > 0 && scratch_layout(ix->dv, nq, k, pcap, R.kcq, nullptr, nullptr) > scratch_bytes) pcap /= 2;
  if (!queries || !l || !h || !out_ids || !out_dist || !scratch ||
      scratch_bytes < scratch_layout(ix->dv, nq, k, pcap, R.kcq, nullptr, nullptr)) {
    set_error("null buffer or scratch too small");
    return UNIFY_EINVAL;
  }
  HIP_OK(hipSetDevice(ix->device));
  rc = ensure_pool(ix);
  if (rc != UNIFY_OK) return rc;
  if (!pool) pool = &ix->pool;
  else if ((rc = pool_ensure(*pool, ix->dv.n)) != UNIFY_OK) return rc;
  Launch X;
  rc = prepare_launch(ix, R, queries, nq, l, h, strategy, out_ids, out_dist, out_strategy, out_stats, scratch, pcap,
                      *pool, X);
  if (rc == UNIFY_OK) rc = make_side_for(pool->side, X);
  if (rc == UNIFY_OK) rc = enqueue_launch(X, reinterpret_cast<hipStream_t>(stream), nullptr, pool->side, pool);
  return rc;
}

size_t noalloc_scratch_bytes() { return NOALLOC_SCRATCH_BYTES; }

// unify_search_ex over the static scratch array: no allocation of any kind.
int search_impl_noalloc(unify_index_t ix, const float* queries, int64_t nq, const int64_t* l, const int64_t* h,
                        int32_t k, int32_t ef, const int8_t* strategy, const unify_params* prm, int64_t* out_ids,
                        float* out_dist, int8_t* out_strategy, int32_t* out_stats, void* stream) {
  if (!ix) {
    set_error("null index");
    return UNIFY_EINVAL;
  }
  std::shared_lock<std::shared_mutex> version(ix->version_mu);
  Resolved R;
  int rc = resolve(ix, nq, k, ef, prm, R);
  if (rc != UNIFY_OK) return rc;
  R.flags &= ~(uint32_t)UNIFY_FLAG_TIMING;  // timing events would be created on first use
  if (nq == 0) return UNIFY_OK;
  if (!queries || !l || !h || !out_ids || !out_dist) {
    set_error("null buffer");
    return UNIFY_EINVAL;
  }
  int64_t pcap = tile_pcap(R, nq);
  while (pcap > 0 && scratch_layout(ix->dv, nq, k, pcap, R.kcq, nullptr, nullptr) > NOALLOC_SCRATCH_BYTES) pcap /= 2;
  const size_t need = scratch_layout(ix->dv, nq, k, pcap, R.kcq, nullptr, nullptr);
  if (need > NOALLOC_SCRATCH_BYTES) {
    set_error("unify_search_ex_noalloc: " + std::to_string(nq) + " queries with k = " + std::to_string(k) +
              " need " + std::to_string(need) + " bytes of scratch, more than the static " +
              std::to_string(NOALLOC_SCRATCH_BYTES) + "; split the batch");
    return UNIFY_EINVAL;
  }
  if (!ix->pool.rows || ix->pool.n != ix->dv.n || !ix->pool.last) {
    set_error("the index has no visited-set memory");
    return UNIFY_EINVAL;
  }
  HIP_OK(hipSetDevice(ix->device));
  void* scratch = nullptr;
  rc = noalloc_scratch(ix->device, &scratch);
  if (rc != UNIFY_OK) return rc;
  Launch X;
  rc = prepare_launch(ix, R, queries, nq, l, h, strategy, out_ids, out_dist, out_strategy, out_stats, scratch, pcap,
                      ix->pool, X, nullptr, nullptr, false);
  if (rc == UNIFY_OK)
    rc = enqueue_launch(X, reinterpret_cast<hipStream_t>(stream), nullptr, ix->pool.side, &ix->pool, true);
  return rc;
}

// ---------------------------------------------------------------------------
// Batched form: every buffer allocated once, the launch sequence captured into
// a HIP graph and replayed.
// ---------------------------------------------------------------------------

int batch_create(unify_index_t ix, const float* queries, int64_t nq, const int64_t* l, const int64_t* h, int32_t k,
                 int32_t ef, const int8_t* strategy, const unify_params* prm, int64_t* out_ids, float* out_dist,
                 int8_t* out_strategy, int32_t* out_stats, unify_batch_t* out) {
  if (!out || !ix) {
    set_error("null index or output");
    return UNIFY_EINVAL;
  }
  std::shared_lock<std::shared_mutex> version(ix->version_mu);
  Resolved R;
  int rc = resolve(ix, nq, k, ef, prm, R);
  if (rc != UNIFY_OK) return rc;
  if (nq < 1 || !queries || !l || !h || !out_ids || !out_dist) {
    set_error("a batch needs nq >= 1 and its query and output buffers");
    return UNIFY_EINVAL;
  }
  R.flags &= ~(uint32_t)UNIFY_FLAG_TIMING;
  HIP_OK(hipSetDevice(ix->device));
  rc = ensure_pool(ix);
  if (rc != UNIFY_OK) return rc;
  unify_batch_t b = new unify_batch();
  b->ix = ix;
  b->version = ix->version;
  auto fail = [&](int code, const char* msg) {
    set_error(msg);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->scratch) (void)hipFree(b->scratch);
    free_side(b->side);
    delete b;
    return code;
  };
  const int64_t pcap = tile_pcap(R, nq);
  if (hipMalloc(&b->scratch, scratch_layout(ix->dv, nq, k, pcap, R.kcq, nullptr, nullptr)) != hipSuccess)
    return fail(UNIFY_ENOMEM, "device allocation failed (batch scratch)");
  Launch X;
  rc = prepare_launch(ix, R, queries, nq, l, h, strategy, out_ids, out_dist, out_strategy, out_stats, b->scratch,
                      pcap, ix->pool, X);
  if (rc != UNIFY_OK) return fail(rc, "batch preparation failed");
  if (make_side_for(b->side, X) != UNIFY_OK) return fail(UNIFY_EDEVICE, "side stream creation failed");
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
    return fail(UNIFY_EDEVICE, "hipStreamCreate failed");
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    rc = enqueue_launch(X, cs, nullptr, b->side);
    const hipError_t e2 = hipStreamEndCapture(cs, &b->graph);
    if (e2 != hipSuccess) e = e2;
  }
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess || rc != UNIFY_OK) return fail(UNIFY_EDEVICE, "capturing the search into a graph failed");
  if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
    return fail(UNIFY_EDEVICE, "hipGraphInstantiate failed");
  *out = b;
  return UNIFY_OK;
}

int batch_run(unify_batch_t b, void* stream) {
  if (!b) {
    set_error("null batch");
    return UNIFY_EINVAL;
  }
  HIP_OK(hipSetDevice(b->ix->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  unify_index_t ix = b->ix;
  std::shared_lock<std::shared_mutex> version(ix->version_mu);
  if (b->version != ix->version) {
    set_error("the index changed (objects were inserted) after this batch was created: create it again");
    return UNIFY_EINVAL;
  }
  std::lock_guard<std::mutex> g(ix->pool.mu);
  HIP_OK(hipStreamWaitEvent(st, ix->pool.last, 0));
  HIP_OK(hipGraphLaunch(b->exec, st));
  HIP_OK(hipEventRecord(ix->pool.last, st));
  return UNIFY_OK;
}

}  // namespace unify
