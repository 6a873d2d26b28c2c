// TEST INFRASTRUCTURE -- NOT PART OF THE PRODUCT.
//
// Plain, slow CPU reference of the HSIG index of UNIFY (Liang, Zhang, Yao,
// Chen, Song, Cheng, "UNIFY: Unified Index for Range Filtered Approximate
// Nearest Neighbors Search", PVLDB 18(4), 2024).  Only the test suite, the
// smoke check and the CPU-baseline leg of the benchmark may load this code; the
// product library shares nothing with it.
//
// What it computes, and where the paper defines it:
//   * attribute segmentation by an equi-depth histogram        (Sec. 3.1; Example 2 of Sec. 3.2)
//   * level draw of an inserted object                          (Alg. 6, "HSIGInsert")
//   * Prune heuristic                                           (Sec. 2.2, text after Alg. 3)
//   * ANNSearch on one layer                                    (Alg. 1)
//   * BackboneConnectionsBuild                                  (Alg. 4)
//   * skip-list connections (Pugh's insertion)                  (Sec. 4.1, "Fusing Skip List Connections")
//   * GlobalEdgeMasking                                         (Alg. 5)
//   * HSIGInsert                                                (Alg. 6)
//   * plain HNSW InsertLayer, for the S = 1 reduction           (Alg. 3)
//   * search strategies A (pre), B (post), C (hybrid, Alg. 7),
//     the hierarchical scheme (Alg. 2) and the range-aware
//     selection rule                                            (Sec. 4.2)
//
// Readings of passages the paper leaves open (each is listed in the design notes):
//   R1  segment boundaries b_j = attr_sorted[floor(j n / S)], j = 1..S-1; segment j
//       is [b_j, b_{j+1}); an object equal to a boundary goes to the higher segment.
//   R2  level = floor(-ln(U) * mL) with U in (0,1] and mL = 1/ln(M); the printed
//       formula places mL inside the logarithm, which is taken as a typesetting slip.
//   R3  one chunk capacity per layer: M0 on layer 0 (default M0 = M), M above.
//   R4  Prune: candidates sorted by (distance, id); r is dropped when an already
//       selected e has d(e, r) < d(v, r) (strict); no refill of pruned candidates.
//   R5  chunks stay sorted by (distance to owner, id) after every insert and prune,
//       since the hybrid search takes the first entries of each chunk.
//   R6  HSIGInsert visits every segment; an empty segment is skipped; when the new
//       object's level exceeds a segment's top level, it connects only on the layers
//       that segment has; the entry of segment j changes only when j is the object's
//       own segment and its level is higher than the segment's top level.
//   R7  global-edge marks are kept as target ids; a mark is dropped when its target
//       is pruned out of the owner's chunks; Alg. 5's re-prune runs over all chunks.
//   R8  the global entry is the first object to reach the global top level.
//   R9  build distances are FP64; search distances are the canonical FP32 distance
//       (dist32 below), so that a GPU implementation can match them bit for bit.
//   R10 every comparison of two objects by distance uses the key (distance, id).
//   R11 hybrid search: the entry is the entry of the active segment with the highest
//       top level (ties: nearer to q, then smaller id); upper layers run the k = 1
//       search over the active chunks with no range test; on layer 0 the entry goes
//       into cand always and into ann only when in range; while ann holds fewer than
//       ef objects its worst distance counts as +infinity; the active segments are
//       those holding at least one in-range object; a chunk shorter than
//       ceil(m/S') contributes all its entries.
//   R12 strategy rule: pre when Y <= floor(tau_A n), post when Y >= ceil(tau_B n),
//       hybrid otherwise (tau_A = 1%, tau_B = 50%).
//   R13 beam width p (an extension for parallel hardware): pop up to p candidates
//       that pass the stopping test, expand them as one batch whose admission test
//       uses the threshold from before the batch.  For p = 1 this gives the same
//       result as the sequential loop of Alg. 7; the tests check that.
//   R14 low-precision stores (not in the paper): the graph searches may rank by
//       distances to a BF16 copy (nearest, ties to even) or an FP8 E4M3 copy
//       (scale max|x|/448 per vector, nearest code, ties to even, clamp at 448);
//       the first 4k in-range results (k = results wanted) are then re-scored with
//       the FP32 distance.  The pre-filter scan stays exact.
//
// Pins (tests/test_oracle_*.py): Definition 1 and Eq. 1 by hand examples and a
// library routine; dist32 by exact integer cases, a crafted rounding case and
// the FP64 error bound; the level law P(level >= l) = M^-l; Prune by hand-built
// cases; Example 2's segments; the S = 1 build against an independent HNSW
// (Alg. 1 and Alg. 3 written separately in the tests) edge for edge; a
// six-object, two-segment build traced by hand through Alg. 4-6 (forward and
// reverse edges, the re-prune of an overflowing chunk, every global-edge mark,
// a mark dropped with its edge); the whole build (chunks, marks, entries)
// against an independent HSIGInsert on integer grids full of distance ties; the
// hybrid entry rule on an index whose two segments share the top level;
// single-segment inclusiveness = 1 and > 80% on 1..8 segments (Sec. 5.4);
// Theorem 1 on this code's exact range search; layer search with ef >= n =
// brute force over the reachable set; pre-filter = exact k-NN; the skip-list
// walk = the attribute slice; the beam form at p = 1 = the sequential loop; the
// BF16 and E4M3 roundings against a library's conversions, every E4M3 code's
// value, and a low-precision search on vectors both formats hold exactly = the
// FP32 search.  Parity unpinned: none of the build's steps; the graphs of the
// large synthetic workloads are checked only by invariants and recall (no
// printed graph exists), which is enough for search parity because the GPU and
// this code search the same file.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <queue>
#include <string>
#include <vector>

namespace {

typedef std::pair<double, int> DI;  // (FP64 distance, id): build-side key
typedef std::pair<float, int> FI;   // (FP32 distance, internal id): search-side key

// ---------------------------------------------------------------------------
// Distances
// ---------------------------------------------------------------------------

// Squared Euclidean distance in FP64 (the paper uses Euclidean distance, Sec. 5.1).
double dist64(const float* a, const float* b, int d) {
  double s = 0.0;
  for (int t = 0; t < d; ++t) {
    double e = (double)a[t] - (double)b[t];
    s += e * e;
  }
  return s;
}

// Canonical FP32 squared distance: e_t = x_t - q_t rounded to FP32; sixteen
// partial sums, partial p takes the 4-element groups g with g mod 16 == p in
// increasing order, each element accumulated with a fused multiply-add; then
// a butterfly P[i] + P[i ^ s] for s = 8, 4, 2, 1.  d must be a multiple of 4.
float dist32(const float* q, const float* x, int d) {
  float P[16];
  for (int i = 0; i < 16; ++i) P[i] = 0.0f;
  const int G = d / 4;
  for (int g = 0; g < G; ++g) {
    float& acc = P[g % 16];
    for (int t = 4 * g; t < 4 * g + 4; ++t) {
      float e = x[t] - q[t];
      acc = std::fma(e, e, acc);
    }
  }
  for (int s = 8; s >= 1; s >>= 1) {
    float T[16];
    for (int i = 0; i < 16; ++i) T[i] = P[i] + P[i ^ s];
    for (int i = 0; i < 16; ++i) P[i] = T[i];
  }
  return P[0];
}

// ---------------------------------------------------------------------------
// Low-precision copies of the vectors (an extension for bandwidth-bound
// hardware; the paper computes plain Euclidean distances, Sec. 5.1).  A graph
// search may rank objects by distances to rounded copies and then re-score its
// best results with the exact FP32 distance.  Each rounding below is written as
// "pick the nearest representable value" over the format's value set, which is
// slow but follows the formats' definitions directly.
// ---------------------------------------------------------------------------

// Value of a non-negative FP32 bit pattern, with the pattern just past the
// largest finite one read as 2^128 (the next step of the significand grid).
double f32_bits_value(uint32_t b) {
  if (b >= 0x7F800000u) return std::ldexp(1.0, 128);
  float f;
  std::memcpy(&f, &b, 4);
  return (double)f;
}

// bfloat16 = the upper 16 bits of an FP32 pattern.  Nearest bfloat16 to x,
// ties to the even significand; returns its bit pattern.
uint16_t bf16_nearest(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if (std::isnan(x)) return (uint16_t)((u >> 16) | 0x0040u);
  const uint32_t sign = u & 0x80000000u, mag = u & 0x7FFFFFFFu;
  if (mag == 0x7F800000u) return (uint16_t)(u >> 16);  // infinities stay
  const uint32_t lo = mag & 0xFFFF0000u, hi = lo + 0x10000u;  // the two bfloat16 neighbours of |x|
  const double a = (double)std::fabs(x), dlo = a - f32_bits_value(lo), dhi = f32_bits_value(hi) - a;
  uint32_t pick;
  if (dlo < dhi) pick = lo;
  else if (dhi < dlo) pick = hi;
  else pick = ((lo >> 16) & 1u) ? hi : lo;  // tie: even significand
  return (uint16_t)((sign | pick) >> 16);
}

float bf16_value(uint16_t b) {
  uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// OCP 8-bit E4M3 ("fn" variant): sign, 4 exponent bits (bias 7), 3 significand
// bits; exponent field 0 holds subnormals m * 2^-9; no infinities; S.1111.111
// is NaN; the largest finite magnitude is 1.75 * 2^8 = 448.
double e4m3_value(uint8_t c) {
  const int e = (c >> 3) & 15, m = c & 7;
  double mag;
  if (e == 15 && m == 7) mag = std::numeric_limits<double>::quiet_NaN();
  else if (e == 0) mag = std::ldexp((double)m, -9);
  else mag = std::ldexp(1.0 + m / 8.0, e - 7);
  return (c & 0x80) ? -mag : mag;
}

// Nearest E4M3 code to y, ties to the even significand; magnitudes beyond 448
// clamp to 448 (reading: a per-vector scale keeps |y| <= 448 up to the rounding
// of the division).  Codes 0x00..0x7E have increasing values.
uint8_t e4m3_nearest(float y) {
  if (std::isnan(y)) return 0x7F;
  const uint8_t sign = std::signbit(y) ? 0x80 : 0x00;
  const double a = std::fabs((double)y);
  if (a >= 448.0) return sign | 0x7E;
  int lo = 0, hi = 0x7E;  // largest code with value <= a
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (e4m3_value((uint8_t)mid) <= a) lo = mid;
    else hi = mid - 1;
  }
  const double dlo = a - e4m3_value((uint8_t)lo), dhi = e4m3_value((uint8_t)(lo + 1)) - a;
  int pick;
  if (dlo < dhi) pick = lo;
  else if (dhi < dlo) pick = lo + 1;
  else pick = (lo & 1) ? lo + 1 : lo;  // tie: even significand (the code's last bit)
  return sign | (uint8_t)pick;
}

// FP8 copy of one vector: scale s = max_t |x_t| / 448 (1 for a zero vector),
// codes of x_t / s, read back as e4m3_value(code) * s in FP32.
float fp8_row(const float* x, int d, uint8_t* codes, float* back) {
  float mx = 0.0f;
  for (int t = 0; t < d; ++t) mx = std::max(mx, std::fabs(x[t]));
  const float s = mx > 0.0f ? mx / 448.0f : 1.0f;
  for (int t = 0; t < d; ++t) {
    codes[t] = e4m3_nearest(x[t] / s);
    back[t] = (float)e4m3_value(codes[t]) * s;
  }
  return s;
}

// Level of an inserted object (Alg. 6, second step; reading R2).
int draw_level(double u, double mL) {
  double lv = std::floor(-std::log(u) * mL);
  return (int)std::min(lv, 30.0);
}

// ---------------------------------------------------------------------------
// Build (external ids, dynamic adjacency)
// ---------------------------------------------------------------------------

struct Builder {
  int64_t n = 0;
  int d = 0, S = 1, M = 16, M0 = 16, efCons = 100;
  double mL = 0.0;
  bool hnsw_mode = false;  // plain HNSW (Alg. 3): one segment, no masking
  std::vector<float> X;        // [n][d], row = external id
  std::vector<int64_t> attr;   // [n]
  std::vector<int64_t> bnd;    // b_1 .. b_{S-1}
  std::vector<int> seg, level;
  // adj[v][l][j] = chunk j of v on layer l, sorted by (distance to v, id)
  std::vector<std::vector<std::vector<std::vector<DI>>>> adj;
  // marks[v][l] = global-edge targets of v on layer l (sorted ids)
  std::vector<std::vector<std::vector<int>>> marks;
  std::vector<int> entry, maxlev;  // per segment
  int gentry = -1, gmax = -1;
  // skip list: next[v][l]; the head is a separate array
  std::vector<std::vector<int>> next;
  std::vector<int> head_next;
  // visited stamps for ANNSearch
  std::vector<uint32_t> stamp;
  uint32_t cur = 0;
  int64_t n_inserted = 0;

  const float* vec(int v) const { return &X[(size_t)v * d]; }
  double dv(int a, int b) const { return dist64(vec(a), vec(b), d); }
  int cap(int l) const { return l == 0 ? M0 : M; }

  void new_visit() {
    if (++cur == 0) {
      std::fill(stamp.begin(), stamp.end(), 0u);
      cur = 1;
    }
  }
  bool seen(int v) const { return stamp[v] == cur; }
  void see(int v) { stamp[v] = cur; }

  int seg_of(int64_t a) const {
    return (int)(std::upper_bound(bnd.begin(), bnd.end(), a) - bnd.begin());
  }

  // Prune heuristic (Sec. 2.2): candidates sorted by distance to v; r is
  // dropped when some already selected e is closer to r than v is.
  std::vector<DI> prune(int v, std::vector<DI> cands, int Mcap) const {
    std::sort(cands.begin(), cands.end());
    std::vector<DI> out;
    for (const DI& r : cands) {
      if ((int)out.size() >= Mcap) break;
      if (r.second == v) continue;
      bool keep = true;
      for (const DI& e : out) {
        if (dv(e.second, r.second) < r.first) {
          keep = false;
          break;
        }
      }
      if (keep) out.push_back(r);
    }
    return out;
  }

  // Alg. 1 (ANNSearch) on layer l, restricted to the sub-graph of segment j:
  // nodes of segment j, edges of their chunk j.
  std::vector<DI> ann_search(const float* q, int ep, int ef, int l, int j) {
    new_visit();
    std::priority_queue<DI, std::vector<DI>, std::greater<DI>> cand;
    std::priority_queue<DI> ann;
    DI e0(dist64(q, vec(ep), d), ep);
    cand.push(e0);
    ann.push(e0);
    see(ep);
    while (!cand.empty()) {
      DI o = cand.top();
      cand.pop();
      if (o > ann.top()) break;
      for (const DI& nb : adj[o.second][l][j]) {
        int v = nb.second;
        if (seen(v)) continue;
        see(v);
        DI kv(dist64(q, vec(v), d), v);
        if ((int)ann.size() < ef || kv < ann.top()) {
          cand.push(kv);
          ann.push(kv);
          if ((int)ann.size() > ef) ann.pop();
        }
      }
    }
    std::vector<DI> out;
    while (!ann.empty()) {
      out.push_back(ann.top());
      ann.pop();
    }
    std::reverse(out.begin(), out.end());
    return out;
  }

  // Removes the marks of v on layer l whose target is no longer in v's chunks.
  void drop_stale_marks(int v, int l, const std::vector<DI>& removed_from) {
    (void)removed_from;
    std::vector<int>& mk = marks[v][l];
    std::vector<int> keep;
    for (int t : mk) {
      bool present = false;
      for (const auto& ch : adj[v][l])
        for (const DI& e : ch)
          if (e.second == t) present = true;
      if (present) keep.push_back(t);
    }
    mk.swap(keep);
  }

  // Inserts (key) into a chunk that is kept sorted (R5).
  static void sorted_insert(std::vector<DI>& ch, DI key) {
    ch.insert(std::upper_bound(ch.begin(), ch.end(), key), key);
  }

  // Alg. 4 (BackboneConnectionsBuild) of object v (segment i) into segment j on layer l.
  std::vector<DI> backbone(int l, int ep, int v, int i, int j) {
    std::vector<DI> ann = ann_search(vec(v), ep, efCons, l, j);
    std::vector<DI> N = prune(v, ann, cap(l));
    adj[v][l][j] = N;  // sorted by (distance to v, id)
    for (const DI& on : N) {
      int o = on.second;
      std::vector<DI>& ch = adj[o][l][i];
      sorted_insert(ch, DI(on.first, v));
      if ((int)ch.size() > cap(l)) {
        std::vector<DI> before = ch;
        ch = prune(o, before, cap(l));
        if (!hnsw_mode) drop_stale_marks(o, l, before);
      }
    }
    return ann;
  }

  std::vector<DI> all_chunks(int v, int l) const {
    std::vector<DI> c;
    for (const auto& ch : adj[v][l]) c.insert(c.end(), ch.begin(), ch.end());
    std::sort(c.begin(), c.end());
    return c;
  }

  static void set_from(std::vector<int>& mk, const std::vector<DI>& N) {
    mk.clear();
    for (const DI& e : N) mk.push_back(e.second);
    std::sort(mk.begin(), mk.end());
  }

  // Alg. 5 (GlobalEdgeMasking) of object v on layer l.
  void global_mask(int l, int v) {
    std::vector<DI> N = prune(v, all_chunks(v, l), M);
    set_from(marks[v][l], N);
    for (const DI& on : N) {
      int o = on.second;
      bool has_v = false;
      for (const auto& ch : adj[o][l])
        for (const DI& e : ch)
          if (e.second == v) has_v = true;
      if (!has_v) continue;
      std::vector<int>& mk = marks[o][l];
      if (!std::binary_search(mk.begin(), mk.end(), v)) {
        mk.insert(std::upper_bound(mk.begin(), mk.end(), v), v);
      }
      if ((int)mk.size() > M) {
        std::vector<DI> N2 = prune(o, all_chunks(o, l), M);
        set_from(mk, N2);
      }
    }
  }

  // Skip-list insertion (Pugh) with the object's HSIG level as its list height;
  // the order is by (attribute, external id).
  bool before_key(int a, int64_t attr_b, int b) const {
    return attr[a] < attr_b || (attr[a] == attr_b && a < b);
  }
  void skiplist_insert(int v) {
    int lev = level[v];
    if ((int)head_next.size() < lev + 1) head_next.resize(lev + 1, -1);
    next[v].assign(lev + 1, -1);
    int top = (int)head_next.size() - 1;
    int x = -1;  // -1 = head
    for (int l = top; l >= 0; --l) {
      while (true) {
        int nx = (x < 0) ? head_next[l] : next[x][l];
        if (nx >= 0 && before_key(nx, attr[v], v)) x = nx;
        else break;
      }
      if (l <= lev) {
        int nx = (x < 0) ? head_next[l] : next[x][l];
        next[v][l] = nx;
        if (x < 0) head_next[l] = v;
        else next[x][l] = v;
      }
    }
  }

  // Alg. 6 (HSIGInsert); with hnsw_mode it is Alg. 3 per layer with one segment.
  void insert(int v, double u) {
    int i = hnsw_mode ? 0 : seg[v];
    int lev = draw_level(u, mL);
    level[v] = lev;
    adj[v].assign(lev + 1, std::vector<std::vector<DI>>(S));
    marks[v].assign(lev + 1, std::vector<int>());
    for (int j = 0; j < S; ++j) {
      if (entry[j] < 0) {
        if (j == i) {
          entry[j] = v;
          maxlev[j] = lev;
        }
        continue;
      }
      int L = maxlev[j];
      int ep = entry[j];
      for (int l = L; l >= lev + 1; --l) ep = ann_search(vec(v), ep, 1, l, j)[0].second;
      for (int l = std::min(lev, L); l >= 0; --l) {
        std::vector<DI> ann = backbone(l, ep, v, i, j);
        ep = ann[0].second;
      }
      if (j == i && lev > L) {
        entry[j] = v;
        maxlev[j] = lev;
      }
    }
    if (!hnsw_mode) {
      skiplist_insert(v);
      for (int l = 0; l <= lev; ++l) global_mask(l, v);
    }
    if (lev > gmax) {
      gmax = lev;
      gentry = v;
    }
    ++n_inserted;
  }

  // Segment boundaries come from the attributes of the first bnd_n objects (all
  // of them when bnd_n <= 0): the objects present when the index is created.
  void init(const float* X_, const int64_t* attr_, int64_t n_, int d_, int S_, int M_, int M0_,
            int efCons_, double mL_, int64_t bnd_n = 0) {
    n = n_;
    d = d_;
    S = S_;
    M = M_;
    M0 = M0_ > 0 ? M0_ : M_;
    efCons = efCons_;
    mL = mL_ > 0 ? mL_ : 1.0 / std::log((double)M_);
    X.assign(X_, X_ + (size_t)n * d);
    attr.assign(attr_, attr_ + n);
    const int64_t nb = bnd_n > 0 && bnd_n < n ? bnd_n : n;
    std::vector<int64_t> srt(attr.begin(), attr.begin() + nb);
    std::sort(srt.begin(), srt.end());
    bnd.clear();
    for (int j = 1; j < S; ++j) bnd.push_back(srt[(size_t)((int64_t)j * nb / S)]);
    seg.resize(n);
    for (int64_t v = 0; v < n; ++v) seg[v] = seg_of(attr[v]);
    level.assign(n, 0);
    adj.assign(n, {});
    marks.assign(n, {});
    entry.assign(S, -1);
    maxlev.assign(S, -1);
    next.assign(n, {});
    head_next.clear();
    stamp.assign(n, 0u);
    cur = 0;
  }

  // Room for m more objects (external ids n .. n + m - 1); the segment
  // boundaries stay as they are.  HSIGInsert then inserts them (Alg. 6).
  void append(const float* X_, const int64_t* attr_, int64_t m) {
    X.insert(X.end(), X_, X_ + (size_t)m * d);
    attr.insert(attr.end(), attr_, attr_ + m);
    n += m;
    seg.resize(n);
    for (int64_t v = n - m; v < n; ++v) seg[v] = hnsw_mode ? 0 : seg_of(attr[v]);
    level.resize(n, 0);
    adj.resize(n);
    marks.resize(n);
    next.resize(n);
    stamp.resize(n, 0u);
  }
};

// ---------------------------------------------------------------------------
// Frozen view: internal ids = rank in (attribute, external id) order.  It is
// also the content of the index file.
// ---------------------------------------------------------------------------

struct View {
  int64_t n = 0;
  int d = 0, S = 0, M0 = 0, MU = 0, L = -1, gentry = -1, efCons = 0;
  double mL = 0;
  uint64_t seed = 0;
  int64_t R = 0;
  int W0 = 0, WU = 0;
  std::vector<int64_t> attr, ext, seg_start;
  std::vector<int32_t> seg_entry, seg_maxlevel;
  std::vector<uint8_t> level;
  std::vector<int32_t> uprow;
  std::vector<float> X;
  std::vector<int32_t> adj0, adjU;
  std::vector<uint32_t> gbits0, gbitsU;
  // Store the graph searches rank by: empty = X itself; else the values of a
  // BF16 or FP8 copy of X, whose best rerank * k results are re-scored on X.
  std::vector<float> XS;
  int rerank = 0;
  // A second attribute per object (internal order; empty when not set) for
  // conjunctive two-attribute queries (the multi-attribute discussion of Sec. 5.9, approach 1).
  std::vector<int64_t> attr2;
  // sorted sample of attr2 for the strategy rule: the value at rank floor(j n / ns)
  // of the sorted attr2, j < ns = min(n, 2048)
  std::vector<int64_t> attr2_sample;
  // z-order composite attribute (the multi-attribute discussion of Sec. 5.9, approach 2):
  // the index's attribute is the key of the pair (A1, A2); both attributes of every
  // object (internal order; empty when not set), the key map, and the pairs of the
  // objects at internal ids floor(j n / ns), j < ns = min(n, 2048), for the strategy rule.
  std::vector<int64_t> za1, za2, zs1, zs2;
  int64_t zbase1 = 0, zbase2 = 0;
  int zshift1 = 0, zshift2 = 0;

  const float* vec(int v) const { return &X[(size_t)v * d]; }
  const float* svec(int v) const { return XS.empty() ? vec(v) : &XS[(size_t)v * d]; }
  int mcap(int l) const { return l == 0 ? M0 : MU; }
  // Pointer to chunk j of v on layer l (mcap(l) entries, -1 padded).
  const int32_t* chunk(int v, int l, int j) const {
    if (l == 0) return &adj0[((size_t)v * S + j) * M0];
    int64_t row = (int64_t)uprow[v] + (l - 1);
    return &adjU[((size_t)row * S + j) * MU];
  }
  const uint32_t* bits(int v, int l) const {
    if (l == 0) return &gbits0[(size_t)v * W0];
    int64_t row = (int64_t)uprow[v] + (l - 1);
    return &gbitsU[(size_t)row * WU];
  }
  // The global (marked) edges of v on layer l, in bit order.
  void glist(int v, int l, std::vector<int>& out) const {
    out.clear();
    const int mc = mcap(l);
    const uint32_t* b = bits(v, l);
    for (int pos = 0; pos < S * mc; ++pos) {
      if (b[pos >> 5] >> (pos & 31) & 1u) {
        int t = chunk(v, l, pos / mc)[pos % mc];
        if (t >= 0) out.push_back(t);
      }
    }
  }
  // Segment of internal id r (the last j whose start is <= r).
  int seg_of_rank(int64_t r) const {
    return (int)(std::upper_bound(seg_start.begin(), seg_start.end(), r) - seg_start.begin()) - 1;
  }
};

void freeze(const Builder& B, View& V, uint64_t seed) {
  const int64_t n = B.n;
  V.n = n;
  V.d = B.d;
  V.S = B.S;
  V.M0 = B.M0;
  V.MU = B.M;
  V.L = B.gmax;
  V.efCons = B.efCons;
  V.mL = B.mL;
  V.seed = seed;
  std::vector<int> order(n);
  for (int64_t v = 0; v < n; ++v) order[v] = (int)v;
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    return B.attr[a] < B.attr[b] || (B.attr[a] == B.attr[b] && a < b);
  });
  std::vector<int> rank(n);
  for (int64_t r = 0; r < n; ++r) rank[order[r]] = (int)r;
  V.attr.resize(n);
  V.ext.resize(n);
  V.level.resize(n);
  V.uprow.resize(n);
  V.X.resize((size_t)n * B.d);
  int64_t R = 0;
  for (int64_t r = 0; r < n; ++r) {
    int v = order[r];
    V.attr[r] = B.attr[v];
    V.ext[r] = v;
    V.level[r] = (uint8_t)B.level[v];
    V.uprow[r] = B.level[v] > 0 ? (int32_t)R : -1;
    R += B.level[v];
    std::memcpy(&V.X[(size_t)r * B.d], B.vec(v), sizeof(float) * B.d);
  }
  V.R = R;
  V.seg_start.assign(B.S + 1, 0);
  for (int j = 1; j < B.S; ++j)
    V.seg_start[j] = std::lower_bound(V.attr.begin(), V.attr.end(), B.bnd[j - 1]) - V.attr.begin();
  V.seg_start[B.S] = n;
  V.seg_entry.resize(B.S);
  V.seg_maxlevel.resize(B.S);
  for (int j = 0; j < B.S; ++j) {
    V.seg_entry[j] = B.entry[j] >= 0 ? rank[B.entry[j]] : -1;
    V.seg_maxlevel[j] = B.maxlev[j];
  }
  V.gentry = B.gentry >= 0 ? rank[B.gentry] : -1;
  V.W0 = (B.S * B.M0 + 31) / 32;
  V.WU = (B.S * B.M + 31) / 32;
  V.adj0.assign((size_t)n * B.S * B.M0, -1);
  V.gbits0.assign((size_t)n * V.W0, 0u);
  V.adjU.assign((size_t)R * B.S * B.M, -1);
  V.gbitsU.assign((size_t)R * V.WU, 0u);
  for (int64_t r = 0; r < n; ++r) {
    int v = order[r];
    for (int l = 0; l <= B.level[v]; ++l) {
      int mc = l == 0 ? B.M0 : B.M;
      int32_t* rowp = l == 0 ? &V.adj0[(size_t)r * B.S * mc]
                             : &V.adjU[(size_t)(V.uprow[r] + l - 1) * B.S * mc];
      uint32_t* bp = l == 0 ? &V.gbits0[(size_t)r * V.W0] : &V.gbitsU[(size_t)(V.uprow[r] + l - 1) * V.WU];
      for (int j = 0; j < B.S; ++j) {
        const auto& ch = B.adj[v][l][j];
        for (size_t t = 0; t < ch.size(); ++t) {
          rowp[j * mc + t] = rank[ch[t].second];
          if (!B.hnsw_mode && std::binary_search(B.marks[v][l].begin(), B.marks[v][l].end(), ch[t].second)) {
            int pos = j * mc + (int)t;
            bp[pos >> 5] |= 1u << (pos & 31);
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Index file (little-endian; 256-byte header; sections 64-byte aligned; CRC-32 footer)
// ---------------------------------------------------------------------------

uint32_t crc32_update(uint32_t c, const uint8_t* p, size_t len) {
  static uint32_t table[256];
  static bool ready = false;
  if (!ready) {
    for (uint32_t i = 0; i < 256; ++i) {
      uint32_t x = i;
      for (int k = 0; k < 8; ++k) x = (x & 1) ? (0xEDB88320u ^ (x >> 1)) : (x >> 1);
      table[i] = x;
    }
    ready = true;
  }
  for (size_t i = 0; i < len; ++i) c = table[(c ^ p[i]) & 0xFFu] ^ (c >> 8);
  return c;
}

struct Writer {
  FILE* f;
  uint32_t crc = 0xFFFFFFFFu;
  uint64_t off = 0;
  bool ok = true;
  void put(const void* p, size_t len) {
    if (len == 0) return;
    if (fwrite(p, 1, len, f) != len) ok = false;
    crc = crc32_update(crc, (const uint8_t*)p, len);
    off += len;
  }
  void align() {
    static const uint8_t z[64] = {0};
    size_t pad = (size_t)((64 - off % 64) % 64);
    put(z, pad);
  }
};

struct Header {
  char magic[8];
  uint32_t version, flags;
  int64_t n;
  int32_t d, S, M0, MU, L, efCons, gentry, reserved;
  double mL;
  uint64_t seed;
  int64_t R;
  int32_t W0, WU;
  uint8_t pad[256 - 8 - 8 - 8 - 32 - 8 - 8 - 8 - 8];
};
static_assert(sizeof(Header) == 256, "header is 256 bytes");

int write_view(const View& V, const char* path) {
  FILE* f = fopen(path, "wb");
  if (!f) return -5;
  Writer w{f};
  Header h;
  std::memset(&h, 0, sizeof h);
  std::memcpy(h.magic, "UNIFYIX1", 8);
  h.version = 1;
  h.n = V.n;
  h.d = V.d;
  h.S = V.S;
  h.M0 = V.M0;
  h.MU = V.MU;
  h.L = V.L;
  h.efCons = V.efCons;
  h.gentry = V.gentry;
  h.mL = V.mL;
  h.seed = V.seed;
  h.R = V.R;
  h.W0 = V.W0;
  h.WU = V.WU;
  w.put(&h, sizeof h);
  auto sec = [&](const void* p, size_t len) {
    w.align();
    w.put(p, len);
  };
  sec(V.attr.data(), 8 * V.n);
  sec(V.ext.data(), 8 * V.n);
  sec(V.seg_start.data(), 8 * (V.S + 1));
  sec(V.seg_entry.data(), 4 * V.S);
  sec(V.seg_maxlevel.data(), 4 * V.S);
  sec(V.level.data(), V.n);
  sec(V.uprow.data(), 4 * V.n);
  sec(V.X.data(), 4 * V.X.size());
  sec(V.adj0.data(), 4 * V.adj0.size());
  sec(V.gbits0.data(), 4 * V.gbits0.size());
  sec(V.adjU.data(), 4 * V.adjU.size());
  sec(V.gbitsU.data(), 4 * V.gbitsU.size());
  w.align();
  uint32_t crc = w.crc ^ 0xFFFFFFFFu;
  bool ok = w.ok && fwrite(&crc, 4, 1, f) == 1;
  ok = (fclose(f) == 0) && ok;
  return ok ? 0 : -5;
}

struct Reader {
  std::vector<uint8_t> buf;
  size_t pos = 0;
  bool ok = true;
  void get(void* p, size_t len) {
    if (pos + len > buf.size()) {
      ok = false;
      return;
    }
    if (len) std::memcpy(p, &buf[pos], len);
    pos += len;
  }
  void align() { pos = (pos + 63) / 64 * 64; }
};

int read_view(const char* path, View& V) {
  FILE* f = fopen(path, "rb");
  if (!f) return -5;
  Reader rd;
  fseek(f, 0, SEEK_END);
  long sz = ftell(f);
  fseek(f, 0, SEEK_SET);
  if (sz < (long)sizeof(Header) + 4) {
    fclose(f);
    return -6;
  }
  rd.buf.resize(sz);
  size_t got = fread(rd.buf.data(), 1, sz, f);
  fclose(f);
  if (got != (size_t)sz) return -5;
  uint32_t stored;
  std::memcpy(&stored, &rd.buf[sz - 4], 4);
  uint32_t crc = crc32_update(0xFFFFFFFFu, rd.buf.data(), sz - 4) ^ 0xFFFFFFFFu;
  Header h;
  rd.get(&h, sizeof h);
  if (std::memcmp(h.magic, "UNIFYIX1", 8) != 0 || h.version != 1) return -6;
  if (crc != stored) return -6;
  if (h.n < 1 || h.d < 4 || h.d % 4 || h.S < 1 || h.M0 < 1 || h.MU < 1 || h.R < 0) return -6;
  V.n = h.n;
  V.d = h.d;
  V.S = h.S;
  V.M0 = h.M0;
  V.MU = h.MU;
  V.L = h.L;
  V.efCons = h.efCons;
  V.gentry = h.gentry;
  V.mL = h.mL;
  V.seed = h.seed;
  V.R = h.R;
  V.W0 = h.W0;
  V.WU = h.WU;
  auto sec = [&](auto& vec, size_t count) {
    rd.align();
    vec.resize(count);
    rd.get(vec.data(), count * sizeof(vec[0]));
  };
  sec(V.attr, V.n);
  sec(V.ext, V.n);
  sec(V.seg_start, V.S + 1);
  sec(V.seg_entry, V.S);
  sec(V.seg_maxlevel, V.S);
  sec(V.level, V.n);
  sec(V.uprow, V.n);
  sec(V.X, (size_t)V.n * V.d);
  sec(V.adj0, (size_t)V.n * V.S * V.M0);
  sec(V.gbits0, (size_t)V.n * V.W0);
  sec(V.adjU, (size_t)V.R * V.S * V.MU);
  sec(V.gbitsU, (size_t)V.R * V.WU);
  rd.align();
  if (!rd.ok || rd.pos + 4 != rd.buf.size()) return -6;
  return 0;
}

// ---------------------------------------------------------------------------
// Search (O2) on a view
// ---------------------------------------------------------------------------

enum { ST_AUTO = 0, ST_PRE = 1, ST_HYBRID = 2, ST_POST = 3 };
enum { C_NDIST = 0, C_NEXP, C_NVISIT0, C_MAXCAND, C_MAXLIVE, C_STRAT, C_LO, C_HI, C_NRERANK, C_ENTRY, C_NCOUNT };

struct Query {
  const View* V;
  const float* q;
  int64_t lo = 0, hi = 0;  // in-range internal ids are [lo, hi)
  int64_t l = 0, h = 0;    // inclusive attribute range
  int a = 0, b = -1;       // active segments
  int c = 0;               // entries per active chunk (selection S2)
  int m = 0;               // neighbours per expansion (selection S1)
  bool s1 = false;         // hybrid neighbour selection S1 instead of S2
  bool multi = false;      // also require l2 <= attr2 <= h2 (conjunctive query)
  int64_t l2 = 0, h2 = 0;
  bool box = false;        // z-order index: require l1 <= A1 <= h1 and l2 <= A2 <= h2
  int64_t l1 = 0, h1 = 0;
  int64_t* cnt;
  bool second_ok(int v) const {
    if (box) return V->za1[v] >= l1 && V->za1[v] <= h1 && V->za2[v] >= l2 && V->za2[v] <= h2;
    return !multi || (V->attr2[v] >= l2 && V->attr2[v] <= h2);
  }
  // the filter of Alg. 7 (its ann admission) and of the post-filter: every range of the query
  bool in_range(int v) const { return V->attr[v] >= l && V->attr[v] <= h && second_ok(v); }
  // distance in the store the graph searches use
  FI key(int v) {
    ++cnt[C_NDIST];
    return FI(dist32(q, V->svec(v), V->d), v);
  }
  // exact FP32 distance
  FI xkey(int v) const { return FI(dist32(q, V->vec(v), V->d), v); }
};

// Neighbours of o on layer l: the first c entries of each active chunk (hybrid),
// or the marked global edges (post).
// Hybrid selections (Sec. 4.2): S2 (default) takes the first ceil(m / S') entries of
// each active chunk; S1 ranks every entry of the active chunks by its distance
// to o and takes the m nearest (key (distance, id); distances in the search's
// store, o's copy standing in for the query).
void neighbours(const Query& Q, bool hybrid, int o, int l, std::vector<int>& out) {
  out.clear();
  if (hybrid && Q.s1) {
    const int mc = Q.V->mcap(l);
    std::vector<FI> all;
    for (int j = Q.a; j <= Q.b; ++j) {
      const int32_t* ch = Q.V->chunk(o, l, j);
      for (int r = 0; r < mc; ++r)
        if (ch[r] >= 0) all.push_back(FI(dist32(Q.V->svec(o), Q.V->svec(ch[r]), Q.V->d), ch[r]));
    }
    std::sort(all.begin(), all.end());
    for (size_t i = 0; i < all.size() && (int)i < Q.m; ++i) out.push_back(all[i].second);
  } else if (hybrid) {
    const int mc = Q.V->mcap(l);
    for (int j = Q.a; j <= Q.b; ++j) {
      const int32_t* ch = Q.V->chunk(o, l, j);
      for (int r = 0; r < Q.c && r < mc; ++r)
        if (ch[r] >= 0) out.push_back(ch[r]);
    }
  } else {
    Q.V->glist(o, l, out);
  }
}

// One layer, sequential (Alg. 1 for post and the upper layers; Alg. 7 on layer
// 0 of the hybrid search).  Returns ann sorted by key.
std::vector<FI> layer_seq(Query& Q, bool hybrid, bool filter, int ep, int l, int ef,
                          std::vector<uint32_t>& stamp, uint32_t& cur) {
  if (++cur == 0) {
    std::fill(stamp.begin(), stamp.end(), 0u);
    cur = 1;
  }
  std::priority_queue<FI, std::vector<FI>, std::greater<FI>> cand;
  std::priority_queue<FI> ann;
  FI e0 = Q.key(ep);
  stamp[ep] = cur;
  cand.push(e0);
  if (!filter || Q.in_range(ep)) ann.push(e0);
  int64_t nvisit = 1;
  std::vector<int> nb;
  while (!cand.empty()) {
    FI o = cand.top();
    cand.pop();
    if ((int)ann.size() == ef && o > ann.top()) break;
    ++Q.cnt[C_NEXP];
    neighbours(Q, hybrid, o.second, l, nb);
    for (int v : nb) {
      if (stamp[v] == cur) continue;
      stamp[v] = cur;
      ++nvisit;
      FI kv = Q.key(v);
      if ((int)ann.size() < ef || kv < ann.top()) {
        cand.push(kv);
        if (!filter || Q.in_range(v)) {
          ann.push(kv);
          if ((int)ann.size() > ef) ann.pop();
        }
      }
    }
    Q.cnt[C_MAXCAND] = std::max<int64_t>(Q.cnt[C_MAXCAND], (int64_t)cand.size());
  }
  if (l == 0) Q.cnt[C_NVISIT0] = nvisit;
  std::vector<FI> out;
  while (!ann.empty()) {
    out.push_back(ann.top());
    ann.pop();
  }
  std::reverse(out.begin(), out.end());
  return out;
}

// Layer 0 with beam width p (R13).  For p == 1 the result equals layer_seq.
std::vector<FI> layer_beam(Query& Q, bool hybrid, bool filter, int ep, int ef, int p,
                           std::vector<uint32_t>& stamp, uint32_t& cur) {
  if (++cur == 0) {
    std::fill(stamp.begin(), stamp.end(), 0u);
    cur = 1;
  }
  std::priority_queue<FI, std::vector<FI>, std::greater<FI>> cand;
  std::priority_queue<FI> ann;
  FI e0 = Q.key(ep);
  stamp[ep] = cur;
  cand.push(e0);
  if (!filter || Q.in_range(ep)) ann.push(e0);
  int64_t nvisit = 1;
  std::vector<int> nb, batch;
  std::vector<int> popped;
  while (!cand.empty()) {
    popped.clear();
    while ((int)popped.size() < p && !cand.empty()) {
      FI o = cand.top();
      if ((int)ann.size() == ef && o > ann.top()) break;
      cand.pop();
      popped.push_back(o.second);
    }
    if (popped.empty()) break;
    const bool full = (int)ann.size() == ef;
    const FI T = full ? ann.top() : FI(0.f, 0);
    batch.clear();
    for (int o : popped) {
      ++Q.cnt[C_NEXP];
      neighbours(Q, hybrid, o, 0, nb);
      for (int v : nb) {
        if (stamp[v] == cur) continue;
        stamp[v] = cur;
        ++nvisit;
        batch.push_back(v);
      }
    }
    for (int v : batch) {
      FI kv = Q.key(v);
      if (!full || kv < T) {
        cand.push(kv);
        if (!filter || Q.in_range(v)) ann.push(kv);
      }
    }
    while ((int)ann.size() > ef) ann.pop();
    Q.cnt[C_MAXCAND] = std::max<int64_t>(Q.cnt[C_MAXCAND], (int64_t)cand.size());
    // live entries: those the search can still expand
    if ((int)ann.size() == ef) {
      int64_t live = 0;
      auto copy = cand;
      while (!copy.empty() && !(copy.top() > ann.top())) {
        ++live;
        copy.pop();
      }
      Q.cnt[C_MAXLIVE] = std::max(Q.cnt[C_MAXLIVE], live);
    } else {
      Q.cnt[C_MAXLIVE] = std::max<int64_t>(Q.cnt[C_MAXLIVE], (int64_t)cand.size());
    }
  }
  Q.cnt[C_NVISIT0] = nvisit;
  std::vector<FI> out;
  while (!ann.empty()) {
    out.push_back(ann.top());
    ann.pop();
  }
  std::reverse(out.begin(), out.end());
  return out;
}

struct Searcher {
  const View* V;
  std::vector<uint32_t> stamp;
  uint32_t cur = 0;
  explicit Searcher(const View* v) : V(v), stamp(v->n, 0u) {}

  void plan(Query& Q, int64_t l, int64_t h) const {
    Q.l = l;
    Q.h = h;
    if (l > h) {
      Q.lo = Q.hi = 0;
      return;
    }
    Q.lo = std::lower_bound(V->attr.begin(), V->attr.end(), l) - V->attr.begin();
    Q.hi = std::upper_bound(V->attr.begin(), V->attr.end(), h) - V->attr.begin();
    if (Q.hi < Q.lo) Q.hi = Q.lo;
    if (Q.hi > Q.lo) {
      Q.a = V->seg_of_rank(Q.lo);
      Q.b = V->seg_of_rank(Q.hi - 1);
    }
  }

  // Strategy A: the slice of objects in [l, h] (the layer-0 skip list from the
  // first object >= l), exact top-k by (dist32, id).
  std::vector<FI> pre(Query& Q, int k) {
    std::vector<FI> all;
    for (int64_t v = Q.lo; v < Q.hi; ++v)
      if (Q.second_ok((int)v)) all.push_back(Q.xkey((int)v));
    Q.cnt[C_NDIST] += Q.hi - Q.lo;
    std::sort(all.begin(), all.end());
    if ((int)all.size() > k) all.resize(k);
    return all;
  }

  // Strategy C: Alg. 2 scheme with Alg. 7 per layer over the active chunks.
  std::vector<FI> hybrid(Query& Q, int k, int ef, int m, int p, bool batch_form) {
    const int Sa = Q.b - Q.a + 1;
    Q.c = (m + Sa - 1) / Sa;
    Q.m = m;
    int top = -1;
    for (int j = Q.a; j <= Q.b; ++j)
      if (V->seg_entry[j] >= 0) top = std::max(top, V->seg_maxlevel[j]);
    if (top < 0) return {};
    FI best(std::numeric_limits<float>::infinity(), -1);
    for (int j = Q.a; j <= Q.b; ++j) {
      if (V->seg_entry[j] < 0 || V->seg_maxlevel[j] != top) continue;
      FI kj = Q.key(V->seg_entry[j]);
      if (best.second < 0 || kj < best) best = kj;
    }
    int ep = best.second;
    Q.cnt[C_ENTRY] = ep;  // the entry the rule chose (internal id), for the tests
    for (int l = top; l >= 1; --l) ep = layer_seq(Q, true, false, ep, l, 1, stamp, cur)[0].second;
    std::vector<FI> ann = (p == 1 && !batch_form) ? layer_seq(Q, true, true, ep, 0, ef, stamp, cur)
                                                  : layer_beam(Q, true, true, ep, ef, p, stamp, cur);
    return finish(Q, ann, k);
  }

  // The k results of a graph search from its ann list (ascending keys): the
  // in-range entries in order.  With a low-precision store, the first
  // rerank * k in-range entries are re-scored with the exact FP32 distance
  // and re-sorted by (distance, id) before the first k are kept.
  std::vector<FI> finish(Query& Q, const std::vector<FI>& ann, int k) const {
    const bool low = !V->XS.empty();
    const size_t R = low ? (size_t)V->rerank * k : (size_t)k;
    std::vector<FI> out;
    for (const FI& e : ann)
      if (Q.in_range(e.second) && out.size() < R) out.push_back(e);
    if (low) {
      for (FI& e : out) e = Q.xkey(e.second);
      Q.cnt[C_NRERANK] += (int64_t)out.size();
      std::sort(out.begin(), out.end());
    }
    if (out.size() > (size_t)k) out.resize(k);
    return out;
  }

  // Strategy B: Alg. 2 over the marked (global) edges, then the range filter.
  std::vector<FI> post(Query& Q, int k, int ef, int p, bool batch_form) {
    if (V->gentry < 0) return {};
    int ep = V->gentry;
    for (int l = V->L; l >= 1; --l) ep = layer_seq(Q, false, false, ep, l, 1, stamp, cur)[0].second;
    std::vector<FI> ann = (p == 1 && !batch_form) ? layer_seq(Q, false, false, ep, 0, ef, stamp, cur)
                                                  : layer_beam(Q, false, false, ep, ef, p, stamp, cur);
    return finish(Q, ann, k);
  }
};

thread_local std::string g_err;

}  // namespace

// ---------------------------------------------------------------------------
// C interface (loaded by the tests through ctypes)
// ---------------------------------------------------------------------------

struct OrcIndex {
  Builder B;
  bool has_builder = false;
  View V;
};

// ---- z-order composite attribute (Sec. 5.9, multiple attributes, approach 2) ----
// Reading: each attribute becomes an order-preserving coordinate on a grid of 2^31 cells,
//   u(x) = 0 if x <= base, else min(scale(x - base), 2^31 - 1)   (x - base modulo 2^64),
// scale(t) = t >> shift for shift >= 0 and t << -shift (2^31 - 1 when that overflows) else,
// with base the attribute's smallest value over the objects and shift = bits(largest - base)
// - 31 (0 when all values are equal), so that both attributes spread over the whole grid
// (the largest value lands in its upper half); the key interleaves the coordinates' bits
// (Orenstein's z-order), bit j of u1 becoming bit 2j + 1 of the key and bit j of u2 bit 2j.
// Every coordinate function is non-decreasing, and so is the key in each coordinate, so
// an object inside the box [l1, h1] x [l2, h2] has a key between key(u1(l1), u2(l2)) and
// key(u1(h1), u2(h2)): the search runs on that key range and admits only box objects.
static uint64_t z_coord(int64_t x, int64_t base, int shift) {
  const uint64_t top = (1ull << 31) - 1;
  if (x <= base) return 0;
  const uint64_t t = (uint64_t)x - (uint64_t)base;
  uint64_t u;
  if (shift >= 0) u = t >> shift;
  else u = t > (top >> -shift) ? top : t << -shift;
  return u < top ? u : top;
}
static int64_t z_key(uint64_t u1, uint64_t u2) {
  uint64_t z = 0;
  for (int j = 0; j < 31; ++j) {
    z |= ((u1 >> j) & 1ull) << (2 * j + 1);
    z |= ((u2 >> j) & 1ull) << (2 * j);
  }
  return (int64_t)z;
}
static void z_axis(const int64_t* a, int64_t n, int64_t& base, int& shift) {
  base = 0;
  shift = 0;
  if (n == 0) return;
  int64_t lo = a[0], hi = a[0];
  for (int64_t i = 1; i < n; ++i) {
    lo = std::min(lo, a[i]);
    hi = std::max(hi, a[i]);
  }
  base = lo;
  const uint64_t span = (uint64_t)hi - (uint64_t)lo;
  if (span == 0) return;
  int bits = 0;
  while (bits < 64 && (span >> bits) != 0) ++bits;
  shift = bits - 31;
}

// Runs one planned query under strategy st and writes its k results (external ids,
// FP32 distances; (-1, +inf) padding) and the strategy and slice counters.
static void run_query(Searcher& srch, Query& qq, int st, int k, int ef, int m, int p, int batch_form,
                      int64_t* out_ids, float* out_dist) {
  const View& V = *qq.V;
  int64_t* cnt = qq.cnt;
  cnt[C_STRAT] = st;
  cnt[C_LO] = qq.lo;
  cnt[C_HI] = qq.hi;
  std::vector<FI> res;
  if (qq.hi > qq.lo) {
    if (st == ST_PRE) res = srch.pre(qq, k);
    else if (st == ST_HYBRID) res = srch.hybrid(qq, k, ef, m, p, batch_form != 0);
    else res = srch.post(qq, k, ef, p, batch_form != 0);
  }
  for (int t = 0; t < k; ++t) {
    if (t < (int)res.size()) {
      out_ids[t] = V.ext[res[t].second];
      out_dist[t] = res[t].first;
    } else {
      out_ids[t] = -1;
      out_dist[t] = std::numeric_limits<float>::infinity();
    }
  }
}

extern "C" {

const char* orc_last_error() { return g_err.c_str(); }

float orc_dist32(const float* q, const float* x, int d) { return dist32(q, x, d); }

void orc_bf16(const float* x, int64_t n, uint16_t* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = bf16_nearest(x[i]);
}
void orc_e4m3_encode(const float* y, int64_t n, uint8_t* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = e4m3_nearest(y[i]);
}
void orc_e4m3_decode(const uint8_t* c, int64_t n, float* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = (float)e4m3_value(c[i]);
}
// FP8 copies of n rows of X [n][d]: codes [n][d], scales [n], values read back [n][d].
void orc_fp8_rows(const float* X, int64_t n, int d, uint8_t* codes, float* scales, float* back) {
  for (int64_t v = 0; v < n; ++v)
    scales[v] = fp8_row(X + v * d, d, codes + v * d, back + v * d);
}
int orc_level_of(double u, double mL) { return draw_level(u, mL); }
double orc_dist64(const float* q, const float* x, int d) { return dist64(q, x, d); }

// Builds an HSIG by inserting objects 0..n-1 in order (Alg. 6).  level_u[v] is
// the uniform variate of object v's level draw.  M0 <= 0 means M0 = M;
// mL <= 0 means 1/ln(M).  hnsw != 0 builds a plain HNSW (Alg. 3) instead.
void* orc_build(const float* X, const int64_t* attr, const double* level_u, int64_t n, int d,
                int S, int M, int M0, int efCons, double mL, uint64_t seed, int hnsw, int64_t bnd_n) {
  if (n < 1 || d < 4 || d % 4 || S < 1 || M < 1 || efCons < 1) {
    g_err = "orc_build: bad arguments";
    return nullptr;
  }
  OrcIndex* ix = new OrcIndex();
  ix->B.hnsw_mode = hnsw != 0;
  ix->B.init(X, attr, n, d, hnsw ? 1 : S, M, M0, efCons, mL, bnd_n);
  if (hnsw) {
    ix->B.bnd.clear();
    std::fill(ix->B.seg.begin(), ix->B.seg.end(), 0);
  }
  for (int64_t v = 0; v < n; ++v) ix->B.insert((int)v, level_u[v]);
  ix->has_builder = true;
  freeze(ix->B, ix->V, seed);
  return ix;
}

// Incremental insertion (Alg. 6) of m more objects into an index this library
// built; they take external ids n .. n + m - 1.  Returns 0, or -1.
int orc_insert(void* h, const float* X, const int64_t* attr, const double* level_u, int64_t m) {
  OrcIndex* ix = (OrcIndex*)h;
  if (!ix->has_builder || m < 0) {
    g_err = "orc_insert: the index was not built here (no builder state)";
    return -1;
  }
  for (int64_t t = 0; t < m; ++t)
    if (!(level_u[t] > 0.0 && level_u[t] <= 1.0)) {
      g_err = "orc_insert: level variates must lie in (0, 1]";
      return -1;
    }
  const int64_t n0 = ix->B.n;
  ix->B.append(X, attr, m);
  for (int64_t t = 0; t < m; ++t) ix->B.insert((int)(n0 + t), level_u[t]);
  const uint64_t seed = ix->V.seed;
  ix->V = View();
  freeze(ix->B, ix->V, seed);
  return 0;
}

void* orc_read(const char* path) {
  OrcIndex* ix = new OrcIndex();
  int rc = read_view(path, ix->V);
  if (rc != 0) {
    g_err = rc == -5 ? "orc_read: I/O error" : "orc_read: bad index file";
    delete ix;
    return nullptr;
  }
  return ix;
}

int orc_write(void* h, const char* path) { return write_view(((OrcIndex*)h)->V, path); }

void orc_free(void* h) { delete (OrcIndex*)h; }

// info: n, d, S, M0, MU, L, gentry, R, efCons
void orc_info(void* h, int64_t* out) {
  const View& V = ((OrcIndex*)h)->V;
  out[0] = V.n;
  out[1] = V.d;
  out[2] = V.S;
  out[3] = V.M0;
  out[4] = V.MU;
  out[5] = V.L;
  out[6] = V.gentry;
  out[7] = V.R;
  out[8] = V.efCons;
}

// Copies of the view's tables (internal ids).
void orc_get_attr(void* h, int64_t* out) {
  const View& V = ((OrcIndex*)h)->V;
  std::copy(V.attr.begin(), V.attr.end(), out);
}
void orc_get_ext(void* h, int64_t* out) {
  const View& V = ((OrcIndex*)h)->V;
  std::copy(V.ext.begin(), V.ext.end(), out);
}
void orc_get_level(void* h, int32_t* out) {
  const View& V = ((OrcIndex*)h)->V;
  for (int64_t i = 0; i < V.n; ++i) out[i] = V.level[i];
}
void orc_get_segments(void* h, int64_t* seg_start, int32_t* entry, int32_t* maxlev) {
  const View& V = ((OrcIndex*)h)->V;
  std::copy(V.seg_start.begin(), V.seg_start.end(), seg_start);
  std::copy(V.seg_entry.begin(), V.seg_entry.end(), entry);
  std::copy(V.seg_maxlevel.begin(), V.seg_maxlevel.end(), maxlev);
}
// Chunk rows of layer l for every node that has layer l: out[n][S][mcap] (-1 rows for absent nodes).
void orc_get_layer(void* h, int l, int32_t* out_adj, int32_t* out_glist) {
  const View& V = ((OrcIndex*)h)->V;
  const int mc = V.mcap(l);
  std::vector<int> g;
  for (int64_t v = 0; v < V.n; ++v) {
    int32_t* row = out_adj + (size_t)v * V.S * mc;
    int32_t* grow = out_glist + (size_t)v * V.S * mc;
    for (int t = 0; t < V.S * mc; ++t) row[t] = grow[t] = -1;
    if (V.level[v] < l) continue;
    for (int j = 0; j < V.S; ++j) std::memcpy(row + j * mc, V.chunk((int)v, l, j), 4 * mc);
    V.glist((int)v, l, g);
    for (size_t t = 0; t < g.size(); ++t) grow[t] = g[t];
  }
}
// The real skip list of the builder, walked on layer 0 from the first object
// with attribute >= l while attribute <= h; writes internal ids (= ranks).
int64_t orc_skiplist_range(void* h, int64_t l, int64_t hh, int64_t* out, int64_t cap) {
  OrcIndex* ix = (OrcIndex*)h;
  if (!ix->has_builder) return -1;
  const Builder& B = ix->B;
  int top = (int)B.head_next.size() - 1;
  int x = -1;
  for (int lv = top; lv >= 0; --lv) {
    while (true) {
      int nx = x < 0 ? B.head_next[lv] : B.next[x][lv];
      if (nx >= 0 && B.attr[nx] < l) x = nx;
      else break;
    }
  }
  int v = x < 0 ? B.head_next[0] : B.next[x][0];
  // map ext -> rank through the view
  std::vector<int64_t> rank(B.n);
  for (int64_t r = 0; r < ix->V.n; ++r) rank[ix->V.ext[r]] = r;
  int64_t cnt = 0;
  while (v >= 0 && B.attr[v] <= hh) {
    if (cnt < cap) out[cnt] = rank[v];
    ++cnt;
    v = B.next[v][0];
  }
  return cnt;
}

// Build-side structures before freezing, by external id (for reduction tests):
// chunk j of v on layer l, as external ids.
int orc_build_chunk(void* h, int64_t v, int l, int j, int64_t* out, int cap) {
  OrcIndex* ix = (OrcIndex*)h;
  if (!ix->has_builder) return -1;
  const Builder& B = ix->B;
  if (v < 0 || v >= B.n || l > B.level[v] || j < 0 || j >= B.S) return -1;
  const auto& ch = B.adj[v][l][j];
  int c = 0;
  for (const DI& e : ch)
    if (c < cap) out[c++] = e.second;
  return (int)ch.size();
}
int orc_build_level(void* h, int64_t v) { return ((OrcIndex*)h)->B.level[v]; }

// Prune (Sec. 2.2) of owner point o against candidate points, FP64 distances;
// writes the indices of the kept candidates in selection order.
int orc_prune(const float* owner, const float* cands, int nc, int d, int Mcap, int32_t* out) {
  std::vector<std::pair<double, int>> c;
  for (int i = 0; i < nc; ++i) c.push_back({dist64(owner, cands + (size_t)i * d, d), i});
  std::sort(c.begin(), c.end());
  int cnt = 0;
  std::vector<int> sel;
  for (auto& r : c) {
    if ((int)sel.size() >= Mcap) break;
    bool keep = true;
    for (int e : sel)
      if (dist64(cands + (size_t)e * d, cands + (size_t)r.second * d, d) < r.first) {
        keep = false;
        break;
      }
    if (keep) {
      sel.push_back(r.second);
      out[cnt++] = r.second;
    }
  }
  return cnt;
}

// Search (O2).  strategy: 0 auto, 1 pre, 2 hybrid, 3 post.  m <= 0 means M0.
// Outputs external ids and FP32 distances, ascending by (distance, internal id),
// padded with (-1, +inf).  counters: [nq][C_NCOUNT] or NULL.  batch_form != 0
// runs layer 0 in the beam form even for p = 1 (and records live-candidate counts).
// L2, H2 (both or neither): the second attribute's inclusive range per query; an
// object qualifies when both of its attributes are in range.  The strategy rule
// looks at the first (indexed) attribute's range only.
int orc_search(void* h, const float* Q, int64_t nq, const int64_t* L, const int64_t* H, int k,
               int ef, int m, int p, int strategy, double tau_a, double tau_b, int64_t* out_ids,
               float* out_dist, int64_t* counters, int batch_form, int select_s1, const int64_t* L2,
               const int64_t* H2) {
  OrcIndex* ix = (OrcIndex*)h;
  const View& V = ix->V;
  if (k < 1 || ef < 1 || p < 1 || strategy < 0 || strategy > 3 || (!L2) != (!H2) ||
      (L2 && V.attr2.empty())) {
    g_err = "orc_search: bad arguments (or a second range without a second attribute)";
    return -22;
  }
  if (m <= 0) m = V.M0;
  const int64_t tA = (int64_t)std::floor(tau_a * (double)V.n);
  const int64_t tB = (int64_t)std::ceil(tau_b * (double)V.n);
  Searcher srch(&V);
  std::vector<int64_t> dummy(C_NCOUNT);
  for (int64_t i = 0; i < nq; ++i) {
    int64_t* cnt = counters ? counters + i * C_NCOUNT : dummy.data();
    for (int t = 0; t < C_NCOUNT; ++t) cnt[t] = 0;
    cnt[C_ENTRY] = -1;
    Query qq;
    qq.V = &V;
    qq.q = Q + (size_t)i * V.d;
    qq.cnt = cnt;
    qq.s1 = select_s1 != 0;
    if (L2) {
      qq.multi = true;
      qq.l2 = L2[i];
      qq.h2 = H2[i];
    }
    srch.plan(qq, L[i], H[i]);
    const int64_t Y = qq.hi - qq.lo;
    int st = strategy;
    if (st == ST_AUTO && qq.multi) {
      // conjunctive query: the rule looks at the estimated count of objects passing both
      // ranges, Y times the fraction of the second attribute's sample inside its range
      const std::vector<int64_t>& sm = V.attr2_sample;
      const int64_t ns = (int64_t)sm.size();
      int64_t c2 = 0;
      for (int64_t j = 0; j < ns; ++j) c2 += sm[j] >= qq.l2 && sm[j] <= qq.h2;
      const int64_t yj = Y * c2;
      st = (Y <= tA || yj <= tA * ns) ? ST_PRE : (yj >= tB * ns ? ST_POST : ST_HYBRID);
    } else if (st == ST_AUTO) {
      st = Y <= tA ? ST_PRE : (Y >= tB ? ST_POST : ST_HYBRID);
    }
    run_query(srch, qq, st, k, ef, m, p, batch_form, out_ids + i * k, out_dist + i * k);
  }
  return 0;
}

// The z-order key map of two attributes given per object: out = {base1, shift1, base2, shift2}.
int orc_zorder_map(const int64_t* a1, const int64_t* a2, int64_t n, int64_t* out) {
  int s1 = 0, s2 = 0;
  z_axis(a1, n, out[0], s1);
  z_axis(a2, n, out[2], s2);
  out[1] = s1;
  out[3] = s2;
  return 0;
}

// z-order keys of n pairs under map {base1, shift1, base2, shift2}.
int orc_zorder_keys(const int64_t* map, const int64_t* a1, const int64_t* a2, int64_t n, int64_t* out) {
  if (map[1] < -30 || map[1] > 63 || map[3] < -30 || map[3] > 63) {
    g_err = "orc_zorder_keys: bad map";
    return -22;
  }
  for (int64_t i = 0; i < n; ++i)
    out[i] = z_key(z_coord(a1[i], map[0], (int)map[1]), z_coord(a2[i], map[2], (int)map[3]));
  return 0;
}

// The key range [out_lo, out_hi] searched for each box (out_lo > out_hi: an empty box).
int orc_zorder_range(const int64_t* map, const int64_t* L1, const int64_t* H1, const int64_t* L2,
                     const int64_t* H2, int64_t nq, int64_t* out_lo, int64_t* out_hi) {
  for (int64_t i = 0; i < nq; ++i) {
    if (L1[i] > H1[i] || L2[i] > H2[i]) {
      out_lo[i] = 1;
      out_hi[i] = 0;
      continue;
    }
    out_lo[i] = z_key(z_coord(L1[i], map[0], (int)map[1]), z_coord(L2[i], map[2], (int)map[3]));
    out_hi[i] = z_key(z_coord(H1[i], map[0], (int)map[1]), z_coord(H2[i], map[2], (int)map[3]));
  }
  return 0;
}

// Attaches the two attributes of a z-order index: a1[e], a2[e] belong to the object with
// external id e (ids 0 .. n-1), and the index's attribute of every object must be the key
// of its pair under map.  Returns 0, or -22.
int orc_set_zorder(void* h, const int64_t* map, const int64_t* a1, const int64_t* a2, int64_t n) {
  View& V = ((OrcIndex*)h)->V;
  if (n != V.n || map[1] < -30 || map[1] > 63 || map[3] < -30 || map[3] > 63) {
    g_err = "orc_set_zorder: one pair per object and a valid map";
    return -22;
  }
  std::vector<int64_t> b1(n), b2(n);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t e = V.ext[i];
    if (e < 0 || e >= n) {
      g_err = "orc_set_zorder: external ids are not 0 .. n-1";
      return -22;
    }
    b1[i] = a1[e];
    b2[i] = a2[e];
    if (V.attr[i] != z_key(z_coord(b1[i], map[0], (int)map[1]), z_coord(b2[i], map[2], (int)map[3]))) {
      g_err = "orc_set_zorder: the index is not built on these pairs' keys";
      return -22;
    }
  }
  const int64_t ns = std::min<int64_t>(n, 2048);
  V.zs1.resize(ns);
  V.zs2.resize(ns);
  for (int64_t j = 0; j < ns; ++j) {
    V.zs1[j] = b1[(size_t)(j * n / ns)];
    V.zs2[j] = b2[(size_t)(j * n / ns)];
  }
  V.za1.swap(b1);
  V.za2.swap(b2);
  V.zbase1 = map[0];
  V.zshift1 = (int)map[1];
  V.zbase2 = map[2];
  V.zshift2 = (int)map[3];
  return 0;
}

// Box search on a z-order index: the k nearest objects with L1 <= A1 <= H1 and
// L2 <= A2 <= H2.  The HSIG is searched on the key range of the box (orc_zorder_range)
// and admits only box objects (Alg. 7's ann admission and the post-filter test; the
// pre-filter scans the key range and keeps box objects).  Strategy rule (auto): with Y
// the objects in the key range and c the sampled pairs inside the box, pre-filter when
// Y <= tau_a n or c n <= tau_a n ns, post-filter when c n >= tau_b n ns, else hybrid.
// Other arguments and outputs as orc_search.
int orc_search_box(void* h, const float* Q, int64_t nq, const int64_t* L1, const int64_t* H1, const int64_t* L2,
                   const int64_t* H2, int k, int ef, int m, int p, int strategy, double tau_a, double tau_b,
                   int64_t* out_ids, float* out_dist, int64_t* counters, int batch_form, int select_s1) {
  OrcIndex* ix = (OrcIndex*)h;
  const View& V = ix->V;
  if (k < 1 || ef < 1 || p < 1 || strategy < 0 || strategy > 3 || V.za1.empty()) {
    g_err = "orc_search_box: bad arguments (or no z-order attributes)";
    return -22;
  }
  if (m <= 0) m = V.M0;
  const int64_t tA = (int64_t)std::floor(tau_a * (double)V.n);
  const int64_t tB = (int64_t)std::ceil(tau_b * (double)V.n);
  const int64_t map[4] = {V.zbase1, V.zshift1, V.zbase2, V.zshift2};
  const int64_t ns = (int64_t)V.zs1.size();
  Searcher srch(&V);
  std::vector<int64_t> dummy(C_NCOUNT);
  for (int64_t i = 0; i < nq; ++i) {
    int64_t* cnt = counters ? counters + i * C_NCOUNT : dummy.data();
    for (int t = 0; t < C_NCOUNT; ++t) cnt[t] = 0;
    cnt[C_ENTRY] = -1;
    Query qq;
    qq.V = &V;
    qq.q = Q + (size_t)i * V.d;
    qq.cnt = cnt;
    qq.s1 = select_s1 != 0;
    qq.box = true;
    qq.l1 = L1[i];
    qq.h1 = H1[i];
    qq.l2 = L2[i];
    qq.h2 = H2[i];
    int64_t zl = 0, zh = 0;
    orc_zorder_range(map, L1 + i, H1 + i, L2 + i, H2 + i, 1, &zl, &zh);
    srch.plan(qq, zl, zh);
    const int64_t Y = qq.hi - qq.lo;
    int st = strategy;
    if (st == ST_AUTO) {
      int64_t c = 0;
      for (int64_t j = 0; j < ns; ++j)
        c += V.zs1[j] >= qq.l1 && V.zs1[j] <= qq.h1 && V.zs2[j] >= qq.l2 && V.zs2[j] <= qq.h2;
      st = (Y <= tA || c * V.n <= tA * ns) ? ST_PRE : (c * V.n >= tB * ns ? ST_POST : ST_HYBRID);
    }
    run_query(srch, qq, st, k, ef, m, p, batch_form, out_ids + i * k, out_dist + i * k);
  }
  return 0;
}

// Sets the second attribute: attr2[e] belongs to the object with external id e
// (external ids must be 0 .. n-1).  Returns 0, or -22.
int orc_set_attr2(void* h, const int64_t* attr2, int64_t n) {
  View& V = ((OrcIndex*)h)->V;
  if (n != V.n) {
    g_err = "orc_set_attr2: one value per object";
    return -22;
  }
  std::vector<int64_t> a(n);
  for (int64_t i = 0; i < n; ++i) {
    if (V.ext[i] < 0 || V.ext[i] >= n) {
      g_err = "orc_set_attr2: external ids are not 0 .. n-1";
      return -22;
    }
    a[i] = attr2[V.ext[i]];
  }
  std::vector<int64_t> srt(a);
  std::sort(srt.begin(), srt.end());
  const int64_t ns = std::min<int64_t>(n, 2048);
  V.attr2_sample.resize(ns);
  for (int64_t j = 0; j < ns; ++j) V.attr2_sample[j] = srt[(size_t)(j * n / ns)];
  V.attr2.swap(a);
  return 0;
}

// Selects the store the graph searches rank by: 0 = the FP32 vectors, 1 = a
// BF16 copy, 2 = an FP8 E4M3 copy with one scale per vector; rerank_mult >= 1
// sets how many results (rerank_mult * k) are re-scored in FP32.
int orc_set_store(void* h, int precision, int rerank_mult) {
  OrcIndex* ix = (OrcIndex*)h;
  View& V = ix->V;
  if (precision < 0 || precision > 2 || (precision > 0 && rerank_mult < 1)) {
    g_err = "orc_set_store: bad arguments";
    return -22;
  }
  V.rerank = rerank_mult;
  if (precision == 0) {
    std::vector<float>().swap(V.XS);
    return 0;
  }
  V.XS.resize(V.X.size());
  if (precision == 1) {
    for (size_t i = 0; i < V.X.size(); ++i) V.XS[i] = bf16_value(bf16_nearest(V.X[i]));
  } else {
    std::vector<uint8_t> codes(V.d);
    for (int64_t v = 0; v < V.n; ++v) fp8_row(&V.X[(size_t)v * V.d], V.d, codes.data(), &V.XS[(size_t)v * V.d]);
  }
  return 0;
}

// One layer search from a given entry (for the reachability tests): hybrid
// (chunk rule with segments [a, b] and c entries each) or post (marked edges);
// filter applies the [l, h] test to ann.  Returns the count, writes internal ids.
int orc_layer_search(void* h, const float* q, int ep, int layer, int ef, int hybrid, int a, int b,
                     int c, int filter, int64_t l, int64_t hh, int32_t* out_ids, float* out_dist) {
  OrcIndex* ix = (OrcIndex*)h;
  const View& V = ix->V;
  Searcher srch(&V);
  std::vector<int64_t> cnt(C_NCOUNT, 0);
  Query qq;
  qq.V = &V;
  qq.q = q;
  qq.cnt = cnt.data();
  qq.l = l;
  qq.h = hh;
  qq.a = a;
  qq.b = b;
  qq.c = c;
  std::vector<FI> r = layer_seq(qq, hybrid != 0, filter != 0, ep, layer, ef, srch.stamp, srch.cur);
  for (size_t t = 0; t < r.size(); ++t) {
    out_ids[t] = r[t].second;
    out_dist[t] = r[t].first;
  }
  return (int)r.size();
}

// The neighbours a hybrid expansion of o on layer l takes with the active
// segments a..b and budget m: selection S1 (s1 != 0) or S2 (Sec. 4.2), in the
// current store.  Writes at most cap ids; returns how many there are.
int orc_neighbours(void* h, int o, int l, int a, int b, int m, int s1, int32_t* out, int cap) {
  const View& V = ((OrcIndex*)h)->V;
  if (o < 0 || o >= V.n || V.level[o] < l || a < 0 || b < a || b >= V.S || m < 1) return -1;
  std::vector<int64_t> cnt(C_NCOUNT, 0);
  Query qq;
  qq.V = &V;
  qq.cnt = cnt.data();
  qq.a = a;
  qq.b = b;
  qq.m = m;
  qq.c = (m + (b - a + 1) - 1) / (b - a + 1);
  qq.s1 = s1 != 0;
  std::vector<int> nb;
  neighbours(qq, true, o, l, nb);
  for (size_t t = 0; t < nb.size() && (int)t < cap; ++t) out[t] = nb[t];
  return (int)nb.size();
}

}  // extern "C"
