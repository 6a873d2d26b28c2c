// Internal declarations shared by the HIP translation units of libunify.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/unify.h"

namespace unify {

// Device-resident index.  Internal ids are ranks in (attribute, external id)
// order, so the objects in an attribute range are one contiguous id interval
// (the layer-0 skip list of Sec. 4.1 becomes "next = id + 1").
struct DevIndex {
  int64_t n;
  int32_t d, S, M0, MU, GC, L, gentry;
  int64_t R;            // rows of the upper-layer tables
  int32_t precision;    // UNIFY_FP32 / BF16 / FP8E4M3: the store the searches rank by
  int32_t pad;
  const int64_t* attr;       // [n] sorted attributes
  const int64_t* ext;        // [n] external id of each internal id
  const int64_t* seg_start;  // [S+1] first internal id of each segment
  const int32_t* seg_entry;  // [S] entry (internal id) of each segment's HNSW, -1 if empty
  const int32_t* seg_maxlevel;  // [S]
  const int32_t* uprow;      // [n] row of (v, layer 1) in the upper tables; rows of layers 2.. follow
  const float* vec;          // [n][d] FP32 store
  const uint16_t* vec_bf16;  // [n][d] BF16 store or null
  const uint8_t* vec_fp8;    // [n][d] FP8 E4M3 store or null
  const float* vec_scale;    // [n] FP8 scale or null
  const float* vec_eps;      // [n] bound on ||copy - FP32 vector|| of the store in use, or null
  const float* vec_nrm;      // [n] squared norm of each row of the store in use (FP32)
  const int32_t* adj0;       // [n][S][M0] layer-0 chunks, -1 padded
  const int32_t* glist0;     // [n][GC] layer-0 global (marked) edges, -1 padded
  const int32_t* adjU;       // [R][S][MU]
  const int32_t* glistU;     // [R][GC]
  const int64_t* attr2;      // [n] second attribute (conjunctive queries), or null
  const int64_t* attr2_sample;  // [n2s] sorted sample of attr2 (selectivity estimates)
  int32_t n2s;
};

// Per-query plan written by the plan kernel.
struct QPlan {
  int32_t lo, hi;   // in-range internal ids [lo, hi)
  int32_t a, b;     // active segments a..b (segments holding an in-range object)
  int32_t strat;    // UNIFY_PRE / HYBRID / POST; -1 when the range is empty
  int32_t nch;      // pre-filter: chunks the slice is split into (1 = one wavefront)
  int32_t clen;     // pre-filter: objects per chunk (the last one may be shorter)
  int32_t pbase;    // pre-filter, nch > 1: first slot of the query's partial top-k lists
  int32_t tsb;      // pre-filter by the matrix-core scan: super-blocks its slice touches (0: not)
  int32_t tbase;    // matrix-core scan: first of the query's tsb candidate records
};

// Host-side tables of an index (the index file content), internal ids.
struct HostIndex {
  int64_t n = 0;
  int32_t d = 0, S = 0, M0 = 0, MU = 0, L = -1, gentry = -1, ef_cons = 0;
  double mL = 0;
  uint64_t seed = 0;
  int64_t R = 0;
  int32_t W0 = 0, WU = 0;
  std::vector<int64_t> attr, ext, seg_start;
  std::vector<int32_t> seg_entry, seg_maxlevel;
  std::vector<uint8_t> level;
  std::vector<int32_t> uprow;
  std::vector<float> vec;
  std::vector<int32_t> adj0, adjU;
  std::vector<uint32_t> gbits0, gbitsU;
};

int read_index_file(const char* path, HostIndex& H, std::string& err);
int write_index_file(const char* path, const HostIndex& H, std::string& err);
int validate_index(const HostIndex& H, std::string& err);

void set_error(const std::string& msg);

// Selects the store the searches rank by, building the BF16 or FP8 copy of the
// resident vectors and its error bounds when it is not resident yet.
int quantize_store(unify_index_t ix, int precision);

// Two more streams with their fork and join events: the cooperative search
// kernel runs on `stream` beside the one-wavefront kernel, the matrix-core
// pre-filter scan on `tstream` beside both.
struct SideStream {
  hipStream_t stream = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  hipStream_t tstream = nullptr;
  hipEvent_t tfork = nullptr, tjoin = nullptr;
};
// Creates the streams and events a launch needs (the cooperative kernel's, the
// matrix-core scan's) if they are not there yet: a process shares a few hardware
// queues among all its streams, so none is made that would stay unused.
int make_side(SideStream& s, bool coop, bool tile);
void free_side(SideStream& s);

// Visited-set memory of the graph searches: one row per persistent wavefront (a
// bitmap of the index's n objects, clear between layer searches, then a log of
// the bitmap words a layer search set), the event of the last search kernel
// enqueued on the rows and the side stream of the cooperative kernel.  Searches
// on one pool are ordered through `last` under `mu`; searches on different
// pools run concurrently.  The index holds one pool, each serving slot its own.
struct VisitPool {
  uint32_t* rows = nullptr;
  int64_t nrows = 0;     // rows made
  int64_t max_rows = 0;  // rows wanted (fewer are made when device memory is short)
  int64_t stride = 0;    // words of a row
  int64_t bwords = 0;    // words of a row's bitmap
  int64_t n = -1;        // objects the rows were made for
  std::mutex mu;
  hipEvent_t last = nullptr;
  SideStream side;
};
// Bytes of one row for an index of n objects.
size_t pool_row_bytes(int64_t n);
// Makes the event, the side stream and max_rows rows for n objects (fewer if a
// quarter of the free device memory does not hold them), all bits clear; rows
// made for another n are freed first, once the searches on them have finished.
int pool_ensure(VisitPool& p, int64_t n);
// Waits for the pool's searches and frees everything it holds.
void pool_free(VisitPool& p);

// Makes the index's visited pool (one row per resident wavefront of the device),
// if it is not there yet for the current index size (called when an index
// version becomes resident).
int ensure_pool(unify_index_t ix);

// The two attributes of an index built on their z-order keys (box searches): device
// arrays in internal-id order, the key map, and the pairs of the objects at internal
// ids floor(j n / ns), j < ns = min(n, 2048), for the strategy rule.
struct ZOrder {
  const int64_t* a1 = nullptr;
  const int64_t* a2 = nullptr;
  const int64_t* s1 = nullptr;
  const int64_t* s2 = nullptr;
  int64_t base1 = 0, base2 = 0;
  int32_t shift1 = 0, shift2 = 0;
  int32_t ns = 0;
};

}  // namespace unify

struct unify_index {
  int device = 0;
  // timing: before the plan, after the work list, after the matrix-core scan's set-up, after its
  // scan, after its results, after the search kernel, after the merge, after the re-run
  hipEvent_t ev[8] = {};
  bool timed = false;
  bool timed_side = false;  // the timed call ran the matrix-core scan beside the graph search
  unify::VisitPool pool;  // the visited rows of searches that bring none of their own
  const float* eps_of[3] = {nullptr, nullptr, nullptr};  // error bounds of the resident BF16 / FP8 copies
  const float* nrm_of[3] = {nullptr, nullptr, nullptr};  // squared row norms of each resident store
  int cus = 0;                                            // compute units of the device
  // An insertion builds a new version of the tables and swaps it in while no
  // search is being enqueued: entry points that read dv hold version_mu shared,
  // the swap holds it exclusively.  version counts the swaps; insert_mu keeps
  // insertions one at a time.
  std::shared_mutex version_mu;
  std::mutex insert_mu;
  uint64_t version = 0;
  std::map<std::pair<const void*, size_t>, int> occupancy;  // (kernel, LDS bytes) -> waves per CU
  unify::DevIndex dv{};
  unify::ZOrder z;        // set by unify_set_zorder; dropped by an insertion
  unify::HostIndex host;  // small tables kept on the host; large ones released after upload
  std::vector<void*> allocs;
};

// A batch: the search over fixed caller buffers captured as a HIP graph.
struct unify_batch {
  unify_index_t ix = nullptr;
  uint64_t version = 0;  // the index version the graph was captured on
  void* scratch = nullptr;
  unify::SideStream side;  // joins the capture when the search forks
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace unify {
int batch_create(unify_index_t ix, const float* queries, int64_t nq, const int64_t* l, const int64_t* h, int32_t k,
                 int32_t ef, const int8_t* strategy, const unify_params* prm, int64_t* out_ids, float* out_dist,
                 int8_t* out_strategy, int32_t* out_stats, unify_batch_t* out);
int batch_run(unify_batch_t b, void* stream);
int insert_impl(unify_index_t ix, const float* vectors, const int64_t* attr, const double* level_u, int64_t m);
int prune_impl(const float* X, int64_t n, int32_t d, const int32_t* owners, const int32_t* cand, int64_t t,
               int32_t c, int32_t M, int32_t* out, void* stream);
}  // namespace unify
