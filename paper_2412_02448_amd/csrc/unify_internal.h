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

// Allocates the index's visited-set memory and its search-ordering event if
// they are not there yet (called when an index version becomes resident).
int ensure_tags(unify_index_t ix);

}  // namespace unify

struct unify_index {
  int device = 0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};  // timing: before the plan, after the work
                                                            // list, after the search, after the re-run
  bool timed = false;
  uint32_t* tags = nullptr;    // visited epochs [nslots][n], allocated when the index becomes resident
  uint32_t* epochs = nullptr;  // [nslots]
  int64_t nslots = 0;
  const float* eps_of[3] = {nullptr, nullptr, nullptr};  // error bounds of the resident BF16 / FP8 copies
  int cus = 0;                                            // compute units of the device
  // The visited tags are shared by every search on the index: the search
  // kernels of successive calls are ordered across streams by this event.
  std::mutex order_mu;
  hipEvent_t last_search = nullptr;
  // An insertion builds a new version of the tables and swaps it in while no
  // search is being enqueued: entry points that read dv hold version_mu shared,
  // the swap holds it exclusively.  version counts the swaps; insert_mu keeps
  // insertions one at a time.
  std::shared_mutex version_mu;
  std::mutex insert_mu;
  uint64_t version = 0;
  std::map<std::pair<const void*, size_t>, int> occupancy;  // (kernel, LDS bytes) -> waves per CU
  unify::DevIndex dv{};
  unify::HostIndex host;  // small tables kept on the host; large ones released after upload
  std::vector<void*> allocs;
};

// A batch: the search over fixed caller buffers captured as a HIP graph.
struct unify_batch {
  unify_index_t ix = nullptr;
  uint64_t version = 0;  // the index version the graph was captured on
  void* scratch = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace unify {
int batch_create(unify_index_t ix, const float* queries, int64_t nq, const int64_t* l, const int64_t* h, int32_t k,
                 int32_t ef, const int8_t* strategy, const unify_params* prm, int64_t* out_ids, float* out_dist,
                 int8_t* out_strategy, int32_t* out_stats, unify_batch_t* out);
int batch_run(unify_batch_t b, void* stream);
int insert_impl(unify_index_t ix, const float* vectors, const int64_t* attr, const double* level_u, int64_t m);
}  // namespace unify
