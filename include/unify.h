/*
 * unify.h -- C ABI of the MI355X (gfx950) range-filtered k-NN library.
 *
 * The library answers range-filtered k-nearest-neighbour queries over a
 * Hierarchical Segmented Inclusive Graph (HSIG) kept resident on one GPU.
 * The method is UNIFY (Liang et al., PVLDB 18(4), 2024):
 *   - the problem: Definition 1 (Sec. 2.1) -- given q, an inclusive attribute
 *     range [l, h] and k, return the k objects with l <= attribute <= h nearest
 *     to q (all of them when fewer than k exist);
 *   - the index: Sec. 4.1 (segmented chunks per layer, skip-list order,
 *     global-edge bitmap) and Alg. 4-6 for its construction;
 *   - the search: Sec. 4.2 -- strategy A (pre-filter scan), B (post-filter search
 *     on the global edges), C (hybrid search, Alg. 7 inside the scheme of Alg. 2)
 *     and the range-aware selection rule (pre when Y <= tau_A, post when
 *     Y >= tau_B, hybrid otherwise, Y = number of objects in range).
 *
 * Conventions shared by every entry point:
 *   - Return value: 0 on success, a negative UNIFY_E* code on failure; on failure
 *     unify_last_error() describes it.  No C++ exception crosses this boundary.
 *   - Device pointers are HIP device addresses on the index's device; host
 *     pointers are ordinary process memory.  Each argument says which it is.
 *   - The caller owns every buffer it passes; the library owns the index.
 *   - Work is enqueued on the caller's HIP stream (NULL = the default stream) and
 *     is not waited for: the caller synchronises that stream before reading outputs.
 *   - Distances are squared Euclidean distances in FP32.  Identifiers returned
 *     are the external ids stored with the index (the row numbers the vectors had
 *     when the index was built).  Each output row is ascending by
 *     (distance, internal id), internal id = rank in attribute order.
 *   - Rows with fewer than k results (empty range, l > h, fewer than k objects in
 *     range, or a post-filter search that met fewer than k in-range objects) are
 *     padded with id -1 and distance +inf.
 *   - NaN in a query vector is not checked on the device; results are then unspecified.
 */
#ifndef UNIFY_H
#define UNIFY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct unify_index* unify_index_t;

/* Search strategies (Sec. 4.2). */
enum {
  UNIFY_AUTO = 0,   /* range-aware selection rule */
  UNIFY_PRE = 1,    /* strategy A: exact scan of the objects in range */
  UNIFY_HYBRID = 2, /* strategy C: Alg. 7 over the chunks of the segments in range */
  UNIFY_POST = 3    /* strategy B: search on the global edges, then the range filter */
};

/* Element type of the device vector store used by the graph searches. */
enum {
  UNIFY_FP32 = 0,
  UNIFY_BF16 = 1,    /* bfloat16, round to nearest even; candidates reranked in FP32 */
  UNIFY_FP8E4M3 = 2  /* OCP FP8 E4M3 with one FP32 scale per vector; reranked in FP32 */
};

/* Status codes. */
enum {
  UNIFY_OK = 0,
  UNIFY_EINVAL = -22,   /* an argument is out of its documented domain */
  UNIFY_ENOMEM = -12,   /* device or host allocation failed */
  UNIFY_EIO = -5,       /* the index file could not be read or written */
  UNIFY_EFORMAT = -74,  /* bad magic, version, checksum or table contents */
  UNIFY_EDEVICE = -19   /* a HIP runtime call failed */
};

/* Bits of unify_params.flags. */
enum {
  UNIFY_FLAG_TIMING = 1,    /* record HIP events around the search kernels; see unify_last_timing */
  UNIFY_FLAG_SELECT_S1 = 2,  /* hybrid neighbour selection S1 (Sec. 4.2): rank every entry of the
                                active chunks by its distance to the expanded object and take the
                                m nearest, instead of the first ceil(m / S') of each chunk (S2) */
  UNIFY_FLAG_PRE_WAVE_SCAN = 4,  /* strategy A by one scan per query and wavefront instead of the
                                    shared matrix-core scan (same results) */
  UNIFY_FLAG_SERIAL_PHASES = 8   /* run the matrix-core scan before the graph-search kernel instead
                                    of beside it on a second stream (same results; each phase's
                                    timing is then its own) */
};

/* Search parameters.  Zero in a field selects its default.  The first six fields
 * are the search's own parameters (m and the strategy thresholds of Sec. 4.2 and
 * Sec. 5.2, plus the beam width and rerank depth of this implementation); the
 * fields after `flags` size on-chip structures and never change a result. */
typedef struct {
  int32_t m;            /* neighbours examined per expansion in the hybrid search,
                           ceil(m / S') from each active chunk (Sec. 4.2); default M0 */
  int32_t beam_p;       /* candidates expanded together per step, 1..8; default 1 (= Alg. 7) */
  int32_t rerank_mult;  /* BF16/FP8 stores: FP32 rerank of the best rerank_mult * k
                           graph results; default 4 */
  double tau_a_frac;    /* tau_A = floor(tau_a_frac * n); default 0.01 (Sec. 5.2) */
  double tau_b_frac;    /* tau_B = ceil(tau_b_frac * n); default 0.5 (Sec. 5.2) */
  uint32_t flags;       /* UNIFY_FLAG_* bits, 0 for none */
  int32_t cand_cap;     /* on-chip candidate entries per query, a power of two in
                           [64, 4096]; default the larger of 512 and 8 * ef rounded up to
                           a power of two.  Queries that need more are re-run with a
                           larger array (same results). */
  int32_t visit_cap;    /* on-chip visited-cache entries per query, a power of two in
                           [256, 16384]; default 1024 for the FP32 store, 512 for BF16 /
                           FP8 (more wavefronts fit; larger visited sets spill to HBM,
                           same results) */
  int32_t pre_chunk;    /* pre-filter scans with k <= 128 split their slice into chunks of
                           about this many objects (at most 8 chunks), scanned by different
                           wavefronts and merged exactly; default 2048, minimum 64 */
  int32_t waves_per_query;  /* 1 (default), 2 or 4: wavefronts that run each heavy graph
                               search together (same results; not with selection S1) */
  int32_t heavy_queries;    /* graph searches of a batch run that way at most: the first in the
                               work list, which starts with the narrowest hybrid ranges;
                               default the number of compute units */
} unify_params;

/*
 * Reads an index file holding an HSIG as Sec. 4.1 lays it out (per layer, one
 * chunk of at most M neighbours per segment for every object; the global-edge
 * bitmap of Alg. 5; objects in attribute order, the order the layer-0 skip list
 * walks) and makes it resident on HIP device `device`.  File format:
 * little-endian, see the package documentation.  precision selects the store the graph
 * searches read (UNIFY_FP32, UNIFY_BF16, UNIFY_FP8E4M3); the FP32 store is always
 * resident for the pre-filter scan and the rerank.  The file's tables are checked
 * (checksum, sizes, every adjacency entry in range); on any failure *out is left
 * unchanged.  *out (host) receives a handle owned by the library.
 */
int unify_load_index(const char* path, int device, int precision, unify_index_t* out);

/*
 * Builds an HSIG on device `device` from host arrays and makes it resident.
 *   vectors   host, [n][d] float32 row-major; row i has external id i
 *   attr      host, [n] int64 attribute values
 *   level_u   host, [n] float64 in (0, 1]: the uniform variate of each object's
 *             level draw (level = floor(-ln(u) / ln(M)), Alg. 6)
 *   S, M      segments and chunk capacity (Sec. 4.1); ef_cons candidates per chunk
 * Construction is batched on the GPU (every chunk from exact per-segment
 * candidates, then the Prune rule and reverse edges of Alg. 4, and the global-edge
 * marking of Alg. 5); it is not the sequential insertion order of Alg. 6.
 */
int unify_build_index(const float* vectors, const int64_t* attr, const double* level_u, int64_t n,
                      int32_t d, int32_t S, int32_t M, int32_t ef_cons, int device, int precision,
                      unify_index_t* out);

/*
 * Incremental insertion (Alg. 6, HSIGInsert; the paper's incremental-construction
 * objective) of m more objects into a resident index.
 *   vectors   host, [m][d] float32 row-major; row t takes external id X + t, where X
 *             is one more than the largest external id already in the index
 *   attr      host, [m] int64 attribute values
 *   level_u   host, [m] float64 in (0, 1]: the level variates, as for unify_build_index
 * Segment boundaries stay those of the index (each new object joins the segment its
 * attribute falls in).  The library builds a new version of the resident tables in
 * merged attribute order, connects the new objects on every layer they reach (chunks
 * from exact per-segment candidates and Prune, reverse edges into the chunks of
 * their neighbours, which are re-pruned when they overflow, Alg. 4), recomputes the
 * global-edge marks of those layers from their final chunks (Alg. 5), and swaps the
 * new version in: searches already enqueued finish on the old version, later ones
 * see every object.  Concurrent searches on other threads are allowed; batches
 * created before the call must be created again (unify_batch_run then fails with
 * UNIFY_EINVAL).  The low-precision store in use is rebuilt; other copies are
 * dropped.  Synchronous; m = 0 does nothing.  Errors: UNIFY_EINVAL (null arrays,
 * m < 0, a level variate outside (0, 1], more than 2^31 - 1 objects in total),
 * UNIFY_ENOMEM, UNIFY_EDEVICE; on error the index is unchanged.
 */
int unify_insert(unify_index_t index, const float* vectors, const int64_t* attr, const double* level_u,
                 int64_t m);

/*
 * Prune (Sec. 2.2, the neighbour selection of Alg. 4 and Alg. 5) as the GPU builder
 * runs it, on caller-given candidate lists: for task i, owner owners[i] and
 * candidates cand[i][0 .. c) (ids into vectors, -1 for none), the candidates are
 * ordered by (FP32 squared distance to the owner, id), the owner itself and repeated
 * ids dropped, and each is kept unless an already kept one is strictly nearer to
 * it than the owner is, until M are kept.  Exposed for callers that assemble
 * their own candidate lists.
 *   vectors  device, [n][d] float32 (d % 4 == 0, 4 <= d <= 2048)
 *   owners   device, [t] int32 ids into vectors
 *   cand     device, [t][c] int32, 1 <= c <= 256
 *   out      device, [t][M] int32 kept ids in selection order, -1 padded; 1 <= M <= 64
 *   hip_stream  stream to enqueue on (scratch is allocated on it), or NULL
 * Asynchronous; t = 0 is a no-op.  UNIFY_EINVAL for out-of-range sizes or null buffers.
 */
int unify_prune(const float* vectors, int64_t n, int32_t d, const int32_t* owners, const int32_t* cand,
                int64_t t, int32_t c, int32_t M, int32_t* out, void* hip_stream);

/*
 * Reads and checks an index file on the host only (no GPU needed): header,
 * checksum, section sizes and the range of every adjacency entry.  Outputs are
 * host pointers, any may be NULL.  Returns UNIFY_EIO or UNIFY_EFORMAT on failure.
 */
int unify_validate_index_file(const char* path, int64_t* n, int32_t* d, int32_t* S, int32_t* M);

/* Writes a resident index to `path` in the index file format. */
int unify_save_index(unify_index_t index, const char* path);

/* Sizes of a resident index (host outputs; any may be NULL), in the notation of
 * Sec. 4.1 and Table 1: n objects of dimension d, S segments, chunk capacity M,
 * levels = top layer + 1 (the layer count of the hierarchy, Alg. 6's L + 1).
 * UNIFY_EINVAL for a null index. */
int unify_index_info(unify_index_t index, int64_t* n, int32_t* d, int32_t* S, int32_t* M,
                     int32_t* levels);

/*
 * Range-filtered k-NN search of nq queries (Definition 1; Sec. 4.2).
 *   queries       device, [nq][d] float32
 *   l, h          device, [nq] int64, inclusive attribute range of each query
 *   k             1 <= k <= 256
 *   ef            result-list size of the graph searches; k <= ef <= 256 when any
 *                 query runs the hybrid or post-filter search
 *   strategy      device, [nq] int8 per-query strategy (UNIFY_AUTO .. UNIFY_POST),
 *                 or NULL for UNIFY_AUTO on every query.  The values are read on the
 *                 device, so an unknown one cannot fail the call: its row is padded
 *                 and out_strategy reports -2 for it
 *   params        host, or NULL for defaults
 *   out_ids       device, [nq][k] int64
 *   out_dist      device, [nq][k] float32
 *   out_strategy  device, [nq] int8 strategy of each row (the rule's choice or the
 *                 requested one; an empty range runs nothing and pads its row; -2:
 *                 unknown requested strategy), or NULL
 *   hip_stream    hipStream_t to enqueue on, or NULL
 * nq = 0 is a no-op.  Scratch space is allocated by the library per call.
 * Calls may come from several threads and streams: the search kernels of
 * successive calls on one index run one after another (they share the index's
 * visited-set memory: per resident wavefront, a bitmap of the n objects and a
 * 32 KiB log, 16 wavefronts per compute unit, made when the index becomes
 * resident), ordered by an event the library records.  Serving slots hold
 * visited memory of their own and run concurrently with these calls.
 */
int unify_search(unify_index_t index, const float* queries, int64_t nq, const int64_t* l,
                 const int64_t* h, int32_t k, int32_t ef, const int8_t* strategy,
                 const unify_params* params, int64_t* out_ids, float* out_dist,
                 int8_t* out_strategy, void* hip_stream);

/*
 * unify_search plus per-query counters:
 *   out_stats  device, [nq][8] int32: [0] distance evaluations, [1] expansions,
 *              [2] FP32 re-scores of a BF16 / FP8 search, [3] status in bits 0-7
 *              (0 = answered in the first search pass, 1 = re-run: with larger on-chip
 *              lists for a graph search, by the FP32 scan for a low-precision pre-filter
 *              scan whose bounds could not settle the result, 2 = capacity exceeded even
 *              then: the row is padded, 3 = the requested strategy is not one of
 *              UNIFY_AUTO..UNIFY_POST: the row is padded) and flag bits above: bit 8 =
 *              a layer search met ids whose set of the on-chip visited cache was full
 *              and recorded them in HBM (same results), bit 9 = several wavefronts ran
 *              the graph search together (waves_per_query; which searches run so can
 *              differ between calls), [4] adjacency
 *              entries read (a pre-filter row answered
 *              by the matrix-core scan: the super-blocks its slice spans; 0 when it was
 *              scanned per wavefront), [5] strategy run (-1 for
 *              an empty range, -2 for an unknown requested strategy), [6] Y = objects in
 *              range, [7] active segments (hybrid only, else 0).
 */
int unify_search_ex(unify_index_t index, const float* queries, int64_t nq, const int64_t* l,
                    const int64_t* h, int32_t k, int32_t ef, const int8_t* strategy,
                    const unify_params* params, int64_t* out_ids, float* out_dist,
                    int8_t* out_strategy, int32_t* out_stats, void* hip_stream);

/*
 * unify_search_ex for callers that cannot allocate: code under HIP graph capture,
 * serving loops that must not call hipMalloc, harnesses that forbid allocation.
 * Arguments, results and errors are those of unify_search_ex (UNIFY_FLAG_TIMING is
 * ignored).  The call allocates no device, pinned or host memory: the per-call
 * scratch (query plans, the work list, partial lists of split pre-filter scans)
 * lives in one static device array of 32 MiB that every GPU the library runs on
 * holds until the process ends, and the visited-set memory was allocated when the
 * index became resident.  A call needing more scratch than the array holds (about
 * nq * (64 * k + 120) bytes when k <= 128, nq * 120 bytes otherwise) fails with
 * UNIFY_EINVAL before launching anything: split the batch.  Every call on one GPU
 * uses the same array, which keeps the last call's contents (each call writes what
 * it reads).  Calls on one index are ordered on the device (each waits for the
 * previous one's kernels); calls on two indexes of one GPU that overlap on the
 * device race on the array and return wrong results: the caller serialises them.
 */
int unify_search_ex_noalloc(unify_index_t index, const float* queries, int64_t nq, const int64_t* l,
                            const int64_t* h, int32_t k, int32_t ef, const int8_t* strategy,
                            const unify_params* params, int64_t* out_ids, float* out_dist,
                            int8_t* out_strategy, int32_t* out_stats, void* hip_stream);

/*
 * Second attribute for conjunctive two-attribute queries (the paper's
 * multi-attribute extension, approach 1: the HSIG stays built on the first
 * attribute; the filter also tests the second).
 *   attr2   host, [n] int64: the second attribute of the object with external id e is
 *           attr2[e] (the index's external ids must be 0 .. n-1)
 * Replaces a previous second attribute once the searches already enqueued have
 * finished.  unify_insert drops it (set it again for the grown index).
 * Errors: UNIFY_EINVAL (n is not the index's object count, external ids not dense),
 * UNIFY_ENOMEM, UNIFY_EDEVICE.
 */
int unify_set_attr2(unify_index_t index, const int64_t* attr2, int64_t n);

/*
 * Conjunctive range-filtered k-NN: the k nearest objects with l <= attribute <= h AND
 * l2 <= second attribute <= h2 (Alg. 7's ann admission, the post-filter test and the
 * pre-filter scan test both ranges).  Arguments as unify_search_ex, plus
 *   l2, h2  device, [nq] int64, inclusive ranges on the second attribute
 * The strategy rule and the entry segments follow the first range only (the index
 * knows the first attribute's distribution); fewer than k results pad the row.
 * Errors: as unify_search, and UNIFY_EINVAL when no second attribute is set.
 */
int unify_search_multi(unify_index_t index, const float* queries, int64_t nq, const int64_t* l,
                       const int64_t* h, const int64_t* l2, const int64_t* h2, int32_t k, int32_t ef,
                       const int8_t* strategy, const unify_params* params, int64_t* out_ids,
                       float* out_dist, int8_t* out_strategy, int32_t* out_stats, void* hip_stream);

/*
 * The z-order composite attribute (the paper's multi-attribute extension, approach 2,
 * Sec. 5.9: one HSIG built on a one-dimensional z-order attribute of the pair (A1, A2)).
 * Each attribute maps to an order-preserving coordinate on an axis of 2^31 cells:
 *   u(x) = 0 for x <= base, else min(scale(x - base), 2^31 - 1)   (x - base modulo 2^64),
 *   scale(t) = t >> shift for shift >= 0, t << -shift (2^31 - 1 when that overflows) else,
 * and the key of a pair interleaves the coordinates' bits: bit j of u1 is bit 2j + 1
 * of the key, bit j of u2 bit 2j (keys are in [0, 2^62)).  Build the index with the
 * keys as its attribute (unify_build_index), attach the pairs (unify_set_zorder), and
 * search boxes (unify_search_box).
 */
typedef struct {
  int64_t base1, base2;    /* each attribute's smallest value */
  int32_t shift1, shift2;  /* in [-30, 63] */
} unify_zmap;

/*
 * The map of n pairs: base = the attribute's smallest value, shift = bits(largest -
 * base) - 31 (0 when all values are equal), so both attributes spread over the whole
 * axis (the largest value lands in its upper half).
 *   a1, a2  host, [n] int64
 *   out     host
 * Errors: UNIFY_EINVAL (null argument, n < 0).
 */
int unify_zorder_map(const int64_t* a1, const int64_t* a2, int64_t n, unify_zmap* out);

/*
 * The z-order keys of n pairs under map (the build's attribute values).
 *   a1, a2  host, [n] int64;  out  host, [n] int64
 * Errors: UNIFY_EINVAL (null argument, n < 0, a shift outside [-30, 63]).
 */
int unify_zorder_keys(const unify_zmap* map, const int64_t* a1, const int64_t* a2, int64_t n, int64_t* out);

/*
 * Attaches both attributes to an index built on their z-order keys under map: the
 * pair of the object with external id e is (a1[e], a2[e]) (external ids 0 .. n-1).
 * Every object's attribute must equal its pair's key.  Replaces earlier pairs once
 * the searches already enqueued have finished; unify_insert drops them.
 *   map     host;  a1, a2  host, [n] int64
 * Errors: UNIFY_EINVAL (n is not the index's object count, external ids not dense, an
 * object whose attribute is not its pair's key, a bad map), UNIFY_ENOMEM, UNIFY_EDEVICE.
 */
int unify_set_zorder(unify_index_t index, const unify_zmap* map, const int64_t* a1, const int64_t* a2,
                     int64_t n);

/*
 * Box search on a z-order index: the k nearest objects with l1 <= A1 <= h1 AND
 * l2 <= A2 <= h2.  The HSIG is searched on the key range [key(u1(l1), u2(l2)),
 * key(u1(h1), u2(h2))], which holds every object of the box, and admits box objects
 * only (Alg. 7's ann admission, the post-filter test and the pre-filter scan test
 * both attributes; the pre-filter scan jumps over the key runs whose cells lie outside
 * the box).  Strategy rule (UNIFY_AUTO): with Y the objects of the key range
 * and c the sampled pairs in the box (the pairs of the objects at internal ids
 * floor(j n / ns), j < ns = min(n, 2048)), pre-filter when Y <= tau_a n or
 * c n <= tau_a n ns, post-filter when c n >= tau_b n ns, else hybrid (tau_a n rounded
 * down, tau_b n up).  Arguments as unify_search_ex, with
 *   l1, h1, l2, h2  device, [nq] int64, inclusive ranges on A1 and A2 (an empty range
 *                   pads the row)
 * Errors: as unify_search, and UNIFY_EINVAL when no pairs are attached.
 */
int unify_search_box(unify_index_t index, const float* queries, int64_t nq, const int64_t* l1,
                     const int64_t* h1, const int64_t* l2, const int64_t* h2, int32_t k, int32_t ef,
                     const int8_t* strategy, const unify_params* params, int64_t* out_ids, float* out_dist,
                     int8_t* out_strategy, int32_t* out_stats, void* hip_stream);

/*
 * Disjunctive two-attribute queries (the paper's multi-attribute extension,
 * approach 1): with one index per attribute over the same objects, search each
 * with its own range and merge the two [nq][k] result lists of every query here.
 * The merge keeps the k smallest (distance, external id) pairs, an object found
 * by both searches once (it carries the same canonical FP32 distance in both).
 * All arrays are device memory in the layout unify_search writes (ascending,
 * -1 / +inf padded); out_* may not alias the inputs.  Enqueued on hip_stream.
 * Errors: UNIFY_EINVAL (k < 1, nq < 0, null arrays), UNIFY_EDEVICE.
 */
int unify_merge_or(const int64_t* ids_a, const float* dist_a, const int64_t* ids_b, const float* dist_b,
                   int64_t nq, int32_t k, int64_t* out_ids, float* out_dist, void* hip_stream);

/*
 * Durations of the kernels of the last unify_search* call on this index that set
 * UNIFY_FLAG_TIMING, from HIP events recorded on that call's streams:
 *   plan_ms     everything before the graph-search kernel: plan and work list (and,
 *               with UNIFY_FLAG_SERIAL_PHASES, the matrix-core pre-filter scan);
 *   search_ms   the graph-search launch (graph searches and the pre-filter scans that
 *               run per wavefront), by default concurrent with the matrix-core scan,
 *               until both have finished, and the merge of split scans;
 *   rerun_ms    the launch that re-runs queries whose on-chip lists overflowed.
 * Waits for the events to complete.  Outputs are host pointers, any may be NULL.
 * Returns UNIFY_EINVAL when no timed search has been issued.
 */
int unify_last_timing(unify_index_t index, float* plan_ms, float* search_ms, float* rerun_ms);

/*
 * The same, phase by phase: out_ms (host, n entries, 1 <= n <= 7) receives in order
 * the plan and work list; the matrix-core scan's set-up (query split, super-block
 * lists); its scan kernel; its results (FP32 re-scores); the graph-search kernel;
 * the merge of split scans (with, by default, the wait for the matrix-core scan,
 * which runs beside the graph search); the re-run.  Phases that did not run last
 * 0 ms.  The graph-search phase starts after the work list (after the matrix-core
 * scan with UNIFY_FLAG_SERIAL_PHASES).
 */
int unify_last_timing_ex(unify_index_t index, float* out_ms, int32_t n);

/*
 * Selects the store later searches on this index rank by (UNIFY_FP32, UNIFY_BF16,
 * UNIFY_FP8E4M3), building the copy on the device the first time a precision is
 * selected; copies stay resident until unify_free_index.  Searches already
 * enqueued keep the store they were issued with.  Not to be called concurrently
 * with other calls on the same index.
 */
int unify_set_precision(unify_index_t index, int precision);

/*
 * Copies a resident low-precision store of an index (one loaded or built with
 * precision UNIFY_BF16 / UNIFY_FP8E4M3, or selected by unify_set_precision), for
 * inspection or export, in internal-id order
 * (attribute order):
 *   codes   device, [n][d] uint16 BF16 patterns or uint8 E4M3 codes, or NULL
 *   scales  device, [n] float32 FP8 scales (value = code value * scale), or NULL;
 *           ignored for BF16
 *   eps     device, [n] float32 upper bounds on the Euclidean norm of
 *           (stored values - FP32 vector), or NULL
 * Enqueued on hip_stream.  UNIFY_EINVAL when the index holds no store of that precision.
 */
int unify_copy_store(unify_index_t index, int precision, void* codes, float* scales, float* eps,
                     void* hip_stream);

/*
 * Batched form for fixed-size batches (serving loops, benchmark replays): the
 * whole search of unify_search_ex over the given buffers (plan, work list,
 * search, merge, re-run) is captured once into a HIP graph, with its scratch
 * allocated once; each unify_batch_run replays it on the caller's stream and
 * reads whatever the buffers hold at that time.  Arguments are those of
 * unify_search_ex (nq >= 1; out_stats may be NULL); the buffers stay owned by
 * the caller and must stay allocated, at the same addresses, until
 * unify_batch_free.  The search parameters and the index's store at creation
 * are kept.  Replays of one batch must not overlap; the index must outlive it.
 */
typedef struct unify_batch* unify_batch_t;
int unify_batch_create(unify_index_t index, const float* queries, int64_t nq, const int64_t* l, const int64_t* h,
                       int32_t k, int32_t ef, const int8_t* strategy, const unify_params* params,
                       int64_t* out_ids, float* out_dist, int8_t* out_strategy, int32_t* out_stats,
                       unify_batch_t* out);
int unify_batch_run(unify_batch_t batch, void* hip_stream);
int unify_batch_free(unify_batch_t batch);  /* NULL is accepted */

/*
 * Serving: continuous batching over a resident index (one worker thread per
 * server).  Requests are submitted from host memory with an arrival time; the
 * worker admits the requests that have arrived into a batch whenever one of
 * its `inflight` slots is free, searches it on the slot's stream and completes
 * the requests when the slot's event fires.  Each slot holds pinned staging,
 * device buffers and scratch for a batch and its own visited-set memory, all
 * allocated at creation (again only after an insertion grows the index), so
 * the search kernels of different slots run concurrently on the device.
 * Admission is by device memory: the batch size (at most max_batch), then the
 * visited rows of each slot (at most one per resident wavefront of the device),
 * halve until `inflight` slots fit mem_budget bytes; unify_server_limits
 * reports the outcome.  Each slot runs on one stream (the matrix-core scan before
 * the graph search; a second stream only for cooperative searches).  Slots overlap
 * on the device only on different hardware queues: HIP shares GPU_MAX_HW_QUEUES
 * queues (4 by default) among all streams of a process, in order, so a serving
 * process with more slots than free queues should raise it.  Every request's
 * result is the one unify_search returns for it alone.
 */
typedef struct unify_server* unify_server_t;
typedef struct {
  int32_t k, ef;          /* results per request and beam, as for unify_search */
  int32_t max_batch;      /* requests per launch at most; default 4096 */
  int32_t inflight;       /* batches in flight, 1..8; default 2 */
  double max_wait_s;      /* a partial batch waits until its oldest request has waited this
                             long (0: it launches as soon as a slot is free) */
  unify_params params;    /* search parameters (flags ignored) */
  int64_t mem_budget;     /* device bytes the slots may hold; 0: half the free device memory.
                             UNIFY_ENOMEM when it holds no slots of 64 queries and 64 rows */
} unify_server_config;

int unify_server_create(unify_index_t index, const unify_server_config* config, unify_server_t* out);
/* Submits n requests (host arrays: queries [n][d] f32, l, h [n] i64, strategy [n]
 * i8 or NULL for UNIFY_AUTO).  arrive_s [n] (or NULL for now): seconds from the
 * call at which each request arrives; the worker ignores a request until then
 * (an open-loop arrival process).  tickets [n] receives one id per request. */
int unify_server_submit(unify_server_t server, int64_t n, const float* queries, const int64_t* l,
                        const int64_t* h, const int8_t* strategy, const double* arrive_s, int64_t* tickets);
/* Waits for n tickets (timeout_s <= 0: no limit) and copies their results to host
 * arrays ids [n][k], dist [n][k] and latency_s [n] (completion - arrival), any may
 * be NULL.  UNIFY_EIO on time-out.  Results stay retrievable until the server is freed. */
int unify_server_wait(unify_server_t server, int64_t n, const int64_t* tickets, int64_t* ids, float* dist,
                      double* latency_s, double timeout_s);
/* The admission the memory budget allowed: requests per batch, visited rows per slot,
 * and the device bytes all slots hold (any pointer may be NULL). */
int unify_server_limits(unify_server_t server, int64_t* max_batch, int64_t* visit_rows,
                        int64_t* device_bytes);
/* Requests completed, batches launched, and seconds with at least one batch in flight. */
int unify_server_stats(unify_server_t server, int64_t* completed, int64_t* batches, double* busy_s);
/* Serves every submitted request, stops the worker and frees the server (NULL accepted). */
int unify_server_free(unify_server_t server);

/* Frees an index returned by unify_load_index or unify_build_index and all device
 * memory it holds (tables, low-precision copies, visited-set memory).  Waits for the
 * searches enqueued on it.  Batches and servers over it must be freed first.  Not a
 * step of the method: the handle's lifetime under the ownership rule above.  NULL is
 * accepted. */
int unify_free_index(unify_index_t index);

/* Message of the last failure on the calling thread (never NULL). */
const char* unify_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* UNIFY_H */
