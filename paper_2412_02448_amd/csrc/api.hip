// C ABI: index residency (load, upload, free, save) and the search entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "unify_internal.h"
#include "zorder.h"

namespace unify {

int build_impl(const float* vectors, const int64_t* attr, const double* level_u, int64_t n, int32_t d, int32_t S,
               int32_t M, int32_t ef_cons, int device, int precision, unify_index_t* out);
int search_impl(unify_index_t ix, const float* queries, int64_t nq, const int64_t* l, const int64_t* h,
                int32_t k, int32_t ef, const int8_t* strategy, const unify_params* prm, int64_t* out_ids,
                float* out_dist, int8_t* out_strategy, int32_t* out_stats, void* stream);
int search_multi_impl(unify_index_t ix, const float* queries, int64_t nq, const int64_t* l, const int64_t* h,
                      const int64_t* l2, const int64_t* h2, int32_t k, int32_t ef, const int8_t* strategy,
                      const unify_params* prm, int64_t* out_ids, float* out_dist, int8_t* out_strategy,
                      int32_t* out_stats, void* stream);
int search_box_impl(unify_index_t ix, const float* queries, int64_t nq, const int64_t* l1, const int64_t* h1,
                    const int64_t* l2, const int64_t* h2, int32_t k, int32_t ef, const int8_t* strategy,
                    const unify_params* prm, int64_t* out_ids, float* out_dist, int8_t* out_strategy,
                    int32_t* out_stats, void* stream);
int search_impl_noalloc(unify_index_t ix, const float* queries, int64_t nq, const int64_t* l, const int64_t* h,
                        int32_t k, int32_t ef, const int8_t* strategy, const unify_params* prm, int64_t* out_ids,
                        float* out_dist, int8_t* out_strategy, int32_t* out_stats, void* stream);

namespace {
thread_local std::string g_error;
}

void set_error(const std::string& msg) { g_error = msg; }

namespace {

template <class T>
int upload(unify_index_t ix, const std::vector<T>& v, const T** out) {
  if (v.empty()) {
    *out = nullptr;
    return UNIFY_OK;
  }
  void* p = nullptr;
  if (hipMalloc(&p, v.size() * sizeof(T)) != hipSuccess) {
    set_error("device allocation failed");
    return UNIFY_ENOMEM;
  }
  ix->allocs.push_back(p);
  if (hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("host-to-device copy failed");
    return UNIFY_EDEVICE;
  }
  *out = static_cast<const T*>(p);
  return UNIFY_OK;
}

// Global edges in bit order, -1 padded to GC entries per row.
void compact_glist(const std::vector<int32_t>& adj, const std::vector<uint32_t>& bits, int64_t rows, int S,
                   int mc, int W, int GC, std::vector<int32_t>& out) {
  out.assign((size_t)rows * GC, -1);
  for (int64_t r = 0; r < rows; ++r) {
    int c = 0;
    for (int w = 0; w < W && c < GC; ++w) {
      for (uint32_t m = bits[(size_t)r * W + w]; m && c < GC; m &= m - 1) {
        const int pos = 32 * w + __builtin_ctz(m);
        if (pos >= S * mc) break;
        const int32_t t = adj[((size_t)r * S) * mc + pos];
        if (t >= 0) out[(size_t)r * GC + c++] = t;
      }
    }
  }
}

}  // namespace

// Makes HostIndex H resident on `device`; takes ownership of H's tables.
int make_resident(HostIndex&& H, int device, int precision, unify_index_t* out) {
  if (precision < UNIFY_FP32 || precision > UNIFY_FP8E4M3) {
    set_error("unknown precision");
    return UNIFY_EINVAL;
  }
  if (hipSetDevice(device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return UNIFY_EDEVICE;
  }
  unify_index_t ix = new unify_index();
  ix->device = device;
  DevIndex& dv = ix->dv;
  dv.n = H.n;
  dv.d = H.d;
  dv.S = H.S;
  dv.M0 = H.M0;
  dv.MU = H.MU;
  dv.L = H.L;
  dv.gentry = H.gentry;
  dv.R = H.R;
  dv.precision = precision;
  // global-edge lists: as wide as the most marks on any row
  int GC = 1;
  auto widest = [&](const std::vector<uint32_t>& bits, int W) {
    size_t rows = W ? bits.size() / W : 0;
    for (size_t r = 0; r < rows; ++r) {
      int c = 0;
      for (int w = 0; w < W; ++w) c += __builtin_popcount(bits[r * W + w]);
      GC = std::max(GC, c);
    }
  };
  widest(H.gbits0, H.W0);
  widest(H.gbitsU, H.WU);
  dv.GC = GC;
  std::vector<int32_t> g0, gU;
  compact_glist(H.adj0, H.gbits0, H.n, H.S, H.M0, H.W0, GC, g0);
  compact_glist(H.adjU, H.gbitsU, H.R, H.S, H.MU, H.WU, GC, gU);
  int rc = UNIFY_OK;
  auto up = [&](auto& vec, auto** dst) {
    if (rc == UNIFY_OK) rc = upload(ix, vec, dst);
  };
  up(H.attr, &dv.attr);
  up(H.ext, &dv.ext);
  up(H.seg_start, &dv.seg_start);
  up(H.seg_entry, &dv.seg_entry);
  up(H.seg_maxlevel, &dv.seg_maxlevel);
  up(H.uprow, &dv.uprow);
  up(H.vec, &dv.vec);
  up(H.adj0, &dv.adj0);
  up(g0, &dv.glist0);
  up(H.adjU, &dv.adjU);
  up(gU, &dv.glistU);
  if (rc == UNIFY_OK) rc = quantize_store(ix, precision);
  if (rc == UNIFY_OK) rc = ensure_pool(ix);
  if (rc != UNIFY_OK) {
    pool_free(ix->pool);
    for (void* p : ix->allocs) (void)hipFree(p);
    delete ix;
    return rc;
  }
  // keep the small tables on the host; drop the big ones
  ix->host = std::move(H);
  std::vector<float>().swap(ix->host.vec);
  std::vector<int32_t>().swap(ix->host.adj0);
  std::vector<int32_t>().swap(ix->host.adjU);
  std::vector<uint32_t>().swap(ix->host.gbits0);
  std::vector<uint32_t>().swap(ix->host.gbitsU);
  *out = ix;
  return UNIFY_OK;
}

}  // namespace unify

using namespace unify;

extern "C" {

const char* unify_last_error(void) { return g_error.c_str(); }

int unify_validate_index_file(const char* path, int64_t* n, int32_t* d, int32_t* S, int32_t* M) {
  if (!path) {
    set_error("null path");
    return UNIFY_EINVAL;
  }
  HostIndex H;
  std::string err;
  int rc = read_index_file(path, H, err);
  if (rc != UNIFY_OK) {
    set_error(err);
    return rc;
  }
  if (n) *n = H.n;
  if (d) *d = H.d;
  if (S) *S = H.S;
  if (M) *M = H.M0;
  return UNIFY_OK;
}

int unify_load_index(const char* path, int device, int precision, unify_index_t* out) {
  if (!path || !out) {
    set_error("null argument");
    return UNIFY_EINVAL;
  }
  HostIndex H;
  std::string err;
  int rc = read_index_file(path, H, err);
  if (rc != UNIFY_OK) {
    set_error(err);
    return rc;
  }
  return make_resident(std::move(H), device, precision, out);
}

int unify_save_index(unify_index_t ix, const char* path) {
  if (!ix || !path) {
    set_error("null argument");
    return UNIFY_EINVAL;
  }
  if (hipSetDevice(ix->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return UNIFY_EDEVICE;
  }
  std::shared_lock<std::shared_mutex> version(ix->version_mu);
  HostIndex H = ix->host;
  const DevIndex& dv = ix->dv;
  H.vec.resize((size_t)dv.n * dv.d);
  H.adj0.resize((size_t)dv.n * dv.S * dv.M0);
  H.adjU.resize((size_t)dv.R * dv.S * dv.MU);
  bool ok = hipMemcpy(H.vec.data(), dv.vec, H.vec.size() * 4, hipMemcpyDeviceToHost) == hipSuccess &&
            hipMemcpy(H.adj0.data(), dv.adj0, H.adj0.size() * 4, hipMemcpyDeviceToHost) == hipSuccess &&
            (H.adjU.empty() ||
             hipMemcpy(H.adjU.data(), dv.adjU, H.adjU.size() * 4, hipMemcpyDeviceToHost) == hipSuccess);
  if (!ok) {
    set_error("device-to-host copy failed");
    return UNIFY_EDEVICE;
  }
  // rebuild the bitmaps from the compacted global-edge lists
  std::vector<int32_t> g0((size_t)dv.n * dv.GC), gU((size_t)dv.R * dv.GC);
  ok = hipMemcpy(g0.data(), dv.glist0, g0.size() * 4, hipMemcpyDeviceToHost) == hipSuccess &&
       (gU.empty() || hipMemcpy(gU.data(), dv.glistU, gU.size() * 4, hipMemcpyDeviceToHost) == hipSuccess);
  if (!ok) {
    set_error("device-to-host copy failed");
    return UNIFY_EDEVICE;
  }
  auto bits_of = [&](const std::vector<int32_t>& adj, const std::vector<int32_t>& gl, int64_t rows, int mc,
                     int W, std::vector<uint32_t>& bits) {
    bits.assign((size_t)rows * W, 0u);
    for (int64_t r = 0; r < rows; ++r) {
      for (int t = 0; t < dv.GC; ++t) {
        int32_t g = gl[(size_t)r * dv.GC + t];
        if (g < 0) continue;
        for (int pos = 0; pos < dv.S * mc; ++pos)
          if (adj[(size_t)r * dv.S * mc + pos] == g) {
            bits[(size_t)r * W + (pos >> 5)] |= 1u << (pos & 31);
            break;
          }
      }
    }
  };
  bits_of(H.adj0, g0, dv.n, dv.M0, H.W0, H.gbits0);
  bits_of(H.adjU, gU, dv.R, dv.MU, H.WU, H.gbitsU);
  std::string err;
  int rc = write_index_file(path, H, err);
  if (rc != UNIFY_OK) set_error(err);
  return rc;
}

int unify_index_info(unify_index_t ix, int64_t* n, int32_t* d, int32_t* S, int32_t* M, int32_t* levels) {
  if (!ix) {
    set_error("null index");
    return UNIFY_EINVAL;
  }
  std::shared_lock<std::shared_mutex> version(ix->version_mu);
  if (n) *n = ix->dv.n;
  if (d) *d = ix->dv.d;
  if (S) *S = ix->dv.S;
  if (M) *M = ix->dv.M0;
  if (levels) *levels = ix->dv.L + 1;
  return UNIFY_OK;
}

int unify_copy_store(unify_index_t ix, int precision, void* codes, float* scales, float* eps, void* hip_stream) {
  if (!ix || precision < UNIFY_BF16 || precision > UNIFY_FP8E4M3 || !ix->eps_of[precision]) {
    set_error("unify_copy_store: the index holds no store of that precision");
    return UNIFY_EINVAL;
  }
  std::shared_lock<std::shared_mutex> version(ix->version_mu);
  const DevIndex& dv = ix->dv;
  hipStream_t st = (hipStream_t)hip_stream;
  const size_t cells = (size_t)dv.n * dv.d;
  bool ok = hipSetDevice(ix->device) == hipSuccess;
  if (ok && codes) {
    const void* src = precision == UNIFY_BF16 ? (const void*)dv.vec_bf16 : (const void*)dv.vec_fp8;
    ok = hipMemcpyAsync(codes, src, cells * (precision == UNIFY_BF16 ? 2 : 1), hipMemcpyDeviceToDevice, st) ==
         hipSuccess;
  }
  if (ok && scales && precision == UNIFY_FP8E4M3)
    ok = hipMemcpyAsync(scales, dv.vec_scale, sizeof(float) * dv.n, hipMemcpyDeviceToDevice, st) == hipSuccess;
  if (ok && eps) ok = hipMemcpyAsync(eps, dv.vec_eps, sizeof(float) * dv.n, hipMemcpyDeviceToDevice, st) == hipSuccess;
  if (!ok) {
    set_error("unify_copy_store: copy failed");
    return UNIFY_EDEVICE;
  }
  return UNIFY_OK;
}

int unify_set_precision(unify_index_t ix, int precision) {
  if (!ix || precision < UNIFY_FP32 || precision > UNIFY_FP8E4M3) {
    set_error("unify_set_precision: bad arguments");
    return UNIFY_EINVAL;
  }
  if (hipSetDevice(ix->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return UNIFY_EDEVICE;
  }
  std::unique_lock<std::shared_mutex> version(ix->version_mu);
  return quantize_store(ix, precision);
}

int unify_search(unify_index_t ix, const float* queries, int64_t nq, const int64_t* l, const int64_t* h,
                 int32_t k, int32_t ef, const int8_t* strategy, const unify_params* params, int64_t* out_ids,
                 float* out_dist, int8_t* out_strategy, void* hip_stream) {
  return search_impl(ix, queries, nq, l, h, k, ef, strategy, params, out_ids, out_dist, out_strategy, nullptr,
                     hip_stream);
}

int unify_search_ex(unify_index_t ix, const float* queries, int64_t nq, const int64_t* l, const int64_t* h,
                    int32_t k, int32_t ef, const int8_t* strategy, const unify_params* params, int64_t* out_ids,
                    float* out_dist, int8_t* out_strategy, int32_t* out_stats, void* hip_stream) {
  return search_impl(ix, queries, nq, l, h, k, ef, strategy, params, out_ids, out_dist, out_strategy, out_stats,
                     hip_stream);
}

int unify_search_ex_noalloc(unify_index_t ix, const float* queries, int64_t nq, const int64_t* l, const int64_t* h,
                            int32_t k, int32_t ef, const int8_t* strategy, const unify_params* params,
                            int64_t* out_ids, float* out_dist, int8_t* out_strategy, int32_t* out_stats,
                            void* hip_stream) {
  return search_impl_noalloc(ix, queries, nq, l, h, k, ef, strategy, params, out_ids, out_dist, out_strategy,
                             out_stats, hip_stream);
}

int unify_search_multi(unify_index_t ix, const float* queries, int64_t nq, const int64_t* l, const int64_t* h,
                       const int64_t* l2, const int64_t* h2, int32_t k, int32_t ef, const int8_t* strategy,
                       const unify_params* params, int64_t* out_ids, float* out_dist, int8_t* out_strategy,
                       int32_t* out_stats, void* hip_stream) {
  return search_multi_impl(ix, queries, nq, l, h, l2, h2, k, ef, strategy, params, out_ids, out_dist, out_strategy,
                           out_stats, hip_stream);
}

int unify_search_box(unify_index_t ix, const float* queries, int64_t nq, const int64_t* l1, const int64_t* h1,
                     const int64_t* l2, const int64_t* h2, int32_t k, int32_t ef, const int8_t* strategy,
                     const unify_params* params, int64_t* out_ids, float* out_dist, int8_t* out_strategy,
                     int32_t* out_stats, void* hip_stream) {
  return search_box_impl(ix, queries, nq, l1, h1, l2, h2, k, ef, strategy, params, out_ids, out_dist, out_strategy,
                         out_stats, hip_stream);
}

int unify_zorder_map(const int64_t* a1, const int64_t* a2, int64_t n, unify_zmap* out) {
  if (!out || n < 0 || (n > 0 && (!a1 || !a2))) {
    set_error("unify_zorder_map: null argument or negative count");
    return UNIFY_EINVAL;
  }
  auto axis = [n](const int64_t* a, int64_t& base, int32_t& shift) {
    base = 0;
    shift = 0;
    if (n == 0) return;
    const auto mm = std::minmax_element(a, a + n);
    base = *mm.first;
    const uint64_t span = static_cast<uint64_t>(*mm.second) - static_cast<uint64_t>(*mm.first);
    // the span's top bit lands on the axis's bit 30
    if (span) shift = (64 - __builtin_clzll(span)) - 31;
  };
  axis(a1, out->base1, out->shift1);
  axis(a2, out->base2, out->shift2);
  return UNIFY_OK;
}

namespace {
bool zmap_ok(const unify_zmap* m) {
  return m && m->shift1 >= -30 && m->shift1 <= 63 && m->shift2 >= -30 && m->shift2 <= 63;
}
}  // namespace

int unify_zorder_keys(const unify_zmap* map, const int64_t* a1, const int64_t* a2, int64_t n, int64_t* out) {
  if (!zmap_ok(map) || n < 0 || (n > 0 && (!a1 || !a2 || !out))) {
    set_error("unify_zorder_keys: null argument, negative count or a shift outside [-30, 63]");
    return UNIFY_EINVAL;
  }
  for (int64_t i = 0; i < n; ++i)
    out[i] = zkey(zcoord(a1[i], map->base1, map->shift1), zcoord(a2[i], map->base2, map->shift2));
  return UNIFY_OK;
}

int unify_set_zorder(unify_index_t ix, const unify_zmap* map, const int64_t* a1, const int64_t* a2, int64_t n) {
  if (!ix || !zmap_ok(map) || (n > 0 && (!a1 || !a2))) {
    set_error("unify_set_zorder: null argument or a shift outside [-30, 63]");
    return UNIFY_EINVAL;
  }
  if (hipSetDevice(ix->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return UNIFY_EDEVICE;
  }
  std::unique_lock<std::shared_mutex> version(ix->version_mu);
  const int64_t N = ix->dv.n;
  if (n != N) {
    set_error("unify_set_zorder: one pair per object of the index");
    return UNIFY_EINVAL;
  }
  const std::vector<int64_t>& ext = ix->host.ext;
  const std::vector<int64_t>& attr = ix->host.attr;
  const int64_t ns = std::min<int64_t>(N, 2048);
  const int64_t Nr = std::max<int64_t>(N, 1);
  // a1, a2 in internal order, then the sampled pairs
  std::vector<int64_t> buf((size_t)(2 * Nr + 2 * ns));
  int64_t* b1 = buf.data();
  int64_t* b2 = b1 + Nr;
  for (int64_t i = 0; i < N; ++i) {
    const int64_t e = ext[i];
    if (e < 0 || e >= N) {
      set_error("unify_set_zorder: the index's external ids are not 0 .. n-1");
      return UNIFY_EINVAL;
    }
    b1[i] = a1[e];
    b2[i] = a2[e];
    if (attr[i] != zkey(zcoord(b1[i], map->base1, map->shift1), zcoord(b2[i], map->base2, map->shift2))) {
      set_error("unify_set_zorder: the index is not built on these pairs' z-order keys");
      return UNIFY_EINVAL;
    }
  }
  int64_t* s1 = b2 + Nr;
  int64_t* s2 = s1 + ns;
  for (int64_t j = 0; j < ns; ++j) {
    s1[j] = b1[j * N / ns];
    s2[j] = b2[j * N / ns];
  }
  void* p = nullptr;
  if (hipMalloc(&p, sizeof(int64_t) * buf.size()) != hipSuccess) {
    set_error("device allocation failed (z-order attributes)");
    return UNIFY_ENOMEM;
  }
  if (hipMemcpy(p, buf.data(), sizeof(int64_t) * buf.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(p);
    set_error("host-to-device copy failed");
    return UNIFY_EDEVICE;
  }
  // searches enqueued before (on any visited pool) may still read the previous arrays
  if (hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(p);
    set_error("hipDeviceSynchronize failed");
    return UNIFY_EDEVICE;
  }
  void* old = const_cast<int64_t*>(ix->z.a1);
  if (old) {
    for (auto& q : ix->allocs)
      if (q == old) q = nullptr;
    (void)hipFree(old);
  }
  ix->allocs.push_back(p);
  const int64_t* d = static_cast<const int64_t*>(p);
  ix->z.a1 = d;
  ix->z.a2 = d + Nr;
  ix->z.s1 = d + 2 * Nr;
  ix->z.s2 = d + 2 * Nr + ns;
  ix->z.ns = (int32_t)ns;
  ix->z.base1 = map->base1;
  ix->z.base2 = map->base2;
  ix->z.shift1 = map->shift1;
  ix->z.shift2 = map->shift2;
  return UNIFY_OK;
}

int unify_set_attr2(unify_index_t ix, const int64_t* attr2, int64_t n) {
  if (!ix || (!attr2 && n > 0)) {
    set_error("unify_set_attr2: null argument");
    return UNIFY_EINVAL;
  }
  if (hipSetDevice(ix->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return UNIFY_EDEVICE;
  }
  std::unique_lock<std::shared_mutex> version(ix->version_mu);
  const int64_t N = ix->dv.n;
  if (n != N) {
    set_error("unify_set_attr2: one value per object of the index");
    return UNIFY_EINVAL;
  }
  const std::vector<int64_t>& ext = ix->host.ext;
  std::vector<int64_t> a((size_t)N);
  for (int64_t i = 0; i < N; ++i) {
    if (ext[i] < 0 || ext[i] >= N) {
      set_error("unify_set_attr2: the index's external ids are not 0 .. n-1");
      return UNIFY_EINVAL;
    }
    a[i] = attr2[ext[i]];
  }
  // sorted sample for the plan's selectivity estimate: the value at rank floor(j n / ns)
  // of the sorted second attributes, j < ns = min(n, 2048)
  const int64_t ns = std::min<int64_t>(N, 2048);
  std::vector<int64_t> srt(a);
  std::sort(srt.begin(), srt.end());
  std::vector<int64_t> smp((size_t)ns);
  for (int64_t j = 0; j < ns; ++j) smp[j] = srt[(size_t)(j * N / ns)];
  void* p = nullptr;
  if (hipMalloc(&p, sizeof(int64_t) * (size_t)(std::max<int64_t>(N, 1) + ns)) != hipSuccess) {
    set_error("device allocation failed (second attribute)");
    return UNIFY_ENOMEM;
  }
  if (hipMemcpy(p, a.data(), sizeof(int64_t) * (size_t)N, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(static_cast<int64_t*>(p) + std::max<int64_t>(N, 1), smp.data(), sizeof(int64_t) * (size_t)ns,
                hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(p);
    set_error("host-to-device copy failed");
    return UNIFY_EDEVICE;
  }
  // searches enqueued before (on any visited pool) may still read the previous array
  if (hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(p);
    set_error("hipDeviceSynchronize failed");
    return UNIFY_EDEVICE;
  }
  void* old = const_cast<int64_t*>(ix->dv.attr2);
  if (old) {
    for (auto& q : ix->allocs)
      if (q == old) q = nullptr;
    (void)hipFree(old);
  }
  ix->allocs.push_back(p);
  ix->dv.attr2 = static_cast<const int64_t*>(p);
  ix->dv.attr2_sample = static_cast<const int64_t*>(p) + std::max<int64_t>(N, 1);
  ix->dv.n2s = (int32_t)ns;
  return UNIFY_OK;
}

int unify_last_timing_ex(unify_index_t ix, float* out_ms, int32_t n) {
  if (!ix || !ix->timed) {
    set_error("no timed search on this index");
    return UNIFY_EINVAL;
  }
  if (!out_ms || n < 1 || n > 7) {
    set_error("unify_last_timing_ex: out_ms needs 1..7 entries");
    return UNIFY_EINVAL;
  }
  if (hipSetDevice(ix->device) != hipSuccess || hipEventSynchronize(ix->ev[7]) != hipSuccess) {
    set_error("hipEventSynchronize failed");
    return UNIFY_EDEVICE;
  }
  for (int i = 0; i < n; ++i) {
    // the graph-search phase starts after the work list when the matrix-core scan ran beside it
    const int from = (i == 4 && ix->timed_side) ? 1 : i;
    if (hipEventElapsedTime(&out_ms[i], ix->ev[from], ix->ev[i + 1]) != hipSuccess) {
      set_error("hipEventElapsedTime failed");
      return UNIFY_EDEVICE;
    }
  }
  return UNIFY_OK;
}

int unify_last_timing(unify_index_t ix, float* plan_ms, float* search_ms, float* rerun_ms) {
  float t[7];
  const int rc = unify_last_timing_ex(ix, t, 7);
  if (rc != UNIFY_OK) return rc;
  const bool side = ix->timed_side;
  if (plan_ms) *plan_ms = side ? t[0] : t[0] + t[1] + t[2] + t[3];
  if (search_ms) *search_ms = t[4] + t[5];
  if (rerun_ms) *rerun_ms = t[6];
  return UNIFY_OK;
}

int unify_batch_create(unify_index_t ix, const float* queries, int64_t nq, const int64_t* l, const int64_t* h,
                       int32_t k, int32_t ef, const int8_t* strategy, const unify_params* params, int64_t* out_ids,
                       float* out_dist, int8_t* out_strategy, int32_t* out_stats, unify_batch_t* out) {
  return batch_create(ix, queries, nq, l, h, k, ef, strategy, params, out_ids, out_dist, out_strategy, out_stats,
                      out);
}

int unify_batch_run(unify_batch_t b, void* hip_stream) { return batch_run(b, hip_stream); }

int unify_batch_free(unify_batch_t b) {
  if (!b) return UNIFY_OK;
  (void)hipSetDevice(b->ix->device);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->scratch) (void)hipFree(b->scratch);
  free_side(b->side);
  delete b;
  return UNIFY_OK;
}

int unify_free_index(unify_index_t ix) {
  if (!ix) return UNIFY_OK;
  (void)hipSetDevice(ix->device);
  for (hipEvent_t e : ix->ev)
    if (e) (void)hipEventDestroy(e);
  pool_free(ix->pool);
  for (void* p : ix->allocs)
    if (p) (void)hipFree(p);
  delete ix;
  return UNIFY_OK;
}

int unify_insert(unify_index_t ix, const float* vectors, const int64_t* attr, const double* level_u, int64_t m) {
  return insert_impl(ix, vectors, attr, level_u, m);
}

int unify_prune(const float* vectors, int64_t n, int32_t d, const int32_t* owners, const int32_t* cand, int64_t t,
                int32_t c, int32_t M, int32_t* out, void* hip_stream) {
  return prune_impl(vectors, n, d, owners, cand, t, c, M, out, hip_stream);
}

int unify_build_index(const float* vectors, const int64_t* attr, const double* level_u, int64_t n, int32_t d,
                      int32_t S, int32_t M, int32_t ef_cons, int device, int precision, unify_index_t* out) {
  return build_impl(vectors, attr, level_u, n, d, S, M, ef_cons, device, precision, out);
}

}  // extern "C"
