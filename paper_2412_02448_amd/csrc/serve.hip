// Serving: continuous batching of range-filtered k-NN requests over a resident
// index.  Requests carry an arrival time; a worker thread admits the requests
// that have arrived into a batch whenever one of its in-flight slots is free,
// launches the search on the slot's stream and harvests finished slots by their
// events.  A slot owns pinned host staging, device buffers, scratch and its own
// visited pool, so the search kernels of different slots run concurrently on
// the device.  The batch size and the pool rows are chosen at creation so that
// the slots fit a device-memory budget.  Per-query results do not depend on
// which other queries share a batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "unify_internal.h"

namespace unify {
int search_impl_scratch(unify_index_t ix, const float* queries, int64_t nq, const int64_t* l, const int64_t* h,
                        int32_t k, int32_t ef, const int8_t* strategy, const unify_params* prm, int64_t* out_ids,
                        float* out_dist, int8_t* out_strategy, int32_t* out_stats, void* scratch,
                        size_t scratch_bytes, VisitPool* pool, void* stream);
size_t search_scratch_bytes(unify_index_t ix, int64_t nq, int32_t k, int32_t ef, const unify_params* prm);
}  // namespace unify

using Clock = std::chrono::steady_clock;

struct unify_server {
  unify_index_t ix = nullptr;
  unify_server_config cfg{};  // cfg.max_batch: the batch size the budget admits
  int d = 0;
  int64_t visit_rows = 0;    // rows of each slot's visited pool
  int64_t device_bytes = 0;  // device memory the slots hold

  struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    // pinned host staging
    float* hq = nullptr;
    int64_t *hl = nullptr, *hh = nullptr, *hids = nullptr;
    int8_t* hs = nullptr;
    float* hdist = nullptr;
    // device
    void* dmem = nullptr;
    float* dq = nullptr;
    int64_t *dl = nullptr, *dh = nullptr, *dids = nullptr;
    int8_t* ds = nullptr;
    float* ddist = nullptr;
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    std::unique_ptr<unify::VisitPool> pool;  // the visited rows of this slot's searches
    std::vector<int64_t> tickets;  // requests of the batch in flight, empty when free
  };
  std::vector<Slot> slots;

  struct Request {
    int64_t ticket;
    Clock::time_point arrive;
  };
  // request inputs, by ticket
  std::vector<float> q;
  std::vector<int64_t> l, h;
  std::vector<int8_t> strat;
  // results, by ticket
  std::vector<int64_t> ids;
  std::vector<float> dist;
  std::vector<double> latency;
  std::vector<uint8_t> done;
  std::vector<Clock::time_point> arrive_at;

  std::deque<Request> future;  // not yet arrived, by arrival time
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  int error = UNIFY_OK;
  std::thread worker;
  int64_t completed = 0, batches = 0;
  double busy_s = 0.0;
};

namespace {

// Device bytes of a slot's query and result buffers for B queries.
size_t io_bytes(int64_t B, int d, int k) {
  const size_t parts[] = {sizeof(float) * B * d, sizeof(int64_t) * B, sizeof(int64_t) * B, (size_t)B,
                          sizeof(int64_t) * B * k, sizeof(float) * B * k};
  size_t total = 0;
  for (size_t p : parts) total += (p + 255) / 256 * 256;
  return total;
}

int slot_init(unify_server* S, unify_server::Slot& s) {
  const int64_t B = S->cfg.max_batch;
  const int k = S->cfg.k, d = S->d;
  s.pool = std::make_unique<unify::VisitPool>();
  s.pool->max_rows = S->visit_rows;
  if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess)
    return UNIFY_EDEVICE;
  auto hm = [](void** p, size_t b) { return hipHostMalloc(p, b, hipHostMallocDefault) == hipSuccess; };
  if (!hm((void**)&s.hq, sizeof(float) * B * d) || !hm((void**)&s.hl, sizeof(int64_t) * B) ||
      !hm((void**)&s.hh, sizeof(int64_t) * B) || !hm((void**)&s.hs, B) ||
      !hm((void**)&s.hids, sizeof(int64_t) * B * k) || !hm((void**)&s.hdist, sizeof(float) * B * k))
    return UNIFY_ENOMEM;
  const size_t parts[] = {sizeof(float) * B * d, sizeof(int64_t) * B, sizeof(int64_t) * B, (size_t)B,
                          sizeof(int64_t) * B * k, sizeof(float) * B * k};
  size_t total = 0, off[6];
  for (int i = 0; i < 6; ++i) {
    off[i] = total;
    total += (parts[i] + 255) / 256 * 256;
  }
  s.scratch_bytes = unify::search_scratch_bytes(S->ix, B, k, S->cfg.ef, &S->cfg.params);
  if (s.scratch_bytes == 0) return UNIFY_EINVAL;
  if (hipMalloc(&s.dmem, total) != hipSuccess || hipMalloc(&s.scratch, s.scratch_bytes) != hipSuccess)
    return UNIFY_ENOMEM;
  const int rc = unify::pool_ensure(*s.pool, S->ix->dv.n);
  if (rc != UNIFY_OK) return rc;
  S->device_bytes += (int64_t)(total + s.scratch_bytes) + s.pool->nrows * (int64_t)unify::pool_row_bytes(s.pool->n);
  char* b = static_cast<char*>(s.dmem);
  s.dq = reinterpret_cast<float*>(b + off[0]);
  s.dl = reinterpret_cast<int64_t*>(b + off[1]);
  s.dh = reinterpret_cast<int64_t*>(b + off[2]);
  s.ds = reinterpret_cast<int8_t*>(b + off[3]);
  s.dids = reinterpret_cast<int64_t*>(b + off[4]);
  s.ddist = reinterpret_cast<float*>(b + off[5]);
  return UNIFY_OK;
}

void slot_free(unify_server::Slot& s) {
  if (s.stream) (void)hipStreamSynchronize(s.stream);
  for (void* p : {(void*)s.hq, (void*)s.hl, (void*)s.hh, (void*)s.hs, (void*)s.hids, (void*)s.hdist})
    if (p) (void)hipHostFree(p);
  if (s.dmem) (void)hipFree(s.dmem);
  if (s.scratch) (void)hipFree(s.scratch);
  if (s.pool) unify::pool_free(*s.pool);
  if (s.done) (void)hipEventDestroy(s.done);
  if (s.stream) (void)hipStreamDestroy(s.stream);
}

// Launches the requests in `batch` on slot s (worker thread; takes the lock
// only to copy the inputs, which submissions may reallocate).
int slot_launch(unify_server* S, unify_server::Slot& s, const std::vector<int64_t>& batch) {
  const int64_t n = (int64_t)batch.size();
  const int k = S->cfg.k, d = S->d;
  {
    std::lock_guard<std::mutex> g(S->mu);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t t = batch[i];
      std::memcpy(s.hq + i * d, S->q.data() + t * d, sizeof(float) * d);
      s.hl[i] = S->l[t];
      s.hh[i] = S->h[t];
      s.hs[i] = S->strat[t];
    }
  }
  hipStream_t st = s.stream;
  if (hipMemcpyAsync(s.dq, s.hq, sizeof(float) * n * d, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(s.dl, s.hl, sizeof(int64_t) * n, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(s.dh, s.hh, sizeof(int64_t) * n, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(s.ds, s.hs, n, hipMemcpyHostToDevice, st) != hipSuccess)
    return UNIFY_EDEVICE;
  int rc = unify::search_impl_scratch(S->ix, s.dq, n, s.dl, s.dh, k, S->cfg.ef, s.ds, &S->cfg.params, s.dids,
                                      s.ddist, nullptr, nullptr, s.scratch, s.scratch_bytes, s.pool.get(), st);
  if (rc != UNIFY_OK) return rc;
  if (hipMemcpyAsync(s.hids, s.dids, sizeof(int64_t) * n * k, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(s.hdist, s.ddist, sizeof(float) * n * k, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipEventRecord(s.done, st) != hipSuccess)
    return UNIFY_EDEVICE;
  return UNIFY_OK;
}

void worker_main(unify_server* S) {
  (void)hipSetDevice(S->ix->device);
  const int64_t B = S->cfg.max_batch;
  const auto max_wait = std::chrono::duration<double>(S->cfg.max_wait_s);
  std::deque<unify_server::Request> ready;
  auto busy_since = Clock::now();
  int inflight = 0;
  while (true) {
    // harvest finished slots
    for (auto& s : S->slots) {
      if (s.tickets.empty() || hipEventQuery(s.done) != hipSuccess) continue;
      const auto now = Clock::now();
      const int k = S->cfg.k;
      {
        std::lock_guard<std::mutex> g(S->mu);
        for (size_t i = 0; i < s.tickets.size(); ++i) {
          const int64_t t = s.tickets[i];
          std::memcpy(S->ids.data() + t * k, s.hids + i * k, sizeof(int64_t) * k);
          std::memcpy(S->dist.data() + t * k, s.hdist + i * k, sizeof(float) * k);
          S->latency[t] = std::chrono::duration<double>(now - S->arrive_at[t]).count();
          S->done[t] = 1;
        }
        S->completed += (int64_t)s.tickets.size();
        if (--inflight == 0) S->busy_s += std::chrono::duration<double>(now - busy_since).count();
      }
      s.tickets.clear();
      S->cv_done.notify_all();
    }
    // admit the requests that have arrived
    bool stop;
    {
      std::unique_lock<std::mutex> g(S->mu);
      const auto now = Clock::now();
      while (!S->future.empty() && S->future.front().arrive <= now) {
        ready.push_back(S->future.front());
        S->future.pop_front();
      }
      stop = S->stop && S->future.empty() && ready.empty() && inflight == 0;
      if (!stop && ready.empty() && inflight == 0) {
        // idle: sleep until the next arrival or a submission
        if (S->future.empty())
          S->cv_work.wait_for(g, std::chrono::milliseconds(50));
        else
          S->cv_work.wait_until(g, S->future.front().arrive);
        continue;
      }
    }
    if (stop) break;
    // launch on a free slot: a full batch at once, a partial one when its oldest
    // request has waited max_wait (0: as soon as a slot is free)
    if (!ready.empty()) {
      const bool full = (int64_t)ready.size() >= B;
      const bool waited = Clock::now() - ready.front().arrive >= max_wait;
      for (auto& s : S->slots) {
        if (!s.tickets.empty() || !(full || waited) || ready.empty()) continue;
        const int64_t n = std::min<int64_t>(B, (int64_t)ready.size());
        std::vector<int64_t> batch(n);
        for (int64_t i = 0; i < n; ++i) {
          batch[i] = ready.front().ticket;
          ready.pop_front();
        }
        const int rc = slot_launch(S, s, batch);
        if (rc != UNIFY_OK) {
          std::lock_guard<std::mutex> g(S->mu);
          S->error = rc;
          S->stop = true;
          for (int64_t t : batch) S->done[t] = 2;
          S->cv_done.notify_all();
          continue;
        }
        if (inflight++ == 0) busy_since = Clock::now();
        {
          std::lock_guard<std::mutex> g(S->mu);
          ++S->batches;
        }
        s.tickets = std::move(batch);
      }
    }
    std::this_thread::yield();
  }
}

}  // namespace

using namespace unify;

extern "C" {

int unify_server_create(unify_index_t ix, const unify_server_config* cfg, unify_server_t* out) {
  if (!ix || !cfg || !out) {
    set_error("unify_server_create: null argument");
    return UNIFY_EINVAL;
  }
  unify_server_config c = *cfg;
  c.params.flags &= ~(uint32_t)UNIFY_FLAG_TIMING;  // timing events belong to the index, not to a server
  // concurrency comes from the slots: each keeps to its one stream (the matrix-core scan
  // before the graph search), since a process's streams share a few hardware queues
  c.params.flags |= UNIFY_FLAG_SERIAL_PHASES;
  if (c.max_batch <= 0) c.max_batch = 4096;
  if (c.inflight <= 0) c.inflight = 2;
  if (c.k < 1 || c.k > 256 || c.ef < c.k || c.ef > 256 || c.max_batch > (1 << 20) || c.inflight > 8 ||
      c.max_wait_s < 0 || c.mem_budget < 0) {
    set_error("unify_server_create: k in [1, 256], ef in [k, 256], max_batch <= 2^20, inflight <= 8, max_wait >= 0, "
              "mem_budget >= 0");
    return UNIFY_EINVAL;
  }
  if (hipSetDevice(ix->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return UNIFY_EDEVICE;
  }
  std::shared_lock<std::shared_mutex> version(ix->version_mu);
  // admission by memory: each slot holds the buffers and scratch of a batch and a
  // visited pool (one row per resident wavefront of the device at most); the batch
  // size, then the rows, halve until `inflight` slots fit the budget
  int cus = 0;
  size_t free_b = 0, total_b = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ix->device) != hipSuccess ||
      hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    set_error("device query failed");
    return UNIFY_EDEVICE;
  }
  const int64_t budget = c.mem_budget > 0 ? c.mem_budget : (int64_t)(free_b / 2);
  const size_t row = pool_row_bytes(ix->dv.n);
  int64_t B = c.max_batch, rows = (int64_t)cus * 16;
  auto slot_bytes = [&](int64_t b, int64_t r) {
    const size_t sc = search_scratch_bytes(ix, b, c.k, c.ef, &c.params);
    return sc == 0 ? INT64_MAX : (int64_t)(io_bytes(b, ix->dv.d, c.k) + sc + (size_t)r * row);
  };
  if (slot_bytes(1, 1) == INT64_MAX) return UNIFY_EINVAL;  // the parameters (message set)
  while (B > 64 && slot_bytes(B, rows) > budget / c.inflight) B = (B + 1) / 2;
  while (rows > 64 && slot_bytes(B, rows) > budget / c.inflight) rows /= 2;
  if (slot_bytes(B, rows) > budget / c.inflight) {
    set_error("unify_server_create: the memory budget (" + std::to_string(budget) + " bytes) holds no " +
              std::to_string(c.inflight) + " slots of " + std::to_string(B) + " queries and " +
              std::to_string(rows) + " visited rows");
    return UNIFY_ENOMEM;
  }
  c.max_batch = (int32_t)B;
  unify_server* S = new unify_server();
  S->ix = ix;
  S->cfg = c;
  S->d = ix->dv.d;
  S->visit_rows = rows;
  S->slots.resize(c.inflight);
  for (auto& s : S->slots) {
    const int rc = slot_init(S, s);
    if (rc != UNIFY_OK) {
      for (auto& t : S->slots) slot_free(t);
      delete S;
      set_error("unify_server_create: slot allocation failed");
      return rc;
    }
  }
  S->worker = std::thread(worker_main, S);
  *out = S;
  return UNIFY_OK;
}

int unify_server_submit(unify_server_t S, int64_t n, const float* queries, const int64_t* l, const int64_t* h,
                        const int8_t* strategy, const double* arrive_s, int64_t* tickets) {
  if (!S || n < 0 || (n > 0 && (!queries || !l || !h || !tickets))) {
    set_error("unify_server_submit: bad arguments");
    return UNIFY_EINVAL;
  }
  const auto now = Clock::now();
  std::lock_guard<std::mutex> g(S->mu);
  if (S->stop) {
    set_error("unify_server_submit: the server has stopped");
    return S->error != UNIFY_OK ? S->error : UNIFY_EINVAL;
  }
  const int64_t t0 = (int64_t)S->l.size();
  const int d = S->d, k = S->cfg.k;
  S->q.insert(S->q.end(), queries, queries + n * d);
  S->l.insert(S->l.end(), l, l + n);
  S->h.insert(S->h.end(), h, h + n);
  for (int64_t i = 0; i < n; ++i) S->strat.push_back(strategy ? strategy[i] : (int8_t)UNIFY_AUTO);
  S->ids.resize((t0 + n) * k);
  S->dist.resize((t0 + n) * k);
  S->latency.resize(t0 + n);
  S->done.resize(t0 + n, 0);
  // arrival times: `now + arrive_s[i]`, kept ordered in the future queue
  std::vector<unify_server::Request> add(n);
  for (int64_t i = 0; i < n; ++i) {
    const double off = arrive_s ? std::max(0.0, arrive_s[i]) : 0.0;
    add[i] = {t0 + i, now + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(off))};
    S->arrive_at.push_back(add[i].arrive);
    tickets[i] = t0 + i;
  }
  std::stable_sort(add.begin(), add.end(), [](const auto& a, const auto& b) { return a.arrive < b.arrive; });
  std::deque<unify_server::Request> merged;
  std::merge(S->future.begin(), S->future.end(), add.begin(), add.end(), std::back_inserter(merged),
             [](const auto& a, const auto& b) { return a.arrive < b.arrive; });
  S->future.swap(merged);
  S->cv_work.notify_one();
  return UNIFY_OK;
}

int unify_server_wait(unify_server_t S, int64_t n, const int64_t* tickets, int64_t* ids, float* dist,
                      double* latency_s, double timeout_s) {
  if (!S || n < 0 || (n > 0 && !tickets)) {
    set_error("unify_server_wait: bad arguments");
    return UNIFY_EINVAL;
  }
  const int k = S->cfg.k;
  const auto deadline = Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                           std::chrono::duration<double>(timeout_s > 0 ? timeout_s : 1e9));
  std::unique_lock<std::mutex> g(S->mu);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t t = tickets[i];
    if (t < 0 || t >= (int64_t)S->done.size()) {
      set_error("unify_server_wait: unknown ticket");
      return UNIFY_EINVAL;
    }
    while (!S->done[t]) {
      if (S->cv_done.wait_until(g, deadline) == std::cv_status::timeout && !S->done[t]) {
        set_error("unify_server_wait: timed out");
        return UNIFY_EIO;
      }
    }
    if (S->done[t] == 2) {
      set_error("unify_server_wait: the batch of this request failed");
      return S->error;
    }
    if (ids) std::memcpy(ids + i * k, S->ids.data() + t * k, sizeof(int64_t) * k);
    if (dist) std::memcpy(dist + i * k, S->dist.data() + t * k, sizeof(float) * k);
    if (latency_s) latency_s[i] = S->latency[t];
  }
  return UNIFY_OK;
}

int unify_server_limits(unify_server_t S, int64_t* max_batch, int64_t* visit_rows, int64_t* device_bytes) {
  if (!S) {
    set_error("null server");
    return UNIFY_EINVAL;
  }
  if (max_batch) *max_batch = S->cfg.max_batch;
  if (visit_rows) *visit_rows = S->slots.empty() ? 0 : S->slots[0].pool->nrows;
  if (device_bytes) *device_bytes = S->device_bytes;
  return UNIFY_OK;
}

int unify_server_stats(unify_server_t S, int64_t* completed, int64_t* batches, double* busy_s) {
  if (!S) {
    set_error("null server");
    return UNIFY_EINVAL;
  }
  std::lock_guard<std::mutex> g(S->mu);
  if (completed) *completed = S->completed;
  if (batches) *batches = S->batches;
  if (busy_s) *busy_s = S->busy_s;
  return UNIFY_OK;
}

int unify_server_free(unify_server_t S) {
  if (!S) return UNIFY_OK;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  (void)hipSetDevice(S->ix->device);
  for (auto& s : S->slots) slot_free(s);
  delete S;
  return UNIFY_OK;
}

}  // extern "C"
