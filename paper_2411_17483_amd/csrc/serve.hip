// serve.hip -- the request loop: continuous batching of exact k-NN queries
// over HBM-resident indexes.
//
// Requests (one query each, any registered collection, any k) wait in a
// queue per collection.  A fixed number of slots run batches; each slot owns
// a HIP stream (default priority), a workspace, pinned staging buffers and a
// host thread, so batches on different slots overlap on the device.
// Whenever a slot is free it takes, among the collections with fewer than
// `per_collection` batches in flight, the queue whose oldest request is the
// oldest overall, up to max_batch requests of it, and admits the batch only
// if the device memory of the server stays within its budget (halving the
// batch, then waiting for memory to free up).  That memory is the slots'
// staging buffers plus, per slot, what its workspace holds: a workspace keeps
// the capacity of its largest batch (its fall-back buffers included), so a
// running slot is charged the larger of that and its batch's bytes, and an
// idle one what it holds.  When a batch does not fit, the idle slots give
// their workspaces back first.  Requests that arrive
// while batches run join the next batch of their collection: batching is
// continuous, not a queue in front of one batch at a time.  A batch of a
// large collection costs about one pass over its rows whatever its size, so
// limiting the batches in flight per collection makes the batches larger
// instead of running many small passes side by side.
//
// A batch runs at the largest k of its requests and each request keeps its
// first k results: the ranking is the total order on (distance, id), so
// those are exactly its own k nearest.  A query's answer therefore does not
// depend on the batch it ran in, and is the same alone and in any mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string.h>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mlp.h"

using namespace sofa;

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

constexpr int kServeMaxN = 1024;

}  // namespace

struct sofa_server {
  struct Coll {
    const sofa_index* ix = nullptr;
    int prune = 0;
    std::map<int, const sofa_radius*> models;  // by k
  };
  struct Req {
    int64_t ticket = 0;
    int coll = 0, k = 0;
    std::vector<float> q;
    double t_submit = 0, t_start = 0, t_done = 0;
    bool done = false;
    sofa_status st = SOFA_OK;
    std::string err;
    std::vector<int64_t> ids;
    std::vector<float> d;
    int batch = 0;
  };
  struct Slot {
    hipStream_t stream = nullptr;
    sofa_workspace* ws = nullptr;
    DevBuf dq, dids, dd;
    float* hq = nullptr;
    int64_t* hids = nullptr;
    float* hd = nullptr;
    std::thread th;
    // guarded by the server's mutex
    bool running = false;
    int64_t held = 0;  // workspace bytes kept after the last batch
    int64_t need = 0;  // bytes of the batch running
  };

  int device = 0;
  int max_batch = 256;
  int per_coll = 1;
  int64_t budget = 0;
  std::vector<Coll> colls;
  std::vector<Slot> slots;

  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_mem;
  std::map<int, std::deque<Req*>> pending;  // per collection
  std::map<int, int> busy;                  // batches in flight per collection
  std::unordered_map<int64_t, Req*> reqs;
  int64_t next_ticket = 1;
  int64_t fixed_bytes = 0;  // staging buffers of the slots
  bool stop = false;
  bool started = false;
  sofa_server_stats stats{};

  void worker(int si);
  void start();
  // device bytes charged to slot t (mutex held)
  int64_t charge(int t) const {
    const Slot& x = slots[t];
    return x.running ? std::max(x.held, x.need) : x.held;
  }
  int64_t charged_except(int si) const {
    int64_t c = fixed_bytes;
    for (int t = 0; t < (int)slots.size(); t++)
      if (t != si) c += charge(t);
    return c;
  }
  bool any_running() const {
    for (const Slot& x : slots)
      if (x.running) return true;
    return false;
  }
};

void sofa_server::start() {
  // called with mu held
  if (started) return;
  started = true;
  for (size_t i = 0; i < slots.size(); i++) slots[i].th = std::thread(&sofa_server::worker, this, (int)i);
}

void sofa_server::worker(int si) {
  (void)hipSetDevice(device);
  Slot& sl = slots[si];
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    // a collection with a request and room for another batch in flight
    auto eligible = [&]() {
      auto best = pending.end();
      for (auto it = pending.begin(); it != pending.end(); ++it) {
        if (busy[it->first] >= per_coll) continue;
        if (best == pending.end() || it->second.front()->t_submit < best->second.front()->t_submit)
          best = it;
      }
      return best;
    };
    cv_work.wait(lk, [&] { return (stop && pending.empty()) || eligible() != pending.end(); });
    auto best = eligible();
    if (best == pending.end()) {
      if (stop && pending.empty()) break;
      continue;
    }
    const int ci = best->first;
    const Coll c = colls[ci];  // a copy: colls may grow once the lock is released
    int b = (int)std::min<size_t>(best->second.size(), (size_t)max_batch);
    // the batch runs at the largest k among its requests
    auto kmax = [&](int cnt) {
      int km = 1;
      for (int i = 0; i < cnt; i++) km = std::max(km, best->second[i]->k);
      return km;
    };
    int k = kmax(b);
    // the parameters the batch runs with (the network's scratch is part of
    // its bytes)
    auto params_for = [&](int kk) {
      sofa_knn_params q{};
      q.prune = c.prune;
      auto m = c.models.find(kk);
      if (m != c.models.end()) q.radius_model = m->second;
      return q;
    };
    int64_t need = 0;
    bool admitted = false;
    for (;;) {
      const sofa_knn_params pq = params_for(k);
      need = knn_workspace_bytes(c.ix, b, k, &pq);
      int64_t others = charged_except(si);
      if (others + std::max(sl.held, need) > budget) {
        // the idle slots give back what they keep from earlier batches
        for (int t = 0; t < (int)slots.size(); t++)
          if (t != si && !slots[t].running && slots[t].held > 0 && workspace_trim(slots[t].ws))
            slots[t].held = 0;
        others = charged_except(si);
        // this slot's own larger buffer from an earlier batch
        if (sl.held > need && others + sl.held > budget && workspace_trim(sl.ws)) sl.held = 0;
      }
      if (others + std::max(sl.held, need) <= budget) {
        admitted = true;
        break;
      }
      if (b > 1) {
        b = std::max(1, b / 2);
        k = kmax(b);
        stats.memory_waits++;
        continue;
      }
      break;
    }
    if (!admitted) {
      if (!any_running()) {
        // one query alone exceeds the budget: fail it instead of waiting forever
        Req* r = best->second.front();
        best->second.pop_front();
        if (best->second.empty()) pending.erase(best);
        r->st = set_error(SOFA_ENOMEM, "a query of collection %d with k=%d needs %lld workspace bytes, "
                                       "budget %lld", ci, k, (long long)need, (long long)budget);
        r->err = sofa_last_error();
        r->done = true;
        r->t_done = now_ms();
        stats.completed++;
        cv_done.notify_all();
        continue;
      }
      stats.memory_waits++;
      cv_mem.wait(lk);
      continue;  // choose again: the queues may have changed
    }
    std::vector<Req*> batch(best->second.begin(), best->second.begin() + b);
    best->second.erase(best->second.begin(), best->second.begin() + b);
    if (best->second.empty()) pending.erase(best);
    sl.running = true;
    sl.need = need;
    busy[ci]++;
    stats.batches++;
    stats.max_batch = std::max<int64_t>(stats.max_batch, b);
    stats.in_flight_bytes_peak = std::max(stats.in_flight_bytes_peak, charged_except(si) + charge(si));
    const double t0 = now_ms();
    for (Req* r : batch) {
      r->t_start = t0;
      r->batch = b;
    }
    lk.unlock();

    // run the batch on this slot's stream
    const int n = c.ix->n;
    for (int i = 0; i < b; i++) memcpy(sl.hq + (size_t)i * n, batch[i]->q.data(), (size_t)n * 4);
    sofa_status st = SOFA_OK;
    if (hipMemcpyAsync(sl.dq.p, sl.hq, (size_t)b * n * 4, hipMemcpyHostToDevice, sl.stream) != hipSuccess)
      st = set_error(SOFA_EDEVICE, "query upload failed");
    sofa_knn_params p = params_for(k);
    p.ws = sl.ws;
    if (st == SOFA_OK)
      st = sofa_knn(c.ix, sl.dq.as<float>(), b, k, &p, sl.dids.as<int64_t>(), sl.dd.as<float>(), sl.stream);
    if (st == SOFA_OK &&
        (hipMemcpyAsync(sl.hids, sl.dids.p, (size_t)b * k * 8, hipMemcpyDeviceToHost, sl.stream) != hipSuccess ||
         hipMemcpyAsync(sl.hd, sl.dd.p, (size_t)b * k * 4, hipMemcpyDeviceToHost, sl.stream) != hipSuccess ||
         hipStreamSynchronize(sl.stream) != hipSuccess))
      st = set_error(SOFA_EDEVICE, "result download failed");
    const double t1 = now_ms();
    const std::string err = st == SOFA_OK ? std::string() : std::string(sofa_last_error());
    // the bytes the batch's search had to read (prune tiers)
    double bytes = 0.0;
    sofa_knn_stats ks{};
    if (st == SOFA_OK && c.prune != 0 && sofa_knn_get_stats(sl.ws, nullptr, &ks) == SOFA_OK)
      bytes = (double)ks.prune_rows_streamed * (double)c.ix->n_pad * (c.prune == 1 ? 2.0 : 1.0) +
              (double)ks.series_refined * 4.0 * (double)c.ix->n_pad;

    lk.lock();
    for (int i = 0; i < b; i++) {
      Req* r = batch[i];
      r->st = st;
      r->err = err;
      if (st == SOFA_OK) {
        // the first r->k of the batch's k results
        r->ids.assign(sl.hids + (size_t)i * k, sl.hids + (size_t)i * k + r->k);
        r->d.assign(sl.hd + (size_t)i * k, sl.hd + (size_t)i * k + r->k);
      }
      r->t_done = t1;
      r->done = true;
    }
    sl.running = false;
    sl.held = workspace_held_bytes(sl.ws);
    busy[ci]--;
    stats.completed += b;
    stats.busy_ms += t1 - t0;
    stats.hbm_bytes += bytes;
    cv_done.notify_all();
    cv_mem.notify_all();
    cv_work.notify_all();  // the collection may take another batch now
  }
}

extern "C" sofa_status sofa_server_create(const sofa_server_params* params, sofa_server** out) {
  if (!out) return set_error(SOFA_EINVAL, "null output");
  *out = nullptr;
  const int n_slots = params && params->slots > 0 ? params->slots : 4;
  const int max_batch = params && params->max_batch > 0 ? params->max_batch : 256;
  const int64_t budget = params && params->memory_budget > 0 ? params->memory_budget : (8ll << 30);
  const int per_coll = params && params->per_collection > 0 ? params->per_collection : 1;
  if (n_slots > 16) return set_error(SOFA_EINVAL, "slots=%d above 16", n_slots);
  if (max_batch > 65535) return set_error(SOFA_EINVAL, "max_batch=%d above 65535", max_batch);
  sofa_server* s = new sofa_server();
  s->max_batch = max_batch;
  s->per_coll = per_coll;
  s->budget = budget;
  (void)hipGetDevice(&s->device);
  s->slots.resize(n_slots);
  sofa_status st = SOFA_OK;
  for (auto& sl : s->slots) {
    if (st == SOFA_OK && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess)
      st = set_error(SOFA_EDEVICE, "stream creation failed");
    if (st == SOFA_OK) st = sofa_workspace_create(0, &sl.ws);
    if (st == SOFA_OK) st = sl.dq.alloc((size_t)max_batch * kServeMaxN * 4);
    if (st == SOFA_OK) st = sl.dids.alloc((size_t)max_batch * kMaxK * 8);
    if (st == SOFA_OK) st = sl.dd.alloc((size_t)max_batch * kMaxK * 4);
    s->fixed_bytes += (int64_t)(sl.dq.bytes + sl.dids.bytes + sl.dd.bytes);
    if (st == SOFA_OK && (hipHostMalloc((void**)&sl.hq, (size_t)max_batch * kServeMaxN * 4) != hipSuccess ||
                          hipHostMalloc((void**)&sl.hids, (size_t)max_batch * kMaxK * 8) != hipSuccess ||
                          hipHostMalloc((void**)&sl.hd, (size_t)max_batch * kMaxK * 4) != hipSuccess))
      st = set_error(SOFA_ENOMEM, "pinned staging allocation failed");
  }
  if (st != SOFA_OK) {
    sofa_server_free(s);
    return st;
  }
  *out = s;
  return SOFA_OK;
}

extern "C" sofa_status sofa_server_add_collection(sofa_server* s, const sofa_index* ix, int32_t prune,
                                                  int32_t* out_id) {
  if (!s || !ix || !out_id) return set_error(SOFA_EINVAL, "null argument");
  if (prune < 0 || prune > 2) return set_error(SOFA_EINVAL, "prune must be 0, 1 or 2");
  if (prune == 1 && !ix->has_bf16) return set_error(SOFA_EINVAL, "the index has no BF16 copy");
  if (prune == 2 && !ix->has_fp8) return set_error(SOFA_EINVAL, "the index has no FP8 copy");
  if (ix->n > kServeMaxN) return set_error(SOFA_EINVAL, "series length %d above %d", ix->n, kServeMaxN);
  std::lock_guard<std::mutex> lk(s->mu);
  sofa_server::Coll c;
  c.ix = ix;
  c.prune = prune;
  s->colls.push_back(c);
  *out_id = (int32_t)s->colls.size() - 1;
  return SOFA_OK;
}

extern "C" sofa_status sofa_server_set_model(sofa_server* s, int32_t coll, const sofa_radius* model) {
  if (!s || !model) return set_error(SOFA_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  if (coll < 0 || coll >= (int32_t)s->colls.size()) return set_error(SOFA_EINVAL, "no collection %d", coll);
  const sofa_index* ix = s->colls[coll].ix;
  if (model->dims.D != 2 * ix->bins.pool)
    return set_error(SOFA_EINVAL, "the model takes %d features, the collection has %d pool values",
                     model->dims.D, 2 * ix->bins.pool);
  s->colls[coll].models[model->k] = model;
  return SOFA_OK;
}

extern "C" sofa_status sofa_server_submit(sofa_server* s, int32_t coll, const float* h_query, int32_t k,
                                          int64_t* ticket) {
  if (!s || !h_query || !ticket) return set_error(SOFA_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return set_error(SOFA_EBUSY, "the server is shutting down");
  if (coll < 0 || coll >= (int32_t)s->colls.size()) return set_error(SOFA_EINVAL, "no collection %d", coll);
  const sofa_index* ix = s->colls[coll].ix;
  if (k < 1 || k > kMaxK || k > ix->N) return set_error(SOFA_EINVAL, "k=%d outside [1, min(N, %d)]", k, kMaxK);
  auto* r = new sofa_server::Req();
  r->ticket = s->next_ticket++;
  r->coll = coll;
  r->k = k;
  r->q.assign(h_query, h_query + ix->n);
  r->t_submit = now_ms();
  s->reqs[r->ticket] = r;
  s->pending[coll].push_back(r);
  s->stats.submitted++;
  s->start();
  s->cv_work.notify_one();
  *ticket = r->ticket;
  return SOFA_OK;
}

extern "C" sofa_status sofa_server_wait(sofa_server* s, int64_t ticket, int64_t* h_ids, float* h_dists,
                                        double* times_ms, int32_t timeout_ms) {
  if (!s) return set_error(SOFA_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return set_error(SOFA_EINVAL, "unknown ticket %lld", (long long)ticket);
  sofa_server::Req* r = it->second;
  auto ready = [&] { return r->done; };
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
    return set_error(SOFA_EBUSY, "ticket %lld not finished", (long long)ticket);
  }
  const sofa_status st = r->st;
  if (st == SOFA_OK) {
    if (h_ids) memcpy(h_ids, r->ids.data(), r->ids.size() * 8);
    if (h_dists) memcpy(h_dists, r->d.data(), r->d.size() * 4);
  }
  if (times_ms) {
    times_ms[0] = r->t_done - r->t_submit;   // latency
    times_ms[1] = r->t_start - r->t_submit;  // queueing
    times_ms[2] = (double)r->batch;          // size of the batch it ran in
  }
  const std::string err = r->err;
  s->reqs.erase(it);
  delete r;
  return st == SOFA_OK ? SOFA_OK : set_error(st, "request %lld failed: %s", (long long)ticket, err.c_str());
}

extern "C" sofa_status sofa_server_get_stats(sofa_server* s, sofa_server_stats* out) {
  if (!s || !out) return set_error(SOFA_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  return SOFA_OK;
}

extern "C" void sofa_server_free(sofa_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  s->cv_mem.notify_all();
  for (auto& sl : s->slots)
    if (sl.th.joinable()) sl.th.join();
  for (auto& kv : s->reqs) delete kv.second;
  for (auto& sl : s->slots) {
    if (sl.ws) sofa_workspace_free(sl.ws);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.hq) (void)hipHostFree(sl.hq);
    if (sl.hids) (void)hipHostFree(sl.hids);
    if (sl.hd) (void)hipHostFree(sl.hd);
  }
  delete s;
}
