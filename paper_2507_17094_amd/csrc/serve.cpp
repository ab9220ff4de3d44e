// Continuous-batching serving loop over a resident index.
//
// Requests (host query rows + k, itopk, T and search parameters) are queued by
// miann_server_submit from any thread. Pending requests wait in one FIFO per
// search shape (k, itopk, T, parameters). A scheduler thread forms batches: it
// takes the shape whose first request is the oldest and coalesces that FIFO's
// requests in arrival order up to max_batch_queries, admitting each only while
// the queries and device bytes already in flight stay within the configured
// limits (forming a batch costs time in its size, not in the queue's length). Each admitted batch runs on one of
// num_streams HIP streams (default priority), so batches that arrive while
// others are running overlap on the device. Every query is searched with its
// index inside its own request as the query key, so a result is the same
// alone and in any mix. Latency runs from submission to the scheduler seeing
// the batch's completion event, on the host's steady clock.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/miann.h"

miann_status miann_fail(miann_status st, const char* fmt, ...);
int miann_index_input_esize(const miann_index* idx, int32_t* d_out);
size_t miann_search_scratch_bytes(const miann_index* ix, int64_t nq, int32_t k, int32_t itopk,
                                  const miann_search_params* sp);

namespace {

using clk = std::chrono::steady_clock;

// Result width the slot buffers are allocated for up front, so that no
// allocation (which can serialise the device) happens while serving.
constexpr int32_t kPreallocK = 128;

struct Request {
  uint64_t ticket = 0;
  int64_t nq = 0;
  int32_t k = 0, itopk = 0, T = 0;
  miann_search_params sp{};
  std::vector<uint8_t> q;  // host copy of the query rows
  std::vector<uint32_t> ids;
  std::vector<uint8_t> dists;
  clk::time_point t_submit, t_done;
  bool done = false;
  miann_status status = MIANN_OK;
  std::string err;
};

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  void* h_in = nullptr;   // pinned: queries then qkeys
  void* h_out = nullptr;  // pinned: ids then dists
  void* d_buf = nullptr;  // device: queries, qkeys, ids, dists
  size_t cap_in = 0, cap_out = 0, cap_dev = 0;
  bool busy = false;
  std::vector<std::shared_ptr<Request>> reqs;
  int64_t nq = 0;
  int32_t k = 0;
  size_t bytes = 0;
  clk::time_point t_launch;
};

bool same_shape(const Request& a, const Request& b) {
  return a.k == b.k && a.itopk == b.itopk && a.T == b.T && std::memcmp(&a.sp, &b.sp, sizeof a.sp) == 0;
}

}  // namespace

struct miann_server {
  const miann_index* idx = nullptr;
  miann_server_config cfg{};
  int esize = 4, d = 0;
  int64_t prealloc_nq = 0;  // queries the slot buffers hold without growing
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  struct ShapeQueue {
    std::shared_ptr<Request> rep;  // a request of this shape (the key)
    std::deque<std::shared_ptr<Request>> q;
  };
  std::vector<ShapeQueue> pending;  // one FIFO per search shape
  int64_t n_pending = 0;
  std::map<uint64_t, std::shared_ptr<Request>> all;
  uint64_t next_ticket = 1;
  int64_t inflight_q = 0;
  size_t inflight_b = 0;
  miann_server_stats stats{};
  bool stop = false;
  std::thread th;
  clk::time_point t0;

  // device bytes of a batch: its staging buffers plus the search's temporaries on the slot's stream
  size_t batch_bytes(int64_t nq, int32_t k, int32_t itopk, const miann_search_params* sp) const {
    return (size_t)nq * ((size_t)d * esize + 8 + (size_t)k * 8) + 4096 +
           miann_search_scratch_bytes(idx, nq, k, itopk, sp);
  }
  size_t batch_bytes(int64_t nq, const Request& r) const { return batch_bytes(nq, r.k, r.itopk, &r.sp); }

  void loop();
  bool reserve(Slot& s, int64_t nq, int32_t k);
  bool launch(Slot& s, std::vector<std::shared_ptr<Request>>& batch);
  void finish(Slot& s, miann_status st, const char* err);
};

bool miann_server::reserve(Slot& s, int64_t nq, int32_t k) {
  const size_t qbytes = (size_t)nq * d * esize, kbytes = (size_t)nq * 8;
  const size_t obytes = (size_t)nq * k * 8;
  if (qbytes + kbytes > s.cap_in) {
    if (s.h_in) hipHostFree(s.h_in);
    s.cap_in = qbytes + kbytes;
    if (hipHostMalloc(&s.h_in, s.cap_in) != hipSuccess) { s.h_in = nullptr; s.cap_in = 0; return false; }
  }
  if (obytes > s.cap_out) {
    if (s.h_out) hipHostFree(s.h_out);
    s.cap_out = obytes;
    if (hipHostMalloc(&s.h_out, s.cap_out) != hipSuccess) { s.h_out = nullptr; s.cap_out = 0; return false; }
  }
  if (qbytes + kbytes + obytes + 1024 > s.cap_dev) {
    if (s.d_buf) { hipStreamSynchronize(s.st); hipFree(s.d_buf); }
    s.cap_dev = qbytes + kbytes + obytes + 1024;
    if (hipMalloc(&s.d_buf, s.cap_dev) != hipSuccess) { s.d_buf = nullptr; s.cap_dev = 0; return false; }
  }
  return true;
}

bool miann_server::launch(Slot& s, std::vector<std::shared_ptr<Request>>& batch) {
  int64_t nq = 0;
  for (auto& r : batch) nq += r->nq;
  const int32_t k = batch[0]->k;
  const size_t qbytes = (size_t)nq * d * esize, kbytes = (size_t)nq * 8;
  // buffers are sized at creation for a full batch of k <= kPreallocK; larger k grows them (a blocking step)
  if (!reserve(s, std::max<int64_t>(nq, prealloc_nq), std::max<int32_t>(k, kPreallocK))) return false;
  char* hi = (char*)s.h_in;
  uint64_t* hk = (uint64_t*)(hi + qbytes);
  int64_t off = 0;
  for (auto& r : batch) {
    std::memcpy(hi + off * d * esize, r->q.data(), r->q.size());
    for (int64_t i = 0; i < r->nq; i++) hk[off + i] = (uint64_t)i;  // key = index within the request
    off += r->nq;
  }
  char* db = (char*)s.d_buf;
  void* dq = db;
  uint64_t* dk = (uint64_t*)(db + ((qbytes + 255) & ~(size_t)255));
  uint32_t* di = (uint32_t*)((char*)dk + ((kbytes + 255) & ~(size_t)255));
  void* dd = (char*)di + (((size_t)nq * k * 4 + 255) & ~(size_t)255);
  miann_search_params sp = batch[0]->sp;
  sp.qkeys = dk;
  s.t_launch = clk::now();
  hipMemcpyAsync(dq, hi, qbytes, hipMemcpyHostToDevice, s.st);
  hipMemcpyAsync(dk, hk, kbytes, hipMemcpyHostToDevice, s.st);
  miann_status rc = miann_search(idx, dq, nq, k, batch[0]->itopk, batch[0]->T, &sp, di, dd, nullptr, s.st);
  if (rc != MIANN_OK) {
    for (auto& r : batch) { r->status = rc; r->err = miann_last_error(); }
  }
  hipMemcpyAsync(s.h_out, di, (size_t)nq * k * 4, hipMemcpyDeviceToHost, s.st);
  hipMemcpyAsync((char*)s.h_out + (size_t)nq * k * 4, dd, (size_t)nq * k * 4, hipMemcpyDeviceToHost, s.st);
  hipEventRecord(s.ev, s.st);
  s.busy = true;
  s.reqs = batch;
  s.nq = nq;
  s.k = k;
  s.bytes = batch_bytes(nq, *batch[0]);
  return true;
}

void miann_server::finish(Slot& s, miann_status st, const char* err) {
  const auto now = clk::now();
  const uint32_t* ids = (const uint32_t*)s.h_out;
  const char* dists = (const char*)s.h_out + (size_t)s.nq * s.k * 4;
  int64_t off = 0;
  std::lock_guard<std::mutex> lk(mu);
  for (auto& r : s.reqs) {
    r->ids.assign(ids + off * s.k, ids + (off + r->nq) * s.k);
    r->dists.assign(dists + off * s.k * 4, dists + (off + r->nq) * s.k * 4);
    if (st != MIANN_OK && r->status == MIANN_OK) { r->status = st; r->err = err ? err : ""; }
    r->t_done = now;
    r->done = true;
    off += r->nq;
    stats.requests_done++;
    stats.queries_done += r->nq;
  }
  inflight_q -= s.nq;
  inflight_b -= s.bytes;
  s.busy = false;
  s.reqs.clear();
  cv_done.notify_all();
}

void miann_server::loop() {
  for (;;) {
    // completions
    for (auto& s : slots) {
      if (!s.busy) continue;
      hipError_t q = hipEventQuery(s.ev);
      if (q == hipSuccess) finish(s, MIANN_OK, nullptr);
      else if (q != hipErrorNotReady) finish(s, MIANN_EDEVICE, hipGetErrorString(q));
    }
    // admission and launch
    std::vector<std::pair<Slot*, std::vector<std::shared_ptr<Request>>>> todo;
    {
      std::unique_lock<std::mutex> lk(mu);
      if (stop && n_pending == 0) {
        bool any = false;
        for (auto& s : slots) any |= s.busy;
        if (!any) return;
      }
      for (auto& s : slots) {
        if (s.busy || n_pending == 0) continue;
        bool claimed = false;
        for (auto& t : todo) claimed |= (t.first == &s);
        if (claimed) continue;
        // the shape whose first request is the oldest
        ShapeQueue* g = nullptr;
        for (auto& x : pending)
          if (!x.q.empty() && (!g || x.q.front()->ticket < g->q.front()->ticket)) g = &x;
        auto head = g->q.front();
        std::vector<std::shared_ptr<Request>> batch;
        int64_t nq = 0;
        while (!g->q.empty()) {
          const auto& r = g->q.front();
          if (nq + r->nq > cfg.max_batch_queries || inflight_q + nq + r->nq > cfg.max_inflight_queries ||
              inflight_b + batch_bytes(nq + r->nq, *head) > (size_t)cfg.memory_budget_bytes)
            break;
          nq += r->nq;
          batch.push_back(r);
          g->q.pop_front();
          n_pending--;
        }
        if (batch.empty()) break;  // the oldest request must wait for capacity
        inflight_q += nq;
        inflight_b += batch_bytes(nq, *head);
        stats.peak_inflight_queries = std::max<int64_t>(stats.peak_inflight_queries, inflight_q);
        stats.peak_inflight_bytes = std::max<int64_t>(stats.peak_inflight_bytes, (int64_t)inflight_b);
        stats.batches++;
        todo.emplace_back(&s, std::move(batch));
      }
      pending.erase(std::remove_if(pending.begin(), pending.end(), [](const ShapeQueue& x) { return x.q.empty(); }),
                    pending.end());
    }
    for (auto& t : todo) {
      if (!launch(*t.first, t.second)) {
        std::lock_guard<std::mutex> lk(mu);
        int64_t nq = 0;
        for (auto& r : t.second) {
          r->status = MIANN_ENOMEM;
          r->err = "miann_server: buffer allocation failed";
          r->done = true;
          r->t_done = clk::now();
          nq += r->nq;
        }
        inflight_q -= nq;
        inflight_b -= batch_bytes(nq, *t.second[0]);
        cv_done.notify_all();
      }
    }
    bool busy = false;
    for (auto& s : slots) busy |= s.busy;
    std::unique_lock<std::mutex> lk(mu);
    if (busy) cv_work.wait_for(lk, std::chrono::microseconds(50));
    else if (n_pending == 0 && !stop) cv_work.wait_for(lk, std::chrono::milliseconds(5));
  }
}

namespace {

void miann_server_destroy_slots(miann_server* s) {
  for (auto& sl : s->slots) {
    if (sl.st) {
      hipStreamSynchronize(sl.st);
      miann_release_scratch(sl.st);  // the searches' kept blocks of this stream go back to the pool
      hipStreamSynchronize(sl.st);
    }
    if (sl.d_buf) hipFree(sl.d_buf);
    if (sl.h_in) hipHostFree(sl.h_in);
    if (sl.h_out) hipHostFree(sl.h_out);
    if (sl.ev) hipEventDestroy(sl.ev);
    if (sl.st) hipStreamDestroy(sl.st);
  }
  s->slots.clear();
}

}  // namespace

extern "C" {

void miann_server_config_default(miann_server_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof *c);
  c->num_streams = 4;
  c->max_batch_queries = 8192;
  c->max_inflight_queries = 65536;
  c->memory_budget_bytes = (int64_t)1 << 30;
}

miann_status miann_server_create(const miann_index* idx, const miann_server_config* cfg, miann_server** out) {
  if (!idx || !out) return miann_fail(MIANN_EINVAL, "miann_server_create: null argument");
  miann_server_config c;
  if (cfg) c = *cfg; else miann_server_config_default(&c);
  if (c.num_streams < 1 || c.num_streams > 32 || c.max_batch_queries < 1 || c.max_inflight_queries < 1 ||
      c.memory_budget_bytes < 1)
    return miann_fail(MIANN_EINVAL, "miann_server_create: configuration out of range");
  auto* s = new miann_server();
  s->idx = idx;
  s->cfg = c;
  s->esize = miann_index_input_esize(idx, &s->d);
  s->slots.resize(c.num_streams);
  for (auto& sl : s->slots) {
    if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess) {
      miann_server_destroy_slots(s);
      delete s;
      return miann_fail(MIANN_EDEVICE, "miann_server_create: stream or event creation failed");
    }
  }
  // full batches up front, as far as the memory budget covers them
  s->prealloc_nq = std::max<int64_t>(1, std::min<int64_t>(c.max_batch_queries, c.memory_budget_bytes /
                                                              (int64_t)s->batch_bytes(1, kPreallocK, kPreallocK,
                                                                                      nullptr)));
  for (auto& sl : s->slots) {
    if (!s->reserve(sl, s->prealloc_nq, kPreallocK)) {
      miann_server_destroy_slots(s);
      delete s;
      return miann_fail(MIANN_ENOMEM, "miann_server_create: slot buffer allocation failed");
    }
  }
  s->t0 = clk::now();
  s->th = std::thread([s] { s->loop(); });
  *out = s;
  return MIANN_OK;
}

miann_status miann_server_submit(miann_server* s, const void* queries, int64_t nq, int32_t k, int32_t itopk,
                                 int32_t max_iters, const miann_search_params* sp, uint64_t* ticket) {
  if (!s || !ticket || (nq > 0 && !queries)) return miann_fail(MIANN_EINVAL, "miann_server_submit: null argument");
  if (nq < 1) return miann_fail(MIANN_EINVAL, "miann_server_submit: nq = %lld < 1", (long long)nq);
  auto r = std::make_shared<Request>();
  if (sp) r->sp = *sp; else miann_search_params_default(&r->sp);
  if (nq > s->cfg.max_batch_queries || nq > s->cfg.max_inflight_queries ||
      s->batch_bytes(nq, k, itopk, &r->sp) > (size_t)s->cfg.memory_budget_bytes)
    return miann_fail(MIANN_EINVAL, "miann_server_submit: a request of %lld queries exceeds the server limits",
                      (long long)nq);
  if (r->sp.qkeys || r->sp.seeds || r->sp.max_iters_per_query || r->sp.phase_ms || r->sp.phase_events)
    return miann_fail(MIANN_EINVAL, "miann_server_submit: per-query device arrays are not accepted by the server");
  // validate the shape with a zero-query search (no device work)
  miann_status rc = miann_search(s->idx, nullptr, 0, k, itopk, max_iters, &r->sp, nullptr, nullptr, nullptr, nullptr);
  if (rc != MIANN_OK) return rc;
  r->nq = nq;
  r->k = k;
  r->itopk = itopk;
  r->T = max_iters;
  r->q.assign((const uint8_t*)queries, (const uint8_t*)queries + (size_t)nq * s->d * s->esize);
  r->t_submit = clk::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return miann_fail(MIANN_ESTATE, "miann_server_submit: server is shutting down");
    r->ticket = s->next_ticket++;
    auto g = std::find_if(s->pending.begin(), s->pending.end(),
                          [&](const miann_server::ShapeQueue& x) { return same_shape(*x.rep, *r); });
    if (g == s->pending.end()) g = s->pending.insert(s->pending.end(), miann_server::ShapeQueue{r, {}});
    g->q.push_back(r);
    s->n_pending++;
    s->all[r->ticket] = r;
  }
  s->cv_work.notify_one();
  *ticket = r->ticket;
  return MIANN_OK;
}

miann_status miann_server_wait(miann_server* s, uint64_t ticket, uint32_t* ids, void* dists, double* latency_ms) {
  if (!s) return miann_fail(MIANN_EINVAL, "miann_server_wait: null server");
  std::shared_ptr<Request> r;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return miann_fail(MIANN_EINVAL, "miann_server_wait: unknown ticket %llu",
                                              (unsigned long long)ticket);
    r = it->second;
    s->cv_done.wait(lk, [&] { return r->done; });
    s->all.erase(it);
  }
  if (r->status != MIANN_OK) return miann_fail(r->status, "miann_server_wait: %s", r->err.c_str());
  if (ids) std::memcpy(ids, r->ids.data(), r->ids.size() * 4);
  if (dists) std::memcpy(dists, r->dists.data(), r->dists.size());
  if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
  return MIANN_OK;
}

miann_status miann_server_warm(miann_server* s, int64_t nq, int32_t k, int32_t itopk, int32_t max_iters,
                               const miann_search_params* sp) {
  if (!s) return miann_fail(MIANN_EINVAL, "miann_server_warm: null server");
  if (nq < 1 || nq > s->cfg.max_batch_queries) return miann_fail(MIANN_EINVAL, "miann_server_warm: nq out of range");
  miann_search_params p;
  if (sp) p = *sp; else miann_search_params_default(&p);
  miann_status rc = miann_search(s->idx, nullptr, 0, k, itopk, max_iters, &p, nullptr, nullptr, nullptr, nullptr);
  if (rc != MIANN_OK) return rc;
  // every stream runs one search of nq zero queries while no batch is in flight, so that the buffers it keeps
  // (slot staging, search scratch) reach this shape's size before requests arrive
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] {
    for (auto& sl : s->slots)
      if (sl.busy) return false;
    return s->n_pending == 0;
  });
  for (auto& sl : s->slots) {
    if (!s->reserve(sl, nq, k)) return miann_fail(MIANN_ENOMEM, "miann_server_warm: buffer allocation failed");
    void* dq = sl.d_buf;
    uint32_t* di = (uint32_t*)((char*)dq + (size_t)nq * s->d * s->esize + (size_t)nq * 8);
    void* dd = (char*)di + (size_t)nq * k * 4;
    hipError_t e = hipMemsetAsync(dq, 0, (size_t)nq * s->d * s->esize, sl.st);
    if (e == hipSuccess) {
      rc = miann_search(s->idx, dq, nq, k, itopk, max_iters, &p, di, dd, nullptr, sl.st);
      if (rc != MIANN_OK) return rc;
      e = hipStreamSynchronize(sl.st);
    }
    if (e != hipSuccess) return miann_fail(MIANN_EDEVICE, "miann_server_warm: %s", hipGetErrorString(e));
  }
  return MIANN_OK;
}

miann_status miann_server_replay(miann_server* s, const void* queries_host, int64_t pool_rows, const int64_t* row_start,
                                 const int64_t* nq, const int32_t* k, const int32_t* itopk, const int32_t* max_iters,
                                 const double* arrival_s, int64_t n_req, const miann_search_params* sp,
                                 double* latency_ms, double* wall_s) {
  if (!s || !queries_host || !row_start || !nq || !k || !itopk || !max_iters || !arrival_s || !latency_ms)
    return miann_fail(MIANN_EINVAL, "miann_server_replay: null argument");
  if (n_req < 0) return miann_fail(MIANN_EINVAL, "miann_server_replay: n_req < 0");
  for (int64_t j = 0; j < n_req; j++)
    if (row_start[j] < 0 || nq[j] < 1 || row_start[j] + nq[j] > pool_rows || (j > 0 && arrival_s[j] < arrival_s[j - 1]))
      return miann_fail(MIANN_EINVAL, "miann_server_replay: request %lld outside the pool or out of order",
                        (long long)j);
  const size_t row_bytes = (size_t)s->d * s->esize;
  std::vector<uint64_t> tickets((size_t)n_req, 0);
  std::vector<std::atomic<int>> ready((size_t)n_req);
  for (auto& r : ready) r.store(0);
  std::atomic<int> failed{0};
  std::string err;
  const auto t0 = clk::now() + std::chrono::milliseconds(2);
  auto at = [&](int64_t j) {
    return t0 + std::chrono::duration_cast<clk::duration>(std::chrono::duration<double>(arrival_s[j]));
  };
  // the arrivals: each request is submitted at its scheduled time (sleep until shortly before it, then spin)
  std::thread sub([&] {
    for (int64_t j = 0; j < n_req; j++) {
      const auto when = at(j);
      const auto early = when - std::chrono::microseconds(200);
      if (clk::now() < early) std::this_thread::sleep_until(early);
      while (clk::now() < when) {
      }
      uint64_t tk = 0;
      const miann_status st = miann_server_submit(s, (const char*)queries_host + (size_t)row_start[j] * row_bytes,
                                                  nq[j], k[j], itopk[j], max_iters[j], sp, &tk);
      if (st != MIANN_OK) {
        if (!failed.exchange(1)) err = miann_last_error();
        ready[(size_t)j].store(2);
        continue;
      }
      tickets[(size_t)j] = tk;
      ready[(size_t)j].store(1);
    }
  });
  // completions, in arrival order: latency from the scheduled arrival to the batch's completion
  for (int64_t j = 0; j < n_req; j++) {
    int rdy;
    while ((rdy = ready[(size_t)j].load()) == 0) std::this_thread::sleep_for(std::chrono::microseconds(20));
    if (rdy != 1) {
      latency_ms[j] = -1.0;
      continue;
    }
    std::shared_ptr<Request> r;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      auto it = s->all.find(tickets[(size_t)j]);
      r = it->second;
      s->cv_done.wait(lk, [&] { return r->done; });
      s->all.erase(it);
    }
    latency_ms[j] = r->status == MIANN_OK ? std::chrono::duration<double, std::milli>(r->t_done - at(j)).count() : -1.0;
    if (r->status != MIANN_OK && !failed.exchange(1)) err = r->err;
  }
  sub.join();
  if (wall_s) *wall_s = std::chrono::duration<double>(clk::now() - t0).count();
  if (failed.load()) return miann_fail(MIANN_EDEVICE, "miann_server_replay: %s", err.c_str());
  return MIANN_OK;
}

miann_status miann_server_get_stats(miann_server* s, miann_server_stats* out) {
  if (!s || !out) return miann_fail(MIANN_EINVAL, "miann_server_get_stats: null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->elapsed_s = std::chrono::duration<double>(clk::now() - s->t0).count();
  return MIANN_OK;
}

void miann_server_destroy(miann_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->th.joinable()) s->th.join();
  miann_server_destroy_slots(s);
  delete s;
}

}  // extern "C"
