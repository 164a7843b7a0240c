// Continuous-batching solve server: requests are admitted into a running
// engine at chunk boundaries while device memory (an arena of fixed size)
// and slots allow; finished solves are retired between chunks.
#include <hip/hip_runtime.h>

#include <algorithm>
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

#include "mb.h"
#include "runtime.hpp"

namespace mb {
int fail(int code, const std::string &msg);
}
using namespace mb;

namespace {

using clk = std::chrono::steady_clock;

struct Request {
  uint64_t ticket = 0;
  SimPlan plan;
  size_t bytes = 0;
  double arrival = 0, t_admit = -1, t_done = -1;
  int32_t state = 0;  // 0 queued, 1 running, 2 done, 3 cancelled, <0 error
  bool cancel = false;
  int engine_id = -1;
  std::vector<std::vector<double>> records;
  std::vector<int64_t> widths;
};

}  // namespace

struct mb_server {
  int device = 0;
  int precision = 32;
  int max_slots = 1;
  int chunk_steps = 32;
  std::unique_ptr<Engine> eng;
  Arena arena;
  hipStream_t stream = nullptr, side = nullptr;
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  bool started = false, stop = false;
  clk::time_point t0;
  uint64_t next_ticket = 1;
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  std::deque<Request *> queue;      // ordered by arrival
  std::vector<Request *> running;
  size_t outstanding = 0;
  double busy_s = 0;
  int64_t chunks = 0;
  std::string worker_error;

  double now() const { return std::chrono::duration<double>(clk::now() - t0).count(); }
  void loop();
  void retire(Request *r, int32_t state);
};

void mb_server::retire(Request *r, int32_t state) {
  Engine &e = *eng;
  if (r->engine_id >= 0) {
    const SimState &s = e.sim(r->engine_id);
    r->records.resize(s.plan.records.size());
    r->widths.resize(s.plan.records.size());
    for (size_t q = 0; q < s.plan.records.size(); ++q) {
      (void)e.read_records(r->engine_id, int(q), r->records[q]);
      r->widths[q] = s.plan.records[q].width;
    }
    e.remove(r->engine_id, &arena);
  }
  r->state = state;
  r->t_done = now();
  if (outstanding) --outstanding;
}

void mb_server::loop() {
  (void)hipSetDevice(device);
  Engine &e = *eng;
  std::unique_lock<std::mutex> lk(mu);
  while (!stop) {
    // admission: arrived requests in arrival order, while slots and memory allow
    double t = now();
    while (!queue.empty()) {
      Request *r = queue.front();
      if (r->cancel) {
        queue.pop_front();
        r->state = 3;
        r->t_done = t;
        if (outstanding) --outstanding;
        continue;
      }
      if (r->arrival > t || int(running.size()) >= max_slots) break;
      if (arena.capacity() - arena.used() < r->bytes) break;
      std::string err;
      int id = e.add(std::move(r->plan), &arena, side, err);
      queue.pop_front();
      if (id == MB_ERR_BUDGET) {  // fragmentation: retry after the next retirement
        queue.push_front(r);
        break;
      }
      if (id < 0) {
        r->state = id;
        r->t_done = t;
        if (outstanding) --outstanding;
        continue;
      }
      r->engine_id = id;
      r->state = 1;
      r->t_admit = now();
      running.push_back(r);
    }
    if (running.empty()) {
      if (queue.empty())
        cv.wait(lk);
      else {
        double wait = std::max(0.0, queue.front()->arrival - now());
        cv.wait_for(lk, std::chrono::duration<double>(std::min(wait, 0.05)));
      }
      continue;
    }
    lk.unlock();
    auto tb = clk::now();
    hipError_t he = hipSuccess;
    int k = e.variant() == MB_VARIANT_PLAIN ? chunk_steps : std::min(chunk_steps, e.chunk_steps());
    int sub = e.variant() == MB_VARIANT_PLAIN ? 1 : std::max(1, chunk_steps / e.chunk_steps());
    he = e.chunk(stream, k, sub);
    if (he == hipSuccess) he = hipStreamSynchronize(stream);
    std::vector<int32_t> status;
    if (he == hipSuccess) he = e.read_status(status);
    busy_s += std::chrono::duration<double>(clk::now() - tb).count();
    lk.lock();
    ++chunks;
    if (he != hipSuccess) {
      worker_error = hipGetErrorString(he);
      for (Request *r : running) retire(r, MB_ERR_HIP);
      running.clear();
      continue;
    }
    for (size_t i = 0; i < running.size();) {
      Request *r = running[i];
      const SimState &s = e.sim(r->engine_id);
      int32_t st = 0;
      if (status[s.status_slot]) st = MB_ERR_NONFINITE;
      else if (r->cancel) st = 3;
      else if (e.finished(r->engine_id)) st = 2;
      if (st) {
        retire(r, st);
        running.erase(running.begin() + long(i));
      } else {
        ++i;
      }
    }
    cv.notify_all();
  }
}

extern "C" {

int mb_server_create(int hip_device, size_t hbm_budget, int32_t max_slots, int32_t precision,
                     int32_t chunk_steps, mb_server **out) {
  if (!out || max_slots < 1 || (precision != 32 && precision != 64) || chunk_steps < 1 || hbm_budget == 0)
    return fail(MB_ERR_ARG, "bad server arguments");
  *out = nullptr;
  auto s = std::make_unique<mb_server>();
  s->device = hip_device;
  s->precision = precision;
  s->max_slots = std::min(max_slots, 4000);
  s->chunk_steps = chunk_steps;
  std::string err;
  if (hipSetDevice(hip_device) != hipSuccess) return fail(MB_ERR_HIP, "hipSetDevice failed");
  int block = 256, halo = 32;
  default_shape(3, precision, block, halo);
  halo = std::min(halo, chunk_steps);
  // waves per cell chosen per launch from the load: a lightly loaded server
  // spreads each cell's density update over more waves
  s->eng = std::make_unique<Engine>(hip_device, precision, MB_VARIANT_BLOCKED, block, halo, false, 0);
  int rc = s->eng->init(err);
  if (rc < 0) return fail(rc, err);
  if ((rc = s->arena.init(hbm_budget, err)) < 0) return fail(rc, err);
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking) != hipSuccess)
    return fail(MB_ERR_HIP, "stream creation failed");
  s->t0 = clk::now();
  *out = s.release();
  return MB_OK;
}

int mb_server_submit(mb_server *s, const mb_device_desc *dev, const mb_scenario_desc *scen, double arrival_s,
                     uint64_t *ticket) {
  if (!s || !ticket) return fail(MB_ERR_ARG, "null argument");
  auto r = std::make_unique<Request>();
  std::string err;
  int rc;
  try {
    rc = build_plan(dev, scen, r->plan, err);
  } catch (...) {
    return fail(MB_ERR_ARG, "exception while planning");
  }
  if (rc < 0) return fail(rc, err);
  r->plan.precision = s->precision;
  r->plan.variant = MB_VARIANT_BLOCKED;
  r->bytes = sim_bytes(r->plan, s->precision, false) + 256;
  if (r->bytes > s->arena.capacity())
    return fail(MB_ERR_BUDGET, "request needs more device memory than the server budget");
  r->arrival = arrival_s;
  std::lock_guard<std::mutex> lk(s->mu);
  r->ticket = s->next_ticket++;
  *ticket = r->ticket;
  Request *raw = r.get();
  s->reqs[r->ticket] = std::move(r);
  auto it = std::upper_bound(s->queue.begin(), s->queue.end(), raw,
                             [](const Request *a, const Request *b) { return a->arrival < b->arrival; });
  s->queue.insert(it, raw);
  ++s->outstanding;
  s->cv.notify_all();
  return MB_OK;
}

int mb_server_start(mb_server *s) {
  if (!s) return fail(MB_ERR_ARG, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->started) return MB_OK;
  s->t0 = clk::now();
  s->started = true;
  s->worker = std::thread([s] { s->loop(); });
  return MB_OK;
}

int mb_server_drain(mb_server *s, double timeout_s) {
  if (!s) return fail(MB_ERR_ARG, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto deadline = clk::now() + std::chrono::duration_cast<clk::duration>(std::chrono::duration<double>(timeout_s));
  while (s->outstanding > 0) {
    if (s->cv.wait_until(lk, deadline) == std::cv_status::timeout && s->outstanding > 0)
      return fail(MB_ERR_STATE, "timeout while draining the server");
  }
  return MB_OK;
}

int mb_server_cancel(mb_server *s, uint64_t ticket) {
  if (!s) return fail(MB_ERR_ARG, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(MB_ERR_ARG, "unknown ticket");
  it->second->cancel = true;
  s->cv.notify_all();
  return MB_OK;
}

int mb_server_status(mb_server *s, uint64_t ticket, int32_t *state, double *t_arrival, double *t_admit,
                     double *t_done) {
  if (!s) return fail(MB_ERR_ARG, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(MB_ERR_ARG, "unknown ticket");
  const Request &r = *it->second;
  if (state) *state = r.state;
  if (t_arrival) *t_arrival = r.arrival;
  if (t_admit) *t_admit = r.t_admit;
  if (t_done) *t_done = r.t_done;
  return MB_OK;
}

int mb_server_record_shape(mb_server *s, uint64_t ticket, int record_id, int64_t *n_samples, int64_t *width) {
  if (!s) return fail(MB_ERR_ARG, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(MB_ERR_ARG, "unknown ticket");
  const Request &r = *it->second;
  if (r.state != 2) return fail(MB_ERR_STATE, "request not done");
  if (record_id < 0 || record_id >= int(r.records.size())) return fail(MB_ERR_ARG, "bad record id");
  int64_t w = std::max<int64_t>(1, r.widths[record_id]);
  if (n_samples) *n_samples = int64_t(r.records[record_id].size()) / w;
  if (width) *width = w;
  return MB_OK;
}

int mb_server_read_records(mb_server *s, uint64_t ticket, int record_id, double *out, int64_t capacity,
                           int64_t *n_out) {
  if (!s) return fail(MB_ERR_ARG, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(MB_ERR_ARG, "unknown ticket");
  const Request &r = *it->second;
  if (r.state != 2) return fail(r.state < 0 ? r.state : MB_ERR_STATE, "request not done");
  if (record_id < 0 || record_id >= int(r.records.size())) return fail(MB_ERR_ARG, "bad record id");
  const auto &v = r.records[record_id];
  if (int64_t(v.size()) > capacity) return fail(MB_ERR_ARG, "output buffer too small");
  if (!v.empty()) std::memcpy(out, v.data(), v.size() * sizeof(double));
  if (n_out) *n_out = int64_t(v.size());
  return MB_OK;
}

int mb_server_stats(mb_server *s, double *cell_updates, double *busy_s, int64_t *chunks) {
  if (!s) return fail(MB_ERR_ARG, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  if (cell_updates) *cell_updates = s->eng->cell_updates();
  if (busy_s) *busy_s = s->busy_s;
  if (chunks) *chunks = s->chunks;
  return MB_OK;
}

int mb_server_destroy(mb_server *s) {
  if (!s) return MB_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->device);
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  s->eng.reset();
  if (s->stream) (void)hipStreamDestroy(s->stream);
  if (s->side) (void)hipStreamDestroy(s->side);
  delete s;
  return MB_OK;
}

}  // extern "C"
