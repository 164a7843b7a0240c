// Continuous-batching solve server: requests are admitted into a running
// engine at chunk boundaries while device memory (an arena of fixed size)
// and slots allow; finished solves are retired between chunks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
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

// Requests of one level count run in their own engine, on their own stream,
// with their own chunk cadence: a slow six-level solve does not hold back the
// two-level solves next to it.
struct Lane {
  int levels = 0;
  std::unique_ptr<Engine> eng;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  int32_t *status = nullptr;  // pinned copy of the status flags, written after each chunk
  bool in_flight = false;
  bool changed = false;       // membership changed since the last chunk
  std::vector<Request *> running;
  double t_launch = 0;        // host time of the chunk in flight
};

// one line of the optional chunk trace (MB_SERVER_TRACE=<file>)
struct ChunkTrace {
  double t_launch, t_done;
  int levels, sims, block, halo, lanes;
  int64_t cells;
};

struct mb_server {
  int device = 0;
  int precision = 32;
  int max_slots = 1;
  int chunk_steps = 32;
  std::map<int, Lane> lanes;  // by level count
  Arena arena;
  // streams created together at start-up (so that they land on different
  // hardware queues).  With at least 8 hardware queues per process every lane
  // gets its own stream (up to 4); with fewer, the lanes of 2 and 3 levels
  // share one stream and those of 4 to 6 levels another, so that a slow lane
  // never queues a fast one behind its chunks.
  static constexpr int kStreams = 4;
  hipStream_t pool[kStreams] = {};
  int n_pool = kStreams;
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  bool started = false, stop = false;
  clk::time_point t0;
  uint64_t next_ticket = 1;
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  std::deque<Request *> queue;      // ordered by arrival
  std::deque<uint64_t> finished;    // tickets that reached a final state, not yet polled
  int n_running = 0;
  size_t outstanding = 0;
  double busy_s = 0;
  int64_t chunks = 0;
  double cell_updates_retired = 0;
  std::string worker_error;
  bool tracing = false;
  std::vector<ChunkTrace> trace;

  double now() const { return std::chrono::duration<double>(clk::now() - t0).count(); }
  void loop();
  void retire(Lane &ln, Request *r, int32_t state);
  int lane_for(int levels, std::string &err);
  hipError_t launch(Lane &ln);
  void finish(Lane &ln, hipError_t he);
};

// Tile shape of one lane for the cells it holds.  Few cells: latency
// shapes (deep halos; large density updates on 128-cell tiles split over up
// to 2 waves per 64 cells, six levels on 64-cell tiles over 4); many cells:
// 256-cell tiles with shallow halos, which redo fewer halo cells.  The split
// itself follows the tile count.
static void server_shape(int levels, int64_t cells, int chunk_steps, int &block, int &halo) {
  const bool busy = cells > (levels >= 4 ? 65536 : 196608);
  if (busy) {
    block = 256;
    halo = 32;
  } else if (levels >= 6) {
    block = 64;  // with 4 wave groups per 64 cells
    halo = 16;
  } else if (levels >= 4) {
    block = 128;
    halo = 32;
  } else {
    block = 256;
    halo = 64;
  }
  halo = std::min(halo, chunk_steps);
}

int mb_server::lane_for(int levels, std::string &err) {
  auto it = lanes.find(levels);
  if (it != lanes.end()) return MB_OK;
  Lane ln;
  ln.levels = levels;
  int block = 256, halo = 32;
  server_shape(levels, 0, chunk_steps, block, halo);
  ln.eng = std::make_unique<Engine>(device, precision, MB_VARIANT_BLOCKED, block, halo, false, 0);
  int rc = ln.eng->init(err);
  if (rc < 0) return rc;
  if (n_pool == kStreams)
    ln.stream = pool[lanes.size() % kStreams];
  else
    ln.stream = pool[levels >= 4 ? 1 : 0];
  if (hipEventCreateWithFlags(&ln.done, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void **>(&ln.status), Engine::kMaxStatusSlots * sizeof(int32_t),
                    hipHostMallocDefault) != hipSuccess) {
    err = "stream or pinned buffer creation failed";
    return MB_ERR_HIP;
  }
  std::memset(ln.status, 0, Engine::kMaxStatusSlots * sizeof(int32_t));
  lanes.emplace(levels, std::move(ln));
  return MB_OK;
}

void mb_server::retire(Lane &ln, Request *r, int32_t state) {
  Engine &e = *ln.eng;
  if (r->engine_id >= 0) {
    const SimState &s = e.sim(r->engine_id);
    r->records.resize(s.plan.records.size());
    r->widths.resize(s.plan.records.size());
    for (size_t q = 0; q < s.plan.records.size(); ++q) {
      (void)e.read_records(r->engine_id, int(q), r->records[q]);
      r->widths[q] = s.plan.records[q].width;
    }
    cell_updates_retired += double(s.done) * double(s.plan.nx);
    e.remove(r->engine_id, &arena);
    ln.changed = true;
  }
  r->state = state;
  r->t_done = now();
  finished.push_back(r->ticket);
  --n_running;
  if (outstanding) --outstanding;
}

// enqueues one chunk (chunk_steps steps) of every simulation of the lane
hipError_t mb_server::launch(Lane &ln) {
  Engine &e = *ln.eng;
  if (ln.changed) {
    int block = 256, halo = 32;
    server_shape(ln.levels, e.total_cells(), chunk_steps, block, halo);
    std::string err;
    (void)e.reshape(block, halo, 0, err);
    ln.changed = false;
  }
  const int k = std::min(chunk_steps, e.chunk_steps());
  const int sub = std::max(1, chunk_steps / e.chunk_steps());
  hipError_t he = e.chunk(ln.stream, k, sub);
  if (he == hipSuccess) he = e.enqueue_status(ln.stream, ln.status);
  if (he == hipSuccess) he = hipEventRecord(ln.done, ln.stream);
  if (he == hipSuccess) {
    ln.in_flight = true;
    ln.t_launch = now();
    ++chunks;
  }
  return he;
}

// after the lane's chunk completed (or failed): status, retirements
void mb_server::finish(Lane &ln, hipError_t he) {
  ln.in_flight = false;
  if (tracing)
    trace.push_back(ChunkTrace{ln.t_launch, now(), ln.levels, int(ln.running.size()), ln.eng->block(),
                               ln.eng->depth(), ln.eng->effective_lanes(ln.levels), ln.eng->total_cells()});
  const int32_t *status = ln.status;
  if (he != hipSuccess) {
    worker_error = hipGetErrorString(he);
    for (Request *r : ln.running) retire(ln, r, MB_ERR_HIP);
    ln.running.clear();
    return;
  }
  for (size_t i = 0; i < ln.running.size();) {
    Request *r = ln.running[i];
    const SimState &s = ln.eng->sim(r->engine_id);
    int32_t st = 0;
    if (status[s.status_slot]) st = MB_ERR_NONFINITE;
    else if (r->cancel) st = 3;
    else if (ln.eng->finished(r->engine_id)) st = 2;
    if (st) {
      retire(ln, r, st);
      ln.running.erase(ln.running.begin() + long(i));
    } else {
      ++i;
    }
  }
}

void mb_server::loop() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  clk::time_point busy_since{};
  bool busy = false;
  while (!stop) {
    // admission: arrived requests in arrival order, while slots and memory
    // allow, into lanes that have no chunk in flight
    double t = now();
    for (auto it = queue.begin(); it != queue.end();) {
      Request *r = *it;
      if (r->cancel) {
        it = queue.erase(it);
        r->state = 3;
        r->t_done = t;
        finished.push_back(r->ticket);
        if (outstanding) --outstanding;
        continue;
      }
      if (r->arrival > t || n_running >= max_slots) break;
      if (arena.capacity() - arena.used() < r->bytes) break;
      const int levels = r->plan.n;
      std::string err;
      int rc = lane_for(levels, err);
      if (rc < 0) {
        it = queue.erase(it);
        r->state = rc;
        r->t_done = t;
        finished.push_back(r->ticket);
        if (outstanding) --outstanding;
        continue;
      }
      Lane &ln = lanes[levels];
      if (ln.in_flight) {
        ++it;
        continue;
      }
      int id = ln.eng->add(std::move(r->plan), &arena, ln.stream, err);
      if (id == MB_ERR_BUDGET) break;  // fragmentation: retry after the next retirement
      it = queue.erase(it);
      if (id < 0) {
        r->state = id;
        r->t_done = t;
        finished.push_back(r->ticket);
        if (outstanding) --outstanding;
        continue;
      }
      r->engine_id = id;
      r->state = 1;
      r->t_admit = now();
      ln.running.push_back(r);
      ln.changed = true;
      ++n_running;
    }
    // launch a chunk in every idle lane with work
    for (auto &[lv, ln] : lanes) {
      if (ln.in_flight || ln.running.empty()) continue;
      hipError_t he = launch(ln);
      if (he != hipSuccess) finish(ln, he);
    }
    bool any = false;
    for (auto &[lv, ln] : lanes) any = any || ln.in_flight;
    if (any && !busy) {
      busy = true;
      busy_since = clk::now();
    }
    if (!any) {
      if (busy) {
        busy = false;
        busy_s += std::chrono::duration<double>(clk::now() - busy_since).count();
      }
      cv.notify_all();
      if (queue.empty())
        cv.wait(lk);
      else {
        double wait = std::max(0.0, queue.front()->arrival - now());
        cv.wait_for(lk, std::chrono::duration<double>(std::min(wait, 0.05)));
      }
      continue;
    }
    // wait for the first lane to complete its chunk (or for a new arrival)
    lk.unlock();
    // poll the lanes' completion events: spinning for the first ~0.5 ms, then
    // in 20 us sleeps
    bool done_any = false;
    const auto w0 = clk::now();
    while (!done_any) {
      for (auto &[lv, ln] : lanes)
        if (ln.in_flight && hipEventQuery(ln.done) != hipErrorNotReady) done_any = true;
      if (!done_any && clk::now() - w0 > std::chrono::microseconds(500))
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    lk.lock();
    for (auto &[lv, ln] : lanes) {
      if (!ln.in_flight) continue;
      hipError_t q = hipEventQuery(ln.done);
      if (q == hipErrorNotReady) continue;
      finish(ln, q);
    }
    cv.notify_all();
  }
  if (busy) busy_s += std::chrono::duration<double>(clk::now() - busy_since).count();
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
  int rc;
  if ((rc = s->arena.init(hbm_budget, err)) < 0) return fail(rc, err);
  {
    const char *hq = std::getenv("GPU_MAX_HW_QUEUES");
    const int queues = hq ? std::atoi(hq) : 4;
    s->n_pool = queues >= 8 ? mb_server::kStreams : 2;
  }
  for (int i = 0; i < s->n_pool; ++i)
    if (hipStreamCreateWithFlags(&s->pool[i], hipStreamNonBlocking) != hipSuccess)
      return fail(MB_ERR_HIP, "stream creation failed");
  s->t0 = clk::now();
  s->tracing = std::getenv("MB_SERVER_TRACE") != nullptr;
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

int mb_server_poll(mb_server *s, uint64_t *done, int32_t capacity, int32_t *n_done) {
  if (!s || !n_done || (capacity > 0 && !done) || capacity < 0) return fail(MB_ERR_ARG, "bad arguments");
  std::lock_guard<std::mutex> lk(s->mu);
  int32_t n = 0;
  while (n < capacity && !s->finished.empty()) {
    done[n++] = s->finished.front();
    s->finished.pop_front();
  }
  *n_done = n;
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
  if (cell_updates) {
    // retired solves plus the progress of the running ones
    double cu = s->cell_updates_retired;
    for (auto &[lv, ln] : s->lanes)
      for (Request *r : ln.running) cu += double(ln.eng->sim(r->engine_id).done) * double(ln.eng->sim(r->engine_id).plan.nx);
    *cell_updates = cu;
  }
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
  if (s->tracing) {
    if (FILE *f = std::fopen(std::getenv("MB_SERVER_TRACE"), "a")) {
      std::fprintf(f, "# server: t_launch t_done levels sims cells block halo lanes\n");
      for (const ChunkTrace &c : s->trace)
        std::fprintf(f, "%.6f %.6f %d %d %lld %d %d %d\n", c.t_launch, c.t_done, c.levels, c.sims,
                     static_cast<long long>(c.cells), c.block, c.halo, c.lanes);
      std::fclose(f);
    }
  }
  (void)hipSetDevice(s->device);
  for (auto &[lv, ln] : s->lanes) {
    if (ln.stream) (void)hipStreamSynchronize(ln.stream);
    ln.eng.reset();
    if (ln.status) (void)hipHostFree(ln.status);
    if (ln.done) (void)hipEventDestroy(ln.done);
  }
  for (auto &q : s->pool)
    if (q) (void)hipStreamDestroy(q);
  delete s;
  return MB_OK;
}

}  // extern "C"
