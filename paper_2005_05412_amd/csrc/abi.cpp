// extern "C" entry points for single simulations and batches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "mb.h"
#include "launch.hpp"
#include "scratch.hpp"
#include "runtime.hpp"
#include "tune.hpp"

namespace mb {
thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}
}  // namespace mb

using namespace mb;

namespace {

// a simulation's device block, rounded to the sub-allocator's granule
constexpr size_t kWorkspaceAlign = 256;
size_t workspace_round(size_t v) { return (v + kWorkspaceAlign - 1) / kWorkspaceAlign * kWorkspaceAlign; }

// One captured run of chunk launches, replayed when the same run (engine
// tables, start step, length) is asked for again, e.g. after mb_reset.
struct GraphCache {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t version = -1, n0 = -1, steps = -1;
  int k = 0;
  void clear() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    version = n0 = steps = -1;
  }
  ~GraphCache() { clear(); }
};

}  // namespace

struct mb_handle {
  int device = 0;
  Arena ws;  // the caller's workspace, if any (declared before eng: outlives it)
  std::unique_ptr<Engine> eng;
  int id = -1;
  hipStream_t last_stream = nullptr;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  double ms_done = 0.0;
  GraphCache gc;
};

struct mb_batch {
  int device = 0;
  std::unique_ptr<Engine> eng;
  std::vector<int> ids;
  hipStream_t last_stream = nullptr;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  double ms_done = 0.0;
  GraphCache gc;
};

namespace {

// Advances the engine by `steps` steps in chunks of at most k.  With
// use_graph the chunk launches are captured into one HIP graph (or the
// cached graph of an identical earlier run is replayed); MB_GRAPHS=0 turns
// capture off (graphs_enabled).

hipError_t run_steps(Engine &eng, hipStream_t st, int64_t steps, int k, bool use_graph, GraphCache &gc) {
  hipError_t e = eng.sync_tables(st);
  use_graph = use_graph && graphs_enabled();
  if (e != hipSuccess) return e;
  // full chunks as persistent launches when every tile fits on the device at
  // once (no graph: one launch covers thousands of chunks), then the tail
  if (eng.persist_ok(k, steps / k)) {
    e = eng.run_persistent(st, k, steps / k);
    if (e == hipSuccess && steps % k) e = eng.chunk(st, int(steps % k));
    return e;
  }
  if (!use_graph) {
    while (steps > 0 && e == hipSuccess) {
      int kk = int(std::min<int64_t>(k, steps));
      e = eng.chunk(st, kk);
      steps -= kk;
    }
    return e;
  }
  const int64_t n0 = eng.engine_step();
  if (gc.exec && gc.version == eng.version() && gc.n0 == n0 && gc.steps == steps && gc.k == k) {
    e = hipGraphLaunch(gc.exec, st);
    for (int64_t left = steps; left > 0 && e == hipSuccess; left -= k) eng.commit_chunk(int(std::min<int64_t>(k, left)));
    return e;
  }
  gc.clear();
  hipStream_t cap;
  if ((e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess) return e;
  e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  // full chunks in one fork/join, then the shorter tail chunk; the host step
  // counters advance only once the graph has been launched
  const int64_t full = steps / k, tail = steps % k;
  const bool plain = eng.variant() == MB_VARIANT_PLAIN;
  if (e == hipSuccess && full > 0) e = eng.launch_only(cap, k, int(full));
  // the tail starts after the full chunks, which are not committed yet
  if (e == hipSuccess && tail > 0)
    e = eng.launch_only(cap, int(tail), 1, full * k, int(plain ? (full * k) & 1 : full & 1));
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(cap, &graph);
  (void)hipStreamDestroy(cap);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(&gc.exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    gc.exec = nullptr;
    return e;
  }
  gc.graph = graph;
  gc.version = eng.version();
  gc.n0 = n0;
  gc.steps = steps;
  gc.k = k;
  e = hipGraphLaunch(gc.exec, st);
  if (e != hipSuccess) {
    gc.clear();
    return e;
  }
  for (int64_t q = 0; q < full; ++q) eng.commit_chunk(k);
  if (tail > 0) eng.commit_chunk(int(tail));
  return hipSuccess;
}

#define MB_GUARD_BEGIN try {
#define MB_GUARD_END                                         \
  }                                                          \
  catch (const std::exception &ex) {                         \
    return fail(MB_ERR_ARG, std::string("exception: ") + ex.what()); \
  }                                                          \
  catch (...) {                                              \
    return fail(MB_ERR_ARG, "unknown exception");            \
  }

int hip_fail(hipError_t e, const char *what) {
  return fail(MB_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int shape_for(const SimPlan &p, int &block, int &halo, int &lanes) {
  default_shape(p.n, p.precision, block, halo);
  lanes = 1;
  if (p.block > 0) block = p.block;
  if (p.depth > 0) halo = p.depth;
  if (p.lanes > 0) lanes = p.lanes;
  if (p.variant == MB_VARIANT_PLAIN) return MB_OK;
  if (!block_supported(block) || halo < 1 || 2 * halo >= block)
    return fail(MB_ERR_ARG, "blocked variant needs block in {64,...,512} and 1 <= depth < block/2");
  return MB_OK;
}

double drain_events(std::vector<std::pair<hipEvent_t, hipEvent_t>> &ev) {
  double total = 0.0;
  for (auto &p : ev) {
    float ms = 0.f;
    if (hipEventSynchronize(p.second) == hipSuccess && hipEventElapsedTime(&ms, p.first, p.second) == hipSuccess)
      total += ms;
    (void)hipEventDestroy(p.first);
    (void)hipEventDestroy(p.second);
  }
  ev.clear();
  return total;
}

}  // namespace

extern "C" {

const char *mb_last_error(void) { return g_last_error.c_str(); }

int mb_device_count(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) return 0;
  return n;
}

int mb_plan_material(const mb_device_desc *dev, const mb_scenario_desc *scen, int32_t material, double *out,
                     int64_t capacity, int64_t *n_out) {
  MB_GUARD_BEGIN
  SimPlan plan;
  std::string err;
  int rc = build_plan(dev, scen, plan, err);
  if (rc < 0) return fail(rc, err);
  if (material < 0 || material >= int(plan.mats.size())) return fail(MB_ERR_ARG, "bad material index");
  const MaterialPlan &mp = plan.mats[material];
  std::vector<double> v;
  if (mp.qm) {
    v.insert(v.end(), mp.lam.begin(), mp.lam.end());
    for (const cd &z : mp.vec) {
      v.push_back(z.real());
      v.push_back(z.imag());
    }
    v.insert(v.end(), mp.kappa.begin(), mp.kappa.end());
    v.push_back(mp.p0);
    for (auto *t : {&mp.at, &mp.ah, &mp.bh, &mp.am, &mp.bf, &mp.t0, &mp.tm, &mp.sm, &mp.as, &mp.bm})
      v.insert(v.end(), t->begin(), t->end());
    for (int l : mp.lvl) v.push_back(double(l));
    v.push_back(plan.block_form ? 1.0 : 0.0);  // the form the kernels run for this simulation
  }
  if (int64_t(v.size()) > capacity) return fail(MB_ERR_ARG, "output buffer too small");
  if (!v.empty()) std::memcpy(out, v.data(), v.size() * sizeof(double));
  if (n_out) *n_out = int64_t(v.size());
  if (rc > 0) fail(rc, "pure dephasing rates admit no completely positive dissipator");
  return rc;
  MB_GUARD_END
}

int mb_plan_readout(const mb_device_desc *dev, const mb_scenario_desc *scen, int32_t record_id, int32_t material,
                    double *out, int64_t capacity) {
  MB_GUARD_BEGIN
  SimPlan plan;
  std::string err;
  int rc = build_plan(dev, scen, plan, err);
  if (rc < 0) return fail(rc, err);
  if (record_id < 0 || record_id >= int(plan.records.size())) return fail(MB_ERR_ARG, "bad record id");
  if (material < 0 || material >= int(plan.mats.size())) return fail(MB_ERR_ARG, "bad material index");
  const RecordPlan &rp = plan.records[record_id];
  const int m1 = ro_len(plan.n);
  if (rp.readout.empty() || !plan.mats[material].qm) return fail(MB_ERR_ARG, "no density readout for this pair");
  if (capacity < m1) return fail(MB_ERR_ARG, "output buffer too small");
  std::memcpy(out, rp.readout.data() + size_t(material) * m1, size_t(m1) * sizeof(double));
  return MB_OK;
  MB_GUARD_END
}

int mb_tile_supported(int32_t levels, int32_t precision, int32_t block, int32_t lanes) {
  if ((levels != 0 && (levels < 2 || levels > 8)) || (precision != 32 && precision != 64)) return 0;
  if (lanes != 1 && lanes != 2 && lanes != 4 && lanes != 8) return 0;
  return shape_supported(levels, precision, block, lanes) ? 1 : 0;
}

int mb_plan_source(const mb_device_desc *dev, const mb_scenario_desc *scen, int32_t source_id, int64_t *node,
                   double *values, int64_t capacity, int64_t *n_out) {
  MB_GUARD_BEGIN
  SimPlan plan;
  std::string err;
  int rc = build_plan(dev, scen, plan, err);
  if (rc < 0) return fail(rc, err);
  if (source_id < 0 || source_id >= int(plan.sources.size())) return fail(MB_ERR_ARG, "bad source id");
  const SourcePlan &sp = plan.sources[source_id];
  if (node) *node = sp.cell;
  const int64_t n = std::min<int64_t>(capacity, int64_t(sp.table.size()));
  if (values && n > 0) std::memcpy(values, sp.table.data(), size_t(n) * sizeof(double));
  if (n_out) *n_out = values ? std::max<int64_t>(n, 0) : 0;
  return rc;
  MB_GUARD_END
}

int mb_workspace_bytes(const mb_device_desc *dev, const mb_scenario_desc *scen, size_t *bytes) {
  MB_GUARD_BEGIN
  if (!bytes) return fail(MB_ERR_ARG, "null output");
  *bytes = 0;
  SimPlan plan;
  std::string err;
  int rc = build_plan(dev, scen, plan, err);
  if (rc < 0) return fail(rc, err);
  *bytes = workspace_round(sim_bytes(plan, plan.precision, plan.variant == MB_VARIANT_PLAIN));
  return MB_OK;
  MB_GUARD_END
}

int mb_setup(int hip_device, const mb_device_desc *dev, const mb_scenario_desc *scen, void *workspace,
             size_t ws_bytes, mb_handle **out) {
  MB_GUARD_BEGIN
  if (!out) return fail(MB_ERR_ARG, "null output handle");
  *out = nullptr;
  SimPlan plan;
  std::string err;
  int rc = build_plan(dev, scen, plan, err);
  if (rc < 0) return fail(rc, err);
  int warn = rc;
  const size_t need = workspace_round(sim_bytes(plan, plan.precision, plan.variant == MB_VARIANT_PLAIN));
  if (workspace) {
    if (reinterpret_cast<uintptr_t>(workspace) % kWorkspaceAlign != 0)
      return fail(MB_ERR_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
      return fail(MB_ERR_ARG, "workspace smaller than mb_workspace_bytes (" + std::to_string(need) + " bytes)");
  }
  int block = 0, halo = 0, lanes = 1;
  bool vc = plan.variant == MB_VARIANT_BLOCKED_REGS, persist = true;
  if ((rc = shape_for(plan, block, halo, lanes)) < 0) return rc;
  if (plan.variant == MB_VARIANT_AUTO && plan.block == 0 && plan.depth == 0 && plan.lanes == 0) {
    if (hipSetDevice(hip_device) != hipSuccess) return fail(MB_ERR_HIP, "hipSetDevice failed");
    Shape sh;
    if ((rc = tune_shape(hip_device, {&plan}, plan.precision, sh, err)) < 0) return fail(rc, err);
    block = sh.block;
    halo = sh.halo;
    vc = sh.vc;
    lanes = sh.lanes;
    persist = sh.persist;
  }
  auto h = std::make_unique<mb_handle>();
  h->device = hip_device;
  int variant = plan.variant == MB_VARIANT_PLAIN ? MB_VARIANT_PLAIN : MB_VARIANT_BLOCKED;
  h->eng = std::make_unique<Engine>(hip_device, plan.precision, variant, block, halo, vc, lanes);
  if ((rc = h->eng->init(err)) < 0) return fail(rc, err);
  h->eng->set_persist(persist);
  hipStream_t st = nullptr;
  if (workspace) h->ws.init_external(workspace, ws_bytes);
  int id = h->eng->add(std::move(plan), workspace ? &h->ws : nullptr, st, err);
  if (id < 0) return fail(id, err);
  h->id = id;
  *out = h.release();
  if (warn > 0) return fail(warn, "pure dephasing rates admit no completely positive dissipator");
  return MB_OK;
  MB_GUARD_END
}

int mb_run(mb_handle *h, int64_t n_steps, void *hip_stream) {
  MB_GUARD_BEGIN
  if (!h) return fail(MB_ERR_ARG, "null handle");
  if (hipSetDevice(h->device) != hipSuccess) return fail(MB_ERR_HIP, "hipSetDevice failed");
  SimState &s = h->eng->sim(h->id);
  int64_t remaining = s.plan.n_steps - s.done;
  if (n_steps < 0 || n_steps > remaining) n_steps = remaining;
  if (n_steps == 0) return MB_OK;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  h->last_stream = st;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
    return fail(MB_ERR_HIP, "hipEventCreate failed");
  hipError_t e = h->eng->sync_tables(st);
  if (e != hipSuccess) return hip_fail(e, "table upload");
  (void)hipEventRecord(a, st);
  const bool plain = h->eng->variant() == MB_VARIANT_PLAIN;
  const int k = plain ? 1 : h->eng->chunk_steps();
  e = run_steps(*h->eng, st, n_steps, k, !plain && n_steps >= 4 * int64_t(k), h->gc);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  (void)hipEventRecord(b, st);
  h->events.emplace_back(a, b);
  return MB_OK;
  MB_GUARD_END
}

int mb_run_static(mb_handle *h, int64_t n_steps, void *hip_stream) {
  MB_GUARD_BEGIN
  if (!h) return fail(MB_ERR_ARG, "null handle");
  if (hipSetDevice(h->device) != hipSuccess) return fail(MB_ERR_HIP, "hipSetDevice failed");
  SimState &s = h->eng->sim(h->id);
  int64_t remaining = s.plan.n_steps - s.done;
  if (n_steps < 0 || n_steps > remaining) n_steps = remaining;
  if (n_steps == 0) return MB_OK;
  std::string err;
  void *base = scratch_address(h->device, err);
  if (!base) return fail(MB_ERR_HIP, err);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (h->last_stream != st) (void)hipStreamSynchronize(h->last_stream);
  h->last_stream = st;
  int rc = MB_OK;
  hipError_t e = h->eng->run_in_tables(st, n_steps, static_cast<char *>(base), scratch_capacity(), rc, err);
  if (rc < 0) return fail(rc, err);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return MB_OK;
  MB_GUARD_END
}

int mb_run_mode(mb_handle *h, int64_t n_steps) {
  MB_GUARD_BEGIN
  if (!h) return fail(MB_ERR_ARG, "null handle");
  if (hipSetDevice(h->device) != hipSuccess) return fail(MB_ERR_HIP, "hipSetDevice failed");
  if (h->eng->variant() == MB_VARIANT_PLAIN) return 0;
  hipError_t e = h->eng->sync_tables(h->last_stream);
  if (e != hipSuccess) return hip_fail(e, "table upload");
  const int k = h->eng->chunk_steps();
  return h->eng->persist_form(k, n_steps / k);
  MB_GUARD_END
}

int mb_reset(mb_handle *h, void *hip_stream) {
  MB_GUARD_BEGIN
  if (!h) return fail(MB_ERR_ARG, "null handle");
  if (hipSetDevice(h->device) != hipSuccess) return fail(MB_ERR_HIP, "hipSetDevice failed");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (h->last_stream != st) (void)hipStreamSynchronize(h->last_stream);
  h->last_stream = st;
  hipError_t e = h->eng->reset(st);
  if (e != hipSuccess) return hip_fail(e, "reset");
  return MB_OK;
  MB_GUARD_END
}

int64_t mb_steps_done(const mb_handle *h) { return h ? h->eng->sim(h->id).done : -1; }

int mb_shape(const mb_handle *h, int32_t *block, int32_t *depth, int32_t *regs, int32_t *lanes) {
  if (!h) return fail(MB_ERR_ARG, "null handle");
  const bool plain = h->eng->variant() == MB_VARIANT_PLAIN;
  if (block) *block = plain ? plain_block() : h->eng->block();
  if (depth) *depth = plain ? 1 : h->eng->chunk_steps();
  if (regs) *regs = h->eng->vc() ? 1 : 0;
  if (lanes) *lanes = plain ? 1 : h->eng->lanes();
  return MB_OK;
}

int mb_batch_shape(const mb_batch *b, int32_t *block, int32_t *depth, int32_t *regs, int32_t *lanes) {
  if (!b) return fail(MB_ERR_ARG, "null batch");
  const bool plain = b->eng->variant() == MB_VARIANT_PLAIN;
  if (block) *block = plain ? plain_block() : b->eng->block();
  if (depth) *depth = plain ? 1 : b->eng->chunk_steps();
  if (regs) *regs = b->eng->vc() ? 1 : 0;
  if (lanes) *lanes = plain ? 1 : b->eng->lanes();
  return MB_OK;
}

int mb_record_shape(const mb_handle *h, int record_id, int64_t *n_samples, int64_t *width) {
  if (!h) return fail(MB_ERR_ARG, "null handle");
  const SimState &s = h->eng->sim(h->id);
  if (record_id < 0 || record_id >= int(s.plan.records.size())) return fail(MB_ERR_ARG, "bad record id");
  const RecordPlan &rp = s.plan.records[record_id];
  if (n_samples) *n_samples = std::min<int64_t>(rp.n_samples, s.done / rp.interval);
  if (width) *width = rp.width;
  return MB_OK;
}

int mb_read_records(mb_handle *h, int record_id, double *out, int64_t capacity, int64_t *n_out) {
  MB_GUARD_BEGIN
  if (!h) return fail(MB_ERR_ARG, "null handle");
  if (hipSetDevice(h->device) != hipSuccess) return fail(MB_ERR_HIP, "hipSetDevice failed");
  SimState &s = h->eng->sim(h->id);
  if (record_id < 0 || record_id >= int(s.plan.records.size())) return fail(MB_ERR_ARG, "bad record id");
  hipError_t e = hipStreamSynchronize(h->last_stream);
  if (e != hipSuccess) return hip_fail(e, "stream synchronize");
  std::vector<double> buf;
  e = h->eng->read_records(h->id, record_id, buf);
  if (e != hipSuccess) return hip_fail(e, "record copy");
  if (int64_t(buf.size()) > capacity) return fail(MB_ERR_ARG, "output buffer too small");
  if (!buf.empty()) std::memcpy(out, buf.data(), buf.size() * sizeof(double));
  if (n_out) *n_out = int64_t(buf.size());
  std::vector<int32_t> st;
  if (h->eng->read_status(st) == hipSuccess && (st[s.status_slot] & kStatusWaitTimeout))
    return fail(MB_ERR_DEVICE, "a tile gave up waiting for its neighbours in a persistent launch");
  if (st[s.status_slot] & kStatusNonFinite)
    return fail(MB_ERR_NONFINITE, "the simulation produced a non-finite field value");
  return MB_OK;
  MB_GUARD_END
}

int mb_read_state(mb_handle *h, double *e, double *hfield, double *rho) {
  MB_GUARD_BEGIN
  if (!h) return fail(MB_ERR_ARG, "null handle");
  if (hipSetDevice(h->device) != hipSuccess) return fail(MB_ERR_HIP, "hipSetDevice failed");
  hipError_t er = hipStreamSynchronize(h->last_stream);
  if (er != hipSuccess) return hip_fail(er, "stream synchronize");
  er = h->eng->read_state(h->id, e, hfield, rho);
  if (er != hipSuccess) return hip_fail(er, "state copy");
  return MB_OK;
  MB_GUARD_END
}

int mb_elapsed_ms(mb_handle *h, double *ms) {
  if (!h || !ms) return fail(MB_ERR_ARG, "null argument");
  h->ms_done += drain_events(h->events);
  *ms = h->ms_done;
  return MB_OK;
}

int mb_destroy(mb_handle *h) {
  if (!h) return MB_OK;
  (void)hipSetDevice(h->device);
  if (h->last_stream) (void)hipStreamSynchronize(h->last_stream);
  drain_events(h->events);
  delete h;
  return MB_OK;
}

// ---------------------------------------------------------------- batches

int mb_batch_setup(int hip_device, int32_t n, const mb_device_desc *devs, const mb_scenario_desc *scens,
                   mb_batch **out) {
  MB_GUARD_BEGIN
  if (!out || n < 1 || !devs || !scens) return fail(MB_ERR_ARG, "bad batch arguments");
  *out = nullptr;
  std::vector<SimPlan> plans(n);
  std::string err;
  for (int i = 0; i < n; ++i) {
    int rc = build_plan(&devs[i], &scens[i], plans[i], err);
    if (rc < 0) return fail(rc, "simulation " + std::to_string(i) + ": " + err);
    if (plans[i].precision != plans[0].precision || (plans[i].variant == MB_VARIANT_PLAIN) != (plans[0].variant == MB_VARIANT_PLAIN))
      return fail(MB_ERR_ARG, "batch members must share precision and variant");
  }
  int block = 0, halo = 0, lanes = 1, rc;
  bool vc = plans[0].variant == MB_VARIANT_BLOCKED_REGS, persist = true;
  int nmax = 0;
  for (auto &p : plans) nmax = std::max(nmax, p.n);
  SimPlan probe;
  probe.n = nmax;
  probe.precision = plans[0].precision;
  probe.variant = plans[0].variant;
  probe.block = plans[0].block;
  probe.depth = plans[0].depth;
  probe.lanes = plans[0].lanes;
  if ((rc = shape_for(probe, block, halo, lanes)) < 0) return rc;
  if (probe.variant == MB_VARIANT_AUTO && probe.block == 0 && probe.depth == 0 && probe.lanes == 0) {
    if (hipSetDevice(hip_device) != hipSuccess) return fail(MB_ERR_HIP, "hipSetDevice failed");
    std::vector<const SimPlan *> ptrs;
    for (auto &p : plans) ptrs.push_back(&p);
    Shape sh;
    if ((rc = tune_shape(hip_device, ptrs, probe.precision, sh, err)) < 0) return fail(rc, err);
    block = sh.block;
    halo = sh.halo;
    vc = sh.vc;
    lanes = sh.lanes;
    persist = sh.persist;
  }
  auto b = std::make_unique<mb_batch>();
  b->device = hip_device;
  int variant = plans[0].variant == MB_VARIANT_PLAIN ? MB_VARIANT_PLAIN : MB_VARIANT_BLOCKED;
  b->eng = std::make_unique<Engine>(hip_device, plans[0].precision, variant, block, halo, vc, lanes);
  if ((rc = b->eng->init(err)) < 0) return fail(rc, err);
  b->eng->set_persist(persist);
  for (int i = 0; i < n; ++i) {
    int id = b->eng->add(std::move(plans[i]), nullptr, nullptr, err);
    if (id < 0) return fail(id, "simulation " + std::to_string(i) + ": " + err);
    b->ids.push_back(id);
  }
  *out = b.release();
  return MB_OK;
  MB_GUARD_END
}

int mb_batch_run(mb_batch *b, void *hip_stream, int32_t use_graph) {
  MB_GUARD_BEGIN
  if (!b) return fail(MB_ERR_ARG, "null batch");
  if (hipSetDevice(b->device) != hipSuccess) return fail(MB_ERR_HIP, "hipSetDevice failed");
  Engine &eng = *b->eng;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  b->last_stream = st;
  int64_t remaining = 0;
  for (int id : b->ids) {
    const SimState &s = eng.sim(id);
    remaining = std::max<int64_t>(remaining, s.plan.n_steps - s.done);
  }
  if (remaining <= 0) return MB_OK;
  hipError_t e = eng.sync_tables(st);
  if (e != hipSuccess) return hip_fail(e, "table upload");
  const bool plain = eng.variant() == MB_VARIANT_PLAIN;
  const int k = plain ? 1 : eng.chunk_steps();
  hipEvent_t ea, eb;
  if (hipEventCreate(&ea) != hipSuccess || hipEventCreate(&eb) != hipSuccess)
    return fail(MB_ERR_HIP, "hipEventCreate failed");
  (void)hipEventRecord(ea, st);
  e = run_steps(eng, st, remaining, k, use_graph != 0 && !plain, b->gc);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  (void)hipEventRecord(eb, st);
  b->events.emplace_back(ea, eb);
  return MB_OK;
  MB_GUARD_END
}

int mb_batch_run_mode(mb_batch *b) {
  MB_GUARD_BEGIN
  if (!b) return fail(MB_ERR_ARG, "null batch");
  if (hipSetDevice(b->device) != hipSuccess) return fail(MB_ERR_HIP, "hipSetDevice failed");
  Engine &eng = *b->eng;
  if (eng.variant() == MB_VARIANT_PLAIN) return 0;
  int64_t remaining = 0;
  for (int id : b->ids) {
    const SimState &s = eng.sim(id);
    remaining = std::max<int64_t>(remaining, s.plan.n_steps - s.done);
  }
  hipError_t e = eng.sync_tables(b->last_stream);
  if (e != hipSuccess) return hip_fail(e, "table upload");
  const int k = eng.chunk_steps();
  return eng.persist_form(k, remaining / k);
  MB_GUARD_END
}

int mb_batch_reset(mb_batch *b, void *hip_stream) {
  MB_GUARD_BEGIN
  if (!b) return fail(MB_ERR_ARG, "null batch");
  if (hipSetDevice(b->device) != hipSuccess) return fail(MB_ERR_HIP, "hipSetDevice failed");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (b->last_stream != st) (void)hipStreamSynchronize(b->last_stream);
  b->last_stream = st;
  hipError_t e = b->eng->reset(st);
  if (e != hipSuccess) return hip_fail(e, "reset");
  return MB_OK;
  MB_GUARD_END
}

int mb_batch_record_shape(const mb_batch *b, int32_t sim, int record_id, int64_t *n_samples, int64_t *width) {
  if (!b || sim < 0 || sim >= int(b->ids.size())) return fail(MB_ERR_ARG, "bad batch member");
  const SimState &s = b->eng->sim(b->ids[sim]);
  if (record_id < 0 || record_id >= int(s.plan.records.size())) return fail(MB_ERR_ARG, "bad record id");
  const RecordPlan &rp = s.plan.records[record_id];
  if (n_samples) *n_samples = std::min<int64_t>(rp.n_samples, s.done / rp.interval);
  if (width) *width = rp.width;
  return MB_OK;
}

int mb_batch_read_records(mb_batch *b, int32_t sim, int record_id, double *out, int64_t capacity, int64_t *n_out) {
  MB_GUARD_BEGIN
  if (!b || sim < 0 || sim >= int(b->ids.size())) return fail(MB_ERR_ARG, "bad batch member");
  if (hipSetDevice(b->device) != hipSuccess) return fail(MB_ERR_HIP, "hipSetDevice failed");
  SimState &s = b->eng->sim(b->ids[sim]);
  if (record_id < 0 || record_id >= int(s.plan.records.size())) return fail(MB_ERR_ARG, "bad record id");
  hipError_t e = hipStreamSynchronize(b->last_stream);
  if (e != hipSuccess) return hip_fail(e, "stream synchronize");
  std::vector<double> buf;
  e = b->eng->read_records(b->ids[sim], record_id, buf);
  if (e != hipSuccess) return hip_fail(e, "record copy");
  if (int64_t(buf.size()) > capacity) return fail(MB_ERR_ARG, "output buffer too small");
  if (!buf.empty()) std::memcpy(out, buf.data(), buf.size() * sizeof(double));
  if (n_out) *n_out = int64_t(buf.size());
  std::vector<int32_t> st;
  if (b->eng->read_status(st) == hipSuccess && (st[s.status_slot] & kStatusWaitTimeout))
    return fail(MB_ERR_DEVICE, "a tile gave up waiting for its neighbours in a persistent launch");
  if (st[s.status_slot] & kStatusNonFinite)
    return fail(MB_ERR_NONFINITE, "the simulation produced a non-finite field value");
  return MB_OK;
  MB_GUARD_END
}

int mb_batch_elapsed_ms(mb_batch *b, double *ms) {
  if (!b || !ms) return fail(MB_ERR_ARG, "null argument");
  b->ms_done += drain_events(b->events);
  *ms = b->ms_done;
  return MB_OK;
}

int mb_batch_destroy(mb_batch *b) {
  if (!b) return MB_OK;
  (void)hipSetDevice(b->device);
  if (b->last_stream) (void)hipStreamSynchronize(b->last_stream);
  drain_events(b->events);
  delete b;
  return MB_OK;
}

}  // extern "C"
