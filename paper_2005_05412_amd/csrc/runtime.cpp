#include "runtime.hpp"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <numeric>

#include "launch.hpp"
#include "scratch.hpp"

namespace mb {

namespace {
constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
constexpr int kStatusSlots = Engine::kMaxStatusSlots;

struct Layout {
  size_t e, h, x, init_e, init_x, p, mat_e, mat_h, mtab, src, src_tab, rec, readout, rec_first, rec_ids, rec_all;
  size_t qs, init_q, qtab;  // strong coupling
  size_t outputs, end_head, total;
  std::vector<size_t> tab_off, ro_off, out_off;
  int n_point = 0, n_all = 0;
};

Layout layout_of(const SimPlan &p, int precision, bool plain) {
  Layout L;
  const size_t rs = precision == 64 ? 8 : 4;
  const size_t nx = size_t(p.nx);
  const size_t m = size_t(p.m);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.e = take(2 * nx * rs);
  L.h = take(2 * nx * rs);
  const size_t planes = size_t(state_planes(p.n, precision));
  L.x = take(std::max<size_t>(1, 2 * planes * nx) * rs);
  L.init_e = take(nx * rs);
  L.init_x = take(std::max<size_t>(1, m * nx) * rs);
  L.p = take(plain ? nx * rs : rs);
  L.mat_e = take(nx);
  L.mat_h = take(nx);
  L.mtab = take(p.mats.size() * size_t(stride_of(p.n, p.block_form)) * rs);
  const bool strong = p.coupling == MB_COUPLING_STRONG && p.n > 0;
  L.qs = take(strong ? 4 * nx * sizeof(double) : sizeof(double));  // tr{mu rho} x 2, then p x 2
  L.init_q = take(strong ? nx * sizeof(double) : sizeof(double));
  L.qtab = take(strong ? p.mats.size() * size_t(ro_len(p.n)) * sizeof(double) : sizeof(double));
  L.src = take(std::max<size_t>(1, p.sources.size()) * sizeof(DevSource));
  for (auto &s : p.sources) L.tab_off.push_back(take(s.table.size() * sizeof(double)));
  L.rec = take(std::max<size_t>(1, p.records.size()) * sizeof(DevRecord));
  for (auto &r : p.records) {
    L.ro_off.push_back(r.readout.empty() ? 0 : take(r.readout.size() * sizeof(double)));
    if (r.cell >= 0)
      ++L.n_point;
    else
      ++L.n_all;
  }
  L.rec_first = L.n_point ? take((nx + 1) * sizeof(int32_t)) : 0;
  L.rec_ids = take(std::max(1, L.n_point) * sizeof(DevRecord));
  L.rec_all = take(std::max(1, L.n_all) * sizeof(int32_t));
  L.end_head = off;
  for (auto &r : p.records) L.out_off.push_back(take(size_t(r.n_samples) * size_t(r.width) * sizeof(double)));
  L.total = off;
  return L;
}

template <typename R>
void fill_mtab(const SimPlan &p, R *out) {
  const int n = p.n, s = stride_of(n, p.block_form), m = mat_m(n);
  for (size_t i = 0; i < p.mats.size(); ++i) {
    const MaterialPlan &mp = p.mats[i];
    R *t = out + i * s;
    t[kCoefA] = R(mp.ca);
    t[kCoefBG] = R(mp.cbg);
    t[kCoefBD] = R(mp.cbd);
    t[kCoefH] = R(mp.ch);
    if (n == 0) continue;
    t[kCoefQM] = mp.qm ? R(1) : R(0);
    if (!mp.qm) continue;  // the table is zero-initialised
    const int k = mat_k(n), w = prop_w(n);
    for (int q = 0; q < n - 1; ++q) t[kCoefKap + q] = R(mp.kappa[q]);
    t[coef_p0(n)] = R(mp.p0);
    for (int a = 0; a < m; ++a) t[coef_at(n) + a] = R(mp.at[a]);
    for (int r = 0; r < k; ++r) t[coef_as(n) + r] = R(mp.as[r]);
    if (p.block_form) {
      auto put = [&](int off, const std::vector<double> &v) {
        for (size_t j = 0; j < v.size(); ++j) t[off + int(j)] = R(v[j]);
      };
      put(bk_bf(n), mp.bfp);
      put(bk_ap(n), mp.ap);
      put(bk_blk(n), mp.blk);
      put(bk_t0(n), mp.t0r);
      put(bk_tp(n), mp.tp);
      put(bk_tr(n), mp.tr);
      put(bk_ti(n), mp.ti);
      put(bk_sp(n), mp.sp);
      put(bk_sr(n), mp.sr);
      put(bk_si(n), mp.si);
      put(bk_sg(n), mp.sigma);
      continue;
    }
    for (int a = 0; a < m; ++a) {
      t[coef_bf(n) + a] = R(mp.bf[a]);
      for (int b = 0; b < m; ++b) t[coef_am(n) + a * w + b] = R(mp.am[size_t(a) * m + b]);
      for (int r = 0; r < k; ++r) t[coef_am(n) + a * w + m + r] = R(mp.bm[size_t(a) * k + r]);
    }
    for (int r = 0; r < k; ++r) {
      t[coef_t0(n) + r] = R(mp.t0[r]);
      for (int b = 0; b < m; ++b) t[coef_tm(n) + r * m + b] = R(mp.tm[size_t(r) * m + b]);
    }
    for (int j = 0; j < n; ++j) t[coef_sg(n) + j] = R(mp.sigma[j]);
  }
}

template <typename R>
void fill_state(const SimPlan &p, char *head, const Layout &L) {
  const size_t nx = size_t(p.nx);
  R *e = reinterpret_cast<R *>(head + L.e);
  R *h = reinterpret_cast<R *>(head + L.h);
  R *x = reinterpret_cast<R *>(head + L.x);
  R *ie = reinterpret_cast<R *>(head + L.init_e);
  R *ix = reinterpret_cast<R *>(head + L.init_x);
  for (size_t c = 0; c < nx; ++c) {
    e[c] = e[nx + c] = ie[c] = R(p.e0[c]);
    h[c] = h[nx + c] = R(0);
  }
  const size_t mn = size_t(p.m) * nx;
  const size_t pn = size_t(state_planes(p.n, sizeof(R) == 4 ? 32 : 64)) * nx;  // planes of one buffer
  for (size_t q = 0; q < mn; ++q) x[q] = x[pn + q] = ix[q] = R(p.x0[q]);
  for (size_t q = mn; q < pn; ++q) x[q] = x[pn + q] = R(0);  // FP32 compensation
  fill_mtab<R>(p, reinterpret_cast<R *>(head + L.mtab));
  if (p.coupling == MB_COUPLING_STRONG && p.n > 0) {
    double *qs = reinterpret_cast<double *>(head + L.qs);
    double *iq = reinterpret_cast<double *>(head + L.init_q);
    for (size_t c = 0; c < nx; ++c) {
      qs[c] = qs[nx + c] = iq[c] = p.q0[c];
      qs[2 * nx + c] = qs[3 * nx + c] = 0.0;  // no polarization current before the first step
    }
    double *qt = reinterpret_cast<double *>(head + L.qtab);
    const size_t rl = size_t(ro_len(p.n)), k = size_t(mat_k(p.n));
    for (size_t i = 0; i < p.mats.size(); ++i) {
      const MaterialPlan &mp = p.mats[i];
      qt[i * rl] = mp.qm ? mp.qc : 0.0;
      for (int a = 0; a < p.m; ++a) qt[i * rl + 1 + a] = mp.qm ? mp.aq[a] : 0.0;
      for (size_t r = 0; r < k; ++r) qt[i * rl + 1 + p.m + r] = mp.qm ? mp.aqs[r] : 0.0;
    }
  }
}

}  // namespace

size_t sim_bytes(const SimPlan &p, int precision, bool plain) { return layout_of(p, precision, plain).total; }

bool graphs_enabled() {
  static const bool on = [] {
    const char *v = std::getenv("MB_GRAPHS");
    return !(v && v[0] == '0');
  }();
  return on;
}

void default_shape(int levels, int precision, int &block, int &halo) {
  (void)precision;
  if (levels >= 5) {
    block = 256;
    halo = 16;
  } else {
    block = 256;
    halo = 32;
  }
}

// ---------------------------------------------------------------- Arena

Arena::~Arena() {
  if (base_ && own_) (void)hipFree(base_);
}

void Arena::init_external(void *base, size_t bytes) {
  base_ = static_cast<char *>(base);
  own_ = false;
  cap_ = bytes / kAlign * kAlign;
  used_ = 0;
  free_.clear();
  live_.clear();
  if (cap_) free_[0] = cap_;
}

int Arena::init(size_t bytes, std::string &err) {
  bytes = align_up(bytes);
  if (hipMalloc(&base_, bytes) != hipSuccess) {
    base_ = nullptr;
    err = "device allocation of the serving budget failed";
    return MB_ERR_OOM;
  }
  cap_ = bytes;
  free_[0] = bytes;
  return MB_OK;
}

void *Arena::alloc(size_t bytes) {
  bytes = align_up(std::max<size_t>(bytes, 1));
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second < bytes) continue;
    size_t off = it->first, sz = it->second;
    free_.erase(it);
    if (sz > bytes) free_[off + bytes] = sz - bytes;
    live_[off] = bytes;
    used_ += bytes;
    return base_ + off;
  }
  return nullptr;
}

void Arena::release(void *p) {
  if (!p) return;
  size_t off = size_t(static_cast<char *>(p) - base_);
  auto it = live_.find(off);
  if (it == live_.end()) return;
  size_t sz = it->second;
  live_.erase(it);
  used_ -= sz;
  auto nx = free_.lower_bound(off);
  if (nx != free_.end() && off + sz == nx->first) {
    sz += nx->second;
    free_.erase(nx);
  }
  auto pv = free_.lower_bound(off);
  if (pv != free_.begin()) {
    --pv;
    if (pv->first + pv->second == off) {
      pv->second += sz;
      return;
    }
  }
  free_[off] = sz;
}

// ---------------------------------------------------------------- Engine

Engine::Engine(int device, int precision, int variant, int block, int halo, bool vc, int lanes)
    : device_(device), precision_(precision), variant_(variant), block_(block), halo_(halo), vc_(vc), lanes_(lanes) {}

Engine::~Engine() {
  for (auto &s : sims_)
    if (s && s->own_block && s->block) (void)hipFree(s->block);
  for (auto &g : groups_) {
    if (g.d_sims) (void)hipFree(g.d_sims);
    if (g.d_tiles) (void)hipFree(g.d_tiles);
    if (g.d_flags) (void)hipFree(g.d_flags);
  }
  if (d_status_) (void)hipFree(d_status_);
  for (hipStream_t q : side_) (void)hipStreamDestroy(q);
  for (hipEvent_t ev : side_done_) (void)hipEventDestroy(ev);
  if (fork_) (void)hipEventDestroy(fork_);
}

int Engine::init(std::string &err) {
  if (hipSetDevice(device_) != hipSuccess) {
    err = "hipSetDevice failed";
    return MB_ERR_HIP;
  }
  if (variant_ != MB_VARIANT_PLAIN) {
    if (!block_supported(block_) || halo_ < 1 || 2 * halo_ >= block_) {
      err = "blocked variant needs block in {64,128,192,256,512} and 1 <= depth < block/2";
      return MB_ERR_ARG;
    }
    if (lanes_ != 0 && lanes_ != 1 && lanes_ != 2 && lanes_ != 4 && lanes_ != 8) {
      err = "lanes must be 0, 1, 2, 4 or 8";
      return MB_ERR_ARG;
    }
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device_) == hipSuccess && prop.multiProcessorCount > 0)
    n_cu_ = prop.multiProcessorCount;
  if (const char *v = std::getenv("MB_PERSIST")) persist_ = std::string(v) != "0";
  // the work-queue form on request: on the 256-member sweep it is 15 % slower
  // than graph-replayed chunks, and the tuner's subset timing can favour it
  if (const char *v = std::getenv("MB_QUEUE")) queue_ = std::string(v) == "1";
  int clock_khz = 0;
  if (hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, device_) != hipSuccess || clock_khz <= 0)
    persist_ = false;
  spin_ticks_ = int64_t(clock_khz) * 1000 * 2;  // two seconds
  if (hipMalloc(&d_status_, kStatusSlots * sizeof(int32_t)) != hipSuccess) {
    err = "device allocation failed";
    return MB_ERR_OOM;
  }
  if (hipMemset(d_status_, 0, kStatusSlots * sizeof(int32_t)) != hipSuccess) {
    err = "device initialisation failed";
    return MB_ERR_HIP;
  }
  status_cap_ = kStatusSlots;
  for (int i = kStatusSlots - 1; i >= 0; --i) free_slots_.push_back(i);
  return MB_OK;
}

Engine::Group &Engine::group_for(int levels, bool strong, bool cayley, bool bk) {
  for (auto &g : groups_)
    if (g.levels == levels && g.strong == strong && g.cayley == cayley && g.bk == bk) return g;
  groups_.push_back(Group());
  groups_.back().levels = levels;
  groups_.back().strong = strong;
  groups_.back().cayley = cayley;
  groups_.back().bk = bk;
  return groups_.back();
}

int Engine::add(SimPlan &&plan, Arena *arena, hipStream_t st, std::string &err) {
  const bool plain = variant_ == MB_VARIANT_PLAIN;
  if (plain && plan.coupling == MB_COUPLING_STRONG) {
    err = "strong coupling runs on the blocked variant";
    return MB_ERR_UNSUPPORTED;
  }
  if (plain && precision_ != 64) {
    err = "the two-launch variant runs in FP64 only";
    return MB_ERR_UNSUPPORTED;
  }
  if (!plain && !shape_supported(plan.n, precision_, block_, 1)) {
    err = "no tile of " + std::to_string(block_) + " cells is built for " + std::to_string(plan.n) +
          " levels in this precision (5 and 6 levels: at most 256; 7 and 8 levels: 128 or 256)";
    return MB_ERR_UNSUPPORTED;
  }
  if (!plain && plan.n >= 7 && (plan.coupling == MB_COUPLING_STRONG || plan.field_step == MB_FIELD_CAYLEY)) {
    err = "7 and 8 levels run with weak coupling and the exact field step";
    return MB_ERR_UNSUPPORTED;
  }
  if (free_slots_.empty()) {
    err = "too many simulations in one engine";
    return MB_ERR_BUDGET;
  }
  Layout L = layout_of(plan, precision_, plain);
  char *block = nullptr;
  if (arena) {
    block = static_cast<char *>(arena->alloc(L.total));
    if (!block) {
      err = "serving budget exhausted";
      return MB_ERR_BUDGET;
    }
  } else if (hipMalloc(&block, L.total) != hipSuccess) {
    err = "device allocation failed";
    return MB_ERR_OOM;
  }
  auto s = std::make_unique<SimState>();
  s->plan = std::move(plan);
  SimPlan &p = s->plan;
  s->bytes = L.total;
  s->init_e = L.init_e;
  s->init_x = L.init_x;
  s->init_q = L.init_q;
  s->out_begin = L.end_head;
  s->block = block;
  s->own_block = arena == nullptr;
  // host image of everything before the record outputs
  std::vector<char> head(L.end_head, 0);
  if (precision_ == 64)
    fill_state<double>(p, head.data(), L);
  else
    fill_state<float>(p, head.data(), L);
  char *dev = s->block;
  std::memcpy(head.data() + L.mat_e, p.mat_e.data(), p.nx);
  std::memcpy(head.data() + L.mat_h, p.mat_h.data(), p.nx);
  DevSource *srcs = reinterpret_cast<DevSource *>(head.data() + L.src);
  for (size_t i = 0; i < p.sources.size(); ++i) {
    srcs[i].cell = p.sources[i].cell;
    srcs[i].hard = p.sources[i].hard;
    srcs[i].table = reinterpret_cast<const double *>(dev + L.tab_off[i]);
    std::memcpy(head.data() + L.tab_off[i], p.sources[i].table.data(), p.sources[i].table.size() * 8);
  }
  DevRecord *recs = reinterpret_cast<DevRecord *>(head.data() + L.rec);
  std::vector<std::vector<int32_t>> per_cell(L.n_point ? p.nx : 0);
  std::vector<int32_t> all_ids;
  for (size_t r = 0; r < p.records.size(); ++r) {
    const RecordPlan &rp = p.records[r];
    recs[r].quantity = rp.quantity;
    recs[r].whole = rp.cell < 0 ? 1 : 0;
    recs[r].cell = rp.cell;
    recs[r].interval = rp.interval;
    recs[r].out = reinterpret_cast<double *>(dev + L.out_off[r]);
    recs[r].readout = rp.readout.empty() ? nullptr : reinterpret_cast<const double *>(dev + L.ro_off[r]);
    if (!rp.readout.empty()) std::memcpy(head.data() + L.ro_off[r], rp.readout.data(), rp.readout.size() * 8);
    if (rp.cell >= 0)
      per_cell[rp.cell].push_back(int32_t(r));
    else
      all_ids.push_back(int32_t(r));
    s->rec_off.push_back(L.out_off[r]);
  }
  if (L.n_point) {
    int32_t *first = reinterpret_cast<int32_t *>(head.data() + L.rec_first);
    DevRecord *cell_recs = reinterpret_cast<DevRecord *>(head.data() + L.rec_ids);
    int32_t k = 0;
    for (int64_t c = 0; c < p.nx; ++c) {
      first[c] = k;
      for (int32_t id : per_cell[c]) cell_recs[k++] = recs[id];
    }
    first[p.nx] = k;
  }
  std::memcpy(head.data() + L.rec_all, all_ids.data(), all_ids.size() * sizeof(int32_t));
  hipError_t he = hipMemcpyAsync(dev, head.data(), head.size(), hipMemcpyHostToDevice, st);
  if (he == hipSuccess && L.total > L.end_head)
    he = hipMemsetAsync(dev + L.end_head, 0, L.total - L.end_head, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (he != hipSuccess) {
    err = std::string("upload failed: ") + hipGetErrorString(he);
    if (arena) arena->release(s->block);
    else (void)hipFree(s->block);
    return MB_ERR_HIP;
  }
  const size_t rs = precision_ == 64 ? 8 : 4;
  const size_t nx = size_t(p.nx);
  DevSim &d = s->ds;
  d.nx = p.nx;
  d.n_steps = p.n_steps;
  d.n_src = int32_t(p.sources.size());
  d.edge_l = p.edge_l;
  d.edge_r = p.edge_r;
  d.kap_l = p.kap_l;
  d.kap_r = p.kap_r;
  d.load_g_l = p.load_g_l;
  d.load_d_l = p.load_d_l;
  d.load_g_r = p.load_g_r;
  d.load_d_r = p.load_d_r;
  d.h_scale = p.h_scale;
  d.e[0] = dev + L.e;
  d.e[1] = dev + L.e + nx * rs;
  d.h[0] = dev + L.h;
  d.h[1] = dev + L.h + nx * rs;
  d.x[0] = dev + L.x;
  d.x[1] = dev + L.x + size_t(state_planes(p.n, precision_)) * nx * rs;
  d.qs[0] = reinterpret_cast<double *>(dev + L.qs);
  d.qs[1] = p.coupling == MB_COUPLING_STRONG && p.n > 0 ? d.qs[0] + nx : d.qs[0];
  d.qtab = reinterpret_cast<const double *>(dev + L.qtab);
  d.p = dev + L.p;
  d.mat_e = reinterpret_cast<const uint8_t *>(dev + L.mat_e);
  d.mat_h = reinterpret_cast<const uint8_t *>(dev + L.mat_h);
  d.mtab = dev + L.mtab;
  d.src = reinterpret_cast<const DevSource *>(dev + L.src);
  d.rec = reinterpret_cast<const DevRecord *>(dev + L.rec);
  d.n_rec = int32_t(p.records.size());
  d.n_rec_all = int32_t(all_ids.size());
  int64_t g = 0;
  for (auto &rp : p.records) g = std::gcd(g, rp.interval);
  d.rec_every = int32_t(g > 0 ? g : 1);
  d.cayley = p.field_step == MB_FIELD_CAYLEY ? 1 : 0;
  d.rec_first = L.n_point ? reinterpret_cast<const int32_t *>(dev + L.rec_first) : nullptr;
  d.rec_cell = reinterpret_cast<const DevRecord *>(dev + L.rec_ids);
  d.rec_all = reinterpret_cast<const int32_t *>(dev + L.rec_all);
  s->status_slot = free_slots_.back();
  free_slots_.pop_back();
  hi_slot_ = std::max(hi_slot_, s->status_slot + 1);
  d.status = d_status_ + s->status_slot;
  int32_t zero = 0;
  (void)hipMemcpy(d.status, &zero, sizeof(zero), hipMemcpyHostToDevice);
  s->start = n0_;
  s->parity_off = parity_;
  d.start = s->start;
  d.parity_off = s->parity_off;
  s->active = true;
  int id = int(sims_.size());
  group_for(p.n, p.coupling == MB_COUPLING_STRONG && p.n > 0, p.field_step == MB_FIELD_CAYLEY && p.n > 0,
            p.block_form && p.n > 0)
      .members.push_back(id);
  sims_.push_back(std::move(s));
  dirty_ = true;
  ++version_;
  return id;
}

void Engine::remove(int id, Arena *arena) {
  SimState &s = *sims_[id];
  if (s.active) {
    for (auto &g : groups_) {
      auto it = std::find(g.members.begin(), g.members.end(), id);
      if (it != g.members.end()) g.members.erase(it);
    }
    s.active = false;
    dirty_ = true;
    ++version_;
  }
  if (s.block) {
    if (s.own_block)
      (void)hipFree(s.block);
    else if (arena)
      arena->release(s.block);
    s.block = nullptr;
  }
  if (s.status_slot >= 0) {
    free_slots_.push_back(s.status_slot);
    s.status_slot = -1;
  }
  s.plan.sources.clear();
}

// the group's simulation descriptors and tiles (T owned cells each, chained
// left/right within a simulation)
void Engine::build_tables(const Group &g, std::vector<DevSim> &hs, std::vector<DevTile> &ht) const {
  hs.clear();
  ht.clear();
  const bool plain = variant_ == MB_VARIANT_PLAIN;
  const int span = plain ? plain_block() : block_ - 2 * halo_;
  for (int id : g.members) {
    const SimState &s = *sims_[id];
    int32_t local = int32_t(hs.size());
    hs.push_back(s.ds);
    const int32_t first = int32_t(ht.size());
    for (int64_t c0 = 0; c0 < s.plan.nx; c0 += span) {
      const int32_t idx = int32_t(ht.size());
      ht.push_back(DevTile{local, int32_t(c0), idx > first ? idx - 1 : -1, -1});
      if (idx > first) ht[idx - 1].right = idx;
    }
  }
}

hipError_t Engine::upload_group(Group &g, hipStream_t st) {
  std::vector<DevSim> hs;
  std::vector<DevTile> ht;
  build_tables(g, hs, ht);
  if (int(hs.size()) > g.cap_sims) {
    if (g.d_sims) (void)hipFree(g.d_sims);
    g.cap_sims = std::max<int>(int(hs.size()), 2 * g.cap_sims);
    if (hipMalloc(&g.d_sims, size_t(g.cap_sims) * sizeof(DevSim)) != hipSuccess) return hipErrorOutOfMemory;
  }
  if (int(ht.size()) > g.cap_tiles) {
    if (g.d_tiles) (void)hipFree(g.d_tiles);
    if (g.d_flags) (void)hipFree(g.d_flags);
    g.d_flags = nullptr;
    g.cap_tiles = std::max<int>(int(ht.size()), 2 * g.cap_tiles);
    if (hipMalloc(&g.d_tiles, size_t(g.cap_tiles) * sizeof(DevTile)) != hipSuccess) return hipErrorOutOfMemory;
    if (hipMalloc(&g.d_flags, size_t(g.cap_tiles + 1) * sizeof(uint32_t)) != hipSuccess) return hipErrorOutOfMemory;
  }
  hipError_t e = hipSuccess;
  if (!hs.empty()) e = hipMemcpyAsync(g.d_sims, hs.data(), hs.size() * sizeof(DevSim), hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !ht.empty())
    e = hipMemcpyAsync(g.d_tiles, ht.data(), ht.size() * sizeof(DevTile), hipMemcpyHostToDevice, st);
  // every tile's flag at the epoch of the next persistent launch (earlier epochs count as finished)
  std::vector<uint32_t> hf(ht.size(), epoch_);
  if (e == hipSuccess && !hf.empty())
    e = hipMemcpyAsync(g.d_flags, hf.data(), hf.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  g.n_tiles = int(ht.size());
  return e;
}

hipError_t Engine::sync_tables(hipStream_t st) {
  if (!dirty_) return hipSuccess;
  for (auto &g : groups_) {
    hipError_t e = upload_group(g, st);
    if (e != hipSuccess) return e;
  }
  dirty_ = false;
  return hipSuccess;
}

int Engine::effective_lanes(int levels) const {
  for (auto &g : groups_)
    if (g.levels == levels && !g.strong) return group_lanes(g);
  return 1;
}

int Engine::group_lanes(const Group &g) const {
  if (g.strong) return 1;  // the strong-coupling field iteration runs in one wave per cell
  int want = lanes_;
  if (want == 0) {
    // enough waves for about two per SIMD (4 SIMDs per compute unit)
    const int64_t waves1 = int64_t(g.n_tiles) * (block_ / 64);
    const int64_t target = 8 * int64_t(n_cu_);
    want = waves1 * 8 <= target ? 8 : waves1 * 4 <= target ? 4 : waves1 * 2 <= target ? 2 : 1;
  }
  for (int l = want; l > 1; l /= 2)
    if (shape_supported(g.levels, precision_, block_, l)) return l;
  return 1;
}

hipError_t Engine::launch_group(Group &g, hipStream_t st, int k, int reps, int64_t step_off, int par_off) {
  const int lanes = variant_ == MB_VARIANT_PLAIN ? 1 : group_lanes(g);
  const int64_t n0 = n0_ + step_off;
  const int par0 = parity_ ^ (par_off & 1);
  for (int r = 0; r < reps; ++r) {
    hipError_t e;
    if (variant_ == MB_VARIANT_PLAIN) {
      for (int s = 0; s < k; ++s) {
        const int64_t step = n0 + int64_t(r) * k + s;
        if ((e = launch_plain(g.levels, g.bk, g.d_sims, g.d_tiles, g.n_tiles, step, int((par0 + r * k + s) & 1), st)) !=
            hipSuccess)
          return e;
      }
    } else if ((e = launch_blocked(g.levels, precision_, block_, lanes, vc_, g.strong, g.cayley, g.bk, g.d_sims, g.d_tiles, g.n_tiles,
                                   n0 + int64_t(r) * k, par0 ^ (r & 1), halo_, k, ChunkSync{nullptr, 0u, 1, 0},
                                   st)) != hipSuccess) {
      return e;
    }
  }
  return hipSuccess;
}

bool Engine::persist_ok(int k, int64_t reps) { return persist_form(k, reps) != 0; }

int Engine::persist_form(int k, int64_t reps) { return flags_ok(k, reps) ? 1 : queue_ok(k, reps) ? 2 : 0; }

bool Engine::queue_ok(int k, int64_t reps) {
  if (!persist_ || !queue_ || variant_ == MB_VARIANT_PLAIN || reps < 2 || k != halo_ || 3 * halo_ > block_ || dirty_)
    return false;
  const Group *two = nullptr, *three = nullptr;
  for (auto &g : groups_) {
    if (g.members.empty()) continue;
    if (g.strong || g.cayley || (g.levels != 2 && g.levels != 3) || group_lanes(g) != 1 || !g.d_flags) return false;
    const Group *&slot = g.levels == 2 ? two : three;
    if (slot) return false;
    slot = &g;
  }
  if (!two && !three) return false;
  if (two && three && two->bk != three->bk) return false;
  const bool bk = two ? two->bk : three->bk;
  if (q_block_ != block_ || q_vc_ != int(vc_) || q_bk_ != int(bk)) {
    q_block_ = block_;
    q_vc_ = int(vc_);
    q_bk_ = int(bk);
    q_per_cu_ = queue_tiles_per_cu(precision_, block_, vc_, bk);
  }
  return q_per_cu_ > 0;
}

hipError_t Engine::run_queue(hipStream_t st, int k, int64_t reps) {
  Group *two = nullptr, *three = nullptr;
  for (auto &g : groups_)
    if (!g.members.empty()) (g.levels == 2 ? two : three) = &g;
  Group *first = two ? two : three;
  const int64_t per_chunk = int64_t(two ? two->n_tiles : 0) + int64_t(three ? three->n_tiles : 0);
  // items of one launch stay below 2^31
  const int64_t cap = std::max<int64_t>(1, std::min<int64_t>(kMaxPersistChunks, (int64_t(1) << 31) / std::max<int64_t>(1, per_chunk)));
  const int grid = int(std::min<int64_t>(int64_t(q_per_cu_) * n_cu_, per_chunk * std::min<int64_t>(reps, cap)));
  hipError_t e = hipSuccess;
  while (reps > 0 && e == hipSuccess) {
    const int n = int(std::min<int64_t>(reps, cap));
    QueueArgs qa{};
    qa.sims[0] = two ? two->d_sims : nullptr;
    qa.tiles[0] = two ? two->d_tiles : nullptr;
    qa.flags[0] = two ? two->d_flags : nullptr;
    qa.n_tiles[0] = two ? two->n_tiles : 0;
    qa.sims[1] = three ? three->d_sims : nullptr;
    qa.tiles[1] = three ? three->d_tiles : nullptr;
    qa.flags[1] = three ? three->d_flags : nullptr;
    qa.n_tiles[1] = three ? three->n_tiles : 0;
    qa.counter = first->d_flags + first->n_tiles;
    qa.epoch = epoch_;
    qa.n_chunks = n;
    qa.spin_ticks = spin_ticks_;
    e = fill_u32(qa.counter, 1, 0u, st);
    if (e == hipSuccess)
      e = launch_queue(precision_, block_, vc_, first->bk, grid, qa, n0_, parity_, halo_, k, st);
    if (e != hipSuccess) return e;
    epoch_ += uint32_t(n);
    for (int r = 0; r < n; ++r) commit_chunk(k);
    reps -= n;
  }
  return e;
}

bool Engine::flags_ok(int k, int64_t reps) {
  if (!persist_ || variant_ == MB_VARIANT_PLAIN || reps < 2 || k != halo_ || 3 * halo_ > block_ || dirty_)
    return false;
  Group *live = nullptr;
  for (auto &g : groups_) {
    if (g.members.empty()) continue;
    if (live) return false;  // groups of different kernels overlap on side streams
    live = &g;
  }
  if (!live || live->n_tiles < 1 || !live->d_flags) return false;
  const int lanes = group_lanes(*live);
  if (live->occ_block != block_ || live->occ_lanes != lanes) {
    live->occ_block = block_;
    live->occ_lanes = lanes;
    live->occ_per_cu = blocked_tiles_per_cu(live->levels, precision_, block_, lanes, vc_, live->strong, live->cayley,
                                            live->bk);
  }
  return int64_t(live->n_tiles) <= int64_t(live->occ_per_cu) * n_cu_;
}

hipError_t Engine::run_persistent(hipStream_t st, int k, int64_t reps) {
  hipError_t e = sync_tables(st);
  if (e != hipSuccess) return e;
  const int form = persist_form(k, reps);
  if (form == 2) return run_queue(st, k, reps);
  if (form != 1) return hipErrorInvalidValue;
  Group *g = nullptr;
  for (auto &q : groups_)
    if (!q.members.empty()) g = &q;
  const int lanes = group_lanes(*g);
  while (reps > 0) {
    const int n = int(std::min<int64_t>(reps, kMaxPersistChunks));
    const ChunkSync cs{g->d_flags, epoch_, n, spin_ticks_};
    e = launch_blocked(g->levels, precision_, block_, lanes, vc_, g->strong, g->cayley, g->bk, g->d_sims, g->d_tiles, g->n_tiles, n0_,
                       parity_, halo_, k, cs, st);
    if (e != hipSuccess) return e;
    epoch_ += uint32_t(n);
    for (int r = 0; r < n; ++r) commit_chunk(k);
    reps -= n;
  }
  return hipSuccess;
}

namespace {
struct TableSpan {
  size_t sims, tiles, flags, end;
};
TableSpan table_span(size_t at, size_t n_sims, size_t n_tiles) {
  TableSpan t;
  t.sims = align_up(at);
  t.tiles = align_up(t.sims + n_sims * sizeof(DevSim));
  t.flags = align_up(t.tiles + n_tiles * sizeof(DevTile));
  t.end = t.flags + (n_tiles + 1) * sizeof(uint32_t);  // flags and the work-queue counter
  return t;
}
}  // namespace

size_t Engine::table_bytes() const {
  size_t at = 0;
  std::vector<DevSim> hs;
  std::vector<DevTile> ht;
  for (const auto &g : groups_) {
    if (g.members.empty()) continue;
    build_tables(g, hs, ht);
    at = table_span(at, hs.size(), ht.size()).end;
  }
  return at;
}

hipError_t Engine::run_in_tables(hipStream_t st, int64_t steps, char *base, size_t bytes, int &rc,
                                 std::string &err) {
  rc = MB_OK;
  const size_t need = table_bytes();
  if (need > bytes) {
    rc = MB_ERR_BUDGET;
    err = "the run's group tables need " + std::to_string(need) + " bytes; the static scratch holds " +
          std::to_string(bytes);
    return hipSuccess;
  }
  struct Saved {
    Group *g;
    DevSim *sims;
    DevTile *tiles;
    uint32_t *flags;
    int n_tiles;
  };
  std::vector<Saved> saved;
  hipError_t e = hipSuccess;
  size_t at = 0;
  // host images of every group's tables, alive until the copies completed
  std::vector<std::vector<DevSim>> hsims;
  std::vector<std::vector<DevTile>> htiles;
  for (auto &g : groups_) {
    if (g.members.empty()) continue;
    hsims.emplace_back();
    htiles.emplace_back();
    std::vector<DevSim> &hs = hsims.back();
    std::vector<DevTile> &ht = htiles.back();
    build_tables(g, hs, ht);
    const TableSpan t = table_span(at, hs.size(), ht.size());
    at = t.end;
    saved.push_back(Saved{&g, g.d_sims, g.d_tiles, g.d_flags, g.n_tiles});
    g.d_sims = reinterpret_cast<DevSim *>(base + t.sims);
    g.d_tiles = reinterpret_cast<DevTile *>(base + t.tiles);
    g.d_flags = reinterpret_cast<uint32_t *>(base + t.flags);
    g.n_tiles = int(ht.size());
    if (e == hipSuccess && !hs.empty())
      e = hipMemcpyAsync(g.d_sims, hs.data(), hs.size() * sizeof(DevSim), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !ht.empty())
      e = hipMemcpyAsync(g.d_tiles, ht.data(), ht.size() * sizeof(DevTile), hipMemcpyHostToDevice, st);
    // every tile's flag at the epoch of the next persistent launch (the
    // scratch keeps whatever the last run on this GPU left there)
    if (e == hipSuccess) e = fill_u32(g.d_flags, ht.size(), epoch_, st);
  }
  // the host vectors are copied before they go out of scope
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) {
    dirty_ = false;
    const int k = variant_ == MB_VARIANT_PLAIN ? 1 : chunk_steps();
    if (variant_ != MB_VARIANT_PLAIN && persist_ok(k, steps / k)) {
      e = run_persistent(st, k, steps / k);
      steps %= k;
    }
    while (e == hipSuccess && steps > 0) {
      const int kk = int(std::min<int64_t>(k, steps));
      e = launch_only(st, kk);
      if (e == hipSuccess) commit_chunk(kk);
      steps -= kk;
    }
  }
  // the engine's own tables are rebuilt at its next ordinary run
  for (const Saved &sv : saved) {
    sv.g->d_sims = sv.sims;
    sv.g->d_tiles = sv.tiles;
    sv.g->d_flags = sv.flags;
    sv.g->n_tiles = sv.n_tiles;
  }
  dirty_ = true;
  return e;
}

hipError_t Engine::launch_only(hipStream_t st, int k, int reps, int64_t step_off, int par_off) {
  std::vector<Group *> live;
  for (auto &g : groups_)
    if (!g.members.empty()) live.push_back(&g);
  if (live.empty()) return hipSuccess;
  if (live.size() == 1) return launch_group(*live[0], st, k, reps, step_off, par_off);
  hipError_t e = hipSuccess;
  if (!fork_) e = hipEventCreateWithFlags(&fork_, hipEventDisableTiming);
  while (e == hipSuccess && side_.size() + 1 < live.size()) {
    hipStream_t q;
    hipEvent_t ev;
    if ((e = hipStreamCreateWithFlags(&q, hipStreamNonBlocking)) != hipSuccess) break;
    side_.push_back(q);
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) break;
    side_done_.push_back(ev);
  }
  if (e != hipSuccess) return e;
  if ((e = hipEventRecord(fork_, st)) != hipSuccess) return e;
  for (size_t i = 1; i < live.size() && e == hipSuccess; ++i) {
    e = hipStreamWaitEvent(side_[i - 1], fork_, 0);
    if (e == hipSuccess) e = launch_group(*live[i], side_[i - 1], k, reps, step_off, par_off);
    if (e == hipSuccess) e = hipEventRecord(side_done_[i - 1], side_[i - 1]);
  }
  if (e == hipSuccess) e = launch_group(*live[0], st, k, reps, step_off, par_off);
  // join every side stream that was forked, also after a failed launch
  for (size_t i = 1; i < live.size(); ++i) {
    hipError_t e2 = hipStreamWaitEvent(st, side_done_[i - 1], 0);
    if (e == hipSuccess) e = e2;
  }
  return e;
}

hipError_t Engine::reset(hipStream_t st) {
  n0_ = 0;
  parity_ = 0;
  cell_updates_ = 0;
  const size_t rs = precision_ == 64 ? 8 : 4;
  for (auto &sp : sims_) {
    SimState &s = *sp;
    if (!s.active || !s.block) continue;
    const size_t nx = size_t(s.plan.nx), m = size_t(s.plan.m);
    hipError_t e = hipSuccess;
    for (int b = 0; b < 2 && e == hipSuccess; ++b) {
      e = hipMemcpyAsync(s.ds.e[b], s.block + s.init_e, nx * rs, hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess) e = hipMemsetAsync(s.ds.h[b], 0, nx * rs, st);
      if (e == hipSuccess && m)
        e = hipMemcpyAsync(s.ds.x[b], s.block + s.init_x, m * nx * rs, hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess && m && precision_ == 32)  // the compensation planes start at zero
        e = hipMemsetAsync(static_cast<char *>(s.ds.x[b]) + m * nx * rs, 0, m * nx * rs, st);
      if (e == hipSuccess && s.plan.coupling == MB_COUPLING_STRONG && m)
        e = hipMemcpyAsync(s.ds.qs[b], s.block + s.init_q, nx * sizeof(double), hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess && s.plan.coupling == MB_COUPLING_STRONG && m)
        e = hipMemsetAsync(s.ds.qs[b] + 2 * nx, 0, nx * sizeof(double), st);
    }
    if (e == hipSuccess && s.bytes > s.out_begin) e = hipMemsetAsync(s.block + s.out_begin, 0, s.bytes - s.out_begin, st);
    if (e == hipSuccess) e = hipMemsetAsync(s.ds.status, 0, sizeof(int32_t), st);
    if (e != hipSuccess) return e;
    s.start = 0;
    s.parity_off = 0;
    s.ds.start = 0;
    s.ds.parity_off = 0;
    s.done = 0;
    s.cur_e = s.cur_h = s.cur_x = 0;
  }
  dirty_ = true;
  return sync_tables(st);
}

void Engine::commit_chunk(int k) {
  const bool plain = variant_ == MB_VARIANT_PLAIN;
  const int sub = plain ? k : 1;          // parity flips per launch
  const int per = plain ? 1 : k;          // steps per launch
  for (int q = 0; q < sub; ++q) {
    for (auto &sp : sims_) {
      SimState &s = *sp;
      if (!s.active) continue;
      int64_t ls = n0_ - s.start;
      if (ls < 0 || ls >= s.plan.n_steps) continue;
      int64_t ks = std::min<int64_t>(per, s.plan.n_steps - ls);
      s.done += ks;
      cell_updates_ += double(ks) * double(s.plan.nx);
      int par = parity_ ^ s.parity_off;
      if (plain) {
        s.cur_e = par ^ 1;
        s.cur_h = 0;
        s.cur_x = 0;
      } else {
        s.cur_e = s.cur_h = s.cur_x = par ^ 1;
      }
    }
    n0_ += per;
    parity_ ^= 1;
  }
}

hipError_t Engine::chunk(hipStream_t st, int k, int reps) {
  if (variant_ != MB_VARIANT_PLAIN && (k < 1 || k > halo_)) return hipErrorInvalidValue;
  if (reps < 1) return hipErrorInvalidValue;
  hipError_t e = sync_tables(st);
  if (e != hipSuccess) return e;
  e = launch_only(st, k, reps);
  if (e != hipSuccess) return e;
  for (int r = 0; r < reps; ++r) commit_chunk(k);
  return hipSuccess;
}

bool Engine::finished(int id) const {
  const SimState &s = *sims_[id];
  return s.done >= s.plan.n_steps;
}

bool Engine::all_finished() const {
  for (auto &s : sims_)
    if (s->active && s->done < s->plan.n_steps) return false;
  return true;
}

hipError_t Engine::enqueue_status(hipStream_t st, int32_t *host) {
  if (hi_slot_ == 0) return hipSuccess;
  return hipMemcpyAsync(host, d_status_, size_t(hi_slot_) * sizeof(int32_t), hipMemcpyDeviceToHost, st);
}

int Engine::reshape(int block, int halo, int lanes, std::string &err) {
  if (variant_ == MB_VARIANT_PLAIN) return MB_OK;
  if (!block_supported(block) || halo < 1 || 2 * halo >= block ||
      (lanes != 0 && lanes != 1 && lanes != 2 && lanes != 4 && lanes != 8)) {
    err = "bad tile shape";
    return MB_ERR_ARG;
  }
  if (block == block_ && halo == halo_ && lanes == lanes_) return MB_OK;
  block_ = block;
  halo_ = halo;
  lanes_ = lanes;
  dirty_ = true;
  ++version_;
  return MB_OK;
}

int64_t Engine::total_cells() const {
  int64_t c = 0;
  for (auto &s : sims_)
    if (s->active) c += s->plan.nx;
  return c;
}

hipError_t Engine::read_status(std::vector<int32_t> &out) {
  out.assign(status_cap_, 0);
  if (hi_slot_ == 0) return hipSuccess;
  return hipMemcpy(out.data(), d_status_, size_t(hi_slot_) * sizeof(int32_t), hipMemcpyDeviceToHost);
}

hipError_t Engine::read_records(int id, int rec, std::vector<double> &out) {
  SimState &s = *sims_[id];
  const RecordPlan &rp = s.plan.records[rec];
  int64_t avail = std::min<int64_t>(rp.n_samples, s.done / rp.interval);
  out.assign(size_t(avail) * size_t(rp.width), 0.0);
  if (out.empty()) return hipSuccess;
  return hipMemcpy(out.data(), s.block + s.rec_off[rec], out.size() * sizeof(double), hipMemcpyDeviceToHost);
}

hipError_t Engine::read_state(int id, double *e, double *h, double *rho) {
  SimState &s = *sims_[id];
  const SimPlan &p = s.plan;
  const size_t nx = size_t(p.nx), m = size_t(p.m);
  const bool f64 = precision_ == 64;
  auto fetch = [&](void *src, size_t count, std::vector<double> &dst) -> hipError_t {
    dst.resize(count);
    if (f64) return hipMemcpy(dst.data(), src, count * 8, hipMemcpyDeviceToHost);
    std::vector<float> tmp(count);
    hipError_t er = hipMemcpy(tmp.data(), src, count * 4, hipMemcpyDeviceToHost);
    for (size_t i = 0; i < count; ++i) dst[i] = tmp[i];
    return er;
  };
  std::vector<double> buf;
  hipError_t er;
  if (e) {
    if ((er = fetch(s.ds.e[s.cur_e], nx, buf)) != hipSuccess) return er;
    std::copy(buf.begin(), buf.end(), e);
  }
  if (h) {
    if ((er = fetch(s.ds.h[s.cur_h], nx, buf)) != hipSuccess) return er;
    for (size_t c = 0; c < nx; ++c) h[c] = buf[c] * p.h_scale;  // the kernels hold eta0 H
    if (nx) h[nx - 1] = 0.0;
  }
  if (rho) {
    const int n = p.n;
    std::fill(rho, rho + nx * n * n * 2, 0.0);
    if (n > 0) {
      // FP32: the entries and their compensation planes (the running sum lacks
      // the compensation: its value is entry - compensation)
      const size_t planes = size_t(state_planes(n, precision_));
      if ((er = fetch(s.ds.x[s.cur_x], planes * nx, buf)) != hipSuccess) return er;
      std::vector<double> sig(m);
      std::vector<cd> r(size_t(n) * n);
      for (size_t c = 0; c < nx; ++c) {
        const MaterialPlan &mp = p.mats[p.mat_e[c]];
        if (!mp.qm) continue;
        for (size_t a = 0; a < m; ++a) sig[a] = buf[a * nx + c] - (planes > m ? buf[(m + a) * nx + c] : 0.0);
        state_to_rho(mp, sig.data(), r.data());
        for (int q = 0; q < n * n; ++q) {
          rho[(c * n * n + q) * 2] = r[q].real();
          rho[(c * n * n + q) * 2 + 1] = r[q].imag();
        }
      }
    }
  }
  return hipSuccess;
}

}  // namespace mb
