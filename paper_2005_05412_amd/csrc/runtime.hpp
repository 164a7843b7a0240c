// Host runtime: simulations resident on one GPU, grouped by level count,
// advanced chunk by chunk.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "engine.hpp"
#include "plan.hpp"

namespace mb {

// First-fit allocator over one device allocation (no hipMalloc/hipFree on
// the serving path, which would synchronise the device).
class Arena {
 public:
  Arena() = default;
  ~Arena();
  int init(size_t bytes, std::string &err);
  // sub-allocates from caller-owned device memory (never freed here); base
  // must be 256-byte aligned
  void init_external(void *base, size_t bytes);
  void *alloc(size_t bytes);
  void release(void *p);
  size_t capacity() const { return cap_; }
  size_t used() const { return used_; }

 private:
  char *base_ = nullptr;
  bool own_ = true;
  size_t cap_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;  // offset -> size
  std::map<size_t, size_t> live_;  // offset -> size
};

struct SimState {
  SimPlan plan;
  size_t bytes = 0;
  char *block = nullptr;       // device memory of this simulation
  bool own_block = false;      // hipMalloc'ed by the engine
  DevSim ds{};
  int64_t start = 0;           // engine step of the simulation's step 0
  int parity_off = 0;
  int cur_e = 0, cur_h = 0, cur_x = 0;  // buffers holding the current state
  int64_t done = 0;            // steps completed (host mirror)
  std::vector<size_t> rec_off; // device offsets of record outputs inside block
  size_t init_e = 0, init_x = 0, init_q = 0, out_begin = 0;  // initial-state images, start of outputs
  bool active = false;
  int status_slot = -1;
};

// Bytes of device memory one simulation needs at a given precision.
size_t sim_bytes(const SimPlan &p, int precision, bool plain);

class Engine {
 public:
  // vc: keep the quantum coefficients of single-material waves in registers;
  // lanes: waves per 64 cells sharing each cell's density update (1, 2, 4, 8;
  // a level count without a kernel for that many uses the next smaller), or
  // 0 to choose per launch from the group's size (more waves per cell while
  // the group has too few tiles to fill the GPU)
  Engine(int device, int precision, int variant, int block, int halo, bool vc = false, int lanes = 1);
  ~Engine();
  int init(std::string &err);

  // Uploads a planned simulation; memory from `arena` when given, else
  // hipMalloc.  Returns the simulation id (>= 0) or a negative error.
  int add(SimPlan &&plan, Arena *arena, hipStream_t st, std::string &err);
  // Frees the simulation's device memory (after its last chunk completed).
  void remove(int id, Arena *arena);

  // Advances every active simulation by reps chunks of up to k steps each
  // (k <= depth for the blocked variant, any k for the two-launch variant).
  // Asynchronous.
  hipError_t chunk(hipStream_t st, int k, int reps = 1);
  // Uploads group tables if membership changed (synchronous copy).
  hipError_t sync_tables(hipStream_t st);

  // Whether reps chunks of k steps can run as persistent launches (k equal to
  // the halo, not switched off by MB_PERSIST=0): one group whose tiles are all
  // resident at once (neighbour flags, each tile runs every chunk), or else
  // a two-level and/or a three-level group of weak coupling and the exact
  // field step with one wave per 64 cells on a tile with a work-queue kernel
  // (with MB_QUEUE=1 set at set-up).  Tables must be current.
  bool persist_ok(int k, int64_t reps);
  // reps chunks of k steps as persistent launches (at most kMaxPersistChunks
  // chunks each); asynchronous, not capturable into graphs
  hipError_t run_persistent(hipStream_t st, int k, int64_t reps);
  // the form persist_ok found: 1 neighbour flags, 2 work queue, 0 none
  int persist_form(int k, int64_t reps);
  // allows (on) or forbids persistent launches (MB_PERSIST=0 forbids them regardless)
  void set_persist(bool on) { persist_ = persist_ && on; }
  static constexpr int kMaxPersistChunks = 4096;

  // Launches of reps chunks of k steps, for graph capture: tables must be
  // current.  Groups of different level counts run on their own streams,
  // forked from and joined back into st, so their kernels overlap.  The first
  // launch starts step_off steps and par_off buffer flips after the engine's
  // committed step (chunks captured ahead of their commit_chunk calls).
  hipError_t launch_only(hipStream_t st, int k, int reps = 1, int64_t step_off = 0, int par_off = 0);
  void commit_chunk(int k);  // host bookkeeping of a chunk launched via launch_only
  // Restores every simulation's initial state from its device image and
  // clears records (asynchronous copies on st, then table upload).
  hipError_t reset(hipStream_t st);
  // Changes whenever tables or the step origin change (graph cache key).
  int64_t version() const { return version_; }

  bool finished(int id) const;
  bool all_finished() const;
  int64_t engine_step() const { return n0_; }
  int depth() const { return halo_; }
  // steps per blocked launch: the halo width, at most 256
  int chunk_steps() const { return halo_ < 256 ? halo_ : 256; }
  int block() const { return block_; }
  int lanes() const { return lanes_; }
  // waves per 64 cells the next launch of the group of this level count uses
  int effective_lanes(int levels) const;
  bool vc() const { return vc_; }
  int variant() const { return variant_; }
  int precision() const { return precision_; }
  SimState &sim(int id) { return *sims_[id]; }
  const SimState &sim(int id) const { return *sims_[id]; }
  int n_sims() const { return int(sims_.size()); }
  // copies the status flags of all simulations to the host (synchronous)
  hipError_t read_status(std::vector<int32_t> &out);
  // enqueues the copy of the status flags in use into `host` (pinned, at
  // least kMaxStatusSlots entries) on st
  hipError_t enqueue_status(hipStream_t st, int32_t *host);
  static constexpr int kMaxStatusSlots = 4096;
  // new tile shape for the following launches (tables are rebuilt at the next
  // chunk); only between chunks
  int reshape(int block, int halo, int lanes, std::string &err);
  int64_t total_cells() const;
  // Runs `steps` steps like chunk()/run_persistent() -- persistent launches
  // when the tiles fit, else one launch per chunk -- with the group tables
  // (simulation descriptors, tiles, neighbour flags) written into the device
  // region [base, base + bytes) instead of the engine's own table buffers:
  // nothing is allocated or freed.  The region is rewritten by every such run
  // (table_bytes() of it).  rc: MB_OK, or MB_ERR_BUDGET when the tables do not fit.
  hipError_t run_in_tables(hipStream_t st, int64_t steps, char *base, size_t bytes, int &rc, std::string &err);
  size_t table_bytes() const;
  hipError_t read_records(int id, int rec, std::vector<double> &out);
  hipError_t read_state(int id, double *e, double *h, double *rho);
  double cell_updates() const { return cell_updates_; }

 private:
  struct Group {
    int levels = 0;
    bool strong = false;  // strong-coupling simulations (their own kernel)
    bool cayley = false;  // Cayley field step (their own kernel)
    bool bk = false;      // density tables in the block form (their own kernel)
    std::vector<int> members;
    DevSim *d_sims = nullptr;
    DevTile *d_tiles = nullptr;
    // per tile: epoch of the last finished chunk (persistent launches), then
    // one more word: the item counter of a work-queue launch
    uint32_t *d_flags = nullptr;
    int n_tiles = 0, cap_sims = 0, cap_tiles = 0;
    int occ_block = 0, occ_lanes = 0, occ_per_cu = 0;  // cached occupancy of the group's kernel
  };
  Group &group_for(int levels, bool strong, bool cayley, bool bk);
  hipError_t upload_group(Group &g, hipStream_t st);
  void build_tables(const Group &g, std::vector<DevSim> &hs, std::vector<DevTile> &ht) const;
  hipError_t launch_group(Group &g, hipStream_t st, int k, int reps, int64_t step_off = 0, int par_off = 0);
  int group_lanes(const Group &g) const;
  bool flags_ok(int k, int64_t reps);
  bool queue_ok(int k, int64_t reps);
  hipError_t run_queue(hipStream_t st, int k, int64_t reps);

  int device_, precision_, variant_, block_, halo_;
  bool vc_ = false;
  int lanes_ = 1;
  int n_cu_ = 256;
  std::vector<std::unique_ptr<SimState>> sims_;
  std::vector<Group> groups_;
  // one stream and completion event per group beyond the first, plus the fork event
  std::vector<hipStream_t> side_;
  std::vector<hipEvent_t> side_done_;
  hipEvent_t fork_ = nullptr;
  bool dirty_ = true;
  int64_t version_ = 0;
  int32_t *d_status_ = nullptr;
  int status_cap_ = 0;
  int hi_slot_ = 0;  // status slots in use lie below this index
  std::vector<int> free_slots_;
  int64_t n0_ = 0;
  int parity_ = 0;
  bool persist_ = true;        // persistent launches allowed
  bool queue_ = false;         // work-queue persistent launches allowed (MB_QUEUE=1)
  int q_block_ = 0, q_vc_ = -1, q_bk_ = -1, q_per_cu_ = 0;  // cached occupancy of the work-queue kernel
  uint32_t epoch_ = 0;         // chunk epoch of the next persistent launch
  int64_t spin_ticks_ = 0;     // device wall-clock ticks of a neighbour wait before giving up
  double cell_updates_ = 0;
};

// false when MB_GRAPHS=0 is set in the environment: runs and the tuner launch
// chunks directly instead of capturing them into HIP graphs (for tools that do
// not follow graph launches)
bool graphs_enabled();

// default tile shape per level count and precision
void default_shape(int levels, int precision, int &block, int &halo);

}  // namespace mb
