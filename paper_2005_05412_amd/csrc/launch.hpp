// Host-side launchers of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "engine.hpp"

namespace mb {

bool block_supported(int block);
// whether the blocked kernel is built for this tile (block cells, lanes wave
// groups per 64 cells: 1, 2 or 4) at this level count and precision
bool shape_supported(int levels, int precision, int block, int lanes);
// whether that tile is also built with register-resident coefficients (a run
// that asks for them on another shape uses scalar coefficient loads)
bool regs_supported(int levels, int precision, int block, int lanes);
int plain_block();

// Temporally blocked launch from engine step n0 with buffer parity `parity`:
// k <= halo steps for every tile; 2*halo < block.  Tiles of `block` cells,
// block*lanes threads.
// vc: quantum coefficients of single-material waves held in registers
// (used for 2 and 3 levels, ignored otherwise).
// strong: strong-coupling simulations (one wave per 64 cells; register
// coefficients only on three-level FP32 tiles of 256 cells)
// cayley: simulations with the Cayley field step (persistent launches with
// one wave per 64 cells only)
// bk: simulations whose density tables are in the block form (engine.hpp)
// cs.n_chunks > 1: a persistent launch of that many chunks of k = halo steps
// (3*halo <= block, cs.flags per tile); all n_tiles tiles must fit on the
// device at once (blocked_tiles_per_cu); cs.n_chunks == 1: one chunk, no flags.
hipError_t launch_blocked(int levels, int precision, int block, int lanes, bool vc, bool strong, bool cayley, bool bk,
                          const DevSim *sims, const DevTile *tiles, int n_tiles, int64_t n0, int parity,
                          int halo, int k, const ChunkSync &cs, hipStream_t st);
// tiles of this shape one compute unit holds at once (0: no such kernel)
int blocked_tiles_per_cu(int levels, int precision, int block, int lanes, bool vc, bool strong, bool cayley, bool bk);
// One time step as two launches (FP64); tiles of plain_block() cells.
hipError_t launch_plain(int levels, bool bk, const DevSim *sims, const DevTile *tiles, int n_tiles,
                        int64_t n0, int parity, hipStream_t st);

// Work-queue persistent launch of a two- and a three-level group (QueueArgs,
// either group may be empty) with `grid` workgroups: one chunk of k = halo
// steps per item, 3*halo <= block, one wave per 64 cells; FP32 tiles of 128,
// 192 or 256 cells, FP64 of 128 or 256.  qa.counter must read zero.
hipError_t launch_queue(int precision, int block, bool vc, bool bk, int grid, const QueueArgs &qa, int64_t n0,
                        int parity, int halo, int k, hipStream_t st);
// workgroups of the work-queue kernel one compute unit holds at once (0: none built)
int queue_tiles_per_cu(int precision, int block, bool vc, bool bk);

}  // namespace mb
