// Host-side launchers of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "engine.hpp"

namespace mb {

bool block_supported(int block);
int plain_block();

// Temporally blocked launch: k <= halo steps for every tile; 2*halo < block.
hipError_t launch_blocked(int levels, int precision, int block, const DevSim *sims,
                          const DevTile *tiles, int n_tiles, const DevClock *clk, int halo, int k,
                          hipStream_t st);
// One time step as two launches (FP64); tiles of plain_block() cells.
hipError_t launch_plain(int levels, const DevSim *sims, const DevTile *tiles, int n_tiles,
                        const DevClock *clk, hipStream_t st);
// clk->n0 += k, clk->parity ^= 1 (one thread).
hipError_t launch_advance(DevClock *clk, int k, hipStream_t st);

}  // namespace mb
