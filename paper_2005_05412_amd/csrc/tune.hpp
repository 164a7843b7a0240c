// Tile-shape autotuner of the blocked kernel.
#pragma once

#include <string>
#include <vector>

#include "runtime.hpp"

namespace mb {

struct Shape {
  int block = 256;  // cells per tile
  int halo = 32;    // halo width = steps per launch (capped at 256)
  bool vc = false;  // quantum coefficients in registers (2 and 3 levels)
  int lanes = 1;    // waves per 64 cells sharing each cell's density update
  bool persist = true;  // full chunks as persistent launches (when the tiles fit on the device)
};

std::vector<Shape> candidate_shapes(int levels, int precision);
std::string tune_key(int device, const std::vector<const SimPlan *> &plans, int precision);
// Picks the fastest candidate shape for these simulations (cached).
int tune_shape(int device, const std::vector<const SimPlan *> &plans, int precision, Shape &best,
               std::string &err);

}  // namespace mb
