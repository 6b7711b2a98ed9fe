// Arguments of the tile kernels (assembly and depth back-substitution).
#pragma once

#include "layout.h"

namespace dpvba {

template <typename T, typename P>
struct TileArgs {
  const P* poses;          // [N,7]
  P* inv_depth;            // [P] (back-substitution writes it)
  const float* patches;    // [P,p,p,2]
  int p;
  const float* target;     // [E,2]
  const float* weight;     // [E,2]
  T fx, fy, cx, cy, z_min, lambda;
  int n_fixed;
  const TileInfo* tiles;
  const int* tile_patch;
  const int* slot_frame;
  const int* slot_blk;
  const int* edge_grid;
  const int* blk_pose;
  T* part_S;
  T* part_vec;
  double* part_cost;
  int* part_invalid;
  const T* dx;             // [6 N'] pose step (back-substitution)
  const int* step_status;  // nonzero: discard this iteration's step
};

}  // namespace dpvba
