// Arguments of the tile kernels and of the single-launch small-problem solver.
#pragma once

#include <hip/hip_runtime.h>

#include "layout.h"

namespace dpvba {

template <typename T>
struct IterArgs {
  const float* patches;
  int p;
  const float* target;
  const float* weight;
  T fx, fy, cx, cy, z_min;
  T lambda;                // additive damping: H~ = H + lam_diag Diag(H) + lambda I
  T lam_diag;              // lambda (Levenberg-Marquardt) or 0 (Levenberg)
  int n_frames, n_fixed, n_free, n_tiles;
  const T* poses_cur;      // [N,7] x_t
  T* poses_next;           // [N,7] x_{t+1} (written by the last workgroup)
  const T* depth_in;       // caller's inverse depths (read when first)
  T* depth_s;              // tile-ordered inverse depths
  T* xh_s;                 // tile-ordered patch rays [.,2]
  T* U_s;                  // stored Schur rows
  T* pscale_s;             // per patch: 1/sqrt(C~), w/sqrt(C~)
  const T* dx_prev;        // previous pose step (applied unless first)
  const int* status_prev;  // nonzero: previous step discarded (entry inst * status_stride)
  int status_stride;       // distance between the problems' status words (0: one problem)
  int first;
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
  // gather lists and per-iteration outputs of the small-problem solver
  const int* s_off;
  const int* s_src;
  const int* v_off;
  const int2* v_src;
  T* dx;
  int* status;
  unsigned int* min_bits;
  double* cost_out;
  int* invalid_out;
  int* dev_err;            // device failure word of the call (bit 4: invalid target / weight)
  int* host_err;           // host-visible sticky copy of the failure bits
  const int* order;        // one launch per pass: workgroup g runs tile order[g] (heaviest first), or g if null
};

// Arguments of the single-launch solver of small problems.
template <typename T>
struct SmallArgs {
  IterArgs<T> it;       // shared fields; per-iteration fields set in the kernel
  T* poses_io;          // caller's poses (read at t = 0, written at the end)
  T* depth_io;          // caller's inverse depths
  T* pbuf0;
  T* pbuf1;
  T* Sp;                // packed reduced system
  T* rhs;
  T* d0;
  int* status;          // per iteration
  unsigned int* min_bits;
  double* cost;         // per iteration, or null
  int* invalid;
  int n_iters;
  unsigned int* bar;       // this launch's grid-barrier slot (arrivals, generation)
  unsigned int* bar_next;  // the next launch's slot, cleared by this one
  int* err;                // this launch's failure word
  int* err_next;           // the next launch's failure word, cleared by this one
};

}  // namespace dpvba
