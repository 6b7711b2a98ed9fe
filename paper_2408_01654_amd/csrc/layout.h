// Layout of the symbolic analysis shared by the host planner and the kernels.
//
// A *tile* is a run of patches owned by one source frame i (all edges of a
// patch leave its owner frame, paper Sec. 3.1).  Its *slots* are the distinct
// target frames of those patches; the edges of the tile form a dense grid
// (patch, slot) whose cells hold the caller's edge index or -1.  The tile's
// *blocks* are the free poses it touches (its source if free, plus its free
// targets), sorted by pose index; the tile writes the upper block pairs of its
// contribution to the reduced camera system into a private partial buffer,
// which a gather pass sums per global block in a fixed order.
#pragma once

#include <stdint.h>

namespace dpvba {

constexpr int kMaxSlots = 64;     // distinct target frames per tile
constexpr int kMaxBlocks = kMaxSlots + 1;
constexpr int kTileThreads = 256;
constexpr int kRedWidth = 28;     // per-slot partial: 21 (M upper) + 6 (v) + 1 (cost)

struct TileInfo {
  int32_t frame;       // source frame i
  int32_t src_blk;     // local block of the source pose, -1 if held
  int32_t n_patch;     // patches in the tile
  int32_t n_slot;      // target frames
  int32_t n_blk;       // free blocks
  int32_t patch_begin; // into tile_patch[]
  int32_t slot_begin;  // into slot_frame[] / slot_blk[]
  int32_t grid_begin;  // into edge_grid[] (n_patch * n_slot cells)
  int32_t blk_begin;   // into blk_pose[]
  int32_t part_begin;  // element offset of the partial block pairs (36 each)
  int32_t vec_begin;   // element offset of the partial vectors (rhs then diag, 6 * n_blk each)
  int32_t pad;
};

// Upper block pair (a <= b) of nb blocks, row-major over the upper triangle.
__host__ __device__ inline int upper_pair_index(int a, int b, int nb) {
  return a * nb - (a * (a - 1)) / 2 + (b - a);
}

}  // namespace dpvba

namespace dpvba {

// Shared-memory plan of the tile kernels, in elements of the compute type T
// followed by small byte tables; the host sizes the dynamic allocation with
// the same function.
struct TileLds {
  int slot, patch, cell, work, m, total_T;  // offsets / total in T elements
  int pair_a, pair_b, blk_s0, blk_s1, slot_blk, total_bytes_tables;
};

__host__ __device__ inline int imax(int a, int b) { return a > b ? a : b; }

__host__ __device__ inline TileLds tile_lds_plan(int K, int Tn, int nb) {
  TileLds L;
  const int npairs = nb * (nb + 1) / 2;
  L.slot = 0;
  L.patch = L.slot + Tn * 18;
  L.cell = L.patch + K * 4;
  L.work = L.cell + imax(K * Tn * 8, Tn * 80);
  L.m = L.work + imax(kTileThreads * kRedWidth, K * 6 * nb);
  L.total_T = L.m + Tn * kRedWidth;
  L.pair_a = 0;
  L.pair_b = L.pair_a + npairs;
  L.blk_s0 = L.pair_b + npairs;
  L.blk_s1 = L.blk_s0 + nb;
  L.slot_blk = L.blk_s1 + nb;
  L.total_bytes_tables = L.slot_blk + Tn;
  return L;
}

__host__ __device__ inline int tile_lds_bytes(int K, int Tn, int nb, int tsize) {
  TileLds L = tile_lds_plan(K, Tn, nb);
  return ((L.total_T * tsize + 15) / 16) * 16 + ((L.total_bytes_tables + 15) / 16) * 16;
}

}  // namespace dpvba
