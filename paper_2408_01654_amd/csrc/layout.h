// Layout of the symbolic analysis shared by the host planner and the kernels.
//
// A *tile* is a run of patches owned by one source frame i (all edges of a
// patch leave its owner frame, paper Sec. 3.1).  Its *slots* are the distinct
// target frames of those patches (a frame appears once per multiplicity of a
// duplicated (patch, frame) edge); the edges of the tile form a dense grid
// (patch, slot) whose cells hold the caller's edge index or -1.  The tile's
// *blocks* are the free poses it touches (its source if free, plus its free
// targets), sorted by pose index.  A tile writes the upper block pairs of its
// share of the reduced camera system into a private partial buffer, which is
// summed per global block in a fixed order.
#pragma once

#include <stdint.h>

namespace dpvba {

// Failure bits of a call's device work (see report_device_error), and the
// number of host-visible words (one per cause).
constexpr int kErrBarrier = 1;  // a grid barrier's bounded wait expired
constexpr int kErrChain = 2;    // a chained triangular solve's bounded wait expired
constexpr int kErrInput = 4;    // a non-finite target / weight or a negative weight
constexpr int kHostErrWords = 3;

constexpr int kMaxSlots = 64;     // slots per tile (one wavefront)
constexpr int kTileThreads = 256;      // float64 tile work and the depth write-back
constexpr int kTileThreadsWide = 512;  // float32 tile work

// Workgroup size of the tile kernel and of the single-launch solver for a
// compute type of tsize bytes (float64 keeps 256: its per-thread partials
// would not fit).  The solver's dense factor works on a 16 x 16 register
// grid of the first 256 threads; the others only meet its barriers.
__host__ __device__ constexpr int tile_threads(int tsize) { return tsize == 4 ? kTileThreadsWide : kTileThreads; }
constexpr int kRedWidth = 28;     // per-slot partial: 21 (M upper) + 6 (v) + 1 (cost)

struct TileInfo {
  int32_t frame;       // source frame i
  int32_t src_blk;     // local block of the source pose, -1 if held
  int32_t n_patch;     // patches in the tile
  int32_t n_slot;      // slots
  int32_t n_blk;       // free blocks
  int32_t max_mult;    // largest slot multiplicity of one frame (1 without duplicate edges)
  int32_t patch_begin; // into the tile-ordered patch arrays
  int32_t slot_begin;  // into slot_frame[] / slot_blk[]
  int32_t grid_begin;  // into edge_grid[] (n_patch * n_slot cells)
  int32_t blk_begin;   // into blk_pose[]
  int32_t part_begin;  // element offset of the partial block pairs (36 each)
  int32_t vec_begin;   // element offset of the partial vectors (rhs then diag, 6 * n_blk each)
  int32_t u_begin;     // element offset of the stored Schur rows (tile_u_rows x tile_u_stride)
  int32_t inst;        // problem of a batch the tile belongs to (0 for one problem)
  int32_t pad[2];
};

// Upper block pair (a <= b) of nb blocks, row-major over the upper triangle.
__host__ __device__ inline int upper_pair_index(int a, int b, int nb) {
  return a * nb - (a * (a - 1)) / 2 + (b - a);
}

__host__ __device__ inline int imax(int a, int b) { return a > b ? a : b; }

// Shared-memory plan of the tile kernel.  Compute-type (T) arrays: slot
// relative poses, patch rays (and, in float32 plans, both again in
// float64 for the residuals), per-patch sums, per-slot sums, and the
// Schur-row matrix U (K_pad x W_pad, rows = patches, columns = 6 n_blk
// block columns plus one column for w / sqrt(C~), padded for 16x16x4
// matrix-core tiles; rows 16-byte aligned), which first holds the
// wavefronts' per-slot partial sums.  Then a byte region of per-cell records (target,
// weight) that each lane overwrites with its edge's results, later reused
// for per-slot source blocks and their sums (and in phase 0 for the block
// step).  Then the block -> slot range tables.
struct TileLds {
  int slot, patch, hp, psum, m, u, total_T; // T offsets
  int K_pad, W_pad;
  int cell_bytes, rec_bytes;                // per cell, region
  int blk_s0, blk_s1, tables;               // byte offsets in the table region
};

__host__ __device__ inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Row stride of a tile's Schur-row matrix; the stored rows of a tile are
// the same K_pad x W_pad matrix (padding included), so they move as
// contiguous 16-byte vectors.
__host__ __device__ inline int tile_u_stride(int nb) { return round_up(6 * nb + 1, 16); }
__host__ __device__ inline int tile_u_rows(int K) { return round_up(K, 4); }

// Per-slot source blocks (Ad^T M, Ad^T M Ad, Ad^T v: 80 entries with
// padding) and, after them, their sums over the slots (36 + 6 + 6).
constexpr int kSlotBlk = 80;
constexpr int kSrcSums = 48;

// Entries of the B-term table of phase 3 after those sums: per block its
// diagonal block (36) and its source-row block (36), then the right-hand
// side and Diag(B) terms of each row (2 x 6 n_blk), then one zero.
__host__ __device__ inline int tile_bterm_entries(int nb) { return 72 * nb + 12 * nb + 1; }

// nthreads: the workgroup size (the per-thread partial sums of phase 1
// share the U region).  Host plans use tile_threads(tsize), never fewer
// than the single-launch solver's, so one allocation fits both kernels.
__host__ __device__ inline TileLds tile_lds_plan(int K, int Tn, int nb, int tsize, int nthreads) {
  TileLds L;
  L.K_pad = tile_u_rows(K);
  L.W_pad = tile_u_stride(nb);
  L.slot = 0;
  L.patch = L.slot + Tn * 18;
  // float32 plans: the slots' relative poses (12 doubles) and the patches'
  // rays (2 doubles) in float64, for the residuals
  L.hp = round_up(L.patch + K * 4, 4);
  L.psum = L.hp + (tsize == 4 ? Tn * 24 + K * 4 : 0);
  L.m = L.psum + K * 8;
  L.u = round_up(L.m + Tn * kRedWidth, 4);
  L.total_T = L.u + imax(L.K_pad * L.W_pad, (nthreads / 64) * Tn * kRedWidth);  // U, or the wavefronts' slot partials
  L.cell_bytes = imax(16, 8 * tsize);
  L.rec_bytes = imax(K * Tn * L.cell_bytes, imax(Tn * kSlotBlk + kSrcSums + tile_bterm_entries(nb), L.W_pad) * tsize);
  L.blk_s0 = 0;
  L.blk_s1 = L.blk_s0 + nb;
  L.tables = L.blk_s1 + nb;
  return L;
}

__host__ __device__ inline int align16(int b) { return (b + 15) / 16 * 16; }

__host__ __device__ inline int tile_lds_bytes(int K, int Tn, int nb, int tsize) {
  TileLds L = tile_lds_plan(K, Tn, nb, tsize, tile_threads(tsize));
  return align16(L.total_T * tsize) + align16(L.rec_bytes) + align16(L.tables);
}

// One problem of a batch: its ranges in the packed arrays and in the
// concatenated analysis (tiles, gather lists, solver scratch).
struct BatchInst {
  int32_t frame_begin, n_frames, n_fixed;
  int32_t free_begin;   // first free pose in the packed step vector (units of poses)
  int32_t n_free;
  int32_t patch_begin, n_patches;
  int32_t edge_begin, n_edges;
  int32_t tile_begin, n_tiles;
  int32_t s_base;       // its lower-block share lists start at s_off[s_base]
  int32_t v_base;       // its pose share lists start at v_off[v_base]
  int32_t pad;
  int64_t scratch_off;  // element offset of its packed float64 system in the scratch
};

// Largest system (n + 1 <= kSmallRows) handled by the single-launch solver,
// whose workgroup 0 factors it in registers (panel_chol_solve); larger
// systems take the separate dense solve.
constexpr int kSmallRows = 96;

// Row capacity 16 MB of the register-blocked dense solve of n unknowns
// (augmented with the right-hand side: n + 1 rows).
__host__ __device__ inline int small_solve_rows(int n) {
  const int n1 = n + 1;
  return n1 <= 32 ? 32 : (n1 <= 64 ? 64 : (n1 <= 80 ? 80 : 96));
}

// Shared memory of the one-workgroup dense solve (register-blocked panels):
// two published panels (2 x NR x 17), the reciprocal diagonal, the damped
// diagonal, the pivots, the factor's rows (NR x NR) and the step.
__host__ __device__ inline int small_solve_lds_bytes(int n, int tsize) {
  const int nr = small_solve_rows(n);
  return (38 * nr + nr * nr) * tsize;
}

// Shared memory of the one-workgroup packed solve (small_chol_solve_kernel):
// four vectors (damped diagonal, 1 / L_jj, pivots, step) and the packed
// lower triangle with the right-hand side appended as row n.
__host__ __device__ inline int packed_solve_lds_bytes(int n, int tsize) {
  return (4 * n + (n + 1) * (n + 2) / 2) * tsize;
}

}  // namespace dpvba
