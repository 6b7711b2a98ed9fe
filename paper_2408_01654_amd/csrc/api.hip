// C ABI of the patch-graph Gauss-Newton BA library: context, symbolic
// analysis of the edge set, and orchestration of the numeric phases on the
// caller's stream.  See include/dpvba.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "dpvba.h"
#include "factor_plan.h"
#include "layout.h"
#include "tileargs.h"

namespace dpvba {

// kernels (tile.hip, assemble.hip, dense.hip)
template <typename T>
hipError_t launch_tile_iterate(const IterArgs<T>& A, int lds_bytes, hipStream_t st);
template <typename T>
hipError_t launch_tile_finalize(const TileInfo* tiles, int n_tiles, int lds_bytes, const int* tile_patch,
                                const int* blk_pose, const T* U_s, const T* pscale_s, const T* depth_s,
                                const T* dx, const int* status, int status_stride, T* depth_out,
                                const T* poses_final, T* poses_out, int n_frames, hipStream_t st);
template <typename T>
hipError_t launch_retract_copy(const T* poses_cur, T* poses_next, T* dx, int n_fixed, int n_frames,
                               const int* status, hipStream_t st, const T* dx_sys = nullptr, const int* pos = nullptr);
template <typename T>
int small_solve_grid(int lds_bytes);
template <typename T>
hipError_t launch_small_solve(const SmallArgs<T>& S, int grid, int lds_bytes, bool cooperative, hipStream_t st);
int small_solve_max_n(int tsize);
hipError_t launch_pgo_init(const double* poses, int n, double* sims, const double* loop_rel, int n_loops, double* C,
                           hipStream_t st);
hipError_t launch_pgo_linearise(const double* sims, const double* C, const int* ea, const int* eb, int n_edges,
                                double* r, double* J, double* cost, hipStream_t st);
hipError_t launch_pgo_normal(const double* J, const double* r, const int* blk_pq, const int* blk_off,
                             const int* blk_src, int n_blocks, const int* pose_off, const int* pose_src, int nf,
                             double lambda, double lam_diag, double* H, double* d0, double* rhs, hipStream_t st);
hipError_t launch_pgo_retract(double* sims, int n, int n_fixed, const double* dx, const int* status, hipStream_t st);
hipError_t launch_pgo_apply(const double* sims, int n, const int* patch_off, float* poses, float* inv_depth,
                            hipStream_t st);
template <typename T>
hipError_t launch_fill(T* x, long long n, T v, hipStream_t st);
hipError_t launch_patch_correlation(int n_edges, int p, int dim, const float* gmap, int n_patches, const float* fmaps,
                                    int n_maps, int H, int W, const int* kk, const int* jj, const float* coords,
                                    float* corr, int* dev_err, int* host_err, hipStream_t st);
hipError_t launch_proximity_edges(const float* poses, int n, const int* patch_off, int first_recent, int min_gap,
                                  float r2, int max_t, int* counts, int* targets, long long* edge_off, int* ii,
                                  int* jj, int* kk, long long max_edges, hipStream_t st);
template <typename T>
hipError_t launch_gather(const T* part_S, const T* part_vec, const int* s_off, const int* s_src,
                         const int* v_off, const int2* v_src, int n_free, T* S, T* rhs, T* dB, T lambda,
                         T lam_diag, int mirror, T* diag_out, hipStream_t st, const int* pos);
template <typename T>
hipError_t launch_gather_env(const T* part_S, const T* part_vec, const int* s_off, const int* s_src,
                             const int* v_off, const int2* v_src, int n_free, const int4* env, int n_env, T* S, T* rhs,
                             T* dB, T lambda, T lam_diag, T* diag_out, hipStream_t st, const int* pos);
template <typename TP, typename T>
hipError_t launch_gather_env_as(const TP* part_S, const TP* part_vec, const int* s_off, const int* s_src,
                                const int* v_off, const int2* v_src, int n_free, const int4* env, int n_env, T* S,
                                T* rhs, T* dB, T lambda, T lam_diag, T* diag_out, hipStream_t st, const int* pos,
                                int mirror);
template <typename T>
hipError_t launch_permute_blocks(const T* src, T* dst, const int* perm, int n_blk, int bw, int to_system,
                                 hipStream_t st);
template <typename T, typename P>
hipError_t launch_edge_cost(const P* poses, const P* inv_depth, const float* patches, int p, const int* ii,
                            const int* jj, const int* kk, const float* target, const float* weight,
                            int n_edges, T fx, T fy, T cx, T cy, T z_min, double* part, hipStream_t st);
hipError_t launch_report_reduce(const double* part_cost, const int* part_invalid, int n, double* cost_out,
                                int* invalid_out, hipStream_t st);
hipError_t launch_reproject(const float* poses, const float* inv_depth, const float* patches, int p,
                            const int* ii, const int* jj, const int* kk, int n_edges, float fx, float fy,
                            float cx, float cy, float z_min, float* coords, uint8_t* valid, hipStream_t st);
template <typename T>
hipError_t launch_chol_solve(T* S, const T* rhs, int n, T* dx, T* work_y, T* Linv_all, const T* d0, int* status,
                             unsigned int* min_bits, int* flags, int epoch, int* err, int* host_err, hipStream_t st,
                             bool cooperative = false, const PanelPlan* plan = nullptr);
hipError_t launch_report_init(int* status, unsigned int* min_bits, int n, hipStream_t st, int* err_clear = nullptr);
template <typename TP, typename T>
hipError_t launch_gather_as(const TP* part_S, const TP* part_vec, const int* s_off, const int* s_src,
                            const int* v_off, const int2* v_src, int n_free, T* S, T* rhs, T* dB, T lambda,
                            T lam_diag, int mirror, T* diag_out, hipStream_t st, const int* pos);
template <typename T>
hipError_t launch_chol_factor(T* S, int n, int nrows, T* Linv_all, const T* d0, int* status, unsigned int* min_bits,
                              hipStream_t st, const PanelPlan* plan);
template <typename T>
hipError_t launch_chol_apply(const T* L, int n, const T* Linv_all, const T* rhs, T* x, T* work_y, int* flags,
                             int epoch, int* err, int* host_err, hipStream_t st, int backward_only = 0,
                             bool cooperative = false, const PanelPlan* plan = nullptr, const int* skip = nullptr);
// mixed-precision helpers (mixed.hip)
template <typename Ti, typename To>
hipError_t launch_convert(const Ti* src, To* dst, long long n, hipStream_t st);
hipError_t launch_lower_to_f32(const double* S64, float* S32, int n, hipStream_t st,
                               const PanelPlan* env = nullptr);
hipError_t launch_residual64(const double* S, const double* s, const double* x, int n, double* r,
                             unsigned long long* maxes, hipStream_t st, const PanelPlan* env = nullptr);
hipError_t launch_accumulate(double* x, const float* c, int n, hipStream_t st, const int* skip = nullptr);
hipError_t launch_refine_check(const unsigned long long* maxes, double tol, int* skip, hipStream_t st);
hipError_t launch_refine_decide(const unsigned long long* maxes, const int* status32, double tol, int force,
                                double* resid_out, int* fallback_out, int* host_flag, hipStream_t st);
hipError_t launch_step_to_f32(const double* x, float* dx, int n, const int* fallback, const int* status64,
                              int* status, hipStream_t st);
// batch kernels (batch.hip)
template <typename TS>
struct BatchArgs {
  const BatchInst* inst;
  const TS* part_S;
  const TS* part_vec;
  const int* s_off;
  const int* s_src;
  const int* v_off;
  const int2* v_src;
  double lambda;
  double lam_diag;
  int n_refine;
  int force_fb;
  const TS* poses_cur;
  TS* poses_next;
  TS* dx;
  int* status;
  unsigned int* min_bits;
  double* refine_resid;
  int* fallback;
  int stride, it;
  double* scratch;
  int lds_factor;
};
template <typename T>
int batch_solve_lds(int n_max, bool mixed, bool* lds_factor);
template <typename T>
hipError_t launch_batch_solve(const BatchArgs<T>& a, int n_inst, int lds_bytes, hipStream_t st);
template <typename TS, typename TA>
hipError_t launch_batch_gather(const BatchArgs<TS>& a, int n_inst, int n_max, hipStream_t st);
hipError_t launch_batch_solve_mixed(const BatchArgs<float>& a, int n_inst, int lds_bytes, hipStream_t st);
hipError_t launch_batch_cost(const BatchInst* inst, int n_inst, const double* part_cost, const int* part_invalid,
                             dpvba_report* rep, int it, hipStream_t st);
template <typename T>
hipError_t launch_batch_report(const BatchInst* inst, int n_inst, const T* poses, const T* inv_depth,
                               const float* patches, int p, const int* ii, const int* jj, const int* kk,
                               const float* target, const float* weight, T fx, T fy, T cx, T cy, T z_min,
                               const int* status, const unsigned int* min_bits, const double* refine,
                               const int* fallback, int stride, int n_iters, dpvba_report* rep, hipStream_t st);
// adjoint kernels (adjoint.hip)
template <typename T>
hipError_t launch_edge_adjoint(const T* poses, const T* depth_t, const int* patch_pos, const float* patches, int p,
                               const int* ii, const int* jj, const int* kk, const float* target,
                               const float* weight, int n_edges, int n_fixed, T fx, T fy, T cx, T cy, T z_min,
                               T lambda, const T* u_pose, const T* u_depth, const T* dxi, const T* dd,
                               const int* status, T* grad_target, T* grad_weight, T* edge_xbar, hipStream_t st);
template <typename T>
hipError_t launch_retract_adjoint(const T* poses_t, const T* dxi, const int* status, int n_fixed, int n_frames,
                                  T* pbar, T* dxi_bar, hipStream_t st);
template <typename T>
hipError_t launch_adjoint_rhs(const TileInfo* tiles, int n_tiles, const T* U_s, const T* pscale_s, const T* dbar,
                              T* part_vec, const int* v_off, const int2* v_src, int n_free, const T* dxi_bar,
                              const int* status, T* rhs, hipStream_t st);
template <typename T>
hipError_t launch_adjoint_backsub(const TileInfo* tiles, int n_tiles, int max_w6, const int* blk_pose,
                                  const T* U_s, const T* pscale_s, const T* dbar, const T* u_pose, const T* dxi,
                                  const int* status, T* u_depth, T* dd, hipStream_t st);
template <typename T>
hipError_t launch_adjoint_reduce(const T* edge_xbar, const int* pose_off, const int* pose_src, int n_fixed,
                                 int n_frames, T* pbar, const int* tile_patch, const int* pcount, const int* pedges,
                                 int n_tp, T* dbar, hipStream_t st);
template <typename T>
hipError_t launch_depth_to_tile(const T* src, const int* tile_patch, int n_tp, T* dst, hipStream_t st);
template <typename T>
hipError_t launch_fill(T* x, long long n, T v, hipStream_t st);
template <typename T>
hipError_t launch_copy(const T* src, T* dst, long long n, hipStream_t st);
hipError_t launch_report_finalize(dpvba_report* rep, const int* status, const unsigned int* min_bits,
                                  int n_iters, const int* err, hipStream_t st, const double* refine = nullptr,
                                  const int* fallback = nullptr);

}  // namespace dpvba

#include "tileargs.h"

using namespace dpvba;

namespace {

// Shared-memory budget of one tile, and default patches per tile for the
// float32 and float64 plans.
constexpr int kLdsBudget = 150 * 1024;
// Tiles of the multi-launch path (systems beyond the single-launch solver)
// are planned to fit two float32 workgroups per CU (160 KiB of LDS): more
// tiles, but two of them in flight per CU hide each other's dependent
// phases.  The single-launch solver keeps one workgroup per CU anyway and
// prefers fewer, larger tiles.
constexpr int kLdsBudgetTwoPerCu = 80 * 1024;
constexpr int kDefaultTilePatches32 = 96;
constexpr int kDefaultTilePatches64 = 32;
// Largest reduced system of one problem of a batch (its workgroup keeps the
// right-hand side on one wavefront, at most 4 entries per lane).
constexpr int kBatchMaxUnknowns = 252;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Bumped whenever a workspace buffer moves: a captured HIP graph that bakes
// in workspace addresses is valid only while it is unchanged.
uint64_t g_workspace_generation = 0;

hipError_t ensure(DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (b.bytes >= bytes) return hipSuccess;
  ++g_workspace_generation;
  if (b.p) {
    hipError_t e = hipFree(b.p);
    if (e != hipSuccess) return e;
    b.p = nullptr;
    b.bytes = 0;
  }
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) { b.p = nullptr; return e; }
  b.bytes = bytes;
  return hipSuccess;
}

template <typename X>
hipError_t upload(DevBuf& b, const std::vector<X>& v, hipStream_t st) {
  hipError_t e = ensure(b, v.size() * sizeof(X));
  if (e != hipSuccess || v.empty()) return e;
  e = hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(X), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

// Static workspace of dpvba_solve_noalloc: the per-call buffers of a
// single-launch solve, carved from one fixed array per device instead of
// the context's allocations.  In host code `scratch` names a host-side
// stand-in; its device address is resolved once per device, with that device
// current, by resolve_scratch (called from dpvba_create), and only that
// address is ever passed to kernels or copies.
constexpr size_t kScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};
hipError_t g_scratch_err[kMaxScratchDevices] = {};
bool g_scratch_done[kMaxScratchDevices] = {};

// Device address of `scratch` on `device`, which must be current.
static hipError_t resolve_scratch(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_done[device]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_err[device] = e;
    g_scratch_ptr[device] = e == hipSuccess ? ptr : nullptr;
    g_scratch_done[device] = true;
  }
  return g_scratch_err[device];
}

static void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_done[device] ? g_scratch_ptr[device] : nullptr;
}

// Device copy of one tiling of the patch graph.
struct Tiling {
  int n_tiles = 0, lds_bytes = 0, max_w6 = 0, max_k = 0;
  long long part_S = 0, part_vec = 0, u_elems = 0, u_alloc = 0, grid_cells = 0, n_tp = 0;
  DevBuf tiles, tile_patch, slot_frame, slot_blk, edge_grid, blk_pose, s_off, s_src, v_off, v_src;
  DevBuf order;  // launch order of the tiles: the heaviest first
  DevBuf* bufs[11] = {&tiles, &tile_patch, &slot_frame, &slot_blk, &edge_grid, &blk_pose, &s_off, &s_src, &v_off,
                      &v_src, &order};
};

// Shared memory of the depth write-back (tile_writeback): the block step
// row [dxi | 1 | 0 ...] of the widest tile and the dots of the largest one.
static int writeback_lds_bytes(const Tiling& tl, int tsize) {
  return (tile_u_stride(tl.max_w6 / 6) + tl.max_k) * tsize;
}

}  // namespace

// Host side of a factor plan (factor_plan.h) and its device lists.
struct PlanStore {
  std::vector<int32_t> reach, blocks_off;
  DevBuf blocks, chain_lo, chain_hi, fq_dev, reach_dev;
  PanelPlan plan{};
  int n = 0;  // the system size the plan is for
};

// Factor plan of an n-row system of pose blocks of width bw whose block row
// P couples first with block column fq[P] (<= P): per 64-column panel k the
// reach and the 64-row blocks below the panel's diagonal block that hold a
// row whose envelope starts in or before the panel (block 0 always listed:
// the trailing update runs its look-ahead there).
static hipError_t build_plan(const std::vector<int32_t>& fq, int bw, int n, PlanStore& ps, hipStream_t st) {
  const int nb = (int)fq.size(), np = (n + 63) / 64;
  std::vector<int32_t> last(nb, -1);
  for (int Pp = 0; Pp < nb; ++Pp) last[fq[Pp]] = std::max(last[fq[Pp]], Pp);
  for (int Qq = 1; Qq < nb; ++Qq) last[Qq] = std::max(last[Qq], last[Qq - 1]);
  std::vector<int32_t> reach(np, n), boff{0}, bl;
  for (int k = 0; k < np; ++k) {
    const int qmax = std::min(64 * k + 63, n - 1) / bw;
    reach[k] = std::min(n, bw * (std::max(last[qmax], qmax) + 1));
    const int t0 = 64 * (k + 1);
    auto active = [&](int r0, int r1) {  // any row of [r0, r1) (clipped to n)
      for (int Pp = r0 / bw; Pp * bw < std::min(r1, n); ++Pp)
        if (fq[Pp] <= qmax) return true;
      return false;
    };
    for (int B = 0; t0 + 64 * B < n; ++B)
      if (B == 0 || active(t0 + 64 * B, t0 + 64 * B + 64)) bl.push_back(B);
    boff.push_back((int32_t)bl.size());
  }
  if (bl.empty()) bl.push_back(0);
  // triangular-solve ranges per pair of 64-row blocks: block I's rows start
  // at column block fcb[I] (the envelope), and the rows that reach block
  // k's columns end at reach[k] (non-decreasing in k)
  std::vector<int32_t> fcb(np);
  for (int I = 0; I < np; ++I) {
    int lo = I;
    for (int Pp = (64 * I) / bw; Pp * bw < std::min(64 * I + 64, n); ++Pp) lo = std::min(lo, (bw * fq[Pp]) / 64);
    fcb[I] = lo;
  }
  const int npair = (np + 1) / 2;
  std::vector<int32_t> plo(npair), phi(npair);
  for (int Q = 0; Q < npair; ++Q) {
    const int I0 = 2 * Q, I1 = std::min(2 * Q + 1, np - 1);
    plo[Q] = std::min(fcb[I0], fcb[I1]) / 2;
    phi[Q] = std::max(Q, std::min(npair - 1, (reach[I1] - 1) / 128));
  }
  hipError_t e;
  if ((e = upload(ps.chain_lo, plo, st)) != hipSuccess) return e;
  if ((e = upload(ps.chain_hi, phi, st)) != hipSuccess) return e;
  if ((e = upload(ps.fq_dev, fq, st)) != hipSuccess) return e;
  if ((e = upload(ps.reach_dev, reach, st)) != hipSuccess) return e;
  if ((e = upload(ps.blocks, bl, st)) != hipSuccess) return e;
  ps.reach = reach;
  ps.blocks_off = boff;
  ps.plan = PanelPlan{ps.reach.data(),          ps.blocks_off.data(),     (const int*)ps.blocks.p,
                      (const int*)ps.chain_lo.p, (const int*)ps.chain_hi.p, (const int*)ps.fq_dev.p,
                      (const int*)ps.reach_dev.p, bw};
  ps.n = n;
  return hipSuccess;
}

struct dpvba_ctx {
  int device = 0;
  // analysed graph
  bool analysed = false;
  int N = 0, P = 0, E = 0, p = 0, n_fixed = 0, n_free = 0;
  const int32_t *ii = nullptr, *jj = nullptr, *kk = nullptr;
  Tiling tl[2];  // [0] float32 plan, [1] float64 plan
  int coop_grid32 = 0, coop_lds32 = -1, coop_grid64 = 0, coop_lds64 = -1;  // co-resident workgroups
  bool coop_launch = false;  // single-launch solver: cooperative launch instead of an ordinary one
  // workspace
  DevBuf part_S, part_vec, part_cost, part_invalid, U_s, pscale_s, depth_s, xh_s, poses_a, poses_b;
  // ticket: grid-barrier slots of the single-launch solver (slot p at
  // ticket[8 p .. 8 p + 1]); dev_err: failure words of a call (small-solve
  // launch parity p at [4 p], large path [8], batch [12]); host_err:
  // host-visible sticky failure words (pinned, mapped), host_err_dev its
  // device address
  DevBuf S, rhs, dB, d0, dx, wb, wy, Linv, edge_part, ticket, dev_err;
  int* host_err = nullptr;
  int* host_err_dev = nullptr;
  long long small_launches = 0;
  DevBuf chain_flags;  // the triangular chain's value-and-epoch words (chain_words_bytes)
  // sparsity plan of the float32 factor (factor_plan.h): per 64-column panel
  // its reach and the 64-row blocks below its diagonal block that hold a row
  // that can be non-zero in it
  PlanStore ba_plan;  // the analysed graph's reduced system
  // system order of the large solves: block p of the factored system is free
  // pose sys_perm[p] (sys_pos its inverse); empty: the poses' own order
  std::vector<int32_t> sys_perm_h;
  DevBuf sys_perm, sys_pos, sys_x, sys_b;
  // blocks of the envelope in the system order (int4: block row, block
  // column, the poses' lower block, transposed) and the element size S was
  // last zeroed for outside the envelope (0: not zeroed)
  DevBuf env_blk;
  int n_env = 0, s_env_elem = 0;
  bool s32_zeroed = false;  // S32 zero outside the envelope (mixed path)
  PlanStore pg_plan;  // the last pose graph's normal equations
  DevBuf one_inst;     // the analysed problem as a one-problem batch (small mixed solves)
  int chain_epoch = 0;
  DevBuf status, min_bits, devrep;
  // edge lists of the adjoint: per patch (pcount / pedges, edge order), per
  // pose (pose_off / pose_src = 2 e + side), tile-order position of a patch
  DevBuf pcount, pedges, pose_off, pose_src, patch_pos;
  // mixed precision: float32 factor, float64 iterate and residual, decision state
  DevBuf S32, x64, r64, rhs32, c32, d0_32, mx_max, mx_resid, mx_fb, mx_flag;
  int* host_flag = nullptr;  // pinned
  // batch analysis
  struct Batch {
    bool analysed = false;
    int B = 0, p = 0, N = 0, P = 0, E = 0, n_max = 0;
    long long n_free = 0, scratch = 0;
    const int32_t *ii = nullptr, *jj = nullptr, *kk = nullptr;
    std::vector<int32_t> frame_off, patch_off, edge_off, n_fixed;
    Tiling tl[2];
    DevBuf inst[2];
    DevBuf status, min_bits, refine, fallback, reps, scratch_buf;
    hipGraphExec_t exec = nullptr;
    std::vector<uint64_t> key;
  } bt;
  // adjoint workspace
  // Sim(3) pose-graph optimisation workspace
  DevBuf pg_C, pg_ea, pg_eb, pg_r, pg_J, pg_H, pg_rhs, pg_dx, pg_d0, pg_wy, pg_Linv, pg_flags, pg_status, pg_mb,
      pg_cost, pg_blk_pq, pg_blk_off, pg_blk_src, pg_pose_off, pg_pose_src, pg_perm, pg_xs;
  int pg_epoch = 0;
  DevBuf bw_poses, bw_depth, bw_dx, bw_pbar, bw_dbar, bw_dxbar, bw_rhs, bw_up, bw_ud, bw_dd, bw_edge, bw_status,
      bw_minbits;
  char err[256] = {0};
  // tracing
  bool tracing = false;
  int trace_every = 1;
  std::vector<hipEvent_t> ev;       // 2 per pair
  // the context's own stream and events for the calls over many contexts
  // (created on first use, default priority)
  hipStream_t aux = nullptr;
  hipEvent_t aux_start = nullptr, aux_done = nullptr;
  std::vector<int> ev_phase;        // phase per pair
  int ev_used = 0;
  long long seen[DPVBA_N_PHASES] = {0};
  int open_pair = -1;
};

// Trace scope: records an event pair around one phase when sampled.
struct TraceScope {
  dpvba_ctx* c;
  hipStream_t st;
  int pair = -1;
  TraceScope(dpvba_ctx* c_, int phase, hipStream_t st_) : c(c_), st(st_) {
    if (!c->tracing) return;
    const long long n = c->seen[phase]++;
    if (n % c->trace_every != 0 || c->ev_used * 2 + 2 > (int)c->ev.size()) return;
    pair = c->ev_used++;
    c->ev_phase[pair] = phase;
    (void)hipEventRecord(c->ev[2 * pair], st);
  }
  ~TraceScope() {
    if (pair >= 0) (void)hipEventRecord(c->ev[2 * pair + 1], st);
  }
};

// Epoch of the next chained triangular solve (never 0, the flags' initial value).
// The factor plan of the analysed graph for a reduced system of n rows (null
// when it was not built for this n: the factor is then dense).
static const PanelPlan* reach_of(const dpvba_ctx* c, int n) {
  return c->ba_plan.n == n && n > 0 ? &c->ba_plan.plan : nullptr;
}

// Bytes of the triangular chain's value words for nblk 64-row blocks: two
// passes, two 64-bit words per row (float64; float32 uses one).
static size_t chain_words_bytes(size_t nblk) { return 2 * nblk * 64 * 2 * 8; }

// The large solves of a reduced system of more than this many unknowns run
// in the system order (the smaller ones are gathered inside their kernels).
constexpr int kPermuteMinUnknowns = kBatchMaxUnknowns;

// System-order permutation (device, block p = free pose perm[p]) of the
// analysed graph's large solves, or null for the poses' own order.
static const int* sys_perm_of(const dpvba_ctx* c) {
  return !c->sys_perm_h.empty() && 6 * c->n_free > kPermuteMinUnknowns ? (const int*)c->sys_perm.p : nullptr;
}
static const int* sys_pos_of(const dpvba_ctx* c) { return sys_perm_of(c) ? (const int*)c->sys_pos.p : nullptr; }

// Gather of the large path's damped reduced system into the context's S in
// the system order: only the envelope's blocks (the rest of S zeroed once
// per analysis and element type), or every lower block for the smaller
// systems.
template <typename T>
static hipError_t gather_system(dpvba_ctx* c, const Tiling& tl, const T* part_S, const T* part_vec, T* S, T* rhs,
                                T lambda, T lam_diag, T* d0, hipStream_t st) {
  const int n = 6 * c->n_free;
  if (c->n_env > 0 && n > kPermuteMinUnknowns && S == (T*)c->S.p) {
    if (c->s_env_elem != (int)sizeof(T)) {
      hipError_t e = launch_fill<T>(S, (long long)n * n, (T)0, st);
      if (e != hipSuccess) return e;
      c->s_env_elem = (int)sizeof(T);
    }
    return launch_gather_env<T>(part_S, part_vec, (const int*)tl.s_off.p, (const int*)tl.s_src.p,
                                (const int*)tl.v_off.p, (const int2*)tl.v_src.p, c->n_free, (const int4*)c->env_blk.p,
                                c->n_env, S, rhs, (T*)c->dB.p, lambda, lam_diag, d0, st, sys_pos_of(c));
  }
  return launch_gather<T>(part_S, part_vec, (const int*)tl.s_off.p, (const int*)tl.s_src.p, (const int*)tl.v_off.p,
                          (const int2*)tl.v_src.p, c->n_free, S, rhs, (T*)c->dB.p, lambda, lam_diag, 0, d0, st,
                          sys_pos_of(c));
}

// Block row P of a symmetric block pattern starts at block column fq[P]
// (<= P): fill of a Cholesky factor stays between it and the diagonal.
static double envelope_cost(const std::vector<int32_t>& fq) {
  double s = 0.0;
  for (size_t P = 0; P < fq.size(); ++P) {
    const double w = (double)(P - fq[P] + 1);
    s += w * w;
  }
  return s;
}

static std::vector<int32_t> first_coupled(const std::vector<std::vector<int32_t>>& adj,
                                          const std::vector<int32_t>& pos) {
  std::vector<int32_t> fq(adj.size());
  for (size_t P = 0; P < adj.size(); ++P) {
    int q = pos[P];
    for (int Q : adj[P]) q = std::min(q, pos[Q]);
    fq[pos[P]] = q;
  }
  return fq;
}

// Reverse Cuthill-McKee order of a graph (George and Liu's profile-reducing
// ordering): per connected component, breadth-first from a pseudo-peripheral
// vertex (the far end of repeated breadth-first sweeps), the unvisited
// neighbours of each vertex queued by increasing degree; the whole order is
// then reversed.  Returns order[p] = vertex at position p.
static std::vector<int32_t> rcm_order(const std::vector<std::vector<int32_t>>& adj) {
  const int nv = (int)adj.size();
  std::vector<int32_t> order, level(nv, -1);
  std::vector<char> done(nv, 0);
  order.reserve(nv);
  auto deg = [&](int v) { return (int)adj[v].size(); };
  // breadth-first levels from r over the vertices not yet ordered; returns
  // the last level's vertex of least degree and the eccentricity
  auto sweep = [&](int r, int* far) {
    std::vector<int32_t> q{r};
    std::fill(level.begin(), level.end(), -1);
    level[r] = 0;
    for (size_t h = 0; h < q.size(); ++h)
      for (int u : adj[q[h]])
        if (!done[u] && level[u] < 0) {
          level[u] = level[q[h]] + 1;
          q.push_back(u);
        }
    const int ecc = level[q.back()];
    int best = q.back();
    for (int v : q)
      if (level[v] == ecc && deg(v) < deg(best)) best = v;
    *far = best;
    return ecc;
  };
  for (;;) {
    int r = -1;
    for (int v = 0; v < nv; ++v)
      if (!done[v] && (r < 0 || deg(v) < deg(r))) r = v;
    if (r < 0) break;
    int far = r, ecc = sweep(r, &far);
    for (int t = 0; t < 8; ++t) {
      int far2 = far;
      const int e2 = sweep(far, &far2);
      if (e2 <= ecc) break;
      r = far;
      ecc = e2;
      far = far2;
    }
    const size_t first = order.size();
    order.push_back(r);
    done[r] = 1;
    std::vector<int32_t> nb;
    for (size_t h = first; h < order.size(); ++h) {
      nb.clear();
      for (int u : adj[order[h]])
        if (!done[u]) {
          done[u] = 1;
          nb.push_back(u);
        }
      std::stable_sort(nb.begin(), nb.end(), [&](int a, int b) { return deg(a) < deg(b); });
      order.insert(order.end(), nb.begin(), nb.end());
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

static int next_epoch(dpvba_ctx* c) {
  c->chain_epoch = c->chain_epoch >= 0x3fffffff ? 1 : c->chain_epoch + 1;
  return c->chain_epoch;
}

static void record_error(dpvba_ctx* c, hipError_t e, const char* where) {
  if (!c) return;
  snprintf(c->err, sizeof(c->err), "%s: %s (%d)", where, hipGetErrorString(e), (int)e);
}

static dpvba_status hip_status(hipError_t e) {
  if (e == hipSuccess) return DPVBA_OK;
  return e == hipErrorOutOfMemory ? DPVBA_ENOMEM : DPVBA_EHIP;
}

#define HIP_TRY(x)                                      \
  do {                                                  \
    hipError_t _e = (x);                                \
    if (_e != hipSuccess) {                             \
      record_error(c, _e, #x);                          \
      return hip_status(_e);                            \
    }                                                   \
  } while (0)

extern "C" {

const char* dpvba_last_error(const dpvba_ctx* c) { return c ? c->err : ""; }

dpvba_status dpvba_get_analysis_info(const dpvba_ctx* c, int32_t precision, dpvba_analysis_info* info) {
  if (!c || !info || (precision != DPVBA_FP32 && precision != DPVBA_FP64)) return DPVBA_EINVAL;
  if (!c->analysed) return DPVBA_ESTATE;
  const Tiling& t = c->tl[precision == DPVBA_FP64 ? 1 : 0];
  info->n_tiles = t.n_tiles;
  info->n_free = c->n_free;
  info->part_S_elems = t.part_S;
  info->part_vec_elems = t.part_vec;
  info->grid_cells = t.grid_cells;
  info->u_elems = t.u_elems;
  info->lds_bytes = t.lds_bytes;
  return DPVBA_OK;
}

dpvba_status dpvba_get_system_order(const dpvba_ctx* c, int32_t* order, int32_t n) {
  if (!c || !order) return DPVBA_EINVAL;
  if (!c->analysed) return DPVBA_ESTATE;
  if (n != c->n_free) return DPVBA_EINVAL;
  const bool perm = sys_perm_of(c) != nullptr;
  for (int p = 0; p < n; ++p) order[p] = perm ? c->sys_perm_h[p] : p;
  return DPVBA_OK;
}

dpvba_status dpvba_set_cooperative(dpvba_ctx* c, int32_t cooperative) {
  if (!c || (cooperative != 0 && cooperative != 1)) return DPVBA_EINVAL;
  c->coop_launch = cooperative == 1;
  return DPVBA_OK;
}

dpvba_status dpvba_trace_begin(dpvba_ctx* c, int32_t sample_every, int32_t max_pairs) {
  if (!c || sample_every < 1 || max_pairs < 1) return DPVBA_EINVAL;
  HIP_TRY(hipSetDevice(c->device));
  if ((int)c->ev.size() < 2 * max_pairs) {
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    c->ev.assign(2 * (size_t)max_pairs, nullptr);
    for (auto& e : c->ev) HIP_TRY(hipEventCreate(&e));
    c->ev_phase.assign(max_pairs, 0);
  }
  c->trace_every = sample_every;
  c->ev_used = 0;
  for (long long& x : c->seen) x = 0;
  c->tracing = true;
  return DPVBA_OK;
}

dpvba_status dpvba_trace_end(dpvba_ctx* c, double* ms, int32_t* n_sampled, int64_t* n_launched) {
  if (!c || !c->tracing) return DPVBA_EINVAL;
  c->tracing = false;
  double tot[DPVBA_N_PHASES] = {0};
  int cnt[DPVBA_N_PHASES] = {0};
  for (int q = 0; q < c->ev_used; ++q) {
    HIP_TRY(hipEventSynchronize(c->ev[2 * q + 1]));
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, c->ev[2 * q], c->ev[2 * q + 1]));
    tot[c->ev_phase[q]] += t;
    cnt[c->ev_phase[q]]++;
  }
  for (int p = 0; p < DPVBA_N_PHASES; ++p) {
    if (ms) ms[p] = tot[p];
    if (n_sampled) n_sampled[p] = cnt[p];
    if (n_launched) n_launched[p] = c->seen[p];
  }
  return DPVBA_OK;
}

const char* dpvba_status_string(dpvba_status s) {
  switch (s) {
    case DPVBA_OK: return "ok";
    case DPVBA_EINVAL: return "invalid argument";
    case DPVBA_ENOTPD: return "reduced camera system not positive definite";
    case DPVBA_ENOMEM: return "out of device memory";
    case DPVBA_EHIP: return "HIP runtime error";
    case DPVBA_ESTATE: return "numeric call without a matching dpvba_analyze";
    case DPVBA_EDEVICE: return "device work of an earlier call failed (see dpvba_device_status)";
    case DPVBA_ELIMIT: return "problem exceeds a fixed capacity (see dpvba_last_error)";
  }
  return "unknown status";
}

dpvba_status dpvba_create(dpvba_ctx** out, int32_t device) {
  if (!out) return DPVBA_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return DPVBA_EINVAL;
  dpvba_ctx* c = new (std::nothrow) dpvba_ctx();
  if (!c) return DPVBA_ENOMEM;
  c->device = device;
  hipError_t e = hipSetDevice(device);
  // the static scratch of dpvba_solve_noalloc: its address on this device,
  // resolved once per device (a failure is kept and returned by that call)
  if (e == hipSuccess) (void)resolve_scratch(device);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&c->host_err, kHostErrWords * sizeof(int), hipHostMallocMapped | hipHostMallocCoherent);
  if (e == hipSuccess) {
    for (int q = 0; q < kHostErrWords; ++q) c->host_err[q] = 0;
    e = hipHostGetDevicePointer((void**)&c->host_err_dev, c->host_err, 0);
  }
  if (e == hipSuccess) e = ensure(c->ticket, 64);
  if (e == hipSuccess) e = ensure(c->dev_err, 64);
  if (e == hipSuccess) e = hipMemset(c->ticket.p, 0, 64);
  if (e == hipSuccess) e = hipMemset(c->dev_err.p, 0, 64);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    dpvba_destroy(c);
    return hip_status(e);
  }
  *out = c;
  return DPVBA_OK;
}

// Failure bits recorded by earlier calls' kernels in the host-visible words.
static int recorded_failure(const dpvba_ctx* c) {
  int bits = 0;
  for (int q = 0; q < kHostErrWords; ++q)
    if (__atomic_load_n(c->host_err + q, __ATOMIC_ACQUIRE)) bits |= 1 << q;
  return bits;
}

dpvba_status dpvba_device_status(dpvba_ctx* c, void* stream, int32_t* cause) {
  if (!c) return DPVBA_EINVAL;
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  const int bits = recorded_failure(c);
  if (cause) *cause = bits;
  if (!bits) return DPVBA_OK;
  // re-arm: barrier slots and failure words start from zero again
  HIP_TRY(hipMemsetAsync(c->ticket.p, 0, 64, (hipStream_t)stream));
  HIP_TRY(hipMemsetAsync(c->dev_err.p, 0, 64, (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  for (int q = 0; q < kHostErrWords; ++q) __atomic_store_n(c->host_err + q, 0, __ATOMIC_RELEASE);
  return DPVBA_EDEVICE;
}

void dpvba_destroy(dpvba_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  DevBuf* bufs[] = {&c->part_S, &c->part_vec, &c->part_cost, &c->part_invalid, &c->U_s, &c->pscale_s,
                    &c->depth_s, &c->xh_s, &c->poses_a, &c->poses_b, &c->S, &c->rhs, &c->dB, &c->d0, &c->dx,
                    &c->wb, &c->wy, &c->Linv, &c->edge_part, &c->ticket, &c->dev_err, &c->status, &c->min_bits, &c->devrep,
                    &c->chain_flags, &c->one_inst, &c->ba_plan.blocks, &c->pg_plan.blocks,
                    &c->ba_plan.chain_lo, &c->ba_plan.chain_hi, &c->pg_plan.chain_lo,
                    &c->pg_plan.chain_hi, &c->ba_plan.fq_dev, &c->ba_plan.reach_dev, &c->pg_plan.fq_dev,
                    &c->pg_plan.reach_dev, &c->sys_perm, &c->sys_pos, &c->sys_x, &c->sys_b, &c->env_blk,
                    &c->pcount, &c->pedges, &c->pose_off, &c->pose_src, &c->patch_pos, &c->bw_poses, &c->bw_depth,
                    &c->bw_dx, &c->bw_pbar, &c->bw_dbar, &c->bw_dxbar, &c->bw_rhs, &c->bw_up, &c->bw_ud, &c->bw_dd,
                    &c->bw_edge, &c->bw_status, &c->bw_minbits, &c->S32, &c->x64, &c->r64, &c->rhs32, &c->c32,
                    &c->d0_32, &c->mx_max, &c->mx_resid, &c->mx_fb, &c->mx_flag, &c->pg_C, &c->pg_ea, &c->pg_eb,
                    &c->pg_r, &c->pg_J, &c->pg_H, &c->pg_rhs, &c->pg_dx, &c->pg_d0, &c->pg_wy, &c->pg_Linv,
                    &c->pg_flags, &c->pg_status, &c->pg_mb, &c->pg_cost, &c->pg_blk_pq, &c->pg_blk_off,
                    &c->pg_blk_src, &c->pg_pose_off, &c->pg_pose_src, &c->pg_perm, &c->pg_xs};
  for (DevBuf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  for (Tiling& t : c->tl)
    for (DevBuf* b : t.bufs)
      if (b->p) (void)hipFree(b->p);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  if (c->aux_start) (void)hipEventDestroy(c->aux_start);
  if (c->aux_done) (void)hipEventDestroy(c->aux_done);
  if (c->aux) (void)hipStreamDestroy(c->aux);
  if (c->host_flag) (void)hipHostFree(c->host_flag);
  if (c->host_err) (void)hipHostFree(c->host_err);
  {
    DevBuf* bb[] = {&c->bt.inst[0], &c->bt.inst[1], &c->bt.status, &c->bt.min_bits, &c->bt.refine, &c->bt.fallback,
                    &c->bt.reps, &c->bt.scratch_buf};
    for (DevBuf* b : bb)
      if (b->p) (void)hipFree(b->p);
    for (Tiling& t : c->bt.tl)
      for (DevBuf* b : t.bufs)
        if (b->p) (void)hipFree(b->p);
    if (c->bt.exec) (void)hipGraphExecDestroy(c->bt.exec);
  }
  delete c;
}

static hipError_t backward_workspace(dpvba_ctx* c, int N, long long ntp, long long E, int n);

static bool graph_sizes_ok(const dpvba_graph* g) {
  if (!g) return false;
  if (g->n_frames < 1 || g->n_patches < 0 || g->n_edges < 0) return false;
  if (g->patch_size < 1 || (g->patch_size % 2) == 0) return false;
  if (g->n_fixed < 0 || g->n_fixed > g->n_frames) return false;
  if (g->n_frames > (1 << 24) || g->n_patches > (1 << 28) || g->n_edges > (1 << 29)) return false;
  if (!(g->fx != 0.f) || !(g->fy != 0.f)) return false;
  if (g->n_edges > 0 && (!g->ii || !g->jj || !g->kk || !g->target || !g->weight)) return false;
  if (g->n_patches > 0 && !g->patches) return false;
  return true;
}

// Targets and weights of E edges copied to the host (synchronising st) and
// checked: every value finite, every weight >= 0.
static hipError_t inputs_valid(const float* target, const float* weight, long long E, hipStream_t st, bool* ok) {
  *ok = true;
  if (E <= 0) return hipSuccess;
  std::vector<float> tw(4 * (size_t)E);
  hipError_t e = hipMemcpyAsync(tw.data(), target, (size_t)E * 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(tw.data() + 2 * E, weight, (size_t)E * 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  for (size_t q = 0; q < 2 * (size_t)E; ++q)
    if (!(std::fabs(tw[q]) <= FLT_MAX)) *ok = false;
  for (size_t q = 2 * (size_t)E; q < 4 * (size_t)E; ++q)
    if (!(tw[q] >= 0.f && tw[q] <= FLT_MAX)) *ok = false;
  return hipSuccess;
}

// Host copy of one tiling.
struct HostTiling {
  std::vector<TileInfo> tiles;
  std::vector<int32_t> tile_patch, slot_frame, slot_blk, edge_grid, blk_pose, s_off, s_src, v_off;
  std::vector<int2> v_src;
  long long part_S = 0, part_vec = 0;
  long long u_elems = 0;  // entries of the stored Schur rows (K 6 n_blk per tile)
  long long u_alloc = 0;  // their padded storage (tile_u_rows x tile_u_stride per tile)
  int lds = 0, max_w6 = 0, max_k = 0;
};

// Edge structure of one problem from host copies of its indices: edges
// grouped by patch (pcount / pedges, original order within a patch) and each
// frame's patches.  False on an index out of range, a self edge or a patch
// whose edges leave different frames.
struct ProblemIndex {
  std::vector<int32_t> pcount, pedges;
  std::vector<std::vector<int32_t>> frame_patches;
};

static bool index_problem(int N, int P, int E, const int32_t* ii, const int32_t* jj, const int32_t* kk,
                          ProblemIndex& X) {
  std::vector<int32_t> owner(P, -1);
  X.pcount.assign(P + 1, 0);
  for (int e = 0; e < E; ++e) {
    const int i = ii[e], j = jj[e], k = kk[e];
    if (i < 0 || i >= N || j < 0 || j >= N || k < 0 || k >= P || i == j) return false;
    if (owner[k] < 0) owner[k] = i;
    else if (owner[k] != i) return false;
    X.pcount[k + 1]++;
  }
  for (int k = 0; k < P; ++k) X.pcount[k + 1] += X.pcount[k];
  X.pedges.assign(E, 0);
  std::vector<int32_t> cur(X.pcount.begin(), X.pcount.end() - 1);
  for (int e = 0; e < E; ++e) X.pedges[cur[kk[e]]++] = e;
  X.frame_patches.assign(N, {});
  for (int k = 0; k < P; ++k)
    if (owner[k] >= 0) X.frame_patches[owner[k]].push_back(k);
  return true;
}

// Split each source frame's patches into tiles of at most `kcap` patches
// whose shared-memory plan (element size tsize) fits the budget, then build
// the gather lists.  Returns false if one patch alone does not fit.
static bool plan_tiling(int N, int nf, const std::vector<int32_t>& jj, const std::vector<int32_t>& pcount,
                        const std::vector<int32_t>& pedges, const std::vector<std::vector<int32_t>>& frame_patches,
                        int kcap, int tsize, HostTiling& H, int lds_budget = kLdsBudget) {
  const int n_free = N - nf;
  auto patch_mult = [&](int k, std::map<int, int>& m) {
    for (int q = pcount[k]; q < pcount[k + 1]; ++q) m[jj[pedges[q]]]++;
  };
  auto plan_of = [&](const std::map<int, int>& mult, int frame, int& Tn, int& nb, int& mm) {
    Tn = 0;
    mm = 1;
    nb = frame >= nf ? 1 : 0;
    for (auto& kv : mult) {
      Tn += kv.second;
      mm = std::max(mm, kv.second);
      if (kv.first >= nf) nb++;
    }
  };
  auto emit = [&](int frame, const std::vector<int32_t>& pl, const std::map<int, int>& mult) {
    TileInfo t{};
    t.frame = frame;
    t.n_patch = (int)pl.size();
    t.patch_begin = (int)H.tile_patch.size();
    t.slot_begin = (int)H.slot_frame.size();
    t.grid_begin = (int)H.edge_grid.size();
    t.blk_begin = (int)H.blk_pose.size();
    std::vector<int> blocks;
    if (frame >= nf) blocks.push_back(frame);
    for (auto& kv : mult)
      if (kv.first >= nf) blocks.push_back(kv.first);
    std::sort(blocks.begin(), blocks.end());
    auto blk_of = [&](int pose) -> int {
      auto it = std::lower_bound(blocks.begin(), blocks.end(), pose);
      return (it != blocks.end() && *it == pose) ? (int)(it - blocks.begin()) : -1;
    };
    t.src_blk = blk_of(frame);
    t.n_blk = (int)blocks.size();
    std::map<int, int> first_slot;
    int Tn = 0, mm = 1;
    for (auto& kv : mult) {
      first_slot[kv.first] = Tn;
      mm = std::max(mm, kv.second);
      for (int m = 0; m < kv.second; ++m) {
        H.slot_frame.push_back(kv.first);
        H.slot_blk.push_back(blk_of(kv.first));
      }
      Tn += kv.second;
    }
    t.n_slot = Tn;
    t.max_mult = mm;
    for (int b : blocks) H.blk_pose.push_back(b - nf);
    const size_t g0 = H.edge_grid.size();
    H.edge_grid.resize(g0 + (size_t)t.n_patch * Tn, -1);
    for (int lp = 0; lp < t.n_patch; ++lp) {
      const int k = pl[lp];
      H.tile_patch.push_back(k);
      std::map<int, int> used;
      for (int q = pcount[k]; q < pcount[k + 1]; ++q) {
        const int e = pedges[q];
        const int s = first_slot[jj[e]] + used[jj[e]]++;
        H.edge_grid[g0 + (size_t)lp * Tn + s] = e;
      }
    }
    t.part_begin = (int)H.part_S;
    t.vec_begin = (int)H.part_vec;
    t.u_begin = (int)H.u_alloc;
    H.part_S += (long long)t.n_blk * (t.n_blk + 1) / 2 * 36;
    H.part_vec += 12LL * t.n_blk;
    H.u_elems += (long long)t.n_patch * 6 * t.n_blk;
    H.u_alloc += (long long)tile_u_rows(t.n_patch) * tile_u_stride(t.n_blk);
    H.lds = std::max(H.lds, tile_lds_bytes(t.n_patch, Tn, t.n_blk, tsize));
    H.max_w6 = std::max(H.max_w6, 6 * t.n_blk);
    H.max_k = std::max(H.max_k, t.n_patch);
    H.tiles.push_back(t);
  };
  for (int f = 0; f < N; ++f) {
    std::vector<int32_t> cur;
    std::map<int, int> cur_mult;
    for (int k : frame_patches[f]) {
      std::map<int, int> km;
      patch_mult(k, km);
      std::map<int, int> merged = cur_mult;
      for (auto& kv : km) merged[kv.first] = std::max(merged[kv.first], kv.second);
      int Tn, nb, mm;
      plan_of(merged, f, Tn, nb, mm);
      const bool fits = Tn <= kMaxSlots && (int)cur.size() + 1 <= kcap &&
                        tile_lds_bytes((int)cur.size() + 1, Tn, nb, tsize) <= lds_budget;
      if (!fits) {
        if (cur.empty()) return false;
        emit(f, cur, cur_mult);
        cur.clear();
        cur_mult.clear();
        merged = km;
        plan_of(merged, f, Tn, nb, mm);
        if (!(Tn <= kMaxSlots && tile_lds_bytes(1, Tn, nb, tsize) <= lds_budget)) return false;
      }
      cur.push_back(k);
      cur_mult = merged;
    }
    if (!cur.empty()) emit(f, cur, cur_mult);
  }
  if (H.part_S > INT32_MAX || H.part_vec > INT32_MAX || H.u_alloc > INT32_MAX) return false;
  // gather lists: lower block (P >= Q) -> tile partial offsets, in tile order
  const long long n_lb = (long long)n_free * (n_free + 1) / 2;
  H.s_off.assign(n_lb + 1, 0);
  H.v_off.assign(n_free + 1, 0);
  for (const TileInfo& t : H.tiles) {
    for (int a = 0; a < t.n_blk; ++a)
      for (int b = a; b < t.n_blk; ++b) {
        const long long Pp = H.blk_pose[t.blk_begin + b], Qq = H.blk_pose[t.blk_begin + a];
        H.s_off[Pp * (Pp + 1) / 2 + Qq + 1]++;
      }
    for (int a = 0; a < t.n_blk; ++a) H.v_off[H.blk_pose[t.blk_begin + a] + 1]++;
  }
  for (long long q = 0; q < n_lb; ++q) H.s_off[q + 1] += H.s_off[q];
  for (int q = 0; q < n_free; ++q) H.v_off[q + 1] += H.v_off[q];
  H.s_src.assign(H.s_off[n_lb], 0);
  H.v_src.assign(H.v_off[n_free], make_int2(0, 0));
  std::vector<int32_t> cs(H.s_off.begin(), H.s_off.end() - 1), cv(H.v_off.begin(), H.v_off.end() - 1);
  for (const TileInfo& t : H.tiles) {
    for (int a = 0; a < t.n_blk; ++a)
      for (int b = a; b < t.n_blk; ++b) {
        const long long Pp = H.blk_pose[t.blk_begin + b], Qq = H.blk_pose[t.blk_begin + a];
        H.s_src[cs[Pp * (Pp + 1) / 2 + Qq]++] = t.part_begin + upper_pair_index(a, b, t.n_blk) * 36;
      }
    for (int a = 0; a < t.n_blk; ++a) {
      const int Pp = H.blk_pose[t.blk_begin + a];
      H.v_src[cv[Pp]++] = make_int2(t.vec_begin + 6 * a, t.vec_begin + 6 * t.n_blk + 6 * a);
    }
  }
  return true;
}

static hipError_t upload_tiling(Tiling& T_, const HostTiling& H, hipStream_t st) {
  hipError_t e;
  if ((e = upload(T_.tiles, H.tiles, st)) != hipSuccess) return e;
  if ((e = upload(T_.tile_patch, H.tile_patch, st)) != hipSuccess) return e;
  if ((e = upload(T_.slot_frame, H.slot_frame, st)) != hipSuccess) return e;
  if ((e = upload(T_.slot_blk, H.slot_blk, st)) != hipSuccess) return e;
  if ((e = upload(T_.edge_grid, H.edge_grid, st)) != hipSuccess) return e;
  if ((e = upload(T_.blk_pose, H.blk_pose, st)) != hipSuccess) return e;
  if ((e = upload(T_.s_off, H.s_off, st)) != hipSuccess) return e;
  if ((e = upload(T_.s_src, H.s_src, st)) != hipSuccess) return e;
  if ((e = upload(T_.v_off, H.v_off, st)) != hipSuccess) return e;
  if ((e = upload(T_.v_src, H.v_src, st)) != hipSuccess) return e;
  {
    // one workgroup per tile: the heaviest tiles go first, so the last ones
    // to start are short (work ~ edge cells + Schur rows + the U^T U product)
    std::vector<int32_t> ord(H.tiles.size());
    std::vector<long long> cost(H.tiles.size());
    for (size_t t = 0; t < H.tiles.size(); ++t) {
      const TileInfo& ti = H.tiles[t];
      ord[t] = (int32_t)t;
      cost[t] = (long long)ti.n_patch * (ti.n_slot + 6 * ti.n_blk) + 18LL * ti.n_blk * (ti.n_blk + 1);
    }
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
    if (ord.empty()) ord.push_back(0);
    if ((e = upload(T_.order, ord, st)) != hipSuccess) return e;
  }
  T_.n_tiles = (int)H.tiles.size();
  T_.lds_bytes = H.lds;
  T_.max_w6 = H.max_w6;
  T_.max_k = H.max_k;
  T_.part_S = H.part_S;
  T_.part_vec = H.part_vec;
  T_.u_elems = H.u_elems;
  T_.u_alloc = H.u_alloc;
  T_.grid_cells = (long long)H.edge_grid.size();
  T_.n_tp = (long long)H.tile_patch.size();
  return hipSuccess;
}

dpvba_status dpvba_analyze_ex(dpvba_ctx* c, const dpvba_graph* g, const dpvba_tuning* tune, void* stream) {
  if (!c || !graph_sizes_ok(g)) return DPVBA_EINVAL;
  int kcap32 = kDefaultTilePatches32, kcap64 = kDefaultTilePatches64;
  if (tune) {
    if (tune->tile_patches_fp32 < 0 || tune->tile_patches_fp64 < 0) return DPVBA_EINVAL;
    if (tune->keep_order != 0 && tune->keep_order != 1) return DPVBA_EINVAL;
    if (tune->tile_patches_fp32 > 0) kcap32 = tune->tile_patches_fp32;
    if (tune->tile_patches_fp64 > 0) kcap64 = tune->tile_patches_fp64;
  }
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(c->device));
  c->analysed = false;
  const int N = g->n_frames, P = g->n_patches, E = g->n_edges, nf = g->n_fixed;
  const int n_free = N - nf;
  if ((long long)n_free * 6 > 46000) return DPVBA_EINVAL;  // dense reduced system must stay addressable
  std::vector<int32_t> ii(E), jj(E), kk(E);
  if (E) {
    HIP_TRY(hipMemcpyAsync(ii.data(), g->ii, E * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(jj.data(), g->jj, E * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(kk.data(), g->kk, E * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  ProblemIndex X;
  if (!index_problem(N, P, E, ii.data(), jj.data(), kk.data(), X)) return DPVBA_EINVAL;
  {
    bool ok = true;
    HIP_TRY(inputs_valid(g->target, g->weight, E, st, &ok));
    if (!ok) return DPVBA_EINVAL;
  }
  const std::vector<int32_t>& pcount = X.pcount;
  const std::vector<int32_t>& pedges = X.pedges;
  const std::vector<std::vector<int32_t>>& frame_patches = X.frame_patches;
  HostTiling H32, H64;
  const bool single_launch = 6 * (long long)n_free + 1 <= kSmallRows;
  if (!plan_tiling(N, nf, jj, pcount, pedges, frame_patches, kcap32, 4, H32,
                   single_launch ? kLdsBudget : kLdsBudgetTwoPerCu))
    return DPVBA_EINVAL;
  if (!plan_tiling(N, nf, jj, pcount, pedges, frame_patches, kcap64, 8, H64)) return DPVBA_EINVAL;
  HIP_TRY(upload_tiling(c->tl[0], H32, st));
  HIP_TRY(upload_tiling(c->tl[1], H64, st));
  {
    // envelope of the reduced system: block row P starts at its first
    // coupled block column fq[P] (a tile contributes to (P, Q)); Cholesky
    // fill stays between that column and the diagonal, so the rows that can
    // be non-zero in block column Q end at the last P with fq[P] <= Q
    std::vector<std::vector<int32_t>> adj(n_free);
    for (int Pp = 0; Pp < n_free; ++Pp) {
      const long long base = (long long)Pp * (Pp + 1) / 2;
      for (int Qq = 0; Qq < Pp; ++Qq)
        if (H32.s_off[base + Qq + 1] > H32.s_off[base + Qq]) {
          adj[Pp].push_back(Qq);
          adj[Qq].push_back(Pp);
        }
    }
    std::vector<int32_t> ident(n_free), pos(n_free);
    for (int Pp = 0; Pp < n_free; ++Pp) ident[Pp] = Pp;
    std::vector<int32_t> fq = first_coupled(adj, ident);
    c->sys_perm_h.clear();
    if (6 * n_free > kPermuteMinUnknowns && !(tune && tune->keep_order)) {
      // a symmetric permutation leaves the solution unchanged and can shrink
      // the envelope (and the factor's work) by orders of magnitude when
      // loop closures couple distant keyframes
      const std::vector<int32_t> order = rcm_order(adj);
      for (int p = 0; p < n_free; ++p) pos[order[p]] = p;
      std::vector<int32_t> fq_r = first_coupled(adj, pos);
      if (envelope_cost(fq_r) < 0.9 * envelope_cost(fq)) {
        c->sys_perm_h = order;
        fq = fq_r;
        HIP_TRY(upload(c->sys_perm, order, st));
        HIP_TRY(upload(c->sys_pos, pos, st));
      }
    }
    c->ba_plan.n = 0;
    HIP_TRY(build_plan(fq, 6, 6 * n_free, c->ba_plan, st));
    c->n_env = 0;
    c->s_env_elem = 0;
    c->s32_zeroed = false;
    if (6 * n_free > kPermuteMinUnknowns) {
      std::vector<int32_t> env;
      const bool perm = !c->sys_perm_h.empty();
      for (int Ps = 0; Ps < n_free; ++Ps)
        for (int Qs = fq[Ps]; Qs <= Ps; ++Qs) {
          const int Pp = perm ? c->sys_perm_h[Ps] : Ps, Qq = perm ? c->sys_perm_h[Qs] : Qs;
          const int a = std::max(Pp, Qq), b = std::min(Pp, Qq);
          env.insert(env.end(), {Ps, Qs, (int32_t)((long long)a * (a + 1) / 2 + b), Pp < Qq ? 1 : 0});
        }
      HIP_TRY(upload(c->env_blk, env, st));
      c->n_env = (int)(env.size() / 4);
    }
  }
  {
    // both plans list the patches in the same order (frame, then patch id)
    if (H32.tile_patch != H64.tile_patch) return DPVBA_EINVAL;
    std::vector<int32_t> pos(P, -1), pose_off(N + 1, 0), pose_src(2 * (size_t)E);
    for (size_t q = 0; q < H32.tile_patch.size(); ++q) pos[H32.tile_patch[q]] = (int32_t)q;
    for (int e = 0; e < E; ++e) {
      pose_off[ii[e] + 1]++;
      pose_off[jj[e] + 1]++;
    }
    for (int f = 0; f < N; ++f) pose_off[f + 1] += pose_off[f];
    std::vector<int32_t> cur(pose_off.begin(), pose_off.end() - 1);
    for (int e = 0; e < E; ++e) {
      pose_src[cur[ii[e]]++] = 2 * e;
      pose_src[cur[jj[e]]++] = 2 * e + 1;
    }
    HIP_TRY(upload(c->pcount, pcount, st));
    HIP_TRY(upload(c->pedges, pedges, st));
    HIP_TRY(upload(c->pose_off, pose_off, st));
    HIP_TRY(upload(c->pose_src, pose_src, st));
    HIP_TRY(upload(c->patch_pos, pos, st));
    BatchInst one{};
    one.n_frames = N;
    one.n_fixed = nf;
    one.n_free = n_free;
    one.n_patches = P;
    one.n_edges = E;
    one.n_tiles = (int)H32.tiles.size();
    HIP_TRY(upload(c->one_inst, std::vector<BatchInst>{one}, st));
  }

  const size_t n = 6 * (size_t)n_free;
  const size_t nblk64 = (n + 63) / 64;
  auto mx = [&](long long a, long long b) { return (size_t)std::max(a, b); };
  HIP_TRY(ensure(c->part_S, std::max(H32.part_S * 4, H64.part_S * 8)));
  HIP_TRY(ensure(c->part_vec, std::max(H32.part_vec * 4, H64.part_vec * 8)));
  HIP_TRY(ensure(c->part_cost, mx(H32.tiles.size(), H64.tiles.size()) * 8));
  HIP_TRY(ensure(c->part_invalid, mx(H32.tiles.size(), H64.tiles.size()) * 4));
  HIP_TRY(ensure(c->U_s, std::max(H32.u_alloc * 4, H64.u_alloc * 8)));
  HIP_TRY(ensure(c->pscale_s, (size_t)P * 2 * 8));
  HIP_TRY(ensure(c->depth_s, (size_t)P * 8));
  HIP_TRY(ensure(c->xh_s, (size_t)P * 2 * 8));
  HIP_TRY(ensure(c->poses_a, (size_t)N * 7 * 8));
  HIP_TRY(ensure(c->poses_b, (size_t)N * 7 * 8));
  HIP_TRY(ensure(c->S, (n + 1) * n * 8));  // the float32 large path appends s as row n
  HIP_TRY(ensure(c->rhs, n * 8));
  HIP_TRY(ensure(c->dB, n * 8));
  HIP_TRY(ensure(c->d0, n * 8));
  HIP_TRY(ensure(c->dx, n * 8));
  HIP_TRY(ensure(c->wb, n * 8));
  HIP_TRY(ensure(c->wy, n * 8));
  HIP_TRY(ensure(c->sys_x, n * 8));
  HIP_TRY(ensure(c->sys_b, n * 8));
  HIP_TRY(ensure(c->Linv, nblk64 * 64 * 64 * 8));
  // the triangular chain's value words: two passes, up to two words per row
  if (c->chain_flags.bytes < chain_words_bytes(nblk64)) {
    HIP_TRY(ensure(c->chain_flags, chain_words_bytes(nblk64)));
    HIP_TRY(hipMemsetAsync(c->chain_flags.p, 0, c->chain_flags.bytes, st));
    HIP_TRY(hipStreamSynchronize(st));
    c->chain_epoch = 0;
  }
  HIP_TRY(ensure(c->edge_part, ((size_t)(E + 255) / 256) * 8));
  HIP_TRY(ensure(c->status, 2 * DPVBA_MAX_ITERS * 4));  // [MAX, 2 MAX): float64 fallback solves
  HIP_TRY(ensure(c->min_bits, 2 * DPVBA_MAX_ITERS * 4));
  HIP_TRY(ensure(c->S32, (n + 1) * n * 4));  // s appended as row n for the first solve
  HIP_TRY(ensure(c->x64, n * 8));
  HIP_TRY(ensure(c->r64, n * 8));
  HIP_TRY(ensure(c->rhs32, n * 4));
  HIP_TRY(ensure(c->c32, n * 4));
  HIP_TRY(ensure(c->d0_32, n * 4));
  HIP_TRY(ensure(c->mx_max, 16));
  HIP_TRY(ensure(c->mx_resid, DPVBA_MAX_ITERS * 8));
  HIP_TRY(ensure(c->mx_fb, DPVBA_MAX_ITERS * 4));
  HIP_TRY(ensure(c->mx_flag, 16));
  if (!c->host_flag) HIP_TRY(hipHostMalloc((void**)&c->host_flag, sizeof(int), hipHostMallocDefault));
  HIP_TRY(ensure(c->devrep, sizeof(dpvba_report)));
  HIP_TRY(backward_workspace(c, N, std::max((long long)H32.tile_patch.size(), (long long)H64.tile_patch.size()), E,
                             (int)n));

  c->N = N; c->P = P; c->E = E; c->p = g->patch_size; c->n_fixed = nf; c->n_free = n_free;
  c->ii = g->ii; c->jj = g->jj; c->kk = g->kk;
  c->analysed = true;
  return DPVBA_OK;
}

dpvba_status dpvba_analyze(dpvba_ctx* c, const dpvba_graph* g, void* stream) {
  return dpvba_analyze_ex(c, g, nullptr, stream);
}

}  // extern "C"

static dpvba_status check_analysed(const dpvba_ctx* c, const dpvba_graph* g) {
  if (!c->analysed) return DPVBA_ESTATE;
  if (g->n_frames != c->N || g->n_patches != c->P || g->n_edges != c->E || g->patch_size != c->p ||
      g->n_fixed != c->n_fixed || g->ii != c->ii || g->jj != c->jj || g->kk != c->kk)
    return DPVBA_ESTATE;
  return DPVBA_OK;
}

// Options of a numeric call; `extra` are the flag bits that call accepts
// besides the damping flag.
static dpvba_status check_opts(const dpvba_opts* o, uint32_t extra = 0) {
  if (!o) return DPVBA_EINVAL;
  if (o->n_iters < 0 || o->n_iters > DPVBA_MAX_ITERS) return DPVBA_EINVAL;
  if (!(o->lambda >= 0.0) || !(o->lambda < (double)FLT_MAX)) return DPVBA_EINVAL;
  if (!(o->z_min >= 0.0) || !(o->z_min < (double)FLT_MAX)) return DPVBA_EINVAL;
  if (o->precision != DPVBA_FP32 && o->precision != DPVBA_MIXED && o->precision != DPVBA_FP64) return DPVBA_EINVAL;
  const uint32_t mixed_only = DPVBA_FLAG_FORCE_FP64_CHOL | DPVBA_FLAG_NO_REFINE;
  if (o->flags & ~(DPVBA_FLAG_LEVENBERG | mixed_only | extra)) return DPVBA_EINVAL;
  if ((o->flags & mixed_only) && o->precision != DPVBA_MIXED) return DPVBA_EINVAL;
  return DPVBA_OK;
}

// Marquardt coefficient of the damping H~ = H + lam_diag Diag(H) + lambda I.
static double lam_diag_of(const dpvba_opts* o) {
  return (o->flags & DPVBA_FLAG_LEVENBERG) ? 0.0 : o->lambda;
}

// Per-call buffers of a solve: the context's workspace (ctx_ws), or slices
// of the static scratch (carve_ws, dpvba_solve_noalloc).
template <typename T>
struct SolveWs {
  T *part_S, *part_vec, *U_s, *pscale_s, *depth_s, *xh_s, *pbuf0, *pbuf1, *S, *rhs, *d0, *dx;
  double *part_cost, *edge_part;
  int *part_invalid, *status;
  unsigned int* min_bits;
  dpvba_report* devrep;
};

template <typename T>
static SolveWs<T> ctx_ws(dpvba_ctx* c) {
  SolveWs<T> w;
  w.part_S = (T*)c->part_S.p;
  w.part_vec = (T*)c->part_vec.p;
  w.U_s = (T*)c->U_s.p;
  w.pscale_s = (T*)c->pscale_s.p;
  w.depth_s = (T*)c->depth_s.p;
  w.xh_s = (T*)c->xh_s.p;
  w.pbuf0 = (T*)c->poses_a.p;
  w.pbuf1 = (T*)c->poses_b.p;
  w.S = (T*)c->S.p;
  w.rhs = (T*)c->rhs.p;
  w.d0 = (T*)c->d0.p;
  w.dx = (T*)c->dx.p;
  w.part_cost = (double*)c->part_cost.p;
  w.edge_part = (double*)c->edge_part.p;
  w.part_invalid = (int*)c->part_invalid.p;
  w.status = (int*)c->status.p;
  w.min_bits = (unsigned int*)c->min_bits.p;
  w.devrep = (dpvba_report*)c->devrep.p;
  return w;
}

// Lays the buffers of a single-launch solve of the analysed problem (plan
// tl, element type T) out from `base` at 256-byte boundaries; returns the
// bytes needed.  With base == nullptr only the size is computed.
template <typename T>
static size_t carve_ws(const dpvba_ctx* c, const Tiling& tl, unsigned char* base, SolveWs<T>* w) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* q = base ? base + off : nullptr;
    off += (std::max<size_t>(bytes, 16) + 255) & ~(size_t)255;
    return (void*)q;
  };
  const size_t n = 6 * (size_t)c->n_free, P = (size_t)c->P, N = (size_t)c->N;
  const size_t ts = sizeof(T);
  SolveWs<T> v;
  v.part_S = (T*)take((size_t)tl.part_S * ts);
  v.part_vec = (T*)take((size_t)tl.part_vec * ts);
  v.U_s = (T*)take((size_t)tl.u_alloc * ts);
  v.pscale_s = (T*)take(P * 2 * ts);
  v.depth_s = (T*)take(P * ts);
  v.xh_s = (T*)take(P * 2 * ts);
  v.pbuf0 = (T*)take(N * 7 * ts);
  v.pbuf1 = (T*)take(N * 7 * ts);
  v.S = (T*)take((n + 1) * n * ts);
  v.rhs = (T*)take(n * ts);
  v.d0 = (T*)take(n * ts);
  v.dx = (T*)take(n * ts);
  v.part_cost = (double*)take((size_t)tl.n_tiles * 8);
  v.edge_part = (double*)take(((size_t)c->E + 255) / 256 * 8);
  v.part_invalid = (int*)take((size_t)tl.n_tiles * 4);
  v.status = (int*)take(DPVBA_MAX_ITERS * 4);
  v.min_bits = (unsigned int*)take(DPVBA_MAX_ITERS * 4);
  v.devrep = (dpvba_report*)take(sizeof(dpvba_report));
  if (w) *w = v;
  return off;
}

template <typename T>
static IterArgs<T> make_iter_args(dpvba_ctx* c, const SolveWs<T>& w, const dpvba_graph* g, const Tiling& tl,
                                  const T* poses_cur, T* poses_next, const T* depth_in, T lambda, T z_min,
                                  T lam_diag, int* dev_err) {
  IterArgs<T> A{};
  A.lam_diag = lam_diag;
  A.dev_err = dev_err;
  A.host_err = c->host_err_dev;
  A.patches = g->patches;
  A.p = g->patch_size;
  A.target = g->target;
  A.weight = g->weight;
  A.fx = g->fx; A.fy = g->fy; A.cx = g->cx; A.cy = g->cy;
  A.z_min = z_min;
  A.lambda = lambda;
  A.n_frames = c->N;
  A.n_fixed = c->n_fixed;
  A.n_free = c->n_free;
  A.n_tiles = tl.n_tiles;
  A.poses_cur = poses_cur;
  A.poses_next = poses_next;
  A.depth_in = depth_in;
  A.depth_s = w.depth_s;
  A.xh_s = w.xh_s;
  A.U_s = w.U_s;
  A.pscale_s = w.pscale_s;
  A.tiles = (const TileInfo*)tl.tiles.p;
  A.tile_patch = (const int*)tl.tile_patch.p;
  A.slot_frame = (const int*)tl.slot_frame.p;
  A.slot_blk = (const int*)tl.slot_blk.p;
  A.edge_grid = (const int*)tl.edge_grid.p;
  A.blk_pose = (const int*)tl.blk_pose.p;
  A.part_S = w.part_S;
  A.part_vec = w.part_vec;
  A.part_cost = w.part_cost;
  A.part_invalid = w.part_invalid;
  A.s_off = (const int*)tl.s_off.p;
  A.s_src = (const int*)tl.s_src.p;
  A.v_off = (const int*)tl.v_off.p;
  A.v_src = (const int2*)tl.v_src.p;
  A.order = (const int*)tl.order.p;
  A.dx = w.dx;
  A.first = 1;
  return A;
}

template <typename T>
static IterArgs<T> make_iter_args(dpvba_ctx* c, const dpvba_graph* g, const Tiling& tl, const T* poses_cur,
                                  T* poses_next, const T* depth_in, T lambda, T z_min, T lam_diag, int* dev_err) {
  return make_iter_args<T>(c, ctx_ws<T>(c), g, tl, poses_cur, poses_next, depth_in, lambda, z_min, lam_diag,
                           dev_err);
}

template <typename T>
static bool use_small_path(const dpvba_ctx* c) {
  const int n = 6 * c->n_free;
  return n + 1 <= kSmallRows && small_solve_lds_bytes(n, (int)sizeof(T)) <= 160 * 1024;
}

// Failure word of the calls that run as several launches (cleared by their
// report initialisation).
static int* large_err(dpvba_ctx* c) { return (int*)c->dev_err.p + 8; }
static int* batch_err(dpvba_ctx* c) { return (int*)c->dev_err.p + 12; }

template <typename T>
static hipError_t reduced_impl(dpvba_ctx* c, const dpvba_graph* g, const T* poses, const T* depth, T lambda,
                               T lam_diag, T z_min, T* S, T* rhs, double* cost_out, hipStream_t st) {
  const Tiling& tl = c->tl[sizeof(T) == 8 ? 1 : 0];
  IterArgs<T> A = make_iter_args<T>(c, g, tl, poses, nullptr, depth, lambda, z_min, lam_diag, large_err(c));
  hipError_t e;
  {
    TraceScope ts(c, DPVBA_PHASE_ASSEMBLE, st);
    e = launch_tile_iterate<T>(A, tl.lds_bytes, st);
  }
  if (e != hipSuccess) return e;
  TraceScope ts(c, DPVBA_PHASE_GATHER, st);
  if (cost_out) {
    e = launch_report_reduce((const double*)c->part_cost.p, (const int*)c->part_invalid.p, tl.n_tiles, cost_out,
                             nullptr, st);
    if (e != hipSuccess) return e;
  }
  return launch_gather<T>((const T*)c->part_S.p, (const T*)c->part_vec.p, (const int*)tl.s_off.p,
                          (const int*)tl.s_src.p, (const int*)tl.v_off.p, (const int2*)tl.v_src.p, c->n_free, S,
                          rhs, (T*)c->dB.p, lambda, lam_diag, 1, (T*)c->d0.p, st, nullptr);
}

// Float32 tile assembly gathered in float64 (the DPVBA_MIXED system).
static hipError_t reduced_mixed_impl(dpvba_ctx* c, const dpvba_graph* g, const float* poses, const float* depth,
                                     float lambda, float lam_diag, float z_min, double* S, double* rhs,
                                     double* cost_out, hipStream_t st) {
  const Tiling& tl = c->tl[0];
  IterArgs<float> A = make_iter_args<float>(c, g, tl, poses, nullptr, depth, lambda, z_min, lam_diag, large_err(c));
  hipError_t e;
  {
    TraceScope ts(c, DPVBA_PHASE_ASSEMBLE, st);
    e = launch_tile_iterate<float>(A, tl.lds_bytes, st);
  }
  if (e != hipSuccess) return e;
  TraceScope ts(c, DPVBA_PHASE_GATHER, st);
  if (cost_out) {
    e = launch_report_reduce((const double*)c->part_cost.p, (const int*)c->part_invalid.p, tl.n_tiles, cost_out,
                             nullptr, st);
    if (e != hipSuccess) return e;
  }
  return launch_gather_as<float, double>((const float*)c->part_S.p, (const float*)c->part_vec.p,
                                         (const int*)tl.s_off.p, (const int*)tl.s_src.p, (const int*)tl.v_off.p,
                                         (const int2*)tl.v_src.p, c->n_free, S, rhs, (double*)c->dB.p,
                                         (double)lambda, (double)lam_diag, 1, (double*)c->d0.p, st, nullptr);
}

template <typename T>
static hipError_t solve_impl(dpvba_ctx* c, const dpvba_graph* g, T* poses, T* depth, const dpvba_opts* o,
                             dpvba_report* report, hipStream_t st, const SolveWs<T>* ws_in = nullptr) {
  const SolveWs<T> ws = ws_in ? *ws_in : ctx_ws<T>(c);
  const T lambda = (T)o->lambda, z_min = (T)o->z_min, lam_diag = (T)lam_diag_of(o);
  const Tiling& tl = c->tl[sizeof(T) == 8 ? 1 : 0];
  const int n = 6 * c->n_free;
  const int nit = o->n_iters;
  const bool small = use_small_path<T>(c);
  dpvba_report* dev = ws.devrep;
  int* status = ws.status;
  unsigned int* mb = ws.min_bits;
  T* pbuf[2] = {ws.pbuf0, ws.pbuf1};
  T* dx = ws.dx;
  // the large iterations solve in the system order (workspaces of the
  // context's own only)
  const int* perm = ws_in ? nullptr : sys_perm_of(c);
  // the float32 blocked factor takes s as row n of S: gather it there
  T* rhs_s = !ws_in && sizeof(T) == 4 && n > small_solve_max_n(4) ? ws.S + (size_t)n * n : ws.rhs;
  hipError_t e;
  // the call's failure word: that of the single launch's parity, else the large path's
  const int parity = (int)(c->small_launches & 1);
  int* err = small && nit > 0 ? (int*)c->dev_err.p + 4 * parity : large_err(c);
  if (small && nit > 0) {
    SmallArgs<T> S{};
    S.it = make_iter_args<T>(c, ws, g, tl, poses, pbuf[0], depth, lambda, z_min, lam_diag, err);
    S.poses_io = poses;
    S.depth_io = depth;
    S.pbuf0 = pbuf[0];
    S.pbuf1 = pbuf[1];
    S.Sp = ws.S;
    S.rhs = ws.rhs;
    S.d0 = ws.d0;
    S.status = status;
    S.min_bits = mb;
    S.cost = dev->cost;
    S.invalid = dev->n_invalid;
    S.n_iters = nit;
    S.bar = (unsigned int*)c->ticket.p + 8 * parity;
    S.bar_next = (unsigned int*)c->ticket.p + 8 * (1 - parity);
    S.err = err;
    S.err_next = (int*)c->dev_err.p + 4 * (1 - parity);
    const int lds_small = std::max(tl.lds_bytes, small_solve_lds_bytes(n, (int)sizeof(T)));
    int& cap = sizeof(T) == 8 ? c->coop_grid64 : c->coop_grid32;
    int& cap_lds = sizeof(T) == 8 ? c->coop_lds64 : c->coop_lds32;
    if (cap_lds != lds_small) {
      cap = small_solve_grid<T>(lds_small);
      cap_lds = lds_small;
    }
    const int grid = std::min(tl.n_tiles, cap);
    if (grid < 1) return hipErrorCooperativeLaunchTooLarge;
    TraceScope ts(c, DPVBA_PHASE_ASSEMBLE, st);
    e = launch_small_solve<T>(S, grid, lds_small, c->coop_launch, st);
    if (e != hipSuccess) return e;
    ++c->small_launches;
  }
  if (!small) {
    e = launch_report_init(status, mb, DPVBA_MAX_ITERS, st, err);
    if (e != hipSuccess) return e;
  }
  for (int it = 0; it < nit && !small; ++it) {
    const T* cur = it == 0 ? poses : pbuf[(it - 1) & 1];
    T* next = pbuf[it & 1];
    IterArgs<T> A = make_iter_args<T>(c, ws, g, tl, cur, next, depth, lambda, z_min, lam_diag, err);
    A.first = it == 0;
    A.dx_prev = it ? dx : nullptr;
    A.status_prev = it ? status + it - 1 : nullptr;
    {
      TraceScope ts(c, DPVBA_PHASE_ASSEMBLE, st);
      e = launch_tile_iterate<T>(A, tl.lds_bytes, st);
    }
    if (e != hipSuccess) return e;
    {
      TraceScope ts(c, DPVBA_PHASE_GATHER, st);
      e = launch_report_reduce(ws.part_cost, ws.part_invalid, tl.n_tiles, &dev->cost[it], &dev->n_invalid[it], st);
      if (e == hipSuccess)
        e = !ws_in ? gather_system<T>(c, tl, ws.part_S, ws.part_vec, ws.S, rhs_s, lambda, lam_diag, ws.d0, st)
                   : launch_gather<T>(ws.part_S, ws.part_vec, (const int*)tl.s_off.p, (const int*)tl.s_src.p,
                                    (const int*)tl.v_off.p, (const int2*)tl.v_src.p, c->n_free, ws.S, ws.rhs,
                                    (T*)c->dB.p, lambda, lam_diag, 0, ws.d0, st, nullptr);
    }
    if (e != hipSuccess) return e;
    {
      TraceScope ts(c, DPVBA_PHASE_FACTOR, st);
      e = launch_chol_solve<T>(ws.S, rhs_s, n, perm ? (T*)c->sys_x.p : dx, (T*)c->wy.p, (T*)c->Linv.p, ws.d0,
                               status + it, mb + it, (int*)c->chain_flags.p, next_epoch(c), err, c->host_err_dev, st,
                               c->coop_launch, reach_of(c, n));
    }
    if (e != hipSuccess) return e;
    {
      TraceScope ts(c, DPVBA_PHASE_RETRACT, st);
      // perm: the step leaves the system order here (stored into dx)
      e = launch_retract_copy<T>(cur, next, dx, c->n_fixed, c->N, status + it, st, perm ? (const T*)c->sys_x.p : nullptr,
                                 perm ? sys_pos_of(c) : nullptr);
    }
    if (e != hipSuccess) return e;
  }
  if (nit > 0 && !small) {
    TraceScope ts(c, DPVBA_PHASE_BACKSUB, st);
    e = launch_tile_finalize<T>((const TileInfo*)tl.tiles.p, tl.n_tiles, writeback_lds_bytes(tl, (int)sizeof(T)), (const int*)tl.tile_patch.p,
                                (const int*)tl.blk_pose.p, ws.U_s, ws.pscale_s, ws.depth_s, dx, status + nit - 1, 0, depth, pbuf[(nit - 1) & 1], poses,
                                c->N, st);
    if (e != hipSuccess) return e;
  }
  if (!report) return hipSuccess;
  {
    TraceScope ts_cost(c, DPVBA_PHASE_COST, st);
    e = launch_edge_cost<T, T>(poses, depth, g->patches, g->patch_size, g->ii, g->jj, g->kk, g->target, g->weight,
                               g->n_edges, (T)g->fx, (T)g->fy, (T)g->cx, (T)g->cy, z_min,
                               ws.edge_part, st);
  }
  if (e != hipSuccess) return e;
  e = launch_report_reduce(ws.edge_part, nullptr, (g->n_edges + 255) / 256, &dev->cost[nit], nullptr, st);
  if (e != hipSuccess) return e;
  e = launch_report_finalize(dev, status, mb, nit, err, st);
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(report, dev, sizeof(dpvba_report), hipMemcpyDeviceToHost, st);
}

// Refinement of the float32 Cholesky solve against the float64 residual:
// fixed number of steps, and the largest accepted relative residual.
constexpr int kRefineSteps = 2;
constexpr double kRefineTol = 1e-8;

// DPVBA_MIXED: float32 state and tile assembly, float64 gather of the
// shares, float32 Cholesky with float64 iterative refinement, float64
// Cholesky when refinement does not reach kRefineTol (decided on the host
// after one stream synchronisation per iteration, unless the fallback is
// forced by DPVBA_FLAG_FORCE_FP64_CHOL).
static hipError_t solve_mixed_impl(dpvba_ctx* c, const dpvba_graph* g, float* poses, float* depth,
                                   const dpvba_opts* o, dpvba_report* report, hipStream_t st) {
  const float lambda = (float)o->lambda, z_min = (float)o->z_min, lam_diag = (float)lam_diag_of(o);
  const bool force_fb = (o->flags & DPVBA_FLAG_FORCE_FP64_CHOL) != 0;
  const int n_refine = (o->flags & DPVBA_FLAG_NO_REFINE) ? 0 : kRefineSteps;
  int* err = large_err(c);
  const Tiling& tl = c->tl[0];
  const int n = 6 * c->n_free;
  const int nit = o->n_iters;
  dpvba_report* dev = (dpvba_report*)c->devrep.p;
  int* status = (int*)c->status.p;
  int* status64 = status + DPVBA_MAX_ITERS;
  unsigned int* mb = (unsigned int*)c->min_bits.p;
  unsigned int* mb64 = mb + DPVBA_MAX_ITERS;
  float* pbuf[2] = {(float*)c->poses_a.p, (float*)c->poses_b.p};
  float* dx = (float*)c->dx.p;
  double* S64 = (double*)c->S.p;
  double* s64 = (double*)c->rhs.p;
  double* d064 = (double*)c->d0.p;
  float* S32 = (float*)c->S32.p;
  float* Linv32 = (float*)c->Linv.p;
  double* x64 = (double*)c->x64.p;
  double* r64 = (double*)c->r64.p;
  float* rhs32 = (float*)c->rhs32.p;
  float* c32 = (float*)c->c32.p;
  float* d032 = (float*)c->d0_32.p;
  unsigned long long* maxes = (unsigned long long*)c->mx_max.p;
  double* resid = (double*)c->mx_resid.p;
  int* fb = (int*)c->mx_fb.p;
  hipError_t e;
  if ((e = launch_report_init(status, mb, 2 * DPVBA_MAX_ITERS, st, err)) != hipSuccess) return e;
  if ((e = launch_fill<double>(resid, DPVBA_MAX_ITERS, 0.0, st)) != hipSuccess) return e;
  if ((e = launch_fill<int>(fb, DPVBA_MAX_ITERS, 0, st)) != hipSuccess) return e;
  for (int it = 0; it < nit; ++it) {
    const float* cur = it == 0 ? poses : pbuf[(it - 1) & 1];
    float* next = pbuf[it & 1];
    IterArgs<float> A = make_iter_args<float>(c, g, tl, cur, next, depth, lambda, z_min, lam_diag, err);
    A.first = it == 0;
    A.dx_prev = it ? dx : nullptr;
    A.status_prev = it ? status + it - 1 : nullptr;
    {
      TraceScope ts(c, DPVBA_PHASE_ASSEMBLE, st);
      if ((e = launch_tile_iterate<float>(A, tl.lds_bytes, st)) != hipSuccess) return e;
    }
    {
      TraceScope ts(c, DPVBA_PHASE_GATHER, st);
      e = launch_report_reduce((const double*)c->part_cost.p, (const int*)c->part_invalid.p, tl.n_tiles,
                               &dev->cost[it], &dev->n_invalid[it], st);
      if (e == hipSuccess && n > kBatchMaxUnknowns) {  // small systems are gathered by the one-problem batch
        if (c->n_env > 0) {
          // the envelope's blocks and their mirror images; S64 zero elsewhere
          if (c->s_env_elem != 8) {
            if ((e = launch_fill<double>(S64, (long long)n * n, 0.0, st)) != hipSuccess) return e;
            c->s_env_elem = 8;
          }
          e = launch_gather_env_as<float, double>((const float*)c->part_S.p, (const float*)c->part_vec.p,
                                                  (const int*)tl.s_off.p, (const int*)tl.s_src.p,
                                                  (const int*)tl.v_off.p, (const int2*)tl.v_src.p, c->n_free,
                                                  (const int4*)c->env_blk.p, c->n_env, S64, s64, (double*)c->dB.p,
                                                  (double)lambda, (double)lam_diag, d064, st, sys_pos_of(c), 1);
        } else {
          e = launch_gather_as<float, double>((const float*)c->part_S.p, (const float*)c->part_vec.p,
                                              (const int*)tl.s_off.p, (const int*)tl.s_src.p, (const int*)tl.v_off.p,
                                              (const int2*)tl.v_src.p, c->n_free, S64, s64, (double*)c->dB.p,
                                              (double)lambda, (double)lam_diag, 1, d064, st, sys_pos_of(c));
          c->s_env_elem = 0;  // S now holds the whole float64 system
        }
      }
      if (e != hipSuccess) return e;
    }
    if (n > 0 && n <= kBatchMaxUnknowns) {
      // one workgroup: float32 panel factor, refinement against the float64
      // residual and the float64 fallback without leaving the kernel; it
      // also writes the step and retracts the poses
      BatchArgs<float> a{};
      a.inst = (const BatchInst*)c->one_inst.p;
      a.part_S = (const float*)c->part_S.p;
      a.part_vec = (const float*)c->part_vec.p;
      a.s_off = (const int*)tl.s_off.p;
      a.s_src = (const int*)tl.s_src.p;
      a.v_off = (const int*)tl.v_off.p;
      a.v_src = (const int2*)tl.v_src.p;
      a.lambda = (double)lambda;
      a.lam_diag = (double)lam_diag;
      a.n_refine = n_refine;
      a.force_fb = force_fb ? 1 : 0;
      a.poses_cur = cur;
      a.poses_next = next;
      a.dx = dx;
      a.status = status;
      a.min_bits = mb;
      a.refine_resid = resid;
      a.fallback = fb;
      a.stride = DPVBA_MAX_ITERS;
      a.it = it;
      a.scratch = S64;  // packed system, s and d0 (float64) of the one problem
      a.lds_factor = 1;
      bool lf = false;
      const int lds_solve = batch_solve_lds<float>(n, true, &lf);
      TraceScope ts(c, DPVBA_PHASE_FACTOR, st);
      if ((e = launch_batch_gather<float, double>(a, 1, n, st)) != hipSuccess) return e;
      if ((e = launch_batch_solve_mixed(a, 1, lds_solve, st)) != hipSuccess) return e;
      continue;
    }
    if (n > 0) {
      TraceScope ts(c, DPVBA_PHASE_FACTOR, st);
      const PanelPlan* env = c->n_env > 0 ? reach_of(c, n) : nullptr;  // envelope-limited conversion and residuals
      if (env && !c->s32_zeroed) {
        if ((e = launch_fill<float>(S32, (long long)n * n, 0.f, st)) != hipSuccess) return e;
        c->s32_zeroed = true;
      }
      if ((e = launch_lower_to_f32(S64, S32, n, st, env)) != hipSuccess) return e;
      if ((e = launch_convert<double, float>(d064, d032, n, st)) != hipSuccess) return e;
      // s rides along as row n: the factor leaves y = L^-1 s there, so the
      // first solve is the backward chain alone
      float* y32 = S32 + (size_t)n * n;
      if ((e = launch_convert<double, float>(s64, y32, n, st)) != hipSuccess) return e;
      if ((e = launch_chol_factor<float>(S32, n, n + 1, Linv32, d032, status + it, mb + it, st, reach_of(c, n))) !=
          hipSuccess)
        return e;
      if ((e = launch_chol_apply<float>(S32, n, Linv32, y32, c32, y32, (int*)c->chain_flags.p, next_epoch(c), err,
                                    c->host_err_dev, st, 1, c->coop_launch, reach_of(c, n))) != hipSuccess)
        return e;
      if ((e = launch_convert<float, double>(c32, x64, n, st)) != hipSuccess) return e;
      int* skip = (int*)c->mx_flag.p + 1;  // set on the device once the residual meets the tolerance
      for (int k = 0; k < n_refine; ++k) {
        if ((e = launch_residual64(S64, s64, x64, n, r64, maxes, st, env)) != hipSuccess) return e;
        // the first step is always taken; a later one only while needed
        if (k > 0 && (e = launch_refine_check(maxes, kRefineTol, skip, st)) != hipSuccess) return e;
        if ((e = launch_convert<double, float>(r64, rhs32, n, st)) != hipSuccess) return e;
        if ((e = launch_chol_apply<float>(S32, n, Linv32, rhs32, c32, (float*)c->wy.p, (int*)c->chain_flags.p,
                                      next_epoch(c), err, c->host_err_dev, st, 0, c->coop_launch, reach_of(c, n),
                                      k > 0 ? skip : nullptr)) != hipSuccess)
          return e;
        if ((e = launch_accumulate(x64, c32, n, st, k > 0 ? skip : nullptr)) != hipSuccess) return e;
      }
      if ((e = launch_residual64(S64, s64, x64, n, r64, maxes, st, env)) != hipSuccess) return e;
      if ((e = launch_refine_decide(maxes, status + it, kRefineTol, force_fb ? 1 : 0, resid + it, fb + it,
                                    (int*)c->mx_flag.p, st)) != hipSuccess)
        return e;
      bool run64 = force_fb;
      if (!force_fb) {
        if ((e = hipMemcpyAsync(c->host_flag, c->mx_flag.p, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess)
          return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        run64 = *c->host_flag != 0;
      }
      if (run64) {
        if ((e = launch_chol_solve<double>(S64, s64, n, x64, (double*)c->wy.p, (double*)c->Linv.p, d064, status64 + it,
                                           mb64 + it, (int*)c->chain_flags.p, next_epoch(c), err, c->host_err_dev,
                                           st, c->coop_launch, reach_of(c, n))) != hipSuccess)
          return e;
      }
      // the step leaves the system order (perm: through c32, free by now)
      const int* perm = sys_perm_of(c);
      if ((e = launch_step_to_f32(x64, perm ? c32 : dx, n, fb + it, status64 + it, status + it, st)) != hipSuccess)
        return e;
      if (perm && (e = launch_permute_blocks<float>(c32, dx, perm, c->n_free, 6, 0, st)) != hipSuccess) return e;
    }
    {
      TraceScope ts(c, DPVBA_PHASE_RETRACT, st);
      if ((e = launch_retract_copy<float>(cur, next, dx, c->n_fixed, c->N, status + it, st)) != hipSuccess) return e;
    }
  }
  if (nit > 0) {
    TraceScope ts(c, DPVBA_PHASE_BACKSUB, st);
    e = launch_tile_finalize<float>((const TileInfo*)tl.tiles.p, tl.n_tiles, writeback_lds_bytes(tl, 4),
                                    (const int*)tl.tile_patch.p, (const int*)tl.blk_pose.p, (const float*)c->U_s.p,
                                    (const float*)c->pscale_s.p, (const float*)c->depth_s.p, dx, status + nit - 1,
                                    0, depth, pbuf[(nit - 1) & 1], poses, c->N, st);
    if (e != hipSuccess) return e;
  }
  if (!report) return hipSuccess;
  {
    TraceScope ts_cost(c, DPVBA_PHASE_COST, st);
    e = launch_edge_cost<float, float>(poses, depth, g->patches, g->patch_size, g->ii, g->jj, g->kk, g->target,
                                       g->weight, g->n_edges, g->fx, g->fy, g->cx, g->cy, z_min,
                                       (double*)c->edge_part.p, st);
  }
  if (e != hipSuccess) return e;
  e = launch_report_reduce((const double*)c->edge_part.p, nullptr, (g->n_edges + 255) / 256, &dev->cost[nit], nullptr,
                           st);
  if (e != hipSuccess) return e;
  e = launch_report_finalize(dev, status, mb, nit, err, st, resid, fb);
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(report, dev, sizeof(dpvba_report), hipMemcpyDeviceToHost, st);
}

// Append one problem's tiling to the batch tiling, rebasing its indices
// into the packed arrays (frames, patches, edges, free poses) and into the
// concatenated share buffers and gather lists.
static bool append_tiling(HostTiling& H, const HostTiling& Hb, int b, int frame_begin, int patch_begin,
                          int edge_begin, int free_begin, BatchInst& I) {
  I.tile_begin = (int)H.tiles.size();
  I.n_tiles = (int)Hb.tiles.size();
  I.s_base = (int)H.s_off.size();
  I.v_base = (int)H.v_off.size();
  const long long tp0 = (long long)H.tile_patch.size(), sl0 = (long long)H.slot_frame.size();
  const long long g0 = (long long)H.edge_grid.size(), bp0 = (long long)H.blk_pose.size();
  const long long ps0 = H.part_S, pv0 = H.part_vec, u0 = H.u_alloc;
  const long long ss0 = (long long)H.s_src.size(), vs0 = (long long)H.v_src.size();
  if (g0 + (long long)Hb.edge_grid.size() > INT32_MAX || ps0 + Hb.part_S > INT32_MAX ||
      pv0 + Hb.part_vec > INT32_MAX || u0 + Hb.u_alloc > INT32_MAX)
    return false;
  for (TileInfo t : Hb.tiles) {
    t.frame += frame_begin;
    t.patch_begin += (int)tp0;
    t.slot_begin += (int)sl0;
    t.grid_begin += (int)g0;
    t.blk_begin += (int)bp0;
    t.part_begin += (int)ps0;
    t.vec_begin += (int)pv0;
    t.u_begin += (int)u0;
    t.inst = b;
    H.tiles.push_back(t);
  }
  for (int32_t k : Hb.tile_patch) H.tile_patch.push_back(k + patch_begin);
  for (int32_t f : Hb.slot_frame) H.slot_frame.push_back(f + frame_begin);
  for (int32_t x : Hb.slot_blk) H.slot_blk.push_back(x);
  for (int32_t e : Hb.edge_grid) H.edge_grid.push_back(e >= 0 ? e + edge_begin : -1);
  for (int32_t f : Hb.blk_pose) H.blk_pose.push_back(f + free_begin);
  for (int32_t o : Hb.s_off) H.s_off.push_back(o + (int)ss0);
  for (int32_t o : Hb.s_src) H.s_src.push_back(o + (int)ps0);
  for (int32_t o : Hb.v_off) H.v_off.push_back(o + (int)vs0);
  for (int2 o : Hb.v_src) H.v_src.push_back(make_int2(o.x + (int)pv0, o.y + (int)pv0));
  H.part_S += Hb.part_S;
  H.part_vec += Hb.part_vec;
  H.u_elems += Hb.u_elems;
  H.u_alloc += Hb.u_alloc;
  H.lds = std::max(H.lds, Hb.lds);
  H.max_w6 = std::max(H.max_w6, Hb.max_w6);
  H.max_k = std::max(H.max_k, Hb.max_k);
  return true;
}

static bool batch_sizes_ok(const dpvba_batch* b) {
  if (!b || b->n_problems < 1 || b->patch_size < 1 || (b->patch_size % 2) == 0) return false;
  if (!b->frame_off || !b->patch_off || !b->edge_off || !b->n_fixed) return false;
  if (!(b->fx != 0.f) || !(b->fy != 0.f)) return false;
  const int B = b->n_problems;
  if (b->frame_off[0] != 0 || b->patch_off[0] != 0 || b->edge_off[0] != 0) return false;
  for (int q = 0; q < B; ++q) {
    if (b->frame_off[q + 1] <= b->frame_off[q] || b->patch_off[q + 1] < b->patch_off[q] ||
        b->edge_off[q + 1] < b->edge_off[q])
      return false;
    const int N = b->frame_off[q + 1] - b->frame_off[q];
    if (b->n_fixed[q] < 0 || b->n_fixed[q] > N) return false;
  }
  if (b->frame_off[B] > (1 << 24) || b->patch_off[B] > (1 << 28) || b->edge_off[B] > (1 << 29)) return false;
  if (b->edge_off[B] > 0 && (!b->ii || !b->jj || !b->kk || !b->target || !b->weight)) return false;
  if (b->patch_off[B] > 0 && !b->patches) return false;
  return true;
}

// Workspace of dpvba_solve_backward for up to DPVBA_MAX_ITERS iterations in
// float64 (float32 uses a prefix of every buffer).
static hipError_t backward_workspace(dpvba_ctx* c, int N, long long ntp, long long E, int n) {
  const size_t ts = 8, np7 = 7 * (size_t)N, it = DPVBA_MAX_ITERS;
  hipError_t e;
  if ((e = ensure(c->bw_poses, (it + 1) * np7 * ts)) != hipSuccess) return e;
  if ((e = ensure(c->bw_depth, it * (size_t)ntp * ts)) != hipSuccess) return e;
  if ((e = ensure(c->bw_dx, it * (size_t)n * ts)) != hipSuccess) return e;
  if ((e = ensure(c->bw_pbar, np7 * ts)) != hipSuccess) return e;
  if ((e = ensure(c->bw_dbar, (size_t)ntp * ts)) != hipSuccess) return e;
  if ((e = ensure(c->bw_dxbar, (size_t)n * ts)) != hipSuccess) return e;
  if ((e = ensure(c->bw_rhs, (size_t)n * ts)) != hipSuccess) return e;
  if ((e = ensure(c->bw_up, (size_t)n * ts)) != hipSuccess) return e;
  if ((e = ensure(c->bw_ud, (size_t)ntp * ts)) != hipSuccess) return e;
  if ((e = ensure(c->bw_dd, (size_t)ntp * ts)) != hipSuccess) return e;
  if ((e = ensure(c->bw_edge, (size_t)E * 15 * ts)) != hipSuccess) return e;
  if ((e = ensure(c->bw_status, 2 * DPVBA_MAX_ITERS * 4)) != hipSuccess) return e;
  return ensure(c->bw_minbits, 2 * DPVBA_MAX_ITERS * 4);
}

// Adjoint of `n_iters` iterations started from (poses0, depth0): replays
// the iterations storing x_t and the pose steps, then walks them backwards
// (see adjoint.hip), recomputing each iteration's Schur system at x_t.
template <typename T>
static hipError_t backward_impl(dpvba_ctx* c, const dpvba_graph* g, const T* poses0, const T* depth0,
                                const dpvba_opts* o, const T* grad_poses, const T* grad_depth, T* grad_target,
                                T* grad_weight, hipStream_t st) {
  const T lambda = (T)o->lambda, z_min = (T)o->z_min, lam_diag = (T)lam_diag_of(o);
  const Tiling& tl = c->tl[sizeof(T) == 8 ? 1 : 0];
  const int N = c->N, nf = c->n_fixed, n = 6 * c->n_free, nit = o->n_iters, E = c->E;
  int* err = large_err(c);
  const long long ntp = tl.n_tp, np7 = 7LL * N;
  const size_t ts = sizeof(T);
  hipError_t e;
  if ((e = launch_fill<T>(grad_target, 2LL * E, (T)0, st)) != hipSuccess) return e;
  if ((e = launch_fill<T>(grad_weight, 2LL * E, (T)0, st)) != hipSuccess) return e;
  if (nit == 0) return hipSuccess;
  // workspace sized by the analysis (backward_workspace) for DPVBA_MAX_ITERS
  if (c->bw_poses.bytes < (size_t)(nit + 1) * np7 * ts || c->bw_depth.bytes < (size_t)nit * ntp * ts ||
      c->bw_edge.bytes < (size_t)E * 15 * ts)
    return hipErrorInvalidValue;
  T* Xp = (T*)c->bw_poses.p;
  T* Xd = (T*)c->bw_depth.p;
  T* DX = (T*)c->bw_dx.p;
  T* pbar = (T*)c->bw_pbar.p;
  T* dbar = (T*)c->bw_dbar.p;
  T* dxbar = (T*)c->bw_dxbar.p;
  T* urhs = (T*)c->bw_rhs.p;
  T* up = (T*)c->bw_up.p;
  T* ud = (T*)c->bw_ud.p;
  T* dd = (T*)c->bw_dd.p;
  T* exb = (T*)c->bw_edge.p;
  int* status = (int*)c->bw_status.p;  // [0, MAX): replayed steps, [MAX, 2 MAX): adjoint solves
  unsigned int* mb = (unsigned int*)c->bw_minbits.p;
  const TileInfo* tiles = (const TileInfo*)tl.tiles.p;
  if ((e = launch_report_init(status, mb, 2 * DPVBA_MAX_ITERS, st, err)) != hipSuccess) return e;
  if ((e = launch_copy<T>(poses0, Xp, np7, st)) != hipSuccess) return e;
  auto gather = [&]() {
    return gather_system<T>(c, tl, (const T*)c->part_S.p, (const T*)c->part_vec.p, (T*)c->S.p, (T*)c->rhs.p, lambda,
                            lam_diag, (T*)c->d0.p, st);
  };
  const int* perm = sys_perm_of(c);
  T* xs = (T*)c->sys_x.p;  // a solve's result in the system order
  T* bs = (T*)c->sys_b.p;  // a right-hand side in the system order
  // replay: x_0 .. x_T, depths d_0 .. d_{T-1} in tile order, steps of the poses
  for (int it = 0; it < nit; ++it) {
    T* xt = Xp + it * np7;
    IterArgs<T> A = make_iter_args<T>(c, g, tl, xt, nullptr, depth0, lambda, z_min, lam_diag, err);
    A.first = it == 0;
    A.dx_prev = it ? DX + (size_t)(it - 1) * n : nullptr;
    A.status_prev = it ? status + it - 1 : nullptr;
    if ((e = launch_tile_iterate<T>(A, tl.lds_bytes, st)) != hipSuccess) return e;
    if ((e = launch_copy<T>((const T*)c->depth_s.p, Xd + it * ntp, ntp, st)) != hipSuccess) return e;
    if ((e = gather()) != hipSuccess) return e;
    if ((e = launch_chol_solve<T>((T*)c->S.p, (const T*)c->rhs.p, n, perm ? xs : DX + (size_t)it * n, (T*)c->wy.p,
                                  (T*)c->Linv.p, (const T*)c->d0.p, status + it, mb + it, (int*)c->chain_flags.p,
                                  next_epoch(c), err, c->host_err_dev, st, c->coop_launch, reach_of(c, n))) !=
        hipSuccess)
      return e;
    if (perm && (e = launch_permute_blocks<T>(xs, DX + (size_t)it * n, perm, c->n_free, 6, 0, st)) != hipSuccess) return e;
    if ((e = launch_retract_copy<T>(xt, xt + np7, DX + (size_t)it * n, nf, N, status + it, st)) != hipSuccess)
      return e;
  }
  // adjoint of x_T
  if (grad_poses) e = launch_copy<T>(grad_poses, pbar, np7, st);
  else e = launch_fill<T>(pbar, np7, (T)0, st);
  if (e != hipSuccess) return e;
  if ((e = launch_depth_to_tile<T>(grad_depth, (const int*)tl.tile_patch.p, (int)ntp, dbar, st)) != hipSuccess)
    return e;
  for (int it = nit - 1; it >= 0; --it) {
    const T* xt = Xp + it * np7;
    const T* dx_t = DX + (size_t)it * n;
    const int* stt = status + it;
    if ((e = launch_retract_adjoint<T>(xt, dx_t, stt, nf, N, pbar, dxbar, st)) != hipSuccess) return e;
    IterArgs<T> A = make_iter_args<T>(c, g, tl, xt, nullptr, depth0, lambda, z_min, lam_diag, err);
    A.first = 0;
    A.dx_prev = nullptr;
    A.depth_s = Xd + it * ntp;
    if ((e = launch_tile_iterate<T>(A, tl.lds_bytes, st)) != hipSuccess) return e;
    if ((e = gather()) != hipSuccess) return e;
    if ((e = launch_adjoint_rhs<T>(tiles, tl.n_tiles, (const T*)c->U_s.p, (const T*)c->pscale_s.p, dbar,
                                   (T*)c->part_vec.p, (const int*)tl.v_off.p, (const int2*)tl.v_src.p, c->n_free,
                                   dxbar, stt, urhs, st)) != hipSuccess)
      return e;
    if (perm && (e = launch_permute_blocks<T>(urhs, bs, perm, c->n_free, 6, 1, st)) != hipSuccess) return e;
    if ((e = launch_chol_solve<T>((T*)c->S.p, perm ? bs : urhs, n, perm ? xs : up, (T*)c->wy.p, (T*)c->Linv.p,
                                  (const T*)c->d0.p, status + DPVBA_MAX_ITERS + it, mb + DPVBA_MAX_ITERS + it,
                                  (int*)c->chain_flags.p, next_epoch(c), err, c->host_err_dev, st, c->coop_launch,
                                  reach_of(c, n))) != hipSuccess)
      return e;
    if (perm && (e = launch_permute_blocks<T>(xs, up, perm, c->n_free, 6, 0, st)) != hipSuccess) return e;
    if ((e = launch_adjoint_backsub<T>(tiles, tl.n_tiles, tl.max_w6, (const int*)tl.blk_pose.p,
                                       (const T*)c->U_s.p, (const T*)c->pscale_s.p, dbar, up, dx_t, stt, ud, dd,
                                       st)) != hipSuccess)
      return e;
    if ((e = launch_edge_adjoint<T>(xt, Xd + it * ntp, (const int*)c->patch_pos.p, g->patches, g->patch_size, g->ii,
                                    g->jj, g->kk, g->target, g->weight, E, nf, (T)g->fx, (T)g->fy, (T)g->cx,
                                    (T)g->cy, z_min, lam_diag, up, ud, dx_t, dd, stt, grad_target, grad_weight, exb,
                                    st)) != hipSuccess)
      return e;
    if ((e = launch_adjoint_reduce<T>(exb, (const int*)c->pose_off.p, (const int*)c->pose_src.p, nf, N, pbar,
                                      (const int*)tl.tile_patch.p, (const int*)c->pcount.p,
                                      (const int*)c->pedges.p, (int)ntp, dbar, st)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

extern "C" {

dpvba_status dpvba_reproject(dpvba_ctx* c, const dpvba_graph* g, const float* poses, const float* inv_depth,
                             float z_min, float* coords, uint8_t* valid, void* stream) {
  if (!c || !graph_sizes_ok(g)) return DPVBA_EINVAL;
  if (!(z_min >= 0.f) || !(z_min < FLT_MAX)) return DPVBA_EINVAL;
  if (g->n_edges > 0 && (!poses || !inv_depth || !coords)) return DPVBA_EINVAL;
  if (recorded_failure(c)) return DPVBA_EDEVICE;
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(launch_reproject(poses, inv_depth, g->patches, g->patch_size, g->ii, g->jj, g->kk, g->n_edges, g->fx,
                           g->fy, g->cx, g->cy, z_min, coords, valid, (hipStream_t)stream));
  return DPVBA_OK;
}

dpvba_status dpvba_pgo_sim3(dpvba_ctx* c, int32_t n_frames, int32_t n_fixed, const double* poses, int32_t n_loops,
                            const int32_t* loop_j, const int32_t* loop_k, const double* loop_rel, int32_t n_iters,
                            double lambda, uint32_t flags, double* sims, double* cost, void* stream) {
  if (!c || n_frames < 1 || n_fixed < 0 || n_fixed > n_frames || n_loops < 0 || !poses || !sims) return DPVBA_EINVAL;
  if (n_iters < 0 || n_iters > DPVBA_MAX_PGO_ITERS || !(lambda >= 0.0) || !(lambda < 1e300)) return DPVBA_EINVAL;
  if (flags & ~DPVBA_FLAG_LEVENBERG) return DPVBA_EINVAL;
  if (n_loops > 0 && (!loop_j || !loop_k || !loop_rel)) return DPVBA_EINVAL;
  const int nf = n_frames - n_fixed;
  if ((long long)nf * 7 > 20000) return DPVBA_EINVAL;  // the dense system must stay a few GB
  for (int l = 0; l < n_loops; ++l)
    if (loop_j[l] < 0 || loop_j[l] >= n_frames || loop_k[l] < 0 || loop_k[l] >= n_frames || loop_j[l] == loop_k[l])
      return DPVBA_EINVAL;
  if (recorded_failure(c)) return DPVBA_EDEVICE;
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  // residual list: the n - 1 smoothness terms, then the loops
  const int E = n_frames - 1 + n_loops;
  std::vector<int32_t> ea(std::max(E, 1)), eb(std::max(E, 1));
  for (int e = 0; e < n_frames - 1; ++e) { ea[e] = e; eb[e] = e + 1; }
  for (int l = 0; l < n_loops; ++l) { ea[n_frames - 1 + l] = loop_j[l]; eb[n_frames - 1 + l] = loop_k[l]; }
  // order of the free poses in the normal equations: a reverse Cuthill-McKee
  // order where it shrinks the envelope (loop closures couple poses far
  // apart in time), else their own; pos[f] = block row of free pose f
  std::vector<int32_t> pos(std::max(nf, 0)), order;
  for (int f = 0; f < nf; ++f) pos[f] = f;
  if (nf > 0) {
    std::vector<std::vector<int32_t>> adj(nf);
    for (int e = 0; e < E; ++e) {
      const int fa = ea[e] - n_fixed, fb = eb[e] - n_fixed;
      if (fa >= 0 && fb >= 0 && fa != fb) {
        adj[fa].push_back(fb);
        adj[fb].push_back(fa);
      }
    }
    for (auto& a : adj) {
      std::sort(a.begin(), a.end());
      a.erase(std::unique(a.begin(), a.end()), a.end());
    }
    const std::vector<int32_t> cand = rcm_order(adj);
    std::vector<int32_t> cpos(nf);
    for (int p = 0; p < nf; ++p) cpos[cand[p]] = p;
    if (envelope_cost(first_coupled(adj, cpos)) < 0.9 * envelope_cost(first_coupled(adj, pos))) {
      order = cand;
      pos = cpos;
    }
  }
  // block lists of the free poses' normal equations (at their block rows),
  // contributions in residual order
  std::map<std::pair<int, int>, std::vector<int32_t>> blocks;
  std::vector<std::vector<int32_t>> pose_list(std::max(nf, 0));
  for (int e = 0; e < E; ++e) {
    const int fa = ea[e] - n_fixed, fb = eb[e] - n_fixed;
    const int pa = fa >= 0 ? pos[fa] : -1, pb = fb >= 0 ? pos[fb] : -1;
    if (fa >= 0) { blocks[{pa, pa}].push_back(4 * e + 0); pose_list[pa].push_back(2 * e); }
    if (fb >= 0) { blocks[{pb, pb}].push_back(4 * e + 3); pose_list[pb].push_back(2 * e + 1); }
    if (fa >= 0 && fb >= 0) {
      if (pa > pb) blocks[{pa, pb}].push_back(4 * e + 1);
      else blocks[{pb, pa}].push_back(4 * e + 2);
    }
  }
  std::vector<int32_t> blk_pq, blk_off{0}, blk_src, pose_off{0}, pose_src;
  for (auto& kv : blocks) {
    blk_pq.push_back(kv.first.first);
    blk_pq.push_back(kv.first.second);
    blk_src.insert(blk_src.end(), kv.second.begin(), kv.second.end());
    blk_off.push_back((int32_t)blk_src.size());
  }
  for (auto& l : pose_list) {
    pose_src.insert(pose_src.end(), l.begin(), l.end());
    pose_off.push_back((int32_t)pose_src.size());
  }
  const size_t n = 7 * (size_t)nf, nblk64 = (n + 63) / 64;
  if (nf > 0) {
    // envelope of the normal equations: each free pose's first coupled free pose
    std::vector<int32_t> fq(nf);
    for (int Pp = 0; Pp < nf; ++Pp) fq[Pp] = Pp;
    for (auto& kv : blocks) fq[kv.first.first] = std::min(fq[kv.first.first], kv.first.second);
    c->pg_plan.n = 0;
    HIP_TRY(build_plan(fq, 7, (int)n, c->pg_plan, st));
  }
  if (!order.empty()) HIP_TRY(upload(c->pg_perm, order, st));
  HIP_TRY(upload(c->pg_ea, ea, st));
  HIP_TRY(upload(c->pg_eb, eb, st));
  HIP_TRY(upload(c->pg_blk_pq, blk_pq, st));
  HIP_TRY(upload(c->pg_blk_off, blk_off, st));
  HIP_TRY(upload(c->pg_blk_src, blk_src, st));
  HIP_TRY(upload(c->pg_pose_off, pose_off, st));
  HIP_TRY(upload(c->pg_pose_src, pose_src, st));
  HIP_TRY(ensure(c->pg_C, (size_t)std::max(E, 1) * 13 * 8));
  HIP_TRY(ensure(c->pg_r, (size_t)std::max(E, 1) * 7 * 8));
  HIP_TRY(ensure(c->pg_J, (size_t)std::max(E, 1) * 7 * 14 * 8));
  HIP_TRY(ensure(c->pg_H, std::max<size_t>(n * n, 1) * 8));
  HIP_TRY(ensure(c->pg_rhs, std::max<size_t>(n, 1) * 8));
  HIP_TRY(ensure(c->pg_dx, std::max<size_t>(n, 1) * 8));
  HIP_TRY(ensure(c->pg_xs, std::max<size_t>(n, 1) * 8));
  HIP_TRY(ensure(c->pg_d0, std::max<size_t>(n, 1) * 8));
  HIP_TRY(ensure(c->pg_wy, std::max<size_t>(n, 1) * 8));
  HIP_TRY(ensure(c->pg_Linv, std::max<size_t>(nblk64, 1) * 64 * 64 * 8));
  if (c->pg_flags.bytes < chain_words_bytes(nblk64)) {
    HIP_TRY(ensure(c->pg_flags, chain_words_bytes(nblk64)));
    HIP_TRY(hipMemsetAsync(c->pg_flags.p, 0, c->pg_flags.bytes, st));
    c->pg_epoch = 0;
  }
  HIP_TRY(ensure(c->pg_status, (DPVBA_MAX_PGO_ITERS + 1) * 4));
  HIP_TRY(ensure(c->pg_mb, (DPVBA_MAX_PGO_ITERS + 1) * 4));
  HIP_TRY(ensure(c->pg_cost, (DPVBA_MAX_PGO_ITERS + 1) * 8));
  int* status = (int*)c->pg_status.p;
  double* costd = (double*)c->pg_cost.p;
  double* H = (double*)c->pg_H.p;
  const double lam_diag = (flags & DPVBA_FLAG_LEVENBERG) ? 0.0 : lambda;
  int* err = large_err(c);
  HIP_TRY(launch_report_init(status, (unsigned int*)c->pg_mb.p, DPVBA_MAX_PGO_ITERS + 1, st, err));
  HIP_TRY(launch_pgo_init(poses, n_frames, sims, loop_rel, n_loops, (double*)c->pg_C.p, st));
  for (int it = 0; it < n_iters; ++it) {
    HIP_TRY(launch_pgo_linearise(sims, (const double*)c->pg_C.p, (const int*)c->pg_ea.p, (const int*)c->pg_eb.p, E,
                                 (double*)c->pg_r.p, (double*)c->pg_J.p, costd + it, st));
    if (nf == 0) continue;
    HIP_TRY(launch_fill<double>(H, (long long)(n * n), 0.0, st));
    HIP_TRY(launch_pgo_normal((const double*)c->pg_J.p, (const double*)c->pg_r.p, (const int*)c->pg_blk_pq.p,
                              (const int*)c->pg_blk_off.p, (const int*)c->pg_blk_src.p, (int)blocks.size(),
                              (const int*)c->pg_pose_off.p, (const int*)c->pg_pose_src.p, nf, lambda, lam_diag, H,
                              (double*)c->pg_d0.p, (double*)c->pg_rhs.p, st));
    c->pg_epoch = c->pg_epoch >= 0x3fffffff ? 1 : c->pg_epoch + 1;
    const bool perm = !order.empty();
    HIP_TRY(launch_chol_solve<double>(H, (const double*)c->pg_rhs.p, (int)n, (double*)(perm ? c->pg_xs.p : c->pg_dx.p),
                                      (double*)c->pg_wy.p, (double*)c->pg_Linv.p, (const double*)c->pg_d0.p,
                                      status + it, (unsigned int*)c->pg_mb.p + it, (int*)c->pg_flags.p, c->pg_epoch,
                                      err, c->host_err_dev, st, c->coop_launch, &c->pg_plan.plan));
    if (perm)
      HIP_TRY(launch_permute_blocks<double>((const double*)c->pg_xs.p, (double*)c->pg_dx.p, (const int*)c->pg_perm.p,
                                            nf, 7, 0, st));
    HIP_TRY(launch_pgo_retract(sims, n_frames, n_fixed, (const double*)c->pg_dx.p, status + it, st));
  }
  HIP_TRY(launch_pgo_linearise(sims, (const double*)c->pg_C.p, (const int*)c->pg_ea.p, (const int*)c->pg_eb.p, E,
                               (double*)c->pg_r.p, (double*)c->pg_J.p, costd + n_iters, st));
  std::vector<int32_t> hs(DPVBA_MAX_PGO_ITERS + 1);
  std::vector<double> hc(DPVBA_MAX_PGO_ITERS + 1);
  HIP_TRY(hipMemcpyAsync(hs.data(), status, hs.size() * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(hc.data(), costd, hc.size() * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (cost)
    for (int it = 0; it <= n_iters; ++it) cost[it] = hc[it];
  if (recorded_failure(c)) return DPVBA_EDEVICE;
  for (int it = 0; it < n_iters; ++it)
    if (hs[it]) return DPVBA_ENOTPD;
  return DPVBA_OK;
}

dpvba_status dpvba_pgo_apply(dpvba_ctx* c, int32_t n_frames, const double* sims, const int32_t* patch_off,
                             float* poses, float* inv_depth, void* stream) {
  if (!c || n_frames < 0 || (n_frames > 0 && (!sims || !patch_off || !poses || !inv_depth))) return DPVBA_EINVAL;
  if (recorded_failure(c)) return DPVBA_EDEVICE;
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(launch_pgo_apply(sims, n_frames, patch_off, poses, inv_depth, (hipStream_t)stream));
  return DPVBA_OK;
}

dpvba_status dpvba_patch_correlation(dpvba_ctx* c, int32_t n_edges, int32_t patch_size, int32_t dim,
                                     const float* gmap, int32_t n_patches, const float* fmaps, int32_t n_maps,
                                     int32_t height, int32_t width, const int32_t* kk, const int32_t* jj,
                                     const float* coords, float* corr, void* stream) {
  if (!c || n_edges < 0 || patch_size < 1 || patch_size % 2 == 0 || patch_size > 15) return DPVBA_EINVAL;
  if (dim < 64 || dim > 256 || dim % 64 != 0 || n_patches < 0 || n_maps < 0 || height < 0 || width < 0)
    return DPVBA_EINVAL;
  if ((long long)height * width * dim > (1LL << 31)) return DPVBA_EINVAL;
  if (n_edges > 0 && (!gmap || !fmaps || !kk || !jj || !coords || !corr)) return DPVBA_EINVAL;
  if ((long long)n_edges * patch_size * patch_size > INT32_MAX) return DPVBA_EINVAL;
  if (recorded_failure(c)) return DPVBA_EDEVICE;
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(launch_patch_correlation(n_edges, patch_size, dim, gmap, n_patches, fmaps, n_maps, height, width, kk, jj,
                                   coords, corr, nullptr, c->host_err_dev, (hipStream_t)stream));
  return DPVBA_OK;
}

dpvba_status dpvba_proximity_edges(dpvba_ctx* c, const float* poses, int32_t n_frames, const int32_t* patch_off,
                                   int32_t first_recent, int32_t min_gap, float radius, int32_t max_targets,
                                   int32_t* counts, int32_t* targets, int64_t* edge_off, int32_t* ii, int32_t* jj,
                                   int32_t* kk, int64_t max_edges, int64_t* n_edges, void* stream) {
  if (!c || !n_edges || n_frames < 0 || !patch_off || !edge_off) return DPVBA_EINVAL;
  if (first_recent < 0 || first_recent > n_frames || min_gap < 0) return DPVBA_EINVAL;
  if (!(radius >= 0.f) || !(radius <= FLT_MAX)) return DPVBA_EINVAL;
  if (max_targets < 0 || max_targets > DPVBA_MAX_LOOP_TARGETS || max_edges < 0) return DPVBA_EINVAL;
  if (n_frames > 0 && (!poses || !counts || (max_targets > 0 && !targets))) return DPVBA_EINVAL;
  if (max_edges > 0 && (!ii || !jj || !kk)) return DPVBA_EINVAL;
  if (recorded_failure(c)) return DPVBA_EDEVICE;
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const float r2 = radius * radius;  // rounded to float, as the decisions are
  HIP_TRY(launch_proximity_edges(poses, n_frames, patch_off, first_recent, min_gap, r2, max_targets, counts, targets,
                                 (long long*)edge_off, ii, jj, kk, (long long)max_edges, st));
  long long total = 0;
  HIP_TRY(hipMemcpyAsync(&total, edge_off + n_frames, sizeof(total), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *n_edges = total;
  if (total > max_edges) {
    snprintf(c->err, sizeof(c->err), "dpvba_proximity_edges: %lld edges exceed max_edges %lld", total,
             (long long)max_edges);
    return DPVBA_ELIMIT;
  }
  return DPVBA_OK;
}

dpvba_status dpvba_reduced_system(dpvba_ctx* c, const dpvba_graph* g, const float* poses, const float* inv_depth,
                                  const dpvba_opts* o, void* S, void* s, double* cost, void* stream) {
  if (!c || !graph_sizes_ok(g)) return DPVBA_EINVAL;
  dpvba_status rc = check_opts(o);
  if (rc != DPVBA_OK) return rc;
  rc = check_analysed(c, g);
  if (rc != DPVBA_OK) return rc;
  if (!poses || (!inv_depth && c->P > 0) || (c->n_free > 0 && (!S || !s))) return DPVBA_EINVAL;
  if (recorded_failure(c)) return DPVBA_EDEVICE;
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  if (o->precision == DPVBA_FP64) {
    HIP_TRY(reduced_impl<double>(c, g, (const double*)(const void*)poses, (const double*)(const void*)inv_depth,
                                 (double)o->lambda, lam_diag_of(o), (double)o->z_min, (double*)S, (double*)s, cost,
                                 st));
  } else if (o->precision == DPVBA_MIXED) {
    HIP_TRY(reduced_mixed_impl(c, g, poses, inv_depth, (float)o->lambda, (float)lam_diag_of(o), (float)o->z_min,
                               (double*)S, (double*)s, cost, st));
  } else {
    HIP_TRY(reduced_impl<float>(c, g, poses, inv_depth, (float)o->lambda, (float)lam_diag_of(o), (float)o->z_min,
                                (float*)S, (float*)s, cost, st));
  }
  return DPVBA_OK;
}

dpvba_status dpvba_solve(dpvba_ctx* c, const dpvba_graph* g, float* poses, float* inv_depth, const dpvba_opts* o,
                         dpvba_report* report, void* stream) {
  if (!c || !graph_sizes_ok(g)) return DPVBA_EINVAL;
  dpvba_status rc = check_opts(o);
  if (rc != DPVBA_OK) return rc;
  rc = check_analysed(c, g);
  if (rc != DPVBA_OK) return rc;
  if (!poses || (!inv_depth && c->P > 0)) return DPVBA_EINVAL;
  if (recorded_failure(c)) return DPVBA_EDEVICE;
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  if (o->precision == DPVBA_FP64) {
    HIP_TRY(solve_impl<double>(c, g, (double*)(void*)poses, (double*)(void*)inv_depth, o, report, st));
  } else if (o->precision == DPVBA_MIXED) {
    HIP_TRY(solve_mixed_impl(c, g, poses, inv_depth, o, report, st));
  } else {
    HIP_TRY(solve_impl<float>(c, g, poses, inv_depth, o, report, st));
  }
  return DPVBA_OK;
}

dpvba_status dpvba_solve_noalloc(dpvba_ctx* c, const dpvba_graph* g, float* poses, float* inv_depth,
                                 const dpvba_opts* o, dpvba_report* report, void* stream) {
  if (!c || !graph_sizes_ok(g)) return DPVBA_EINVAL;
  dpvba_status rc = check_opts(o);
  if (rc != DPVBA_OK) return rc;
  if (o->precision == DPVBA_MIXED) return DPVBA_EINVAL;
  rc = check_analysed(c, g);
  if (rc != DPVBA_OK) return rc;
  if (!poses || (!inv_depth && c->P > 0)) return DPVBA_EINVAL;
  if (recorded_failure(c)) return DPVBA_EDEVICE;
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const bool f64 = o->precision == DPVBA_FP64;
  const bool small = f64 ? use_small_path<double>(c) : use_small_path<float>(c);
  if (!small || o->n_iters == 0) {
    snprintf(c->err, sizeof(c->err),
             "dpvba_solve_noalloc: %s", o->n_iters == 0 ? "n_iters must be >= 1"
                                                      : "reduced system beyond the single-launch solver (6 free poses + 1 > 96)");
    return o->n_iters == 0 ? DPVBA_EINVAL : DPVBA_ELIMIT;
  }
  unsigned char* base = (unsigned char*)scratch_ptr(c->device);
  if (!base) {
    const hipError_t e = c->device < kMaxScratchDevices ? g_scratch_err[c->device] : hipErrorInvalidDevice;
    record_error(c, e == hipSuccess ? hipErrorInvalidSymbol : e, "dpvba_solve_noalloc: static scratch address");
    return DPVBA_EHIP;
  }
  const Tiling& tl = c->tl[f64 ? 1 : 0];
  const size_t need = f64 ? carve_ws<double>(c, tl, nullptr, nullptr) : carve_ws<float>(c, tl, nullptr, nullptr);
  if (need > kScratchBytes) {
    snprintf(c->err, sizeof(c->err), "dpvba_solve_noalloc: workspace of %zu bytes exceeds the static scratch of %zu",
             need, kScratchBytes);
    return DPVBA_ELIMIT;
  }
  if (f64) {
    SolveWs<double> w;
    carve_ws<double>(c, tl, base, &w);
    HIP_TRY(solve_impl<double>(c, g, (double*)(void*)poses, (double*)(void*)inv_depth, o, report, st, &w));
  } else {
    SolveWs<float> w;
    carve_ws<float>(c, tl, base, &w);
    HIP_TRY(solve_impl<float>(c, g, poses, inv_depth, o, report, st, &w));
  }
  return DPVBA_OK;
}

dpvba_status dpvba_solve_backward(dpvba_ctx* c, const dpvba_graph* g, const float* poses0,
                                  const float* inv_depth0, const dpvba_opts* o, const float* grad_poses,
                                  const float* grad_inv_depth, float* grad_target, float* grad_weight,
                                  void* stream) {
  if (!c || !graph_sizes_ok(g)) return DPVBA_EINVAL;
  dpvba_status rc = check_opts(o);
  if (rc != DPVBA_OK) return rc;
  rc = check_analysed(c, g);
  if (rc != DPVBA_OK) return rc;
  if (!poses0 || (!inv_depth0 && c->P > 0)) return DPVBA_EINVAL;
  if (c->E > 0 && (!grad_target || !grad_weight)) return DPVBA_EINVAL;
  if (o->precision == DPVBA_MIXED) return DPVBA_EINVAL;
  if (recorded_failure(c)) return DPVBA_EDEVICE;
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  if (o->precision == DPVBA_FP64) {
    HIP_TRY(backward_impl<double>(c, g, (const double*)(const void*)poses0, (const double*)(const void*)inv_depth0,
                                  o, (const double*)(const void*)grad_poses,
                                  (const double*)(const void*)grad_inv_depth, (double*)(void*)grad_target,
                                  (double*)(void*)grad_weight, st));
  } else {
    HIP_TRY(backward_impl<float>(c, g, poses0, inv_depth0, o, grad_poses, grad_inv_depth, grad_target, grad_weight,
                                 st));
  }
  return DPVBA_OK;
}

}  // extern "C"

// Runs fn(i, stream_i) for the n contexts concurrently: each on its own
// stream, after the work already enqueued on `st`, and makes `st` wait for
// all of them.  The contexts must be distinct (a context's workspace serves
// one call at a time) and on one device.  Returns the first failure; the
// joins are enqueued whatever happens.
template <typename F>
static dpvba_status fan_out(int32_t n, dpvba_ctx* const* ctxs, hipStream_t st, F&& fn) {
  if (n < 1 || !ctxs) return DPVBA_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i] || ctxs[i]->device != ctxs[0]->device) return DPVBA_EINVAL;
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return DPVBA_EINVAL;
  }
  dpvba_ctx* c = ctxs[0];  // failures of the shared steps are recorded here
  HIP_TRY(hipSetDevice(c->device));
  for (int i = 0; i < n; ++i) {
    dpvba_ctx* ci = ctxs[i];
    if (!ci->aux) HIP_TRY(hipStreamCreateWithFlags(&ci->aux, hipStreamNonBlocking));
    if (!ci->aux_start) HIP_TRY(hipEventCreateWithFlags(&ci->aux_start, hipEventDisableTiming));
    if (!ci->aux_done) HIP_TRY(hipEventCreateWithFlags(&ci->aux_done, hipEventDisableTiming));
  }
  HIP_TRY(hipEventRecord(c->aux_start, st));
  dpvba_status first = DPVBA_OK;
  for (int i = 0; i < n; ++i) {
    dpvba_ctx* ci = ctxs[i];
    HIP_TRY(hipStreamWaitEvent(ci->aux, c->aux_start, 0));
    // launches that wait for other workgroups of their grid go cooperative:
    // concurrent grids could otherwise hold the slots a waiting grid needs
    const bool coop = ci->coop_launch;
    ci->coop_launch = true;
    const dpvba_status rc = fn(i, (void*)ci->aux);
    ci->coop_launch = coop;
    if (rc != DPVBA_OK && first == DPVBA_OK) first = rc;
    HIP_TRY(hipEventRecord(ci->aux_done, ci->aux));
    HIP_TRY(hipStreamWaitEvent(st, ci->aux_done, 0));
  }
  return first;
}

extern "C" {

dpvba_status dpvba_solve_many(int32_t n, dpvba_ctx* const* ctxs, const dpvba_graph* graphs, float* const* poses,
                              float* const* inv_depth, const dpvba_opts* opts, dpvba_report* reports, void* stream) {
  if (!graphs || !poses || !inv_depth) return DPVBA_EINVAL;
  return fan_out(n, ctxs, (hipStream_t)stream, [&](int i, void* s) {
    return dpvba_solve(ctxs[i], &graphs[i], poses[i], inv_depth[i], opts, reports ? &reports[i] : nullptr, s);
  });
}

dpvba_status dpvba_solve_backward_many(int32_t n, dpvba_ctx* const* ctxs, const dpvba_graph* graphs,
                                       const float* const* poses0, const float* const* inv_depth0,
                                       const dpvba_opts* opts, const float* const* grad_poses,
                                       const float* const* grad_inv_depth, float* const* grad_target,
                                       float* const* grad_weight, void* stream) {
  if (!graphs || !poses0 || !inv_depth0 || !grad_target || !grad_weight) return DPVBA_EINVAL;
  return fan_out(n, ctxs, (hipStream_t)stream, [&](int i, void* s) {
    return dpvba_solve_backward(ctxs[i], &graphs[i], poses0[i], inv_depth0[i], opts,
                                grad_poses ? grad_poses[i] : nullptr, grad_inv_depth ? grad_inv_depth[i] : nullptr,
                                grad_target[i], grad_weight[i], s);
  });
}

}  // extern "C"

// Iterations of an analysed batch (one precision; see dpvba_solve_batch).
template <typename T>
static hipError_t batch_impl(dpvba_ctx* c, const dpvba_batch* b, T* poses, T* depth, const dpvba_opts* o,
                             bool mixed, hipStream_t st) {
  auto& B = c->bt;
  const int ti = sizeof(T) == 8 ? 1 : 0;
  const Tiling& tl = B.tl[ti];
  const T lambda = (T)o->lambda, z_min = (T)o->z_min, lam_diag = (T)lam_diag_of(o);
  const int nit = o->n_iters;
  const int stride = DPVBA_MAX_ITERS;
  int* status = (int*)B.status.p;
  unsigned int* mb = (unsigned int*)B.min_bits.p;
  T* pbuf[2] = {(T*)c->poses_a.p, (T*)c->poses_b.p};
  int* err = batch_err(c);
  hipError_t e;
  if ((e = launch_report_init(status, mb, B.B * stride, st, err)) != hipSuccess) return e;
  bool lds_factor = false;
  const int lds_solve = batch_solve_lds<T>(B.n_max, mixed, &lds_factor);
  for (int it = 0; it < nit; ++it) {
    const T* cur = it == 0 ? poses : pbuf[(it - 1) & 1];
    T* next = pbuf[it & 1];
    IterArgs<T> A{};
    A.patches = b->patches;
    A.p = b->patch_size;
    A.target = b->target;
    A.weight = b->weight;
    A.fx = b->fx; A.fy = b->fy; A.cx = b->cx; A.cy = b->cy;
    A.z_min = z_min;
    A.lambda = lambda;
    A.lam_diag = lam_diag;
    A.dev_err = err;
    A.host_err = c->host_err_dev;
    A.n_tiles = tl.n_tiles;
    A.poses_cur = cur;
    A.depth_in = depth;
    A.depth_s = (T*)c->depth_s.p;
    A.xh_s = (T*)c->xh_s.p;
    A.U_s = (T*)c->U_s.p;
    A.pscale_s = (T*)c->pscale_s.p;
    A.tiles = (const TileInfo*)tl.tiles.p;
    A.tile_patch = (const int*)tl.tile_patch.p;
    A.slot_frame = (const int*)tl.slot_frame.p;
    A.slot_blk = (const int*)tl.slot_blk.p;
    A.edge_grid = (const int*)tl.edge_grid.p;
    A.blk_pose = (const int*)tl.blk_pose.p;
    A.part_S = (T*)c->part_S.p;
    A.part_vec = (T*)c->part_vec.p;
    A.part_cost = (double*)c->part_cost.p;
    A.part_invalid = (int*)c->part_invalid.p;
    A.first = it == 0;
    A.dx_prev = it ? (const T*)c->dx.p : nullptr;
    A.status_prev = it ? status + it - 1 : nullptr;
    A.status_stride = stride;
    {
      TraceScope ts(c, DPVBA_PHASE_ASSEMBLE, st);
      if ((e = launch_tile_iterate<T>(A, tl.lds_bytes, st)) != hipSuccess) return e;
    }
    if ((e = launch_batch_cost((const BatchInst*)B.inst[ti].p, B.B, (const double*)c->part_cost.p,
                               (const int*)c->part_invalid.p, (dpvba_report*)B.reps.p, it, st)) != hipSuccess)
      return e;
    BatchArgs<T> a{};
    a.inst = (const BatchInst*)B.inst[ti].p;
    a.part_S = (const T*)c->part_S.p;
    a.part_vec = (const T*)c->part_vec.p;
    a.s_off = (const int*)tl.s_off.p;
    a.s_src = (const int*)tl.s_src.p;
    a.v_off = (const int*)tl.v_off.p;
    a.v_src = (const int2*)tl.v_src.p;
    a.lambda = (double)lambda;
    a.lam_diag = (double)lam_diag;
    a.n_refine = (o->flags & DPVBA_FLAG_NO_REFINE) ? 0 : 2;
    a.force_fb = (o->flags & DPVBA_FLAG_FORCE_FP64_CHOL) ? 1 : 0;
    a.poses_cur = cur;
    a.poses_next = next;
    a.dx = (T*)c->dx.p;
    a.status = status;
    a.min_bits = mb;
    a.refine_resid = (double*)B.refine.p;
    a.fallback = (int*)B.fallback.p;
    a.stride = stride;
    a.it = it;
    a.scratch = (double*)B.scratch_buf.p;
    a.lds_factor = lds_factor ? 1 : 0;
    {
      TraceScope tg(c, DPVBA_PHASE_GATHER, st);
      if constexpr (sizeof(T) == 4)
        e = mixed ? launch_batch_gather<float, double>(a, B.B, B.n_max, st)
                  : launch_batch_gather<float, float>(a, B.B, B.n_max, st);
      else
        e = launch_batch_gather<double, double>(a, B.B, B.n_max, st);
      if (e != hipSuccess) return e;
    }
    TraceScope ts(c, DPVBA_PHASE_FACTOR, st);
    if constexpr (sizeof(T) == 4) {
      if (mixed) e = launch_batch_solve_mixed(a, B.B, lds_solve, st);
      else e = launch_batch_solve<T>(a, B.B, lds_solve, st);
    } else {
      e = launch_batch_solve<T>(a, B.B, lds_solve, st);
    }
    if (e != hipSuccess) return e;
  }
  if (nit > 0) {
    TraceScope ts(c, DPVBA_PHASE_BACKSUB, st);
    e = launch_tile_finalize<T>((const TileInfo*)tl.tiles.p, tl.n_tiles, writeback_lds_bytes(tl, (int)sizeof(T)), (const int*)tl.tile_patch.p,
                                (const int*)tl.blk_pose.p, (const T*)c->U_s.p, (const T*)c->pscale_s.p,
                                (const T*)c->depth_s.p, (const T*)c->dx.p, status + nit - 1, stride, depth,
                                pbuf[(nit - 1) & 1], poses, B.N, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
static hipError_t batch_report(dpvba_ctx* c, const dpvba_batch* b, const T* poses, const T* depth,
                               const dpvba_opts* o, bool mixed, dpvba_report* reports, hipStream_t st) {
  auto& B = c->bt;
  const int ti = sizeof(T) == 8 ? 1 : 0;
  hipError_t e = launch_batch_report<T>((const BatchInst*)B.inst[ti].p, B.B, poses, depth, b->patches, b->patch_size,
                                        b->ii, b->jj, b->kk, b->target, b->weight, (T)b->fx, (T)b->fy, (T)b->cx,
                                        (T)b->cy, (T)o->z_min, (const int*)B.status.p,
                                        (const unsigned int*)B.min_bits.p, mixed ? (const double*)B.refine.p : nullptr,
                                        mixed ? (const int*)B.fallback.p : nullptr, DPVBA_MAX_ITERS, o->n_iters,
                                        (dpvba_report*)B.reps.p, st);
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(reports, B.reps.p, sizeof(dpvba_report) * (size_t)B.B, hipMemcpyDeviceToHost, st);
}

extern "C" {

dpvba_status dpvba_analyze_batch(dpvba_ctx* c, const dpvba_batch* b, const int32_t* tile_patches, void* stream) {
  if (!c || !batch_sizes_ok(b)) return DPVBA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(c->device));
  auto& Bt = c->bt;
  Bt.analysed = false;
  if (Bt.exec) {
    HIP_TRY(hipGraphExecDestroy(Bt.exec));
    Bt.exec = nullptr;
  }
  const int NB = b->n_problems;
  const int N = b->frame_off[NB], P = b->patch_off[NB], E = b->edge_off[NB];
  std::vector<int32_t> ii(E), jj(E), kk(E);
  if (E) {
    HIP_TRY(hipMemcpyAsync(ii.data(), b->ii, (size_t)E * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(jj.data(), b->jj, (size_t)E * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(kk.data(), b->kk, (size_t)E * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  {
    bool ok = true;
    HIP_TRY(inputs_valid(b->target, b->weight, E, st, &ok));
    if (!ok) return DPVBA_EINVAL;
  }
  HostTiling H[2];
  std::vector<BatchInst> inst[2];
  inst[0].resize(NB);
  inst[1].resize(NB);
  long long free_begin = 0, scratch = 0;
  int n_max = 0;
  for (int q = 0; q < NB; ++q) {
    const int f0 = b->frame_off[q], Nq = b->frame_off[q + 1] - f0;
    const int p0 = b->patch_off[q], Pq = b->patch_off[q + 1] - p0;
    const int e0 = b->edge_off[q], Eq = b->edge_off[q + 1] - e0;
    const int nf = b->n_fixed[q];
    ProblemIndex X;
    if (!index_problem(Nq, Pq, Eq, ii.data() + e0, jj.data() + e0, kk.data() + e0, X)) return DPVBA_EINVAL;
    std::vector<int32_t> jq(jj.begin() + e0, jj.begin() + e0 + Eq);
    const int kcap32 = (tile_patches && tile_patches[q] > 0) ? tile_patches[q] : kDefaultTilePatches32;
    for (int t = 0; t < 2; ++t) {
      HostTiling Hq;
      if (!plan_tiling(Nq, nf, jq, X.pcount, X.pedges, X.frame_patches, t ? kDefaultTilePatches64 : kcap32,
                       t ? 8 : 4, Hq))
        return DPVBA_EINVAL;
      BatchInst& I = inst[t][q];
      I.frame_begin = f0;
      I.n_frames = Nq;
      I.n_fixed = nf;
      I.free_begin = (int)free_begin;
      I.n_free = Nq - nf;
      I.patch_begin = p0;
      I.n_patches = Pq;
      I.edge_begin = e0;
      I.n_edges = Eq;
      I.scratch_off = scratch;
      if (!append_tiling(H[t], Hq, q, f0, p0, e0, (int)free_begin, I)) return DPVBA_EINVAL;
    }
    const long long n = 6LL * (Nq - nf);
    if (n > kBatchMaxUnknowns) return DPVBA_EINVAL;
    n_max = std::max(n_max, (int)n);
    scratch += n * (n + 1) / 2 + 2 * n;
    free_begin += Nq - nf;
  }
  // the per-problem solve keeps a float32 factor of the widest problem in shared memory
  if (n_max > 0) {
    bool lf = false;
    if (batch_solve_lds<float>(n_max, true, &lf) > 150 * 1024) return DPVBA_EINVAL;
  }
  HIP_TRY(upload_tiling(Bt.tl[0], H[0], st));
  HIP_TRY(upload_tiling(Bt.tl[1], H[1], st));
  HIP_TRY(upload(Bt.inst[0], inst[0], st));
  HIP_TRY(upload(Bt.inst[1], inst[1], st));
  const size_t nfree6 = 6 * (size_t)free_begin;
  HIP_TRY(ensure(c->part_S, std::max(H[0].part_S * 4, H[1].part_S * 8)));
  HIP_TRY(ensure(c->part_vec, std::max(H[0].part_vec * 4, H[1].part_vec * 8)));
  HIP_TRY(ensure(c->part_cost, std::max(H[0].tiles.size(), H[1].tiles.size()) * 8));
  HIP_TRY(ensure(c->part_invalid, std::max(H[0].tiles.size(), H[1].tiles.size()) * 4));
  HIP_TRY(ensure(c->U_s, std::max(H[0].u_alloc * 4, H[1].u_alloc * 8)));
  HIP_TRY(ensure(c->pscale_s, (size_t)P * 2 * 8));
  HIP_TRY(ensure(c->depth_s, (size_t)P * 8));
  HIP_TRY(ensure(c->xh_s, (size_t)P * 2 * 8));
  HIP_TRY(ensure(c->poses_a, (size_t)N * 7 * 8));
  HIP_TRY(ensure(c->poses_b, (size_t)N * 7 * 8));
  HIP_TRY(ensure(c->dx, nfree6 * 8));
  HIP_TRY(ensure(Bt.status, (size_t)NB * DPVBA_MAX_ITERS * 4));
  HIP_TRY(ensure(Bt.min_bits, (size_t)NB * DPVBA_MAX_ITERS * 4));
  HIP_TRY(ensure(Bt.refine, (size_t)NB * DPVBA_MAX_ITERS * 8));
  HIP_TRY(ensure(Bt.fallback, (size_t)NB * DPVBA_MAX_ITERS * 4));
  HIP_TRY(ensure(Bt.reps, (size_t)NB * sizeof(dpvba_report)));
  HIP_TRY(ensure(Bt.scratch_buf, (size_t)scratch * 8));
  Bt.B = NB;
  Bt.p = b->patch_size;
  Bt.N = N;
  Bt.P = P;
  Bt.E = E;
  Bt.n_max = n_max;
  Bt.n_free = free_begin;
  Bt.scratch = scratch;
  Bt.ii = b->ii;
  Bt.jj = b->jj;
  Bt.kk = b->kk;
  Bt.frame_off.assign(b->frame_off, b->frame_off + NB + 1);
  Bt.patch_off.assign(b->patch_off, b->patch_off + NB + 1);
  Bt.edge_off.assign(b->edge_off, b->edge_off + NB + 1);
  Bt.n_fixed.assign(b->n_fixed, b->n_fixed + NB);
  Bt.key.clear();
  Bt.analysed = true;
  return DPVBA_OK;
}

dpvba_status dpvba_solve_batch(dpvba_ctx* c, const dpvba_batch* b, float* poses, float* inv_depth,
                               const dpvba_opts* o, dpvba_report* reports, void* stream) {
  if (!c || !batch_sizes_ok(b) || !o) return DPVBA_EINVAL;
  auto& Bt = c->bt;
  if (!Bt.analysed) return DPVBA_ESTATE;
  const int NB = b->n_problems;
  if (NB != Bt.B || b->patch_size != Bt.p || b->ii != Bt.ii || b->jj != Bt.jj || b->kk != Bt.kk ||
      !std::equal(Bt.frame_off.begin(), Bt.frame_off.end(), b->frame_off) ||
      !std::equal(Bt.patch_off.begin(), Bt.patch_off.end(), b->patch_off) ||
      !std::equal(Bt.edge_off.begin(), Bt.edge_off.end(), b->edge_off) ||
      !std::equal(Bt.n_fixed.begin(), Bt.n_fixed.end(), b->n_fixed))
    return DPVBA_ESTATE;
  const bool graph = (o->flags & DPVBA_FLAG_GRAPH) != 0;
  dpvba_status rc = check_opts(o, DPVBA_FLAG_GRAPH);
  if (rc != DPVBA_OK) return rc;
  if (!poses || (!inv_depth && Bt.P > 0)) return DPVBA_EINVAL;
  if (recorded_failure(c)) return DPVBA_EDEVICE;
  if (graph && !stream) return DPVBA_EINVAL;
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const bool mixed = o->precision == DPVBA_MIXED;
  const bool f64 = o->precision == DPVBA_FP64;
  auto enqueue = [&]() -> hipError_t {
    if (f64) return batch_impl<double>(c, b, (double*)(void*)poses, (double*)(void*)inv_depth, o, false, st);
    return batch_impl<float>(c, b, poses, inv_depth, o, mixed, st);
  };
  if (graph && !c->tracing) {
    // everything the recorded launches bake in: the caller's pointers, the
    // options, the camera, the stream, and the workspace addresses (any
    // reallocation of a workspace buffer, by either analysis, changes the
    // generation)
    double lam = o->lambda, zm = o->z_min;
    uint64_t lb, zb;
    std::memcpy(&lb, &lam, 8);
    std::memcpy(&zb, &zm, 8);
    float cam[4] = {b->fx, b->fy, b->cx, b->cy};
    uint64_t cb[2];
    std::memcpy(cb, cam, 16);
    std::vector<uint64_t> key = {(uint64_t)(uintptr_t)poses, (uint64_t)(uintptr_t)inv_depth,
                                 (uint64_t)(uintptr_t)b->patches, (uint64_t)(uintptr_t)b->target,
                                 (uint64_t)(uintptr_t)b->weight, (uint64_t)o->n_iters, (uint64_t)o->precision, lb,
                                 zb, (uint64_t)o->flags, cb[0], cb[1], (uint64_t)(uintptr_t)st,
                                 g_workspace_generation};
    if (!Bt.exec || key != Bt.key) {
      if (Bt.exec) {
        HIP_TRY(hipGraphExecDestroy(Bt.exec));
        Bt.exec = nullptr;
      }
      HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
      hipError_t e = enqueue();
      hipGraph_t gr = nullptr;
      hipError_t e2 = hipStreamEndCapture(st, &gr);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        HIP_TRY(e != hipSuccess ? e : e2);
      }
      hipError_t e3 = hipGraphInstantiate(&Bt.exec, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      HIP_TRY(e3);
      Bt.key = key;
    }
    HIP_TRY(hipGraphLaunch(Bt.exec, st));
  } else {
    HIP_TRY(enqueue());
  }
  if (reports) {
    if (f64) HIP_TRY(batch_report<double>(c, b, (const double*)(const void*)poses, (const double*)(const void*)inv_depth,
                                          o, false, reports, st));
    else HIP_TRY(batch_report<float>(c, b, poses, inv_depth, o, mixed, reports, st));
  }
  return DPVBA_OK;
}

}  // extern "C"
