// C ABI of the patch-graph Gauss-Newton BA library: context, symbolic
// analysis of the edge set, and orchestration of the numeric phases on the
// caller's stream.  See include/dpvba.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "dpvba.h"
#include "layout.h"
#include "tileargs.h"

namespace dpvba {

// kernels (tile.hip, assemble.hip, dense.hip)
template <typename T>
hipError_t launch_tile_iterate(const IterArgs<T>& A, int lds_bytes, hipStream_t st);
template <typename T>
hipError_t launch_tile_finalize(const TileInfo* tiles, int n_tiles, int lds_bytes, const int* tile_patch,
                                const int* blk_pose, const T* U_s, const T* pscale_s, const T* depth_s,
                                const T* dx, const int* status, T* depth_out, const T* poses_final,
                                T* poses_out, int n_frames, hipStream_t st);
template <typename T>
hipError_t launch_retract_copy(const T* poses_cur, T* poses_next, const T* dx, int n_fixed, int n_frames,
                               const int* status, hipStream_t st);
template <typename T>
int small_solve_grid(int lds_bytes);
template <typename T>
hipError_t launch_small_solve(const SmallArgs<T>& S, int grid, int lds_bytes, hipStream_t st);
int small_solve_max_n(int tsize);
template <typename T>
hipError_t launch_gather(const T* part_S, const T* part_vec, const int* s_off, const int* s_src,
                         const int* v_off, const int2* v_src, int n_free, T* S, T* rhs, T* dB, T lambda,
                         int mirror, T* diag_out, hipStream_t st);
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
hipError_t launch_chol_solve(T* S, const T* rhs, int n, T* dx, T* work_b, T* work_y, T* Linv_all, const T* d0,
                             int* status, unsigned int* min_bits, hipStream_t st);
hipError_t launch_report_init(int* status, unsigned int* min_bits, int n, hipStream_t st);
hipError_t launch_report_finalize(dpvba_report* rep, const int* status, const unsigned int* min_bits,
                                  int n_iters, const int* err, hipStream_t st);

}  // namespace dpvba

#include "tileargs.h"

using namespace dpvba;

namespace {

// Shared-memory budget of one tile, and default patches per tile for the
// float32 and float64 plans.
constexpr int kLdsBudget = 150 * 1024;
constexpr int kDefaultTilePatches32 = 96;
constexpr int kDefaultTilePatches64 = 32;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

hipError_t ensure(DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (b.bytes >= bytes) return hipSuccess;
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

// Device copy of one tiling of the patch graph.
struct Tiling {
  int n_tiles = 0, lds_bytes = 0, max_w6 = 0;
  long long part_S = 0, part_vec = 0, u_elems = 0, grid_cells = 0, n_tp = 0;
  DevBuf tiles, tile_patch, slot_frame, slot_blk, edge_grid, blk_pose, s_off, s_src, v_off, v_src;
  DevBuf* bufs[10] = {&tiles, &tile_patch, &slot_frame, &slot_blk, &edge_grid, &blk_pose, &s_off, &s_src, &v_off,
                      &v_src};
};

}  // namespace

struct dpvba_ctx {
  int device = 0;
  // analysed graph
  bool analysed = false;
  int N = 0, P = 0, E = 0, p = 0, n_fixed = 0, n_free = 0;
  const int32_t *ii = nullptr, *jj = nullptr, *kk = nullptr;
  Tiling tl[2];  // [0] float32 plan, [1] float64 plan
  int coop_grid32 = 0, coop_lds32 = -1, coop_grid64 = 0, coop_lds64 = -1;  // co-resident workgroups
  // workspace
  DevBuf part_S, part_vec, part_cost, part_invalid, U_s, pscale_s, depth_s, xh_s, poses_a, poses_b;
  DevBuf S, rhs, dB, d0, dx, wb, wy, Linv, edge_part, ticket, dev_err;
  DevBuf status, min_bits, devrep;
  char err[256] = {0};
  // tracing
  bool tracing = false;
  int trace_every = 1;
  std::vector<hipEvent_t> ev;       // 2 per pair
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
  *out = c;
  return DPVBA_OK;
}

void dpvba_destroy(dpvba_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  DevBuf* bufs[] = {&c->part_S, &c->part_vec, &c->part_cost, &c->part_invalid, &c->U_s, &c->pscale_s,
                    &c->depth_s, &c->xh_s, &c->poses_a, &c->poses_b, &c->S, &c->rhs, &c->dB, &c->d0, &c->dx,
                    &c->wb, &c->wy, &c->Linv, &c->edge_part, &c->ticket, &c->dev_err, &c->status, &c->min_bits, &c->devrep};
  for (DevBuf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  for (Tiling& t : c->tl)
    for (DevBuf* b : t.bufs)
      if (b->p) (void)hipFree(b->p);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  delete c;
}

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

// Host copy of one tiling.
struct HostTiling {
  std::vector<TileInfo> tiles;
  std::vector<int32_t> tile_patch, slot_frame, slot_blk, edge_grid, blk_pose, s_off, s_src, v_off;
  std::vector<int2> v_src;
  long long part_S = 0, part_vec = 0, u_elems = 0;
  int lds = 0, max_w6 = 0;
};

// Split each source frame's patches into tiles of at most `kcap` patches
// whose shared-memory plan (element size tsize) fits the budget, then build
// the gather lists.  Returns false if one patch alone does not fit.
static bool plan_tiling(int N, int nf, const std::vector<int32_t>& jj, const std::vector<int32_t>& pcount,
                        const std::vector<int32_t>& pedges, const std::vector<std::vector<int32_t>>& frame_patches,
                        int kcap, int tsize, HostTiling& H) {
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
    t.u_begin = (int)H.u_elems;
    H.part_S += (long long)t.n_blk * (t.n_blk + 1) / 2 * 36;
    H.part_vec += 12LL * t.n_blk;
    H.u_elems += (long long)t.n_patch * 6 * t.n_blk;
    H.lds = std::max(H.lds, tile_lds_bytes(t.n_patch, Tn, t.n_blk, tsize));
    H.max_w6 = std::max(H.max_w6, 6 * t.n_blk);
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
                        tile_lds_bytes((int)cur.size() + 1, Tn, nb, tsize) <= kLdsBudget;
      if (!fits) {
        if (cur.empty()) return false;
        emit(f, cur, cur_mult);
        cur.clear();
        cur_mult.clear();
        merged = km;
        plan_of(merged, f, Tn, nb, mm);
        if (!(Tn <= kMaxSlots && tile_lds_bytes(1, Tn, nb, tsize) <= kLdsBudget)) return false;
      }
      cur.push_back(k);
      cur_mult = merged;
    }
    if (!cur.empty()) emit(f, cur, cur_mult);
  }
  if (H.part_S > INT32_MAX || H.part_vec > INT32_MAX || H.u_elems > INT32_MAX) return false;
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
  T_.n_tiles = (int)H.tiles.size();
  T_.lds_bytes = H.lds;
  T_.max_w6 = H.max_w6;
  T_.part_S = H.part_S;
  T_.part_vec = H.part_vec;
  T_.u_elems = H.u_elems;
  T_.grid_cells = (long long)H.edge_grid.size();
  T_.n_tp = (long long)H.tile_patch.size();
  return hipSuccess;
}

dpvba_status dpvba_analyze_ex(dpvba_ctx* c, const dpvba_graph* g, const dpvba_tuning* tune, void* stream) {
  if (!c || !graph_sizes_ok(g)) return DPVBA_EINVAL;
  int kcap32 = kDefaultTilePatches32, kcap64 = kDefaultTilePatches64;
  if (tune) {
    if (tune->tile_patches_fp32 < 0 || tune->tile_patches_fp64 < 0) return DPVBA_EINVAL;
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
  std::vector<int32_t> owner(P, -1), pcount(P + 1, 0);
  for (int e = 0; e < E; ++e) {
    const int i = ii[e], j = jj[e], k = kk[e];
    if (i < 0 || i >= N || j < 0 || j >= N || k < 0 || k >= P || i == j) return DPVBA_EINVAL;
    if (owner[k] < 0) owner[k] = i;
    else if (owner[k] != i) return DPVBA_EINVAL;
    pcount[k + 1]++;
  }
  for (int k = 0; k < P; ++k) pcount[k + 1] += pcount[k];
  std::vector<int32_t> pedges(E);
  {
    std::vector<int32_t> cur(pcount.begin(), pcount.end() - 1);
    for (int e = 0; e < E; ++e) pedges[cur[kk[e]]++] = e;  // stable: original order within a patch
  }
  std::vector<std::vector<int32_t>> frame_patches(N);
  for (int k = 0; k < P; ++k)
    if (owner[k] >= 0) frame_patches[owner[k]].push_back(k);
  HostTiling H32, H64;
  if (!plan_tiling(N, nf, jj, pcount, pedges, frame_patches, kcap32, 4, H32)) return DPVBA_EINVAL;
  if (!plan_tiling(N, nf, jj, pcount, pedges, frame_patches, kcap64, 8, H64)) return DPVBA_EINVAL;
  HIP_TRY(upload_tiling(c->tl[0], H32, st));
  HIP_TRY(upload_tiling(c->tl[1], H64, st));

  const size_t n = 6 * (size_t)n_free;
  const size_t nblk64 = (n + 63) / 64;
  auto mx = [&](long long a, long long b) { return (size_t)std::max(a, b); };
  HIP_TRY(ensure(c->part_S, std::max(H32.part_S * 4, H64.part_S * 8)));
  HIP_TRY(ensure(c->part_vec, std::max(H32.part_vec * 4, H64.part_vec * 8)));
  HIP_TRY(ensure(c->part_cost, mx(H32.tiles.size(), H64.tiles.size()) * 8));
  HIP_TRY(ensure(c->part_invalid, mx(H32.tiles.size(), H64.tiles.size()) * 4));
  HIP_TRY(ensure(c->U_s, std::max(H32.u_elems * 4, H64.u_elems * 8)));
  HIP_TRY(ensure(c->pscale_s, (size_t)P * 2 * 8));
  HIP_TRY(ensure(c->depth_s, (size_t)P * 8));
  HIP_TRY(ensure(c->xh_s, (size_t)P * 2 * 8));
  HIP_TRY(ensure(c->poses_a, (size_t)N * 7 * 8));
  HIP_TRY(ensure(c->poses_b, (size_t)N * 7 * 8));
  HIP_TRY(ensure(c->S, n * n * 8));
  HIP_TRY(ensure(c->rhs, n * 8));
  HIP_TRY(ensure(c->dB, n * 8));
  HIP_TRY(ensure(c->d0, n * 8));
  HIP_TRY(ensure(c->dx, n * 8));
  HIP_TRY(ensure(c->wb, n * 8));
  HIP_TRY(ensure(c->wy, n * 8));
  HIP_TRY(ensure(c->Linv, nblk64 * 64 * 64 * 8));
  HIP_TRY(ensure(c->edge_part, ((size_t)(E + 255) / 256) * 8));
  if (!c->ticket.p) {
    HIP_TRY(ensure(c->ticket, 64));
    HIP_TRY(ensure(c->dev_err, 64));
    HIP_TRY(hipMemsetAsync(c->ticket.p, 0, 64, st));
    HIP_TRY(hipMemsetAsync(c->dev_err.p, 0, 64, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  HIP_TRY(ensure(c->status, DPVBA_MAX_ITERS * 4));
  HIP_TRY(ensure(c->min_bits, DPVBA_MAX_ITERS * 4));
  HIP_TRY(ensure(c->devrep, sizeof(dpvba_report)));

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

static dpvba_status check_opts(const dpvba_opts* o) {
  if (!o) return DPVBA_EINVAL;
  if (o->n_iters < 0 || o->n_iters > DPVBA_MAX_ITERS) return DPVBA_EINVAL;
  if (!(o->lambda >= 0.0) || !(o->lambda < (double)FLT_MAX)) return DPVBA_EINVAL;
  if (!(o->z_min >= 0.0) || !(o->z_min < (double)FLT_MAX)) return DPVBA_EINVAL;
  if (o->precision != DPVBA_FP32 && o->precision != DPVBA_FP64) return DPVBA_EINVAL;
  if (o->flags != 0) return DPVBA_EINVAL;
  return DPVBA_OK;
}

template <typename T>
static IterArgs<T> make_iter_args(dpvba_ctx* c, const dpvba_graph* g, const Tiling& tl, const T* poses_cur,
                                  T* poses_next, const T* depth_in, T lambda, T z_min) {
  IterArgs<T> A{};
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
  A.s_off = (const int*)tl.s_off.p;
  A.s_src = (const int*)tl.s_src.p;
  A.v_off = (const int*)tl.v_off.p;
  A.v_src = (const int2*)tl.v_src.p;
  A.dx = (T*)c->dx.p;
  A.first = 1;
  return A;
}

template <typename T>
static bool use_small_path(const dpvba_ctx* c) {
  const int n = 6 * c->n_free;
  return n + 1 <= kSmallRows && small_solve_lds_bytes(n, (int)sizeof(T)) <= 160 * 1024;
}

template <typename T>
static hipError_t reduced_impl(dpvba_ctx* c, const dpvba_graph* g, const T* poses, const T* depth, T lambda,
                               T z_min, T* S, T* rhs, double* cost_out, hipStream_t st) {
  const Tiling& tl = c->tl[sizeof(T) == 8 ? 1 : 0];
  IterArgs<T> A = make_iter_args<T>(c, g, tl, poses, nullptr, depth, lambda, z_min);
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
                          rhs, (T*)c->dB.p, lambda, 1, (T*)c->d0.p, st);
}

template <typename T>
static hipError_t solve_impl(dpvba_ctx* c, const dpvba_graph* g, T* poses, T* depth, const dpvba_opts* o,
                             dpvba_report* report, hipStream_t st) {
  const T lambda = (T)o->lambda, z_min = (T)o->z_min;
  const Tiling& tl = c->tl[sizeof(T) == 8 ? 1 : 0];
  const int n = 6 * c->n_free;
  const int nit = o->n_iters;
  const bool small = use_small_path<T>(c);
  dpvba_report* dev = (dpvba_report*)c->devrep.p;
  int* status = (int*)c->status.p;
  unsigned int* mb = (unsigned int*)c->min_bits.p;
  T* pbuf[2] = {(T*)c->poses_a.p, (T*)c->poses_b.p};
  T* dx = (T*)c->dx.p;
  hipError_t e;
  if (small && nit > 0) {
    SmallArgs<T> S{};
    S.it = make_iter_args<T>(c, g, tl, poses, pbuf[0], depth, lambda, z_min);
    S.poses_io = poses;
    S.depth_io = depth;
    S.pbuf0 = pbuf[0];
    S.pbuf1 = pbuf[1];
    S.Sp = (T*)c->S.p;
    S.rhs = (T*)c->rhs.p;
    S.d0 = (T*)c->d0.p;
    S.status = status;
    S.min_bits = mb;
    S.cost = dev->cost;
    S.invalid = dev->n_invalid;
    S.n_iters = nit;
    S.bar = (unsigned int*)c->ticket.p;
    S.err = (int*)c->dev_err.p;
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
    e = launch_small_solve<T>(S, grid, lds_small, st);
    if (e != hipSuccess) return e;
  }
  if (!small) {
    e = launch_report_init(status, mb, DPVBA_MAX_ITERS, st);
    if (e != hipSuccess) return e;
  }
  for (int it = 0; it < nit && !small; ++it) {
    const T* cur = it == 0 ? poses : pbuf[(it - 1) & 1];
    T* next = pbuf[it & 1];
    IterArgs<T> A = make_iter_args<T>(c, g, tl, cur, next, depth, lambda, z_min);
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
      e = launch_report_reduce((const double*)c->part_cost.p, (const int*)c->part_invalid.p, tl.n_tiles,
                               &dev->cost[it], &dev->n_invalid[it], st);
      if (e == hipSuccess)
        e = launch_gather<T>((const T*)c->part_S.p, (const T*)c->part_vec.p, (const int*)tl.s_off.p,
                             (const int*)tl.s_src.p, (const int*)tl.v_off.p, (const int2*)tl.v_src.p, c->n_free,
                             (T*)c->S.p, (T*)c->rhs.p, (T*)c->dB.p, lambda, 0, (T*)c->d0.p, st);
    }
    if (e != hipSuccess) return e;
    {
      TraceScope ts(c, DPVBA_PHASE_FACTOR, st);
      e = launch_chol_solve<T>((T*)c->S.p, (const T*)c->rhs.p, n, dx, (T*)c->wb.p, (T*)c->wy.p, (T*)c->Linv.p,
                               (const T*)c->d0.p, status + it, mb + it, st);
    }
    if (e != hipSuccess) return e;
    {
      TraceScope ts(c, DPVBA_PHASE_RETRACT, st);
      e = launch_retract_copy<T>(cur, next, dx, c->n_fixed, c->N, status + it, st);
    }
    if (e != hipSuccess) return e;
  }
  if (nit > 0 && !small) {
    TraceScope ts(c, DPVBA_PHASE_BACKSUB, st);
    e = launch_tile_finalize<T>((const TileInfo*)tl.tiles.p, tl.n_tiles, tl.lds_bytes, (const int*)tl.tile_patch.p,
                                (const int*)tl.blk_pose.p, (const T*)c->U_s.p, (const T*)c->pscale_s.p,
                                (const T*)c->depth_s.p, dx, status + nit - 1, depth, pbuf[(nit - 1) & 1], poses,
                                c->N, st);
    if (e != hipSuccess) return e;
  }
  if (!report) return hipSuccess;
  {
    TraceScope ts_cost(c, DPVBA_PHASE_COST, st);
    e = launch_edge_cost<T, T>(poses, depth, g->patches, g->patch_size, g->ii, g->jj, g->kk, g->target, g->weight,
                               g->n_edges, (T)g->fx, (T)g->fy, (T)g->cx, (T)g->cy, z_min,
                               (double*)c->edge_part.p, st);
  }
  if (e != hipSuccess) return e;
  e = launch_report_reduce((const double*)c->edge_part.p, nullptr, (g->n_edges + 255) / 256, &dev->cost[nit],
                           nullptr, st);
  if (e != hipSuccess) return e;
  e = launch_report_finalize(dev, status, mb, nit, (const int*)c->dev_err.p, st);
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(report, dev, sizeof(dpvba_report), hipMemcpyDeviceToHost, st);
}

extern "C" {

dpvba_status dpvba_reproject(dpvba_ctx* c, const dpvba_graph* g, const float* poses, const float* inv_depth,
                             float z_min, float* coords, uint8_t* valid, void* stream) {
  if (!c || !graph_sizes_ok(g)) return DPVBA_EINVAL;
  if (!(z_min >= 0.f) || !(z_min < FLT_MAX)) return DPVBA_EINVAL;
  if (g->n_edges > 0 && (!poses || !inv_depth || !coords)) return DPVBA_EINVAL;
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(launch_reproject(poses, inv_depth, g->patches, g->patch_size, g->ii, g->jj, g->kk, g->n_edges, g->fx,
                           g->fy, g->cx, g->cy, z_min, coords, valid, (hipStream_t)stream));
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
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  if (o->precision == DPVBA_FP64) {
    HIP_TRY(reduced_impl<double>(c, g, (const double*)(const void*)poses, (const double*)(const void*)inv_depth,
                                 (double)o->lambda, (double)o->z_min, (double*)S, (double*)s, cost, st));
  } else {
    HIP_TRY(reduced_impl<float>(c, g, poses, inv_depth, (float)o->lambda, (float)o->z_min, (float*)S, (float*)s,
                                cost, st));
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
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  if (o->precision == DPVBA_FP64) {
    HIP_TRY(solve_impl<double>(c, g, (double*)(void*)poses, (double*)(void*)inv_depth, o, report, st));
  } else {
    HIP_TRY(solve_impl<float>(c, g, poses, inv_depth, o, report, st));
  }
  return DPVBA_OK;
}

}  // extern "C"
