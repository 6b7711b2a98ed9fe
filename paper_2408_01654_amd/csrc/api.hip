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

#include "../../include/dpvba.h"
#include "layout.h"

namespace dpvba {

// kernels (assemble.hip, dense.hip)
template <typename T, typename P> struct TileArgs;
template <typename T, typename P>
hipError_t launch_tile_assemble(const TileArgs<T, P>& A, int n_tiles, int lds_bytes, hipStream_t st);
template <typename T, typename P>
hipError_t launch_tile_backsub(const TileArgs<T, P>& A, int n_tiles, int lds_bytes, hipStream_t st);
template <typename T, typename P>
hipError_t launch_retract(P* poses, const T* dx, int n_fixed, int n_free, const int* status, hipStream_t st);
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
                                  int n_iters, hipStream_t st);

}  // namespace dpvba

#include "tileargs.h"

using namespace dpvba;

namespace {

// Shared-memory budget of one tile in float64 (float32 tiles use half).
constexpr int kLdsBudget64 = 150 * 1024;
constexpr int kMaxPatchesPerTile = 32;

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

}  // namespace

struct dpvba_ctx {
  int device = 0;
  // analysed graph
  bool analysed = false;
  int N = 0, P = 0, E = 0, p = 0, n_fixed = 0, n_free = 0;
  const int32_t *ii = nullptr, *jj = nullptr, *kk = nullptr;
  int n_tiles = 0;
  int lds_f32 = 0, lds_f64 = 0;
  size_t part_S_elems = 0, part_vec_elems = 0;
  DevBuf tiles, tile_patch, slot_frame, slot_blk, edge_grid, blk_pose, s_off, s_src, v_off, v_src;
  // workspace
  DevBuf part_S, part_vec, part_cost, part_invalid, S, rhs, dB, d0, dx, wb, wy, Linv, edge_part;
  DevBuf status, min_bits, devrep;
  char err[256] = {0};
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
  DevBuf* bufs[] = {&c->tiles, &c->tile_patch, &c->slot_frame, &c->slot_blk, &c->edge_grid, &c->blk_pose,
                    &c->s_off, &c->s_src, &c->v_off, &c->v_src, &c->part_S, &c->part_vec, &c->part_cost,
                    &c->part_invalid, &c->S, &c->rhs, &c->dB, &c->d0, &c->dx, &c->wb, &c->wy, &c->Linv,
                    &c->edge_part, &c->status, &c->min_bits, &c->devrep};
  for (DevBuf* b : bufs)
    if (b->p) (void)hipFree(b->p);
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

dpvba_status dpvba_analyze(dpvba_ctx* c, const dpvba_graph* g, void* stream) {
  if (!c || !graph_sizes_ok(g)) return DPVBA_EINVAL;
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
  // patches with edges, grouped by owner frame (ascending patch index)
  std::vector<std::vector<int32_t>> frame_patches(N);
  for (int k = 0; k < P; ++k)
    if (owner[k] >= 0) frame_patches[owner[k]].push_back(k);

  std::vector<TileInfo> tiles;
  std::vector<int32_t> tile_patch, slot_frame, slot_blk, edge_grid, blk_pose;
  long long part_S = 0, part_vec = 0;
  int max_lds64 = 0, max_lds32 = 0;

  auto patch_mult = [&](int k, std::map<int, int>& m) {
    for (int q = pcount[k]; q < pcount[k + 1]; ++q) m[jj[pedges[q]]]++;
  };
  auto plan_of = [&](const std::map<int, int>& mult, int frame, int& Tn, int& nb) {
    Tn = 0;
    nb = frame >= nf ? 1 : 0;
    for (auto& kv : mult) {
      Tn += kv.second;
      if (kv.first >= nf) nb++;
    }
  };
  auto emit_tile = [&](int frame, const std::vector<int32_t>& pl, const std::map<int, int>& mult) {
    TileInfo t{};
    t.frame = frame;
    t.n_patch = (int)pl.size();
    t.patch_begin = (int)tile_patch.size();
    t.slot_begin = (int)slot_frame.size();
    t.grid_begin = (int)edge_grid.size();
    t.blk_begin = (int)blk_pose.size();
    // blocks: free poses among {frame} U targets, ascending
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
    int Tn = 0;
    for (auto& kv : mult) {
      first_slot[kv.first] = Tn;
      for (int m = 0; m < kv.second; ++m) {
        slot_frame.push_back(kv.first);
        slot_blk.push_back(blk_of(kv.first));
      }
      Tn += kv.second;
    }
    t.n_slot = Tn;
    for (int b : blocks) blk_pose.push_back(b - nf);
    const size_t g0 = edge_grid.size();
    edge_grid.resize(g0 + (size_t)t.n_patch * Tn, -1);
    for (int lp = 0; lp < t.n_patch; ++lp) {
      const int k = pl[lp];
      tile_patch.push_back(k);
      std::map<int, int> used;
      for (int q = pcount[k]; q < pcount[k + 1]; ++q) {
        const int e = pedges[q];
        const int s = first_slot[jj[e]] + used[jj[e]]++;
        edge_grid[g0 + (size_t)lp * Tn + s] = e;
      }
    }
    t.part_begin = (int)part_S;
    t.vec_begin = (int)part_vec;
    part_S += (long long)t.n_blk * (t.n_blk + 1) / 2 * 36;
    part_vec += 12LL * t.n_blk;
    max_lds64 = std::max(max_lds64, tile_lds_bytes(t.n_patch, Tn, t.n_blk, 8));
    max_lds32 = std::max(max_lds32, tile_lds_bytes(t.n_patch, Tn, t.n_blk, 4));
    tiles.push_back(t);
  };

  for (int f = 0; f < N; ++f) {
    std::vector<int32_t> cur;
    std::map<int, int> cur_mult;
    for (int k : frame_patches[f]) {
      std::map<int, int> km;
      patch_mult(k, km);
      std::map<int, int> merged = cur_mult;
      for (auto& kv : km) merged[kv.first] = std::max(merged[kv.first], kv.second);
      int Tn, nb;
      plan_of(merged, f, Tn, nb);
      const bool fits = Tn <= kMaxSlots && (int)cur.size() + 1 <= kMaxPatchesPerTile &&
                        tile_lds_bytes((int)cur.size() + 1, Tn, nb, 8) <= kLdsBudget64;
      if (!fits) {
        if (cur.empty()) return DPVBA_EINVAL;  // one patch alone exceeds the tile limits
        emit_tile(f, cur, cur_mult);
        cur.clear();
        cur_mult.clear();
        merged = km;
        plan_of(merged, f, Tn, nb);
        if (!(Tn <= kMaxSlots && tile_lds_bytes(1, Tn, nb, 8) <= kLdsBudget64)) return DPVBA_EINVAL;
      }
      cur.push_back(k);
      cur_mult = merged;
    }
    if (!cur.empty()) emit_tile(f, cur, cur_mult);
  }
  if (part_S > INT32_MAX || part_vec > INT32_MAX) return DPVBA_EINVAL;

  // gather lists: lower block (P >= Q) -> tile partial offsets, tile order
  const long long n_lb = (long long)n_free * (n_free + 1) / 2;
  std::vector<int32_t> s_off(n_lb + 1, 0), v_off(n_free + 1, 0);
  for (const TileInfo& t : tiles) {
    for (int a = 0; a < t.n_blk; ++a)
      for (int b = a; b < t.n_blk; ++b) {
        const long long Pp = blk_pose[t.blk_begin + b], Qq = blk_pose[t.blk_begin + a];
        s_off[Pp * (Pp + 1) / 2 + Qq + 1]++;
      }
    for (int a = 0; a < t.n_blk; ++a) v_off[blk_pose[t.blk_begin + a] + 1]++;
  }
  for (long long q = 0; q < n_lb; ++q) s_off[q + 1] += s_off[q];
  for (int q = 0; q < n_free; ++q) v_off[q + 1] += v_off[q];
  std::vector<int32_t> s_src(s_off[n_lb]);
  std::vector<int2> v_src(v_off[n_free]);
  {
    std::vector<int32_t> cs(s_off.begin(), s_off.end() - 1), cv(v_off.begin(), v_off.end() - 1);
    for (const TileInfo& t : tiles) {
      for (int a = 0; a < t.n_blk; ++a)
        for (int b = a; b < t.n_blk; ++b) {
          const long long Pp = blk_pose[t.blk_begin + b], Qq = blk_pose[t.blk_begin + a];
          s_src[cs[Pp * (Pp + 1) / 2 + Qq]++] = t.part_begin + upper_pair_index(a, b, t.n_blk) * 36;
        }
      for (int a = 0; a < t.n_blk; ++a) {
        const int Pp = blk_pose[t.blk_begin + a];
        v_src[cv[Pp]++] = make_int2(t.vec_begin + 6 * a, t.vec_begin + 6 * t.n_blk + 6 * a);
      }
    }
  }

  HIP_TRY(upload(c->tiles, tiles, st));
  HIP_TRY(upload(c->tile_patch, tile_patch, st));
  HIP_TRY(upload(c->slot_frame, slot_frame, st));
  HIP_TRY(upload(c->slot_blk, slot_blk, st));
  HIP_TRY(upload(c->edge_grid, edge_grid, st));
  HIP_TRY(upload(c->blk_pose, blk_pose, st));
  HIP_TRY(upload(c->s_off, s_off, st));
  HIP_TRY(upload(c->s_src, s_src, st));
  HIP_TRY(upload(c->v_off, v_off, st));
  HIP_TRY(upload(c->v_src, v_src, st));

  const size_t n = 6 * (size_t)n_free;
  const size_t nblk64 = (n + 63) / 64;
  HIP_TRY(ensure(c->part_S, (size_t)part_S * 8));
  HIP_TRY(ensure(c->part_vec, (size_t)part_vec * 8));
  HIP_TRY(ensure(c->part_cost, tiles.size() * 8));
  HIP_TRY(ensure(c->part_invalid, tiles.size() * 4));
  HIP_TRY(ensure(c->S, n * n * 8));
  HIP_TRY(ensure(c->rhs, n * 8));
  HIP_TRY(ensure(c->dB, n * 8));
  HIP_TRY(ensure(c->d0, n * 8));
  HIP_TRY(ensure(c->dx, n * 8));
  HIP_TRY(ensure(c->wb, n * 8));
  HIP_TRY(ensure(c->wy, n * 8));
  HIP_TRY(ensure(c->Linv, nblk64 * 64 * 64 * 8));
  HIP_TRY(ensure(c->edge_part, ((size_t)(E + 255) / 256) * 8));
  HIP_TRY(ensure(c->status, DPVBA_MAX_ITERS * 4));
  HIP_TRY(ensure(c->min_bits, DPVBA_MAX_ITERS * 4));
  HIP_TRY(ensure(c->devrep, sizeof(dpvba_report)));

  c->N = N; c->P = P; c->E = E; c->p = g->patch_size; c->n_fixed = nf; c->n_free = n_free;
  c->ii = g->ii; c->jj = g->jj; c->kk = g->kk;
  c->n_tiles = (int)tiles.size();
  c->lds_f32 = max_lds32;
  c->lds_f64 = max_lds64;
  c->part_S_elems = (size_t)part_S;
  c->part_vec_elems = (size_t)part_vec;
  c->analysed = true;
  return DPVBA_OK;
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
static TileArgs<T, T> make_args(dpvba_ctx* c, const dpvba_graph* g, const T* poses, T* depth, T lambda,
                                T z_min) {
  TileArgs<T, T> A{};
  A.poses = poses;
  A.inv_depth = depth;
  A.patches = g->patches;
  A.p = g->patch_size;
  A.target = g->target;
  A.weight = g->weight;
  A.fx = g->fx; A.fy = g->fy; A.cx = g->cx; A.cy = g->cy;
  A.z_min = z_min;
  A.lambda = lambda;
  A.n_fixed = c->n_fixed;
  A.tiles = (const TileInfo*)c->tiles.p;
  A.tile_patch = (const int*)c->tile_patch.p;
  A.slot_frame = (const int*)c->slot_frame.p;
  A.slot_blk = (const int*)c->slot_blk.p;
  A.edge_grid = (const int*)c->edge_grid.p;
  A.blk_pose = (const int*)c->blk_pose.p;
  A.part_S = (T*)c->part_S.p;
  A.part_vec = (T*)c->part_vec.p;
  A.part_cost = (double*)c->part_cost.p;
  A.part_invalid = (int*)c->part_invalid.p;
  return A;
}

template <typename T>
static hipError_t assemble_and_gather(dpvba_ctx* c, const dpvba_graph* g, const T* poses, T* depth, T lambda,
                                      T z_min, T* S, T* rhs, int mirror, double* cost_out, int* invalid_out,
                                      hipStream_t st) {
  TileArgs<T, T> A = make_args<T>(c, g, poses, depth, lambda, z_min);
  const int lds = sizeof(T) == 8 ? c->lds_f64 : c->lds_f32;
  hipError_t e = launch_tile_assemble<T, T>(A, c->n_tiles, lds, st);
  if (e != hipSuccess) return e;
  if (cost_out) {
    if (c->n_tiles) {
      e = launch_report_reduce((const double*)c->part_cost.p, (const int*)c->part_invalid.p, c->n_tiles,
                               cost_out, invalid_out, st);
    } else {
      e = launch_report_reduce((const double*)c->part_cost.p, nullptr, 0, cost_out, invalid_out, st);
    }
    if (e != hipSuccess) return e;
  }
  return launch_gather<T>((const T*)c->part_S.p, (const T*)c->part_vec.p, (const int*)c->s_off.p,
                          (const int*)c->s_src.p, (const int*)c->v_off.p, (const int2*)c->v_src.p, c->n_free,
                          S, rhs, (T*)c->dB.p, lambda, mirror, (T*)c->d0.p, st);
}

template <typename T>
static hipError_t solve_impl(dpvba_ctx* c, const dpvba_graph* g, T* poses, T* depth, const dpvba_opts* o,
                             dpvba_report* report, hipStream_t st) {
  const T lambda = (T)o->lambda, z_min = (T)o->z_min;
  const int n = 6 * c->n_free;
  dpvba_report* dev = (dpvba_report*)c->devrep.p;
  int* status = (int*)c->status.p;
  unsigned int* mb = (unsigned int*)c->min_bits.p;
  hipError_t e = launch_report_init(status, mb, DPVBA_MAX_ITERS, st);
  if (e != hipSuccess) return e;
  const int lds = sizeof(T) == 8 ? c->lds_f64 : c->lds_f32;
  for (int it = 0; it < o->n_iters; ++it) {
    e = assemble_and_gather<T>(c, g, poses, depth, lambda, z_min, (T*)c->S.p, (T*)c->rhs.p, 0,
                               &dev->cost[it], &dev->n_invalid[it], st);
    if (e != hipSuccess) return e;
    e = launch_chol_solve<T>((T*)c->S.p, (const T*)c->rhs.p, n, (T*)c->dx.p, (T*)c->wb.p, (T*)c->wy.p,
                             (T*)c->Linv.p, (const T*)c->d0.p, status + it, mb + it, st);
    if (e != hipSuccess) return e;
    TileArgs<T, T> A = make_args<T>(c, g, poses, depth, lambda, z_min);
    A.dx = (const T*)c->dx.p;
    A.step_status = status + it;
    e = launch_tile_backsub<T, T>(A, c->n_tiles, lds, st);
    if (e != hipSuccess) return e;
    e = launch_retract<T, T>(poses, (const T*)c->dx.p, c->n_fixed, c->n_free, status + it, st);
    if (e != hipSuccess) return e;
  }
  e = launch_edge_cost<T, T>(poses, depth, g->patches, g->patch_size, g->ii, g->jj, g->kk, g->target, g->weight,
                             g->n_edges, (T)g->fx, (T)g->fy, (T)g->cx, (T)g->cy, z_min, (double*)c->edge_part.p,
                             st);
  if (e != hipSuccess) return e;
  e = launch_report_reduce((const double*)c->edge_part.p, nullptr, (g->n_edges + 255) / 256,
                           &dev->cost[o->n_iters], nullptr, st);
  if (e != hipSuccess) return e;
  e = launch_report_finalize(dev, status, mb, o->n_iters, st);
  if (e != hipSuccess) return e;
  if (report) {
    e = hipMemcpyAsync(report, dev, sizeof(dpvba_report), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
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
    HIP_TRY(assemble_and_gather<double>(c, g, (const double*)(const void*)poses, (double*)(void*)inv_depth,
                                        (double)o->lambda, (double)o->z_min, (double*)S, (double*)s, 1, cost,
                                        nullptr, st));
  } else {
    HIP_TRY(assemble_and_gather<float>(c, g, poses, (float*)inv_depth, (float)o->lambda, (float)o->z_min, (float*)S,
                                       (float*)s, 1, cost, nullptr, st));
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
