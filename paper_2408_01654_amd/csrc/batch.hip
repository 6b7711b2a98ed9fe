// Batched solve: many independent BA problems (uneven sliding windows) in
// the same launches.  The tiles of every problem form one grid, so the
// assembly of all problems is load-balanced by the hardware dispatcher (the
// tile kernel is unchanged; a tile knows its problem).  Then one wavefront
// per 6x6 block of every problem gathers the damped reduced camera systems
// (DPV-SLAM Appendix A) from the tiles' shares into the problems' scratch
// slices, and one workgroup per problem factors its system, solves it and
// retracts its poses.
//
// Precision modes of the per-problem solve:
//   float32  shares, packed factor and solve in float32 (shared memory);
//   float64  all float64, packed factor in shared memory when it fits, else
//            in the problem's slice of the global scratch;
//   mixed    float32 shares gathered in float64 into the scratch, float32
//            factor in shared memory, kRefine steps of iterative refinement
//            against the float64 residual, and a float64 factorisation of the
//            scratch copy when the refined residual stays above the tolerance
//            or a float32 pivot failed.
#include "edge.h"
#include <cfloat>

#include "packed.h"
#include "dpvba.h"

namespace dpvba {

constexpr int kBatchThreads = 256;
constexpr int kBatchRefine = 2;
constexpr double kBatchRefineTol = 1e-8;

template <typename TS>
struct BatchArgs {
  const BatchInst* inst;
  const TS* part_S;
  const TS* part_vec;
  const int* s_off;
  const int* s_src;
  const int* v_off;
  const int2* v_src;
  double lambda;          // H~ = H + lam_diag Diag(H) + lambda I
  double lam_diag;
  int n_refine;           // mixed: refinement steps
  int force_fb;           // mixed: always take the float64 factorisation
  const TS* poses_cur;
  TS* poses_next;
  TS* dx;
  int* status;            // [problem * stride + iteration]
  unsigned int* min_bits;
  double* refine_resid;
  int* fallback;
  int stride, it;
  double* scratch;        // packed float64 systems
  int lds_factor;         // packed factor in shared memory
};

// Damped system of every problem, one wavefront per lower 6x6 block
// (P >= Q) of problem blockIdx.y: the block is summed from its tiles' shares
// in tile order (share offsets loaded once per wavefront and broadcast,
// eight independent loads in flight), the diagonal gets lam (Diag(B) + 1),
// and the problem's scratch slice receives, in type TA, the packed lower
// matrix, then s, then the damped diagonal d0.
template <typename TS, typename TA>
__global__ void __launch_bounds__(256) batch_gather_kernel(BatchArgs<TS> a) {
  const BatchInst I = a.inst[blockIdx.y];
  const int nf = I.n_free;
  const int blk = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (blk >= nf * (nf + 1) / 2) return;  // whole wavefronts; the kernel has no barrier
  const int lane = threadIdx.x & 63;
  const int n = 6 * nf;
  TA* A = reinterpret_cast<TA*>(a.scratch + I.scratch_off);
  TA* sv_out = A + (size_t)n * (n + 1) / 2;
  TA* d0_out = sv_out + n;
  int P, Q;
  lower_block_of(blk, P, Q);
  const int r = lane / 6, c = lane - (lane / 6) * 6;
  const bool lower = lane < 36 && (P > Q || r >= c);
  const int eo = c * 6 + r;  // the shares hold upper entries: (r, c) of S_PQ is [c][r] of a share
  TA v = (TA)0;
  const int lo = a.s_off[I.s_base + blk], hi = a.s_off[I.s_base + blk + 1];
  for (int b0 = lo; b0 < hi; b0 += 64) {
    const int o_l = b0 + lane < hi ? a.s_src[b0 + lane] : 0;
    const int nq = min(64, hi - b0);
    for (int q0 = 0; q0 < nq; q0 += 8) {
      TA part[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int o = __shfl(o_l, (q0 + u) & 63);
        part[u] = (lower && q0 + u < nq) ? (TA)a.part_S[o + eo] : (TA)0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) v += part[u];
    }
  }
  const int row = 6 * P + r, col = 6 * Q + c;
  if (P == Q) {
    // Diag(B) (lanes on the diagonal) and s (lanes 36..41) of pose P
    const int m = lane < 36 ? r : lane - 36;
    const bool want_d = lane < 36 && r == c, want_s = lane >= 36 && lane < 42;
    const int vlo = a.v_off[I.v_base + P], vhi = a.v_off[I.v_base + P + 1];
    TA db = (TA)0, sv = (TA)0;
    for (int b0 = vlo; b0 < vhi; b0 += 64) {
      const int2 o_l = b0 + lane < vhi ? a.v_src[b0 + lane] : make_int2(0, 0);
      const int nq = min(64, vhi - b0);
      for (int q0 = 0; q0 < nq; q0 += 8) {
        TA pd[8], ps[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int ox = __shfl(o_l.x, (q0 + u) & 63), oy = __shfl(o_l.y, (q0 + u) & 63);
          const bool in = q0 + u < nq;
          pd[u] = (want_d && in) ? (TA)a.part_vec[oy + m] : (TA)0;
          ps[u] = (want_s && in) ? (TA)a.part_vec[ox + m] : (TA)0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          db += pd[u];
          sv += ps[u];
        }
      }
    }
    if (want_s) sv_out[6 * P + m] = sv;
    if (want_d) {
      v += (TA)a.lam_diag * db + (TA)a.lambda;
      d0_out[row] = v;
    }
  }
  if (lower) A[packed_index(row, col)] = v;
}

// count entries from global memory into LDS, eight independent loads in
// flight per thread.
template <typename TD, typename TSRC>
__device__ __forceinline__ void copy_in(const TSRC* src, TD* dst, int count) {
  for (int q0 = threadIdx.x; q0 < count; q0 += 8 * blockDim.x) {
    TSRC v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = q0 + u * blockDim.x;
      v[u] = q < count ? src[q] : (TSRC)0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = q0 + u * blockDim.x;
      if (q < count) dst[q] = (TD)v[u];
    }
  }
}

// Write the step and retract the problem's free poses.
template <typename TS, typename TX>
__device__ __forceinline__ void batch_apply(const BatchArgs<TS>& a, const BatchInst& I, const TX* x, bool bad) {
  const int n = 6 * I.n_free;
  for (int q = threadIdx.x; q < n; q += blockDim.x) a.dx[6 * (size_t)I.free_begin + q] = bad ? (TS)0 : (TS)x[q];
  for (int f = threadIdx.x; f < I.n_frames; f += blockDim.x) {
    const size_t g = (size_t)(I.frame_begin + f);
    TS* pn = a.poses_next + 7 * g;
    for (int m = 0; m < 7; ++m) pn[m] = a.poses_cur[7 * g + m];
    if (f >= I.n_fixed && !bad) {
      TS xi[6];
      for (int m = 0; m < 6; ++m) xi[m] = (TS)x[6 * (f - I.n_fixed) + m];
      retract_pose<TS, TS>(pn, xi);
    }
  }
}

__device__ __forceinline__ void batch_pivot_min(unsigned int* min_bits, float ratio) {
  if (!(ratio >= 0.f)) ratio = 0.f;
  atomicMin(min_bits, __float_as_uint(ratio));
}

// float32 or float64: one precision throughout.  With the factor in shared
// memory: the gathered system with s appended as row n is factored by
// packed_panel_factor (row n ends as y = L^-1 s) and L^T x = y is solved by
// one wavefront.  Otherwise (float64 systems too wide for shared memory) the
// packed factor works in the problem's scratch slice.
template <typename T>
__global__ void __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(1, 1)))
batch_solve_kernel(BatchArgs<T> a) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ int bad;
  __shared__ float minr;
  __shared__ unsigned int minr_bits;
  const BatchInst I = a.inst[blockIdx.x];
  const int n = 6 * I.n_free;
  T* G = reinterpret_cast<T*>(a.scratch + I.scratch_off);  // gathered: packed, s, d0
  int* st = a.status + blockIdx.x * a.stride + a.it;
  if (n == 0) {
    batch_apply<T, T>(a, I, reinterpret_cast<T*>(lds), false);
    return;
  }
  const int np = n * (n + 1) / 2;
  if (a.lds_factor) {
    T* d0 = reinterpret_cast<T*>(lds);
    T* invd = d0 + n;
    T* piv = invd + n;
    T* x = piv + n;
    T* A = x + n;  // packed, n + 1 rows
    copy_in<T, T>(G, A, np + n);  // the packed rows, then s as row n
    copy_in<T, T>(G + np + n, d0, n);
    if (threadIdx.x == 0) {
      A[np + n] = (T)0;
      bad = 0;
      minr_bits = __float_as_uint(3.0e38f);
    }
    __syncthreads();
    packed_panel_factor<T>(A, n, n + 1, invd, piv, &bad);
    pivot_ratio_min<T>(piv, d0, n, &minr_bits);  // smallest pivot / damped diagonal
    packed_back_solve<T>(A, n, invd, A + np, x);
    __syncthreads();
    const bool failed = bad != 0;
    batch_apply<T, T>(a, I, x, failed);
    if (threadIdx.x == 0) {
      *st = failed;
      batch_pivot_min(a.min_bits + blockIdx.x * a.stride + a.it, __uint_as_float(minr_bits));
    }
    return;
  }
  T* vb = reinterpret_cast<T*>(lds);
  T* d0 = vb + n;
  copy_in<T, T>(G + np, vb, 2 * n);  // s and d0
  __syncthreads();
  packed_cholesky<T>(G, n, d0, &bad, &minr);
  packed_solve<T, T>(G, vb, n);
  const bool failed = bad != 0;
  batch_apply<T, T>(a, I, vb, failed);
  if (threadIdx.x == 0) {
    *st = failed;
    batch_pivot_min(a.min_bits + blockIdx.x * a.stride + a.it, minr);
  }
}

// r = s - S x for the packed symmetric S (float64).  A wavefront takes
// eight rows at a time, lanes along the rows (entry (i, j) read from row i
// for j <= i, else from row j; every load of a step in flight together), and
// sums the eight rows over its lanes together in a halving butterfly.
// Returns max |r| (all threads), reduced in a fixed order through `red`.
__device__ __forceinline__ double batch_residual(const double* S, const double* s, const double* x, double* r, int n, double* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
  double mx = 0.0;
  for (int i0 = 8 * wv; i0 < n; i0 += 8 * nwv) {
    double part[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) part[u] = 0.0;
    for (int j = lane; j < n; j += 64) {
      const double xj = x[j];
      double a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = min(i0 + u, n - 1);
        a[u] = j <= i ? S[packed_index(i, j)] : S[packed_index(j, i)];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) part[u] += a[u] * xj;
    }
    // after the butterfly lane l holds the total of row i0 + 4 b5 + 2 b4 + b3
    double h4[4], h2[2];
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double give = b5 ? part[q] : part[4 + q];
      h4[q] = (b5 ? part[4 + q] : part[q]) + __shfl_xor(give, 32);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const double give = b4 ? h4[q] : h4[2 + q];
      h2[q] = (b4 ? h4[2 + q] : h4[q]) + __shfl_xor(give, 16);
    }
    double h = (b3 ? h2[1] : h2[0]) + __shfl_xor(b3 ? h2[0] : h2[1], 8);
    h += __shfl_xor(h, 4);
    h += __shfl_xor(h, 2);
    h += __shfl_xor(h, 1);
    const int row = i0 + 4 * (b5 ? 1 : 0) + 2 * (b4 ? 1 : 0) + (b3 ? 1 : 0);
    if ((lane & 7) == 0 && row < n) {
      const double ri = s[row] - h;
      r[row] = ri;
      if (ri != ri) mx = ri;  // a NaN sticks
      else if (mx == mx) mx = fmax(mx, fabs(ri));
    }
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const double o = red[threadIdx.x + w];
      red[threadIdx.x] = (o != o || o > red[threadIdx.x]) ? o : red[threadIdx.x];
    }
    __syncthreads();
  }
  const double out = red[0];
  __syncthreads();
  return out;
}

// Mixed precision: float32 state and shares, float64 system in the scratch.
// (Both solve kernels run one workgroup per problem and take the whole
// register file: their shared memory allows about one workgroup per CU.)
__global__ void __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(1, 1)))
batch_solve_mixed_kernel(BatchArgs<float> a) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ int bad;
  __shared__ float minr;
  __shared__ double red[kBatchThreads];
  const BatchInst I = a.inst[blockIdx.x];
  const int n = 6 * I.n_free;
  double* x64 = reinterpret_cast<double*>(lds);  // [n]
  double* r64 = x64 + n;                          // [n]
  double* b64 = r64 + n;                          // [n] copy of s for the float64 fallback
  float* c32 = reinterpret_cast<float*>(b64 + n); // [n]
  float* d32 = c32 + n;                           // [n]
  float* invd32 = d32 + n;                        // [n]
  float* piv32 = invd32 + n;                      // [n]
  float* A32 = piv32 + n;                         // packed, n + 1 rows (s appended)
  double* S64 = a.scratch + I.scratch_off;        // packed, then s [n], then d0 [n]
  double* s64 = S64 + (size_t)n * (n + 1) / 2;
  double* d064 = s64 + n;
  __shared__ int bad32;
  __shared__ unsigned int minr_bits;
  const int idx_st = blockIdx.x * a.stride + a.it;
  if (n == 0) {
    batch_apply<float, float>(a, I, c32, false);
    if (threadIdx.x == 0) {
      a.refine_resid[idx_st] = 0.0;
      a.fallback[idx_st] = 0;
    }
    return;
  }
  const int np = n * (n + 1) / 2;
  copy_in<float, double>(S64, A32, np + n);  // gathered in float64: the packed rows, then s as row n
  copy_in<float, double>(d064, d32, n);
  if (threadIdx.x == 0) {
    A32[np + n] = 0.f;
    bad32 = 0;
    minr_bits = __float_as_uint(3.0e38f);
  }
  __syncthreads();
  packed_panel_factor<float>(A32, n, n + 1, invd32, piv32, &bad32);
  pivot_ratio_min<float>(piv32, d32, n, &minr_bits);
  packed_back_solve<float>(A32, n, invd32, A32 + np, c32);
  __syncthreads();
  const float minr32 = __uint_as_float(minr_bits);
  for (int q = threadIdx.x; q < n; q += blockDim.x) x64[q] = (double)c32[q];
  __syncthreads();
  double smax = 0.0;
  {
    double mx = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) mx = fmax(mx, fabs(s64[i]));
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
      __syncthreads();
    }
    smax = red[0];
    __syncthreads();
  }
#pragma unroll 1
  for (int k = 0; k < a.n_refine; ++k) {
    batch_residual(S64, s64, x64, r64, n, red);
    for (int q = threadIdx.x; q < n; q += blockDim.x) c32[q] = (float)r64[q];
    __syncthreads();
    packed_fwd_solve<float>(A32, n, invd32, c32, c32);
    __syncthreads();
    packed_back_solve<float>(A32, n, invd32, c32, c32);
    __syncthreads();
    for (int q = threadIdx.x; q < n; q += blockDim.x) x64[q] += (double)c32[q];
    __syncthreads();
  }
  const double rmax = batch_residual(S64, s64, x64, r64, n, red);
  const double rel = smax > 0.0 ? rmax / smax : rmax;
  const bool fb = a.force_fb || bad32 != 0 || !(rel <= kBatchRefineTol);
  bool failed = false;
  if (fb) {  // float64 factorisation of the scratch copy
    for (int q = threadIdx.x; q < n; q += blockDim.x) b64[q] = s64[q];
    __syncthreads();
    packed_cholesky<double>(S64, n, d064, &bad, &minr);
    failed = bad != 0;
    packed_solve<double, double>(S64, b64, n);
    for (int q = threadIdx.x; q < n; q += blockDim.x) x64[q] = b64[q];
    __syncthreads();
  }
  batch_apply<float, double>(a, I, x64, failed);
  if (threadIdx.x == 0) {
    a.status[idx_st] = failed;
    a.refine_resid[idx_st] = rel;
    a.fallback[idx_st] = fb;
    batch_pivot_min(a.min_bits + idx_st, minr32);
  }
}

// Per problem: sum its tiles' costs and invalid counts of one iteration.
__global__ void batch_cost_kernel(const BatchInst* inst, int n_inst, const double* part_cost,
                                  const int* part_invalid, dpvba_report* rep, int it) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_inst) return;
  const BatchInst I = inst[b];
  double c = 0.0;
  int v = 0;
  for (int t = I.tile_begin; t < I.tile_begin + I.n_tiles; ++t) {
    c += part_cost[t];
    v += part_invalid[t];
  }
  rep[b].cost[it] = c;
  rep[b].n_invalid[it] = v;
}

// Per problem (one workgroup): cost at the final iterate and the report.
template <typename T>
__global__ void __launch_bounds__(256) batch_report_kernel(
    const BatchInst* inst, const T* poses, const T* inv_depth, const float* patches, int p, const int* ii,
    const int* jj, const int* kk, const float* target, const float* weight, T fx, T fy, T cx, T cy, T z_min,
    const int* status, const unsigned int* min_bits, const double* refine, const int* fallback, int stride,
    int n_iters, dpvba_report* rep) {
  __shared__ double sred[256];
  __shared__ int bad_in;
  const BatchInst I = inst[blockIdx.x];
  if (threadIdx.x == 0) bad_in = 0;
  __syncthreads();
  double cst = 0.0;
  bool bad = false;
  for (int q = threadIdx.x; q < I.n_edges; q += blockDim.x) {
    const int e = I.edge_begin + q;
    T Ri[9], Rj[9], ti_[3], tj[3], Rt[12];
    const T* pi = poses + 7 * (size_t)(I.frame_begin + ii[e]);
    const T* pj = poses + 7 * (size_t)(I.frame_begin + jj[e]);
    quat_to_rot<T, T>(pi + 3, Ri);
    quat_to_rot<T, T>(pj + 3, Rj);
    for (int m = 0; m < 3; ++m) { ti_[m] = pi[m]; tj[m] = pj[m]; }
    relative_pose<T>(Ri, ti_, Rj, tj, Rt, Rt + 9);
    const int k = I.patch_begin + kk[e], c = (p - 1) / 2;
    const float* cen = patches + ((size_t)k * p * p + (size_t)c * p + c) * 2;
    EdgeTerms<T> o;
    const float2 tg = reinterpret_cast<const float2*>(target)[e];
    const float2 wt = reinterpret_cast<const float2*>(weight)[e];
    bad |= !(wt.x >= 0.f && wt.y >= 0.f && wt.x <= FLT_MAX && wt.y <= FLT_MAX && fabsf(tg.x) <= FLT_MAX &&
             fabsf(tg.y) <= FLT_MAX);
    if (edge_eval<T>(Rt, ((T)cen[0] - cx) / fx, ((T)cen[1] - cy) / fy, inv_depth[k], fx, fy, cx, cy, z_min, tg.x,
                     tg.y, wt.x, wt.y, o))
      cst += 0.5 * ((double)o.w[0] * o.r[0] * o.r[0] + (double)o.w[1] * o.r[1] * o.r[1]);
  }
  if (bad) bad_in = 1;
  sred[threadIdx.x] = cst;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sred[threadIdx.x] += sred[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  dpvba_report* R = rep + blockIdx.x;
  R->cost[n_iters] = sred[0];
  int s = DPVBA_OK;
  for (int t = 0; t < n_iters; ++t) {
    const int q = blockIdx.x * stride + t;
    if (status[q]) s = DPVBA_ENOTPD;
    R->min_pivot[t] = (double)__uint_as_float(min_bits[q]);
    R->refine_resid[t] = refine ? refine[q] : 0.0;
    R->fp64_fallback[t] = fallback ? fallback[q] : 0;
  }
  if (bad_in) s = DPVBA_EINVAL;  // a target or weight outside the documented range
  R->status = s;
  R->n_iters = n_iters;
}

// ---------------------------------------------------------------- launchers

template <typename T>
int batch_solve_lds(int n_max, bool mixed, bool* lds_factor) {
  const int np1 = (n_max + 1) * (n_max + 2) / 2;  // packed, s appended as row n
  if (mixed) {
    *lds_factor = true;
    return 3 * n_max * 8 + 4 * n_max * 4 + np1 * 4;
  }
  const int full = (4 * n_max + np1) * (int)sizeof(T);
  *lds_factor = full <= 150 * 1024;
  return *lds_factor ? full : 2 * n_max * (int)sizeof(T);
}

template <typename TS, typename TA>
hipError_t launch_batch_gather(const BatchArgs<TS>& a, int n_inst, int n_max, hipStream_t st) {
  const int nf = n_max / 6, nlb = nf * (nf + 1) / 2;
  if (n_inst == 0 || nlb == 0) return hipSuccess;
  hipLaunchKernelGGL((batch_gather_kernel<TS, TA>), dim3((nlb + 3) / 4, n_inst), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_solve(const BatchArgs<T>& a, int n_inst, int lds_bytes, hipStream_t st) {
  if (n_inst == 0) return hipSuccess;
  hipError_t e = opt_in_lds((const void*)batch_solve_kernel<T>, lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((batch_solve_kernel<T>), dim3(n_inst), dim3(kBatchThreads), lds_bytes, st, a);
  return hipGetLastError();
}

hipError_t launch_batch_solve_mixed(const BatchArgs<float>& a, int n_inst, int lds_bytes, hipStream_t st) {
  if (n_inst == 0) return hipSuccess;
  hipError_t e = opt_in_lds((const void*)batch_solve_mixed_kernel, lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(batch_solve_mixed_kernel, dim3(n_inst), dim3(kBatchThreads), lds_bytes, st, a);
  return hipGetLastError();
}

hipError_t launch_batch_cost(const BatchInst* inst, int n_inst, const double* part_cost, const int* part_invalid,
                             dpvba_report* rep, int it, hipStream_t st) {
  if (n_inst == 0) return hipSuccess;
  hipLaunchKernelGGL(batch_cost_kernel, dim3((n_inst + 63) / 64), dim3(64), 0, st, inst, n_inst, part_cost,
                     part_invalid, rep, it);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_report(const BatchInst* inst, int n_inst, const T* poses, const T* inv_depth,
                               const float* patches, int p, const int* ii, const int* jj, const int* kk,
                               const float* target, const float* weight, T fx, T fy, T cx, T cy, T z_min,
                               const int* status, const unsigned int* min_bits, const double* refine,
                               const int* fallback, int stride, int n_iters, dpvba_report* rep, hipStream_t st) {
  if (n_inst == 0) return hipSuccess;
  hipLaunchKernelGGL((batch_report_kernel<T>), dim3(n_inst), dim3(256), 0, st, inst, poses, inv_depth, patches, p,
                     ii, jj, kk, target, weight, fx, fy, cx, cy, z_min, status, min_bits, refine, fallback, stride,
                     n_iters, rep);
  return hipGetLastError();
}

#define DPVBA_BATCH_INST(T)                                                                                       \
  template int batch_solve_lds<T>(int, bool, bool*);                                                             \
  template hipError_t launch_batch_solve<T>(const BatchArgs<T>&, int, int, hipStream_t);                         \
  template hipError_t launch_batch_report<T>(const BatchInst*, int, const T*, const T*, const float*, int,       \
                                             const int*, const int*, const int*, const float*, const float*, T, \
                                             T, T, T, T, const int*, const unsigned int*, const double*,         \
                                             const int*, int, int, dpvba_report*, hipStream_t);
DPVBA_BATCH_INST(float)
DPVBA_BATCH_INST(double)
#undef DPVBA_BATCH_INST
template hipError_t launch_batch_gather<float, float>(const BatchArgs<float>&, int, int, hipStream_t);
template hipError_t launch_batch_gather<float, double>(const BatchArgs<float>&, int, int, hipStream_t);
template hipError_t launch_batch_gather<double, double>(const BatchArgs<double>&, int, int, hipStream_t);

}  // namespace dpvba
