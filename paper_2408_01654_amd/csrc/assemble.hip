// Large-path and auxiliary kernels: gather of the tiles' shares into the
// dense damped reduced camera system (DPV-SLAM Appendix A), per-edge cost of
// eq. (3) at an iterate, report reductions, and the full-patch reprojection
// of eq. (2).
#include "edge.h"
#include "dpvba.h"

namespace dpvba {

// Gather of the per-tile vectors into the right-hand side s and Diag(B):
// one wavefront per free pose P, lane l summing the pose's shares l, l + 64,
// ... (six right-hand-side and six Diag(B) entries each), then a butterfly
// over the lanes; fixed order, so the result is reproducible.  The shares
// (type TP) are summed in the output type T, so float shares gathered into
// double are combined without further rounding error.  With pos, free pose
// P's rows go to block row pos[P] (a symmetric permutation of the system;
// null: the poses' own order).
template <typename TP, typename T>
__global__ void __launch_bounds__(256) gather_vec_kernel(const TP* part_vec, const int* off, const int2* src,
                                                         int n_free, T* rhs, T* dB, const int* pos) {
  const int P_ = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (P_ >= n_free) return;
  T v[6], d[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) v[m] = d[m] = (T)0;
  for (int q = off[P_] + lane; q < off[P_ + 1]; q += 64) {
    const int2 sq = src[q];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      v[m] += (T)part_vec[sq.x + m];
      d[m] += (T)part_vec[sq.y + m];
    }
  }
#pragma unroll
  for (int h = 32; h >= 1; h >>= 1)
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      v[m] += __shfl_xor(v[m], h);
      d[m] += __shfl_xor(d[m], h);
    }
  if (lane < 6) {
    T vv = v[0], dd = d[0];
#pragma unroll
    for (int m = 1; m < 6; ++m)
      if (lane == m) {
        vv = v[m];
        dd = d[m];
      }
    const int xd = 6 * (pos ? pos[P_] : P_) + lane;
    rhs[xd] = vv;
    dB[xd] = dd;
  }
}

// Gather of every lower 6x6 block (P >= Q) of the damped reduced system from
// the tile partials (zero where no tile contributes), with the damping
// lam_diag Diag(B) + lambda added to the diagonal.  `mirror` also writes the
// upper triangle.  With pos, block (P, Q) goes to (pos[P], pos[Q]), as its
// transpose into the lower triangle where pos[P] < pos[Q]; dB is then in
// the permuted order (gather_vec_kernel with the same pos).
template <typename TP, typename T>
__global__ void gather_S_kernel(const TP* part_S, const int* off, const int* src, int n_free, T* S,
                                const T* dB, T lambda, T lam_diag, int mirror, T* diag_out, const int* pos) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nblk = (long long)n_free * (n_free + 1) / 2;
  if (g >= nblk * 36) return;
  const int blk = (int)(g / 36), e = (int)(g % 36), r = e / 6, c = e % 6;
  int Pb, Qb;
  lower_block_of(blk, Pb, Qb);
  if (Pb == Qb && r < c) return;
  T v = (T)0;
  const int lo = off[blk], hi = off[blk + 1];
  const int eo = c * 6 + r;  // the tiles store upper entries of their block pairs
  int q = lo;
  for (; q + 4 <= hi; q += 4) {
    const T v0 = (T)part_S[src[q] + eo], v1 = (T)part_S[src[q + 1] + eo];
    const T v2 = (T)part_S[src[q + 2] + eo], v3 = (T)part_S[src[q + 3] + eo];
    v += v0; v += v1; v += v2; v += v3;
  }
  for (; q < hi; ++q) v += (T)part_S[src[q] + eo];
  const int n = 6 * n_free;
  int row = 6 * Pb + r, col = 6 * Qb + c;
  if (pos) {
    const int Pd = pos[Pb], Qd = pos[Qb];
    row = Pd >= Qd ? 6 * Pd + r : 6 * Qd + c;
    col = Pd >= Qd ? 6 * Qd + c : 6 * Pd + r;
  }
  if (row == col) {
    v += lam_diag * dB[row] + lambda;
    if (diag_out) diag_out[row] = v;
  }
  S[(size_t)row * n + col] = v;
  if (mirror && row != col) S[(size_t)col * n + row] = v;
}

// Gather of the blocks inside the envelope of the reduced system in its
// system order only (env: per block its block row and column in that order,
// the poses' lower block it comes from and whether it is that block's
// transpose); the entries outside the envelope are zero and stay zero
// through the factorisation, so the caller zeroes them once.  Same sums in
// the same order as gather_S_kernel.  `mirror` also writes the upper
// triangle.
template <typename TP, typename T>
__global__ void gather_S_env_kernel(const TP* part_S, const int* off, const int* src, const int4* env, int n_env,
                                    int n, T* S, const T* dB, T lambda, T lam_diag, T* diag_out, int mirror) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (long long)n_env * 36) return;
  const int b = (int)(g / 36), e = (int)(g % 36), r = e / 6, c = e % 6;
  const int4 E = env[b];
  if (E.x == E.y && r < c) return;
  const int eo = E.w ? r * 6 + c : c * 6 + r;  // the tiles store upper entries of their block pairs
  const int lo = off[E.z], hi = off[E.z + 1];
  T v = (T)0;
  int q = lo;
  for (; q + 4 <= hi; q += 4) {
    const T v0 = (T)part_S[src[q] + eo], v1 = (T)part_S[src[q + 1] + eo];
    const T v2 = (T)part_S[src[q + 2] + eo], v3 = (T)part_S[src[q + 3] + eo];
    v += v0; v += v1; v += v2; v += v3;
  }
  for (; q < hi; ++q) v += (T)part_S[src[q] + eo];
  const int row = 6 * E.x + r, col = 6 * E.y + c;
  if (row == col) {
    v += lam_diag * dB[row] + lambda;
    if (diag_out) diag_out[row] = v;
  }
  S[(size_t)row * n + col] = v;
  if (mirror && row != col) S[(size_t)col * n + row] = v;
}

// Cost of every edge at an iterate, summed per block in a fixed order.
template <typename T, typename P>
__global__ void __launch_bounds__(256) edge_cost_kernel(const P* poses, const P* inv_depth,
                                                         const float* patches, int p, const int* ii,
                                                         const int* jj, const int* kk,
                                                         const float* target, const float* weight,
                                                         int n_edges, T fx, T fy, T cx, T cy, T z_min,
                                                         double* part) {
  __shared__ double sred[256];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  double cst = 0.0;
  if (e < n_edges) {
    T Ri[9], Rj[9], ti_[3], tj[3], Rt[12];
    const P* pi = poses + 7 * (size_t)ii[e];
    const P* pj = poses + 7 * (size_t)jj[e];
    quat_to_rot<T, P>(pi + 3, Ri);
    quat_to_rot<T, P>(pj + 3, Rj);
    for (int m = 0; m < 3; ++m) { ti_[m] = (T)pi[m]; tj[m] = (T)pj[m]; }
    relative_pose<T>(Ri, ti_, Rj, tj, Rt, Rt + 9);
    const int k = kk[e], c = (p - 1) / 2;
    const float* cen = patches + ((size_t)k * p * p + (size_t)c * p + c) * 2;
    EdgeTerms<T> o;
    const float2 tg = reinterpret_cast<const float2*>(target)[e];
    const float2 wt = reinterpret_cast<const float2*>(weight)[e];
    if (edge_eval<T>(Rt, ((T)cen[0] - cx) / fx, ((T)cen[1] - cy) / fy, (T)inv_depth[k], fx, fy, cx,
                     cy, z_min, tg.x, tg.y, wt.x, wt.y, o))
      cst = 0.5 * ((double)o.w[0] * o.r[0] * o.r[0] + (double)o.w[1] * o.r[1] * o.r[1]);
  }
  sred[threadIdx.x] = cst;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sred[threadIdx.x] += sred[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sred[0];
}

// Reduce per-tile costs / invalid counts of one iteration into the report.
__global__ void report_reduce_kernel(const double* part_cost, const int* part_invalid, int n,
                                     double* cost_out, int* invalid_out) {
  __shared__ double sc[256];
  __shared__ int si[256];
  double c = 0.0;
  int v = 0;
  // fixed partition: thread t sums a contiguous range, then a fixed tree
  const int per = (n + 255) / 256;
  const int lo = threadIdx.x * per, hi = min(n, lo + per);
  for (int q = lo; q < hi; ++q) {
    c += part_cost[q];
    if (part_invalid) v += part_invalid[q];
  }
  sc[threadIdx.x] = c;
  si[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sc[threadIdx.x] += sc[threadIdx.x + w];
      si[threadIdx.x] += si[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *cost_out = sc[0];
    if (invalid_out) *invalid_out = si[0];
  }
}

// Reprojection of every pixel of every edge's patch (eq. 2).
template <typename T>
__global__ void reproject_kernel(const float* poses, const float* inv_depth, const float* patches,
                                 int p, const int* ii, const int* jj, const int* kk, int n_edges,
                                 T fx, T fy, T cx, T cy, T z_min, float* coords, uint8_t* valid) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_edges) return;
  T Ri[9], Rj[9], ti_[3], tj[3], R[9], t[3];
  const float* pi = poses + 7 * (size_t)ii[e];
  const float* pj = poses + 7 * (size_t)jj[e];
  quat_to_rot<T, float>(pi + 3, Ri);
  quat_to_rot<T, float>(pj + 3, Rj);
  for (int m = 0; m < 3; ++m) { ti_[m] = pi[m]; tj[m] = pj[m]; }
  relative_pose<T>(Ri, ti_, Rj, tj, R, t);
  const int k = kk[e];
  const T d = inv_depth[k];
  const float* pk = patches + (size_t)k * p * p * 2;
  float* out = coords + (size_t)e * p * p * 2;
  const int c = (p - 1) / 2;
  for (int px = 0; px < p * p; ++px) {
    const T x = ((T)pk[2 * px] - cx) / fx, y = ((T)pk[2 * px + 1] - cy) / fy;
    const T q0 = R[0] * x + R[1] * y + R[2] + t[0] * d;
    const T q1 = R[3] * x + R[4] * y + R[5] + t[1] * d;
    const T q2 = R[6] * x + R[7] * y + R[8] + t[2] * d;
    out[2 * px] = (float)(fx * q0 / q2 + cx);
    out[2 * px + 1] = (float)(fy * q1 / q2 + cy);
    if (valid && px == c * p + c) valid[e] = (d > (T)0 && q2 > z_min * d) ? 1 : 0;
  }
}


// Per-solve report state: step status words and pivot minima per iteration.
__global__ void report_init_kernel(int* status, unsigned int* min_bits, int n, int* err_clear) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    status[i] = 0;
    min_bits[i] = 0x7f7fffffu;  // bits of FLT_MAX
  }
  if (i == 0 && err_clear) *err_clear = 0;
}

__global__ void report_finalize_kernel(dpvba_report* rep, const int* status, const unsigned int* min_bits,
                                       int n_iters, const int* err, const double* refine, const int* fallback) {
  if (threadIdx.x != 0) return;
  int st = DPVBA_OK;
  for (int t = 0; t < n_iters; ++t) {
    if (status[t]) st = DPVBA_ENOTPD;
    rep->min_pivot[t] = (double)__uint_as_float(min_bits[t]);
    rep->refine_resid[t] = refine ? refine[t] : 0.0;
    rep->fp64_fallback[t] = fallback ? fallback[t] : 0;
  }
  if (err && (*err & kErrInput)) st = DPVBA_EINVAL;
  if (err && (*err & (kErrBarrier | kErrChain))) st = DPVBA_EHIP;
  rep->status = st;
  rep->n_iters = n_iters;
}

hipError_t launch_report_init(int* status, unsigned int* min_bits, int n, hipStream_t st, int* err_clear) {
  hipLaunchKernelGGL(report_init_kernel, dim3((n + 63) / 64), dim3(64), 0, st, status, min_bits, n, err_clear);
  return hipGetLastError();
}

hipError_t launch_report_finalize(dpvba_report* rep, const int* status, const unsigned int* min_bits,
                                  int n_iters, const int* err, hipStream_t st, const double* refine,
                                  const int* fallback) {
  hipLaunchKernelGGL(report_finalize_kernel, dim3(1), dim3(64), 0, st, rep, status, min_bits, n_iters, err, refine,
                     fallback);
  return hipGetLastError();
}

// ---------------------------------------------------------------- launchers

template <typename TP, typename T>
hipError_t launch_gather_as(const TP* part_S, const TP* part_vec, const int* s_off, const int* s_src,
                            const int* v_off, const int2* v_src, int n_free, T* S, T* rhs, T* dB, T lambda,
                            T lam_diag, int mirror, T* diag_out, hipStream_t st, const int* pos) {
  if (n_free == 0) return hipSuccess;
  hipLaunchKernelGGL((gather_vec_kernel<TP, T>), dim3((n_free + 3) / 4), dim3(256), 0, st, part_vec, v_off,
                     v_src, n_free, rhs, dB, pos);
  const long long tot = (long long)n_free * (n_free + 1) / 2 * 36;
  hipLaunchKernelGGL((gather_S_kernel<TP, T>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, part_S,
                     s_off, s_src, n_free, S, dB, lambda, lam_diag, mirror, diag_out, pos);
  return hipGetLastError();
}

template <typename TP, typename T>
hipError_t launch_gather_env_as(const TP* part_S, const TP* part_vec, const int* s_off, const int* s_src,
                                const int* v_off, const int2* v_src, int n_free, const int4* env, int n_env, T* S,
                                T* rhs, T* dB, T lambda, T lam_diag, T* diag_out, hipStream_t st, const int* pos,
                                int mirror) {
  if (n_free == 0) return hipSuccess;
  const int n = 6 * n_free;
  hipLaunchKernelGGL((gather_vec_kernel<TP, T>), dim3((n_free + 3) / 4), dim3(256), 0, st, part_vec, v_off, v_src,
                     n_free, rhs, dB, pos);
  const long long tot = (long long)n_env * 36;
  if (tot > 0)
    hipLaunchKernelGGL((gather_S_env_kernel<TP, T>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, part_S,
                       s_off, s_src, env, n_env, n, S, dB, lambda, lam_diag, diag_out, mirror);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather_env(const T* part_S, const T* part_vec, const int* s_off, const int* s_src,
                             const int* v_off, const int2* v_src, int n_free, const int4* env, int n_env, T* S, T* rhs,
                             T* dB, T lambda, T lam_diag, T* diag_out, hipStream_t st, const int* pos) {
  return launch_gather_env_as<T, T>(part_S, part_vec, s_off, s_src, v_off, v_src, n_free, env, n_env, S, rhs, dB,
                                    lambda, lam_diag, diag_out, st, pos, 0);
}

template <typename T>
hipError_t launch_gather(const T* part_S, const T* part_vec, const int* s_off, const int* s_src,
                         const int* v_off, const int2* v_src, int n_free, T* S, T* rhs, T* dB, T lambda,
                         T lam_diag, int mirror, T* diag_out, hipStream_t st, const int* pos) {
  return launch_gather_as<T, T>(part_S, part_vec, s_off, s_src, v_off, v_src, n_free, S, rhs, dB, lambda, lam_diag,
                                mirror, diag_out, st, pos);
}

// Row blocks of width bw between the poses' order and a permuted system
// order: block p of the system is pose perm[p].  to_system: dst block p =
// src block perm[p]; else dst block perm[p] = src block p.
template <typename T>
__global__ void permute_blocks_kernel(const T* src, T* dst, const int* perm, int n_blk, int bw, int to_system) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= bw * n_blk) return;
  const int p = x / bw, m = x - bw * p, q = bw * perm[p] + m;
  if (to_system) dst[x] = src[q];
  else dst[q] = src[x];
}

template <typename T>
hipError_t launch_permute_blocks(const T* src, T* dst, const int* perm, int n_blk, int bw, int to_system,
                                 hipStream_t st) {
  if (n_blk == 0) return hipSuccess;
  hipLaunchKernelGGL((permute_blocks_kernel<T>), dim3((bw * n_blk + 255) / 256), dim3(256), 0, st, src, dst, perm,
                     n_blk, bw, to_system);
  return hipGetLastError();
}

template <typename T, typename P>
hipError_t launch_edge_cost(const P* poses, const P* inv_depth, const float* patches, int p, const int* ii,
                            const int* jj, const int* kk, const float* target, const float* weight,
                            int n_edges, T fx, T fy, T cx, T cy, T z_min, double* part, hipStream_t st) {
  const int nblk = (n_edges + 255) / 256;
  if (nblk == 0) return hipSuccess;
  hipLaunchKernelGGL((edge_cost_kernel<T, P>), dim3(nblk), dim3(256), 0, st, poses, inv_depth, patches, p,
                     ii, jj, kk, target, weight, n_edges, fx, fy, cx, cy, z_min, part);
  return hipGetLastError();
}

hipError_t launch_report_reduce(const double* part_cost, const int* part_invalid, int n, double* cost_out,
                                int* invalid_out, hipStream_t st) {
  hipLaunchKernelGGL(report_reduce_kernel, dim3(1), dim3(256), 0, st, part_cost, part_invalid, n, cost_out,
                     invalid_out);
  return hipGetLastError();
}

hipError_t launch_reproject(const float* poses, const float* inv_depth, const float* patches, int p,
                            const int* ii, const int* jj, const int* kk, int n_edges, float fx, float fy,
                            float cx, float cy, float z_min, float* coords, uint8_t* valid, hipStream_t st) {
  if (n_edges == 0) return hipSuccess;
  hipLaunchKernelGGL((reproject_kernel<float>), dim3((n_edges + 255) / 256), dim3(256), 0, st, poses,
                     inv_depth, patches, p, ii, jj, kk, n_edges, fx, fy, cx, cy, z_min, coords, valid);
  return hipGetLastError();
}

#define DPVBA_INSTANTIATE(T, P)                                                                        \
  template hipError_t launch_edge_cost<T, P>(const P*, const P*, const float*, int, const int*,        \
                                             const int*, const int*, const float*, const float*, int,  \
                                             T, T, T, T, T, double*, hipStream_t);

DPVBA_INSTANTIATE(float, float)
DPVBA_INSTANTIATE(double, double)
template hipError_t launch_gather<float>(const float*, const float*, const int*, const int*, const int*,
                                         const int2*, int, float*, float*, float*, float, float, int, float*,
                                         hipStream_t, const int*);
template hipError_t launch_gather<double>(const double*, const double*, const int*, const int*, const int*,
                                          const int2*, int, double*, double*, double*, double, double, int,
                                          double*, hipStream_t, const int*);
template hipError_t launch_gather_as<float, double>(const float*, const float*, const int*, const int*,
                                                    const int*, const int2*, int, double*, double*, double*,
                                                    double, double, int, double*, hipStream_t, const int*);
template hipError_t launch_gather_env<float>(const float*, const float*, const int*, const int*, const int*,
                                             const int2*, int, const int4*, int, float*, float*, float*, float, float,
                                             float*, hipStream_t, const int*);
template hipError_t launch_gather_env<double>(const double*, const double*, const int*, const int*, const int*,
                                              const int2*, int, const int4*, int, double*, double*, double*, double,
                                              double, double*, hipStream_t, const int*);
template hipError_t launch_gather_env_as<float, double>(const float*, const float*, const int*, const int*,
                                                        const int*, const int2*, int, const int4*, int, double*,
                                                        double*, double*, double, double, double*, hipStream_t,
                                                        const int*, int);
template hipError_t launch_permute_blocks<float>(const float*, float*, const int*, int, int, int, hipStream_t);
template hipError_t launch_permute_blocks<double>(const double*, double*, const int*, int, int, int, hipStream_t);

}  // namespace dpvba
