// Adjoint of the unrolled Gauss-Newton iterations: gradients of a loss on
// the final poses and inverse depths with respect to the edge targets and
// confidence weights (the differentiable BA layer that supervises the
// predicted poses, Sec. 2; objective eq. 3).
//
// One iteration maps x_t = (poses, depths) to x_{t+1} = x_t (+) Delta with
// H~ Delta = -g, H~ = H + lam (Diag(H) + I), H = sum_e J_e^T W_e J_e and
// g = sum_e J_e^T W_e r_e over the free variables.  Walking the iterations
// backwards with the adjoint xbar of x_{t+1}:
//   1. retraction:  Deltabar = (dx_{t+1}/dDelta)^T xbar,  xbar_t = (dx_{t+1}/dx_t)^T xbar
//      (poses carry their adjoint in the stored (t, q) coordinates; the
//      differential of the retraction comes from dual-number evaluation);
//   2. solve:       u = H~^-1 Deltabar (Schur elimination with the stored
//      rows E_k / sqrt(C~_k), and a Cholesky solve of the reduced system),
//      so gbar = -u and H~bar = -u Delta^T;
//   3. damping:     Hbar = H~bar + lam Diag(H~bar);
//   4. per edge, on its 13 variables (xi_i, xi_j, d_k), per row c:
//        a_c = J_c u,  b_c = J_c Delta,
//        wbar_c   += -a_c b_c - lam sum_m J_cm^2 u_m Delta_m - r_c a_c,
//        taubar_c += w_c a_c            (r = pi - tau),
//        Jbar_c    = w_c (-(r_c + b_c) u - a_c Delta - 2 lam J_c o u o Delta),
//        rbar_c    = -w_c a_c;
//   5. xbar_t += d/dx [sum_c Jbar_c . J_c(x) + rbar_c r_c(x)], one dual
//      evaluation of the edge per coordinate of (t_i, q_i, t_j, q_j, d_k).
// Per-edge results are summed per pose and per patch in a fixed order.
#include "dual.h"
#include "edge.h"
#include "layout.h"

namespace dpvba {

constexpr int kEdgeAdj = 15;  // (t_i, q_i) 7, (t_j, q_j) 7, d_k 1

// Residual and the 2 x 13 Jacobian (J_i | J_j | J_d) of one edge at poses
// (t, q) of frames i and j and inverse depth d; false if the edge is invalid.
template <typename T>
__device__ __forceinline__ bool edge_full(const T* pi, const T* pj, T d, T xh0, T xh1, T fx, T fy, T cx, T cy,
                                          T z_min, float tx, float ty, T r[2], T J[2][13]) {
  T Ri[9], Rj[9], ti[3], tj[3], Rt[12];
  quat_to_rot<T, T>(pi + 3, Ri);
  quat_to_rot<T, T>(pj + 3, Rj);
  for (int m = 0; m < 3; ++m) { ti[m] = pi[m]; tj[m] = pj[m]; }
  relative_pose<T>(Ri, ti, Rj, tj, Rt, Rt + 9);
  EdgeTerms<T> o;
  if (!edge_eval<T>(Rt, xh0, xh1, d, fx, fy, cx, cy, z_min, tx, ty, 1.f, 1.f, o)) return false;
  for (int c = 0; c < 2; ++c) {
    T ji[6];
    adjoint_transpose_apply<T>(Rt, Rt + 9, o.Jj[c], ji);
    for (int m = 0; m < 6; ++m) {
      J[c][m] = -ji[m];
      J[c][6 + m] = o.Jj[c][m];
    }
    J[c][12] = o.Jd[c];
    r[c] = o.r[c];
  }
  return true;
}

// Step 4 and 5 for every edge.  u and Delta of the poses are indexed by free
// pose, of the depths by tile-order position.  Accumulates taubar and wbar
// into the caller's gradients and writes the edge's xbar contributions.
template <typename T>
__global__ void __launch_bounds__(128) edge_adjoint_kernel(
    const T* poses, const T* depth_t, const int* patch_pos, const float* patches, int p, const int* ii,
    const int* jj, const int* kk, const float* target, const float* weight, int n_edges, int n_fixed, T fx, T fy,
    T cx, T cy, T z_min, T lam_diag, const T* u_pose, const T* u_depth, const T* dxi, const T* dd,
    const int* status, T* grad_target, T* grad_weight, T* edge_xbar) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_edges) return;
  T* xb = edge_xbar + (size_t)kEdgeAdj * e;
  const bool skip = status && *status;
  const int i = ii[e], j = jj[e], k = kk[e];
  const int pos = patch_pos[k];
  const int c0 = (p - 1) / 2;
  const float* cen = patches + ((size_t)k * p * p + (size_t)c0 * p + c0) * 2;
  const T xh0 = ((T)cen[0] - cx) / fx, xh1 = ((T)cen[1] - cy) / fy;
  const T* pi = poses + 7 * (size_t)i;
  const T* pj = poses + 7 * (size_t)j;
  const T d = depth_t[pos];
  T r[2], J[2][13];
  const bool ok = !skip && edge_full<T>(pi, pj, d, xh0, xh1, fx, fy, cx, cy, z_min, target[2 * e],
                                        target[2 * e + 1], r, J);
  if (!ok) {
    for (int m = 0; m < kEdgeAdj; ++m) xb[m] = (T)0;
    return;
  }
  const bool fi = i >= n_fixed, fj = j >= n_fixed;
  T u[13], D[13];
  for (int m = 0; m < 6; ++m) {
    u[m] = fi ? u_pose[6 * (i - n_fixed) + m] : (T)0;
    D[m] = fi ? dxi[6 * (i - n_fixed) + m] : (T)0;
    u[6 + m] = fj ? u_pose[6 * (j - n_fixed) + m] : (T)0;
    D[6 + m] = fj ? dxi[6 * (j - n_fixed) + m] : (T)0;
  }
  u[12] = u_depth[pos];
  D[12] = dd[pos];
  T Jb[2][13], rb[2];
  for (int c = 0; c < 2; ++c) {
    const T w = (T)weight[2 * e + c];
    T a = (T)0, b = (T)0, sd = (T)0;
    for (int m = 0; m < 13; ++m) {
      a += J[c][m] * u[m];
      b += J[c][m] * D[m];
      sd += J[c][m] * J[c][m] * u[m] * D[m];
    }
    grad_weight[2 * e + c] += -a * b - lam_diag * sd - r[c] * a;
    grad_target[2 * e + c] += w * a;
    rb[c] = -w * a;
    for (int m = 0; m < 13; ++m)
      Jb[c][m] = w * (-(r[c] + b) * u[m] - a * D[m] - (T)2 * lam_diag * J[c][m] * u[m] * D[m]);
  }
  // directional derivatives of (r, J) along each stored coordinate
  using D1 = Dual<T>;
  for (int dir = 0; dir < kEdgeAdj; ++dir) {
    if ((dir < 7 && !fi) || (dir >= 7 && dir < 14 && !fj)) {
      xb[dir] = (T)0;
      continue;
    }
    D1 Pi[7], Pj[7];
    for (int m = 0; m < 7; ++m) {
      Pi[m] = D1(pi[m], dir == m ? (T)1 : (T)0);
      Pj[m] = D1(pj[m], dir == 7 + m ? (T)1 : (T)0);
    }
    const D1 dD(d, dir == 14 ? (T)1 : (T)0);
    D1 rD[2], JD[2][13];
    edge_full<D1>(Pi, Pj, dD, D1(xh0, (T)0), D1(xh1, (T)0), D1(fx, (T)0), D1(fy, (T)0), D1(cx, (T)0),
                  D1(cy, (T)0), D1(z_min, (T)0), target[2 * e], target[2 * e + 1], rD, JD);
    T acc = (T)0;
    for (int c = 0; c < 2; ++c) {
      acc += rb[c] * rD[c].d;
      for (int m = 0; m < 13; ++m) acc += Jb[c][m] * JD[c][m].d;
    }
    xb[dir] = acc;
  }
}

// Step 1 for every free pose: xbar of (t, q) before the retraction and the
// adjoint of its step, from the adjoint after it (in place in `pbar`).
template <typename T>
__global__ void retract_adjoint_kernel(const T* poses_t, const T* dxi, const int* status, int n_fixed, int n_frames,
                                       T* pbar, T* dxi_bar) {
  const int f = n_fixed + blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_frames) return;
  const int fr = f - n_fixed;
  T* pb = pbar + 7 * (size_t)f;
  if (status && *status) {  // the iteration was skipped: identity map
    for (int m = 0; m < 6; ++m) dxi_bar[6 * fr + m] = (T)0;
    return;
  }
  T out_bar[7];
  for (int m = 0; m < 7; ++m) out_bar[m] = pb[m];
  const T* x = poses_t + 7 * (size_t)f;
  const T* s = dxi + 6 * (size_t)fr;
  using D1 = Dual<T>;
  T res[13];
  for (int dir = 0; dir < 13; ++dir) {
    D1 pose[7], xi[6];
    for (int m = 0; m < 7; ++m) pose[m] = D1(x[m], dir == m ? (T)1 : (T)0);
    for (int m = 0; m < 6; ++m) xi[m] = D1(s[m], dir == 7 + m ? (T)1 : (T)0);
    retract_pose<D1, D1>(pose, xi);
    T acc = (T)0;
    for (int m = 0; m < 7; ++m) acc += out_bar[m] * pose[m].d;
    res[dir] = acc;
  }
  for (int m = 0; m < 7; ++m) pb[m] = res[m];
  for (int m = 0; m < 6; ++m) dxi_bar[6 * fr + m] = res[7 + m];
}

// Step 2, first half: per tile and block column x, the tile's share of
// -E C~^-1 Deltabar_d = -sum_k U_kx (1 / sqrt(C~_k)) Deltabar_d,k, written to
// the right-hand-side part of the tile's partial vector.
template <typename T>
__global__ void __launch_bounds__(256) tile_adjoint_rhs_kernel(const TileInfo* tiles, const T* U_s,
                                                               const T* pscale_s, const T* dbar, T* part_vec) {
  const TileInfo ti = tiles[blockIdx.x];
  const int W6 = 6 * ti.n_blk, Ws = tile_u_stride(ti.n_blk);
  const T* U = U_s + ti.u_begin;
  for (int x = threadIdx.x; x < W6; x += blockDim.x) {
    T v = (T)0;
    for (int k = 0; k < ti.n_patch; ++k) {
      const int q = ti.patch_begin + k;
      v += U[(size_t)k * Ws + x] * (pscale_s[2 * q] * dbar[q]);
    }
    part_vec[ti.vec_begin + x] = -v;
  }
}

// rhs = Deltabar_xi + the tiles' shares, summed per free pose in tile order.
template <typename T>
__global__ void vec_gather_add_kernel(const T* part_vec, const int* off, const int2* src, int n, const T* add,
                                      const int* status, T* out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  const int P_ = x / 6, m = x % 6;
  T v = add[x];
  for (int q = off[P_]; q < off[P_ + 1]; ++q) v += part_vec[src[q].x + m];
  out[x] = (status && *status) ? (T)0 : v;
}

// Step 2, second half, per patch of a tile: the depth part of u,
// u_d = C~^-1 (Deltabar_d - E^T u_p), and the forward depth step
// Delta_d = C~^-1 (-w - E^T Delta_xi), both from the stored rows.
template <typename T>
__global__ void __launch_bounds__(256) tile_adjoint_backsub_kernel(
    const TileInfo* tiles, const int* blk_pose, const T* U_s, const T* pscale_s, const T* dbar, const T* u_pose,
    const T* dxi, const int* status, T* u_depth, T* dd) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* sU = reinterpret_cast<T*>(lds_raw);
  const TileInfo ti = tiles[blockIdx.x];
  const int W6 = 6 * ti.n_blk, Ws = tile_u_stride(ti.n_blk);
  T* sX = sU + W6;
  for (int x = threadIdx.x; x < W6; x += blockDim.x) {
    const int f = blk_pose[ti.blk_begin + x / 6];
    sU[x] = u_pose[6 * f + x % 6];
    sX[x] = dxi[6 * f + x % 6];
  }
  __syncthreads();
  const bool skip = status && *status;
  const T* U = U_s + ti.u_begin;
  for (int k = threadIdx.x; k < ti.n_patch; k += blockDim.x) {
    const int q = ti.patch_begin + k;
    const T is = pscale_s[2 * q], rs = pscale_s[2 * q + 1];
    T du = (T)0, dx = (T)0;
    for (int x = 0; x < W6; ++x) {
      const T uk = U[(size_t)k * Ws + x];
      du += uk * sU[x];
      dx += uk * sX[x];
    }
    u_depth[q] = skip ? (T)0 : is * (dbar[q] * is - du);
    dd[q] = skip ? (T)0 : -(rs + dx) * is;
  }
}

// Step 5 sums.  Poses: xbar_t of every free pose gets its edges' shares
// (pose_src holds 2 e + side, side 0 = source, 1 = target); one workgroup
// per pose, thread t takes list entries t, t + 256, ... and the partial
// sums are combined by a fixed tree, so the result does not depend on timing.
template <typename T>
__global__ void __launch_bounds__(256) pose_reduce_kernel(const T* edge_xbar, const int* pose_off,
                                                          const int* pose_src, int n_fixed, T* pbar) {
  __shared__ T red[7][256];
  const int f = n_fixed + blockIdx.x;
  T v[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int q = pose_off[f] + threadIdx.x; q < pose_off[f + 1]; q += blockDim.x) {
    const int s = pose_src[q];
    const T* x = edge_xbar + (size_t)kEdgeAdj * (s >> 1) + 7 * (s & 1);
#pragma unroll
    for (int m = 0; m < 7; ++m) v[m] += x[m];
  }
#pragma unroll
  for (int m = 0; m < 7; ++m) red[m][threadIdx.x] = v[m];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int m = 0; m < 7; ++m) red[m][threadIdx.x] += red[m][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 7) pbar[7 * (size_t)f + threadIdx.x] += red[threadIdx.x][0];
}

// Depths: per tile-order patch position, its edges in edge order.
template <typename T>
__global__ void patch_reduce_kernel(const T* edge_xbar, const int* tile_patch, const int* pcount, const int* pedges,
                                    int n_tp, T* dbar) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_tp) return;
  const int k = tile_patch[q];
  T v = (T)0;
  for (int a = pcount[k]; a < pcount[k + 1]; ++a) v += edge_xbar[(size_t)kEdgeAdj * pedges[a] + 14];
  dbar[q] += v;
}

// Caller-order depth adjoint to tile order (zero without one).
template <typename T>
__global__ void depth_to_tile_kernel(const T* src, const int* tile_patch, int n_tp, T* dst) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_tp) return;
  dst[q] = src ? src[tile_patch[q]] : (T)0;
}

template <typename T>
__global__ void fill_kernel(T* x, long long n, T v) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) x[q] = v;
}

template <typename T>
__global__ void copy_kernel(const T* src, T* dst, long long n) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) dst[q] = src[q];
}

// ---------------------------------------------------------------- launchers

static inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename T>
hipError_t launch_edge_adjoint(const T* poses, const T* depth_t, const int* patch_pos, const float* patches, int p,
                               const int* ii, const int* jj, const int* kk, const float* target,
                               const float* weight, int n_edges, int n_fixed, T fx, T fy, T cx, T cy, T z_min,
                               T lambda, const T* u_pose, const T* u_depth, const T* dxi, const T* dd,
                               const int* status, T* grad_target, T* grad_weight, T* edge_xbar, hipStream_t st) {
  if (n_edges == 0) return hipSuccess;
  hipLaunchKernelGGL((edge_adjoint_kernel<T>), dim3(blocks_for(n_edges, 128)), dim3(128), 0, st, poses, depth_t,
                     patch_pos, patches, p, ii, jj, kk, target, weight, n_edges, n_fixed, fx, fy, cx, cy, z_min,
                     lambda, u_pose, u_depth, dxi, dd, status, grad_target, grad_weight, edge_xbar);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_retract_adjoint(const T* poses_t, const T* dxi, const int* status, int n_fixed, int n_frames,
                                  T* pbar, T* dxi_bar, hipStream_t st) {
  const int nf = n_frames - n_fixed;
  if (nf <= 0) return hipSuccess;
  hipLaunchKernelGGL((retract_adjoint_kernel<T>), dim3(blocks_for(nf, 64)), dim3(64), 0, st, poses_t, dxi, status,
                     n_fixed, n_frames, pbar, dxi_bar);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_rhs(const TileInfo* tiles, int n_tiles, const T* U_s, const T* pscale_s, const T* dbar,
                              T* part_vec, const int* v_off, const int2* v_src, int n_free, const T* dxi_bar,
                              const int* status, T* rhs, hipStream_t st) {
  if (n_tiles > 0)
    hipLaunchKernelGGL((tile_adjoint_rhs_kernel<T>), dim3(n_tiles), dim3(256), 0, st, tiles, U_s, pscale_s, dbar,
                       part_vec);
  const int n = 6 * n_free;
  if (n > 0)
    hipLaunchKernelGGL((vec_gather_add_kernel<T>), dim3(blocks_for(n, 256)), dim3(256), 0, st, part_vec, v_off,
                       v_src, n, dxi_bar, status, rhs);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_backsub(const TileInfo* tiles, int n_tiles, int max_w6, const int* blk_pose,
                                  const T* U_s, const T* pscale_s, const T* dbar, const T* u_pose, const T* dxi,
                                  const int* status, T* u_depth, T* dd, hipStream_t st) {
  if (n_tiles == 0) return hipSuccess;
  const int lds = 2 * max_w6 * (int)sizeof(T);
  hipLaunchKernelGGL((tile_adjoint_backsub_kernel<T>), dim3(n_tiles), dim3(256), lds, st, tiles, blk_pose, U_s,
                     pscale_s, dbar, u_pose, dxi, status, u_depth, dd);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_reduce(const T* edge_xbar, const int* pose_off, const int* pose_src, int n_fixed,
                                 int n_frames, T* pbar, const int* tile_patch, const int* pcount, const int* pedges,
                                 int n_tp, T* dbar, hipStream_t st) {
  const int nfree = n_frames - n_fixed;
  if (nfree > 0)
    hipLaunchKernelGGL((pose_reduce_kernel<T>), dim3(nfree), dim3(256), 0, st, edge_xbar, pose_off, pose_src,
                       n_fixed, pbar);
  if (n_tp > 0)
    hipLaunchKernelGGL((patch_reduce_kernel<T>), dim3(blocks_for(n_tp, 128)), dim3(128), 0, st, edge_xbar,
                       tile_patch, pcount, pedges, n_tp, dbar);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_depth_to_tile(const T* src, const int* tile_patch, int n_tp, T* dst, hipStream_t st) {
  if (n_tp == 0) return hipSuccess;
  hipLaunchKernelGGL((depth_to_tile_kernel<T>), dim3(blocks_for(n_tp, 256)), dim3(256), 0, st, src, tile_patch,
                     n_tp, dst);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T* x, long long n, T v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((fill_kernel<T>), dim3(blocks_for(n, 256)), dim3(256), 0, st, x, n, v);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_copy(const T* src, T* dst, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((copy_kernel<T>), dim3(blocks_for(n, 256)), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

#define DPVBA_ADJ_INST(T)                                                                                          \
  template hipError_t launch_edge_adjoint<T>(const T*, const T*, const int*, const float*, int, const int*,       \
                                             const int*, const int*, const float*, const float*, int, int, T, T, \
                                             T, T, T, T, const T*, const T*, const T*, const T*, const int*, T*, \
                                             T*, T*, hipStream_t);                                                \
  template hipError_t launch_retract_adjoint<T>(const T*, const T*, const int*, int, int, T*, T*, hipStream_t);   \
  template hipError_t launch_adjoint_rhs<T>(const TileInfo*, int, const T*, const T*, const T*, T*, const int*,   \
                                            const int2*, int, const T*, const int*, T*, hipStream_t);            \
  template hipError_t launch_adjoint_backsub<T>(const TileInfo*, int, int, const int*, const T*, const T*,       \
                                                const T*, const T*, const T*, const int*, T*, T*, hipStream_t);  \
  template hipError_t launch_adjoint_reduce<T>(const T*, const int*, const int*, int, int, T*, const int*,       \
                                               const int*, const int*, int, T*, hipStream_t);                    \
  template hipError_t launch_depth_to_tile<T>(const T*, const int*, int, T*, hipStream_t);                        \
  template hipError_t launch_fill<T>(T*, long long, T, hipStream_t);                                              \
  template hipError_t launch_copy<T>(const T*, T*, long long, hipStream_t);
DPVBA_ADJ_INST(float)
DPVBA_ADJ_INST(double)
template hipError_t launch_fill<int>(int*, long long, int, hipStream_t);
#undef DPVBA_ADJ_INST

}  // namespace dpvba
