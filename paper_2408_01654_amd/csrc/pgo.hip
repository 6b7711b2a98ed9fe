// Sim(3) pose-graph optimisation of the classical loop closure (DPV-SLAM
// Sec. 3.3, "Optimization", eq. 5-7): absolute similarities S_i, smoothness
// residuals r_i = log(DeltaS_(i,i+1)^-1 S_i^-1 S_(i+1)) between successive
// keyframes and loop residuals r_jk = log(DeltaS^loop_jk S_j^-1 S_k), the sum
// of squares minimised by damped Gauss-Newton (Levenberg-Marquardt with a
// fixed damping), then G_i <- (t_i, R_i) and d <- d / s_i.
//
// Conventions (include/dpvba.h, dpvba_pgo_sim3): S = (R, t, s) maps x to
// s R x + t and is stored (t, q, s); tangent xi = (rho, phi, sigma); Exp(xi)
// = expm of [[sigma I + [phi]x, rho], [0, 0]]; right perturbations.  Every
// residual is written r_e = log(C_e S_a^-1 S_b) with a constant C_e
// (DeltaS^-1 of the initial successive similarities, or DeltaS^loop).
//
// Float64 throughout.  The Jacobian columns of each residual come from one
// forward-mode dual-number evaluation per perturbation direction (14 per
// residual), so they are exact derivatives of the computed residual.  The
// normal equations are assembled per 7 x 7 block in a fixed order (block
// lists from the host), damped, and solved by the library's dense Cholesky.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"
#include "dual.h"

namespace dpvba {

typedef Dual<double> D1;

template <typename T>
struct Sim3 {
  T R[9], t[3], s;
};

template <typename T>
__device__ __forceinline__ void mat3_mul(const T A[9], const T B[9], T C[9]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

template <typename T>
__device__ __forceinline__ Sim3<T> sim3_compose(const Sim3<T>& a, const Sim3<T>& b) {
  Sim3<T> c;
  mat3_mul<T>(a.R, b.R, c.R);
  for (int i = 0; i < 3; ++i)
    c.t[i] = a.s * (a.R[3 * i] * b.t[0] + a.R[3 * i + 1] * b.t[1] + a.R[3 * i + 2] * b.t[2]) + a.t[i];
  c.s = a.s * b.s;
  return c;
}

template <typename T>
__device__ __forceinline__ Sim3<T> sim3_inverse(const Sim3<T>& a) {
  Sim3<T> c;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) c.R[3 * i + j] = a.R[3 * j + i];
  const T is = (T)1 / a.s;
  for (int i = 0; i < 3; ++i)
    c.t[i] = -(c.R[3 * i] * a.t[0] + c.R[3 * i + 1] * a.t[1] + c.R[3 * i + 2] * a.t[2]) * is;
  c.s = is;
  return c;
}

// E = expm(A) and W = int_0^1 expm(tau A) dtau of a 3 x 3 matrix: Taylor
// series of A / 2^k (|A| / 2^k <= 1/2, 16 terms) and k doublings
// W(2B) = (I + e^B) W(B) / 2, e^(2B) = e^B e^B.  Polynomial operations
// only, so dual numbers carry exact derivatives through it.
template <typename T>
__device__ void expm_w3(const T A_in[9], T E[9], T W[9]) {
  double nrm = 0.0;
  for (int i = 0; i < 9; ++i) nrm += fabs(value_of(A_in[i]));
  int k = 0;
  while (nrm > 0.5 && k < 60) {
    nrm *= 0.5;
    ++k;
  }
  const double sc = ldexp(1.0, -k);
  T A[9], P[9], Q[9];
  for (int i = 0; i < 9; ++i) {
    A[i] = A_in[i] * sc;
    P[i] = (i % 4 == 0) ? (T)1 : (T)0;
    E[i] = P[i];
    W[i] = P[i];
  }
  for (int j = 1; j <= 16; ++j) {
    mat3_mul<T>(P, A, Q);
    const double inv = 1.0 / j, inv1 = 1.0 / (j + 1);
    for (int i = 0; i < 9; ++i) {
      P[i] = Q[i] * inv;
      E[i] += P[i];
      W[i] += P[i] * inv1;
    }
  }
  for (int m = 0; m < k; ++m) {
    T IE[9];
    for (int i = 0; i < 9; ++i) IE[i] = (E[i] + ((i % 4 == 0) ? (T)1 : (T)0)) * 0.5;
    mat3_mul<T>(IE, W, Q);
    for (int i = 0; i < 9; ++i) W[i] = Q[i];
    mat3_mul<T>(E, E, Q);
    for (int i = 0; i < 9; ++i) E[i] = Q[i];
  }
}

template <typename T>
__device__ __forceinline__ void sim3_generator(const T phi[3], T sigma, T M[9]) {
  M[0] = sigma;   M[1] = -phi[2]; M[2] = phi[1];
  M[3] = phi[2];  M[4] = sigma;   M[5] = -phi[0];
  M[6] = -phi[1]; M[7] = phi[0];  M[8] = sigma;
}

// Exp(xi), xi = (rho, phi, sigma): R = expm([phi]x), s = e^sigma,
// t = W(sigma I + [phi]x) rho.
template <typename T>
__device__ Sim3<T> sim3_exp(const T xi[7]) {
  Sim3<T> S;
  T M[9], E[9], W[9], Wr[9];
  const T z = (T)0;
  const T phi[3] = {xi[3], xi[4], xi[5]};
  sim3_generator<T>(phi, z, M);
  expm_w3<T>(M, S.R, Wr);
  sim3_generator<T>(phi, xi[6], M);
  expm_w3<T>(M, E, W);
  for (int i = 0; i < 3; ++i) S.t[i] = W[3 * i] * xi[0] + W[3 * i + 1] * xi[1] + W[3 * i + 2] * xi[2];
  S.s = exp(xi[6]);
  return S;
}

// log of (R, t, s) near the identity: phi from R (rotation angle below pi),
// sigma = log s, rho = W(sigma I + [phi]x)^-1 t.
template <typename T>
__device__ void sim3_log(const Sim3<T>& S, T xi[7]) {
  const T v[3] = {(S.R[7] - S.R[5]) * 0.5, (S.R[2] - S.R[6]) * 0.5, (S.R[3] - S.R[1]) * 0.5};
  const T s2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  const T c = (S.R[0] + S.R[4] + S.R[8] - (T)1) * 0.5;
  T f;  // theta / sin(theta)
  if (value_of(s2) < 1e-16) {
    f = (T)1 + s2 * (1.0 / 6.0);
  } else {
    const T sn = sqrt(s2);
    f = atan2(sn, c) / sn;
  }
  const T phi[3] = {f * v[0], f * v[1], f * v[2]};
  const T sigma = log(S.s);
  T M[9], E[9], W[9];
  sim3_generator<T>(phi, sigma, M);
  expm_w3<T>(M, E, W);
  // rho = W^-1 t by the adjugate
  const T c00 = W[4] * W[8] - W[5] * W[7], c01 = W[5] * W[6] - W[3] * W[8], c02 = W[3] * W[7] - W[4] * W[6];
  const T c10 = W[2] * W[7] - W[1] * W[8], c11 = W[0] * W[8] - W[2] * W[6], c12 = W[1] * W[6] - W[0] * W[7];
  const T c20 = W[1] * W[5] - W[2] * W[4], c21 = W[2] * W[3] - W[0] * W[5], c22 = W[0] * W[4] - W[1] * W[3];
  const T idet = (T)1 / (W[0] * c00 + W[1] * c01 + W[2] * c02);
  xi[0] = (c00 * S.t[0] + c10 * S.t[1] + c20 * S.t[2]) * idet;
  xi[1] = (c01 * S.t[0] + c11 * S.t[1] + c21 * S.t[2]) * idet;
  xi[2] = (c02 * S.t[0] + c12 * S.t[1] + c22 * S.t[2]) * idet;
  xi[3] = phi[0];
  xi[4] = phi[1];
  xi[5] = phi[2];
  xi[6] = sigma;
}

// Stored similarity (t, q, s) [8] -> Sim3.
template <typename T>
__device__ __forceinline__ Sim3<T> sim3_load(const double* p) {
  Sim3<T> S;
  double R[9];
  quat_to_rot<double, double>(p + 3, R);
  for (int i = 0; i < 9; ++i) S.R[i] = (T)R[i];
  for (int i = 0; i < 3; ++i) S.t[i] = (T)p[i];
  S.s = (T)p[7];
  return S;
}

// Initial similarities (t, q, 1) of the poses, and the smoothness constants
// C_i = DeltaS_(i,i+1)^-1 = S_(i+1)^-1 S_i (stored (t, q, s) by rotation
// matrix + quaternion of the pose pair's relative rotation).
__global__ void pgo_init_kernel(const double* poses, int n, double* sims) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int m = 0; m < 7; ++m) sims[8 * i + m] = poses[7 * i + m];
  sims[8 * i + 7] = 1.0;
}

// Constants of the residuals kept as rotation matrices: C [E, 13] = (R (9), t (3), s).
__global__ void pgo_constants_kernel(const double* sims, int n, const double* loop_rel, int n_loops, double* C) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n - 1 + n_loops) return;
  Sim3<double> c;
  if (e < n - 1) {
    const Sim3<double> a = sim3_load<double>(sims + 8 * e), b = sim3_load<double>(sims + 8 * (e + 1));
    c = sim3_compose<double>(sim3_inverse<double>(b), a);
  } else {
    c = sim3_load<double>(loop_rel + 8 * (e - (n - 1)));
  }
  double* o = C + 13 * (size_t)e;
  for (int i = 0; i < 9; ++i) o[i] = c.R[i];
  for (int i = 0; i < 3; ++i) o[9 + i] = c.t[i];
  o[12] = c.s;
}

// Thread (e, d): residual e differentiated along direction d of (delta_a,
// delta_b) (d < 7: delta_a, else delta_b).  r [E, 7]; J [E, 7, 14].
__global__ void __launch_bounds__(256) pgo_edge_kernel(const double* sims, const double* C, const int* ea,
                                                       const int* eb, int n_edges, double* r, double* J) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n_edges * 14) return;
  const int e = x / 14, d = x - (x / 14) * 14;
  Sim3<D1> Sa = sim3_load<D1>(sims + 8 * (size_t)ea[e]);
  Sim3<D1> Sb = sim3_load<D1>(sims + 8 * (size_t)eb[e]);
  D1 da[7], db[7];
  for (int m = 0; m < 7; ++m) {
    da[m] = D1(0.0, d == m ? 1.0 : 0.0);
    db[m] = D1(0.0, d == m + 7 ? 1.0 : 0.0);
  }
  Sa = sim3_compose<D1>(Sa, sim3_exp<D1>(da));
  Sb = sim3_compose<D1>(Sb, sim3_exp<D1>(db));
  Sim3<D1> Cs;
  const double* c = C + 13 * (size_t)e;
  for (int i = 0; i < 9; ++i) Cs.R[i] = D1(c[i]);
  for (int i = 0; i < 3; ++i) Cs.t[i] = D1(c[9 + i]);
  Cs.s = D1(c[12]);
  const Sim3<D1> X = sim3_compose<D1>(Cs, sim3_compose<D1>(sim3_inverse<D1>(Sa), Sb));
  D1 xi[7];
  sim3_log<D1>(X, xi);
  for (int m = 0; m < 7; ++m) J[((size_t)e * 7 + m) * 14 + d] = xi[m].d;
  if (d == 0)
    for (int m = 0; m < 7; ++m) r[7 * (size_t)e + m] = xi[m].v;
}

// sum of r^2 over all residuals, one workgroup, fixed order
__global__ void __launch_bounds__(256) pgo_cost_kernel(const double* r, int n, double* out) {
  __shared__ double part[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += r[i] * r[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = part[0];
}

// One workgroup of 64 threads per 7 x 7 block (p >= q) of the free poses:
// H_pq = sum over its contributions (e, side_p, side_q) of J_side_p^T J_side_q,
// in list order; diagonal blocks add the damping lambda (H_ii + 1) (lam_diag
// = lambda for Levenberg-Marquardt, 0 for additive damping) and report the
// damped diagonal.  Row-major n x n, lower blocks.
__global__ void __launch_bounds__(64) pgo_assemble_kernel(const double* J, const int* blk_pq, const int* blk_off,
                                                          const int* blk_src, int n, double lambda,
                                                          double lam_diag, double* H, double* d0) {
  const int b = blockIdx.x, t = threadIdx.x;
  if (t >= 49) return;
  const int p = blk_pq[2 * b], q = blk_pq[2 * b + 1];
  const int rr = t / 7, cc = t - (t / 7) * 7;
  double s = 0.0;
  for (int x = blk_off[b]; x < blk_off[b + 1]; ++x) {
    const int src = blk_src[x];
    const int e = src >> 2, sp = (src >> 1) & 1, sq = src & 1;
    const double* Je = J + (size_t)e * 7 * 14;
    for (int i = 0; i < 7; ++i) s += Je[i * 14 + 7 * sp + rr] * Je[i * 14 + 7 * sq + cc];
  }
  if (p == q && rr == cc) {
    s += lam_diag * s + lambda;
    d0[7 * p + rr] = s;
  }
  H[(size_t)(7 * p + rr) * n + 7 * q + cc] = s;
}

// rhs = -g over the free poses: g_p = sum over (e, side) of J_side^T r_e.
__global__ void pgo_gradient_kernel(const double* J, const double* r, const int* pose_off, const int* pose_src,
                                    int nf, double* rhs) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= 7 * nf) return;
  const int p = x / 7, c = x - (x / 7) * 7;
  double s = 0.0;
  for (int y = pose_off[p]; y < pose_off[p + 1]; ++y) {
    const int e = pose_src[y] >> 1, side = pose_src[y] & 1;
    for (int i = 0; i < 7; ++i) s += J[((size_t)e * 7 + i) * 14 + 7 * side + c] * r[7 * (size_t)e + i];
  }
  rhs[x] = -s;
}

// S_i <- S_i Exp(delta_i) for the free poses (quaternion composed with the
// rotation's half-angle quaternion, renormalised); skipped if the solve failed.
__global__ void pgo_retract_kernel(double* sims, int n, int n_fixed, const double* dx, const int* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || i < n_fixed || (status && *status)) return;
  double* S = sims + 8 * (size_t)i;
  const double* xi = dx + 7 * (size_t)(i - n_fixed);
  double R[9];
  quat_to_rot<double, double>(S + 3, R);
  // t <- s R (W rho) + t
  double M[9], E[9], W[9];
  const double phi[3] = {xi[3], xi[4], xi[5]};
  sim3_generator<double>(phi, xi[6], M);
  expm_w3<double>(M, E, W);
  double tw[3];
  for (int m = 0; m < 3; ++m) tw[m] = W[3 * m] * xi[0] + W[3 * m + 1] * xi[1] + W[3 * m + 2] * xi[2];
  const double s = S[7];
  for (int m = 0; m < 3; ++m) S[m] += s * (R[3 * m] * tw[0] + R[3 * m + 1] * tw[1] + R[3 * m + 2] * tw[2]);
  double h, ch, B, Cc;
  exp_coeffs<double>(phi, h, ch, B, Cc);
  const double qx = S[3], qy = S[4], qz = S[5], qw = S[6];
  const double dx_ = h * phi[0], dy = h * phi[1], dz = h * phi[2], dw = ch;
  double nx = qw * dx_ + qx * dw + qy * dz - qz * dy;
  double ny = qw * dy - qx * dz + qy * dw + qz * dx_;
  double nz = qw * dz + qx * dy - qy * dx_ + qz * dw;
  double nw = qw * dw - qx * dx_ - qy * dy - qz * dz;
  const double inv = 1.0 / sqrt(nx * nx + ny * ny + nz * nz + nw * nw);
  S[3] = nx * inv; S[4] = ny * inv; S[5] = nz * inv; S[6] = nw * inv;
  S[7] = s * exp(xi[6]);
}

// G_i <- (t_i, q_i) and d_k <- d_k / s_owner(k) (patches of frame i are
// [patch_off[i], patch_off[i+1])).
__global__ void pgo_apply_kernel(const double* sims, int n, const int* patch_off, float* poses, float* inv_depth) {
  const int i = blockIdx.x;
  if (i >= n) return;
  const double* S = sims + 8 * (size_t)i;
  if (threadIdx.x < 7) poses[7 * (size_t)i + threadIdx.x] = (float)S[threadIdx.x];
  const double is = 1.0 / S[7];
  for (int k = patch_off[i] + threadIdx.x; k < patch_off[i + 1]; k += blockDim.x)
    inv_depth[k] = (float)((double)inv_depth[k] * is);
}

hipError_t launch_pgo_init(const double* poses, int n, double* sims, const double* loop_rel, int n_loops, double* C,
                           hipStream_t st) {
  hipLaunchKernelGGL(pgo_init_kernel, dim3((n + 255) / 256), dim3(256), 0, st, poses, n, sims);
  const int E = n - 1 + n_loops;
  if (E > 0)
    hipLaunchKernelGGL(pgo_constants_kernel, dim3((E + 255) / 256), dim3(256), 0, st, sims, n, loop_rel, n_loops, C);
  return hipGetLastError();
}

hipError_t launch_pgo_linearise(const double* sims, const double* C, const int* ea, const int* eb, int n_edges,
                                double* r, double* J, double* cost, hipStream_t st) {
  if (n_edges > 0)
    hipLaunchKernelGGL(pgo_edge_kernel, dim3((n_edges * 14 + 255) / 256), dim3(256), 0, st, sims, C, ea, eb, n_edges,
                       r, J);
  if (cost) hipLaunchKernelGGL(pgo_cost_kernel, dim3(1), dim3(256), 0, st, r, 7 * n_edges, cost);
  return hipGetLastError();
}

hipError_t launch_pgo_normal(const double* J, const double* r, const int* blk_pq, const int* blk_off,
                             const int* blk_src, int n_blocks, const int* pose_off, const int* pose_src, int nf,
                             double lambda, double lam_diag, double* H, double* d0, double* rhs, hipStream_t st) {
  const int n = 7 * nf;
  if (n_blocks > 0)
    hipLaunchKernelGGL(pgo_assemble_kernel, dim3(n_blocks), dim3(64), 0, st, J, blk_pq, blk_off, blk_src, n, lambda,
                       lam_diag, H, d0);
  if (nf > 0)
    hipLaunchKernelGGL(pgo_gradient_kernel, dim3((n + 255) / 256), dim3(256), 0, st, J, r, pose_off, pose_src, nf,
                       rhs);
  return hipGetLastError();
}

hipError_t launch_pgo_retract(double* sims, int n, int n_fixed, const double* dx, const int* status, hipStream_t st) {
  hipLaunchKernelGGL(pgo_retract_kernel, dim3((n + 255) / 256), dim3(256), 0, st, sims, n, n_fixed, dx, status);
  return hipGetLastError();
}

hipError_t launch_pgo_apply(const double* sims, int n, const int* patch_off, float* poses, float* inv_depth,
                            hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(pgo_apply_kernel, dim3(n), dim3(128), 0, st, sims, n, patch_off, poses, inv_depth);
  return hipGetLastError();
}

}  // namespace dpvba
