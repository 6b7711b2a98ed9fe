// Per-edge residual and Jacobians (DPV-SLAM eq. 2-3).
//
// For an edge e = (i, k, j) with relative pose T_ji = (R, t), patch-centre
// ray x^ = ((u - cx)/fx, (v - cy)/fy, 1) and inverse depth d:
//   q = R x^ + t d,  pi = (fx qx/qz + cx, fy qy/qz + cy),  r = pi - target,
//   J_d = Jpi t,  J_j = Jpi [ -d I | [q]x ]  (right perturbation of G_j),
// and J_i = -J_j Ad(T_ji) for the source pose.  The edge is valid iff d > 0
// and q_z > z_min d.
#pragma once

#include "common.h"

namespace dpvba {

template <typename T>
struct EdgeTerms {
  T Jj[2][6];
  T Jd[2];
  T r[2];
  T w[2];
};

template <typename T>
__device__ __forceinline__ bool edge_eval(const T* Rt, T xh0, T xh1, T d, T fx, T fy, T cx, T cy,
                                          T z_min, float tx, float ty, float wx, float wy,
                                          EdgeTerms<T>& o) {
  const T* R = Rt;
  const T* t = Rt + 9;
  const T q0 = R[0] * xh0 + R[1] * xh1 + R[2] + t[0] * d;
  const T q1 = R[3] * xh0 + R[4] * xh1 + R[5] + t[1] * d;
  const T q2 = R[6] * xh0 + R[7] * xh1 + R[8] + t[2] * d;
  if (!(d > (T)0) || !(q2 > z_min * d)) return false;
  const T iz = (T)1 / q2;
  const T ax0 = fx * iz, ax2 = -fx * q0 * iz * iz;  // Jpi row 0: (ax0, 0, ax2)
  const T by1 = fy * iz, by2 = -fy * q1 * iz * iz;  // Jpi row 1: (0, by1, by2)
  o.r[0] = fx * q0 * iz + cx - (T)tx;
  o.r[1] = fy * q1 * iz + cy - (T)ty;
  o.w[0] = (T)wx;
  o.w[1] = (T)wy;
  o.Jd[0] = ax0 * t[0] + ax2 * t[2];
  o.Jd[1] = by1 * t[1] + by2 * t[2];
  // translational part: -d Jpi
  o.Jj[0][0] = -d * ax0; o.Jj[0][1] = (T)0;     o.Jj[0][2] = -d * ax2;
  o.Jj[1][0] = (T)0;     o.Jj[1][1] = -d * by1; o.Jj[1][2] = -d * by2;
  // rotational part: row a of Jpi times [q]x is a x q
  o.Jj[0][3] = -ax2 * q1;
  o.Jj[0][4] = ax2 * q0 - ax0 * q2;
  o.Jj[0][5] = ax0 * q1;
  o.Jj[1][3] = by1 * q2 - by2 * q1;
  o.Jj[1][4] = by2 * q0;
  o.Jj[1][5] = -by1 * q0;
  return true;
}

// float32 terms with the residual evaluated in float64: the relative pose
// R64 / t64 (Rt64, 12 doubles) and the ray (x64_0, x64_1) in float64, the
// projection and its difference to the target rounded to float32 once.
// In float32 the projection (hundreds of pixels) would carry rounding errors
// of about 2^-24 of its size into a residual of a fraction of a pixel, and
// weakly observed depths amplify them.  Validity is decided in float64;
// the Jacobians use the float32 relative pose and the rounded point.
__device__ __forceinline__ bool edge_eval_r64(const float* Rt, const double* Rt64, double x64_0, double x64_1,
                                              float d, float fx, float fy, float cx, float cy, float z_min,
                                              float tx, float ty, float wx, float wy, EdgeTerms<float>& o) {
  const double* R = Rt64;
  const double* t = Rt64 + 9;
  const double dd = (double)d;
  const double q0 = R[0] * x64_0 + R[1] * x64_1 + R[2] + t[0] * dd;
  const double q1 = R[3] * x64_0 + R[4] * x64_1 + R[5] + t[1] * dd;
  const double q2 = R[6] * x64_0 + R[7] * x64_1 + R[8] + t[2] * dd;
  if (!(d > 0.f) || !(q2 > (double)z_min * dd)) return false;
  const double iz64 = 1.0 / q2;
  o.r[0] = (float)((double)fx * q0 * iz64 + (double)cx - (double)tx);
  o.r[1] = (float)((double)fy * q1 * iz64 + (double)cy - (double)ty);
  const float* tf = Rt + 9;
  const float p0 = (float)q0, p1 = (float)q1, p2 = (float)q2;
  const float iz = 1.f / p2;
  const float ax0 = fx * iz, ax2 = -fx * p0 * iz * iz;
  const float by1 = fy * iz, by2 = -fy * p1 * iz * iz;
  o.w[0] = wx;
  o.w[1] = wy;
  o.Jd[0] = ax0 * tf[0] + ax2 * tf[2];
  o.Jd[1] = by1 * tf[1] + by2 * tf[2];
  o.Jj[0][0] = -d * ax0; o.Jj[0][1] = 0.f;      o.Jj[0][2] = -d * ax2;
  o.Jj[1][0] = 0.f;      o.Jj[1][1] = -d * by1; o.Jj[1][2] = -d * by2;
  o.Jj[0][3] = -ax2 * p1;
  o.Jj[0][4] = ax2 * p0 - ax0 * p2;
  o.Jj[0][5] = ax0 * p1;
  o.Jj[1][3] = by1 * p2 - by2 * p1;
  o.Jj[1][4] = by2 * p0;
  o.Jj[1][5] = -by1 * p0;
  return true;
}

__device__ __forceinline__ int tri_index(int r, int c) {  // upper 6x6, r <= c
  return r * 6 - (r * (r - 1)) / 2 + (c - r);
}

template <typename T>
__device__ __forceinline__ T sym6(const T* M21, int r, int c) {
  return r <= c ? M21[tri_index(r, c)] : M21[tri_index(c, r)];
}

// Lower block (P >= Q) of a packed enumeration blk = P (P + 1) / 2 + Q.
__device__ __forceinline__ void lower_block_of(int blk, int& P, int& Q) {
  int p = (int)((sqrtf(8.0f * (float)blk + 1.0f) - 1.0f) * 0.5f);
  while (p * (p + 1) / 2 > blk) --p;
  while ((p + 1) * (p + 2) / 2 <= blk) ++p;
  P = p;
  Q = blk - p * (p + 1) / 2;
}

}  // namespace dpvba
