// Device-side helpers shared by the kernels of the patch-graph BA library.
//
// Geometry: poses are camera-to-world (t, q), q = (x, y, z, w); perturbations
// act on the right, G <- G Exp(xi), xi = (rho, phi).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.h"

namespace dpvba {

// Raise a kernel's dynamic shared-memory limit when it needs more than the
// default 64 KiB (gfx950 has 160 KiB of LDS per compute unit).
inline hipError_t opt_in_lds(const void* fn, int bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <typename T>
__device__ __forceinline__ T dsqrt(T x) { return sqrt(x); }

// Failure bits of a call's device work.  The kernel that meets one ORs it
// into the call's device word (read by the report) and stores 1 into the
// context's host-visible word of that cause (host memory mapped into the
// device's address space: a plain store, no read-modify-write across the
// bus), which the host checks before every later call.
__device__ __forceinline__ void report_device_error(int* dev_err, int* host_err, int bit) {
  if (dev_err) atomicOr(dev_err, bit);
  if (host_err) {
    const int word = bit == kErrBarrier ? 0 : (bit == kErrChain ? 1 : 2);
    __hip_atomic_store(host_err + word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// Rotation matrix (row-major) of a quaternion (x, y, z, w), normalised first.
template <typename T, typename Q>
__device__ __forceinline__ void quat_to_rot(const Q* q, T R[9]) {
  T x = (T)q[0], y = (T)q[1], z = (T)q[2], w = (T)q[3];
  T n = (T)1 / dsqrt(x * x + y * y + z * z + w * w);
  x *= n; y *= n; z *= n; w *= n;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - z * w);     R[2] = 2 * (x * z + y * w);
  R[3] = 2 * (x * y + z * w);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - x * w);
  R[6] = 2 * (x * z - y * w);     R[7] = 2 * (y * z + x * w);     R[8] = 1 - 2 * (x * x + y * y);
}

// Relative pose T_ji = G_j^-1 G_i of eq. (2): R = R_j^T R_i, t = R_j^T (t_i - t_j).
template <typename T>
__device__ __forceinline__ void relative_pose(const T Ri[9], const T ti[3], const T Rj[9],
                                              const T tj[3], T R[9], T t[3]) {
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b < 3; ++b)
      R[3 * a + b] = Rj[a] * Ri[b] + Rj[3 + a] * Ri[3 + b] + Rj[6 + a] * Ri[6 + b];
    t[a] = Rj[a] * (ti[0] - tj[0]) + Rj[3 + a] * (ti[1] - tj[1]) + Rj[6 + a] * (ti[2] - tj[2]);
  }
}

// Ad(T)^T applied to (a; b) for T = (R, t): (R^T a ; R^T (b - t x a)).
template <typename T>
__device__ __forceinline__ void adjoint_transpose_apply(const T R[9], const T t[3], const T in[6],
                                                        T out[6]) {
  const T a0 = in[0], a1 = in[1], a2 = in[2];
  const T b0 = in[3] - (t[1] * a2 - t[2] * a1);
  const T b1 = in[4] - (t[2] * a0 - t[0] * a2);
  const T b2 = in[5] - (t[0] * a1 - t[1] * a0);
  out[0] = R[0] * a0 + R[3] * a1 + R[6] * a2;
  out[1] = R[1] * a0 + R[4] * a1 + R[7] * a2;
  out[2] = R[2] * a0 + R[5] * a1 + R[8] * a2;
  out[3] = R[0] * b0 + R[3] * b1 + R[6] * b2;
  out[4] = R[1] * b0 + R[4] * b1 + R[7] * b2;
  out[5] = R[2] * b0 + R[5] * b1 + R[8] * b2;
}

// Ad(T) applied to (a; b): (R a + t x (R b) ; R b).
template <typename T>
__device__ __forceinline__ void adjoint_apply(const T R[9], const T t[3], const T in[6], T out[6]) {
  T Ra[3], Rb[3];
  for (int m = 0; m < 3; ++m) {
    Ra[m] = R[3 * m] * in[0] + R[3 * m + 1] * in[1] + R[3 * m + 2] * in[2];
    Rb[m] = R[3 * m] * in[3] + R[3 * m + 1] * in[4] + R[3 * m + 2] * in[5];
  }
  out[0] = Ra[0] + (t[1] * Rb[2] - t[2] * Rb[1]);
  out[1] = Ra[1] + (t[2] * Rb[0] - t[0] * Rb[2]);
  out[2] = Ra[2] + (t[0] * Rb[1] - t[1] * Rb[0]);
  out[3] = Rb[0]; out[4] = Rb[1]; out[5] = Rb[2];
}

// Series coefficients of the SO(3)/SE(3) exponential for theta = |phi|:
//   h = sin(theta/2) / theta   (quaternion of Exp(phi) = (h phi, cos(theta/2)))
//   B = (1 - cos theta) / theta^2 = 2 h^2
//   C = (theta - sin theta) / theta^3
// B is formed from h, which has no cancellation; C uses its Taylor series
// below a precision-dependent angle, where the direct form would lose digits.
template <typename T> struct ExpSeries;
template <> struct ExpSeries<float> { static constexpr float kSmall2 = 0.25f; };
template <> struct ExpSeries<double> { static constexpr double kSmall2 = 1e-4; };

template <typename T>
__device__ __forceinline__ void exp_coeffs(const T phi[3], T& h, T& ch, T& B, T& C) {
  const T th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
  if (th2 < ExpSeries<T>::kSmall2) {
    // sin(x/2)/x = 1/2 - x^2/48 + x^4/3840 - x^6/645120
    h = (T)0.5 + th2 * ((T)(-1.0 / 48) + th2 * ((T)(1.0 / 3840) + th2 * (T)(-1.0 / 645120)));
    // cos(x/2) = 1 - x^2/8 + x^4/384 - x^6/46080
    ch = (T)1 + th2 * ((T)(-1.0 / 8) + th2 * ((T)(1.0 / 384) + th2 * (T)(-1.0 / 46080)));
    // (x - sin x)/x^3 = 1/6 - x^2/120 + x^4/5040 - x^6/362880
    C = (T)(1.0 / 6) + th2 * ((T)(-1.0 / 120) + th2 * ((T)(1.0 / 5040) + th2 * (T)(-1.0 / 362880)));
  } else {
    const T th = dsqrt(th2);
    T s2, c2;
    s2 = sin(th * (T)0.5);
    c2 = cos(th * (T)0.5);
    h = s2 / th;
    ch = c2;
    C = (th - sin(th)) / (th2 * th);
  }
  B = (T)2 * h * h;
}

// Right retraction of a pose stored as (t, q): G <- G Exp(xi).
//   q <- q (x) (h phi, cos(theta/2)),  t <- t + R V(phi) rho,
//   V(phi) rho = rho + B phi x rho + C phi x (phi x rho).
// The quaternion is renormalised.
template <typename T, typename P>
__device__ __forceinline__ void retract_pose(P* pose, const T xi[6]) {
  const T rho[3] = {xi[0], xi[1], xi[2]};
  const T phi[3] = {xi[3], xi[4], xi[5]};
  T h, ch, B, C;
  exp_coeffs<T>(phi, h, ch, B, C);
  T R[9];
  quat_to_rot<T, P>(pose + 3, R);
  T c1[3] = {phi[1] * rho[2] - phi[2] * rho[1], phi[2] * rho[0] - phi[0] * rho[2],
             phi[0] * rho[1] - phi[1] * rho[0]};
  T c2[3] = {phi[1] * c1[2] - phi[2] * c1[1], phi[2] * c1[0] - phi[0] * c1[2],
             phi[0] * c1[1] - phi[1] * c1[0]};
  T Vr[3];
  for (int m = 0; m < 3; ++m) Vr[m] = rho[m] + B * c1[m] + C * c2[m];
  for (int m = 0; m < 3; ++m)
    pose[m] = (P)((T)pose[m] + R[3 * m] * Vr[0] + R[3 * m + 1] * Vr[1] + R[3 * m + 2] * Vr[2]);
  // quaternion product q * dq, both (x, y, z, w)
  const T qx = (T)pose[3], qy = (T)pose[4], qz = (T)pose[5], qw = (T)pose[6];
  const T dx = h * phi[0], dy = h * phi[1], dz = h * phi[2], dw = ch;
  T nx = qw * dx + qx * dw + qy * dz - qz * dy;
  T ny = qw * dy - qx * dz + qy * dw + qz * dx;
  T nz = qw * dz + qx * dy - qy * dx + qz * dw;
  T nw = qw * dw - qx * dx - qy * dy - qz * dz;
  const T inv = (T)1 / dsqrt(nx * nx + ny * ny + nz * nz + nw * nw);
  pose[3] = (P)(nx * inv); pose[4] = (P)(ny * inv); pose[5] = (P)(nz * inv); pose[6] = (P)(nw * inv);
}

}  // namespace dpvba
