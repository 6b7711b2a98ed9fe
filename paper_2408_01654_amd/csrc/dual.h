// Forward-mode dual numbers a + b eps (eps^2 = 0) for the adjoint kernels
// and the Jacobians of the pose-graph residuals.
//
// Evaluating a function on Dual<S> arguments seeded with one unit tangent
// returns its value and its directional derivative along that tangent.  The
// adjoint of the unrolled Gauss-Newton iterations uses this for the second
// derivatives of the projection (the Jacobians' own dependence on the poses
// and depths) and for the differential of the SE(3) retraction, evaluating
// the same device functions the forward path runs.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace dpvba {

template <typename S>
struct Dual {
  S v, d;
  __device__ __forceinline__ Dual() : v(0), d(0) {}
  __device__ __forceinline__ Dual(S v_, S d_) : v(v_), d(d_) {}
  __device__ __forceinline__ Dual(float x) : v((S)x), d(0) {}
  __device__ __forceinline__ Dual(double x) : v((S)x), d(0) {}
  __device__ __forceinline__ Dual(int x) : v((S)x), d(0) {}
  __device__ __forceinline__ explicit operator S() const { return v; }
  __device__ __forceinline__ Dual& operator+=(const Dual& o) { v += o.v; d += o.d; return *this; }
  __device__ __forceinline__ Dual& operator-=(const Dual& o) { v -= o.v; d -= o.d; return *this; }
  __device__ __forceinline__ Dual& operator*=(const Dual& o) { d = d * o.v + v * o.d; v *= o.v; return *this; }

  // Non-template friends, so plain constants on either side convert.
  friend __device__ __forceinline__ Dual operator+(const Dual& a, const Dual& b) { return {a.v + b.v, a.d + b.d}; }
  friend __device__ __forceinline__ Dual operator-(const Dual& a, const Dual& b) { return {a.v - b.v, a.d - b.d}; }
  friend __device__ __forceinline__ Dual operator-(const Dual& a) { return {-a.v, -a.d}; }
  friend __device__ __forceinline__ Dual operator*(const Dual& a, const Dual& b) {
    return {a.v * b.v, a.d * b.v + a.v * b.d};
  }
  friend __device__ __forceinline__ Dual operator/(const Dual& a, const Dual& b) {
    const S inv = (S)1 / b.v;
    const S q = a.v * inv;
    return {q, (a.d - q * b.d) * inv};
  }
  friend __device__ __forceinline__ bool operator<(const Dual& a, const Dual& b) { return a.v < b.v; }
  friend __device__ __forceinline__ bool operator>(const Dual& a, const Dual& b) { return a.v > b.v; }
  friend __device__ __forceinline__ Dual sqrt(const Dual& a) {
    const S s = ::sqrt(a.v);
    return {s, a.d / (s + s)};
  }
  friend __device__ __forceinline__ Dual sin(const Dual& a) { return {::sin(a.v), ::cos(a.v) * a.d}; }
  friend __device__ __forceinline__ Dual cos(const Dual& a) { return {::cos(a.v), -::sin(a.v) * a.d}; }
  friend __device__ __forceinline__ Dual exp(const Dual& a) {
    const S e = ::exp(a.v);
    return {e, e * a.d};
  }
  friend __device__ __forceinline__ Dual log(const Dual& a) { return {::log(a.v), a.d / a.v}; }
  friend __device__ __forceinline__ Dual atan2(const Dual& y, const Dual& x) {
    const S r2 = x.v * x.v + y.v * y.v;
    return {::atan2(y.v, x.v), (x.v * y.d - y.v * x.d) / r2};
  }
};

// Value part of a plain or dual scalar (for decisions taken on values).
__device__ __forceinline__ double value_of(double x) { return x; }
__device__ __forceinline__ float value_of(float x) { return x; }
template <typename S>
__device__ __forceinline__ S value_of(const Dual<S>& x) { return x.v; }

template <typename S>
struct ExpSeries<Dual<S>> {
  static constexpr S kSmall2 = ExpSeries<S>::kSmall2;
};

}  // namespace dpvba
