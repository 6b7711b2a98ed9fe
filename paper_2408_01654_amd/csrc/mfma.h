// Matrix-core (MFMA) helpers for gfx950.
#pragma once

#include <hip/hip_runtime.h>

namespace dpvba {

typedef float floatx4_t __attribute__((ext_vector_type(4)));
typedef double doublex4_t __attribute__((ext_vector_type(4)));

// 16x16x4 matrix-core step D = A B + C: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; its v-th accumulator (v = 0..3) holds
// D[row(l, v)][l % 16], with row = 4 (l / 16) + v for float32 and
// row = l / 16 + 4 v for float64 (checked on gfx950).
template <typename T> struct Mfma;
template <> struct Mfma<float> {
  typedef floatx4_t acc_t;
  static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct Mfma<double> {
  typedef doublex4_t acc_t;
  static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};


// C (64 x 64) = X Y^T for row-major 64 x 64 blocks X, Y in LDS with row
// stride ld: wavefront w computes rows 16 w .. 16 w + 15 as four 16 x 16
// tiles; acc[t] holds tile t (columns 16 t .. 16 t + 15).
template <typename T>
__device__ __forceinline__ void gemm_nt_64(const T* X, const T* Y, int ld, int kdim,
                                           typename Mfma<T>::acc_t acc[4]) {
  const int lane = threadIdx.x & 63, w = (threadIdx.x >> 6) & 3;
  const T* xr = X + (16 * w + (lane & 15)) * ld + (lane >> 4);
  const T* yr = Y + (lane & 15) * ld + (lane >> 4);
  for (int k0 = 0; k0 < kdim; k0 += 4) {
    const T a = xr[k0];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = Mfma<T>::step(a, yr[16 * t * ld + k0], acc[t]);
  }
}

}  // namespace dpvba
