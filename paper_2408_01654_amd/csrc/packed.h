// Dense Cholesky factorisation and solves of one small symmetric system held
// as a packed lower triangle (row i at i (i + 1) / 2), by one workgroup.
// The storage may be shared memory or global memory private to the
// workgroup; every thread of the workgroup calls these functions.
#pragma once

#include "common.h"

namespace dpvba {

__device__ __forceinline__ int packed_index(int i, int j) { return i * (i + 1) / 2 + j; }

// In-place A = L L^T (right-looking, one column at a time).  A pivot that is
// not positive or not finite is replaced by 1 and counted in *bad; *minr
// receives the smallest pivot / d0 ratio.  bad and minr live in shared memory.
template <typename TA>
__device__ void packed_cholesky(TA* A, int n, const TA* d0, int* bad, float* minr) {
  const int tid = threadIdx.x;
  if (tid == 0) { *bad = 0; *minr = 3.0e38f; }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const int jj = packed_index(j, j);
    if (tid == 0) {
      TA piv = A[jj];
      const float ratio = (float)(piv / d0[j]);
      if (ratio < *minr || !(ratio == ratio)) *minr = ratio == ratio ? ratio : 0.f;
      if (!(piv > (TA)0) || !(piv < (TA)3.0e38)) { *bad = 1; piv = (TA)1; }
      A[jj] = dsqrt(piv);
    }
    __syncthreads();
    const TA ljj = A[jj];
    for (int i = j + 1 + tid; i < n; i += blockDim.x) A[packed_index(i, j)] /= ljj;
    __syncthreads();
    const int m = n - j - 1;
    for (int idx = tid; idx < m * m; idx += blockDim.x) {
      const int i = j + 1 + idx / m, k = j + 1 + idx % m;
      if (k <= i) A[packed_index(i, k)] -= A[packed_index(i, j)] * A[packed_index(k, j)];
    }
    __syncthreads();
  }
}

// b <- (L L^T)^-1 b in place (forward then backward substitution).
template <typename TA, typename TB>
__device__ void packed_solve(const TA* L, TB* b, int n) {
  const int tid = threadIdx.x;
  for (int j = 0; j < n; ++j) {
    if (tid == 0) b[j] /= (TB)L[packed_index(j, j)];
    __syncthreads();
    const TB yj = b[j];
    for (int i = j + 1 + tid; i < n; i += blockDim.x) b[i] -= (TB)L[packed_index(i, j)] * yj;
    __syncthreads();
  }
  for (int j = n - 1; j >= 0; --j) {
    if (tid == 0) b[j] /= (TB)L[packed_index(j, j)];
    __syncthreads();
    const TB xj = b[j];
    const TA* rowj = L + packed_index(j, 0);
    for (int i = tid; i < j; i += blockDim.x) b[i] -= (TB)rowj[i] * xj;
    __syncthreads();
  }
}

}  // namespace dpvba
