// Dense Cholesky factorisation and solves of one small symmetric system held
// as a packed lower triangle (row i at i (i + 1) / 2), by one workgroup.
// The storage may be shared memory or global memory private to the
// workgroup; every thread of the workgroup calls these functions.
#pragma once

#include "common.h"

namespace dpvba {

// 1 / sqrt(d) of a positive pivot: the hardware reciprocal square root for
// float32 (within about one unit in the last place, far inside the float32
// path's tolerance; it keeps the per-column dependency chain short); the
// correctly rounded form for float64.
template <typename T>
__device__ __forceinline__ T pivot_rsqrt(T d) {
  if constexpr (sizeof(T) == 4) return __builtin_amdgcn_rsqf(d);
  else return (T)1 / sqrt(d);
}

// Smallest pivot / damped-diagonal ratio of columns 0..n-1 (the bits of a
// non-negative float, a NaN counting as 0) combined into *min_bits: every
// thread takes columns tid, tid + blockDim.x, ..., each wavefront reduces its
// lanes with shuffles, and one lane per wavefront issues the atomic minimum
// (one LDS atomic per wavefront instead of one per column).  Called by every
// thread of the workgroup.
template <typename T>
__device__ __forceinline__ void pivot_ratio_min(const T* piv, const T* dd, int n, unsigned int* min_bits,
                                                int first = -1, int stride = 0) {
  unsigned int m = __float_as_uint(3.0e38f);
  if (first < 0) {
    first = threadIdx.x;
    stride = blockDim.x;
  }
  for (int j = first; j < n; j += stride) {
    const float ratio = (float)(piv[j] / dd[j]);
    m = min(m, __float_as_uint(ratio == ratio ? fmaxf(ratio, 0.f) : 0.f));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = min(m, (unsigned int)__shfl_xor((int)m, o));
  if ((threadIdx.x & 63) == 0) atomicMin(min_bits, m);
}

__device__ __forceinline__ int packed_index(int i, int j) { return i * (i + 1) / 2 + j; }

// In-place A = L L^T, right-looking with the column scaling deferred: step j
// subtracts A_ij A_kj / d_j from the trailing entries (j < k <= i), where
// d_j = A_jj after the earlier steps, so one barrier per column suffices;
// a final pass scales column j by 1 / sqrt(d_j).  The trailing entries are
// spread over a 16 x 16 thread grid (entry (i, k) on the thread with
// i = ty, k = tx mod 16), which needs blockDim.x >= 256 (threads beyond 256
// idle).  A pivot that is not positive or not finite is replaced by 1 and
// counted in *bad; *minr receives the smallest pivot / d0 ratio.  bad and
// minr live in shared memory.
template <typename TA>
__device__ __forceinline__ TA packed_pivot(TA d) {
  return (d > (TA)0 && d < (TA)3.0e38) ? d : (TA)1;
}

template <typename TA>
__device__ void packed_cholesky(TA* A, int n, const TA* d0, int* bad, float* minr) {
  const int tid = threadIdx.x;
  const int ty = tid & 15, tx = (tid >> 4) & 15;
  const bool worker = tid < 256;
  if (tid == 0) { *bad = 0; *minr = 3.0e38f; }
  __syncthreads();
  const int nb = (n + 15) >> 4;
  for (int j = 0; j < n; ++j) {
    const TA dj = A[packed_index(j, j)];
    if (tid == 0) {
      const float ratio = (float)(dj / d0[j]);
      if (ratio < *minr || !(ratio == ratio)) *minr = ratio == ratio ? ratio : 0.f;
      if (!(dj > (TA)0) || !(dj < (TA)3.0e38)) *bad = 1;
    }
    const TA inv = (TA)1 / packed_pivot(dj);
    if (worker) {
      for (int bi = (j + 1) >> 4; bi < nb; ++bi) {
        const int i = 16 * bi + ty;
        if (i <= j || i >= n) continue;
        const TA aij = A[packed_index(i, j)] * inv;
        TA* row = A + packed_index(i, 0);
        for (int bk = (j + 1) >> 4; bk <= bi; ++bk) {
          const int k = 16 * bk + tx;
          if (k > j && k <= i) row[k] -= aij * A[packed_index(k, j)];
        }
      }
    }
    __syncthreads();
  }
  // L_ij = A_ij / sqrt(d_j) (i > j), L_jj = sqrt(d_j)
  for (int i = tid; i < n; i += blockDim.x) {
    TA* row = A + packed_index(i, 0);
    for (int j = 0; j < i; ++j) row[j] /= dsqrt(packed_pivot(A[packed_index(j, j)]));
  }
  __syncthreads();
  for (int j = tid; j < n; j += blockDim.x) A[packed_index(j, j)] = dsqrt(packed_pivot(A[packed_index(j, j)]));
  __syncthreads();
}

// b <- (L L^T)^-1 b in place (n <= 256): both substitutions run in the
// first wavefront with b held in registers (row i on lane i mod 64) and
// each solved entry broadcast by a lane shuffle; no workgroup barrier inside.
template <typename TA, typename TB>
__device__ void packed_solve(const TA* L, TB* b, int n) {
  const int lane = threadIdx.x;
  if (lane < 64) {
    TB r[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] = (lane + 64 * q < n) ? b[lane + 64 * q] : (TB)0;
    // forward: L y = b
    for (int j = 0; j < n; ++j) {
      const int qj = j >> 6;
      TB bj = (TB)0;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q == qj) bj = r[q];
      const TB yj = __shfl(bj, j & 63) / (TB)L[packed_index(j, j)];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = lane + 64 * q;
        if (i == j) r[q] = yj;
        else if (i > j && i < n) r[q] -= (TB)L[packed_index(i, j)] * yj;
      }
    }
    // backward: L^T x = y
    for (int j = n - 1; j >= 0; --j) {
      const int qj = j >> 6;
      TB yj = (TB)0;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q == qj) yj = r[q];
      const TB xj = __shfl(yj, j & 63) / (TB)L[packed_index(j, j)];
      const TA* rowj = L + packed_index(j, 0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = lane + 64 * q;
        if (i == j) r[q] = xj;
        else if (i < j) r[q] -= (TB)rowj[i] * xj;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (lane + 64 * q < n) b[lane + 64 * q] = r[q];
  }
  __syncthreads();
}

// Cholesky of the augmented matrix [[S, .], [s^T, .]] (n + 1 <= NMAX rows)
// by the first wavefront alone, with no workgroup barrier: lane l keeps rows
// l and l + 64 in registers (entry k of a row in register k, so every index
// is a compile-time constant).  Column j: the pivot is read from its lane
// (v_readlane), every lane scales its column-j entries, then subtracts
// l_ij l_kj from its entries k > j, taking each l_kj from lane k mod 64 by
// v_readlane (no LDS round trip on the elimination's critical path).  Entries above a row's diagonal receive the
// same arithmetic and are never read, so no lane needs a predicate.  The
// last row ends as y = L^-1 s.  Then L^T dxi = y on the same wavefront with
// one pivot broadcast per row.  Returns the step in x[0..n) (LDS, zero if a
// pivot was not positive).
template <int NMAX>
__device__ __forceinline__ void wave_chol_solve(int n_in, const float* Sp_g, const float* rhs_g, const float* d0_g, float* cb,
                                float* Lrow, float* x, float* invd, int* bad_out, float* minr_out) {
  constexpr int N1 = NMAX < 64 ? NMAX : 64;  // columns held for rows < 64
  constexpr int N2 = NMAX > 64 ? NMAX : 1;   // columns held for rows >= 64
  const int n = __builtin_amdgcn_readfirstlane(n_in);  // uniform: loop guards stay scalar
  const int lane = threadIdx.x;
  const int r0 = lane, r1 = lane + 64;
  float a0[N1], a1[N2];
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    float v = 0.f;
    if (k <= r0 && r0 < n) v = Sp_g[r0 * (r0 + 1) / 2 + k];
    else if (r0 == n && k < n) v = rhs_g[k];
    a0[k] = v;
  }
#pragma unroll
  for (int k = 0; k < N2; ++k) {
    float v = 0.f;
    if (NMAX > 64) {
      if (k <= r1 && r1 < n) v = Sp_g[r1 * (r1 + 1) / 2 + k];
      else if (r1 == n && k < n) v = rhs_g[k];
    }
    a1[k] = v;
  }
  const float dd0 = r0 < n ? d0_g[r0] : 1.f;
  const float dd1 = r1 < n ? d0_g[r1] : 1.f;
  int bad = 0;
  float minr = 3.0e38f;
#pragma unroll
  for (int j = 0; j < NMAX - 1; ++j) {
    if (j >= n) continue;  // uniform; keeps the loop fully unrolled
    float d, d0j;
    if (j < 64) {
      d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a0[j < N1 ? j : 0]), j & 63));
      d0j = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(dd0), j & 63));
    } else {
      d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a1[j < N2 ? j : 0]), j & 63));
      d0j = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(dd1), j & 63));
    }
    const float ratio = d / d0j;
    if (!(ratio >= minr)) minr = ratio == ratio ? fmaxf(ratio, 0.f) : 0.f;
    if (!(d > 0.f) || !(d < 3.0e38f)) {
      bad = 1;
      d = 1.f;
    }
    const float rs = 1.f / sqrtf(d);
    if (lane == 0) invd[j] = rs;
    // scale column j (row j's diagonal becomes L_jj = sqrt(d)) and publish it
    float l0 = 0.f, l1 = 0.f;
    if (j < N1) {
      l0 = a0[j < N1 ? j : 0] * rs;
      a0[j < N1 ? j : 0] = l0;
    }
    if (NMAX > 64) {
      l1 = a1[j < N2 ? j : 0] * rs;
      a1[j < N2 ? j : 0] = l1;
    }
    // trailing update of entries k > j; l_kj comes from lane k mod 64 by
    // v_readlane (rows above k receive arithmetic on entries above their
    // diagonal, which are never read; columns k > n touch unused entries)
#pragma unroll
    for (int k = j + 1; k < NMAX; ++k) {
      const float lk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(k < 64 ? l0 : l1), k & 63));
      if (k < N1) a0[k < N1 ? k : 0] -= l0 * lk;
      if (NMAX > 64) a1[k < N2 ? k : 0] -= l1 * lk;
    }
  }
  // rows of L (and y in row n) to LDS, row-major with stride NMAX
#pragma unroll
  for (int k = 0; k < N1; ++k)
    if (r0 < NMAX) Lrow[r0 * NMAX + k] = a0[k];
  if (NMAX > 64) {
#pragma unroll
    for (int k = 0; k < N2; ++k)
      if (r1 < NMAX) Lrow[r1 * NMAX + k] = a1[k];
  }
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  // backward substitution L^T x = y; lane l holds entries l and l + 64
  float y0 = r0 < n ? Lrow[n * NMAX + r0] : 0.f;
  float y1 = (NMAX > 64 && r1 < n) ? Lrow[n * NMAX + r1] : 0.f;
  for (int i = n - 1; i >= 0; --i) {
    const float yv = i >= 64 ? y1 : y0;
    const float xi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(yv), i & 63)) * invd[i];
    const float* Li = Lrow + i * NMAX;
    if (r0 < i) y0 -= Li[r0] * xi;
    if (r1 < i) y1 -= Li[r1] * xi;
    if (r0 == i) y0 = xi;
    if (r1 == i) y1 = xi;
  }
  if (r0 < n) x[r0] = bad ? 0.f : y0;
  if (r1 < n) x[r1] = bad ? 0.f : y1;
  if (lane == 0) {
    *bad_out = bad;
    *minr_out = minr;
  }
}


// Cholesky of the augmented matrix [[S, .], [s^T, .]] (n + 1 <= 16 MB rows)
// by a 256-thread workgroup with the matrix in registers: thread
// (ty, tx) = (tid mod 16, tid / 16) holds entries (16 bi + ty, 16 bk + tx)
// for all bi, bk < MB, so every register index is a compile-time constant.
// Column j (loop fully unrolled): the 16 owners of column j (one wavefront)
// take the pivot by v_readlane, scale their column-j entries and publish the
// scaled column in a double-buffered LDS vector with zeros at rows <= j;
// after one barrier every thread subtracts cb_i cb_k from all of its
// entries.  The zeros make the update a no-op wherever it must not act
// (finished columns and rows), so no thread needs a predicate, and entries
// above the diagonal receive arithmetic that is never read.  The last row
// ends as y = L^-1 s; then L^T x = y on one wavefront.  Returns the step in
// x[0..n) (LDS; zero if a pivot was not positive).
template <typename T, int MB>
__device__ __forceinline__ void block_chol_solve(int n_in, const T* Sp_g, const T* rhs_g, const T* d0_g,
                                                 unsigned char* lds, T* x, int* bad_out, float* minr_out) {
  constexpr int NR = 16 * MB;
  const int n = __builtin_amdgcn_readfirstlane(n_in);
  const int tid = threadIdx.x;
  const int ty = tid & 15, tx = tid >> 4;
  T* cb = reinterpret_cast<T*>(lds);  // [2][NR]
  T* invd = cb + 2 * NR;             // [NR]
  T* dd = invd + NR;                 // [NR] damped diagonal (pivot monitor)
  T* Lrow = dd + NR;                 // [NR][NR] rows of L, then y
  for (int i = tid; i < n; i += blockDim.x) dd[i] = d0_g[i];
  T a[MB][MB];
#pragma unroll
  for (int bi = 0; bi < MB; ++bi)
#pragma unroll
    for (int bk = 0; bk < MB; ++bk) {
      const int i = 16 * bi + ty, k = 16 * bk + tx;
      T v = (T)0;
      if (k <= i && i < n) v = Sp_g[i * (i + 1) / 2 + k];
      else if (i == n && k < n) v = rhs_g[k];
      a[bi][bk] = v;
    }
  int bad = 0;
  float minr = 3.0e38f;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NR - 1; ++j) {
    if (j >= n) continue;  // uniform
    const int bj = j >> 4, jm = j & 15;
    T* cbj = cb + (j & 1) * NR;
    if (tx == jm) {  // one wavefront: threads 16 jm .. 16 jm + 15
      // pivot a_jj lives on the owner with ty == jm: lane (16 jm + jm) mod 64
      T d;
      if constexpr (sizeof(T) == 4) {
        d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a[bj][bj]), (16 * jm + jm) & 63));
      } else {
        const long long bits = __double_as_longlong(a[bj][bj]);
        const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), (16 * jm + jm) & 63);
        const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), (16 * jm + jm) & 63);
        d = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
      }
      if (ty == jm) {
        const float ratio = (float)(d / dd[j]);
        if (!(ratio >= minr)) minr = ratio == ratio ? fmaxf(ratio, 0.f) : 0.f;
        if (!(d > (T)0) || !(d < (T)3.0e38)) bad = 1;
      }
      if (!(d > (T)0) || !(d < (T)3.0e38)) d = (T)1;
      const T rs = (T)1 / dsqrt(d);
      if (ty == jm) invd[j] = rs;
#pragma unroll
      for (int bi = 0; bi < MB; ++bi) {
        const int i = 16 * bi + ty;
        const T l = a[bi][bj] * rs;
        if (i >= j) a[bi][bj] = l;
        cbj[i] = i > j ? l : (T)0;
      }
    }
    __syncthreads();
    T ci[MB], ck[MB];
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      ci[b] = cbj[16 * b + ty];
      ck[b] = cbj[16 * b + tx];
    }
#pragma unroll
    for (int bi = 0; bi < MB; ++bi)
#pragma unroll
      for (int bk = 0; bk < MB; ++bk) a[bi][bk] -= ci[bi] * ck[bk];
  }
  // rows of L (and y in row n) to LDS
#pragma unroll
  for (int bi = 0; bi < MB; ++bi)
#pragma unroll
    for (int bk = 0; bk < MB; ++bk) Lrow[(16 * bi + ty) * NR + 16 * bk + tx] = a[bi][bk];
  __syncthreads();
  if (tid < 64) {  // backward substitution L^T x = y; lane l holds entries l, l + 64
    const int r0 = tid, r1 = tid + 64;
    T y0 = r0 < n ? Lrow[n * NR + r0] : (T)0;
    T y1 = r1 < n ? Lrow[n * NR + r1] : (T)0;
    for (int i = n - 1; i >= 0; --i) {
      const T yv = i >= 64 ? y1 : y0;
      T yi;
      if constexpr (sizeof(T) == 4) {
        yi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(yv), i & 63));
      } else {
        const long long bits = __double_as_longlong(yv);
        const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), i & 63);
        const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), i & 63);
        yi = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
      }
      const T xi = yi * invd[i];
      const T* Li = Lrow + i * NR;
      if (r0 < i) y0 -= Li[r0] * xi;
      if (r1 < i) y1 -= Li[r1] * xi;
      if (r0 == i) y0 = xi;
      if (r1 == i) y1 = xi;
    }
    if (r0 < n) x[r0] = y0;
    if (r1 < n) x[r1] = y1;
  }
  // bad and minr are known to the owners' threads: combine through LDS
  __shared__ int bad_s;
  __shared__ float minr_s;
  if (tid == 0) { bad_s = 0; minr_s = 3.0e38f; }
  __syncthreads();
  if (bad) atomicOr(&bad_s, 1);
  if (minr < 3.0e38f) atomicMin(reinterpret_cast<unsigned int*>(&minr_s), __float_as_uint(minr));
  __syncthreads();
  if (tid < n && bad_s) x[tid] = (T)0;
  if (tid + 256 < n && bad_s) x[tid + 256] = (T)0;
  if (tid == 0) {
    *bad_out = bad_s;
    *minr_out = minr_s;
  }
  __syncthreads();
}


// Sixteen steps i = i_hi, i_hi - 1, ... (i < n) of L^T x = y on one
// wavefront: x_i = y_i / L_ii with y_i broadcast from `src` (the half that
// holds rows i), then y_r -= L_ir x_i (l0 / l1: L_ir of the lane's two
// rows, zero unless r < i).  x_i is kept by the lane of row i, off the chain.
template <typename T>
__device__ __forceinline__ void back_sub16(int i_hi, int n, const T* l0, const T* l1, const T* iv, const T& src,
                                           T& y0, T& y1, T& x0, T& x1, int r0, int r1) {
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const int i = i_hi - c;
    if (i >= n) continue;  // uniform
    T yi;
    if constexpr (sizeof(T) == 4) {
      yi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(src), i & 63));
    } else {
      const long long bits = __double_as_longlong(src);
      const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), i & 63);
      const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), i & 63);
      yi = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    }
    const T xi = yi * iv[c];
    y0 -= l0[c] * xi;
    y1 -= l1[c] * xi;
    x0 = r0 == i ? xi : x0;
    x1 = r1 == i ? xi : x1;
  }
}

// Cholesky of the augmented matrix [[S, .], [s^T, .]] (n + 1 <= 16 MB rows)
// in panels of 16 columns, by a 256-thread workgroup with the matrix in
// registers: thread (ty, tx) = (tid mod 16, tid / 16) holds entries
// (16 bi + ty, 16 bk + tx), bi, bk < MB (the panel loop is unrolled, so every
// register index is a compile-time constant).  Panel p: the threads publish
// its column block in LDS; one wavefront factors the 16 columns on its own
// (rows on lanes, pivots and column entries broadcast by v_readlane, no
// barrier inside); after one barrier every thread takes back its factored
// entries and applies the rank-16 update to its blocks right of and below
// the panel.  Two barriers per panel instead of one per column.  The last
// row ends as y = L^-1 s; then L^T x = y on one wavefront.  Returns the step
// in x[0..n) (LDS; zero if a pivot was not positive).
// ld > 0: Sp_g is instead a dense row-major matrix with row stride ld (its
// lower triangle is read) and d0_g may be null (the damped diagonal is then
// that matrix's diagonal).
template <typename T, int MB>
__device__ __forceinline__ void panel_chol_solve(int n_in, const T* Sp_g, const T* rhs_g, const T* d0_g,
                                                 unsigned char* lds, T* x, int* bad_out, float* minr_out,
                                                 int ld = 0) {
  constexpr int NR = 16 * MB;
  const int n = __builtin_amdgcn_readfirstlane(n_in);
  const int tid = threadIdx.x;
  const int ty = tid & 15, tx = tid >> 4;
  const int lane = tid & 63, wave = tid >> 6;
  const bool grid = tid < 256;  // the 16 x 16 register grid (larger workgroups: the rest only meet the barriers)
  T* PB = reinterpret_cast<T*>(lds);  // [2][NR][17] published panel
  T* invd = PB + 2 * NR * 17;         // [NR] 1 / L_jj
  T* dd = invd + NR;                  // [NR] damped diagonal (pivot report)
  T* piv = dd + NR;                   // [NR] pivots before the square root
  T* Lrow = piv + NR;                 // [NR][NR]
  for (int i = tid; i < n; i += blockDim.x) dd[i] = d0_g ? d0_g[i] : Sp_g[(size_t)i * ld + i];
  T a[MB][MB];
#pragma unroll
  for (int bi = 0; bi < MB; ++bi)
#pragma unroll
    for (int bk = 0; bk < MB; ++bk) {
      const int i = 16 * bi + ty, k = 16 * bk + tx;
      T v = (T)0;
      if (grid && k <= i && i < n) v = ld > 0 ? Sp_g[(size_t)i * ld + k] : Sp_g[i * (i + 1) / 2 + k];
      else if (grid && i == n && k < n) v = rhs_g[k];
      a[bi][bk] = v;
    }
  int bad = 0;
#pragma unroll
  for (int p = 0; p < MB; ++p) {
    if (16 * p >= n) continue;  // uniform: no pivot left
    T* P = PB + (p & 1) * NR * 17;
    // publish the panel's column block (rows >= 16 p)
    if (grid)
#pragma unroll
      for (int bi = p; bi < MB; ++bi) P[(16 * bi + ty) * 17 + tx] = a[bi][p];
    __syncthreads();
    if (wave == (p & 3)) {
      // lane l holds rows 16 p + l and 16 p + l + 64 of the panel
      const int rA = 16 * p + lane, rB = rA + 64;
      const bool hasB = 16 * p + 64 < NR;  // compile-time: rows in the second half exist
      T ra[16], rb[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        ra[c] = rA < NR ? P[rA * 17 + c] : (T)0;
        rb[c] = (hasB && rB < NR) ? P[rB * 17 + c] : (T)0;
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const int j = 16 * p + c;
        if (j >= n) continue;  // uniform
        T d;
        if constexpr (sizeof(T) == 4) {
          d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ra[c]), c));
        } else {
          const long long bits = __double_as_longlong(ra[c]);
          const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), c);
          const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), c);
          d = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
        }
        if (lane == 0) piv[j] = d;
        if (!(d > (T)0) || !(d < (T)3.0e38)) {
          bad = 1;
          d = (T)1;
        }
        const T rs = pivot_rsqrt<T>(d);
        if (lane == 0) invd[j] = rs;
        ra[c] *= rs;  // row j's own entry becomes L_jj = sqrt(d)
        if (hasB) rb[c] *= rs;
#pragma unroll
        for (int c2 = c + 1; c2 < 16; ++c2) {
          T lk;  // l_{16p + c2, j}: lane c2's entry of column c
          if constexpr (sizeof(T) == 4) {
            lk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ra[c]), c2));
          } else {
            const long long bits = __double_as_longlong(ra[c]);
            const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), c2);
            const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), c2);
            lk = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
          }
          ra[c2] -= ra[c] * lk;
          if (hasB) rb[c2] -= rb[c] * lk;
        }
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        if (rA < NR) P[rA * 17 + c] = ra[c];
        if (hasB && rB < NR) P[rB * 17 + c] = rb[c];
      }
    }
    __syncthreads();
    // factored entries back, then the rank-16 update right of and below the panel
    if (grid) {
#pragma unroll
      for (int bi = p; bi < MB; ++bi) a[bi][p] = P[(16 * bi + ty) * 17 + tx];
#pragma unroll
      for (int bi = p + 1; bi < MB; ++bi) {
        T li[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) li[c] = P[(16 * bi + ty) * 17 + c];
#pragma unroll
        for (int bk = p + 1; bk <= bi; ++bk) {
          T acc = (T)0;
#pragma unroll
          for (int c = 0; c < 16; ++c) acc += li[c] * P[(16 * bk + tx) * 17 + c];
          a[bi][bk] -= acc;
        }
      }
    }
  }
  // rows of L (and y in row n) to LDS
  if (grid)
#pragma unroll
    for (int bi = 0; bi < MB; ++bi)
#pragma unroll
      for (int bk = 0; bk < MB; ++bk) Lrow[(16 * bi + ty) * NR + 16 * bk + tx] = a[bi][bk];
  __shared__ int bad_s;
  __shared__ unsigned int minr_s;
  if (tid == 0) { bad_s = 0; minr_s = __float_as_uint(3.0e38f); }
  __syncthreads();
  if (bad) atomicOr(&bad_s, 1);
  // pivot report (smallest pivot / damped diagonal) on the wavefronts other
  // than the first, while the first runs the backward substitution
  if (tid >= 64) pivot_ratio_min<T>(piv, dd, n, &minr_s, tid - 64, (int)blockDim.x - 64);
  if (tid < 64) {  // backward substitution L^T x = y; lane l holds entries l, l + 64
    const int r0 = tid, r1 = tid + 64;
    T y0 = r0 < n ? Lrow[n * NR + r0] : (T)0;
    T y1 = r1 < n ? Lrow[n * NR + r1] : (T)0;
    T x0 = (T)0, x1 = (T)0;
    // blocks of 16 rows from the last; a block lies in one half (64 is a
    // multiple of 16), so the broadcast source is fixed per block
#pragma unroll
    for (int blk = MB - 1; blk >= 0; --blk) {
      if (16 * blk >= n) continue;  // uniform
      T l0[16], l1[16], iv[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) {  // L_ir for r < i only (zero otherwise), loaded off the chain
        const int i = 16 * blk + 15 - c;
        const int ic = min(i, NR - 1);
        l0[c] = r0 < i && i < n ? Lrow[ic * NR + r0] : (T)0;
        l1[c] = r1 < i && i < n ? Lrow[ic * NR + r1] : (T)0;
        iv[c] = invd[ic];
      }
      if (blk >= 4) back_sub16<T>(16 * blk + 15, n, l0, l1, iv, y1, y0, y1, x0, x1, r0, r1);
      else back_sub16<T>(16 * blk + 15, n, l0, l1, iv, y0, y0, y1, x0, x1, r0, r1);
    }
    if (r0 < n) x[r0] = x0;
    if (r1 < n) x[r1] = x1;
  }
  __syncthreads();
  if (tid < n && bad_s) x[tid] = (T)0;
  if (tid == 0) {
    *bad_out = bad_s;
    *minr_out = __uint_as_float(minr_s);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Packed systems of up to 255 unknowns on one workgroup of 256 threads or
// more: blocked factor and wavefront substitutions.

// Value of v on lane c of each 16-lane row, for every lane of that row
// (the DPP row broadcast of CDNA; c must fold to a constant).  The result
// stays in a vector register: no scalar register, no readlane hazard.
template <int C>
__device__ __forceinline__ int row_bcast_bits(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x150 + C, 0xF, 0xF, true);
}
__device__ __forceinline__ int row_bcast_i(int v, int c) {
  switch (c) {
    case 0: return row_bcast_bits<0>(v);
    case 1: return row_bcast_bits<1>(v);
    case 2: return row_bcast_bits<2>(v);
    case 3: return row_bcast_bits<3>(v);
    case 4: return row_bcast_bits<4>(v);
    case 5: return row_bcast_bits<5>(v);
    case 6: return row_bcast_bits<6>(v);
    case 7: return row_bcast_bits<7>(v);
    case 8: return row_bcast_bits<8>(v);
    case 9: return row_bcast_bits<9>(v);
    case 10: return row_bcast_bits<10>(v);
    case 11: return row_bcast_bits<11>(v);
    case 12: return row_bcast_bits<12>(v);
    case 13: return row_bcast_bits<13>(v);
    case 14: return row_bcast_bits<14>(v);
    default: return row_bcast_bits<15>(v);
  }
}
template <typename T>
__device__ __forceinline__ T row_bcast(T v, int c) {
  if constexpr (sizeof(T) == 4) {
    return __int_as_float(row_bcast_i(__float_as_int(v), c));
  } else {
    const long long bits = __double_as_longlong(v);
    const int lo = row_bcast_i((int)(bits & 0xffffffffLL), c);
    const int hi = row_bcast_i((int)(bits >> 32), c);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  }
}

// Value of v on lane l (uniform) of the wavefront.
template <typename T>
__device__ __forceinline__ T lane_bcast(T v, int l) {
  if constexpr (sizeof(T) == 4) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
  } else {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), l);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  }
}

// In-place Cholesky of the packed lower triangle of rows 0..nr-1 of an
// n-column system (nr = n, or n + 1 with the right-hand side appended as row
// n, which then ends as y = L^-1 s; nr <= 256), in panels of 16 columns.
// Panel j0: the first wavefront takes the panel's rows (row j0 + l + 64 t on
// lane l, t < 4), factors its 16 columns alone (pivots and column entries
// broadcast by v_readlane) and writes them back; after a barrier the first
// 256 threads subtract the panel's rank-16 product from the trailing
// triangle, thread (ty, tx) = (tid mod 16, tid / 16 mod 16) owning entry
// (16 bi + ty, 16 bk + tx) of each 16 x 16 block.  Two barriers per panel.
// invd[j] = 1 / L_jj and piv[j] = the pivot before its square root; a pivot
// that is not positive or not finite is replaced by 1 and sets *bad (shared,
// cleared by the caller).
template <typename T>
__device__ __forceinline__ void packed_panel_factor(T* A, int n_in, int nr_in, T* invd, T* piv, int* bad) {
  const int n = __builtin_amdgcn_readfirstlane(n_in);
  const int nr = __builtin_amdgcn_readfirstlane(nr_in);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int ty = tid & 15, tx = (tid >> 4) & 15;
  for (int j0 = 0; j0 < n; j0 += 16) {
    if (tid < 64) {
      T ra[4][16];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int i = j0 + lane + 64 * t;
#pragma unroll
        for (int c = 0; c < 16; ++c)
          ra[t][c] = (i < nr && j0 + c <= i && j0 + c < n) ? A[packed_index(i, j0 + c)] : (T)0;
      }
      int badl = 0;
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const int j = j0 + c;
        if (j >= n) continue;  // uniform
        T d = lane_bcast(ra[0][c], c);
        if (lane == 0) piv[j] = d;
        if (!(d > (T)0) || !(d < (T)3.0e38)) {
          badl = 1;
          d = (T)1;
        }
        const T rs = pivot_rsqrt<T>(d);
        if (lane == 0) invd[j] = rs;
#pragma unroll
        for (int t = 0; t < 4; ++t) ra[t][c] *= rs;
#pragma unroll
        for (int c2 = c + 1; c2 < 16; ++c2) {
          const T lk = lane_bcast(ra[0][c], c2);  // entry (j0 + c2, j) of the panel
#pragma unroll
          for (int t = 0; t < 4; ++t) ra[t][c2] -= ra[t][c] * lk;
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int i = j0 + lane + 64 * t;
#pragma unroll
        for (int c = 0; c < 16; ++c)
          if (i < nr && j0 + c <= i && j0 + c < n) A[packed_index(i, j0 + c)] = ra[t][c];
      }
      if (badl && lane == 0) *bad = 1;
    }
    __syncthreads();
    const int s0 = j0 + 16;  // trailing rows s0 .. nr - 1, columns s0 .. min(i, n - 1)
    if (tid < 256 && s0 < nr) {
      const int nbr = (nr - s0 + 15) >> 4;
      for (int bi = 0; bi < nbr; ++bi) {
        const int i = s0 + 16 * bi + ty;
        if (i >= nr) continue;
        T li[16];
        const T* Li = A + packed_index(i, j0);
#pragma unroll
        for (int c = 0; c < 16; ++c) li[c] = Li[c];
        for (int bk = 0; bk <= bi; ++bk) {
          const int k = s0 + 16 * bk + tx;
          if (k > i || k >= n) continue;
          const T* Lk = A + packed_index(k, j0);
          T acc = (T)0;
#pragma unroll
          for (int c = 0; c < 16; ++c) acc += li[c] * Lk[c];
          A[packed_index(i, k)] -= acc;
        }
      }
    }
    __syncthreads();
  }
}

// Sixteen backward steps i = i_hi, i_hi - 1, ... (i < n) with row i held in
// register set TI: x_i = y_i / L_ii, then y_r -= L_ir x_i on every lane (l:
// L_ir of the lane's four rows, zero unless r < i); x_i is kept by the lane
// of row i.
template <typename T, int TI>
__device__ __forceinline__ void packed_back16(int i_hi, int n, const T (*l)[16], const T* iv, T* y, T* xk,
                                              int lane) {
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const int i = i_hi - c;
    if (i >= n) continue;  // uniform
    const T xi = lane_bcast(y[TI], i & 63) * iv[c];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      y[t] -= l[t][c] * xi;
      xk[t] = lane + 64 * t == i ? xi : xk[t];
    }
  }
}

// L^T x = y on the first wavefront for a packed factor with invd[j] = 1 /
// L_jj (n <= 256; y and x may alias).  Rows r = l + 64 t sit on lane l;
// blocks of 16 rows from the last, whose L entries are loaded before the
// dependent chain.  The other threads return at once (no barrier inside).
template <typename T>
__device__ __forceinline__ void packed_back_solve(const T* A, int n_in, const T* invd, const T* y_in, T* x) {
  if (threadIdx.x >= 64) return;
  const int n = __builtin_amdgcn_readfirstlane(n_in);
  const int lane = threadIdx.x;
  T y[4], xk[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    y[t] = lane + 64 * t < n ? y_in[lane + 64 * t] : (T)0;
    xk[t] = (T)0;
  }
  for (int blk = (n - 1) >> 4; blk >= 0; --blk) {
    T l[4][16], iv[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const int i = 16 * blk + 15 - c, ic = min(i, n - 1);
      iv[c] = invd[ic];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = lane + 64 * t;
        l[t][c] = (r < i && i < n) ? A[packed_index(ic, r)] : (T)0;
      }
    }
    switch (blk >> 2) {  // the set that holds rows 16 blk .. 16 blk + 15
      case 0: packed_back16<T, 0>(16 * blk + 15, n, l, iv, y, xk, lane); break;
      case 1: packed_back16<T, 1>(16 * blk + 15, n, l, iv, y, xk, lane); break;
      case 2: packed_back16<T, 2>(16 * blk + 15, n, l, iv, y, xk, lane); break;
      default: packed_back16<T, 3>(16 * blk + 15, n, l, iv, y, xk, lane); break;
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
    if (lane + 64 * t < n) x[lane + 64 * t] = xk[t];
}

// Sixteen forward steps i = i_lo, i_lo + 1, ... (i < n), row i in set TI:
// y_i = b_i / L_ii, then b_r -= L_ri y_i (l: L_ri, zero unless r > i).
template <typename T, int TI>
__device__ __forceinline__ void packed_fwd16(int i_lo, int n, const T (*l)[16], const T* iv, T* b, T* yk,
                                             int lane) {
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const int i = i_lo + c;
    if (i >= n) continue;  // uniform
    const T yi = lane_bcast(b[TI], i & 63) * iv[c];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      b[t] -= l[t][c] * yi;
      yk[t] = lane + 64 * t == i ? yi : yk[t];
    }
  }
}

// L y = b on the first wavefront (the companion of packed_back_solve; b and
// y may alias).
template <typename T>
__device__ __forceinline__ void packed_fwd_solve(const T* A, int n_in, const T* invd, const T* b_in, T* y) {
  if (threadIdx.x >= 64) return;
  const int n = __builtin_amdgcn_readfirstlane(n_in);
  const int lane = threadIdx.x;
  T b[4], yk[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    b[t] = lane + 64 * t < n ? b_in[lane + 64 * t] : (T)0;
    yk[t] = (T)0;
  }
  for (int blk = 0; 16 * blk < n; ++blk) {
    T l[4][16], iv[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const int i = 16 * blk + c, ic = min(i, n - 1);
      iv[c] = invd[ic];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = lane + 64 * t;
        l[t][c] = (r > i && r < n) ? A[packed_index(r, ic)] : (T)0;
      }
    }
    switch (blk >> 2) {
      case 0: packed_fwd16<T, 0>(16 * blk, n, l, iv, b, yk, lane); break;
      case 1: packed_fwd16<T, 1>(16 * blk, n, l, iv, b, yk, lane); break;
      case 2: packed_fwd16<T, 2>(16 * blk, n, l, iv, b, yk, lane); break;
      default: packed_fwd16<T, 3>(16 * blk, n, l, iv, b, yk, lane); break;
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
    if (lane + 64 * t < n) y[lane + 64 * t] = yk[t];
}

}  // namespace dpvba
