// Damped solve of the reduced camera system S dxi = s (DPV-SLAM Appendix A:
// the Cholesky factorisation of the pose block of the Schur complement).
//
// S is dense row-major n x n; only its lower triangle is read.  Two paths:
//  * small n: one workgroup factors S in LDS (packed lower triangle) and runs
//    both triangular solves;
//  * large n: blocked right-looking Cholesky with 64-wide panels (diagonal
//    block factor and inverse, panel solve as a product with that inverse,
//    trailing symmetric update), then blocked triangular solves that reuse the
//    stored diagonal-block inverses.
// A pivot that is not positive (or not finite) sets *status and is replaced
// by 1 so the arithmetic stays finite; the caller then discards the step.
// min_pivot receives the smallest L_ii^2 / S_ii (as ordered bits of a
// non-negative float, combined with an integer atomic minimum, which is
// order-independent).
#include <algorithm>

#include "common.h"
#include "factor_plan.h"
#include "mfma.h"
#include "packed.h"

namespace dpvba {

constexpr int kNB = 64;

// Two consecutive entries of the compute type (rows of S start on an even
// element, since n = 6 n_free, so the pair loads are aligned).
template <typename T> struct Pair2 { typedef T type __attribute__((ext_vector_type(2))); };

// rows x cols (<= 64 x 64, cols even) block at src (row stride ld) into
// dst[64][65], zero outside: each thread issues its eight pair loads before
// any store, so the block arrives in one memory round trip.
template <typename T, int NT>
__device__ __forceinline__ void load_block64_nt(const T* src, size_t ld, int rows, int cols, T (*dst)[kNB + 1]) {
  typedef typename Pair2<T>::type T2;
  constexpr int PER = kNB * kNB / 2 / NT;
  const int tid = threadIdx.x;
  T2 v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int q = tid + NT * u, r = q / (kNB / 2), c = 2 * (q % (kNB / 2));
    v[u] = (r < rows && c < cols) ? *reinterpret_cast<const T2*>(src + (size_t)r * ld + c) : T2{0, 0};
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int q = tid + NT * u, r = q / (kNB / 2), c = 2 * (q % (kNB / 2));
    dst[r][c] = v[u].x;
    dst[r][c + 1] = v[u].y;
  }
}

template <typename T>
__device__ __forceinline__ void load_block64(const T* src, size_t ld, int rows, int cols, T (*dst)[kNB + 1]) {
  load_block64_nt<T, 256>(src, ld, rows, cols, dst);
}

__device__ __forceinline__ void pivot_min(unsigned int* min_bits, float ratio) {
  if (!(ratio >= 0.f)) ratio = 0.f;
  atomicMin(min_bits, __float_as_uint(ratio));
}

// ------------------------------------------------------------------ small path

template <typename T>
__global__ void __launch_bounds__(256) small_chol_solve_kernel(const T* S, const T* rhs, int n, T* dx,
                                                               int* status, unsigned int* min_bits) {
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  T* d0 = reinterpret_cast<T*>(dyn_lds);  // [n] damped diagonal (pivot report)
  T* invd = d0 + n;                       // [n]
  T* piv = invd + n;                      // [n]
  T* x = piv + n;                         // [n]
  T* A = x + n;                           // packed lower, row i at i(i+1)/2; s appended as row n
  __shared__ int bad;
  __shared__ unsigned int minr_bits;
  const int tid = threadIdx.x;
  if (n + 1 <= kSmallRows) {  // the register-resident panel solver
    __shared__ float minr;
    const int nr = small_solve_rows(n);
    T* xr = reinterpret_cast<T*>(dyn_lds) + 37 * nr + nr * nr;  // after the solver's own arrays
    if (nr == 32) panel_chol_solve<T, 2>(n, S, rhs, nullptr, dyn_lds, xr, &bad, &minr, n);
    else if (nr == 64) panel_chol_solve<T, 4>(n, S, rhs, nullptr, dyn_lds, xr, &bad, &minr, n);
    else if (nr == 80) panel_chol_solve<T, 5>(n, S, rhs, nullptr, dyn_lds, xr, &bad, &minr, n);
    else panel_chol_solve<T, 6>(n, S, rhs, nullptr, dyn_lds, xr, &bad, &minr, n);
    for (int i = tid; i < n; i += blockDim.x) dx[i] = xr[i];  // zero when a pivot failed
    if (tid == 0) {
      if (bad) atomicOr(status, 1);
      pivot_min(min_bits, minr);
    }
    return;
  }
  const int np = n * (n + 1) / 2;
  // lower triangle of the dense row-major S, eight independent loads in
  // flight per thread
  const int nn = n * n;
  for (int q0 = tid; q0 < nn; q0 += 8 * blockDim.x) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = q0 + u * blockDim.x, i = q / n, j = q - (q / n) * n;
      v[u] = (q < nn && j <= i) ? S[q] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = q0 + u * blockDim.x, i = q / n, j = q - (q / n) * n;
      if (q < nn && j <= i) {
        A[packed_index(i, j)] = v[u];
        if (i == j) d0[i] = v[u];
      }
    }
  }
  for (int i = tid; i < n; i += blockDim.x) A[np + i] = rhs[i];
  if (tid == 0) {
    A[np + n] = (T)0;
    bad = 0;
    minr_bits = __float_as_uint(3.0e38f);
  }
  __syncthreads();
  packed_panel_factor<T>(A, n, n + 1, invd, piv, &bad);  // row n ends as y = L^-1 s
  pivot_ratio_min<T>(piv, d0, n, &minr_bits);              // smallest pivot / damped diagonal
  packed_back_solve<T>(A, n, invd, A + np, x);
  __syncthreads();
  for (int i = tid; i < n; i += blockDim.x) dx[i] = bad ? (T)0 : x[i];
  if (tid == 0) {
    if (bad) atomicOr(status, 1);
    pivot_min(min_bits, __uint_as_float(minr_bits));
  }
}

// ------------------------------------------------------------------ large path

// Factor the diagonal block at k0 (kb <= 64), write L back to S, and write
// inv(L_kk) (lower, kb x kb, stride 64, zeros above the diagonal) to Linv.
// The block is factored together with an identity appended below it: the
// Cholesky factor of [[A, I], [I, .]] has L^-T in its lower-left block, so
// one elimination gives both L and its inverse.  The 128 x 64 working
// matrix W (rows 0..63 the block, rows 64..127 the identity, row stride
// kWld) lives in LDS, filled by the caller (fill_diag_w): the block's lower
// triangle in rows and columns below kb, zeros elsewhere, and ones on the
// diagonal of the padding (rows kb..63) and of the identity, so that every
// panel takes all of its columns without a branch (the padding is never
// stored).  Columns go in panels of 16 (p = 0..3, a
// loop, not unrolled: the code is run once per launch and has to come into
// the instruction cache every time):
//   1. wavefront 0 factors the panel: lane l holds row l mod 16 of the
//      16 x 16 diagonal block (ra: each 16-lane row of the wavefront a full
//      copy) and one row of the panel below it (rb: lane row q takes row
//      block q of the four that can be non-zero -- the A rows of the later
//      blocks, the identity rows of the earlier panels and of this one; the
//      identity rows of later panels are still zero in this column block).
//      Column entries travel by the DPP row broadcast, a vector-register
//      move within each 16-lane row, so the chain of 16 pivots takes no
//      scalar registers and no barrier; the panel is written back;
//   2. after one barrier, the four wavefronts update the next column block
//      by the panel (one matrix-core product per 16 x 16 block, one block
//      each), which is all the next panel's chain needs; a second barrier
//      closes the panel.  The rest of the panel's rank-16 update (the later
//      column blocks, on the rows that can be non-zero) and the store of its
//      finished column block are done by wavefronts 1..3 while wavefront 0
//      factors the next panel, off the chain of dependent steps.
// ddv: this thread's entry of the damped diagonal (thread t < kb: column
// t), for the pivot report, which wavefront 0 forms panel by panel from the
// pivots it holds and issues at the end (no closing barrier).  Entries above the diagonal of the A part are
// never read as results.
constexpr int kWld = kNB + 1;

// Rank-16 update of diag_factor's working matrix by panel p on the matrix
// cores: the 16 x 16 blocks (bi, bk), bk = bk_lo .. bk_hi (<= 3), bi = bk ..
// 4 + p (the rows whose panel-p entries can be non-zero), bk-major, go to the
// wavefronts first, first + nwav, ...: W_(bi,bk) -= W_(bi,p) W_(bk,p)^T.
template <typename T>
__device__ __forceinline__ void diag_update_blocks(T* W, int p, int bk_lo, int first, int nwav, int bk_hi = 3) {
  const int lane = threadIdx.x & 63, c0 = 16 * p;
  int count = 0;
  for (int bk = bk_lo; bk <= bk_hi; ++bk) count += 5 + p - bk;
  for (int q = first; q < count; q += nwav) {
    int bk = bk_lo, rem = q;
    while (rem >= 5 + p - bk) {
      rem -= 5 + p - bk;
      ++bk;
    }
    const int bi = bk + rem;
    const T* xr = W + (16 * bi + (lane & 15)) * kWld + c0 + (lane >> 4);
    const T* yr = W + (16 * bk + (lane & 15)) * kWld + c0 + (lane >> 4);
    typename Mfma<T>::acc_t acc = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 16; k += 4) acc = Mfma<T>::step(xr[k], yr[k], acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) W[(16 * bi + Mfma<T>::row(lane, v)) * kWld + 16 * bk + (lane & 15)] -= acc[v];
  }
}

// Store of a finished column block (columns c0 .. c0 + 15) of diag_factor's
// working matrix: L rows c0 .. kb - 1 into S, and rows c0 .. c0 + 15 of
// L^-1 (zeros above its diagonal) into Linv; threads t0, t0 + nthr, ...
template <typename T>
__device__ __forceinline__ void diag_store_block(const T* W, T* S, int n, int k0, int kb, T* Linv, int c0, int t0,
                                                 int nthr) {
  if (t0 < 0) return;
  for (int e = t0; e < 1024; e += nthr) {
    const int r = e >> 4, c = c0 + (e & 15);
    if (r < kb && c <= r) S[(size_t)(k0 + r) * n + k0 + c] = W[r * kWld + c];
    const int kr = c0 + (e >> 6), rr = e & 63;  // Linv row kr, column rr
    if (kr < kb && rr < kb) Linv[kr * kNB + rr] = kr >= rr ? W[(kNB + rr) * kWld + kr] : (T)0;
  }
}


template <typename T>
__device__ __forceinline__ void diag_factor(T* W, T* S, int n, int k0, int kb_in, T* Linv, T ddv, int* status,
                                            unsigned int* min_bits) {
  __shared__ T dd[kNB];
  const int kb = __builtin_amdgcn_readfirstlane(kb_in);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  if (tid < kb) dd[tid] = ddv;  // wavefront 0, which alone reads it
  int bad = 0, last = 0;
  unsigned int minr = __float_as_uint(3.0e38f);  // wavefront 0: smallest pivot / damped diagonal
  for (int p = 0; 16 * p < kb; ++p) {
    const int c0 = 16 * p;
    // 1. the panel on wavefront 0
    if (wave == 0) {
      const int s = lane & 15, q = lane >> 4;
      // row block of rb: the A blocks p + 1 .. 3, then the identity blocks 4 .. 4 + p
      const int bq = q < 3 - p ? p + 1 + q : 4 + (q - (3 - p));
      T* wa = W + (c0 + s) * kWld + c0;
      T* wb = W + (16 * bq + s) * kWld + c0;
      T ra[16], rb[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        ra[c] = wa[c];
        rb[c] = wb[c];
      }
      T dpiv = (T)0;  // lane c: the pivot of column c
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const T d = row_bcast(ra[c], c);
        dpiv = s == c ? d : dpiv;
        const bool ok = d > (T)0 && d < (T)3.0e38;
        bad |= !ok;
        const T rs = ok ? pivot_rsqrt<T>(d) : (T)1;
        ra[c] *= rs;
        rb[c] *= rs;
#pragma unroll
        for (int c2 = c + 1; c2 < 16; ++c2) {
          const T l = row_bcast(ra[c], c2);  // L(c0 + c2, c0 + c)
          ra[c2] -= ra[c] * l;
          rb[c2] -= rb[c] * l;
        }
      }
      if (q == 0) {
#pragma unroll
        for (int c = 0; c < 16; ++c) wa[c] = ra[c];
      }
      // pivot report of the panel: lane s takes column c0 + s (a NaN counts as 0)
      {
        const float ratio = c0 + s < kb ? (float)(dpiv / dd[c0 + s]) : 3.0e38f;
        unsigned int m = __float_as_uint(ratio == ratio ? fmaxf(ratio, 0.f) : 0.f);
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) m = min(m, (unsigned int)__shfl_xor((int)m, o));
        minr = min(minr, m);
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) wb[c] = rb[c];
    } else if (p > 0) {
      // meanwhile wavefronts 1..3 finish panel p - 1: its update of the
      // column blocks p + 1 .. 3 and the store of its column block
      diag_update_blocks<T>(W, p - 1, p + 1, wave - 1, 3);
      diag_store_block<T>(W, S, n, k0, kb, Linv, 16 * (p - 1), tid - 64, 192);
    }
    __syncthreads();
    // 2. what the next panel needs first: column block p + 1 updated by
    // this panel (one 16 x 16 block per wavefront)
    if (16 * (p + 1) < kb) diag_update_blocks<T>(W, p, p + 1, wave, 4, p + 1);
    __syncthreads();
    last = p;
  }
  // the last panel's column block (its later column blocks are padding)
  diag_store_block<T>(W, S, n, k0, kb, Linv, 16 * last, tid, 256);
  if (tid == 0) {  // wavefront 0 holds the report; no barrier needed
    if (bad) atomicOr(status, 1);
    pivot_min(min_bits, __uint_as_float(minr));
  }
}

// Entry (i, c), i < 64, of diag_factor's working matrix, given the block's
// entry a (only read for i < kb, c <= i).
template <typename T>
__device__ __forceinline__ T diag_w_entry(int i, int c, int kb, T a) {
  return (i < kb && c <= i) ? a : (T)(i == c && i >= kb ? 1 : 0);
}

// The identity half of W (rows 64..127); every thread of the workgroup.
template <typename T>
__device__ __forceinline__ void fill_diag_identity(T* W) {
  const int r = threadIdx.x >> 2, c0 = 16 * (threadIdx.x & 3);
  T* w = W + (kNB + r) * kWld + c0;
#pragma unroll
  for (int c = 0; c < 16; ++c) w[c] = (T)(c0 + c == r ? 1 : 0);
}

// W from the kb x kb block of S at (k0, k0) (its lower triangle).
template <typename T>
__device__ __forceinline__ void fill_diag_w(const T* S, int n, int k0, int kb, T* W) {
  for (int e = threadIdx.x; e < kNB * kNB; e += blockDim.x) {
    const int i = e >> 6, c = e & 63;
    T a = (T)0;
    if (i < kb && c <= i) a = S[(size_t)(k0 + i) * n + k0 + c];
    W[i * kWld + c] = diag_w_entry<T>(i, c, kb, a);
  }
  fill_diag_identity<T>(W);
}

template <typename T>
__global__ void __launch_bounds__(256) potrf_diag_kernel(T* S, int n, int k0, int kb, T* Linv, const T* d0,
                                                         int* status, unsigned int* min_bits) {
  __shared__ T W[2 * kNB * kWld];
  const T ddv = threadIdx.x < kb ? d0[k0 + threadIdx.x] : (T)0;
  fill_diag_w<T>(S, n, k0, kb, W);
  __syncthreads();
  diag_factor<T>(W, S, n, k0, kb, Linv, ddv, status, min_bits);
}

// Panel solve below the diagonal block: L_ik = A_ik inv(L_kk)^T, one 64-row
// block per workgroup of sixteen wavefronts (one 16 x 16 output tile each,
// so the product's matrix-core chain is a quarter of that of four
// wavefronts; the panel solves sit on the factor's serial path), on the
// matrix cores: the blocks of rows [k0 + kb, R)
// that can be non-zero in the panel (R: the panel's reach, n for a dense
// matrix; with a list, only the listed blocks), then the appended rows
// [n, nrows).  With lead set, the workgroup of the first block below the
// diagonal block (rows t0 = k0 + kb ..) also updates the next diagonal block
// by the panel, A_t0t0 -= L_t0k L_t0k^T (its lower triangle), from the L
// block it has just formed: the next diagonal factor then starts from S
// alone.
template <typename T>
__global__ void __launch_bounds__(1024) trsm_panel_kernel(T* S, int n, int nrows, int R, int k0, int kb,
                                                         const T* Linv, const int* blocks, int n_main, int lead) {
  __shared__ T Ab[kNB][kNB + 1];
  __shared__ T Li[kNB][kNB + 1];
  const int t0 = k0 + kb;
  const int b = blockIdx.x;
  const int i0 = b < n_main ? t0 + (blocks ? blocks[b] : b) * kNB : n + (b - n_main) * kNB;
  const int rows = min(kNB, (b < n_main ? R : nrows) - i0);
  const int tid = threadIdx.x;
  // sixteen wavefronts: output tile (w mod 4, w / 4)
  const int lane = tid & 63, w = tid >> 6, wr = w & 3, wc = w >> 2;
  const bool lead_blk = lead && b < n_main && i0 == t0;
  const int rb = min(kNB, n - t0);
  // lower 16 x 16 tile w (< 10) of the next diagonal block, (di, dj): the ten
  // go to wavefronts 0..9, i.e. at most three per SIMD
  int di = 0;
  while ((di + 1) * (di + 2) / 2 <= w) ++di;
  const int dj = w - di * (di + 1) / 2;
  T dv[4];  // the next diagonal block's entries at that tile's product positions
  if (lead_blk) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * di + Mfma<T>::row(lane, v), c = 16 * dj + (lane & 15);
      dv[v] = (w < 10 && r < rb && c <= r) ? S[(size_t)(t0 + r) * n + t0 + c] : (T)0;
    }
  }
  load_block64_nt<T, 1024>(S + (size_t)i0 * n + k0, (size_t)n, rows, kb, Ab);
  load_block64_nt<T, 1024>(Linv, (size_t)kNB, kb, kb, Li);
  __syncthreads();
  typename Mfma<T>::acc_t acc = typename Mfma<T>::acc_t{0, 0, 0, 0};
  {
    const T* xr = &Ab[0][0] + (16 * wr + (lane & 15)) * (kNB + 1) + (lane >> 4);
    const T* yr = &Li[0][0] + (16 * wc + (lane & 15)) * (kNB + 1) + (lane >> 4);
    for (int kk = 0; kk < kNB; kk += 4) acc = Mfma<T>::step(xr[kk], yr[kk], acc);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = 16 * wr + Mfma<T>::row(lane, v), c = 16 * wc + (lane & 15);
    if (r < rows && c < kb) S[(size_t)(i0 + r) * n + k0 + c] = acc[v];
  }
  if (!lead_blk) return;
  // the L block (zero outside rows < rows, columns < kb) replaces A in LDS,
  // then the lower 16 x 16 tiles of L L^T, summed from zero and subtracted
  // once
  __syncthreads();
#pragma unroll
  for (int v = 0; v < 4; ++v) Ab[16 * wr + Mfma<T>::row(lane, v)][16 * wc + (lane & 15)] = acc[v];
  __syncthreads();
  if (w >= 10) return;
  typename Mfma<T>::acc_t p = typename Mfma<T>::acc_t{0, 0, 0, 0};
  {
    const T* xr = &Ab[0][0] + (16 * di + (lane & 15)) * (kNB + 1) + (lane >> 4);
    const T* yr = &Ab[0][0] + (16 * dj + (lane & 15)) * (kNB + 1) + (lane >> 4);
    for (int kk = 0; kk < kNB; kk += 4) p = Mfma<T>::step(xr[kk], yr[kk], p);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = 16 * di + Mfma<T>::row(lane, v), c = 16 * dj + (lane & 15);
    if (r < rb && c <= r) S[(size_t)(t0 + r) * n + t0 + c] = dv[v] - p[v];
  }
}

// Trailing update A_IJ -= L_Ik L_Jk^T for 64x64 blocks I >= J of the trailing
// matrix, on the matrix cores; blockIdx.x enumerates the lower block pairs,
// of all trailing blocks or, with act, of the listed ones (the blocks that
// hold a row non-zero in the panel, ascending, block 0 first: a pair with an
// all-zero side has a zero update).
// float32: at least three wavefronts per SIMD (at most 170 registers), so
// the trailing update keeps its occupancy although workgroup 0 also runs the
// register-heavy diagonal factor (which still fits without spilling).
template <typename T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 1)))
syrk_update_kernel(T* S, int n, int k0, int kb, T* Linv_next, const T* d0, int* status, unsigned int* min_bits,
                   const int* act) {
  __shared__ T Lij[2][kNB][kNB + 1];  // contiguous: the look-ahead's W after the update
  T (*Li)[kNB + 1] = Lij[0];
  T (*Lj)[kNB + 1] = Lij[1];
  const int t0 = k0 + kb;
  const int blk = blockIdx.x;
  int a = (int)((sqrt(8.0 * blk + 1.0) - 1.0) * 0.5);
  while (a * (a + 1) / 2 > blk) --a;
  while ((a + 1) * (a + 2) / 2 <= blk) ++a;
  const int b = blk - a * (a + 1) / 2;
  const int I = act ? act[a] : a, J = act ? act[b] : b;
  const int i0 = t0 + I * kNB, j0 = t0 + J * kNB;
  const int ri = min(kNB, n - i0), rj = min(kNB, n - j0);
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  typename Mfma<T>::acc_t acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = typename Mfma<T>::acc_t{0, 0, 0, 0};
  if (blk == 0 && Linv_next) {
    // workgroup 0: the next diagonal block (pair (0, 0)), A - L_0 L_0^T formed
    // straight into the factor's working matrix and factored at once, while
    // the other workgroups finish the trailing update (look-ahead of one
    // panel); the factor stores the block
    T sv[4][4];  // the block's entries at this lane's product positions
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * w + Mfma<T>::row(lane, v), c = 16 * t + (lane & 15);
        sv[t][v] = (r < ri && c <= r) ? S[(size_t)(i0 + r) * n + i0 + c] : (T)0;
      }
    const T ddv = tid < ri ? d0[t0 + tid] : (T)0;
    load_block64<T>(S + (size_t)i0 * n + k0, (size_t)n, ri, kb, Li);
    __syncthreads();
    gemm_nt_64<T>(&Li[0][0], &Li[0][0], kNB + 1, kNB, acc);
    __syncthreads();  // Li is overwritten by the working matrix
    T* W = &Lij[0][0][0];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * w + Mfma<T>::row(lane, v), c = 16 * t + (lane & 15);
        W[r * kWld + c] = diag_w_entry<T>(r, c, ri, sv[t][v] - acc[t][v]);
      }
    fill_diag_identity<T>(W);
    __syncthreads();
    diag_factor<T>(W, S, n, t0, ri, Linv_next, ddv, status, min_bits);
    return;
  }
  load_block64<T>(S + (size_t)i0 * n + k0, (size_t)n, ri, kb, Li);
  load_block64<T>(S + (size_t)j0 * n + k0, (size_t)n, rj, kb, Lj);
  __syncthreads();
  gemm_nt_64<T>(&Li[0][0], &Lj[0][0], kNB + 1, kNB, acc);
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * w + Mfma<T>::row(lane, v), c = 16 * t + (lane & 15);
      if (r < ri && c < rj && (I != J || c <= r)) S[(size_t)(i0 + r) * n + j0 + c] -= acc[t][v];
    }
}

// Trailing update of the float32 factor: A_IJ -= L_Ik L_Jk^T for the lower
// pairs (I, J) of 64-row blocks of the trailing rows and columns [t0, R),
// K = 64 (one panel), one workgroup per pair.  R is the panel's reach: the
// rows below it have no entry in the panel (the envelope of a sparse reduced
// system: fill stays between a row's first non-zero and the diagonal), so
// their update is exactly zero and is skipped; R = n for a dense matrix.
// With a list of the active blocks (those holding a row that is non-zero in
// the panel, factor_plan.h) only their pairs are launched: a pair with an
// all-zero side has a zero update.  Each of the four wavefronts takes one
// 32 x 32 quadrant as 2 x 2 matrix-core tiles accumulating L_I L_J^T; the
// quadrant above the diagonal of a diagonal pair is skipped.  The products
// are then staged in LDS and A is read and written as contiguous 256-byte
// rows: A - L_I L_J^T.  The pairs are 64 rows high, not 128: a trailing
// update of the sparse system has only a few active rows per panel, so a
// launch holds far fewer workgroups than the chip has CUs and each
// workgroup's latency (its loads and its products on one CU) is what counts.
// The right-hand side appended as row n (nrows = n + 1) is updated by the
// diagonal pairs: s_J -= L_J l_n, from the panel rows they hold anyway.
//
// Look-ahead: with Linv_next, workgroup 0 factors the next diagonal block at
// once (pair (0, 0), whose workgroup only updates the right-hand side here),
// so the factor of the next panel starts with the launch instead of after the
// update.  The panel solve before this launch (its lead workgroup) has
// already subtracted the panel's share from that block.
constexpr int kTB = 64;     // trailing-update tile: one pair of 64-row blocks
constexpr int kPanLd = 68;  // LDS row stride of the staged panel rows and products
constexpr int kPiFloats = 2 * kNB * kWld;  // the look-ahead's working matrix, or a tile's row-block panel rows
constexpr int kPjFloats = kTB * kPanLd;
constexpr int kSyrk64Lds = (kPiFloats + kPjFloats) * 4;
static_assert(kPiFloats >= kTB * kPanLd, "LDS regions");

// Two wavefronts per SIMD (at most 256 registers), so two workgroups share a
// CU although workgroup 0 also runs the register-heavy diagonal factor.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
syrk64_kernel(float* S, int n, int nrows, int R, int k0, int kb, float* Linv_next, const float* d0, int* status,
               unsigned int* min_bits, const int* act) {
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  __shared__ float lrhs[kNB];  // l_n: the right-hand-side row's panel entries
  typedef float f2 __attribute__((ext_vector_type(2)));
  float* Pi = reinterpret_cast<float*>(dyn_lds);
  float* Pj = Pi + kPiFloats;
  const int t0 = k0 + kb;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const bool look = Linv_next != nullptr;
  if (look && blockIdx.x == 0) {
    // next diagonal block, already updated by the panel (the panel solve's
    // lead workgroup): its lower triangle into W, then its factor
    float* W = Pi;
    const int rb = min(kNB, n - t0);
    const float ddv = tid < rb ? d0[t0 + tid] : 0.f;
    float av[16];  // rows w + 4 u, column lane: one 256-byte row per access
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int r = w + 4 * u;
      av[u] = (r < rb && lane <= r) ? S[(size_t)(t0 + r) * n + t0 + lane] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int r = w + 4 * u;
      W[r * kWld + lane] = diag_w_entry<float>(r, lane, rb, av[u]);
    }
    fill_diag_identity<float>(W);
    __syncthreads();
    diag_factor<float>(W, S, n, t0, rb, Linv_next, ddv, status, min_bits);
    return;
  }
  const int blk = blockIdx.x - (look ? 1 : 0);
  int a = (int)((sqrt(8.0 * blk + 1.0) - 1.0) * 0.5);
  while (a * (a + 1) / 2 > blk) --a;
  while ((a + 1) * (a + 2) / 2 <= blk) ++a;
  const int b = blk - a * (a + 1) / 2;
  // pair (a, b), b <= a, of the active blocks (all blocks up to the reach without a list)
  const int I = act ? act[a] : a, J = act ? act[b] : b;
  const int i0 = t0 + I * kTB, j0 = t0 + J * kTB;
  const int ri = min(kTB, R - i0), rj = min(kTB, R - j0);
  const bool rhs_row = I == J && nrows > n;
  if (rhs_row && tid < kNB) lrhs[tid] = tid < kb ? S[(size_t)n * n + k0 + tid] : 0.f;
  // the next diagonal block (pair (0, 0)) is the look-ahead's: here only its
  // share of the right-hand-side row
  const bool lead = look && I == 0 && J == 0;
  const int wr = w >> 1, wc = w & 1;
  const bool active = !lead && !(I == J && wr < wc);
  const float* PJ = I == J ? Pi : Pj;  // a diagonal pair stages its panel rows once
  // accumulators (lane: column 16 tj + (lane & 15), rows 4 (lane >> 4) + v of
  // tile ti of the wavefront's 32 x 32 quadrant) collect L_I L_J^T from zero
  // and are subtracted from A once: starting them from A would round every
  // step at the size of A, which the update nearly cancels on the
  // ill-conditioned directions
  floatx4_t acc[2][2];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = floatx4_t{0.f, 0.f, 0.f, 0.f};
  // the tile's own entries, read at once so that their latency overlaps the
  // panel loads and the products: thread t takes rows (t >> 5) + 8 u,
  // columns 2 (t & 31) and 2 (t & 31) + 1 (each access instruction covers
  // two contiguous 256-byte rows)
  const int cc = 2 * (tid & 31), rr = tid >> 5;
  f2 av[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int r = rr + 8 * u;
    av[u] = (!lead && r < ri && cc < rj) ? *reinterpret_cast<const f2*>(S + (size_t)(i0 + r) * n + j0 + cc)
                                         : f2{0.f, 0.f};  // rj is even: n and j0 are
  }
  // panel rows: 64 x kb of columns k0.. for the row block and the column block
  {
    f2 va[8], vb[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = tid + 256 * u, r = q >> 5, c = 2 * (q & 31);
      va[u] = (r < ri && c < kb) ? *reinterpret_cast<const f2*>(S + (size_t)(i0 + r) * n + k0 + c) : f2{0.f, 0.f};
      vb[u] = (I != J && r < rj && c < kb) ? *reinterpret_cast<const f2*>(S + (size_t)(j0 + r) * n + k0 + c)
                                           : f2{0.f, 0.f};
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = tid + 256 * u, r = q >> 5, c = 2 * (q & 31);
      *reinterpret_cast<f2*>(Pi + r * kPanLd + c) = va[u];
      if (I != J) *reinterpret_cast<f2*>(Pj + r * kPanLd + c) = vb[u];
    }
  }
  __syncthreads();
  if (active) {
    const float* pa = Pi + (32 * wr + (lane & 15)) * kPanLd + (lane >> 4);
    const float* pb = PJ + (32 * wc + (lane & 15)) * kPanLd + (lane >> 4);
    for (int k = 0; k < kNB; k += 4) {
      float x[2], y[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        x[t] = pa[16 * t * kPanLd + k];
        y[t] = pb[16 * t * kPanLd + k];
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[ti], y[tj], acc[ti][tj], 0, 0, 0);
    }
  }
  if (rhs_row) {
    // s_(j0 + c) -= sum_k L_(j0 + c, k) l_n(k): thread (c, q) takes 16 k
    const int c = tid >> 2, h = tid & 3;
    const float* pr = PJ + c * kPanLd + 16 * h;
    float sum = 0.f;
#pragma unroll
    for (int k = 0; k < 16; ++k) sum += pr[k] * lrhs[16 * h + k];
    sum += __shfl_xor(sum, 1);
    sum += __shfl_xor(sum, 2);
    if (h == 0 && c < rj) S[(size_t)n * n + j0 + c] -= sum;
  }
  if (lead) return;
  __syncthreads();  // the panel rows are dead: their LDS takes the products
  float* Out = Pi;  // [64][kPanLd]
  if (active) {
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 32 * wr + 16 * ti + 4 * (lane >> 4) + v, c = 32 * wc + 16 * tj + (lane & 15);
          Out[r * kPanLd + c] = acc[ti][tj][v];
        }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int r = rr + 8 * u;
    if (r >= ri || cc >= rj) continue;
    const float* o = Out + r * kPanLd + cc;
    const f2 nv = av[u] - f2{o[0], o[1]};
    float* dst = S + (size_t)(i0 + r) * n + j0 + cc;
    if (I != J || cc + 1 <= r) {
      *reinterpret_cast<f2*>(dst) = nv;
    } else if (cc == r) {
      dst[0] = nv.x;
    }
  }
}

// Both triangular solves of a blocked factor in one cooperative launch.
// The 64-row blocks go in pairs (2P, 2P + 1), and workgroup g owns the pairs
// P = g, g + G, ...  Forward (L y = b): pair Q subtracts L_IK y_K (I in the
// pair, K in an earlier pair) as each earlier pair is published, solves its
// first block with inv(L_II), subtracts that block's share from the second
// inside the workgroup and solves the second; backward (L^T x = y) runs the
// same chain from the last pair down with L_KI^T and inv(L_II)^T.  Pairing
// halves the number of inter-workgroup hops on the dependent chain.  A pair
// is published through its solved values themselves (below).  Every wait is
// bounded: on timeout *err is set and the workgroup returns, so every
// workgroup exits; a wait also gives up as soon as another workgroup's wait
// (or a grid barrier of the call) has expired, but not for an input-range
// report, which leaves the arithmetic valid.  The L blocks are loaded before
// the wait for the vector they multiply, so the chain only carries the
// dependent part.  With pair_lo / pair_hi (a factor plan's envelope) a pair
// takes only the earlier pairs from pair_lo[Q] (forward) and the later ones
// up to pair_hi[Q] (backward): the other blocks of L it would multiply are
// zero.  With *skip set on the device the whole call is a no-op (every
// workgroup returns before any wait).
constexpr long long kChainSpin = 1LL << 22;

// The solved values of both passes travel with the call's epoch in 64-bit
// words (32 value bits low, the epoch high: one word per float32 value, two
// per float64 value, low half first; separate word arrays for the forward
// and the backward pass), stored and polled as single-copy-atomic
// agent-scope words, so a value is its own flag: no release of the
// producer's cache, no acquire on the consumer's, and the data arrives with
// the signal.
template <typename T>
__device__ __forceinline__ void chain_put_x(unsigned long long* xw, int row, T v, int epoch) {
  const unsigned long long tag = (unsigned long long)(unsigned)epoch << 32;
  if constexpr (sizeof(T) == 4) {
    __hip_atomic_store(xw + row, tag | (unsigned long long)__float_as_uint(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  } else {
    const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
    __hip_atomic_store(xw + 2 * (size_t)row, tag | (bits & 0xffffffffull), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(xw + 2 * (size_t)row + 1, tag | (bits >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// One word polled until it carries `epoch` (bounded); false on a timeout or
// another wait's failure (reported).
__device__ __forceinline__ bool chain_poll_word(const unsigned long long* w, int epoch, int* err, int* host_err,
                                                unsigned long long* out) {
  unsigned long long word = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  long long spins = 0;
  while ((int)(word >> 32) != epoch) {
    __builtin_amdgcn_s_sleep(1);
    if (++spins > kChainSpin ||
        (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & (kErrChain | kErrBarrier))) {
      report_device_error(err, host_err, kErrChain);
      return false;
    }
    word = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  *out = word;
  return true;
}

// vk[h][t] = the values of rows k0 + t (h = 0, t < kb0) and k1 + t (h = 1,
// t < kb1), each polled until it carries `epoch`.
template <typename T>
__device__ __forceinline__ bool chain_get_x(const unsigned long long* xw, int k0, int kb0, int k1, int kb1,
                                            int epoch, int* err, int* host_err, T (*vk)[kNB]) {
  __shared__ int fail_s;
  const int tid = threadIdx.x;
  if (tid == 0) fail_s = 0;
  __syncthreads();
  if (tid < 2 * kNB) {
    const int h = tid >> 6, t = tid & 63;
    const int rows = h ? kb1 : kb0;
    T v = (T)0;
    if (t < rows) {
      const int row = (h ? k1 : k0) + t;
      unsigned long long lo = 0, hi = 0;
      if constexpr (sizeof(T) == 4) {
        if (chain_poll_word(xw + row, epoch, err, host_err, &lo)) v = __uint_as_float((unsigned)(lo & 0xffffffffull));
        else fail_s = 1;
      } else {
        if (chain_poll_word(xw + 2 * (size_t)row, epoch, err, host_err, &lo) &&
            chain_poll_word(xw + 2 * (size_t)row + 1, epoch, err, host_err, &hi))
          v = __longlong_as_double((long long)(((hi & 0xffffffffull) << 32) | (lo & 0xffffffffull)));
        else
          fail_s = 1;
      }
    }
    vk[h][t] = v;
  }
  __syncthreads();
  return fail_s == 0;
}

template <typename T>
__global__ void __launch_bounds__(256) trsv_chain_kernel(const T* L, int n, const T* Linv_all, const T* b, T* y,
                                                         T* x, int* flags, int epoch, int* err, int* host_err,
                                                         int backward_only, const int* pair_lo,
                                                         const int* pair_hi, const int* skip) {
  if (skip && *skip) return;
  __shared__ T Li[2][kNB][kNB + 1];  // inverses of the pair's diagonal blocks
  __shared__ T acc[2][kNB];
  __shared__ T vk[2][kNB];
  __shared__ T part[2][4][kNB + 1];
  const int nblk = (n + kNB - 1) / kNB;
  const int npair = (nblk + 1) / 2;
  const int tid = threadIdx.x;
  const int G = gridDim.x;
  // the backward and forward passes' value words (flags is 8-byte aligned;
  // the caller sizes it for them)
  constexpr int kWords = sizeof(T) == 4 ? 1 : 2;
  unsigned long long* xw = reinterpret_cast<unsigned long long*>(flags);
  unsigned long long* yw = xw + (size_t)nblk * kNB * kWords;
  // ---- forward: thread (r, q) = (tid / 4, tid mod 4) takes row r, columns 16 q .. 16 q + 15
  // (skipped when the factor already produced y = L^-1 b in y)
  for (int Q = backward_only ? npair : blockIdx.x; Q < npair; Q += G) {
    const int I0 = 2 * Q, I1 = 2 * Q + 1;
    const int i0 = I0 * kNB, rows0 = min(kNB, n - i0);
    const int i1 = I1 * kNB, rows1 = I1 < nblk ? min(kNB, n - i1) : 0;
    if (tid < kNB) {
      acc[0][tid] = tid < rows0 ? b[i0 + tid] : (T)0;
      acc[1][tid] = tid < rows1 ? b[i1 + tid] : (T)0;
    }
    for (int idx = tid; idx < kNB * kNB; idx += blockDim.x) {  // entries outside a partial block are never written
      const int ra = idx / kNB, cb = idx % kNB;
      Li[0][ra][cb] = (ra < rows0 && cb < rows0) ? Linv_all[(size_t)I0 * kNB * kNB + idx] : (T)0;
      Li[1][ra][cb] = (ra < rows1 && cb < rows1) ? Linv_all[(size_t)I1 * kNB * kNB + idx] : (T)0;
    }
    const int r = tid >> 2, q = tid & 3;
    T lc[16];  // L_{I1, I0}: the in-pair block
#pragma unroll
    for (int m = 0; m < 16; ++m) lc[m] = r < rows1 ? L[(size_t)(i1 + r) * n + i0 + 16 * q + m] : (T)0;
    for (int P = pair_lo ? pair_lo[Q] : 0; P < Q; ++P) {
      const int k0 = 2 * P * kNB;  // both blocks of an earlier pair are full
      T la[32], lb[32];
#pragma unroll
      for (int m = 0; m < 32; ++m) {
        const int col = k0 + (m >> 4) * kNB + 16 * q + (m & 15);
        la[m] = r < rows0 ? L[(size_t)(i0 + r) * n + col] : (T)0;
        lb[m] = r < rows1 ? L[(size_t)(i1 + r) * n + col] : (T)0;
      }
      if (!chain_get_x<T>(yw, k0, kNB, k0 + kNB, kNB, epoch, err, host_err, vk)) return;
      T va = (T)0, vb = (T)0;
#pragma unroll
      for (int m = 0; m < 32; ++m) {
        const T v = vk[m >> 4][16 * q + (m & 15)];
        va += la[m] * v;
        vb += lb[m] * v;
      }
      part[0][q][r] = va;
      part[1][q][r] = vb;
      __syncthreads();
      if (tid < 2 * kNB) {
        const int h = tid >> 6, t = tid & 63;
        acc[h][t] -= (part[h][0][t] + part[h][1][t]) + (part[h][2][t] + part[h][3][t]);
      }
      __syncthreads();
    }
    __syncthreads();
    {  // first block: y = inv(L_II) acc (thread (r, q): 16 terms of row r), kept in vk[0]
      T v = (T)0;
#pragma unroll
      for (int m = 0; m < 16; ++m) v += Li[0][r][16 * q + m] * acc[0][16 * q + m];
      part[0][q][r] = v;
      __syncthreads();
      if (tid < kNB) {
        const T w = (part[0][0][tid] + part[0][1][tid]) + (part[0][2][tid] + part[0][3][tid]);
        vk[0][tid] = tid < rows0 ? w : (T)0;
        if (tid < rows0) {
          y[i0 + tid] = w;
          chain_put_x<T>(yw, i0 + tid, w, epoch);
        }
      }
      __syncthreads();
    }
    if (rows1) {
      T v = (T)0;
#pragma unroll
      for (int m = 0; m < 16; ++m) v += lc[m] * vk[0][16 * q + m];
      part[1][q][r] = v;
      __syncthreads();
      if (tid < kNB) acc[1][tid] -= (part[1][0][tid] + part[1][1][tid]) + (part[1][2][tid] + part[1][3][tid]);
      __syncthreads();
      T w = (T)0;
#pragma unroll
      for (int m = 0; m < 16; ++m) w += Li[1][r][16 * q + m] * acc[1][16 * q + m];
      part[0][q][r] = w;
      __syncthreads();
      if (tid < rows1) {
        const T v1 = (part[0][0][tid] + part[0][1][tid]) + (part[0][2][tid] + part[0][3][tid]);
        y[i1 + tid] = v1;
        chain_put_x<T>(yw, i1 + tid, v1, epoch);
      }
    }

  }
  // ---- backward, pairs in decreasing order: thread (c, q) = (tid mod 64, tid / 64)
  // takes column c and rows 16 q .. 16 q + 15 of a block
  const int last = blockIdx.x + ((npair - 1 - blockIdx.x) / G) * G;
  for (int Q = last; Q >= 0 && blockIdx.x < npair; Q -= G) {
    const int I0 = 2 * Q, I1 = 2 * Q + 1;
    const int i0 = I0 * kNB, rows0 = min(kNB, n - i0);
    const int i1 = I1 * kNB, rows1 = I1 < nblk ? min(kNB, n - i1) : 0;
    if (tid < kNB) {
      acc[0][tid] = tid < rows0 ? y[i0 + tid] : (T)0;
      acc[1][tid] = tid < rows1 ? y[i1 + tid] : (T)0;
    }
    for (int idx = tid; idx < kNB * kNB; idx += blockDim.x) {  // entries outside a partial block are never written
      const int ra = idx / kNB, cb = idx % kNB;
      Li[0][ra][cb] = (ra < rows0 && cb < rows0) ? Linv_all[(size_t)I0 * kNB * kNB + idx] : (T)0;
      Li[1][ra][cb] = (ra < rows1 && cb < rows1) ? Linv_all[(size_t)I1 * kNB * kNB + idx] : (T)0;
    }
    const int c = tid & 63, q = tid >> 6;
    T lc[16];  // column c of L_{I1, I0}^T = L_{I1, I0} rows 16 q .., column c
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int rr = 16 * q + m;
      lc[m] = (rr < rows1 && c < rows0) ? L[(size_t)(i1 + rr) * n + i0 + c] : (T)0;
    }
    for (int P = pair_hi ? pair_hi[Q] : npair - 1; P > Q; --P) {
      const int K0 = 2 * P, K1 = 2 * P + 1;
      const int k0 = K0 * kNB, kb0 = min(kNB, n - k0);
      const int k1 = K1 * kNB, kb1 = K1 < nblk ? min(kNB, n - k1) : 0;
      T la[32], lb[32];  // columns c of blocks I0 / I1, rows of K0 (m < 16) and K1 (m >= 16)
#pragma unroll
      for (int m = 0; m < 32; ++m) {
        const int rr = 16 * q + (m & 15);
        const int kb = m < 16 ? kb0 : kb1, kr = m < 16 ? k0 : k1;
        la[m] = (rr < kb && c < rows0) ? L[(size_t)(kr + rr) * n + i0 + c] : (T)0;
        lb[m] = (rr < kb && c < rows1) ? L[(size_t)(kr + rr) * n + i1 + c] : (T)0;
      }
      if (!chain_get_x<T>(xw, k0, kb0, k1, kb1, epoch, err, host_err, vk)) return;
      T va = (T)0, vb = (T)0;
#pragma unroll
      for (int m = 0; m < 32; ++m) {
        const T v = vk[m >> 4][16 * q + (m & 15)];
        va += la[m] * v;
        vb += lb[m] * v;
      }
      part[0][q][c] = va;
      part[1][q][c] = vb;
      __syncthreads();
      if (tid < 2 * kNB) {
        const int h = tid >> 6, t = tid & 63;
        acc[h][t] -= (part[h][0][t] + part[h][1][t]) + (part[h][2][t] + part[h][3][t]);
      }
      __syncthreads();
    }
    __syncthreads();
    if (rows1) {  // second block first: x = inv(L_II)^T acc (thread (c, q): 16 terms of column c), kept in vk[1]
      T v = (T)0;
#pragma unroll
      for (int m = 0; m < 16; ++m) v += Li[1][16 * q + m][c] * acc[1][16 * q + m];
      part[1][q][c] = v;
      __syncthreads();
      if (tid < kNB) {
        const T w = (part[1][0][tid] + part[1][1][tid]) + (part[1][2][tid] + part[1][3][tid]);
        vk[1][tid] = tid < rows1 ? w : (T)0;
        if (tid < rows1) {
          x[i1 + tid] = w;
          chain_put_x<T>(xw, i1 + tid, w, epoch);
        }
      }
      __syncthreads();
      T u = (T)0;
#pragma unroll
      for (int m = 0; m < 16; ++m) u += lc[m] * vk[1][16 * q + m];
      part[0][q][c] = u;
      __syncthreads();
      if (tid < kNB) acc[0][tid] -= (part[0][0][tid] + part[0][1][tid]) + (part[0][2][tid] + part[0][3][tid]);
      __syncthreads();
    }
    {
      T v = (T)0;
#pragma unroll
      for (int m = 0; m < 16; ++m) v += Li[0][16 * q + m][c] * acc[0][16 * q + m];
      part[1][q][c] = v;
      __syncthreads();
      if (tid < rows0) {
        const T v0 = (part[1][0][tid] + part[1][1][tid]) + (part[1][2][tid] + part[1][3][tid]);
        x[i0 + tid] = v0;
        chain_put_x<T>(xw, i0 + tid, v0, epoch);
      }
    }

  }
}

template <typename T>
__global__ void copy_vec_kernel(T* dst, const T* src, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

template <typename T>
__global__ void zero_on_status_kernel(T* dx, int n, const int* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && *status) dx[i] = (T)0;
}


// ------------------------------------------------------------------ launchers

// packed panel factor in LDS; the substitutions keep the vector on one
// wavefront (n <= 255)
int small_solve_max_n(int tsize) { return tsize == 4 ? 240 : 160; }

// Blocked factorisation in place (lower triangle of S becomes L) with the
// diagonal-block inverses in Linv_all.  nrows >= n rows of S (row stride n)
// take part: with the right-hand side appended as row n (nrows = n + 1,
// float32 only) that row ends as y = L^-1 s, the forward substitution
// done by the factorisation's own panel solves and trailing updates.
template <typename T>
hipError_t launch_chol_factor(T* S, int n, int nrows, T* Linv_all, const T* d0, int* status,
                              unsigned int* min_bits, hipStream_t st, const PanelPlan* plan) {
  const int nblk = (n + kNB - 1) / kNB;
  if (nblk == 0) return hipSuccess;
  if (sizeof(T) == 8 && nrows != n) return hipErrorInvalidValue;
  if (nrows != n && nrows != n + 1) return hipErrorInvalidValue;  // at most the right-hand side appended
  // with a plan only the 64-row blocks that hold a row non-zero in the panel
  // are solved and updated; float32 also stops at the panel's reach (the last
  // row that can be non-zero in it)
  const bool sparse = plan != nullptr;
  auto reach_of = [&](int k) { return sparse && sizeof(T) == 4 ? std::min(n, std::max(plan->reach[k], 0)) : n; };
  hipLaunchKernelGGL((potrf_diag_kernel<T>), dim3(1), dim3(256), 0, st, S, n, 0, min(kNB, n), Linv_all, d0, status,
                     min_bits);
  if constexpr (sizeof(T) == 4) {
    hipError_t e = opt_in_lds((const void*)syrk64_kernel, kSyrk64Lds);
    if (e != hipSuccess) return e;
  }
  for (int k = 0; k + 1 < nblk; ++k) {
    const int k0 = k * kNB, kb = min(kNB, n - k0);
    T* Linv = Linv_all + (size_t)k * kNB * kNB;
    const int t0 = k0 + kb;
    const int R = reach_of(k);
    const int n_main = sparse ? plan->blocks_off[k + 1] - plan->blocks_off[k]
                              : (R > t0 ? (R - t0 + kNB - 1) / kNB : 0);
    if (n_main + nrows - n > 0)
      hipLaunchKernelGGL((trsm_panel_kernel<T>), dim3(n_main + nrows - n), dim3(1024), 0, st, S, n, nrows, R, k0, kb,
                         Linv, sparse ? plan->blocks + plan->blocks_off[k] : (const int*)nullptr, n_main,
                         sizeof(T) == 4 ? 1 : 0);
    // the trailing update also factors diagonal block k + 1 (its workgroup 0)
    if constexpr (sizeof(T) == 4) {
      const int pairs = n_main * (n_main + 1) / 2;
      hipLaunchKernelGGL(syrk64_kernel, dim3(pairs + 1), dim3(256), kSyrk64Lds, st, S, n, nrows, R, k0, kb,
                         Linv + kNB * kNB, d0, status, min_bits,
                         sparse ? plan->blocks + plan->blocks_off[k] : (const int*)nullptr);
    } else {
      const int rest = sparse ? n_main : nblk - k - 1;
      hipLaunchKernelGGL((syrk_update_kernel<T>), dim3(rest * (rest + 1) / 2), dim3(256), 0, st, S, n, k0, kb,
                         Linv + kNB * kNB, d0, status, min_bits,
                         sparse ? plan->blocks + plan->blocks_off[k] : (const int*)nullptr);
    }
  }
  if (nrows > n) {  // the appended rows below the last diagonal block: their last panel solve
    const int k0 = (nblk - 1) * kNB;
    hipLaunchKernelGGL((trsm_panel_kernel<T>), dim3((nrows - n + kNB - 1) / kNB), dim3(1024), 0, st, S, n, nrows, n,
                       k0, n - k0, Linv_all + (size_t)(nblk - 1) * kNB * kNB, (const int*)nullptr, 0, 0);
  }
  return hipGetLastError();
}

// x = (L L^T)^-1 rhs with a factor from launch_chol_factor.
template <typename T>
int trsv_chain_grid(int nblk) {
  int per_cu = 0, dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)trsv_chain_kernel<T>, 256, 0) !=
      hipSuccess)
    return 0;
  return std::min((nblk + 1) / 2, per_cu * cus);  // one workgroup per pair of blocks at most
}

// x = (L L^T)^-1 rhs with a factor from launch_chol_factor: one cooperative
// launch (trsv_chain_kernel).  flags (8-byte aligned) holds the two passes'
// value words, 2 x 64 ceil(n / 64) x (1 for float32, 2 for float64) 64-bit
// words that the library never resets: each call passes a fresh epoch.
// backward_only: work_y already holds y = L^-1 rhs (rhs unused).  The grid
// never exceeds the workgroups the device holds at once (at most one per
// pair of 64-row blocks).  cooperative = false (the default): an ordinary
// launch, relying on the device placing every workgroup while the others
// wait for their predecessors -- true when the device's other work finishes;
// every wait is bounded, so a violation is reported (kErrChain), never a
// hang.  cooperative = true: the runtime guarantees co-residency, at the
// cost of a cooperative launch.
template <typename T>
hipError_t launch_chol_apply(const T* L, int n, const T* Linv_all, const T* rhs, T* x, T* work_y, int* flags,
                             int epoch, int* err, int* host_err, hipStream_t st, int backward_only = 0,
                             bool cooperative = false, const PanelPlan* plan = nullptr, const int* skip = nullptr) {
  const int nblk = (n + kNB - 1) / kNB;
  const int grid = trsv_chain_grid<T>(nblk);
  if (grid < 1) return hipErrorCooperativeLaunchTooLarge;
  const int* pair_lo = plan ? plan->chain_lo : nullptr;
  const int* pair_hi = plan ? plan->chain_hi : nullptr;
  if (!cooperative) {
    hipLaunchKernelGGL((trsv_chain_kernel<T>), dim3(grid), dim3(256), 0, st, L, n, Linv_all, rhs, work_y, x, flags,
                       epoch, err, host_err, backward_only, pair_lo, pair_hi, skip);
    return hipGetLastError();
  }
  void* args[] = {(void*)&L,     (void*)&n,   (void*)&Linv_all, (void*)&rhs,           (void*)&work_y,
                  (void*)&x,     (void*)&flags, (void*)&epoch,  (void*)&err,           (void*)&host_err,
                  (void*)&backward_only, (void*)&pair_lo, (void*)&pair_hi, (void*)&skip};
  return hipLaunchCooperativeKernel((const void*)trsv_chain_kernel<T>, dim3(grid), dim3(256), args, 0, st);
}

template <typename T>
hipError_t launch_chol_solve(T* S, const T* rhs, int n, T* dx, T* work_y, T* Linv_all, const T* d0, int* status,
                             unsigned int* min_bits, int* flags, int epoch, int* err, int* host_err,
                             hipStream_t st, bool cooperative, const PanelPlan* plan) {
  if (n == 0) return hipSuccess;
  if (n <= small_solve_max_n(sizeof(T))) {
    const int lds = n + 1 <= kSmallRows
                        ? std::max(packed_solve_lds_bytes(n, sizeof(T)), small_solve_lds_bytes(n, sizeof(T)))
                        : packed_solve_lds_bytes(n, sizeof(T));
    {
      hipError_t e = opt_in_lds((const void*)small_chol_solve_kernel<T>, lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((small_chol_solve_kernel<T>), dim3(1), dim3(256), lds, st, S, rhs, n, dx, status, min_bits);
    return hipGetLastError();
  }
  hipError_t e;
  if constexpr (sizeof(T) == 4) {
    // s appended as row n of S (which has room for n + 1 rows): the factor
    // leaves y = L^-1 s there and only the backward chain remains
    T* yrow = S + (size_t)n * n;
    if (rhs != yrow)  // a caller may have gathered s straight into that row
      hipLaunchKernelGGL((copy_vec_kernel<T>), dim3((n + 255) / 256), dim3(256), 0, st, yrow, rhs, n);
    e = launch_chol_factor<T>(S, n, n + 1, Linv_all, d0, status, min_bits, st, plan);
    if (e != hipSuccess) return e;
    e = launch_chol_apply<T>(S, n, Linv_all, rhs, dx, yrow, flags, epoch, err, host_err, st, 1, cooperative, plan);
  } else {
    e = launch_chol_factor<T>(S, n, n, Linv_all, d0, status, min_bits, st, plan);
    if (e != hipSuccess) return e;
    e = launch_chol_apply<T>(S, n, Linv_all, rhs, dx, work_y, flags, epoch, err, host_err, st, 0, cooperative, plan);
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((zero_on_status_kernel<T>), dim3((n + 255) / 256), dim3(256), 0, st, dx, n, status);
  return hipGetLastError();
}

template hipError_t launch_chol_solve<float>(float*, const float*, int, float*, float*, float*, const float*, int*,
                                             unsigned int*, int*, int, int*, int*, hipStream_t, bool,
                                             const PanelPlan*);
template hipError_t launch_chol_solve<double>(double*, const double*, int, double*, double*, double*, const double*,
                                              int*, unsigned int*, int*, int, int*, int*, hipStream_t, bool,
                                              const PanelPlan*);
template hipError_t launch_chol_factor<float>(float*, int, int, float*, const float*, int*, unsigned int*,
                                              hipStream_t, const PanelPlan*);
template hipError_t launch_chol_apply<float>(const float*, int, const float*, const float*, float*, float*, int*, int,
                                             int*, int*, hipStream_t, int, bool, const PanelPlan*, const int*);

}  // namespace dpvba
