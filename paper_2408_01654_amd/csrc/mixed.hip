// Mixed-precision solve of the reduced camera system (DPV-SLAM Appendix A:
// the Cholesky factorisation of the Schur complement's pose block, here in
// float32 on the matrix cores, with float64 iterative refinement).
//
// Given S64 (float64, both triangles) and s64 gathered from the float32 tile
// shares: factor S32 = fl32(S64) once, solve, then repeat
//   r = s64 - S64 x   (float64),   x += (L L^T)^-1 fl32(r)
// a fixed number of times.  The iteration is accepted when
// max |r| <= tol max |s64| after the last step; otherwise (or when the
// float32 factorisation met a non-positive pivot) the caller re-solves with
// a float64 Cholesky of S64.
#include "common.h"
#include "factor_plan.h"

namespace dpvba {

template <typename Ti, typename To>
__global__ void convert_kernel(const Ti* src, To* dst, long long n) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) dst[q] = (To)src[q];
}

// Lower triangle (row-major, full storage) of S64 into S32; with an
// envelope (fq, bw: row r starts at column bw fq[r / bw]) only the entries
// from the row's first column on (the caller keeps S32 zero before it).
__global__ void lower_to_f32_kernel(const double* S64, float* S32, int n, const int* fq, int bw) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long long)n * n) return;
  const int r = (int)(q / n), c = (int)(q - (long long)r * n);
  if (c <= r && (!fq || c >= bw * fq[r / bw])) S32[q] = (float)S64[q];
}

// r = s - S x, one wavefront per row, summed in a fixed order; the largest
// |r_i| and |s_i| are kept as ordered bits of non-negative doubles (integer
// maxima, independent of the order of the atomics).
// With an envelope (fq, bw, reach) a row's non-zero entries lie in columns
// [bw fq[row / bw], reach[row / 64]) of the symmetric S, and only those
// are read.
__global__ void __launch_bounds__(256) residual64_kernel(const double* S, const double* s, const double* x, int n,
                                                         double* r, unsigned long long* rmax,
                                                         unsigned long long* smax, const int* fq, int bw,
                                                         const int* reach) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const double* Sr = S + (size_t)row * n;
  const int c0 = fq ? bw * fq[row / bw] : 0, c1 = fq ? min(n, reach[row / 64]) : n;
  double v = 0.0;
  for (int c = c0 + lane; c < c1; c += 64) v += Sr[c] * x[c];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (lane == 0) {
    const double rv = s[row] - v;
    r[row] = rv;
    atomicMax(rmax, (unsigned long long)__double_as_longlong(fabs(rv)));
    atomicMax(smax, (unsigned long long)__double_as_longlong(fabs(s[row])));
  }
}

__global__ void clear_max_kernel(unsigned long long* m) {
  if (threadIdx.x < 2) m[threadIdx.x] = 0ull;
}

// x64 += c32 (nothing when *skip: that refinement step was not taken)
__global__ void accumulate_kernel(double* x, const float* c, int n, const int* skip) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n && !(skip && *skip)) x[q] += (double)c[q];
}

// *skip = the relative residual (largest |r_i| / largest |s_i|) already
// meets the tolerance: the remaining refinement steps are not taken.
__global__ void refine_check_kernel(const unsigned long long* m, double tol, int* skip) {
  if (threadIdx.x != 0) return;
  const double rmax = __longlong_as_double((long long)m[0]);
  const double smax = __longlong_as_double((long long)m[1]);
  *skip = (smax > 0.0 ? rmax / smax : rmax) <= tol;
}

// Accept or fall back; records the relative residual and the decision.
__global__ void refine_decide_kernel(const unsigned long long* m, const int* status32, double tol, int force,
                                     double* resid_out, int* fallback_out, int* host_flag) {
  if (threadIdx.x != 0) return;
  const double rmax = __longlong_as_double((long long)m[0]);
  const double smax = __longlong_as_double((long long)m[1]);
  const double rel = smax > 0.0 ? rmax / smax : rmax;
  const int fb = force || (*status32 != 0) || !(rel <= tol);
  *resid_out = rel;
  *fallback_out = fb;
  *host_flag = fb;
}

// Final step in the state precision.  The iteration's status becomes that of
// the solve actually used: the float32 one when accepted (then clean), else
// the float64 fallback's; a failed fallback leaves a zero step.
__global__ void step_to_f32_kernel(const double* x, float* dx, int n, const int* fallback, const int* status64,
                                   int* status) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int fb = *fallback;
  const int bad = fb && *status64;
  if (q < n) dx[q] = bad ? 0.f : (float)x[q];
  if (q == 0) *status = fb ? *status64 : 0;
}

static inline unsigned nblocks(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename Ti, typename To>
hipError_t launch_convert(const Ti* src, To* dst, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((convert_kernel<Ti, To>), dim3(nblocks(n, 256)), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_lower_to_f32(const double* S64, float* S32, int n, hipStream_t st, const PanelPlan* env) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(lower_to_f32_kernel, dim3(nblocks((long long)n * n, 256)), dim3(256), 0, st, S64, S32, n,
                     env ? env->fq_dev : (const int*)nullptr, env ? env->bw : 1);
  return hipGetLastError();
}

hipError_t launch_residual64(const double* S, const double* s, const double* x, int n, double* r,
                             unsigned long long* maxes, hipStream_t st, const PanelPlan* env) {
  hipLaunchKernelGGL(clear_max_kernel, dim3(1), dim3(64), 0, st, maxes);
  if (n > 0)
    hipLaunchKernelGGL(residual64_kernel, dim3(nblocks(n, 4)), dim3(256), 0, st, S, s, x, n, r, maxes, maxes + 1,
                       env ? env->fq_dev : (const int*)nullptr, env ? env->bw : 1,
                       env ? env->reach_dev : (const int*)nullptr);
  return hipGetLastError();
}

hipError_t launch_refine_check(const unsigned long long* maxes, double tol, int* skip, hipStream_t st) {
  hipLaunchKernelGGL(refine_check_kernel, dim3(1), dim3(64), 0, st, maxes, tol, skip);
  return hipGetLastError();
}

hipError_t launch_accumulate(double* x, const float* c, int n, hipStream_t st, const int* skip) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(accumulate_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, x, c, n, skip);
  return hipGetLastError();
}

hipError_t launch_refine_decide(const unsigned long long* maxes, const int* status32, double tol, int force,
                                double* resid_out, int* fallback_out, int* host_flag, hipStream_t st) {
  hipLaunchKernelGGL(refine_decide_kernel, dim3(1), dim3(64), 0, st, maxes, status32, tol, force, resid_out,
                     fallback_out, host_flag);
  return hipGetLastError();
}

hipError_t launch_step_to_f32(const double* x, float* dx, int n, const int* fallback, const int* status64,
                              int* status, hipStream_t st) {
  hipLaunchKernelGGL(step_to_f32_kernel, dim3(nblocks(n > 0 ? n : 1, 256)), dim3(256), 0, st, x, dx, n, fallback,
                     status64, status);
  return hipGetLastError();
}

template hipError_t launch_convert<double, float>(const double*, float*, long long, hipStream_t);
template hipError_t launch_convert<float, double>(const float*, double*, long long, hipStream_t);

}  // namespace dpvba
