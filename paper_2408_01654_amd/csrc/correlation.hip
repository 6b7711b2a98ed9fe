// Patch correlation of DPV-SLAM eq. 4 (Sec. 3.1, "Patch correlation"):
//   C(u, v, a, b) = < g(u, v), f(P'(u, v) + Delta_ab) >
// for every edge (i, k, j): g the p x p patch features of patch k, f the
// feature map of the edge's target frame sampled bilinearly (zero outside)
// at the reprojected patch pixel shifted by the 7 x 7 grid of offsets
// Delta_ab = (a - 3, b - 3).
//
// All 49 samples of one patch pixel share the fractional position of the
// reprojected point, so their four-pixel footprints cover one 8 x 8 window of
// the map: the kernel takes 64 dot products (window pixel . g) and combines
// them bilinearly, instead of 196 four-pixel samples.  One wavefront per
// (edge, patch pixel): lanes split the feature dimension (D / 64 channels
// each), every window pixel arrives as one contiguous D-vector load per
// wavefront, each lane keeps 64 partial dots, and a halving butterfly (63
// shuffles) leaves window pixel l's total on lane l; lane 8 b + a then reads
// its three neighbours and writes C(u, v, a, b).  The four wavefronts of a
// workgroup take consecutive patch pixels of one edge, which share most of
// their windows in the caches.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"
#include "layout.h"

namespace dpvba {

constexpr int kCorrR = 3;               // offsets -3 .. 3
constexpr int kCorrGrid = 2 * kCorrR + 1;

template <int VPL>  // channels per lane (D = 64 VPL)
__global__ void __launch_bounds__(256) patch_corr_kernel(int n_items, int p2, const float* __restrict__ gmap,
                                                         int n_patches, const float* __restrict__ fmaps, int n_maps,
                                                         int H, int W, const int* __restrict__ kk,
                                                         const int* __restrict__ jj, const float* __restrict__ coords,
                                                         float* __restrict__ corr, int* dev_err, int* host_err) {
  constexpr int D = 64 * VPL;
  const int lane = threadIdx.x & 63;
  const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (item >= n_items) return;  // whole wavefront
  const int e = item / p2, pix = item - (item / p2) * p2;
  const int k = kk[e], fj = jj[e];
  float* out = corr + (size_t)item * (kCorrGrid * kCorrGrid);
  if (k < 0 || k >= n_patches || fj < 0 || fj >= n_maps) {
    if (lane < kCorrGrid * kCorrGrid) out[lane] = 0.f;
    if (lane == 0) report_device_error(dev_err, host_err, kErrInput);
    return;
  }
  const float x = coords[2 * (size_t)item], y = coords[2 * (size_t)item + 1];
  const float xf = floorf(x), yf = floorf(y);
  const float fx = x - xf, fy = y - yf;
  // window of 8 x 8 map pixels starting at (floor(x) - 3, floor(y) - 3); points
  // far outside the map (or not finite) leave every window pixel outside
  const bool finite = fabsf(x) < 1e9f && fabsf(y) < 1e9f;
  const int wx0 = finite ? (int)xf - kCorrR : -(1 << 30), wy0 = finite ? (int)yf - kCorrR : -(1 << 30);
  float g[VPL];
  {
    const float* gp = gmap + ((size_t)k * p2 + pix) * D + lane * VPL;
#pragma unroll
    for (int m = 0; m < VPL; ++m) g[m] = gp[m];
  }
  const float* fm = fmaps + (size_t)fj * H * W * D + lane * VPL;
  float part[64];
#pragma unroll
  for (int w = 0; w < 64; ++w) {
    const int xx = wx0 + (w & 7), yy = wy0 + (w >> 3);
    float s = 0.f;
    if (xx >= 0 && xx < W && yy >= 0 && yy < H) {
      const float* fp = fm + ((size_t)yy * W + xx) * D;
#pragma unroll
      for (int m = 0; m < VPL; ++m) s += g[m] * fp[m];
    }
    part[w] = s;
  }
  // halving butterfly: after level s lane l holds the partial totals of the
  // window pixels whose top s index bits equal l's
#pragma unroll
  for (int h = 32; h >= 1; h >>= 1) {
    const bool hi = lane & h;
#pragma unroll
    for (int i = 0; i < h; ++i) {
      const float keep = hi ? part[h + i] : part[i];
      const float give = hi ? part[i] : part[h + i];
      part[i] = keep + __shfl_xor(give, h);
    }
  }
  const float d00 = part[0];
  const float d01 = __shfl(d00, (lane + 1) & 63);
  const float d10 = __shfl(d00, (lane + 8) & 63);
  const float d11 = __shfl(d00, (lane + 9) & 63);
  const int a = lane & 7, b = lane >> 3;  // window column (x offset), row (y offset)
  if (a < kCorrGrid && b < kCorrGrid) {
    const float c = (1.f - fx) * (1.f - fy) * d00 + fx * (1.f - fy) * d01 + (1.f - fx) * fy * d10 + fx * fy * d11;
    out[a * kCorrGrid + b] = c;
  }
}

hipError_t launch_patch_correlation(int n_edges, int p, int dim, const float* gmap, int n_patches, const float* fmaps,
                                    int n_maps, int H, int W, const int* kk, const int* jj, const float* coords,
                                    float* corr, int* dev_err, int* host_err, hipStream_t st) {
  const int p2 = p * p;
  const long long items = (long long)n_edges * p2;
  if (items == 0) return hipSuccess;
  const int grid = (int)((items + 3) / 4);
  switch (dim / 64) {
#define DPVBA_CORR_CASE(V)                                                                                         \
  case V:                                                                                                          \
    hipLaunchKernelGGL(patch_corr_kernel<V>, dim3(grid), dim3(256), 0, st, (int)items, p2, gmap, n_patches, fmaps, \
                       n_maps, H, W, kk, jj, coords, corr, dev_err, host_err);                                     \
    break;
    DPVBA_CORR_CASE(1)
    DPVBA_CORR_CASE(2)
    DPVBA_CORR_CASE(3)
    DPVBA_CORR_CASE(4)
#undef DPVBA_CORR_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace dpvba
