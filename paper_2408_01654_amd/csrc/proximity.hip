// Proximity loop-closure edges of the patch graph (DPV-SLAM Sec. 3.2,
// "Proximity Loop Closure" and "Constructing the Patch Graph"): loops are
// detected from the cameras' proximity to previously visited locations, and
// every patch of an old frame gets a uni-directional edge to each recent
// frame found near it (the correlation of eq. 4 needs only the destination
// frame's dense features).
//
// Rule (see include/dpvba.h, dpvba_proximity_edges): frame i may link to a
// recent frame j >= first_recent with j - i > min_gap whose camera centre is
// closer than the radius; it keeps its max_targets nearest ones (ties to the
// lower index), listed in increasing frame order.  The decisions are integer
// results of float comparisons: d2 = (dx*dx + dy*dy) + dz*dz is evaluated with
// explicitly rounded operations (no fused multiply-add), compared strictly
// with r2 = radius*radius rounded to float32.
//
// Three launches: selection (one wavefront per old frame, max_targets rounds
// of a wavefront minimum over the frame's candidates: no per-lane lists, no
// sort), an exclusive scan of the edge counts, and the edge writes.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dpvba {

constexpr int kMaxLoopTargets = 32;

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off);
    v = o < v ? o : v;
  }
  return v;
}

// Squared distance of two camera centres (the translations of
// camera-to-world poses [.,7]) with every operation rounded on its own.
__device__ __forceinline__ float centre_d2(const float* a, const float* b) {
  const float dx = __fsub_rn(b[0], a[0]), dy = __fsub_rn(b[1], a[1]), dz = __fsub_rn(b[2], a[2]);
  return __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
}

// Four wavefronts per workgroup, one old frame each.  Keys order the
// candidates by (d2, j): d2 >= 0, so its bit pattern orders like its value.
__global__ void __launch_bounds__(256) loop_select_kernel(const float* poses, int n, int first_recent, int min_gap,
                                                          float r2, int max_t, int* counts, int* targets) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;  // whole wavefront
  const float* ci = poses + 7 * (size_t)i;
  const int j0 = max(first_recent, i + min_gap + 1);
  unsigned long long last = 0ull;  // keys above the previous pick (none is 0: j0 >= 1)
  int cnt = 0, mine = -1;          // lane t keeps the t-th pick's frame
  for (int t = 0; t < max_t; ++t) {
    unsigned long long best = ~0ull;
    for (int j = j0 + lane; j < n; j += 64) {
      const float d2 = centre_d2(ci, poses + 7 * (size_t)j);
      if (!(d2 < r2)) continue;
      const unsigned long long key = ((unsigned long long)__float_as_uint(d2) << 32) | (unsigned int)j;
      if (key > last && key < best) best = key;
    }
    best = wave_min_u64(best);
    if (best == ~0ull) break;  // uniform
    if (lane == t) mine = (int)(best & 0xffffffffu);
    last = best;
    ++cnt;
  }
  // increasing frame order: the rank of each pick among the picks
  int rank = 0;
  for (int s = 0; s < cnt; ++s) {
    const int js = __shfl(mine, s);
    rank += (lane < cnt && js < mine) ? 1 : 0;
  }
  int* out = targets + (size_t)i * max_t;
  if (lane < cnt) out[rank] = mine;
  for (int t = cnt + lane; t < max_t; t += 64) out[t] = -1;
  if (lane == 0) counts[i] = cnt;
}

// Exclusive scan of counts[i] x patches of frame i into edge_off [n + 1]
// (one workgroup; each thread scans a contiguous chunk).
__global__ void __launch_bounds__(1024) loop_offsets_kernel(const int* counts, const int* patch_off, int n,
                                                            long long* edge_off) {
  __shared__ long long part[1024];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int chunk = (n + nt - 1) / nt;
  const int a = min(n, tid * chunk), b = min(n, a + chunk);
  long long s = 0;
  for (int f = a; f < b; ++f) s += (long long)counts[f] * (long long)max(0, patch_off[f + 1] - patch_off[f]);
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < nt; off <<= 1) {  // inclusive Hillis-Steele scan of the chunk sums
    const long long v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  long long run = tid ? part[tid - 1] : 0;
  for (int f = a; f < b; ++f) {
    edge_off[f] = run;
    run += (long long)counts[f] * (long long)max(0, patch_off[f + 1] - patch_off[f]);
  }
  if (tid == nt - 1) edge_off[n] = part[nt - 1];
}

// One workgroup per old frame: edges (i, patch, target) by patch, then target.
__global__ void __launch_bounds__(256) loop_emit_kernel(const int* counts, const int* targets, int max_t,
                                                        const int* patch_off, const long long* edge_off,
                                                        long long max_edges, int* ii, int* jj, int* kk) {
  const int i = blockIdx.x;
  const int cnt = counts[i];
  if (cnt == 0) return;
  const int p0 = patch_off[i], np = max(0, patch_off[i + 1] - p0);
  const long long e0 = edge_off[i];
  const int total = np * cnt;
  for (int x = threadIdx.x; x < total; x += blockDim.x) {
    const long long e = e0 + x;
    if (e >= max_edges) break;
    const int p = x / cnt, t = x - (x / cnt) * cnt;
    ii[e] = i;
    kk[e] = p0 + p;
    jj[e] = targets[(size_t)i * max_t + t];
  }
}

hipError_t launch_proximity_edges(const float* poses, int n, const int* patch_off, int first_recent, int min_gap,
                                  float r2, int max_t, int* counts, int* targets, long long* edge_off, int* ii,
                                  int* jj, int* kk, long long max_edges, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(loop_select_kernel, dim3((n + 3) / 4), dim3(256), 0, st, poses, n, first_recent, min_gap, r2,
                       max_t, counts, targets);
  hipLaunchKernelGGL(loop_offsets_kernel, dim3(1), dim3(1024), 0, st, counts, patch_off, n, edge_off);
  if (n > 0 && max_edges > 0)
    hipLaunchKernelGGL(loop_emit_kernel, dim3(n), dim3(256), 0, st, counts, targets, max_t, patch_off, edge_off,
                       max_edges, ii, jj, kk);
  return hipGetLastError();
}

}  // namespace dpvba
