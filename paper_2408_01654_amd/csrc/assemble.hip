// Per-tile assembly of the reduced camera system, its gather into the dense
// damped Schur complement, back-substitution of the depths and the SE(3)
// retraction of the free poses.
//
// Mathematics (DPV-SLAM eq. 2-3, Appendix A).  For an edge e = (i, k, j) with
// relative pose T_ji = (R, t), patch-centre ray x^ and inverse depth d:
//   q = R x^ + t d,  pi = (fx qx/qz + cx, fy qy/qz + cy),  r = pi - target,
//   J_d = Jpi t,  J_j = Jpi [ -d I | [q]x ],  J_i = -J_j Ad(T_ji).
// The last identity lets a tile reduce, per (source i, target j) pair, only
//   M_ij = sum J_j^T W J_j,  v_ij = sum J_j^T W r
// and recover the source-pose blocks as Ad^T M Ad, -Ad^T M, -Ad^T v.  Per
// patch, with E_j = J_j^T W J_d per edge and E_i = -sum Ad^T E_j,
//   C~ = (1 + lam) sum J_d^T W J_d + lam,   w = sum J_d^T W r,
// and the Schur term -E C~^-1 E^T is the product U^T U of the rows
// u_k = E_k / sqrt(C~_k).  Every reduction runs in a fixed order, so results
// are bitwise reproducible; no floating-point atomics are used.
#include "common.h"
#include "tileargs.h"
#include "../../include/dpvba.h"

namespace dpvba {


// Everything one edge contributes, from the slot's relative pose (R, t), the
// patch ray (xh0, xh1, 1), inverse depth d, target and weight.
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

template <typename T>
__device__ __forceinline__ T* lds_T() {
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  return reinterpret_cast<T*>(dyn_lds);
}

// Shared prologue: slot relative poses and patch rays into LDS.
template <typename T, typename P>
__device__ __forceinline__ void load_tile_geometry(const TileArgs<T, P>& A, const TileInfo& ti,
                                                   T* sSlot, T* sPatch) {
  const int tid = threadIdx.x;
  const int K = ti.n_patch, Tn = ti.n_slot;
  for (int s = tid; s < Tn; s += blockDim.x) {
    const int j = A.slot_frame[ti.slot_begin + s];
    T Ri[9], ti_[3], Rj[9], tj[3];
    const P* pi = A.poses + 7 * (size_t)ti.frame;
    const P* pj = A.poses + 7 * (size_t)j;
    quat_to_rot<T, P>(pi + 3, Ri);
    quat_to_rot<T, P>(pj + 3, Rj);
    for (int m = 0; m < 3; ++m) { ti_[m] = (T)pi[m]; tj[m] = (T)pj[m]; }
    relative_pose<T>(Ri, ti_, Rj, tj, sSlot + 18 * s, sSlot + 18 * s + 9);
  }
  const int p = A.p, c = (p - 1) / 2;
  for (int k = tid; k < K; k += blockDim.x) {
    const int pk = A.tile_patch[ti.patch_begin + k];
    const float* cen = A.patches + ((size_t)pk * p * p + (size_t)c * p + c) * 2;
    sPatch[4 * k + 0] = ((T)cen[0] - A.cx) / A.fx;
    sPatch[4 * k + 1] = ((T)cen[1] - A.cy) / A.fy;
    sPatch[4 * k + 2] = (T)A.inv_depth[pk];
    sPatch[4 * k + 3] = (T)0;
  }
}

__device__ __forceinline__ int tri_index(int r, int c) {  // r <= c < 6
  return r * 6 - (r * (r - 1)) / 2 + (c - r);
}

template <typename T>
__device__ __forceinline__ T sym6(const T* M21, int r, int c) {
  return r <= c ? M21[tri_index(r, c)] : M21[tri_index(c, r)];
}

template <typename T, typename P>
__global__ void __launch_bounds__(kTileThreads) tile_assemble_kernel(TileArgs<T, P> A) {
  const TileInfo ti = A.tiles[blockIdx.x];
  const int tid = threadIdx.x;
  const int K = ti.n_patch, Tn = ti.n_slot, nb = ti.n_blk;
  const int npairs = nb * (nb + 1) / 2;
  const TileLds L = tile_lds_plan(K, Tn, nb);
  T* base = lds_T<T>();
  T* sSlot = base + L.slot;
  T* sPatch = base + L.patch;
  T* sCell = base + L.cell;
  T* sWork = base + L.work;
  T* sM = base + L.m;
  unsigned char* tab = reinterpret_cast<unsigned char*>(base) + ((L.total_T * (int)sizeof(T) + 15) / 16) * 16;
  unsigned char* sPairA = tab + L.pair_a;
  unsigned char* sPairB = tab + L.pair_b;
  unsigned char* sBlkS0 = tab + L.blk_s0;
  unsigned char* sBlkS1 = tab + L.blk_s1;
  signed char* sSlotBlk = reinterpret_cast<signed char*>(tab + L.slot_blk);
  __shared__ int sInvalid;

  // ---- phase 0: geometry and index tables
  if (tid == 0) sInvalid = 0;
  load_tile_geometry<T, P>(A, ti, sSlot, sPatch);
  for (int a = tid; a < nb; a += blockDim.x) {
    for (int b = a; b < nb; ++b) {
      const int pi = upper_pair_index(a, b, nb);
      sPairA[pi] = (unsigned char)a;
      sPairB[pi] = (unsigned char)b;
    }
    sBlkS0[a] = 255; sBlkS1[a] = 0;
  }
  for (int s = tid; s < Tn; s += blockDim.x) sSlotBlk[s] = (signed char)A.slot_blk[ti.slot_begin + s];
  __syncthreads();
  if (tid == 0) {
    // slots of one frame are adjacent (sorted by frame): block -> slot range
    for (int s = 0; s < Tn; ++s) {
      const int b = sSlotBlk[s];
      if (b < 0) continue;
      if (sBlkS0[b] == 255) sBlkS0[b] = (unsigned char)s;
      sBlkS1[b] = (unsigned char)(s + 1);
    }
  }

  // ---- phase 1: edge grid; per-thread partial sums for one slot
  const int G = kTileThreads / Tn;
  const int g = tid / Tn, s = tid % Tn;
  T acc[kRedWidth];
#pragma unroll
  for (int m = 0; m < kRedWidth; ++m) acc[m] = (T)0;
  int n_invalid = 0;
  if (g < G) {
    const T* Rt = sSlot + 18 * s;
    for (int k = g; k < K; k += G) {
      T* cell = sCell + 8 * (k * Tn + s);
      const int e = A.edge_grid[ti.grid_begin + k * Tn + s];
      EdgeTerms<T> o;
      bool ok = false;
      if (e >= 0) {
        const float2 tg = reinterpret_cast<const float2*>(A.target)[e];
        const float2 wt = reinterpret_cast<const float2*>(A.weight)[e];
        ok = edge_eval<T>(Rt, sPatch[4 * k], sPatch[4 * k + 1], sPatch[4 * k + 2], A.fx, A.fy,
                          A.cx, A.cy, A.z_min, tg.x, tg.y, wt.x, wt.y, o);
        if (!ok) ++n_invalid;
      }
      if (!ok) {
#pragma unroll
        for (int m = 0; m < 8; ++m) cell[m] = (T)0;
        continue;
      }
      const T wr0 = o.w[0] * o.r[0], wr1 = o.w[1] * o.r[1];
      const T wd0 = o.w[0] * o.Jd[0], wd1 = o.w[1] * o.Jd[1];
      int idx = 0;
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        const T a0 = o.w[0] * o.Jj[0][r], a1 = o.w[1] * o.Jj[1][r];
#pragma unroll
        for (int c = r; c < 6; ++c) acc[idx++] += a0 * o.Jj[0][c] + a1 * o.Jj[1][c];
      }
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        acc[21 + r] += o.Jj[0][r] * wr0 + o.Jj[1][r] * wr1;
        cell[r] = o.Jj[0][r] * wd0 + o.Jj[1][r] * wd1;
      }
      acc[27] += (T)0.5 * (wr0 * o.r[0] + wr1 * o.r[1]);
      cell[6] = o.Jd[0] * wd0 + o.Jd[1] * wd1;
      cell[7] = o.Jd[0] * wr0 + o.Jd[1] * wr1;
    }
  }
  if (n_invalid) atomicAdd(&sInvalid, n_invalid);
#pragma unroll
  for (int m = 0; m < kRedWidth; ++m) sWork[tid * kRedWidth + m] = acc[m];
  __syncthreads();

  // ---- phase 2a: per-slot totals, groups summed in order
  for (int idx = tid; idx < Tn * kRedWidth; idx += blockDim.x) {
    const int ss = idx / kRedWidth, m = idx % kRedWidth;
    T v = (T)0;
    for (int gg = 0; gg < G; ++gg) v += sWork[(gg * Tn + ss) * kRedWidth + m];
    sM[ss * kRedWidth + m] = v;
  }
  __syncthreads();

  // ---- phase 2b: per patch depth terms and Schur rows u_k = E_k / sqrt(C~_k)
  T* sU = sWork;  // [K][6 nb]
  const int W6 = 6 * nb;
  for (int k = tid; k < K; k += blockDim.x) {
    T C = (T)0, w = (T)0;
    T Ei[6] = {0, 0, 0, 0, 0, 0};
    T* row = sU + k * W6;
    for (int m = 0; m < W6; ++m) row[m] = (T)0;
    for (int ss = 0; ss < Tn; ++ss) {
      const T* cell = sCell + 8 * (k * Tn + ss);
      C += cell[6];
      w += cell[7];
      T tmp[6];
      adjoint_transpose_apply<T>(sSlot + 18 * ss, sSlot + 18 * ss + 9, cell, tmp);
#pragma unroll
      for (int m = 0; m < 6; ++m) Ei[m] -= tmp[m];
    }
    const T Ct = C * ((T)1 + A.lambda) + A.lambda;
    const T is = (T)1 / dsqrt(Ct);
    for (int ss = 0; ss < Tn; ++ss) {
      const int b = sSlotBlk[ss];
      if (b < 0) continue;
      const T* cell = sCell + 8 * (k * Tn + ss);
#pragma unroll
      for (int m = 0; m < 6; ++m) row[6 * b + m] += cell[m] * is;
    }
    if (ti.src_blk >= 0) {
#pragma unroll
      for (int m = 0; m < 6; ++m) row[6 * ti.src_blk + m] = Ei[m] * is;
    }
    sPatch[4 * k + 3] = w * is;
  }
  __syncthreads();

  // ---- phase 2c: per-slot source-side blocks  Ad^T M, Ad^T M Ad, Ad^T v
  T* sB = sCell;  // [Tn][80]
  for (int ss = tid; ss < Tn; ss += blockDim.x) {
    const T* R = sSlot + 18 * ss;
    const T* t = R + 9;
    const T* M21 = sM + ss * kRedWidth;
    T* out = sB + 80 * ss;
    T col[6], res[6];
    for (int c = 0; c < 6; ++c) {  // column c of M -> column c of Ad^T M
      for (int r = 0; r < 6; ++r) col[r] = sym6<T>(M21, r, c);
      adjoint_transpose_apply<T>(R, t, col, res);
      for (int r = 0; r < 6; ++r) out[r * 6 + c] = res[r];
    }
    for (int r = 0; r < 6; ++r) {  // row r of (Ad^T M) Ad = (Ad^T (row r)^T)^T
      for (int c = 0; c < 6; ++c) col[c] = out[r * 6 + c];
      adjoint_transpose_apply<T>(R, t, col, res);
      for (int c = 0; c < 6; ++c) out[36 + r * 6 + c] = res[c];
    }
    adjoint_transpose_apply<T>(R, t, M21 + 21, out + 72);
  }
  __syncthreads();

  // ---- phase 3: partial reduced system of this tile (upper block pairs)
  T* outS = A.part_S + ti.part_begin;
  const int src = ti.src_blk;
  for (int idx = tid; idx < npairs * 36; idx += blockDim.x) {
    const int pr = idx / 36, rc = idx % 36, r = rc / 6, c = rc % 6;
    const int a = sPairA[pr], b = sPairB[pr];
    T v = (T)0;
    for (int k = 0; k < K; ++k) v -= sU[k * W6 + 6 * a + r] * sU[k * W6 + 6 * b + c];
    if (a == b) {
      if (a == src) {
        for (int ss = 0; ss < Tn; ++ss) v += sB[80 * ss + 36 + rc];
      } else {
        for (int ss = sBlkS0[a]; ss < sBlkS1[a]; ++ss) v += sym6<T>(sM + ss * kRedWidth, r, c);
      }
    } else if (a == src) {
      for (int ss = sBlkS0[b]; ss < sBlkS1[b]; ++ss) v -= sB[80 * ss + rc];
    } else if (b == src) {
      for (int ss = sBlkS0[a]; ss < sBlkS1[a]; ++ss) v -= sB[80 * ss + c * 6 + r];
    }
    outS[idx] = v;
  }
  T* outV = A.part_vec + ti.vec_begin;
  for (int idx = tid; idx < W6; idx += blockDim.x) {
    const int b = idx / 6, m = idx % 6;
    T vb = (T)0, db = (T)0;
    if (b == src) {
      for (int ss = 0; ss < Tn; ++ss) {
        vb -= sB[80 * ss + 72 + m];
        db += sB[80 * ss + 36 + m * 7];
      }
    } else {
      for (int ss = sBlkS0[b]; ss < sBlkS1[b]; ++ss) {
        vb += sM[ss * kRedWidth + 21 + m];
        db += sM[ss * kRedWidth + tri_index(m, m)];
      }
    }
    T rhs = -vb;
    for (int k = 0; k < K; ++k) rhs += sU[k * W6 + idx] * sPatch[4 * k + 3];
    outV[idx] = rhs;
    outV[W6 + idx] = db;
  }
  if (tid == 0) {
    double cst = 0.0;
    for (int ss = 0; ss < Tn; ++ss) cst += (double)sM[ss * kRedWidth + 27];
    A.part_cost[blockIdx.x] = cst;
    A.part_invalid[blockIdx.x] = sInvalid;
  }
}

// Depth back-substitution  dd_k = C~_k^-1 (-w_k - E_k^T dxi), recomputed from
// the edge stream at the same iterate.  With E_i = -sum Ad^T E_j,
//   E_k^T dxi = sum_j E_j . (dxi_j - Ad(T_ji) dxi_i).
template <typename T, typename P>
__global__ void __launch_bounds__(kTileThreads) tile_backsub_kernel(TileArgs<T, P> A) {
  const TileInfo ti = A.tiles[blockIdx.x];
  const int tid = threadIdx.x;
  const int K = ti.n_patch, Tn = ti.n_slot;
  const TileLds L = tile_lds_plan(K, Tn, ti.n_blk);
  T* base = lds_T<T>();
  T* sSlot = base + L.slot;   // [Tn][18]: R(9) t(3) delta(6)
  T* sPatch = base + L.patch;
  T* sCell = base + L.cell;   // [K][Tn][3]
  const bool skip = A.step_status && *A.step_status;

  load_tile_geometry<T, P>(A, ti, sSlot, sPatch);
  __syncthreads();
  for (int s = tid; s < Tn; s += blockDim.x) {
    const int j = A.slot_frame[ti.slot_begin + s];
    T xi_i[6] = {0, 0, 0, 0, 0, 0}, xi_j[6] = {0, 0, 0, 0, 0, 0}, adx[6];
    if (!skip) {
      if (ti.frame >= A.n_fixed)
        for (int m = 0; m < 6; ++m) xi_i[m] = A.dx[6 * (ti.frame - A.n_fixed) + m];
      if (j >= A.n_fixed)
        for (int m = 0; m < 6; ++m) xi_j[m] = A.dx[6 * (j - A.n_fixed) + m];
    }
    adjoint_apply<T>(sSlot + 18 * s, sSlot + 18 * s + 9, xi_i, adx);
    for (int m = 0; m < 6; ++m) sSlot[18 * s + 12 + m] = xi_j[m] - adx[m];
  }
  __syncthreads();

  const int G = kTileThreads / Tn;
  const int g = tid / Tn, s = tid % Tn;
  if (g < G) {
    const T* Rt = sSlot + 18 * s;
    for (int k = g; k < K; k += G) {
      T* cell = sCell + 3 * (k * Tn + s);
      const int e = A.edge_grid[ti.grid_begin + k * Tn + s];
      EdgeTerms<T> o;
      bool ok = false;
      if (e >= 0) {
        const float2 tg = reinterpret_cast<const float2*>(A.target)[e];
        const float2 wt = reinterpret_cast<const float2*>(A.weight)[e];
        ok = edge_eval<T>(Rt, sPatch[4 * k], sPatch[4 * k + 1], sPatch[4 * k + 2], A.fx, A.fy,
                          A.cx, A.cy, A.z_min, tg.x, tg.y, wt.x, wt.y, o);
      }
      if (!ok) { cell[0] = cell[1] = cell[2] = (T)0; continue; }
      const T wr0 = o.w[0] * o.r[0], wr1 = o.w[1] * o.r[1];
      const T wd0 = o.w[0] * o.Jd[0], wd1 = o.w[1] * o.Jd[1];
      T ed = (T)0;
#pragma unroll
      for (int r = 0; r < 6; ++r) ed += (o.Jj[0][r] * wd0 + o.Jj[1][r] * wd1) * Rt[12 + r];
      cell[0] = o.Jd[0] * wd0 + o.Jd[1] * wd1;
      cell[1] = o.Jd[0] * wr0 + o.Jd[1] * wr1;
      cell[2] = ed;
    }
  }
  __syncthreads();
  for (int k = tid; k < K; k += blockDim.x) {
    T C = (T)0, w = (T)0, ed = (T)0;
    for (int ss = 0; ss < Tn; ++ss) {
      const T* cell = sCell + 3 * (k * Tn + ss);
      C += cell[0]; w += cell[1]; ed += cell[2];
    }
    const T Ct = C * ((T)1 + A.lambda) + A.lambda;
    const int pk = A.tile_patch[ti.patch_begin + k];
    if (!skip) A.inv_depth[pk] = (P)(sPatch[4 * k + 2] + (-w - ed) / Ct);
  }
}

// Retraction G <- G Exp(dxi) of every free pose.
template <typename T, typename P>
__global__ void retract_kernel(P* poses, const T* dx, int n_fixed, int n_free, const int* step_status) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_free) return;
  if (step_status && *step_status) return;
  T xi[6];
  for (int m = 0; m < 6; ++m) xi[m] = dx[6 * a + m];
  retract_pose<T, P>(poses + 7 * (size_t)(n_fixed + a), xi);
}

// Gather of the per-tile vectors into the right-hand side s and Diag(B).
template <typename T>
__global__ void gather_vec_kernel(const T* part_vec, const int* off, const int2* src, int n, T* rhs,
                                  T* dB) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  const int P_ = x / 6, m = x % 6;
  T v = (T)0, d = (T)0;
  for (int q = off[P_]; q < off[P_ + 1]; ++q) {
    v += part_vec[src[q].x + m];
    d += part_vec[src[q].y + m];
  }
  rhs[x] = v;
  dB[x] = d;
}

// Gather of every lower 6x6 block (P >= Q) of the damped reduced system from
// the tile partials (zero where no tile contributes), with the Marquardt
// diagonal lam (Diag(B) + 1) added.  `mirror` also writes the upper triangle.
template <typename T>
__global__ void gather_S_kernel(const T* part_S, const int* off, const int* src, int n_free, T* S,
                                const T* dB, T lambda, int mirror, T* diag_out) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nblk = (long long)n_free * (n_free + 1) / 2;
  if (g >= nblk * 36) return;
  const int blk = (int)(g / 36), e = (int)(g % 36), r = e / 6, c = e % 6;
  int Pb = (int)((sqrt(8.0 * (double)blk + 1.0) - 1.0) * 0.5);
  while ((long long)Pb * (Pb + 1) / 2 > blk) --Pb;
  while ((long long)(Pb + 1) * (Pb + 2) / 2 <= blk) ++Pb;
  const int Qb = blk - Pb * (Pb + 1) / 2;
  if (Pb == Qb && r < c) return;
  T v = (T)0;
  const int lo = off[blk], hi = off[blk + 1];
  if (Pb == Qb) {
    for (int q = lo; q < hi; ++q) v += part_S[src[q] + r * 6 + c];
  } else {
    for (int q = lo; q < hi; ++q) v += part_S[src[q] + c * 6 + r];
  }
  const int n = 6 * n_free;
  const int row = 6 * Pb + r, col = 6 * Qb + c;
  if (row == col) {
    v += lambda * (dB[row] + (T)1);
    if (diag_out) diag_out[row] = v;
  }
  S[(size_t)row * n + col] = v;
  if (mirror && row != col) S[(size_t)col * n + row] = v;
}

// Cost of every edge at an iterate, summed per block in a fixed order.
template <typename T, typename P>
__global__ void __launch_bounds__(256) edge_cost_kernel(const P* poses, const P* inv_depth,
                                                         const float* patches, int p, const int* ii,
                                                         const int* jj, const int* kk,
                                                         const float* target, const float* weight,
                                                         int n_edges, T fx, T fy, T cx, T cy, T z_min,
                                                         double* part) {
  __shared__ double sred[256];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  double cst = 0.0;
  if (e < n_edges) {
    T Ri[9], Rj[9], ti_[3], tj[3], Rt[12];
    const P* pi = poses + 7 * (size_t)ii[e];
    const P* pj = poses + 7 * (size_t)jj[e];
    quat_to_rot<T, P>(pi + 3, Ri);
    quat_to_rot<T, P>(pj + 3, Rj);
    for (int m = 0; m < 3; ++m) { ti_[m] = (T)pi[m]; tj[m] = (T)pj[m]; }
    relative_pose<T>(Ri, ti_, Rj, tj, Rt, Rt + 9);
    const int k = kk[e], c = (p - 1) / 2;
    const float* cen = patches + ((size_t)k * p * p + (size_t)c * p + c) * 2;
    EdgeTerms<T> o;
    const float2 tg = reinterpret_cast<const float2*>(target)[e];
    const float2 wt = reinterpret_cast<const float2*>(weight)[e];
    if (edge_eval<T>(Rt, ((T)cen[0] - cx) / fx, ((T)cen[1] - cy) / fy, (T)inv_depth[k], fx, fy, cx,
                     cy, z_min, tg.x, tg.y, wt.x, wt.y, o))
      cst = 0.5 * ((double)o.w[0] * o.r[0] * o.r[0] + (double)o.w[1] * o.r[1] * o.r[1]);
  }
  sred[threadIdx.x] = cst;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sred[threadIdx.x] += sred[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sred[0];
}

// Reduce per-tile costs / invalid counts of one iteration into the report.
__global__ void report_reduce_kernel(const double* part_cost, const int* part_invalid, int n,
                                     double* cost_out, int* invalid_out) {
  __shared__ double sc[256];
  __shared__ int si[256];
  double c = 0.0;
  int v = 0;
  // fixed partition: thread t sums a contiguous range, then a fixed tree
  const int per = (n + 255) / 256;
  const int lo = threadIdx.x * per, hi = min(n, lo + per);
  for (int q = lo; q < hi; ++q) {
    c += part_cost[q];
    if (part_invalid) v += part_invalid[q];
  }
  sc[threadIdx.x] = c;
  si[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sc[threadIdx.x] += sc[threadIdx.x + w];
      si[threadIdx.x] += si[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *cost_out = sc[0];
    if (invalid_out) *invalid_out = si[0];
  }
}

// Reprojection of every pixel of every edge's patch (eq. 2).
template <typename T>
__global__ void reproject_kernel(const float* poses, const float* inv_depth, const float* patches,
                                 int p, const int* ii, const int* jj, const int* kk, int n_edges,
                                 T fx, T fy, T cx, T cy, T z_min, float* coords, uint8_t* valid) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_edges) return;
  T Ri[9], Rj[9], ti_[3], tj[3], R[9], t[3];
  const float* pi = poses + 7 * (size_t)ii[e];
  const float* pj = poses + 7 * (size_t)jj[e];
  quat_to_rot<T, float>(pi + 3, Ri);
  quat_to_rot<T, float>(pj + 3, Rj);
  for (int m = 0; m < 3; ++m) { ti_[m] = pi[m]; tj[m] = pj[m]; }
  relative_pose<T>(Ri, ti_, Rj, tj, R, t);
  const int k = kk[e];
  const T d = inv_depth[k];
  const float* pk = patches + (size_t)k * p * p * 2;
  float* out = coords + (size_t)e * p * p * 2;
  const int c = (p - 1) / 2;
  for (int px = 0; px < p * p; ++px) {
    const T x = ((T)pk[2 * px] - cx) / fx, y = ((T)pk[2 * px + 1] - cy) / fy;
    const T q0 = R[0] * x + R[1] * y + R[2] + t[0] * d;
    const T q1 = R[3] * x + R[4] * y + R[5] + t[1] * d;
    const T q2 = R[6] * x + R[7] * y + R[8] + t[2] * d;
    out[2 * px] = (float)(fx * q0 / q2 + cx);
    out[2 * px + 1] = (float)(fy * q1 / q2 + cy);
    if (valid && px == c * p + c) valid[e] = (d > (T)0 && q2 > z_min * d) ? 1 : 0;
  }
}


// Per-solve report state: step status words and pivot minima per iteration.
__global__ void report_init_kernel(int* status, unsigned int* min_bits, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    status[i] = 0;
    min_bits[i] = 0x7f7fffffu;  // bits of FLT_MAX
  }
}

__global__ void report_finalize_kernel(dpvba_report* rep, const int* status, const unsigned int* min_bits,
                                       int n_iters) {
  if (threadIdx.x != 0) return;
  int st = DPVBA_OK;
  for (int t = 0; t < n_iters; ++t) {
    if (status[t]) st = DPVBA_ENOTPD;
    rep->min_pivot[t] = (double)__uint_as_float(min_bits[t]);
  }
  rep->status = st;
  rep->n_iters = n_iters;
}

hipError_t launch_report_init(int* status, unsigned int* min_bits, int n, hipStream_t st) {
  hipLaunchKernelGGL(report_init_kernel, dim3((n + 63) / 64), dim3(64), 0, st, status, min_bits, n);
  return hipGetLastError();
}

hipError_t launch_report_finalize(dpvba_report* rep, const int* status, const unsigned int* min_bits,
                                  int n_iters, hipStream_t st) {
  hipLaunchKernelGGL(report_finalize_kernel, dim3(1), dim3(64), 0, st, rep, status, min_bits, n_iters);
  return hipGetLastError();
}

// ---------------------------------------------------------------- launchers

template <typename T, typename P>
hipError_t launch_tile_assemble(const TileArgs<T, P>& A, int n_tiles, int lds_bytes, hipStream_t st) {
  if (n_tiles == 0) return hipSuccess;
  {
    hipError_t e = opt_in_lds((const void*)tile_assemble_kernel<T, P>, lds_bytes);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((tile_assemble_kernel<T, P>), dim3(n_tiles), dim3(kTileThreads), lds_bytes, st, A);
  return hipGetLastError();
}

template <typename T, typename P>
hipError_t launch_tile_backsub(const TileArgs<T, P>& A, int n_tiles, int lds_bytes, hipStream_t st) {
  if (n_tiles == 0) return hipSuccess;
  {
    hipError_t e = opt_in_lds((const void*)tile_backsub_kernel<T, P>, lds_bytes);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((tile_backsub_kernel<T, P>), dim3(n_tiles), dim3(kTileThreads), lds_bytes, st, A);
  return hipGetLastError();
}

template <typename T, typename P>
hipError_t launch_retract(P* poses, const T* dx, int n_fixed, int n_free, const int* status, hipStream_t st) {
  if (n_free == 0) return hipSuccess;
  hipLaunchKernelGGL((retract_kernel<T, P>), dim3((n_free + 127) / 128), dim3(128), 0, st, poses, dx,
                     n_fixed, n_free, status);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather(const T* part_S, const T* part_vec, const int* s_off, const int* s_src,
                         const int* v_off, const int2* v_src, int n_free, T* S, T* rhs, T* dB, T lambda,
                         int mirror, T* diag_out, hipStream_t st) {
  if (n_free == 0) return hipSuccess;
  const int n = 6 * n_free;
  hipLaunchKernelGGL((gather_vec_kernel<T>), dim3((n + 255) / 256), dim3(256), 0, st, part_vec, v_off,
                     v_src, n, rhs, dB);
  const long long tot = (long long)n_free * (n_free + 1) / 2 * 36;
  hipLaunchKernelGGL((gather_S_kernel<T>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, part_S,
                     s_off, s_src, n_free, S, dB, lambda, mirror, diag_out);
  return hipGetLastError();
}

template <typename T, typename P>
hipError_t launch_edge_cost(const P* poses, const P* inv_depth, const float* patches, int p, const int* ii,
                            const int* jj, const int* kk, const float* target, const float* weight,
                            int n_edges, T fx, T fy, T cx, T cy, T z_min, double* part, hipStream_t st) {
  const int nblk = (n_edges + 255) / 256;
  if (nblk == 0) return hipSuccess;
  hipLaunchKernelGGL((edge_cost_kernel<T, P>), dim3(nblk), dim3(256), 0, st, poses, inv_depth, patches, p,
                     ii, jj, kk, target, weight, n_edges, fx, fy, cx, cy, z_min, part);
  return hipGetLastError();
}

hipError_t launch_report_reduce(const double* part_cost, const int* part_invalid, int n, double* cost_out,
                                int* invalid_out, hipStream_t st) {
  hipLaunchKernelGGL(report_reduce_kernel, dim3(1), dim3(256), 0, st, part_cost, part_invalid, n, cost_out,
                     invalid_out);
  return hipGetLastError();
}

hipError_t launch_reproject(const float* poses, const float* inv_depth, const float* patches, int p,
                            const int* ii, const int* jj, const int* kk, int n_edges, float fx, float fy,
                            float cx, float cy, float z_min, float* coords, uint8_t* valid, hipStream_t st) {
  if (n_edges == 0) return hipSuccess;
  hipLaunchKernelGGL((reproject_kernel<float>), dim3((n_edges + 255) / 256), dim3(256), 0, st, poses,
                     inv_depth, patches, p, ii, jj, kk, n_edges, fx, fy, cx, cy, z_min, coords, valid);
  return hipGetLastError();
}

#define DPVBA_INSTANTIATE(T, P)                                                                        \
  template hipError_t launch_tile_assemble<T, P>(const TileArgs<T, P>&, int, int, hipStream_t);        \
  template hipError_t launch_tile_backsub<T, P>(const TileArgs<T, P>&, int, int, hipStream_t);         \
  template hipError_t launch_retract<T, P>(P*, const T*, int, int, const int*, hipStream_t);           \
  template hipError_t launch_edge_cost<T, P>(const P*, const P*, const float*, int, const int*,        \
                                             const int*, const int*, const float*, const float*, int,  \
                                             T, T, T, T, T, double*, hipStream_t);

DPVBA_INSTANTIATE(float, float)
DPVBA_INSTANTIATE(double, double)
template hipError_t launch_gather<float>(const float*, const float*, const int*, const int*, const int*,
                                         const int2*, int, float*, float*, float*, float, int, float*,
                                         hipStream_t);
template hipError_t launch_gather<double>(const double*, const double*, const int*, const int*, const int*,
                                          const int2*, int, double*, double*, double*, double, int, double*,
                                          hipStream_t);

}  // namespace dpvba
