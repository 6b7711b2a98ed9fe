// One Gauss-Newton iteration over the tiles of a patch graph, and the
// single-launch solver of small problems.
//
// Each workgroup owns one tile (a run of one source frame's patches):
//  0. back-substitutes the previous iteration's depth step for its patches
//     from the stored Schur rows: dd_k = C~_k^-1 (-w_k - E_k^T dxi) =
//     -(w_k / sqrt(C~_k) + u_k . dxi) / sqrt(C~_k), and prefetches the
//     (target, weight) record of every (patch, slot) cell in one pass;
//  1. evaluates every edge: per (source, target) pair it accumulates
//     M = sum J_j^T W J_j and v = sum J_j^T W r in registers, and per edge it
//     leaves E_j = J_j^T W J_d, J_d^T W J_d and J_d^T W r in the edge's cell;
//  2. per patch: C~ = (1 + lam) C + lam, E_i = -sum_j Ad(T_ji)^T E_j and the
//     Schur row u_k = E_k / sqrt(C~_k), with w_k / sqrt(C~_k) appended;
//  3. forms U^T U on the matrix cores (16x16x4 tiles): its block part is the
//     Schur term E C~^-1 E^T and its appended column is E C~^-1 w; adds
//     B = sum J^T W J (the source-pose blocks from J_i = -J_j Ad(T_ji):
//     Ad^T M Ad, -Ad^T M, -Ad^T v) and writes the tile's share of
//     S = B~ - E C~^-1 E^T (upper entries of its block pairs),
//     s = -v + E C~^-1 w and Diag(B).
// All sums run in a fixed order, so results are reproducible bit for bit; no
// floating-point atomics are used.
#include <cfloat>

#include "edge.h"
#include "mfma.h"
#include "packed.h"
#include "tileargs.h"
#include "dpvba.h"

namespace dpvba {

// 16-byte vector of the compute type.
template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct Vec16<double> { typedef double type __attribute__((ext_vector_type(2))); };

// dots[k * ds] = [u_k | w_k / sqrt(C~_k)] . sX for the K stored Schur rows
// of one tile (row stride Ws, a multiple of 16).  With sX = [dxi | 1 | 0...]
// the depth step is dd_k = -dots[k] / sqrt(C~_k).  A wavefront takes eight
// rows at a time, lanes along the rows with 16-byte loads (all eight in
// flight), and sums the eight rows over its lanes together; sX lives in LDS.
template <typename T>
__device__ void schur_row_dots(const T* U, int K, int Ws, const T* sX, T* dots, int ds) {
  typedef typename Vec16<T>::type vec_t;
  constexpr int V = 16 / (int)sizeof(T);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
  const int nv = Ws / V;
  for (int k0 = 8 * wv; k0 < K; k0 += 8 * nwv) {
    T part[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) part[u] = (T)0;
    for (int c = lane; c < nv; c += 64) {
      vec_t x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (k0 + u < K) x[u] = reinterpret_cast<const vec_t*>(U + (size_t)(k0 + u) * Ws)[c];
        else x[u] = vec_t{};
      }
      const vec_t y = reinterpret_cast<const vec_t*>(sX)[c];
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int e = 0; e < V; ++e) part[u] += x[u][e] * y[e];
    }
    // halving butterfly: after it lane l holds the total of row
    // 4 b5 + 2 b4 + b3 (b = bits of l)
    T h4[4], h2[2];
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const T give = b5 ? part[j] : part[4 + j];
      h4[j] = (b5 ? part[4 + j] : part[j]) + __shfl_xor(give, 32);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const T give = b4 ? h4[j] : h4[2 + j];
      h2[j] = (b4 ? h4[2 + j] : h4[j]) + __shfl_xor(give, 16);
    }
    T h = (b3 ? h2[1] : h2[0]) + __shfl_xor(b3 ? h2[0] : h2[1], 8);
    h += __shfl_xor(h, 4);
    h += __shfl_xor(h, 2);
    h += __shfl_xor(h, 1);
    const int row = k0 + 4 * (b5 ? 1 : 0) + 2 * (b4 ? 1 : 0) + (b3 ? 1 : 0);
    if ((lane & 7) == 0 && row < K) dots[(size_t)row * ds] = h;
  }
}

// NT 16x16 tiles of U^T U that share the row tile: acc[t] = sum over the
// rows k of U[k][ua-tile]^T U[k][ub-tile + t] (16x16x4 steps, rows in
// groups of four).
template <typename T, int NT>
__device__ __forceinline__ void utu_unit(const T* ua, const T* ub, int nk, int Wp,
                                         typename Mfma<T>::acc_t* acc) {
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = typename Mfma<T>::acc_t{0, 0, 0, 0};
  // operands of step kq + 1 are loaded before the products of step kq
  T fa = ua[0], fb[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) fb[t] = ub[16 * t];
  for (int kq = 0; kq < nk; ++kq) {
    const int kn = min(kq + 1, nk - 1);  // the last step reloads its own operands
    const T na = ua[kn * 4 * Wp];
    T nb[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) nb[t] = ub[kn * 4 * Wp + 16 * t];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = Mfma<T>::step(fa, fb[t], acc[t]);
    fa = na;
#pragma unroll
    for (int t = 0; t < NT; ++t) fb[t] = nb[t];
  }
}

// Phases 0-3 for one tile; the caller synchronises before reusing `lds`.
// NT: the workgroup size.
template <typename T, int NT>
__device__ __forceinline__ void tile_assemble(const IterArgs<T>& A, int tile, unsigned char* lds) {
  const TileInfo ti = A.tiles[tile];
  const int tid = threadIdx.x;
  const int K = ti.n_patch, Tn = ti.n_slot, nb = ti.n_blk, W6 = 6 * nb;
  const TileLds L = tile_lds_plan(K, Tn, nb, (int)sizeof(T), NT);
  const int Kp = L.K_pad, Wp = L.W_pad;
  T* base = reinterpret_cast<T*>(lds);
  T* sSlot = base + L.slot;   // [Tn][18]: R_ji (9), t_ji (3)
  T* sPatch = base + L.patch; // [K][4]: x^0, x^1, d, w / sqrt(C~)
  double* sSlot64 = reinterpret_cast<double*>(base + L.hp);  // float32 plans: [Tn][12] R_ji, t_ji in float64
  double* sRay64 = sSlot64 + 12 * Tn;                         // float32 plans: [K][2] x^ in float64
  T* sPs = base + L.psum;     // [K][8]: C (then 1 / sqrt(C~)), w, -sum_j Ad^T E_j (phase 0: row dots)
  T* sM = base + L.m;         // [Tn][28]
  T* sU = base + L.u;         // [Kp][Wp]; first the per-thread partial sums
  T* sWork = sU;
  unsigned char* rec = lds + align16(L.total_T * (int)sizeof(T));
  const int cellT = L.cell_bytes / (int)sizeof(T);
  T* sCell = reinterpret_cast<T*>(rec);  // [K*Tn][cellT]
  T* sB = reinterpret_cast<T*>(rec);     // phase 2c: [Tn][kSlotBlk], then kSrcSums sums
  T* sDx = reinterpret_cast<T*>(rec);    // phase 0: [Wp] block step
  unsigned char* tab = rec + align16(L.rec_bytes);
  unsigned char* sBlkS0 = tab + L.blk_s0;  // first slot of each block (its slots are consecutive)
  unsigned char* sBlkS1 = tab + L.blk_s1;  // one past its last slot
  __shared__ int sInvalid;

  // ---- phase 0: block -> slot ranges, slot relative poses, previous depth step
  if (tid == 0) {
    sInvalid = 0;
    if (ti.src_blk >= 0) {  // the source pose is never a slot
      sBlkS0[ti.src_blk] = 0;
      sBlkS1[ti.src_blk] = 0;
    }
  }
  const int* slot_blk = A.slot_blk + ti.slot_begin;
  for (int s = tid; s < Tn; s += blockDim.x) {
    const int b = slot_blk[s];
    if (b >= 0) {  // slots follow the frame order, so a block's slots are consecutive
      if (s == 0 || slot_blk[s - 1] != b) sBlkS0[b] = (unsigned char)s;
      if (s == Tn - 1 || slot_blk[s + 1] != b) sBlkS1[b] = (unsigned char)(s + 1);
    }
    const int j = A.slot_frame[ti.slot_begin + s];
    T Ri[9], tiv[3], Rj[9], tj[3];
    const T* pi = A.poses_cur + 7 * (size_t)ti.frame;
    const T* pj = A.poses_cur + 7 * (size_t)j;
    quat_to_rot<T, T>(pi + 3, Ri);
    quat_to_rot<T, T>(pj + 3, Rj);
    for (int m = 0; m < 3; ++m) { tiv[m] = pi[m]; tj[m] = pj[m]; }
    relative_pose<T>(Ri, tiv, Rj, tj, sSlot + 18 * s, sSlot + 18 * s + 9);
    if constexpr (sizeof(T) == 4) {
      double Ri64[9], ti64[3], Rj64[9], tj64[3];
      quat_to_rot<double, T>(pi + 3, Ri64);
      quat_to_rot<double, T>(pj + 3, Rj64);
      for (int m = 0; m < 3; ++m) { ti64[m] = (double)pi[m]; tj64[m] = (double)pj[m]; }
      relative_pose<double>(Ri64, ti64, Rj64, tj64, sSlot64 + 12 * s, sSlot64 + 12 * s + 9);
    }
  }
  const bool apply_prev =
      !A.first && A.dx_prev && !(A.status_prev && A.status_prev[ti.inst * A.status_stride]);
  const int pb = ti.patch_begin;
  for (int k = tid; k < K; k += blockDim.x) {
    T x0, x1, d, is = (T)0;
    if (A.first) {
      const int pk = A.tile_patch[pb + k];
      const int c = (A.p - 1) / 2;
      const float* cen = A.patches + ((size_t)pk * A.p * A.p + (size_t)c * A.p + c) * 2;
      x0 = ((T)cen[0] - A.cx) / A.fx;
      x1 = ((T)cen[1] - A.cy) / A.fy;
      d = A.depth_in[pk];
      A.xh_s[2 * (pb + k)] = x0;
      A.xh_s[2 * (pb + k) + 1] = x1;
    } else {
      x0 = A.xh_s[2 * (pb + k)];
      x1 = A.xh_s[2 * (pb + k) + 1];
      d = A.depth_s[pb + k];
      if (apply_prev) is = A.pscale_s[2 * (pb + k)];
    }
    sPatch[4 * k] = x0;
    sPatch[4 * k + 1] = x1;
    sPatch[4 * k + 2] = d;
    sPatch[4 * k + 3] = is;
    if constexpr (sizeof(T) == 4) {  // the ray again in float64, from the centre pixel
      const int pk = A.tile_patch[pb + k];
      const int c = (A.p - 1) / 2;
      const float* cen = A.patches + ((size_t)pk * A.p * A.p + (size_t)c * A.p + c) * 2;
      sRay64[2 * k] = ((double)cen[0] - (double)A.cx) / (double)A.fx;
      sRay64[2 * k + 1] = ((double)cen[1] - (double)A.cy) / (double)A.fy;
    }
  }
  if (apply_prev)  // [dxi of the tile's blocks | 1 | 0 ...]
    for (int x = tid; x < Wp; x += blockDim.x)
      sDx[x] = x < W6 ? A.dx_prev[6 * A.blk_pose[ti.blk_begin + x / 6] + x % 6] : (x == W6 ? (T)1 : (T)0);
  __syncthreads();
  if (apply_prev) {
    schur_row_dots<T>(A.U_s + ti.u_begin, K, Wp, sDx, sPs, 8);
    __syncthreads();
  }
  for (int k = tid; k < K; k += blockDim.x) {
    T d = sPatch[4 * k + 2];
    if (apply_prev) {
      d -= sPs[8 * k] * sPatch[4 * k + 3];
      sPatch[4 * k + 2] = d;
    }
    if (A.first || apply_prev) A.depth_s[pb + k] = d;
    sPatch[4 * k + 3] = (T)0;
  }
  __syncthreads();
  // records: (target, weight) per cell and, after them, whether the cell
  // holds an edge (cells without one are marked by the edge id, never by
  // a value); batches of 8 cells per thread keep the index loads and the
  // dependent record loads in flight together.  A non-finite target or
  // weight, or a negative weight, is used as given and reported.
  {
    const int ncell = K * Tn;
    const int* grid = A.edge_grid + ti.grid_begin;
    const float2* tgt = reinterpret_cast<const float2*>(A.target);
    const float2* wgt = reinterpret_cast<const float2*>(A.weight);
    bool bad_in = false;
    for (int c0 = tid; c0 < ncell; c0 += 8 * NT) {
      int e[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = c0 + u * NT;
        e[u] = c < ncell ? grid[c] : -1;
      }
      float2 tg[8], wt[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        tg[u] = e[u] >= 0 ? tgt[e[u]] : make_float2(0.f, 0.f);
        wt[u] = e[u] >= 0 ? wgt[e[u]] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = c0 + u * NT;
        if (c < ncell) {
          unsigned char* cell = rec + (size_t)c * L.cell_bytes;
          *reinterpret_cast<float4*>(cell) = make_float4(tg[u].x, tg[u].y, wt[u].x, wt[u].y);
          *reinterpret_cast<int*>(cell + 16) = e[u] >= 0;
          bad_in |= e[u] >= 0 && !(wt[u].x >= 0.f && wt[u].y >= 0.f && wt[u].x <= FLT_MAX && wt[u].y <= FLT_MAX &&
                                   fabsf(tg[u].x) <= FLT_MAX && fabsf(tg[u].y) <= FLT_MAX);
        }
      }
    }
    if (bad_in) report_device_error(A.dev_err, A.host_err, kErrInput);
  }
  __syncthreads();

  // ---- phase 1: edges.  Thread (g, s) takes slot s of patches g, g + G, ...
  const int G = NT / Tn;
  const int g = tid / Tn, s = tid - (tid / Tn) * Tn;
  T acc[kRedWidth];
#pragma unroll
  for (int m = 0; m < kRedWidth; ++m) acc[m] = (T)0;
  int n_invalid = 0;
  if (g < G) {
    const T* Rt = sSlot + 18 * s;
    for (int k = g; k < K; k += G) {
      T* cell = sCell + (size_t)(k * Tn + s) * cellT;
      const float4 r4 = *reinterpret_cast<const float4*>(cell);
      const bool has = *reinterpret_cast<const int*>(reinterpret_cast<const unsigned char*>(cell) + 16) != 0;
      EdgeTerms<T> o;
      bool ok;
      if constexpr (sizeof(T) == 4)
        ok = has && edge_eval_r64(Rt, sSlot64 + 12 * s, sRay64[2 * k], sRay64[2 * k + 1], sPatch[4 * k + 2], A.fx,
                                  A.fy, A.cx, A.cy, A.z_min, r4.x, r4.y, r4.z, r4.w, o);
      else
        ok = has && edge_eval<T>(Rt, sPatch[4 * k], sPatch[4 * k + 1], sPatch[4 * k + 2], A.fx, A.fy, A.cx, A.cy,
                                 A.z_min, r4.x, r4.y, r4.z, r4.w, o);
      if (has && !ok) ++n_invalid;
      T out[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (ok) {
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
          out[r] = o.Jj[0][r] * wd0 + o.Jj[1][r] * wd1;
        }
        acc[27] += (T)0.5 * (wr0 * o.r[0] + wr1 * o.r[1]);
        out[6] = o.Jd[0] * wd0 + o.Jd[1] * wd1;
        out[7] = o.Jd[0] * wr0 + o.Jd[1] * wr1;
      }
#pragma unroll
      for (int m = 0; m < 8; ++m) cell[m] = out[m];
    }
  }
  if (n_invalid) atomicAdd(&sInvalid, n_invalid);
  // per-slot partials within each wavefront: lanes l, l + Tn, l + 2 Tn, ...
  // hold the same slot, so a tree over offsets Tn, 2 Tn, 4 Tn leaves the
  // wavefront's total of each slot on its first Tn lanes (partners past the
  // last thread group, or past the wavefront, add nothing)
  {
    const int lane = tid & 63, wv = tid >> 6;
    const int valid_lanes = min(64, G * Tn - 64 * wv);  // lanes of this wavefront holding a thread group
    for (int off = Tn; off < 64; off <<= 1) {
      const bool take = lane + off < valid_lanes;
#pragma unroll
      for (int m = 0; m < kRedWidth; ++m) {
        const T o = __shfl(acc[m], min(lane + off, 63));
        acc[m] += take ? o : (T)0;
      }
    }
    if (lane < Tn && lane < valid_lanes) {
      const int ss = (64 * wv + lane) % Tn;
#pragma unroll
      for (int m = 0; m < kRedWidth; ++m) sWork[(wv * Tn + ss) * kRedWidth + m] = acc[m];
    }
  }
  __syncthreads();

  // ---- phase 2a: per-slot totals, the wavefronts' partials summed in order
  {
    const int nwv = (G * Tn + 63) / 64;  // wavefronts holding thread groups
    for (int idx = tid; idx < Tn * kRedWidth; idx += blockDim.x) {
      const int ss = idx / kRedWidth, m = idx % kRedWidth;
      T v = (T)0;
      for (int w = 0; w < nwv; ++w) {
        // slot ss appears among the first Tn lanes of wavefront w unless the
        // wavefront holds fewer lanes than that
        const int first = (ss - (64 * w) % Tn + Tn) % Tn;  // its first lane in wavefront w
        if (first < min(64, G * Tn - 64 * w)) v += sWork[(w * Tn + ss) * kRedWidth + m];
      }
      sM[ss * kRedWidth + m] = v;
    }
  }
  __syncthreads();

  // ---- phase 2b: Schur rows u_k = E_k / sqrt(C~_k), appended w_k / sqrt(C~_k).
  // (i) two threads per patch k sum (C, w, -sum_j Ad(T_ji)^T E_j) over its
  //     slots in slot order, one the rotation part (with C and w), the other
  //     the translation part; (ii) C~, 1 / sqrt(C~) and w / sqrt(C~).
  const int src = ti.src_blk;
  for (int idx = tid; idx < 2 * K; idx += blockDim.x) {
    const int k = idx >> 1;
    const bool tpart = idx & 1;  // 0: C, w and the rotation part; 1: the translation part
    T v[5] = {0, 0, 0, 0, 0};
    for (int ss = 0; ss < Tn; ++ss) {
      const T* cell = sCell + (size_t)(k * Tn + ss) * cellT;
      const T* R = sSlot + 18 * ss;
      const T* tt = R + 9;
      T c[8];
      if (!tpart) {
#pragma unroll
        for (int m = 0; m < 3; ++m) c[m] = cell[m];
        c[6] = cell[6];
        c[7] = cell[7];
        v[0] += c[6];
        v[1] += c[7];
#pragma unroll
        for (int q = 0; q < 3; ++q) v[2 + q] -= R[q] * c[0] + R[3 + q] * c[1] + R[6 + q] * c[2];
      } else {
#pragma unroll
        for (int m = 0; m < 6; ++m) c[m] = cell[m];
        const T b0 = c[3] - (tt[1] * c[2] - tt[2] * c[1]);
        const T b1 = c[4] - (tt[2] * c[0] - tt[0] * c[2]);
        const T b2 = c[5] - (tt[0] * c[1] - tt[1] * c[0]);
#pragma unroll
        for (int q = 0; q < 3; ++q) v[q] -= R[q] * b0 + R[3 + q] * b1 + R[6 + q] * b2;
      }
    }
    if (!tpart) {
#pragma unroll
      for (int m = 0; m < 5; ++m) sPs[8 * k + m] = v[m];
    } else {
#pragma unroll
      for (int m = 0; m < 3; ++m) sPs[8 * k + 5 + m] = v[m];
    }
  }
  __syncthreads();
  for (int k = tid; k < K; k += blockDim.x) {
    const T Ct = sPs[8 * k] * ((T)1 + A.lam_diag) + A.lambda;
    const T is = (T)1 / dsqrt(Ct);
    const T rs = sPs[8 * k + 1] * is;
    sPs[8 * k] = is;
    sPatch[4 * k + 3] = rs;
    A.pscale_s[2 * (pb + k)] = is;
    A.pscale_s[2 * (pb + k) + 1] = rs;
  }
  __syncthreads();
  // (iii) row k, block column b (6 entries; b == nb: the appended column
  //       and the padding), zero rows beyond K
  const int nbx = nb + 1;
  for (int idx = tid; idx < Kp * nbx; idx += blockDim.x) {
    const int k = idx / nbx, b = idx - k * nbx;
    T* urow = sU + k * Wp;
    if (b == nb) {
      const T rs = k < K ? sPatch[4 * k + 3] : (T)0;
      for (int x = W6; x < Wp; ++x) urow[x] = x == W6 ? rs : (T)0;
      continue;
    }
    T v[6] = {0, 0, 0, 0, 0, 0};
    if (k < K) {
      const T is = sPs[8 * k];
      if (b == src) {
#pragma unroll
        for (int m = 0; m < 6; ++m) v[m] = sPs[8 * k + 2 + m] * is;
      } else {
        for (int ss = sBlkS0[b]; ss < sBlkS1[b]; ++ss) {
          const T* cell = sCell + (size_t)(k * Tn + ss) * cellT;
#pragma unroll
          for (int m = 0; m < 6; ++m) v[m] += cell[m];
        }
#pragma unroll
        for (int m = 0; m < 6; ++m) v[m] *= is;
      }
    }
#pragma unroll
    for (int m = 0; m < 6; ++m) urow[6 * b + m] = v[m];
  }
  __syncthreads();

  // ---- phase 2c: stored rows (the padded matrix as 16-byte vectors); per-slot
  // source blocks Ad^T M, Ad^T M Ad and Ad^T v, then their sums over the
  // slots in slot order
  {
    typedef typename Vec16<T>::type vec_t;
    const int nvec = Kp * Wp * (int)sizeof(T) / 16;
    const vec_t* from = reinterpret_cast<const vec_t*>(sU);
    vec_t* to = reinterpret_cast<vec_t*>(A.U_s + ti.u_begin);
    for (int x = tid; x < nvec; x += blockDim.x) to[x] = from[x];
  }
  for (int idx = tid; idx < Tn * 7; idx += blockDim.x) {  // column c of Ad^T M (c = 6: Ad^T v)
    const int ss = idx / 7, c = idx - ss * 7;
    const T* R = sSlot + 18 * ss;
    const T* t = R + 9;
    const T* M21 = sM + ss * kRedWidth;
    T* out = sB + kSlotBlk * ss;
    if (c == 6) {
      adjoint_transpose_apply<T>(R, t, M21 + 21, out + 72);
    } else {
      T col[6], res[6];
#pragma unroll
      for (int r = 0; r < 6; ++r) col[r] = sym6<T>(M21, r, c);
      adjoint_transpose_apply<T>(R, t, col, res);
#pragma unroll
      for (int r = 0; r < 6; ++r) out[r * 6 + c] = res[r];
    }
  }
  __syncthreads();
  for (int idx = tid; idx < Tn * 6; idx += blockDim.x) {  // row r of (Ad^T M) Ad
    const int ss = idx / 6, r = idx - ss * 6;
    const T* R = sSlot + 18 * ss;
    const T* t = R + 9;
    T* out = sB + kSlotBlk * ss;
    T col[6], res[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) col[c] = out[r * 6 + c];
    adjoint_transpose_apply<T>(R, t, col, res);
#pragma unroll
    for (int c = 0; c < 6; ++c) out[36 + r * 6 + c] = res[c];
  }
  __syncthreads();
  T* sSrc = sB + kSlotBlk * Tn;  // sum of Ad^T M Ad (36), of Ad^T v (6), Diag of Ad^T M Ad (6)
  for (int i = tid; i < kSrcSums; i += blockDim.x) {
    const int off = i < 36 ? 36 + i : (i < 42 ? 72 + (i - 36) : 36 + 7 * (i - 42));
    T v = (T)0;
    for (int ss = 0; ss < Tn; ++ss) v += sB[kSlotBlk * ss + off];
    sSrc[i] = v;
  }
  __syncthreads();
  // B-term table: what phase 3 adds to -U^T U.  Diagonal block of a (the
  // source: sum of Ad^T M Ad; a target: sum of its slots' M), source-row
  // block (src, b) = -sum of b's slots' Ad^T M, then per row x the
  // right-hand-side term (-v_x; the source: +sum Ad^T v) and Diag(B)_x.
  T* sBt = sSrc + kSrcSums;
  T* sDg = sBt;             // [nb][36]
  T* sSr = sBt + 36 * nb;   // [nb][36]
  T* sRv = sBt + 72 * nb;   // [6 nb]
  T* sDv = sRv + W6;        // [6 nb]
  T* sZero = sDv + W6;      // one zero (pairs without a B term)
  for (int i = tid; i < 72 * nb + 1; i += blockDim.x) {
    if (i == 72 * nb) {
      *sZero = (T)0;
      continue;
    }
    const int blk = i / 36, rc = i - blk * 36, which = blk / nb, a = blk - which * nb;
    const int r = rc / 6, c = rc - r * 6;
    T v = (T)0;
    if (which == 0) {
      if (a == src) v = sSrc[rc];
      else
        for (int ss = sBlkS0[a]; ss < sBlkS1[a]; ++ss) v += sym6<T>(sM + ss * kRedWidth, r, c);
    } else if (a != src) {
      for (int ss = sBlkS0[a]; ss < sBlkS1[a]; ++ss) v -= sB[kSlotBlk * ss + rc];
    }
    sBt[i] = v;
  }
  for (int x = tid; x < W6; x += blockDim.x) {
    const int a = x / 6, r = x - a * 6;
    T rv = (T)0, dv = (T)0;
    if (a == src) {
      rv = sSrc[36 + r];
      dv = sSrc[42 + r];
    } else {
      for (int ss = sBlkS0[a]; ss < sBlkS1[a]; ++ss) {
        rv -= sM[ss * kRedWidth + 21 + r];
        dv += sM[ss * kRedWidth + tri_index(r, r)];
      }
    }
    sRv[x] = rv;
    sDv[x] = dv;
  }
  __syncthreads();

  // ---- phase 3: U^T U on the matrix cores, plus B; upper entries only.
  // A work unit is row tile ta against up to four column tiles tb0 ..: the
  // row operand is loaded once per step and the four accumulators are
  // independent, so the loads of one step overlap the products of another.
  T* outS = A.part_S + ti.part_begin;
  T* outV = A.part_vec + ti.vec_begin;
  const int T16 = Wp / 16;
  const int nk = Kp / 4;
  const int lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: scalar unit loop
  for (int unit = wv;; unit += NT / 64) {
    int ta = 0, rem = unit;
    while (ta < T16 && rem >= (T16 - ta + 3) / 4) {
      rem -= (T16 - ta + 3) / 4;
      ++ta;
    }
    if (ta >= T16) break;
    const int tb0 = ta + 4 * rem, nt = min(4, T16 - tb0);
    typename Mfma<T>::acc_t acc[4];
    const T* ua = sU + (lane >> 4) * Wp + ta * 16 + (lane & 15);
    const T* ub = sU + (lane >> 4) * Wp + tb0 * 16 + (lane & 15);
    switch (nt) {
      case 1: utu_unit<T, 1>(ua, ub, nk, Wp, acc); break;
      case 2: utu_unit<T, 2>(ua, ub, nk, Wp, acc); break;
      case 3: utu_unit<T, 3>(ua, ub, nk, Wp, acc); break;
      default: utu_unit<T, 4>(ua, ub, nk, Wp, acc); break;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t >= nt) continue;
      const int tb = tb0 + t;
      const typename Mfma<T>::acc_t accv = acc[t];
      // addresses of the four values' B terms first (no branches), so the
      // LDS reads issue together
      const T* t1[4];
      const T* t2[4];
      bool ok[4], rhs[4];
      int dst[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = ta * 16 + Mfma<T>::row(lane, v), col = tb * 16 + (lane & 15);
        ok[v] = row <= col && row < W6 && col <= W6;
        rhs[v] = col == W6;  // right-hand side and Diag(B) of row `row`
        const int a = min(row, W6 - 1) / 6, r = min(row, W6 - 1) - 6 * (min(row, W6 - 1) / 6);
        const int b = min(col, W6 - 1) / 6, c = min(col, W6 - 1) - 6 * (min(col, W6 - 1) / 6);
        const int rc = r * 6 + c;
        const T* term = a == b ? sDg + 36 * a + rc
                               : (a == src ? sSr + 36 * b + rc : (b == src ? sSr + 36 * a + c * 6 + r : sZero));
        t1[v] = !ok[v] ? sZero : (rhs[v] ? sRv + row : term);
        t2[v] = ok[v] && rhs[v] ? sDv + row : sZero;
        dst[v] = rhs[v] ? row : upper_pair_index(a, b, nb) * 36 + rc;
      }
      T x1[4], x2[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        x1[v] = *t1[v];
        x2[v] = *t2[v];
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (!ok[v]) continue;
        if (rhs[v]) {
          outV[dst[v]] = accv[v] + x1[v];
          outV[W6 + dst[v]] = x2[v];
        } else {
          outS[dst[v]] = x1[v] - accv[v];
        }
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    double cst = 0.0;
    for (int ss = 0; ss < Tn; ++ss) cst += (double)sM[ss * kRedWidth + 27];
    A.part_cost[tile] = cst;
    A.part_invalid[tile] = sInvalid;
  }
}

template <typename T>
__global__ void __launch_bounds__(tile_threads(sizeof(T))) tile_iterate_kernel(IterArgs<T> A) {
  extern __shared__ __align__(16) unsigned char lds[];
  tile_assemble<T, tile_threads(sizeof(T))>(A, A.order ? A.order[blockIdx.x] : (int)blockIdx.x, lds);
}

// Damped reduced system of a small problem (packed lower triangle, row i at
// i (i + 1) / 2), summed from the tiles' shares in tile order.  One
// wavefront per lower 6x6 block (P >= Q): the block's share offsets are
// loaded once and broadcast, so every share load of a lane is independent.
// Diagonal entries get lam (Diag(B) + 1) and are kept in d0; the diagonal
// blocks also produce s.
template <typename T>
__device__ __forceinline__ void gather_slice(const IterArgs<T>& A, T* Sp, T* rhs, T* d0, int wave, int nwaves) {
  const int nf = A.n_free;
  const int lane = threadIdx.x & 63;
  const int r = lane / 6, c = lane - (lane / 6) * 6;
  const int nlb = nf * (nf + 1) / 2;
  for (int blk = wave; blk < nlb; blk += nwaves) {
    int P, Q;
    lower_block_of(blk, P, Q);
    const int lo = A.s_off[blk], hi = A.s_off[blk + 1];
    const bool lower = lane < 36 && (P > Q || r >= c);
    const int eo = c * 6 + r;  // the shares hold upper entries: (r, c) of S_PQ is [c][r] of a share
    T v = (T)0;
    for (int b0 = lo; b0 < hi; b0 += 64) {
      const int o_l = b0 + lane < hi ? A.s_src[b0 + lane] : 0;
      const int nq = min(64, hi - b0);
      for (int q0 = 0; q0 < nq; q0 += 8) {  // 8 independent loads in flight, summed in order
        T part[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int o = __shfl(o_l, (q0 + u) & 63);
          part[u] = (lower && q0 + u < nq) ? A.part_S[o + eo] : (T)0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) v += part[u];
      }
    }
    const int row = 6 * P + r, col = 6 * Q + c;
    if (P == Q) {
      // Diag(B) (lanes on the diagonal) and s (lanes 36..41) of pose P
      const int m = lane < 36 ? r : lane - 36;
      const bool want_d = lane < 36 && r == c, want_s = lane >= 36 && lane < 42;
      const int vlo = A.v_off[P], vhi = A.v_off[P + 1];
      T db = (T)0, sv = (T)0;
      for (int b0 = vlo; b0 < vhi; b0 += 64) {
        const int2 o_l = b0 + lane < vhi ? A.v_src[b0 + lane] : make_int2(0, 0);
        const int nq = min(64, vhi - b0);
        for (int q0 = 0; q0 < nq; q0 += 8) {
          T pd[8], ps[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int ox = __shfl(o_l.x, (q0 + u) & 63), oy = __shfl(o_l.y, (q0 + u) & 63);
            const bool in = q0 + u < nq;
            pd[u] = (want_d && in) ? A.part_vec[oy + m] : (T)0;
            ps[u] = (want_s && in) ? A.part_vec[ox + m] : (T)0;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            db += pd[u];
            sv += ps[u];
          }
        }
      }
      if (want_s) rhs[6 * P + m] = sv;
      if (want_d) {
        v += A.lam_diag * db + A.lambda;
        d0[row] = v;
      }
    }
    if (lower) Sp[row * (row + 1) / 2 + col] = v;
  }
}

// Factor and solve the gathered system in workgroup 0 and retract the free
// poses (panel_chol_solve: matrix in registers, 16-column panels factored by
// one wavefront, two barriers per panel; n + 1 <= 96).  A non-positive
// pivot discards the step (dxi = 0, *A.status = 1).
template <typename T>
__device__ __forceinline__ void factor_solve_retract(const IterArgs<T>& A, const T* Sp_g, const T* rhs_g,
                                                     const T* d0_g, unsigned char* lds) {
  const int tid = threadIdx.x;
  const int n = 6 * A.n_free;
  __shared__ int bad;
  __shared__ float minr;
  const int nr = small_solve_rows(n);
  T* x = reinterpret_cast<T*>(lds) + 37 * nr + nr * nr;  // after the solver's own arrays
  // The tiles' costs and invalid-edge counts of this iteration: loaded in
  // parallel before the factor (their latency overlaps it), summed in tile
  // order after it.  At most 256 are staged; any beyond are read in order.
  const int n_cost = A.cost_out ? A.n_tiles : 0;
  const int n_stage = n_cost < 256 ? n_cost : 256;
  double pcost = 0.0;
  int pinv = 0;
  if (tid < n_stage) {
    pcost = A.part_cost[tid];
    pinv = A.part_invalid[tid];
  }
  if (nr == 32) panel_chol_solve<T, 2>(n, Sp_g, rhs_g, d0_g, lds, x, &bad, &minr);
  else if (nr == 64) panel_chol_solve<T, 4>(n, Sp_g, rhs_g, d0_g, lds, x, &bad, &minr);
  else if (nr == 80) panel_chol_solve<T, 5>(n, Sp_g, rhs_g, d0_g, lds, x, &bad, &minr);
  else panel_chol_solve<T, 6>(n, Sp_g, rhs_g, d0_g, lds, x, &bad, &minr);
  // the published-panel area (2 x 32 x 17 values or more) is free after the factor
  double* cost_s = reinterpret_cast<double*>(lds);
  int* inv_s = reinterpret_cast<int*>(cost_s + 256);
  if (tid < n_stage) {
    cost_s[tid] = pcost;
    inv_s[tid] = pinv;
  }
  __syncthreads();
  for (int i = tid; i < n; i += blockDim.x) A.dx[i] = x[i];
  for (int i = tid; i < A.n_frames; i += blockDim.x) {
    const T* pc = A.poses_cur + 7 * (size_t)i;
    T* pn = A.poses_next + 7 * (size_t)i;
    for (int m = 0; m < 7; ++m) pn[m] = pc[m];
    if (i >= A.n_fixed && !bad) retract_pose<T, T>(pn, x + 6 * (i - A.n_fixed));
  }
  if (tid == 0) {
    *A.status = bad;
    *A.min_bits = __float_as_uint(minr >= 0.f ? minr : 0.f);
    if (A.cost_out) {
      double cc = 0.0;
      int inv = 0;
      for (int t = 0; t < n_stage; ++t) {
        cc += cost_s[t];
        inv += inv_s[t];
      }
      for (int t = n_stage; t < n_cost; ++t) {
        cc += A.part_cost[t];
        inv += A.part_invalid[t];
      }
      *A.cost_out = cc;
      if (A.invalid_out) *A.invalid_out = inv;
    }
  }
  __syncthreads();
}

// Grid-wide barrier of the single-launch solver: bar[0] counts arrivals,
// bar[1] is the generation.  Every wait is bounded; on timeout the failure
// is recorded and false returned, so no workgroup can spin forever.  A
// launch uses one of two slots and clears the other for the next launch on
// the stream, so arrivals left behind by a launch whose wait expired never
// reach a later launch's barriers.
constexpr long long kSpinLimit = 1LL << 19;  // polls of ~1000 cycles each: a timeout after ~0.2 s

__device__ bool grid_sync(unsigned int* bar, unsigned int nblocks, int* err, int* host_err) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    ok = 1;
    __threadfence();
    const unsigned int gen = __hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned int arrived = atomicAdd(&bar[0], 1u);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      long long spins = 0;
      while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(16);  // few polls of the shared word while workgroup 0 factors
        if (++spins > kSpinLimit) {
          ok = 0;
          report_device_error(err, host_err, kErrBarrier);
          break;
        }
      }
    }
    __threadfence();
  }
  __syncthreads();
  return ok;
}

// Depth write-back of one tile after the last iteration: apply its step
// dd_k = -(w_k / sqrt(C~_k) + u_k . dxi) / sqrt(C~_k) and scatter to the
// caller's array.  lds holds tile_u_stride(n_blk) + n_patch entries.
template <typename T>
__device__ void tile_writeback(const TileInfo& ti, const int* tile_patch, const int* blk_pose, const T* U_s,
                               const T* pscale_s, const T* depth_s, const T* dx, bool apply, T* depth_out,
                               T* lds) {
  const int W6 = 6 * ti.n_blk, Ws = tile_u_stride(ti.n_blk);
  T* sX = lds;
  T* sDot = lds + Ws;
  if (apply) {
    for (int x = threadIdx.x; x < Ws; x += blockDim.x)
      sX[x] = x < W6 ? dx[6 * blk_pose[ti.blk_begin + x / 6] + x % 6] : (x == W6 ? (T)1 : (T)0);
    __syncthreads();
    schur_row_dots<T>(U_s + ti.u_begin, ti.n_patch, Ws, sX, sDot, 1);
  }
  __syncthreads();
  const int pb = ti.patch_begin;
  for (int k = threadIdx.x; k < ti.n_patch; k += blockDim.x) {
    T d = depth_s[pb + k];
    if (apply) d -= sDot[k] * pscale_s[2 * (pb + k)];
    depth_out[tile_patch[pb + k]] = d;
  }
  __syncthreads();
}

// Whole solve of a small problem in one launch: per iteration
// every workgroup assembles its tiles, all wavefronts gather the damped
// reduced system, workgroup 0 factors, solves and retracts; finally the
// depths are written back.  Poses ping-pong between two buffers.
template <typename T>
__global__ void __launch_bounds__(tile_threads(sizeof(T)))
__attribute__((amdgpu_waves_per_eu(tile_threads(sizeof(T)) / 256, tile_threads(sizeof(T)) / 256)))
small_solve_kernel(SmallArgs<T> S) {
  extern __shared__ __align__(16) unsigned char lds[];
  IterArgs<T> A = S.it;
  const unsigned int nb = gridDim.x;
  const int w = blockIdx.x * blockDim.x + threadIdx.x, nw = gridDim.x * blockDim.x;
  const int wave = w >> 6, nwaves = nw >> 6;
  // the other slot: no launch uses it before this one ends
  if (blockIdx.x == 0 && threadIdx.x < 2) S.bar_next[threadIdx.x] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 2) *S.err_next = 0;
  for (int t = 0; t < S.n_iters; ++t) {
    A.first = t == 0;
    A.poses_cur = t == 0 ? S.poses_io : ((t - 1) & 1 ? S.pbuf1 : S.pbuf0);
    A.poses_next = (t & 1) ? S.pbuf1 : S.pbuf0;
    A.depth_in = S.depth_io;
    A.dx_prev = t ? A.dx : nullptr;
    A.status_prev = t ? S.status + t - 1 : nullptr;
    A.status = S.status + t;
    A.min_bits = S.min_bits + t;
    A.cost_out = S.cost ? S.cost + t : nullptr;
    A.invalid_out = S.invalid ? S.invalid + t : nullptr;
    for (int tile = blockIdx.x; tile < A.n_tiles; tile += nb) {
      tile_assemble<T, tile_threads(sizeof(T))>(A, tile, lds);
      __syncthreads();
    }
    if (!grid_sync(S.bar, nb, S.err, A.host_err)) return;
    gather_slice<T>(A, S.Sp, S.rhs, S.d0, wave, nwaves);
    if (!grid_sync(S.bar, nb, S.err, A.host_err)) return;
    if (blockIdx.x == 0) factor_solve_retract<T>(A, S.Sp, S.rhs, S.d0, lds);
    if (!grid_sync(S.bar, nb, S.err, A.host_err)) return;
  }
  if (S.n_iters == 0) return;
  const T* fin = ((S.n_iters - 1) & 1) ? S.pbuf1 : S.pbuf0;
  const bool apply = !S.status[S.n_iters - 1];
  T* sDx = reinterpret_cast<T*>(lds);
  for (int tile = blockIdx.x; tile < A.n_tiles; tile += nb)
    tile_writeback<T>(A.tiles[tile], A.tile_patch, A.blk_pose, A.U_s, A.pscale_s, A.depth_s, A.dx, apply,
                      S.depth_io, sDx);
  for (int x = w; x < 7 * A.n_frames; x += nw) S.poses_io[x] = fin[x];
}

// Apply the last iteration's depth step and write the results back.
template <typename T>
__global__ void __launch_bounds__(kTileThreads) tile_finalize_kernel(
    const TileInfo* tiles, const int* tile_patch, const int* blk_pose, const T* U_s, const T* pscale_s,
    const T* depth_s, const T* dx, const int* status, int status_stride, T* depth_out, const T* poses_final,
    T* poses_out, int n_frames) {
  extern __shared__ __align__(16) unsigned char lds[];
  const TileInfo ti = tiles[blockIdx.x];
  tile_writeback<T>(ti, tile_patch, blk_pose, U_s, pscale_s, depth_s, dx,
                    !(status && status[ti.inst * status_stride]), depth_out, reinterpret_cast<T*>(lds));
  if (blockIdx.x == 0 && poses_final != poses_out)
    for (int x = threadIdx.x; x < 7 * n_frames; x += blockDim.x) poses_out[x] = poses_final[x];
}

// Pose update of the large path: x_{t+1} = x_t Exp(dxi) for free poses.
template <typename T>
__global__ void retract_copy_kernel(const T* poses_cur, T* poses_next, T* dx, int n_fixed, int n_frames,
                                    const int* status, const T* dx_sys, const int* pos) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_frames) return;
  const T* pc = poses_cur + 7 * (size_t)i;
  T* pn = poses_next + 7 * (size_t)i;
  for (int m = 0; m < 7; ++m) pn[m] = pc[m];
  if (i < n_fixed) return;
  const int f = i - n_fixed;
  T xi[6];
  if (dx_sys) {  // the step in the system order: free pose f's block is pos[f]; stored back in the poses' order
    for (int m = 0; m < 6; ++m) {
      xi[m] = dx_sys[6 * pos[f] + m];
      dx[6 * f + m] = xi[m];
    }
  } else {
    for (int m = 0; m < 6; ++m) xi[m] = dx[6 * f + m];
  }
  if (!(status && *status)) retract_pose<T, T>(pn, xi);
}

// ---------------------------------------------------------------- launchers

template <typename T>
hipError_t launch_tile_iterate(const IterArgs<T>& A, int lds_bytes, hipStream_t st) {
  if (A.n_tiles == 0) return hipSuccess;
  hipError_t e = opt_in_lds((const void*)tile_iterate_kernel<T>, lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((tile_iterate_kernel<T>), dim3(A.n_tiles), dim3(tile_threads(sizeof(T))), lds_bytes, st, A);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tile_finalize(const TileInfo* tiles, int n_tiles, int lds_bytes, const int* tile_patch,
                                const int* blk_pose, const T* U_s, const T* pscale_s, const T* depth_s,
                                const T* dx, const int* status, int status_stride, T* depth_out,
                                const T* poses_final, T* poses_out, int n_frames, hipStream_t st) {
  if (n_tiles == 0) {
    if (poses_final != poses_out)
      return hipMemcpyAsync(poses_out, poses_final, sizeof(T) * 7 * (size_t)n_frames, hipMemcpyDeviceToDevice, st);
    return hipSuccess;
  }
  hipError_t e = opt_in_lds((const void*)tile_finalize_kernel<T>, lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((tile_finalize_kernel<T>), dim3(n_tiles), dim3(kTileThreads), lds_bytes, st, tiles,
                     tile_patch, blk_pose, U_s, pscale_s, depth_s, dx, status, status_stride, depth_out, poses_final,
                     poses_out, n_frames);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_retract_copy(const T* poses_cur, T* poses_next, T* dx, int n_fixed, int n_frames,
                               const int* status, hipStream_t st, const T* dx_sys, const int* pos) {
  hipLaunchKernelGGL((retract_copy_kernel<T>), dim3((n_frames + 127) / 128), dim3(128), 0, st, poses_cur,
                     poses_next, dx, n_fixed, n_frames, status, dx_sys, pos);
  return hipGetLastError();
}

template <typename T>
int small_solve_grid(int lds_bytes) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (opt_in_lds((const void*)small_solve_kernel<T>, lds_bytes) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)small_solve_kernel<T>, tile_threads(sizeof(T)),
                                                   lds_bytes) != hipSuccess)
    return 0;
  return cus * per_cu;
}

// grid never exceeds small_solve_grid (the workgroups the device holds at
// once).  The ordinary launch relies on the dispatcher placing every
// workgroup while the first ones wait at a grid barrier, which holds on a
// device whose other work finishes; the bounded waits of grid_sync turn a
// violation into an error, never a hang.  The cooperative launch has the
// runtime guarantee co-residency, at a higher launch cost.
template <typename T>
hipError_t launch_small_solve(const SmallArgs<T>& S, int grid, int lds_bytes, bool cooperative, hipStream_t st) {
  hipError_t e = opt_in_lds((const void*)small_solve_kernel<T>, lds_bytes);
  if (e != hipSuccess) return e;
  SmallArgs<T> copy = S;
  if (!cooperative) {
    hipLaunchKernelGGL((small_solve_kernel<T>), dim3(grid), dim3(tile_threads(sizeof(T))), lds_bytes, st, copy);
    return hipGetLastError();
  }
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel((const void*)small_solve_kernel<T>, dim3(grid), dim3(tile_threads(sizeof(T))), args,
                                    lds_bytes, st);
}

#define DPVBA_TILE_INSTANTIATE(T)                                                                          \
  template hipError_t launch_tile_iterate<T>(const IterArgs<T>&, int, hipStream_t);                       \
  template hipError_t launch_tile_finalize<T>(const TileInfo*, int, int, const int*, const int*, const T*, \
                                              const T*, const T*, const T*, const int*, int, T*, const T*, \
                                              T*, int, hipStream_t);                                       \
  template hipError_t launch_retract_copy<T>(const T*, T*, T*, int, int, const int*, hipStream_t, const T*,    \
                                             const int*);                                                  \
  template int small_solve_grid<T>(int);                                                                  \
  template hipError_t launch_small_solve<T>(const SmallArgs<T>&, int, int, bool, hipStream_t);

DPVBA_TILE_INSTANTIATE(float)
DPVBA_TILE_INSTANTIATE(double)

}  // namespace dpvba
