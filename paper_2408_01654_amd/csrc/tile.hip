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
#include "edge.h"
#include "mfma.h"
#include "packed.h"
#include "tileargs.h"
#include "dpvba.h"

namespace dpvba {

// Phases 0-3 for one tile; the caller synchronises before reusing `lds`.
template <typename T>
__device__ void tile_assemble(const IterArgs<T>& A, int tile, unsigned char* lds) {
  const TileInfo ti = A.tiles[tile];
  const int tid = threadIdx.x;
  const int K = ti.n_patch, Tn = ti.n_slot, nb = ti.n_blk, W6 = 6 * nb;
  const TileLds L = tile_lds_plan(K, Tn, nb, (int)sizeof(T));
  const int Kp = L.K_pad, Wp = L.W_pad;
  T* base = reinterpret_cast<T*>(lds);
  T* sSlot = base + L.slot;   // [Tn][18]: R_ji (9), t_ji (3)
  T* sPatch = base + L.patch; // [K][4]: x^0, x^1, d, w / sqrt(C~)
  T* sPs = base + L.psum;     // [K][8]: C (then 1 / sqrt(C~)), w, -sum_j Ad^T E_j
  T* sM = base + L.m;         // [Tn][28]
  T* sU = base + L.u;         // [Kp][Wp]; first the per-thread partial sums
  T* sWork = sU;
  unsigned char* rec = lds + align16(L.total_T * (int)sizeof(T));
  const int cellT = L.cell_bytes / (int)sizeof(T);
  T* sCell = reinterpret_cast<T*>(rec);  // [K*Tn][cellT]
  T* sB = reinterpret_cast<T*>(rec);     // later: [Tn][80]
  T* sDx = reinterpret_cast<T*>(rec);    // phase 0: [W6]
  unsigned char* tab = rec + align16(L.rec_bytes);
  unsigned char* sPairA = tab + L.pair_a;
  unsigned char* sPairB = tab + L.pair_b;
  unsigned char* sBlkS0 = tab + L.blk_s0;
  unsigned char* sBlkS1 = tab + L.blk_s1;
  signed char* sSlotBlk = reinterpret_cast<signed char*>(tab + L.slot_blk);
  __shared__ int sInvalid;

  // ---- phase 0: index tables, slot relative poses, previous depth step, records
  if (tid == 0) sInvalid = 0;
  for (int a = tid; a < nb; a += blockDim.x) {
    for (int b = a; b < nb; ++b) {
      const int q = upper_pair_index(a, b, nb);
      sPairA[q] = (unsigned char)a;
      sPairB[q] = (unsigned char)b;
    }
    sBlkS0[a] = 255;
    sBlkS1[a] = 0;
  }
  for (int s = tid; s < Tn; s += blockDim.x) {
    sSlotBlk[s] = (signed char)A.slot_blk[ti.slot_begin + s];
    const int j = A.slot_frame[ti.slot_begin + s];
    T Ri[9], tiv[3], Rj[9], tj[3];
    const T* pi = A.poses_cur + 7 * (size_t)ti.frame;
    const T* pj = A.poses_cur + 7 * (size_t)j;
    quat_to_rot<T, T>(pi + 3, Ri);
    quat_to_rot<T, T>(pj + 3, Rj);
    for (int m = 0; m < 3; ++m) { tiv[m] = pi[m]; tj[m] = pj[m]; }
    relative_pose<T>(Ri, tiv, Rj, tj, sSlot + 18 * s, sSlot + 18 * s + 9);
  }
  const bool apply_prev =
      !A.first && A.dx_prev && !(A.status_prev && A.status_prev[ti.inst * A.status_stride]);
  if (apply_prev) {
    for (int x = tid; x < W6; x += blockDim.x) sDx[x] = A.dx_prev[6 * A.blk_pose[ti.blk_begin + x / 6] + x % 6];
    const T* src_u = A.U_s + ti.u_begin;
    for (int x = tid; x < K * W6; x += blockDim.x) sU[(x / W6) * Wp + x % W6] = src_u[x];
  }
  __syncthreads();
  if (tid == 0) {
    for (int s = 0; s < Tn; ++s) {
      const int b = sSlotBlk[s];
      if (b < 0) continue;
      if (sBlkS0[b] == 255) sBlkS0[b] = (unsigned char)s;
      sBlkS1[b] = (unsigned char)(s + 1);
    }
  }
  const int pb = ti.patch_begin;
  for (int k = tid; k < K; k += blockDim.x) {
    T x0, x1, d;
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
      if (apply_prev) {
        const T* u = sU + k * Wp;
        T dot = (T)0;
        for (int x = 0; x < W6; ++x) dot += u[x] * sDx[x];
        d -= (A.pscale_s[2 * (pb + k) + 1] + dot) * A.pscale_s[2 * (pb + k)];
      }
    }
    if (A.first || apply_prev) A.depth_s[pb + k] = d;
    sPatch[4 * k] = x0;
    sPatch[4 * k + 1] = x1;
    sPatch[4 * k + 2] = d;
    sPatch[4 * k + 3] = (T)0;
  }
  __syncthreads();
  // records: (target, weight) per cell, weight -1 marks a cell without an
  // edge; batches of 8 cells per thread keep the index loads and the
  // dependent record loads in flight together
  {
    const int ncell = K * Tn;
    const int* grid = A.edge_grid + ti.grid_begin;
    const float2* tgt = reinterpret_cast<const float2*>(A.target);
    const float2* wgt = reinterpret_cast<const float2*>(A.weight);
    for (int c0 = tid; c0 < ncell; c0 += 8 * kTileThreads) {
      int e[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = c0 + u * kTileThreads;
        e[u] = c < ncell ? grid[c] : -1;
      }
      float2 tg[8], wt[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        tg[u] = e[u] >= 0 ? tgt[e[u]] : make_float2(0.f, 0.f);
        wt[u] = e[u] >= 0 ? wgt[e[u]] : make_float2(-1.f, -1.f);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = c0 + u * kTileThreads;
        if (c < ncell)
          *reinterpret_cast<float4*>(rec + (size_t)c * L.cell_bytes) = make_float4(tg[u].x, tg[u].y, wt[u].x, wt[u].y);
      }
    }
  }
  __syncthreads();

  // ---- phase 1: edges.  Thread (g, s) takes slot s of patches g, g + G, ...
  const int G = kTileThreads / Tn;
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
      const bool has = r4.z >= 0.f;
      EdgeTerms<T> o;
      const bool ok = has && edge_eval<T>(Rt, sPatch[4 * k], sPatch[4 * k + 1], sPatch[4 * k + 2], A.fx, A.fy,
                                          A.cx, A.cy, A.z_min, r4.x, r4.y, r4.z, r4.w, o);
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
#pragma unroll
  for (int m = 0; m < kRedWidth; ++m) sWork[tid * kRedWidth + m] = acc[m];
  __syncthreads();

  // ---- phase 2a: per-slot totals, thread groups summed in order
  for (int idx = tid; idx < Tn * kRedWidth; idx += blockDim.x) {
    const int ss = idx / kRedWidth, m = idx % kRedWidth;
    T v = (T)0;
    for (int gg = 0; gg < G; ++gg) v += sWork[(gg * Tn + ss) * kRedWidth + m];
    sM[ss * kRedWidth + m] = v;
  }
  __syncthreads();

  // ---- phase 2b: Schur rows u_k = E_k / sqrt(C~_k), appended w_k / sqrt(C~_k).
  // (i) thread k sums (C, w, -sum_j Ad(T_ji)^T E_j) of patch k over its slots
  //     in slot order (the slot poses are read by every lane at once);
  //     (ii) thread (k, x) writes row entry x.
  const int src = ti.src_blk;
  for (int k = tid; k < K; k += blockDim.x) {
    T v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int ss = 0; ss < Tn; ++ss) {
      const T* cell = sCell + (size_t)(k * Tn + ss) * cellT;
      T c[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) c[m] = cell[m];
      const T* R = sSlot + 18 * ss;
      const T* tt = R + 9;
      v[0] += c[6];
      v[1] += c[7];
#pragma unroll
      for (int q = 0; q < 3; ++q) v[2 + q] -= R[q] * c[0] + R[3 + q] * c[1] + R[6 + q] * c[2];
      const T b0 = c[3] - (tt[1] * c[2] - tt[2] * c[1]);
      const T b1 = c[4] - (tt[2] * c[0] - tt[0] * c[2]);
      const T b2 = c[5] - (tt[0] * c[1] - tt[1] * c[0]);
#pragma unroll
      for (int q = 0; q < 3; ++q) v[5 + q] -= R[q] * b0 + R[3 + q] * b1 + R[6 + q] * b2;
    }
#pragma unroll
    for (int m = 0; m < 8; ++m) sPs[8 * k + m] = v[m];
  }
  __syncthreads();
  for (int k = tid; k < K; k += blockDim.x) {
    const T Ct = sPs[8 * k] * ((T)1 + A.lambda) + A.lambda;
    const T is = (T)1 / dsqrt(Ct);
    const T rs = sPs[8 * k + 1] * is;
    sPs[8 * k] = is;
    sPatch[4 * k + 3] = rs;
    A.pscale_s[2 * (pb + k)] = is;
    A.pscale_s[2 * (pb + k) + 1] = rs;
  }
  __syncthreads();
  for (int idx = tid; idx < Kp * Wp; idx += blockDim.x) {
    const int k = idx / Wp, x = idx - (idx / Wp) * Wp;
    T v = (T)0;
    if (k < K && x <= W6) {
      const T rs = sPatch[4 * k + 3];
      if (x == W6) {
        v = rs;
      } else {
        const int b = x / 6, m = x - (x / 6) * 6;
        const T is = sPs[8 * k];
        if (b == src) {
          v = sPs[8 * k + 2 + m] * is;
        } else {
          for (int ss = sBlkS0[b]; ss < sBlkS1[b]; ++ss) v += sCell[(size_t)(k * Tn + ss) * cellT + m];
          v *= is;
        }
      }
    }
    sU[idx] = v;
  }
  __syncthreads();

  // ---- phase 2c: stored rows; per-slot source blocks Ad^T M, Ad^T M Ad, Ad^T v
  for (int x = tid; x < K * W6; x += blockDim.x) A.U_s[ti.u_begin + x] = sU[(x / W6) * Wp + x % W6];
  for (int ss = tid; ss < Tn; ss += blockDim.x) {
    const T* R = sSlot + 18 * ss;
    const T* t = R + 9;
    const T* M21 = sM + ss * kRedWidth;
    T* out = sB + 80 * ss;
    T col[6], res[6];
    for (int c = 0; c < 6; ++c) {
      for (int r = 0; r < 6; ++r) col[r] = sym6<T>(M21, r, c);
      adjoint_transpose_apply<T>(R, t, col, res);
      for (int r = 0; r < 6; ++r) out[r * 6 + c] = res[r];
    }
    for (int r = 0; r < 6; ++r) {
      for (int c = 0; c < 6; ++c) col[c] = out[r * 6 + c];
      adjoint_transpose_apply<T>(R, t, col, res);
      for (int c = 0; c < 6; ++c) out[36 + r * 6 + c] = res[c];
    }
    adjoint_transpose_apply<T>(R, t, M21 + 21, out + 72);
  }
  __syncthreads();

  // ---- phase 3: U^T U on the matrix cores, plus B; upper entries only
  T* outS = A.part_S + ti.part_begin;
  T* outV = A.part_vec + ti.vec_begin;
  const int T16 = Wp / 16;
  const int lane = tid & 63, wv = tid >> 6;
  for (int tp = wv; tp < T16 * (T16 + 1) / 2; tp += kTileThreads / 64) {
    int ta = 0, rem = tp;
    while (rem >= T16 - ta) { rem -= T16 - ta; ++ta; }
    const int tb = ta + rem;
    typename Mfma<T>::acc_t accv = {0, 0, 0, 0};
    const T* ua = sU + (lane >> 4) * Wp + ta * 16 + (lane & 15);
    const T* ub = sU + (lane >> 4) * Wp + tb * 16 + (lane & 15);
    for (int k0 = 0; k0 < Kp; k0 += 4) accv = Mfma<T>::step(ua[k0 * Wp], ub[k0 * Wp], accv);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = ta * 16 + Mfma<T>::row(lane, v), col = tb * 16 + (lane & 15);
      if (row > col || row >= W6 || col > W6) continue;
      const int a = row / 6, r = row % 6;
      if (col == W6) {  // right-hand side and Diag(B) of row `row`
        T vb = (T)0, db = (T)0;
        if (a == src) {
          for (int ss = 0; ss < Tn; ++ss) {
            vb -= sB[80 * ss + 72 + r];
            db += sB[80 * ss + 36 + r * 7];
          }
        } else {
          for (int ss = sBlkS0[a]; ss < sBlkS1[a]; ++ss) {
            vb += sM[ss * kRedWidth + 21 + r];
            db += sM[ss * kRedWidth + tri_index(r, r)];
          }
        }
        outV[row] = accv[v] - vb;
        outV[W6 + row] = db;
        continue;
      }
      const int b = col / 6, c = col % 6, rc = r * 6 + c;
      T val = -accv[v];
      if (a == b) {
        if (a == src) {
          for (int ss = 0; ss < Tn; ++ss) val += sB[80 * ss + 36 + rc];
        } else {
          for (int ss = sBlkS0[a]; ss < sBlkS1[a]; ++ss) val += sym6<T>(sM + ss * kRedWidth, r, c);
        }
      } else if (a == src) {
        for (int ss = sBlkS0[b]; ss < sBlkS1[b]; ++ss) val -= sB[80 * ss + rc];
      } else if (b == src) {
        for (int ss = sBlkS0[a]; ss < sBlkS1[a]; ++ss) val -= sB[80 * ss + c * 6 + r];
      }
      outS[upper_pair_index(a, b, nb) * 36 + rc] = val;
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
__global__ void __launch_bounds__(kTileThreads) tile_iterate_kernel(IterArgs<T> A) {
  extern __shared__ __align__(16) unsigned char lds[];
  tile_assemble<T>(A, blockIdx.x, lds);
}

// Damped reduced system of a small problem (packed lower triangle, row i at
// i (i + 1) / 2), summed from the tiles' shares in tile order.  One
// wavefront per lower 6x6 block (P >= Q): the block's share offsets are
// loaded once and broadcast, so every share load of a lane is independent.
// Diagonal entries get lam (Diag(B) + 1) and are kept in d0; the diagonal
// blocks also produce s.
template <typename T>
__device__ void gather_slice(const IterArgs<T>& A, T* Sp, T* rhs, T* d0, int wave, int nwaves) {
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
        v += A.lambda * (db + (T)1);
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
  T* x = reinterpret_cast<T*>(lds) + 36 * nr + nr * nr;  // after the solver's own arrays
  if (nr == 32) panel_chol_solve<T, 2>(n, Sp_g, rhs_g, d0_g, lds, x, &bad, &minr);
  else if (nr == 64) panel_chol_solve<T, 4>(n, Sp_g, rhs_g, d0_g, lds, x, &bad, &minr);
  else if (nr == 80) panel_chol_solve<T, 5>(n, Sp_g, rhs_g, d0_g, lds, x, &bad, &minr);
  else panel_chol_solve<T, 6>(n, Sp_g, rhs_g, d0_g, lds, x, &bad, &minr);
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
      for (int t = 0; t < A.n_tiles; ++t) {
        cc += A.part_cost[t];
        inv += A.part_invalid[t];
      }
      *A.cost_out = cc;
      if (A.invalid_out) *A.invalid_out = inv;
    }
  }
  __syncthreads();
}

// Grid-wide barrier of a cooperative launch: bar[0] counts arrivals,
// bar[1] is the generation.  Every wait is bounded; on timeout *err is set
// and false returned, so no workgroup can spin forever.
constexpr long long kSpinLimit = 1LL << 22;

__device__ bool grid_sync(unsigned int* bar, unsigned int nblocks, int* err) {
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
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) {
          ok = 0;
          atomicOr(err, 1);
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
// caller's array.
template <typename T>
__device__ void tile_writeback(const TileInfo& ti, const int* tile_patch, const int* blk_pose, const T* U_s,
                               const T* pscale_s, const T* depth_s, const T* dx, bool apply, T* depth_out,
                               T* sDx) {
  const int W6 = 6 * ti.n_blk;
  T* sU = sDx + W6;  // the tile's Schur rows, copied once
  if (apply) {
    for (int x = threadIdx.x; x < W6; x += blockDim.x) sDx[x] = dx[6 * blk_pose[ti.blk_begin + x / 6] + x % 6];
    for (int x = threadIdx.x; x < ti.n_patch * W6; x += blockDim.x) sU[x] = U_s[ti.u_begin + x];
  }
  __syncthreads();
  const int pb = ti.patch_begin;
  for (int k = threadIdx.x; k < ti.n_patch; k += blockDim.x) {
    T d = depth_s[pb + k];
    if (apply) {
      const T* u = sU + k * W6;
      T dot = (T)0;
      for (int xx = 0; xx < W6; ++xx) dot += u[xx] * sDx[xx];
      d -= (pscale_s[2 * (pb + k) + 1] + dot) * pscale_s[2 * (pb + k)];
    }
    depth_out[tile_patch[pb + k]] = d;
  }
  __syncthreads();
}

// Whole solve of a small problem in one cooperative launch: per iteration
// every workgroup assembles its tiles, all wavefronts gather the damped
// reduced system, workgroup 0 factors, solves and retracts; finally the
// depths are written back.  Poses ping-pong between two buffers.
template <typename T>
__global__ void __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(1, 1)))
small_solve_kernel(SmallArgs<T> S) {
  extern __shared__ __align__(16) unsigned char lds[];
  IterArgs<T> A = S.it;
  const unsigned int nb = gridDim.x;
  const int w = blockIdx.x * blockDim.x + threadIdx.x, nw = gridDim.x * blockDim.x;
  const int wave = w >> 6, nwaves = nw >> 6;
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
      tile_assemble<T>(A, tile, lds);
      __syncthreads();
    }
    if (!grid_sync(S.bar, nb, S.err)) return;
    gather_slice<T>(A, S.Sp, S.rhs, S.d0, wave, nwaves);
    if (!grid_sync(S.bar, nb, S.err)) return;
    if (blockIdx.x == 0) factor_solve_retract<T>(A, S.Sp, S.rhs, S.d0, lds);
    if (!grid_sync(S.bar, nb, S.err)) return;
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
__global__ void retract_copy_kernel(const T* poses_cur, T* poses_next, const T* dx, int n_fixed, int n_frames,
                                    const int* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_frames) return;
  const T* pc = poses_cur + 7 * (size_t)i;
  T* pn = poses_next + 7 * (size_t)i;
  for (int m = 0; m < 7; ++m) pn[m] = pc[m];
  if (i >= n_fixed && !(status && *status)) {
    T xi[6];
    for (int m = 0; m < 6; ++m) xi[m] = dx[6 * (i - n_fixed) + m];
    retract_pose<T, T>(pn, xi);
  }
}

// ---------------------------------------------------------------- launchers

template <typename T>
hipError_t launch_tile_iterate(const IterArgs<T>& A, int lds_bytes, hipStream_t st) {
  if (A.n_tiles == 0) return hipSuccess;
  hipError_t e = opt_in_lds((const void*)tile_iterate_kernel<T>, lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((tile_iterate_kernel<T>), dim3(A.n_tiles), dim3(kTileThreads), lds_bytes, st, A);
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
hipError_t launch_retract_copy(const T* poses_cur, T* poses_next, const T* dx, int n_fixed, int n_frames,
                               const int* status, hipStream_t st) {
  hipLaunchKernelGGL((retract_copy_kernel<T>), dim3((n_frames + 127) / 128), dim3(128), 0, st, poses_cur,
                     poses_next, dx, n_fixed, n_frames, status);
  return hipGetLastError();
}

template <typename T>
int small_solve_grid(int lds_bytes) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (opt_in_lds((const void*)small_solve_kernel<T>, lds_bytes) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)small_solve_kernel<T>, kTileThreads,
                                                   lds_bytes) != hipSuccess)
    return 0;
  return cus * per_cu;
}

template <typename T>
hipError_t launch_small_solve(const SmallArgs<T>& S, int grid, int lds_bytes, hipStream_t st) {
  hipError_t e = opt_in_lds((const void*)small_solve_kernel<T>, lds_bytes);
  if (e != hipSuccess) return e;
  SmallArgs<T> copy = S;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel((const void*)small_solve_kernel<T>, dim3(grid), dim3(kTileThreads), args,
                                    lds_bytes, st);
}

#define DPVBA_TILE_INSTANTIATE(T)                                                                          \
  template hipError_t launch_tile_iterate<T>(const IterArgs<T>&, int, hipStream_t);                       \
  template hipError_t launch_tile_finalize<T>(const TileInfo*, int, int, const int*, const int*, const T*, \
                                              const T*, const T*, const T*, const int*, int, T*, const T*, \
                                              T*, int, hipStream_t);                                       \
  template hipError_t launch_retract_copy<T>(const T*, T*, const T*, int, int, const int*, hipStream_t);  \
  template int small_solve_grid<T>(int);                                                                  \
  template hipError_t launch_small_solve<T>(const SmallArgs<T>&, int, int, hipStream_t);

DPVBA_TILE_INSTANTIATE(float)
DPVBA_TILE_INSTANTIATE(double)

}  // namespace dpvba
