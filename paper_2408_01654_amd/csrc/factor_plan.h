// Sparsity plan of the blocked Cholesky of the reduced camera
// system, built by the analysis from the structure of S (which 6 x 6 blocks
// any tile contributes to).  Row r's envelope starts at the first column of
// the first pose block its pose shares a patch with; Cholesky fill stays
// between that column and the diagonal, so in panel k (columns 64 k ..
// 64 k + 63) exactly the rows whose envelope starts inside or before the
// panel can be non-zero.  The factor solves and updates only those: the
// 64-row blocks below the panel's diagonal block that hold such a row
// (block indices count from t0 = 64 (k + 1)); every other
// update is an exact zero (float32 factors also stop each panel at its
// reach).  The triangular solves skip the blocks of L outside the envelope.  Host arrays have one entry per panel (offsets one more); the
// lists themselves are in device memory.
#pragma once

namespace dpvba {

struct PanelPlan {
  const int* reach;       // host [nblk]: one past the last such row (n if none beyond)
  const int* blocks_off;  // host [nblk + 1]: panel k's active blocks are blocks[blocks_off[k] ..]
  const int* blocks;      // device: 64-row block indices, ascending
  // device, one entry per pair of 64-row blocks (2P, 2P + 1): the first pair
  // whose columns the pair's rows reach (forward substitution) and the last
  // pair whose rows reach the pair's columns (backward substitution)
  const int* chain_lo;
  const int* chain_hi;
  // device: per block row of width bw, its first coupled block column (fq),
  // and per 64-column panel the reach; row r's entries lie in columns
  // [bw fq[r / bw], reach[r / 64]) of the symmetric matrix
  const int* fq_dev;
  const int* reach_dev;
  int bw;
};

}  // namespace dpvba
