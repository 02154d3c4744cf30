// Round structure of one truncated low-rank addition (Sec. 4: truncated
// SVD after every addition into a low-rank block), shared by the device
// kernel (kernels_hlu.hip) and the host replay that checks termination
// (hlu_check_trunc_rounds in api.cpp).
//
// An op adds the parts sum_p alpha_p X_p Y_p^T to the block C = X_C Y_C^T.
// The kernel's LDS holds kTruncCols columns, so the parts are absorbed in
// rounds: a round stacks the r current columns of C with part columns taken
// from a cursor, truncates the stack, and the kept rank becomes r for the
// next round.  While parts remain, a round keeps at most
// kTruncCols - kTruncMinAbsorb columns, so the next round absorbs at least
// kTruncMinAbsorb part columns: every op ends after at most
// trunc_max_rounds rounds.  A rank cut by that limit, like a rank cut by
// the block's capacity, is counted as a rank overflow.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.h"

namespace hlu {

constexpr int kTruncCols = 64;        // columns of one round (LDS capacity)
constexpr int kTruncMinAbsorb = 1;    // part columns a round absorbs while parts remain

__host__ __device__ inline int dim_of(int32_t code, const int32_t* dims) {
  return code >= 0 ? code : dims[-code - 1];
}

// Position of the next unabsorbed part column.
struct TruncCursor {
  int part, col;
};

// Column list of the next round: the r current columns of C, then part
// columns from the cursor until `cols` (<= kTruncCols, normally equal)
// columns or the parts run out.
// emit(k, p, c) receives stack position k and its source: p = -1 for column
// c of C, else column c of part p.  Advances the cursor past the absorbed
// columns (and past parts of rank 0), sets *done when no part column is
// left, returns the number of columns K.
template <class Emit>
__host__ __device__ inline int trunc_round_columns(const TruncOp& op, const TruncPart* parts,
                                                   const int32_t* dims, int r, int cols, TruncCursor* cur,
                                                   bool* done, Emit&& emit) {
  int K = 0;
  for (int a = 0; a < r; ++a) emit(K++, -1, a);
  int p = cur->part, c = cur->col;
  while (p < op.np && K < cols) {
    if (c >= dim_of(parts[op.p0 + p].X.cols, dims)) {
      ++p;
      c = 0;
      continue;
    }
    emit(K++, p, c);
    ++c;
  }
  while (p < op.np && c >= dim_of(parts[op.p0 + p].X.cols, dims)) {
    ++p;
    c = 0;
  }
  cur->part = p;
  cur->col = c;
  *done = p >= op.np;
  return K;
}

// Largest rank a round of `cols` columns may keep: the block's capacity in
// the last round, otherwise at most cols - kTruncMinAbsorb.
__host__ __device__ inline int trunc_rank_limit(const TruncOp& op, bool done, int cols) {
  const int lim = cols - kTruncMinAbsorb;
  return done ? op.cap : (op.cap < lim ? op.cap : lim);
}

// Bound on the rounds of an op: the first round may absorb nothing (C
// already at the round's columns), every later round but the last absorbs
// at least kTruncMinAbsorb part columns.
__host__ __device__ inline int trunc_max_rounds(const TruncOp& op, const TruncPart* parts, const int32_t* dims) {
  int64_t cols = 0;
  for (int p = 0; p < op.np; ++p) cols += dim_of(parts[op.p0 + p].X.cols, dims);
  return 2 + (int)((cols + kTruncMinAbsorb - 1) / kTruncMinAbsorb);
}

}  // namespace hlu
