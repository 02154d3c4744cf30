// Task schedule of the persistent H-triangular solve (Algorithm 1, step III:
// z = U^{-1}(L^{-1} r)).
//
// The forward sweep visits the leaf clusters in order; the task of leaf j
// pulls every contribution of the blocks of L in its block row (dense:
// L_b y[sigma]; low-rank: X_b (Y_b^T y[sigma]) with the small product
// Y_b^T y[sigma] computed once per block by a T-product task), then solves
// with the unit lower triangle of the diagonal leaf.  The backward sweep is
// the mirror image with U.  This is the left-looking form of the recursive
// H-forward/backward substitution: the same arithmetic, summed per row.
#pragma once
#include <cstdint>
#include <vector>

#include "plan.h"
#include "structure.h"

namespace hlu {

struct SLeaf {
  int32_t row0, m;     // rows in cluster order
  int64_t diag;        // diagonal leaf (column-major, leading dimension m)
  int32_t d0, nd;      // dense contributions
  int32_t l0, nl;      // low-rank contributions
};
struct SDense {        // block rows of leaf j: off + i + k*ld, k < ncols
  int64_t off;
  int32_t ld, col0, ncols, lf0, lf1;   // columns [col0, col0+ncols) = leaves [lf0, lf1)
  int32_t pad;
};
struct SLow {          // X rows of leaf j: xoff + i + kk*ldx
  int64_t xoff;
  int32_t ldx, tp;
};
struct STprod {        // T = Y^T y[cols]: Y at yoff + r + kk*ldy
  int64_t yoff;
  int64_t toff;        // T (cap x nrhs, leading dimension cap) in the T buffer
  int32_t ldy, col0, ncols, slot, lf0, lf1, cap, pad;
};
enum STaskKind : int32_t { kFwdLeaf = 0, kFwdTprod = 1, kBwdLeaf = 2, kBwdTprod = 3 };
struct STask {
  int32_t kind, idx;
};

struct SolveSched {
  int32_t L = 0;                  // leaf clusters
  std::vector<SLeaf> leaves;      // [0, L) forward, [L, 2L) backward
  std::vector<SDense> dense;
  std::vector<SLow> low;
  std::vector<STprod> tprod;
  std::vector<STask> tasks;       // claim order
  int32_t n_fwd_tasks = 0;
  int64_t tbuf_per_rhs = 0;       // doubles of the T buffer per right-hand side
  int32_t max_m = 0;
  // algorithmic element reads of one application (both sweeps), for the
  // roofline: dense entries read + low-rank capacity entries touched is
  // counted by the caller from the realised ranks
};

void build_solve_sched(const Structure& S, const StoragePlan& st, SolveSched* out);

}  // namespace hlu
