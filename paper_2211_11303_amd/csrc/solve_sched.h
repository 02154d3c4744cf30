// Task schedule of the persistent H-triangular solve (Algorithm 1, step III:
// z = U^{-1}(L^{-1} r)).
//
// The forward sweep visits the leaf clusters in order; leaf j's solution
// row is y_j = L_jj^{-1} (b_j - sum over the blocks of L in its block row).
// Low-rank blocks contribute X_b (Y_b^T y[sigma]), the small product being
// formed once per block by a T-product task.  Every dense block L_b y[sigma]
// is formed into its own partial-sum record: by the task of leaf j-1 for the
// block coupling j to j-1 (on the critical path) and, with it, for the block
// coupling j+1 to j-1, otherwise by the push task of the leaf that completes
// sigma.  The task of leaf j then adds its
// records in a fixed order.  The backward sweep mirrors this with U.  This
// is the left-looking form of the recursive H-forward/backward
// substitution: the same arithmetic, summed per row.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "plan.h"
#include "structure.h"

namespace hlu {

struct SLeaf {
  int32_t row0, m;     // rows in cluster order
  int64_t diag;        // diagonal leaf (column-major, leading dimension m)
  int64_t inv;         // its triangle inverses in the inverse buffer (m x m, leading dimension m)
  int32_t d0, nd;      // dense contributions (partial-sum records) of this row
  int32_t l0, nl;      // low-rank contributions
  int32_t next_rec;    // dense record this leaf task computes after solving (-1: none)
  int32_t prev_rec;    // record of this row formed by the preceding leaf task (-1: none)
  int32_t tq0, ntq;    // T-product chunks this leaf task computes after solving
                       // (leaf_tq[tq0 .. tq0 + ntq)): chunks of exactly this leaf's
                       // rows whose block is needed within kNearLeaves leaves
  int64_t nm;          // the neighbour records' blocks times this leaf's triangle
                       // inverse in the NM buffer (rows of next_rec, then of
                       // next_rec2, x m, leading dimension = those rows; -1: the
                       // record is formed from the solution instead)
  int32_t next_rec2;   // with nm: the record of the leaf after next (second
                       // neighbour) coupled to this leaf alone, formed in the same
                       // product (-1: none; otherwise a push task forms it)
  int32_t nm_rows;     // rows of the NM block (0 without nm)
};
struct SDense {        // block rows of leaf j: off + i + k*ld, k < ncols
  int64_t off;
  int32_t ld, col0, ncols, lf0, lf1;   // columns [col0, col0+ncols) = leaves [lf0, lf1)
  int32_t m;           // rows (= size of leaf j)
  int32_t row0;        // first row of leaf j
  int32_t pad;
};
struct SLow {          // X rows of leaf j: xoff + i + kk*ldx; T = sum of ntp chunk products from tp
  int64_t xoff;
  int32_t ldx, tp, ntp, pad;
};
// One row chunk of a low-rank block's product T = Y^T y[sigma]: the chunk
// covers the leaves [lf0, lf1) of sigma, rows [col0, col0 + ncols); Y of
// the chunk at yoff + r + kk*ldy.  The chunks of a block are summed by the
// consumer, so a long sigma is reduced by several workgroups, each as soon
// as its own leaves are solved.
struct STprod {
  int64_t yoff;
  int64_t toff;        // chunk product (cap x nrhs, leading dimension cap) in the T buffer
  int32_t ldy, col0, ncols, slot, lf0, lf1, cap, pad;
};
constexpr int32_t kTprodChunkRows = 1 << 30; // rows of sigma per T-product chunk (no row split)
constexpr int32_t kNearLeaves = 2;          // consumers this close get the chunk from the leaf task
constexpr int32_t kPushChunk = 2;   // partial-sum records per push task
constexpr int32_t kTprodGroup = 8;  // T-products of blocks sharing sigma's rows per task
enum STaskKind : int32_t { kFwdLeaf = 0, kFwdTprod = 1, kBwdLeaf = 2, kBwdTprod = 3, kFwdPush = 4, kBwdPush = 5 };
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
  std::vector<int32_t> push0;     // per push task: first record in push_recs (size #push + 1)
  std::vector<int32_t> push_recs; // dense records computed by push tasks
  std::vector<int32_t> leaf_tq;   // T-product chunks computed by leaf tasks
  std::vector<int32_t> tg0;       // per T-product task: first entry in tg_list (size #tasks + 1)
  std::vector<int32_t> tg_list;   // T-products of each T-product task, in order
  int32_t n_fwd_tasks = 0;
  int64_t tbuf_per_rhs = 0;       // doubles of the T buffer per right-hand side
  int64_t inv_elems = 0;          // elements of the inverse buffer (sum of m^2 over leaves)
  int64_t nm_elems = 0;           // elements of the NM buffer
  int32_t max_m = 0;
  // algorithmic element reads of one application (both sweeps), for the
  // roofline: dense entries read + low-rank capacity entries touched is
  // counted by the caller from the realised ranks
};

void build_solve_sched(const Structure& S, const StoragePlan& st, SolveSched* out);
// Throws unless every flag a task waits on is set by one earlier task.
void check_solve_waits(const SolveSched& sc);

// Device copy of a schedule and the buffers of the persistent solve.
struct SolveDev {
  const STask* tasks;
  const SLeaf* leaves;
  const SDense* dense;
  const SLow* low;
  const STprod* tprod;
  void* inv;            // triangle inverses of the diagonal leaves (factor storage type)
  void* nm;             // neighbour blocks times the inverses (factor storage type)
  double* pivots;       // U_ii of every diagonal leaf, cluster order (N)
  double* y;
  double* tbuf;
  int32_t* leaf_flag;
  int32_t* tp_flag;
  int32_t* ctr;
  const int32_t* push0;
  const int32_t* push_recs;
  const int32_t* leaf_tq;
  const int32_t* tg0;
  const int32_t* tg_list;
  double* pbuf;
  int32_t* pflag;
  int64_t pstride;
  int64_t* trace;
  int64_t wait_ticks;   // longest wait of a task, in device wall-clock ticks
  int32_t ntasks, n_fwd, L, max_m, max_rhs;
};

// Both triangle inverses of every diagonal leaf (arena storage type T,
// arithmetic in FP64), written to d.inv, and the pivots U_ii to d.pivots;
// then, for every leaf task with a neighbour record, that record's block
// times the leaf's inverse (d.nm).  Run after each factorization.
template <class T>
hipError_t diag_inverse_launch(const T* arena, const SolveDev& d, hipStream_t s);

// z = U^{-1} L^{-1} y for the nrhs columns of d.y (cluster order), in place.
template <class T>
hipError_t solve_persistent_launch(const T* arena, const int32_t* dims, const SolveDev& d, int32_t N,
                                   int32_t nrhs, int32_t epoch, int32_t grid, hipStream_t s);

}  // namespace hlu
