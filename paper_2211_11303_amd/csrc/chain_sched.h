// Schedule of the persistent H-triangular solve (Algorithm 1, step III:
// z = U^{-1}(L^{-1} r)) in chain form.
//
// A sweep visits the leaf clusters in order (forward: ascending, the block
// rows of L; backward: descending, the block rows of U).  At sweep position
// p the solution rows of leaf f(p) are y_f = T_ff^{-1} (r_f - sum over the
// blocks of its block row), T = L or U.  The contributions are split by the
// distance d = p - q between the consuming position p and the position q of
// the source leaf whose solution they multiply:
//
//   near  (d <= kChainWindow): applied by the chain itself.  For every
//         source leaf the blocks it feeds within the window (dense pieces,
//         and low-rank pieces X_b[k] Y_b[f]^T expanded) are stacked under
//         the leaf's triangle inverse and premultiplied by it once per
//         factorisation: S_f = [T_ff^{-1}; B_{k1 f} T_ff^{-1}; ...].  One
//         product S_f r_f then gives y_f and the near contributions, which
//         stay in the chain's LDS until their target comes up.
//   late  (kChainWindow < d <= kLateWindow): one gather task per target
//         leaf and distance, i.e. per single source leaf, multiplies that
//         one piece (dense, or low-rank formed inline as X (Y^T y)) into a
//         record as soon as the source is solved.
//   mid (kLateWindow < d <= kMidWindow) and far (d > kMidWindow): two more
//         gather tasks per target leaf sum the dense pieces and the
//         low-rank blocks through their products T_b = Y_b^T y[sigma],
//         formed once per block chunk by T-product tasks.  Splitting by
//         distance lets the bulk of the work (far) start long before the
//         chain needs it, and keeps the gathers that start late small.
//
// Chains are workgroups that each own a group of right-hand-side columns
// and run both sweeps; they publish their progress (positions done) per
// sweep.  Helper tasks (T-products, gathers) are claimed in order of the
// latest source position they read, so whatever runs, the earliest
// unfinished helper only waits on chain progress that the chains have
// already made, and a chain only waits on gathers of sources at least
// kChainWindow + 1 positions back.  The summation order of every output is
// fixed by the schedule, never by timing.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "plan.h"
#include "structure.h"

namespace hlu {

constexpr int32_t kChainWindow = 3;    // near: sources this many positions back at most
constexpr int32_t kLateWindow = 8;     // sources up to this many positions back: one gather per distance
constexpr int32_t kMidWindow = 24;     // then one gather up to this distance, one beyond it
constexpr int32_t kGatherClasses = kLateWindow - kChainWindow + 2;
constexpr int32_t kTprodRows = 256;    // rows of sigma per T-product piece (whole leaves; one leaf may exceed it)
constexpr int32_t kGatherBudget = 320; // work of one gather, in columns staged through LDS (dense columns;
                                       // low-rank inputs counted by an estimate of their columns)
constexpr int32_t kMaxRecords = 8;     // gather records a chain reads per position at most
constexpr int32_t kMaxTargets = 64;    // near targets of one stacked operator at most
constexpr int32_t kChainCols = 4;      // right-hand-side columns per chain
constexpr int32_t kMaxStackRows = 256; // rows of a stacked operator (one per thread)
constexpr int32_t kMaxLeafRows = 64;   // rows of a leaf cluster the chain keeps in registers
constexpr size_t kChainArgBytes = 1024;  // device copy of a solve launch's arguments

// One position of a sweep ([0, L) forward, [L, 2L) backward).
struct CLeaf {
  int32_t row0, m;       // rows of the leaf, cluster order
  int32_t leaf;          // leaf index (ascending cluster order)
  int32_t srows;         // rows of the stacked operator (m + near target rows)
  int64_t stack;         // its element offset in the stack buffer (column-major, ld srows, m columns)
  int64_t inv;           // the leaf's triangle inverses in the inverse buffer (m x m)
  int64_t diag;          // the dense diagonal leaf in the arena (m x m, ld m)
  int32_t t0, nt;        // near targets tgt[t0 .. t0 + nt)
  int32_t rec0, nrec;    // gather records [rec0, rec0 + nrec) added into this leaf: late by distance, then
                         // the last gathers of the mid and far classes (each class is split into gathers of
                         // bounded work, each adding its predecessor's record)
  int32_t pad;
};

// Rows [srow0, srow0 + m) of a stacked operator: the block from the source
// leaf to the leaf dpos positions later, times the source's inverse.
struct CTarget {
  int32_t dpos, srow0, m, kind;   // kind: 0 dense piece, 1 low-rank piece
  int64_t off;                    // dense: element (0, 0) of the piece; low-rank: X rows of the target
  int64_t yoff;                   // low-rank: Y rows of the source
  int32_t ld, ldy, slot, pad;     // dense / X leading dimension; Y leading dimension; rank slot
};

// Gather inputs.
struct GDense {          // D (m x ncols) at off, leading dimension ld, times y rows [col0, col0 + ncols)
  int64_t off;
  int32_t ld, col0, ncols, pmax;  // pmax: latest source position read
};
struct GLow {            // X rows of the target (m x k) times the sum of T-product chunks tp .. tp + ntp
  int64_t xoff;
  int32_t ldx, tp, ntp, pad;
};
struct GInline {         // X rows of the target times (Y rows [ycol0 ..)^T y rows [col0, col0 + ncols))
  int64_t xoff, yoff;
  int32_t ldx, ldy, slot, col0, ncols, pmax;
};
struct CGather {
  int32_t pos;           // sweep position of the target leaf ([0, 2L))
  int32_t member;        // problem of a batch (chains member * n_chain ...)
  int32_t m, row0;       // rows of the target leaf
  int32_t d0, nd, l0, nl, i0, ni;
  int32_t rec;           // output record
  int32_t prev;          // record of the previous gather of the same class and leaf, added in (-1: none)
};
// One row chunk of a low-rank block's product T = Y^T y[chunk rows]
// (k x nrhs, leading dimension cap) in the T buffer.
struct CTprod {
  int64_t yoff;
  int64_t toff;
  int32_t ldy, col0, ncols, slot, cap, pmax, sweep, member;
};

enum CTaskKind : int32_t { kTaskTprod = 0, kTaskGather = 1 };
struct CTask {
  int32_t kind, idx;     // T-product group (tg0/tg_list) or gather
};

struct ChainSched {
  int32_t L = 0;                  // leaf clusters (sum over the members of a batch)
  int32_t members = 1;
  std::vector<int32_t> member_L;  // leaves of each member
  std::vector<int32_t> member_pos0;   // first forward position of each member (its leaves are contiguous)
  std::vector<CLeaf> leaves;      // 2L positions: member p's forward positions [pos0, pos0 + L_p) in [0, L),
                                  // backward ones at the same indices + L
  std::vector<CTarget> tgt;
  std::vector<GDense> gdense;
  std::vector<GLow> glow;
  std::vector<GInline> ginl;
  std::vector<CGather> gathers;
  std::vector<CTprod> tprod;
  std::vector<int32_t> tg0, tg_list;  // T-product groups (tasks) -> T-products
  std::vector<CTask> tasks;           // helper tasks in claim order
  int64_t stack_elems = 0;        // elements of the stack buffer
  int64_t inv_elems = 0;          // elements of the inverse buffer
  int64_t tbuf_per_rhs = 0;       // doubles of the T buffer per right-hand side
  int32_t max_m = 0;
  int32_t num_recs = 0;           // gather records
};

// Builds one problem's chain schedule from its block tree and arena layout.
void build_chain_sched(const Structure& S, const StoragePlan& st, ChainSched* out);
// Union of several problems' schedules (a batch): arena element offsets a,
// rank slot shifts d, stacked-vector row offsets o.
void merge_chain_scheds(const std::vector<const ChainSched*>& S, const std::vector<int64_t>& a,
                        const std::vector<int32_t>& d, const std::vector<int32_t>& o, ChainSched* out);
// Throws unless the claim order makes every wait point backwards (see the
// file comment).
void check_chain_sched(const ChainSched& sc);

// Device view of a schedule and its buffers.
struct ChainDev {
  const CLeaf* leaves;
  const CTarget* tgt;
  const GDense* gdense;
  const GLow* glow;
  const GInline* ginl;
  const CGather* gathers;
  const CTprod* tprod;
  const int32_t* tg0;
  const int32_t* tg_list;
  const CTask* tasks;
  const int32_t* member_L;
  const int32_t* member_pos0;
  void* stack;          // stacked operators (factor storage type)
  void* inv;            // triangle inverses of the diagonal leaves (factor storage type)
  double* pivots;       // U_ii of every diagonal leaf, cluster order
  double* y;            // stacked vectors, cluster order, N x max_rhs
  double* tbuf;         // T products
  double* fbuf;         // gather records, rstride doubles each (m x nrhs, leading dimension m)
  int32_t* tp_flag;     // per T-product
  int32_t* g_flag;      // per gather record
  int32_t* prog;        // chain progress: [chain * 2 + sweep], reset per launch
  int32_t* ctr;         // [0] claim counter, [1] unused, [2] error of the launch, [3] error since read, [4] left
  int64_t rstride;
  int64_t wait_ticks;
  int64_t* trace;       // debug (HLU_DEBUG_SOLVE_TRACE): 5 words per position of chain 0, or null
  void* kargs;          // device copy of a launch's arguments (kChainArgBytes)
  int32_t ntasks, L, members, max_m, max_rhs;
};

// Triangle inverses of every diagonal leaf (FP64 arithmetic, stored in T)
// and the pivots U_ii; then the stacked operators of every position.  Run
// after each factorisation.
template <class T>
hipError_t chain_prepare_launch(const T* arena, const int32_t* dims, const ChainDev& d, int32_t num_leaves,
                                hipStream_t s);

// y := U^{-1} L^{-1} y for nrhs columns (cluster order, stacked members), in
// place.
template <class T>
hipError_t chain_solve_launch(const T* arena, const int32_t* dims, const ChainDev& d, int32_t N, int32_t nrhs,
                              int32_t epoch, hipStream_t s);

}  // namespace hlu
