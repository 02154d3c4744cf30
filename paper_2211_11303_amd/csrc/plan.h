// Task plans for the H-LU factorisation, the H-triangular solves and the
// product L U, built on the host from the block tree and executed on the GPU
// as batched waves of independent tasks.
#pragma once
#include <cstdint>
#include <vector>

#include "structure.h"

namespace hlu {

// ------------------------------------------------------- device descriptors
// A strided matrix in the arena: element (i, j) at arena[off + i*rs + j*cs].
// rows/cols >= 0 are static extents; a negative value -(s+1) means the
// extent is dims[s], a rank known only on the device.
struct MatRef {
  int64_t off;
  int32_t rs, cs;
  int32_t rows, cols;
};

struct GemmTerm {  // C += alpha * A (m x k) * B (k x n)
  MatRef A, B;
  double alpha;
};
struct GemmOp {    // C = beta * C + sum of terms
  MatRef C;
  double beta;
  int32_t t0, nt;
};

enum TriMode : int32_t {
  kSolveUnitLower = 0,  // V := L^{-1} V, L = unit lower triangle of T
  kSolveUpperT = 1,     // V := U^{-T} V, U = upper triangle of T
  kSolveUpper = 2,      // V := U^{-1} V
  kMulUpper = 3,        // W := U V
  kMulUnitLower = 4     // W := L V
};
struct TriOp {
  int64_t tri;         // dense diagonal leaf (column-major, leading dim ld)
  int32_t ld, m, mode, pad;
  MatRef V, W;         // W used by the multiply modes only
};

struct GetrfOp {
  int64_t off;
  int32_t m, ld, leaf, pad;
};

struct TruncPart {   // adds alpha * Xp Yp^T, Xp placed at row_off, Yp at col_off
  MatRef X, Y;
  int32_t row_off, col_off;
  double alpha;
};
struct TruncOp {     // low-rank C (X: m x cap, Y: n x cap, rank dims[slot])
  int64_t xoff, yoff;
  int32_t m, n, ldx, ldy, slot, cap, p0, np;
};
// Launch order of the truncations of one wave, largest first: a truncation
// workgroup holds a compute unit alone and workgroups start in index order,
// so long ones (many rows, many parts) must not queue behind short ones.
// The ops of a wave touch disjoint data, so the order changes no result.
inline int64_t trunc_launch_cost(const TruncOp& t) { return (int64_t)(t.m + t.n) * (t.np + 1); }
inline bool trunc_launch_before(const TruncOp& a, const TruncOp& b) {
  return trunc_launch_cost(a) > trunc_launch_cost(b);
}
// Debug trace of a truncation op: m, n, rounds | K << 8 | r1 << 20, final
// rank | Jacobi sweeps << 16, start and end clocks, then the clocks spent in
// the Gram products, the pivoted Cholesky, the core and its compression,
// the eigensolver, the rank choice with the small products, the rebuild.
constexpr int kTruncTraceFields = 12;

struct FillOp {
  MatRef M;
  double value;
};

enum OpKind : int32_t { kGetrf = 0, kTri = 1, kGemm = 2, kTrunc = 3, kFill = 4, kNumKinds = 5 };

// Status words of a factor workspace (int32): [0] zero pivots, [1] rank
// overflows, [2] truncations past their round bound; from word kFlopWord0
// on, kFlopSpread uint64 counters per kind of the nominal flops executed
// (summed on the host).
constexpr int kStatusWords = 256;
constexpr int kFlopWord0 = 16;
constexpr int kFlopSpread = 16;
enum FlopKind : int { kFlopGetrf = 0, kFlopTri = 1, kFlopGemm = 2, kFlopTrunc = 3, kNumFlopKinds = 4 };
static_assert(kFlopWord0 + 2 * kFlopSpread * kNumFlopKinds <= kStatusWords, "status words");

// One wave: for each kind, a range of ops in the kind's array.
struct Wave {
  int32_t begin[kNumKinds];
  int32_t count[kNumKinds];
  int32_t gemm_tiles;          // sum of tiles of the wave's GEMM ops
};

struct Plan {
  std::vector<GetrfOp> getrf;
  std::vector<TriOp> tri;
  std::vector<GemmOp> gemm;
  std::vector<GemmTerm> terms;
  std::vector<TruncOp> trunc;
  std::vector<TruncPart> parts;
  std::vector<FillOp> fill;
  std::vector<int32_t> gemm_tile_op;   // per tile: gemm op index
  std::vector<int32_t> gemm_tile_ij;   // per tile: (tile_i << 16) | tile_j
  std::vector<Wave> waves;
  int64_t num_tasks = 0;
};

// Device copies of a plan's task arrays.
struct DevPlan {
  const GetrfOp* getrf;
  const TriOp* tri;
  const GemmOp* gemm;
  const GemmTerm* terms;
  const TruncOp* trunc;
  const TruncPart* parts;
  const FillOp* fill;
  const int32_t* tile_op;
  const int32_t* tile_ij;
};

// ------------------------------------------------------------ the planner
struct StoragePlan {
  // per block-tree leaf (indexed by leaf ordinal)
  std::vector<int64_t> off;     // dense: block; low-rank: X
  std::vector<int64_t> yoff;    // low-rank: Y
  std::vector<int32_t> cap;     // low-rank capacity
  std::vector<int32_t> slot;    // low-rank rank slot
  int64_t identity_off = 0;     // kIdentity x kIdentity identity matrix
  int32_t identity_n = 0;
  int64_t data_elems = 0;       // dense + low-rank + identity
  int64_t temp_elems = 0;       // factor temporaries
  int64_t solve_temp_elems = 0; // temporaries of the solve/apply plans (per rhs capacity)
  int32_t num_slots = 0;        // ranks of leaves and temporaries
  int32_t nrhs_slot = 0;        // dims slot holding the solve's column count
  int64_t vec_off = 0;          // solve vector block (N x max_rhs) in cluster order
  int64_t vec2_off = 0;         // second vector block (apply L U)
  int32_t max_rhs = 0;
  int64_t total_elems = 0;
};

// Admissible leaves that hold entries of the sparse matrix (only possible
// for small leaf clusters) start from a dense staging block that the first
// task of the factor plan truncates into low-rank form.
struct InitBlock {
  int32_t leaf;       // block-tree leaf ordinal
  int64_t off;        // staging block (m x n, column-major) in the arena
};

// Plans of the H-matrix inverse by the Schulz iteration (Sec. 3): four
// H-matrices on one block tree share the per-leaf layout of store (matrix
// m's leaf l at store.off[l] + m * mat_elems, its rank in slot
// store.slot[l] + m * mat_slots): 0 = A_H, 1 and 3 = the iterates X_k, 2 =
// Z = 2I - A_H X_k.  step[s] maps X in matrix 1 + 2s to matrix 3 - 2s
// (matrix 2 and the target zero, ranks from temp_slot0 on zero);
// apply[s] forms W = X V for X in matrix 1 + 2s (V at store.vec_off, W at
// store.vec2_off, cluster order); amul forms U = A_H W at vec3_off.
struct InversePlanSet {
  StoragePlan store;
  Plan step[2], apply[2], amul;
  int64_t mat0_off = 0;     // first element of matrix 0's leaves
  int64_t mat_elems = 0;
  int32_t mat_slots = 0;
  int32_t temp_slot0 = 0;
  int64_t vec3_off = 0;
  int32_t kcap = 64;
};

struct PlanSet {
  StoragePlan store;
  std::vector<InitBlock> init_blocks;
  Plan factor, fwd_bwd, apply;
  int32_t kcap = 64;
};

// Builds storage and the three plans.  kcap: rank capacity per block
// (capped at min(m, n)); max_rhs: column capacity of the solve plans;
// nonzero_admissible: leaf ordinals of admissible blocks holding entries.
void build_inverse_plans(const Structure& S, int32_t kcap, int32_t max_rhs, InversePlanSet* out);
// slot_cap (optional, one entry per rank slot of the factor, i.e. the
// num_slots of a plan of the same structure before the solve's slot): fitted
// capacities, each block's or temporary's capacity min(m, n, kcap, slot_cap).
void build_plans(const Structure& S, int32_t kcap, int32_t max_rhs,
                 const std::vector<int32_t>& nonzero_admissible, PlanSet* out,
                 const std::vector<int32_t>* slot_cap = nullptr);

}  // namespace hlu
