// Planner: unrolls the recursive H-LU (Algorithm 1, step II, in the 2 x 2
// block form L11 U11 = A11, U12 = L11^{-1} A12, L21 = A21 U11^{-1},
// A22 <- A22 - L21 U12, then the same on A22), the H-triangular solves of
// Algorithm 1, step III, and the product L U into lists of primitive tasks:
//
//   GETRF  unpivoted LU of a dense diagonal leaf
//   TRI    triangular solve / multiply with a dense diagonal leaf
//   GEMM   C = beta C + sum_t alpha_t A_t B_t  (one output tile list)
//   TRUNC  low-rank C <- best approximation of C + sum_p alpha_p X_p Y_p^T
//          within the block's rank rule (truncated SVD, Sec. 4)
//   FILL   constant fill
//
// Tasks are emitted in the order of the sequential recursion.  Each task
// records which memory segments it reads and writes (a segment is the part
// of a buffer that belongs to one leaf cluster in each spatial dimension);
// it is placed in the earliest wave after every earlier task it conflicts
// with (read-after-write, write-after-read, write-after-write).  Tasks of
// one wave touch disjoint data and run as batched launches, so executing the
// waves in order gives exactly the sequential result.
//
// Products of H-blocks with blocks of vectors (H-matrix times matrix) are
// emitted in two phases: first T_l = Y_l^T V for every low-rank leaf l, then
// one GEMM task per leaf-cluster segment of the output that sums all dense
// leaf products D V and low-rank products X_l T_l landing there.
#include "plan.h"

#include <algorithm>
#include <climits>
#include <map>
#include <queue>
#include <set>
#include <tuple>

#include "common.h"

namespace hlu {
namespace {

constexpr int kTile = 64;

struct Buf {
  int32_t rl0, nrl;   // first leaf ordinal and count along buffer rows (nrl = 0: not spatial)
  int32_t cl0, ncl;   // same along buffer columns
  int64_t seg0;
};

struct View {
  int64_t off;
  int32_t rs, cs;
  int32_t rows, cols;       // logical dim codes
  int32_t rows_s, cols_s;   // logical static extents (capacities)
  int32_t r0, c0;           // logical absolute positions of row/col 0 (-1: not spatial)
  int32_t buf;              // -1: constant data, not tracked
  bool tr;                  // logical = transpose of the buffer orientation
  MatRef ref() const { return MatRef{off, rs, cs, rows, cols}; }
};

View transpose(View v) {
  std::swap(v.rs, v.cs);
  std::swap(v.rows, v.cols);
  std::swap(v.rows_s, v.cols_s);
  std::swap(v.r0, v.c0);
  v.tr = !v.tr;
  return v;
}

View sub_rows(View v, int32_t a0, int32_t a1) {
  HLU_REQUIRE(v.r0 >= 0 && a0 >= v.r0 && a1 <= v.r0 + v.rows_s && a0 < a1, HLU_ERR_INVALID_ARG,
              "planner: bad row restriction");
  v.off += (int64_t)(a0 - v.r0) * v.rs;
  v.rows = v.rows_s = a1 - a0;
  v.r0 = a0;
  return v;
}

View sub_cols(View v, int32_t a0, int32_t a1) {
  HLU_REQUIRE(v.c0 >= 0 && a0 >= v.c0 && a1 <= v.c0 + v.cols_s && a0 < a1, HLU_ERR_INVALID_ARG,
              "planner: bad column restriction");
  v.off += (int64_t)(a0 - v.c0) * v.cs;
  v.cols = v.cols_s = a1 - a0;
  v.c0 = a0;
  return v;
}

int32_t dyn(int32_t slot) { return -(slot + 1); }

// H-block handle: a node of the block tree or a temporary low-rank block.
struct HB {
  BlockKind kind;
  int32_t node;      // block-tree node id (-1 for a quadrant of a low-rank block)
  int32_t r0, r1, c0, c1;
  View D, X, Y;      // storage of leaves
  int32_t slot = -1, cap = 0;
  // low-rank updates land in the low-rank leaf `root` (a block-tree node),
  // at row/column offset (roff, coff) inside it
  int32_t root = -1, roff = 0, coff = 0;
  int32_t mat = 0;   // which H-matrix on the block tree (several share one layout)
};

struct Access {
  View v;
  bool write;
};

class Planner {
 public:
  Planner(const Structure& S, StoragePlan& st) : S_(S), st_(st) {
    leaf_of_pos_.resize(S.N);
    for (size_t l = 0; l < S.leaf_clusters.size(); ++l) {
      const ClusterNode& c = S.clusters[S.leaf_clusters[l]];
      for (int32_t p = c.begin; p < c.end; ++p) leaf_of_pos_[p] = (int32_t)l;
    }
  }

  // ------------------------------------------------------------ storage
  // Storage of `nmat` H-matrices on the block tree, one after the other
  // with the same per-leaf layout (matrix m's leaf storage and rank slots are
  // matrix 0's shifted by m * mat_stride_ and m * mat_slots_), then the
  // staging blocks of matrix 0's admissible blocks that hold entries.
  void layout(int32_t kcap, const std::vector<int32_t>& nz_adm, std::vector<InitBlock>* inits, int32_t nmat = 1) {
    const int32_t nleaf = (int32_t)S_.leaves.size();
    st_.off.assign(nleaf, -1);
    st_.yoff.assign(nleaf, -1);
    st_.cap.assign(nleaf, 0);
    st_.slot.assign(nleaf, -1);
    int64_t top = 0;
    int32_t slots = 0;
    leaf_buf_.assign(nleaf, -1);
    leaf_ybuf_.assign(nleaf, -1);
    int32_t maxleaf = 1;
    for (int32_t c : S_.leaf_clusters) maxleaf = std::max(maxleaf, S_.clusters[c].size());
    for (int32_t l : nz_adm) {
      const BlockNode& b = S_.blocks[S_.leaves[l]];
      maxleaf = std::max(maxleaf, std::min(S_.clusters[b.row].size(), S_.clusters[b.col].size()));
    }
    st_.identity_n = maxleaf;
    st_.identity_off = top;
    top += align((int64_t)maxleaf * maxleaf);
    const int64_t mat_begin = top;
    for (int32_t l = 0; l < nleaf; ++l) {
      const BlockNode& b = S_.blocks[S_.leaves[l]];
      const ClusterNode& rc = S_.clusters[b.row];
      const ClusterNode& cc = S_.clusters[b.col];
      const int32_t m = rc.size(), n = cc.size();
      if (b.kind == kDense) {
        st_.off[l] = top;
        top += align((int64_t)m * n);
        leaf_buf_[l] = new_buf(rc.leaf_first, rc.leaf_last - rc.leaf_first, cc.leaf_first,
                               cc.leaf_last - cc.leaf_first);
      } else {
        const int32_t cap = cap_for(m, n, kcap, slots);
        st_.cap[l] = cap;
        st_.slot[l] = slots++;
        st_.off[l] = top;
        top += align((int64_t)m * cap);
        st_.yoff[l] = top;
        top += align((int64_t)n * cap);
        leaf_buf_[l] = new_buf(rc.leaf_first, rc.leaf_last - rc.leaf_first, 0, 0);
        leaf_ybuf_[l] = new_buf(cc.leaf_first, cc.leaf_last - cc.leaf_first, 0, 0);
      }
    }
    mat_begin_ = mat_begin;
    mat_stride_ = top - mat_begin;
    mat_slots_ = slots;
    mbuf_.assign(nmat, leaf_buf_);
    mybuf_.assign(nmat, leaf_ybuf_);
    for (int32_t m = 1; m < nmat; ++m) {
      for (int32_t l = 0; l < nleaf; ++l) {
        const BlockNode& b = S_.blocks[S_.leaves[l]];
        const ClusterNode& rc = S_.clusters[b.row];
        const ClusterNode& cc = S_.clusters[b.col];
        if (b.kind == kDense) {
          mbuf_[m][l] = new_buf(rc.leaf_first, rc.leaf_last - rc.leaf_first, cc.leaf_first,
                                cc.leaf_last - cc.leaf_first);
        } else {
          mbuf_[m][l] = new_buf(rc.leaf_first, rc.leaf_last - rc.leaf_first, 0, 0);
          mybuf_[m][l] = new_buf(cc.leaf_first, cc.leaf_last - cc.leaf_first, 0, 0);
        }
      }
      top += mat_stride_;
      slots += mat_slots_;
    }
    for (int32_t l : nz_adm) {
      const BlockNode& b = S_.blocks[S_.leaves[l]];
      HLU_REQUIRE(b.kind == kLowRank, HLU_ERR_INVALID_ARG, "planner: init block is not admissible");
      const ClusterNode& rc = S_.clusters[b.row];
      const ClusterNode& cc = S_.clusters[b.col];
      InitBlock ib{l, top};
      top += align((int64_t)rc.size() * cc.size());
      inits->push_back(ib);
      init_buf_.push_back(new_buf(rc.leaf_first, rc.leaf_last - rc.leaf_first, cc.leaf_first,
                                  cc.leaf_last - cc.leaf_first));
    }
    st_.data_elems = top;
    st_.num_slots = slots;
    persistent_bufs_ = (int32_t)bufs_.size();
    persistent_segs_ = nseg_;
  }

  HB block(int32_t node, int32_t mat = 0) const {
    const BlockNode& b = S_.blocks[node];
    const ClusterNode& rc = S_.clusters[b.row];
    const ClusterNode& cc = S_.clusters[b.col];
    HB h;
    h.kind = b.kind;
    h.node = node;
    h.r0 = rc.begin;
    h.r1 = rc.end;
    h.c0 = cc.begin;
    h.c1 = cc.end;
    h.mat = mat;
    const int32_t m = rc.size(), n = cc.size();
    const int64_t shift = (int64_t)mat * mat_stride_;
    if (b.kind == kDense) {
      const int32_t l = b.leaf_id;
      h.D = View{st_.off[l] + shift, 1, m, m, n, m, n, rc.begin, cc.begin, mbuf_[mat][l], false};
    } else if (b.kind == kLowRank) {
      const int32_t l = b.leaf_id;
      h.slot = st_.slot[l] + mat * mat_slots_;
      h.cap = st_.cap[l];
      h.X = View{st_.off[l] + shift, 1, m, m, dyn(h.slot), m, h.cap, rc.begin, -1, mbuf_[mat][l], false};
      h.Y = View{st_.yoff[l] + shift, 1, n, n, dyn(h.slot), n, h.cap, cc.begin, -1, mybuf_[mat][l], false};
      h.root = node;
    }
    return h;
  }

  HB son(const HB& h, int i, int j) const { return block(S_.blocks[h.node].son[2 * i + j], h.mat); }

  View identity(int32_t n) const {
    return View{st_.identity_off, 1, st_.identity_n, n, n, n, n, -1, -1, -1, false};
  }

  // --------------------------------------------------------- plan control
  void begin_plan(Plan* P, int64_t temp_base) {
    P_ = P;
    bufs_.resize(persistent_bufs_);
    nseg_ = persistent_segs_;
    last_w_.assign(nseg_, -1);
    last_r_.assign(nseg_, -1);
    temp_base_ = temp_base;
    temp_top_ = temp_base;
    temps_.clear();
    temp_of_buf_.clear();
    max_peak_ = 0;
    ops_.clear();
    max_wave_ = -1;
  }

  // Sort the emitted tasks into waves and fill the plan arrays.
  void end_plan() {
    Plan& P = *P_;
    temp_peak_ = assign_temps();
    remap_plan(P);
    // bucket the tasks by (wave, kind), keeping program order inside a bucket
    const int32_t nw = max_wave_ + 1;
    std::vector<int64_t> start((size_t)nw * kNumKinds + 1, 0);
    for (const Rec& r : ops_) start[(size_t)r.wave * kNumKinds + r.kind + 1]++;
    for (size_t i = 1; i < start.size(); ++i) start[i] += start[i - 1];
    std::vector<int32_t> sorted(ops_.size());
    {
      std::vector<int64_t> fillp(start.begin(), start.end() - 1);
      for (size_t i = 0; i < ops_.size(); ++i) {
        const Rec& r = ops_[i];
        sorted[fillp[(size_t)r.wave * kNumKinds + r.kind]++] = (int32_t)i;
      }
    }
    std::vector<GetrfOp> getrf;
    std::vector<TriOp> tri;
    std::vector<GemmOp> gemm;
    std::vector<TruncOp> trunc;
    std::vector<FillOp> fill;
    getrf.reserve(P.getrf.size());
    tri.reserve(P.tri.size());
    gemm.reserve(P.gemm.size());
    trunc.reserve(P.trunc.size());
    fill.reserve(P.fill.size());
    P.waves.assign(nw, Wave{});
    for (int32_t w = 0; w < nw; ++w) {
      Wave& W = P.waves[w];
      W.gemm_tiles = 0;
      for (int k = 0; k < kNumKinds; ++k) {
        const int64_t b0 = start[(size_t)w * kNumKinds + k], b1 = start[(size_t)w * kNumKinds + k + 1];
        switch (k) {
          case kGetrf: W.begin[k] = (int32_t)getrf.size(); break;
          case kTri: W.begin[k] = (int32_t)tri.size(); break;
          case kGemm: W.begin[k] = (int32_t)gemm.size(); break;
          case kTrunc: W.begin[k] = (int32_t)trunc.size(); break;
          default: W.begin[k] = (int32_t)fill.size(); break;
        }
        W.count[k] = (int32_t)(b1 - b0);
        for (int64_t q = b0; q < b1; ++q) {
          const Rec& r = ops_[sorted[q]];
          switch (k) {
            case kGetrf: getrf.push_back(P.getrf[r.idx]); break;
            case kTri: tri.push_back(P.tri[r.idx]); break;
            case kGemm: {
              const GemmOp& g = P.gemm[r.idx];
              const int32_t gi = (int32_t)gemm.size();
              gemm.push_back(g);
              const int32_t rs = cap_of(g.C.rows, r.rows_s), cs = cap_of(g.C.cols, r.cols_s);
              const int32_t ti = (rs + kTile - 1) / kTile, tj = (cs + kTile - 1) / kTile;
              for (int32_t a = 0; a < ti; ++a)
                for (int32_t b = 0; b < tj; ++b) {
                  P.gemm_tile_op.push_back(gi);
                  P.gemm_tile_ij.push_back((a << 16) | b);
                }
              W.gemm_tiles += ti * tj;
              break;
            }
            case kTrunc: trunc.push_back(P.trunc[r.idx]); break;
            default: fill.push_back(P.fill[r.idx]); break;
          }
        }
        if (k == kTrunc) std::stable_sort(trunc.begin() + W.begin[k], trunc.end(), trunc_launch_before);
      }
    }
    P.getrf.swap(getrf);
    P.tri.swap(tri);
    P.gemm.swap(gemm);
    P.trunc.swap(trunc);
    P.fill.swap(fill);
    P.num_tasks = (int64_t)ops_.size();
  }

  int64_t temp_used() const { return temp_peak_; }

  // ----------------------------------------------------- the factorisation
  // Algorithm 1, step I for admissible blocks holding matrix entries: the
  // staged dense block S becomes S I^T (or I S^T^T), truncated.
  void init_lowrank(const std::vector<InitBlock>& inits) {
    for (size_t i = 0; i < inits.size(); ++i) {
      const BlockNode& b = S_.blocks[S_.leaves[inits[i].leaf]];
      HB C = block(S_.leaves[inits[i].leaf]);
      const int32_t m = C.r1 - C.r0, n = C.c1 - C.c0;
      View Sv{inits[i].off, 1, m, m, n, m, n, C.r0, C.c0, init_buf_[i], false};
      (void)b;
      if (n <= m) defer(C, Sv, identity(n), 1.0);
      else defer(C, identity(m), transpose(Sv), 1.0);
    }
  }

  void hlu(const HB& D) {
    if (D.kind == kDense) {
      GetrfOp g{D.D.off, D.D.rows, D.D.cs, S_.blocks[D.node].leaf_id, 0};
      emit(kGetrf, (int32_t)P_->getrf.size(), {{D.D, true}}, 0, 0);
      P_->getrf.push_back(g);
      return;
    }
    HB D00 = son(D, 0, 0), D01 = son(D, 0, 1), D10 = son(D, 1, 0), D11 = son(D, 1, 1);
    hlu(D00);
    trsm_lower(D00, D01);
    trsm_upper(D00, D10);
    gemm(D11, D10, D01);
    hlu(D11);
  }

  void trsm_lower(const HB& Ld, const HB& B) {
    if (B.kind == kLowRank) {
      flush(B);
      hsolve_lower(Ld, B.X);
    } else if (B.kind == kDense) {
      hsolve_lower(Ld, B.D);
    } else {
      HB L00 = son(Ld, 0, 0), L10 = son(Ld, 1, 0), L11 = son(Ld, 1, 1);
      for (int j = 0; j < 2; ++j) {
        HB B0 = son(B, 0, j), B1 = son(B, 1, j);
        trsm_lower(L00, B0);
        gemm(B1, L10, B0);
        trsm_lower(L11, B1);
      }
    }
  }

  void trsm_upper(const HB& Ud, const HB& B) {
    if (B.kind == kLowRank) {
      flush(B);
      hsolve_upper_T(Ud, B.Y);
    } else if (B.kind == kDense) {
      hsolve_upper_T(Ud, transpose(B.D));
    } else {
      HB U00 = son(Ud, 0, 0), U01 = son(Ud, 0, 1), U11 = son(Ud, 1, 1);
      for (int i = 0; i < 2; ++i) {
        HB B0 = son(B, i, 0), B1 = son(B, i, 1);
        trsm_upper(U00, B0);
        gemm(B1, B0, U01);
        trsm_upper(U11, B1);
      }
    }
  }

  // V := L^{-1} V in place (V's rows = the diagonal block's rows)
  void hsolve_lower(const HB& Ld, const View& V) {
    if (Ld.kind == kDense) {
      tri_op(kSolveUnitLower, Ld, V, V);
      return;
    }
    HB L00 = son(Ld, 0, 0), L10 = son(Ld, 1, 0), L11 = son(Ld, 1, 1);
    View V0 = sub_rows(V, L00.r0, L00.r1), V1 = sub_rows(V, L11.r0, L11.r1);
    hsolve_lower(L00, V0);
    hmv(L10, false, V0, V1, -1.0, 1.0);
    hsolve_lower(L11, V1);
  }

  // V := U^{-T} V in place
  void hsolve_upper_T(const HB& Ud, const View& V) {
    if (Ud.kind == kDense) {
      tri_op(kSolveUpperT, Ud, V, V);
      return;
    }
    HB U00 = son(Ud, 0, 0), U01 = son(Ud, 0, 1), U11 = son(Ud, 1, 1);
    View V0 = sub_rows(V, U00.r0, U00.r1), V1 = sub_rows(V, U11.r0, U11.r1);
    hsolve_upper_T(U00, V0);
    hmv(U01, true, V0, V1, -1.0, 1.0);
    hsolve_upper_T(U11, V1);
  }

  // V := U^{-1} V in place
  void hsolve_upper(const HB& Ud, const View& V) {
    if (Ud.kind == kDense) {
      tri_op(kSolveUpper, Ud, V, V);
      return;
    }
    HB U00 = son(Ud, 0, 0), U01 = son(Ud, 0, 1), U11 = son(Ud, 1, 1);
    View V0 = sub_rows(V, U00.r0, U00.r1), V1 = sub_rows(V, U11.r0, U11.r1);
    hsolve_upper(U11, V1);
    hmv(U01, false, V1, V0, -1.0, 1.0);
    hsolve_upper(U00, V0);
  }

  // W := U V (upper triangle of the diagonal block, diagonal included)
  void apply_upper(const HB& Ud, const View& V, const View& W) {
    if (Ud.kind == kDense) {
      tri_op(kMulUpper, Ud, V, W);
      return;
    }
    HB U00 = son(Ud, 0, 0), U01 = son(Ud, 0, 1), U11 = son(Ud, 1, 1);
    apply_upper(U00, sub_rows(V, U00.r0, U00.r1), sub_rows(W, U00.r0, U00.r1));
    hmv(U01, false, sub_rows(V, U11.r0, U11.r1), sub_rows(W, U00.r0, U00.r1), 1.0, 1.0);
    apply_upper(U11, sub_rows(V, U11.r0, U11.r1), sub_rows(W, U11.r0, U11.r1));
  }

  // W := L V (unit lower triangle of the diagonal block)
  void apply_lower(const HB& Ld, const View& V, const View& W) {
    if (Ld.kind == kDense) {
      tri_op(kMulUnitLower, Ld, V, W);
      return;
    }
    HB L00 = son(Ld, 0, 0), L10 = son(Ld, 1, 0), L11 = son(Ld, 1, 1);
    apply_lower(L00, sub_rows(V, L00.r0, L00.r1), sub_rows(W, L00.r0, L00.r1));
    apply_lower(L11, sub_rows(V, L11.r0, L11.r1), sub_rows(W, L11.r0, L11.r1));
    hmv(L10, false, sub_rows(V, L00.r0, L00.r1), sub_rows(W, L11.r0, L11.r1), 1.0, 1.0);
  }

  // C += alpha A B in H-arithmetic (alpha = -1: the H-LU's update).
  void gemm(const HB& C, const HB& A, const HB& B, double alpha = -1.0) {
    if (A.kind == kLowRank) flush(A);
    if (B.kind == kLowRank) flush(B);
    if (A.kind == kLowRank) {
      View W = temp_spatial(C.c0, C.c1 - C.c0, A.X.cols, A.cap);
      hmv(B, true, A.Y, W, 1.0, 0.0);
      add_lowrank(C, A.X, W, alpha);
    } else if (B.kind == kLowRank) {
      View W = temp_spatial(C.r0, C.r1 - C.r0, B.X.cols, B.cap);
      hmv(A, false, B.X, W, 1.0, 0.0);
      add_lowrank(C, W, B.Y, alpha);
    } else if (A.kind == kDense && B.kind == kDense) {
      if (C.kind == kDense) {
        gemm_op(C.D, 1.0, {{A.D, B.D, alpha}});
      } else {
        add_lowrank(C, A.D, transpose(B.D), alpha);
      }
    } else if (A.kind == kDense) {  // B subdivided: rows of C form a leaf cluster
      if (C.kind == kDense) {
        hmv(B, true, transpose(A.D), transpose(C.D), alpha, 1.0);
      } else {
        View W = temp_spatial(C.c0, C.c1 - C.c0, A.D.rows, A.D.rows_s);
        hmv(B, true, transpose(A.D), W, 1.0, 0.0);
        add_lowrank(C, identity(A.D.rows), W, alpha);
      }
    } else if (B.kind == kDense) {  // A subdivided: cols of C form a leaf cluster
      if (C.kind == kDense) {
        hmv(A, false, B.D, C.D, alpha, 1.0);
      } else {
        View W = temp_spatial(C.r0, C.r1 - C.r0, B.D.cols, B.D.cols_s);
        hmv(A, false, B.D, W, 1.0, 0.0);
        add_lowrank(C, W, identity(B.D.cols), alpha);
      }
    } else if (C.kind == kSub) {
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
          for (int k = 0; k < 2; ++k) gemm(son(C, i, j), son(A, i, k), son(B, k, j), alpha);
    } else if (C.kind == kLowRank) {
      // both factors subdivided, low-rank target: accumulate the product on
      // the four quadrants as temporary low-rank blocks, then add them to C
      // with one truncation.
      std::vector<PartSpec> parts;
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          HB Ai0 = son(A, i, 0), B0j = son(B, 0, j);
          HB Q = temp_lowrank(Ai0.r0, Ai0.r1, B0j.c0, B0j.c1);
          for (int k = 0; k < 2; ++k) gemm(Q, son(A, i, k), son(B, k, j), alpha);
          flush(Q);
          parts.push_back({Q.X, Q.Y, C.roff + Q.r0 - C.r0, C.coff + Q.c0 - C.c0, 1.0});
        }
      flush(C);
      trunc_op(root_of(C), parts);
    } else {
      fail(HLU_ERR_INVALID_ARG, "planner: dense target with two subdivided factors");
    }
  }

  // One Schulz step (Sec. 3) between matrices of the layout: with A_H in
  // matrix 0, X_k in matrix xin and matrices 2 and xout zero,
  //   Z := -A_H X_k;  Z += 2 I;  X_{k+1} := X_k Z    (Z in matrix 2).
  void schulz_step(int32_t xin, int32_t xout) {
    gemm(block(0, 2), block(0, 0), block(0, xin), -1.0);
    flush_all();
    for (size_t l = 0; l < S_.leaves.size(); ++l) {
      const BlockNode& b = S_.blocks[S_.leaves[l]];
      if (b.row != b.col) continue;
      const HB d = block(S_.leaves[l], 2);
      const int32_t m = d.r1 - d.r0;
      gemm_op(d.D, 1.0, {{identity(m), identity(m), 2.0}});
    }
    gemm(block(0, xout), block(0, xin), block(0, 2), 1.0);
    flush_all();
  }

  int64_t mat_stride() const { return mat_stride_; }
  int64_t mat_begin() const { return mat_begin_; }
  int32_t mat_slots() const { return mat_slots_; }

  // C += alpha X Y^T, truncating in every low-rank leaf of C.
  void add_lowrank(const HB& C, const View& X, const View& Y, double alpha) {
    if (C.kind == kDense) {
      gemm_op(C.D, 1.0, {{X, transpose(Y), alpha}});
    } else if (C.kind == kLowRank) {
      defer(C, X, Y, alpha);
    } else {
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          HB s = son(C, i, j);
          add_lowrank(s, rows_of(X, C.r0, s.r0, s.r1), rows_of(Y, C.c0, s.c0, s.c1), alpha);
        }
    }
  }

  // W = beta W + alpha op(B) V, op(B) = B or B^T, for an H-block B.
  void hmv(const HB& B, bool trans, const View& V, const View& W, double alpha, double beta) {
    std::vector<HB> lv;
    collect_leaves(B, &lv);
    for (const HB& l : lv)
      if (l.kind == kLowRank) flush(l);
    const int32_t out0 = trans ? B.c0 : B.r0, out1 = trans ? B.c1 : B.r1;
    const int32_t in0 = trans ? B.r0 : B.c0;
    const int32_t lf0 = leaf_of_pos_[out0], lf1 = leaf_of_pos_[out1 - 1] + 1;
    std::vector<std::vector<TermSpec>> seg_terms(lf1 - lf0);
    // V rows are indexed by in-positions; W rows by out-positions
    auto Vin = [&](int32_t a0, int32_t a1) { return rows_of(V, in0, a0, a1); };
    for (const HB& l : lv) {
      const int32_t lo0 = trans ? l.c0 : l.r0, lo1 = trans ? l.c1 : l.r1;
      const int32_t li0 = trans ? l.r0 : l.c0, li1 = trans ? l.r1 : l.c1;
      if (l.kind == kDense) {
        View A = trans ? transpose(l.D) : l.D;   // rows = out positions
        View Vl = Vin(li0, li1);
        for (int32_t f = leaf_of_pos_[lo0]; f <= leaf_of_pos_[lo1 - 1]; ++f) {
          const ClusterNode& c = S_.clusters[S_.leaf_clusters[f]];
          seg_terms[f - lf0].push_back({sub_rows(A, c.begin, c.end), Vl, alpha});
        }
      } else {
        // phase 1: T = (trans ? X : Y)^T V_l   (rank x p)
        View F = trans ? l.X : l.Y;   // rows = in positions
        View G = trans ? l.Y : l.X;   // rows = out positions
        View T = temp_plain(F.cols, l.cap, V.cols, V.cols_s);
        gemm_op(T, 0.0, {{transpose(F), Vin(li0, li1), 1.0}});
        for (int32_t f = leaf_of_pos_[lo0]; f <= leaf_of_pos_[lo1 - 1]; ++f) {
          const ClusterNode& c = S_.clusters[S_.leaf_clusters[f]];
          seg_terms[f - lf0].push_back({sub_rows(G, c.begin, c.end), T, alpha});
        }
      }
    }
    // phase 2: one task per output segment
    for (int32_t f = lf0; f < lf1; ++f) {
      const ClusterNode& c = S_.clusters[S_.leaf_clusters[f]];
      gemm_op(rows_of(W, out0, c.begin, c.end), beta, seg_terms[f - lf0]);
    }
  }

 private:
  struct TermSpec {
    View A, B;
    double alpha;
  };
  struct PartSpec {
    View X, Y;
    int32_t row_off, col_off;
    double alpha;
  };
  struct Rec {
    int32_t kind, idx, wave;
    int32_t rows_s, cols_s;
  };

  static int64_t align(int64_t e) { return (e + 31) & ~int64_t(31); }

  static int32_t cap_of(int32_t code, int32_t s) { return code >= 0 ? code : s; }

  // rank capacity of a low-rank block or temporary m x n with rank slot
  // `slot`: min(m, n, kcap), lowered to the slot's fitted capacity if given
  int32_t cap_for(int32_t m, int32_t n, int32_t kcap, int32_t slot) const {
    int32_t c = std::min(std::min(m, n), kcap);
    if (slot_cap_ && slot < (int32_t)slot_cap_->size()) c = std::min(c, (*slot_cap_)[slot]);
    return std::max(1, c);
  }

  // restriction of a view whose row 0 sits at absolute position base
  View rows_of(const View& v, int32_t base, int32_t a0, int32_t a1) const {
    if (v.r0 >= 0) return sub_rows(v, a0, a1);
    // a non-spatial view (identity): plain row offset
    View w = v;
    w.off += (int64_t)(a0 - base) * v.rs;
    w.rows = w.rows_s = a1 - a0;
    return w;
  }

  void collect_leaves(const HB& B, std::vector<HB>* out) const {
    if (B.kind != kSub) {
      out->push_back(B);
      return;
    }
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) collect_leaves(son(B, i, j), out);
  }

  int32_t new_buf(int32_t rl0, int32_t nrl, int32_t cl0, int32_t ncl) {
    Buf b{rl0, nrl, cl0, ncl, nseg_};
    nseg_ += (int64_t)std::max(nrl, 1) * std::max(ncl, 1);
    bufs_.push_back(b);
    return (int32_t)bufs_.size() - 1;
  }

  // temporary with spatial rows [pos0, pos0 + m) and `cols` columns
  View temp_spatial(int32_t pos0, int32_t m, int32_t cols, int32_t cols_s) {
    const int32_t lf0 = leaf_of_pos_[pos0], lf1 = leaf_of_pos_[pos0 + m - 1] + 1;
    int32_t b = new_buf(lf0, lf1 - lf0, 0, 0);
    grow_segments();
    View v{temp_top_, 1, m, m, cols, m, cols_s, pos0, -1, b, false};
    add_temp(b, align((int64_t)m * std::max(cols_s, 1)));
    return v;
  }

  View temp_plain(int32_t rows, int32_t rows_s, int32_t cols, int32_t cols_s) {
    int32_t b = new_buf(0, 0, 0, 0);
    grow_segments();
    const int32_t ld = std::max(rows_s, 1);
    View v{temp_top_, 1, ld, rows, cols, rows_s, cols_s, -1, -1, b, false};
    add_temp(b, align((int64_t)ld * std::max(cols_s, 1)));
    return v;
  }

  struct Temp {
    int64_t vbegin, size;
    int32_t first = INT32_MAX, last = -1;
    int64_t phys = -1;
  };

  void add_temp(int32_t buf, int64_t size) {
    if ((int32_t)temp_of_buf_.size() <= buf) temp_of_buf_.resize(buf + 1, -1);
    temp_of_buf_[buf] = (int32_t)temps_.size();
    temps_.push_back(Temp{temp_top_, size});
    temp_top_ += size;
  }

  // Give every temporary physical memory, reusing space of temporaries whose
  // last task ran in an earlier wave (best fit, coalescing free ranges);
  // returns the peak size.
  int64_t assign_temps() {
    std::vector<int32_t> order;
    order.reserve(temps_.size());
    for (size_t i = 0; i < temps_.size(); ++i) {
      if (temps_[i].last < 0) temps_[i].phys = 0;   // never touched
      else order.push_back((int32_t)i);
    }
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
      return temps_[a].first != temps_[b].first ? temps_[a].first < temps_[b].first : a < b;
    });
    // free ranges, by offset (-> size, insertion order) and by (size,
    // insertion order, offset): best fit takes the smallest size that fits,
    // the oldest free range among equal sizes
    using Key = std::tuple<int64_t, int64_t, int64_t>;
    std::map<int64_t, std::pair<int64_t, int64_t>> by_off;
    std::set<Key> by_size;
    int64_t seq = 0;
    auto add_free = [&](int64_t off, int64_t size) {
      by_off[off] = {size, seq};
      by_size.insert(Key{size, seq, off});
      ++seq;
    };
    auto erase_size = [&](std::map<int64_t, std::pair<int64_t, int64_t>>::iterator it) {
      by_size.erase(Key{it->second.first, it->second.second, it->first});
    };
    int64_t peak = 0;
    auto release = [&](int64_t off, int64_t size) {
      auto next = by_off.lower_bound(off);
      if (next != by_off.end() && next->first == off + size) {
        size += next->second.first;
        erase_size(next);
        next = by_off.erase(next);
      }
      if (next != by_off.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second.first == off) {
          erase_size(prev);
          off = prev->first;
          size += prev->second.first;
          by_off.erase(prev);
        }
      }
      if (off + size == peak) {   // give it back to the top
        peak = off;
        return;
      }
      add_free(off, size);
    };
    using Ev = std::pair<int32_t, int32_t>;   // (last wave, temp)
    std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> live;
    for (int32_t t : order) {
      Temp& T = temps_[t];
      while (!live.empty() && live.top().first < T.first) {
        const Temp& L = temps_[live.top().second];
        release(L.phys, L.size);
        live.pop();
      }
      auto it = by_size.lower_bound(Key{T.size, INT64_MIN, INT64_MIN});
      if (it != by_size.end()) {
        const int64_t size = std::get<0>(*it), off = std::get<2>(*it);
        by_size.erase(it);
        by_off.erase(off);
        T.phys = off;
        if (size > T.size) add_free(off + T.size, size - T.size);
      } else {
        T.phys = peak;
        peak += T.size;
      }
      max_peak_ = std::max(max_peak_, peak);
      live.push({T.last, t});
    }
    return max_peak_;
  }

  // Physical offset of a virtual temporary offset: the temporary is found
  // by binary search over the (increasing) virtual begins, kept in their own
  // dense array while the plan is remapped.
  int64_t remap(int64_t off) const {
    if (off < temp_base_ || off >= temp_top_ || temps_.empty()) return off;
    const size_t u = (size_t)(std::upper_bound(vbegin_.begin(), vbegin_.end(), off) - vbegin_.begin());
    const size_t t = u > 0 ? u - 1 : 0;
    return temp_base_ + temps_[t].phys + (off - vbegin_[t]);
  }

  void remap_plan(Plan& P) {
    vbegin_.resize(temps_.size());
    for (size_t i = 0; i < temps_.size(); ++i) vbegin_[i] = temps_[i].vbegin;
    auto R = [&](MatRef& m) { m.off = remap(m.off); };
    for (auto& g : P.gemm) R(g.C);
    for (auto& t : P.terms) {
      R(t.A);
      R(t.B);
    }
    for (auto& t : P.tri) {
      R(t.V);
      R(t.W);
    }
    for (auto& t : P.trunc) {
      t.xoff = remap(t.xoff);
      t.yoff = remap(t.yoff);
    }
    for (auto& p : P.parts) {
      R(p.X);
      R(p.Y);
    }
    for (auto& f : P.fill) R(f.M);
    std::vector<int64_t>().swap(vbegin_);
  }

  HB temp_lowrank(int32_t r0, int32_t r1, int32_t c0, int32_t c1) {
    HB h;
    h.kind = kLowRank;
    h.node = -1;
    h.r0 = r0;
    h.r1 = r1;
    h.c0 = c0;
    h.c1 = c1;
    const int32_t m = r1 - r0, n = c1 - c0;
    h.slot = st_.num_slots++;
    h.cap = cap_for(m, n, kcap_, h.slot);
    h.X = temp_spatial(r0, m, dyn(h.slot), h.cap);
    h.Y = temp_spatial(c0, n, dyn(h.slot), h.cap);
    h.root = -2 - h.slot;              // temporaries are their own root
    temp_hb_[h.root] = h;
    return h;
  }

  HB root_of(const HB& C) const {
    if (C.root >= 0) return block(C.root, C.mat);
    return temp_hb_.at(C.root);
  }

  // key of a low-rank root among the pending updates: block-tree node and
  // matrix, or the (negative) id of a temporary
  int64_t root_key(const HB& C) const {
    return C.root >= 0 ? (int64_t)C.mat * (int64_t)S_.blocks.size() + C.root : (int64_t)C.root;
  }
  HB root_of_key(int64_t key) const {
    HB h;
    if (key >= 0) {
      h.root = (int32_t)(key % (int64_t)S_.blocks.size());
      h.mat = (int32_t)(key / (int64_t)S_.blocks.size());
    } else {
      h.root = (int32_t)key;
    }
    return h;
  }

  HB quadrant(const HB& C, int32_t r0, int32_t r1, int32_t c0, int32_t c1) const {
    HB q;
    q.kind = kLowRank;
    q.node = -1;
    q.r0 = r0;
    q.r1 = r1;
    q.c0 = c0;
    q.c1 = c1;
    q.root = C.root;
    q.mat = C.mat;
    q.roff = C.roff + (r0 - C.r0);
    q.coff = C.coff + (c0 - C.c0);
    return q;
  }

 public:
  // Record the low-rank term alpha X Y^T of the low-rank leaf (or quadrant
  // of a leaf) C; the recorded terms are truncated into C together when C
  // is next read or when kMaxPending terms have accumulated.
  static constexpr size_t kMaxPending = 1;
  void defer(const HB& C, const View& X, const View& Y, double alpha) {
    auto& v = pending_[root_key(C)];
    v.push_back({X, Y, C.roff, C.coff, alpha});
    if (v.size() >= kMaxPending) flush(C);
  }

  void flush(const HB& C) {
    if (C.root == -1) return;
    auto it = pending_.find(root_key(C));
    if (it == pending_.end()) return;
    std::vector<PartSpec> parts;
    parts.swap(it->second);
    pending_.erase(it);
    trunc_op(root_of(C), parts);
  }

  void flush_all() {
    std::vector<int64_t> keys;
    for (auto& kv : pending_) keys.push_back(kv.first);
    std::sort(keys.begin(), keys.end());
    for (int64_t k : keys) flush(root_of_key(k));
  }

 private:
  void grow_segments() {
    if ((int64_t)last_w_.size() < nseg_) {
      last_w_.resize(nseg_, -1);
      last_r_.resize(nseg_, -1);
    }
  }

  template <class F>
  void for_segments(const View& v, F f) const {
    if (v.buf < 0) return;
    const Buf& b = bufs_[v.buf];
    // buffer orientation
    const int32_t br0 = v.tr ? v.c0 : v.r0, brs = v.tr ? v.cols_s : v.rows_s;
    const int32_t bc0 = v.tr ? v.r0 : v.c0, bcs = v.tr ? v.rows_s : v.cols_s;
    int32_t rlo = 0, rhi = 1, clo = 0, chi = 1;
    if (b.nrl > 0) {
      if (br0 >= 0) {
        rlo = leaf_of_pos_[br0] - b.rl0;
        rhi = leaf_of_pos_[br0 + brs - 1] - b.rl0 + 1;
      } else {
        rhi = b.nrl;
      }
    }
    if (b.ncl > 0) {
      if (bc0 >= 0) {
        clo = leaf_of_pos_[bc0] - b.cl0;
        chi = leaf_of_pos_[bc0 + bcs - 1] - b.cl0 + 1;
      } else {
        chi = b.ncl;
      }
    }
    const int32_t ncl = std::max(b.ncl, 1);
    for (int32_t r = rlo; r < rhi; ++r)
      for (int32_t c = clo; c < chi; ++c) f(b.seg0 + (int64_t)r * ncl + c);
  }

  void emit(int32_t kind, int32_t idx, std::initializer_list<Access> acc, int32_t rows_s, int32_t cols_s) {
    std::vector<Access> v(acc);
    emit_v(kind, idx, v, rows_s, cols_s);
  }

  void emit_v(int32_t kind, int32_t idx, const std::vector<Access>& acc, int32_t rows_s, int32_t cols_s) {
    int32_t w = 0;
    for (const Access& a : acc)
      for_segments(a.v, [&](int64_t s) {
        w = std::max(w, last_w_[s] + 1);
        if (a.write) w = std::max(w, last_r_[s] + 1);
      });
    for (const Access& a : acc) {
      for_segments(a.v, [&](int64_t s) {
        if (a.write) last_w_[s] = w;
        else last_r_[s] = std::max(last_r_[s], w);
      });
      if (a.v.buf >= 0 && a.v.buf < (int32_t)temp_of_buf_.size() && temp_of_buf_[a.v.buf] >= 0) {
        Temp& T = temps_[temp_of_buf_[a.v.buf]];
        T.first = std::min(T.first, w);
        T.last = std::max(T.last, w);
      }
    }
    ops_.push_back(Rec{kind, idx, w, rows_s, cols_s});
    max_wave_ = std::max(max_wave_, w);
  }

  void tri_op(int32_t mode, const HB& Dg, const View& V, const View& W) {
    TriOp t;
    t.tri = Dg.D.off;
    t.ld = Dg.D.cs;
    t.m = Dg.D.rows;
    t.mode = mode;
    t.pad = 0;
    t.V = V.ref();
    t.W = W.ref();
    std::vector<Access> acc;
    acc.push_back({Dg.D, false});
    if (mode == kMulUpper || mode == kMulUnitLower) {
      acc.push_back({V, false});
      acc.push_back({W, true});
    } else {
      acc.push_back({V, true});
    }
    emit_v(kTri, (int32_t)P_->tri.size(), acc, 0, 0);
    P_->tri.push_back(t);
  }

  void gemm_op(const View& C, double beta, const std::vector<TermSpec>& terms) {
    GemmOp g;
    g.C = C.ref();
    g.beta = beta;
    g.t0 = (int32_t)P_->terms.size();
    g.nt = (int32_t)terms.size();
    std::vector<Access> acc;
    acc.push_back({C, true});
    for (const TermSpec& t : terms) {
      P_->terms.push_back(GemmTerm{t.A.ref(), t.B.ref(), t.alpha});
      acc.push_back({t.A, false});
      acc.push_back({t.B, false});
    }
    emit_v(kGemm, (int32_t)P_->gemm.size(), acc, C.rows_s, C.cols_s);
    P_->gemm.push_back(g);
  }

  void trunc_op(const HB& C, const std::vector<PartSpec>& parts) {
    TruncOp t;
    t.xoff = C.X.off;
    t.yoff = C.Y.off;
    t.m = C.r1 - C.r0;
    t.n = C.c1 - C.c0;
    t.ldx = C.X.cs;
    t.ldy = C.Y.cs;
    t.slot = C.slot;
    t.cap = C.cap;
    t.p0 = (int32_t)P_->parts.size();
    t.np = (int32_t)parts.size();
    std::vector<Access> acc;
    acc.push_back({C.X, true});
    acc.push_back({C.Y, true});
    for (const PartSpec& p : parts) {
      P_->parts.push_back(TruncPart{p.X.ref(), p.Y.ref(), p.row_off, p.col_off, p.alpha});
      acc.push_back({p.X, false});
      acc.push_back({p.Y, false});
    }
    emit_v(kTrunc, (int32_t)P_->trunc.size(), acc, 0, 0);
    P_->trunc.push_back(t);
  }

 public:
  int32_t kcap_ = 64;
  const std::vector<int32_t>* slot_cap_ = nullptr;   // fitted capacity per rank slot (null: uniform)

  View vector_view(int64_t off, int32_t max_rhs, int32_t nrhs_slot, int32_t buf) const {
    return View{off, 1, S_.N, S_.N, dyn(nrhs_slot), S_.N, max_rhs, 0, -1, buf, false};
  }
  int32_t vector_buf() {
    int32_t b = new_buf(0, (int32_t)S_.leaf_clusters.size(), 0, 0);
    grow_segments();
    return b;
  }

 private:
  const Structure& S_;
  StoragePlan& st_;
  Plan* P_ = nullptr;
  std::vector<int32_t> leaf_of_pos_;
  std::vector<int32_t> leaf_buf_, leaf_ybuf_, init_buf_;
  std::vector<std::vector<int32_t>> mbuf_, mybuf_;   // per matrix: buffers of the leaves (X, then Y)
  int64_t mat_begin_ = 0, mat_stride_ = 0;
  int32_t mat_slots_ = 0;
  std::vector<Temp> temps_;
  std::vector<int64_t> vbegin_;   // virtual begins of temps_, filled while the plan is remapped
  std::map<int64_t, std::vector<PartSpec>> pending_;
  std::map<int32_t, HB> temp_hb_;
  std::vector<int32_t> temp_of_buf_;
  int64_t temp_peak_ = 0;
  int64_t max_peak_ = 0;
  std::vector<Buf> bufs_;
  int32_t persistent_bufs_ = 0;
  int64_t persistent_segs_ = 0;
  int64_t nseg_ = 0;
  std::vector<int32_t> last_w_, last_r_;
  int64_t temp_base_ = 0, temp_top_ = 0;
  std::vector<Rec> ops_;
  int32_t max_wave_ = -1;
};

}  // namespace

void build_plans(const Structure& S, int32_t kcap, int32_t max_rhs,
                 const std::vector<int32_t>& nonzero_admissible, PlanSet* out,
                 const std::vector<int32_t>* slot_cap) {
  HLU_REQUIRE(kcap >= 1 && max_rhs >= 1, HLU_ERR_INVALID_ARG, "build_plans: bad capacity");
  PlanSet& ps = *out;
  ps = PlanSet{};
  ps.kcap = kcap;
  StoragePlan& st = ps.store;
  Planner pl(S, st);
  pl.kcap_ = kcap;
  pl.slot_cap_ = slot_cap;
  pl.layout(kcap, nonzero_admissible, &ps.init_blocks);

  // factorisation plan; temporaries follow the data
  const int64_t temp_base = st.data_elems;
  pl.begin_plan(&ps.factor, temp_base);
  pl.init_lowrank(ps.init_blocks);
  pl.hlu(pl.block(0));
  pl.flush_all();
  pl.end_plan();
  st.temp_elems = pl.temp_used();

  // the rank slots of blocks and temporaries depend on the structure only,
  // so a fitted capacity table matches them one to one
  HLU_REQUIRE(!slot_cap || (int64_t)slot_cap->size() == st.num_slots, HLU_ERR_INVALID_ARG,
              "build_plans: fitted capacities do not match the rank slots of this structure");

  // solve plans: vectors and their temporaries after the factor temporaries
  st.max_rhs = max_rhs;
  st.nrhs_slot = st.num_slots++;
  int64_t top = temp_base + st.temp_elems;
  st.vec_off = top;
  top += ((int64_t)S.N * max_rhs + 31) & ~int64_t(31);
  st.vec2_off = top;
  top += ((int64_t)S.N * max_rhs + 31) & ~int64_t(31);
  const int64_t solve_base = top;

  pl.begin_plan(&ps.fwd_bwd, solve_base);
  {
    int32_t vb = pl.vector_buf();
    auto V = pl.vector_view(st.vec_off, max_rhs, st.nrhs_slot, vb);
    pl.hsolve_lower(pl.block(0), V);
    pl.hsolve_upper(pl.block(0), V);
  }
  pl.end_plan();
  int64_t solve_used = pl.temp_used();

  pl.begin_plan(&ps.apply, solve_base);
  {
    int32_t vb = pl.vector_buf();
    int32_t wb = pl.vector_buf();
    auto V = pl.vector_view(st.vec_off, max_rhs, st.nrhs_slot, vb);
    auto W = pl.vector_view(st.vec2_off, max_rhs, st.nrhs_slot, wb);
    pl.apply_upper(pl.block(0), V, W);   // W = U V
    pl.apply_lower(pl.block(0), W, V);   // V = L W
  }
  pl.end_plan();
  solve_used = std::max(solve_used, pl.temp_used());
  st.solve_temp_elems = solve_used;
  st.total_elems = solve_base + solve_used;
}

void build_inverse_plans(const Structure& S, int32_t kcap, int32_t max_rhs, InversePlanSet* out) {
  HLU_REQUIRE(kcap >= 1 && max_rhs >= 1, HLU_ERR_INVALID_ARG, "build_inverse_plans: bad capacity");
  InversePlanSet& ip = *out;
  ip = InversePlanSet{};
  ip.kcap = kcap;
  StoragePlan& st = ip.store;
  Planner pl(S, st);
  pl.kcap_ = kcap;
  std::vector<InitBlock> inits;
  pl.layout(kcap, {}, &inits, 4);
  ip.mat_elems = pl.mat_stride();
  ip.mat0_off = pl.mat_begin();
  ip.mat_slots = pl.mat_slots();
  // vectors (cluster order): V, W = X V, U = A_H W; then the temporaries
  st.max_rhs = max_rhs;
  st.nrhs_slot = st.num_slots++;
  const int64_t vblock = ((int64_t)S.N * max_rhs + 31) & ~int64_t(31);
  st.vec_off = st.data_elems;
  st.vec2_off = st.vec_off + vblock;
  ip.vec3_off = st.vec2_off + vblock;
  const int64_t temp_base = ip.vec3_off + vblock;
  ip.temp_slot0 = st.num_slots;
  int64_t used = 0;
  for (int s = 0; s < 2; ++s) {
    pl.begin_plan(&ip.step[s], temp_base);
    pl.schulz_step(1 + 2 * s, 3 - 2 * s);
    pl.end_plan();
    used = std::max(used, pl.temp_used());
  }
  for (int s = 0; s < 2; ++s) {
    pl.begin_plan(&ip.apply[s], temp_base);
    {
      const int32_t vb = pl.vector_buf(), wb = pl.vector_buf();
      pl.hmv(pl.block(0, 1 + 2 * s), false, pl.vector_view(st.vec_off, max_rhs, st.nrhs_slot, vb),
             pl.vector_view(st.vec2_off, max_rhs, st.nrhs_slot, wb), 1.0, 0.0);
    }
    pl.end_plan();
    used = std::max(used, pl.temp_used());
  }
  pl.begin_plan(&ip.amul, temp_base);
  {
    const int32_t wb = pl.vector_buf(), ub = pl.vector_buf();
    pl.hmv(pl.block(0, 0), false, pl.vector_view(st.vec2_off, max_rhs, st.nrhs_slot, wb),
           pl.vector_view(ip.vec3_off, max_rhs, st.nrhs_slot, ub), 1.0, 0.0);
  }
  pl.end_plan();
  used = std::max(used, pl.temp_used());
  st.temp_elems = used;
  st.total_elems = temp_base + used;
}

}  // namespace hlu
