// Cluster tree and eta-admissible block cluster tree (Sec. 3, Definition 1;
// geometric cluster tree and eta = 2 of Sec. 4), integer-exact.
#pragma once
#include <array>
#include <cstdint>
#include <vector>

namespace hlu {

struct ClusterNode {
  int32_t begin, end;          // index range in cluster order
  int32_t level;
  int32_t son[2] = {-1, -1};
  int32_t leaf_first, leaf_last;  // range of leaf-cluster ordinals covered [first, last)
  std::array<int32_t, 3> lo, hi;  // tight box of doubled midpoints (splitting)
  std::array<int32_t, 3> alo, ahi;  // box of the admissibility test: the midpoint box, or the
                                    // union of the indices' own boxes (supports) when given
  bool is_leaf() const { return son[0] < 0; }
  int32_t size() const { return end - begin; }
};

enum BlockKind : int32_t { kDense = 0, kLowRank = 1, kSub = 2 };

struct BlockNode {
  int32_t row, col;            // cluster ids
  BlockKind kind;
  int32_t son[4] = {-1, -1, -1, -1};  // (0,0),(0,1),(1,0),(1,1) for kSub
  int32_t leaf_id = -1;        // ordinal among leaves (pre-order) for kDense/kLowRank
};

struct Structure {
  int32_t N = 0, leaf_size = 0;
  double eta = 2.0;
  std::vector<int32_t> perm;           // cluster position -> natural index
  std::vector<ClusterNode> clusters;   // pre-order, root = 0
  std::vector<int32_t> leaf_clusters;  // ids of leaf clusters in order
  std::vector<BlockNode> blocks;       // all block-tree nodes, root = 0
  std::vector<int32_t> leaves;         // block-tree leaves (node ids) in pre-order
  int32_t depth = 0;

  // box_lo2/box_hi2 (N x 3, doubled lattice units, may be null): a box per
  // index for the admissibility test, e.g. the support of its basis
  // function; null: the midpoints themselves.
  void build(const int32_t* mid2, int32_t N, int32_t leaf, double eta, const int32_t* box_lo2 = nullptr,
             const int32_t* box_hi2 = nullptr);
};

}  // namespace hlu
