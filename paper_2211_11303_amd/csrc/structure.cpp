// Geometric cluster tree and block cluster tree.
//
// Cluster tree: a cluster with at most `leaf` indices is a leaf; otherwise
// the tight box [lo, hi] of its doubled midpoints is split at its centre
// along the axis of largest extent (lowest axis on ties): indices with
// 2 c_axis < lo_axis + hi_axis form the first son, the rest the second, each
// keeping the parent's order.  Block tree: (tau, sigma) is an admissible
// (low-rank) leaf if dist > 0 and min(diam tau, diam sigma) <= eta dist,
// with diam the box diagonal and dist the gap between the two boxes,
// compared in squares; else a dense leaf if tau or sigma is a leaf cluster;
// else it splits into the four products of the sons.  The boxes of the
// admissibility test are the midpoint boxes, or, when a box per index is
// given (the support of each basis function), the union of those boxes:
// blocks of disjoint supports are admissible only if the supports, not
// just the midpoints, are far apart.
#include "structure.h"

#include <algorithm>

#include "common.h"

namespace hlu {
namespace {

int64_t diam2(const ClusterNode& c) {
  int64_t s = 0;
  for (int a = 0; a < 3; ++a) {
    int64_t d = c.ahi[a] - c.alo[a];
    s += d * d;
  }
  return s;
}

int64_t dist2(const ClusterNode& x, const ClusterNode& y) {
  int64_t s = 0;
  for (int a = 0; a < 3; ++a) {
    int64_t g = std::max<int64_t>(0, std::max<int64_t>(y.alo[a] - x.ahi[a], x.alo[a] - y.ahi[a]));
    s += g * g;
  }
  return s;
}

}  // namespace

void Structure::build(const int32_t* mid2, int32_t n, int32_t leaf, double eta_, const int32_t* box_lo2,
                      const int32_t* box_hi2) {
  HLU_REQUIRE(n > 0 && leaf > 0 && eta_ > 0, HLU_ERR_INVALID_ARG, "hlu_build: N, leaf_size and eta must be positive");
  N = n;
  leaf_size = leaf;
  eta = eta_;
  perm.resize(N);
  clusters.clear();
  leaf_clusters.clear();
  blocks.clear();
  leaves.clear();
  depth = 0;

  std::vector<int32_t> idx(N), tmp(N);
  for (int32_t i = 0; i < N; ++i) idx[i] = i;
  // explicit stack to avoid deep recursion: (begin, end, level, parent, which son)
  struct Item { int32_t b, e, level, parent, which; };
  std::vector<Item> stack;
  stack.push_back({0, N, 0, -1, 0});
  while (!stack.empty()) {
    Item it = stack.back();
    stack.pop_back();
    ClusterNode c;
    c.begin = it.b;
    c.end = it.e;
    c.level = it.level;
    depth = std::max(depth, it.level);
    for (int a = 0; a < 3; ++a) {
      c.lo[a] = INT32_MAX;
      c.hi[a] = INT32_MIN;
    }
    for (int32_t i = it.b; i < it.e; ++i)
      for (int a = 0; a < 3; ++a) {
        int32_t v = mid2[3 * (int64_t)idx[i] + a];
        c.lo[a] = std::min(c.lo[a], v);
        c.hi[a] = std::max(c.hi[a], v);
      }
    c.alo = c.lo;
    c.ahi = c.hi;
    if (box_lo2) {
      for (int a = 0; a < 3; ++a) {
        c.alo[a] = INT32_MAX;
        c.ahi[a] = INT32_MIN;
      }
      for (int32_t i = it.b; i < it.e; ++i)
        for (int a = 0; a < 3; ++a) {
          c.alo[a] = std::min(c.alo[a], box_lo2[3 * (int64_t)idx[i] + a]);
          c.ahi[a] = std::max(c.ahi[a], box_hi2[3 * (int64_t)idx[i] + a]);
        }
    }
    int32_t id = (int32_t)clusters.size();
    clusters.push_back(c);
    if (it.parent >= 0) clusters[it.parent].son[it.which] = id;
    if (it.e - it.b <= leaf) {
      for (int32_t i = it.b; i < it.e; ++i) perm[i] = idx[i];
      continue;
    }
    int ax = 0;
    for (int a = 1; a < 3; ++a)
      if (c.hi[a] - c.lo[a] > c.hi[ax] - c.lo[ax]) ax = a;
    const int64_t mid = (int64_t)c.lo[ax] + c.hi[ax];
    int32_t nl = 0, nr = 0;
    for (int32_t i = it.b; i < it.e; ++i)
      if (2 * (int64_t)mid2[3 * (int64_t)idx[i] + ax] < mid) idx[it.b + nl++] = idx[i];
      else tmp[nr++] = idx[i];
    for (int32_t i = 0; i < nr; ++i) idx[it.b + nl + i] = tmp[i];
    HLU_REQUIRE(nl > 0 && nr > 0, HLU_ERR_INVALID_ARG, "hlu_build: coincident midpoints cannot be split");
    // pre-order: first son handled first, so push the second son first
    stack.push_back({it.b + nl, it.e, it.level + 1, id, 1});
    stack.push_back({it.b, it.b + nl, it.level + 1, id, 0});
  }
  // leaf ordinals and covered leaf ranges (post-order pass over pre-order list)
  for (size_t i = 0; i < clusters.size(); ++i)
    if (clusters[i].is_leaf()) leaf_clusters.push_back((int32_t)i);
  std::vector<int32_t> leaf_ord(clusters.size(), -1);
  for (size_t l = 0; l < leaf_clusters.size(); ++l) leaf_ord[leaf_clusters[l]] = (int32_t)l;
  for (int64_t i = (int64_t)clusters.size() - 1; i >= 0; --i) {
    ClusterNode& c = clusters[i];
    if (c.is_leaf()) {
      c.leaf_first = leaf_ord[i];
      c.leaf_last = leaf_ord[i] + 1;
    } else {
      c.leaf_first = clusters[c.son[0]].leaf_first;
      c.leaf_last = clusters[c.son[1]].leaf_last;
    }
  }

  // block tree, pre-order
  const double eta2 = eta * eta;
  struct BItem { int32_t r, c, parent, which; };
  std::vector<BItem> bst;
  bst.push_back({0, 0, -1, 0});
  while (!bst.empty()) {
    BItem it = bst.back();
    bst.pop_back();
    const ClusterNode& t = clusters[it.r];
    const ClusterNode& s = clusters[it.c];
    BlockNode b;
    b.row = it.r;
    b.col = it.c;
    int64_t d2 = dist2(t, s);
    bool adm = d2 > 0 && double(std::min(diam2(t), diam2(s))) <= eta2 * double(d2);
    int32_t id = (int32_t)blocks.size();
    if (adm) b.kind = kLowRank;
    else if (t.is_leaf() || s.is_leaf()) b.kind = kDense;
    else b.kind = kSub;
    if (b.kind != kSub) {
      b.leaf_id = (int32_t)leaves.size();
      leaves.push_back(id);
    }
    blocks.push_back(b);
    if (it.parent >= 0) blocks[it.parent].son[it.which] = id;
    if (b.kind == kSub) {
      for (int q = 3; q >= 0; --q)
        bst.push_back({t.son[q / 2], s.son[q % 2], id, q});
    }
  }
}

}  // namespace hlu
