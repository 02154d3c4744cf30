// Builds the persistent H-solve schedule from the block tree and the arena
// layout of the factors.
#include "solve_sched.h"

#include <algorithm>

#include "common.h"

namespace hlu {

void build_solve_sched(const Structure& S, const StoragePlan& st, SolveSched* out) {
  SolveSched& sc = *out;
  sc = SolveSched{};
  const int32_t L = (int32_t)S.leaf_clusters.size();
  sc.L = L;
  std::vector<std::vector<SDense>> dl(2 * L);
  std::vector<std::vector<SLow>> ll(2 * L);
  std::vector<int64_t> diag(L, -1);
  std::vector<int32_t> leaf_of_cluster(S.clusters.size(), -1);
  for (int32_t l = 0; l < L; ++l) leaf_of_cluster[S.leaf_clusters[l]] = l;
  std::vector<std::vector<int32_t>> tp_after(2 * L);   // T-products to run after leaf task
  int64_t toff = 0;
  for (size_t b = 0; b < S.leaves.size(); ++b) {
    const BlockNode& B = S.blocks[S.leaves[b]];
    const ClusterNode& rc = S.clusters[B.row];
    const ClusterNode& cc = S.clusters[B.col];
    if (B.row == B.col) {
      HLU_REQUIRE(B.kind == kDense && rc.is_leaf(), HLU_ERR_INVALID_ARG, "solve schedule: bad diagonal block");
      diag[leaf_of_cluster[B.row]] = st.off[b];
      continue;
    }
    const bool lower = cc.end <= rc.begin;
    HLU_REQUIRE(lower || rc.end <= cc.begin, HLU_ERR_INVALID_ARG, "solve schedule: overlapping block");
    const int32_t side = lower ? 0 : L;   // forward (L) or backward (U) sweep
    if (B.kind == kDense) {
      for (int32_t f = rc.leaf_first; f < rc.leaf_last; ++f) {
        const ClusterNode& lc = S.clusters[S.leaf_clusters[f]];
        SDense d{};
        d.off = st.off[b] + (lc.begin - rc.begin);
        d.ld = rc.size();
        d.m = lc.size();
        d.row0 = lc.begin;
        d.col0 = cc.begin;
        d.ncols = cc.size();
        d.lf0 = cc.leaf_first;
        d.lf1 = cc.leaf_last;
        dl[side + f].push_back(d);
      }
    } else {
      STprod t{};
      t.yoff = st.yoff[b];
      t.ldy = cc.size();
      t.col0 = cc.begin;
      t.ncols = cc.size();
      t.slot = st.slot[b];
      t.lf0 = cc.leaf_first;
      t.lf1 = cc.leaf_last;
      t.cap = st.cap[b];
      t.toff = toff;
      toff += t.cap;
      const int32_t tp = (int32_t)sc.tprod.size();
      sc.tprod.push_back(t);
      // forward: ready after the last leaf of sigma; backward: after the first
      if (lower) tp_after[cc.leaf_last - 1].push_back(tp);
      else tp_after[L + cc.leaf_first].push_back(tp);
      for (int32_t f = rc.leaf_first; f < rc.leaf_last; ++f) {
        const ClusterNode& lc = S.clusters[S.leaf_clusters[f]];
        SLow w{};
        w.xoff = st.off[b] + (lc.begin - rc.begin);
        w.ldx = rc.size();
        w.tp = tp;
        ll[side + f].push_back(w);
      }
    }
  }
  sc.tbuf_per_rhs = toff;
  sc.leaves.resize(2 * L);
  for (int32_t s = 0; s < 2 * L; ++s) {
    const int32_t f = s % L;
    const ClusterNode& lc = S.clusters[S.leaf_clusters[f]];
    SLeaf& lf = sc.leaves[s];
    lf.row0 = lc.begin;
    lf.m = lc.size();
    lf.diag = diag[f];
    HLU_REQUIRE(lf.diag >= 0, HLU_ERR_INVALID_ARG, "solve schedule: missing diagonal leaf");
    lf.d0 = (int32_t)sc.dense.size();
    lf.nd = (int32_t)dl[s].size();
    sc.dense.insert(sc.dense.end(), dl[s].begin(), dl[s].end());
    lf.l0 = (int32_t)sc.low.size();
    lf.nl = (int32_t)ll[s].size();
    sc.low.insert(sc.low.end(), ll[s].begin(), ll[s].end());
    sc.max_m = std::max(sc.max_m, lf.m);
  }
  // producers of the dense records: the leaf task of the preceding leaf for
  // the block coupling neighbours, otherwise the push task of the leaf that
  // completes sigma
  std::vector<std::vector<int32_t>> push(2 * L);
  for (int32_t s = 0; s < 2 * L; ++s) sc.leaves[s].next_rec = -1;
  for (int32_t s = 0; s < 2 * L; ++s) {
    const bool fwd = s < L;
    const int32_t j = s % L;
    const SLeaf& lf = sc.leaves[s];
    for (int32_t r = lf.d0; r < lf.d0 + lf.nd; ++r) {
      const SDense& d = sc.dense[r];
      const int32_t prod = fwd ? d.lf1 - 1 : d.lf0;     // leaf that completes sigma
      const bool neighbour = (d.lf1 - d.lf0 == 1) && (fwd ? prod == j - 1 : prod == j + 1);
      const int32_t ps = (fwd ? 0 : L) + prod;
      if (neighbour && sc.leaves[ps].next_rec < 0) sc.leaves[ps].next_rec = r;
      else push[ps].push_back(r);
    }
  }
  auto add_push = [&](int32_t s) {
    if (push[s].empty()) return -1;
    const int32_t id = (int32_t)sc.push0.size();
    sc.push0.push_back((int32_t)sc.push_recs.size());
    sc.push_recs.insert(sc.push_recs.end(), push[s].begin(), push[s].end());
    return id;
  };
  for (int32_t f = 0; f < L; ++f) {
    sc.tasks.push_back({kFwdLeaf, f});
    const int32_t id = add_push(f);
    if (id >= 0) sc.tasks.push_back({kFwdPush, id});
    for (int32_t tp : tp_after[f]) sc.tasks.push_back({kFwdTprod, tp});
  }
  sc.n_fwd_tasks = (int32_t)sc.tasks.size();
  for (int32_t f = L - 1; f >= 0; --f) {
    sc.tasks.push_back({kBwdLeaf, L + f});
    const int32_t id = add_push(L + f);
    if (id >= 0) sc.tasks.push_back({kBwdPush, id});
    for (int32_t tp : tp_after[L + f]) sc.tasks.push_back({kBwdTprod, tp});
  }
  sc.push0.push_back((int32_t)sc.push_recs.size());
}

}  // namespace hlu
