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
  std::vector<int32_t> tp_need;                        // sweep position of the first consumer
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
      // forward: ready after the last leaf of sigma; backward: after the first.
      // The key is the first row leaf that needs it in sweep order.
      if (lower) tp_after[cc.leaf_last - 1].push_back(tp);
      else tp_after[L + cc.leaf_first].push_back(tp);
      tp_need.push_back(lower ? rc.leaf_first : L - rc.leaf_last);
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
  std::vector<int64_t> inv(L);
  for (int32_t f = 0; f < L; ++f) {
    inv[f] = sc.inv_elems;
    const int64_t m = S.clusters[S.leaf_clusters[f]].size();
    sc.inv_elems += m * m;
  }
  for (int32_t s = 0; s < 2 * L; ++s) {
    const int32_t f = s % L;
    const ClusterNode& lc = S.clusters[S.leaf_clusters[f]];
    SLeaf& lf = sc.leaves[s];
    lf.row0 = lc.begin;
    lf.m = lc.size();
    lf.diag = diag[f];
    lf.inv = inv[f];
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
  // Work released by one leaf is queued in the order its consumers come in
  // the sweep (forward: ascending rows, backward: descending), and the
  // records are split into tasks of kPushChunk so that several workgroups
  // form them together.
  auto emit = [&](int32_t s, int32_t push_kind, int32_t tp_kind) {
    const bool fwd = s < L;
    std::vector<int32_t>& pr = push[s];
    std::stable_sort(pr.begin(), pr.end(), [&](int32_t x, int32_t y) {
      return fwd ? sc.dense[x].row0 < sc.dense[y].row0 : sc.dense[x].row0 > sc.dense[y].row0;
    });
    std::vector<int32_t>& tl = tp_after[s];
    std::stable_sort(tl.begin(), tl.end(), [&](int32_t x, int32_t y) { return tp_need[x] < tp_need[y]; });
    for (size_t c = 0; c < pr.size(); c += kPushChunk) {
      const int32_t id = (int32_t)sc.push0.size();
      sc.push0.push_back((int32_t)sc.push_recs.size());
      const size_t e = std::min(pr.size(), c + kPushChunk);
      sc.push_recs.insert(sc.push_recs.end(), pr.begin() + c, pr.begin() + e);
      sc.tasks.push_back({push_kind, id});
    }
    for (int32_t tp : tl) sc.tasks.push_back({tp_kind, tp});
  };
  for (int32_t f = 0; f < L; ++f) {
    sc.tasks.push_back({kFwdLeaf, f});
    emit(f, kFwdPush, kFwdTprod);
  }
  sc.n_fwd_tasks = (int32_t)sc.tasks.size();
  for (int32_t f = L - 1; f >= 0; --f) {
    sc.tasks.push_back({kBwdLeaf, L + f});
    emit(L + f, kBwdPush, kBwdTprod);
  }
  sc.push0.push_back((int32_t)sc.push_recs.size());
}

}  // namespace hlu
