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
  std::vector<std::vector<int32_t>> by_leaf(2 * L);    // chunks computed by leaf tasks
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
      // row chunks of whole leaves of sigma, each about kTprodChunkRows.  If
      // rho starts within kNearLeaves leaves of the sweep after sigma's
      // completing leaf p, the chunk of leaf p alone is computed by p's own
      // leaf task (a separate task would sit on the sweep's critical path).
      const int32_t p_end = lower ? cc.leaf_last - 1 : cc.leaf_first;
      const bool next_needs = lower ? rc.leaf_first - cc.leaf_last < kNearLeaves
                                    : cc.leaf_first - rc.leaf_last < kNearLeaves;
      const int32_t tp0 = (int32_t)sc.tprod.size();
      for (int32_t f0 = cc.leaf_first; f0 < cc.leaf_last;) {
        const int32_t r0 = S.clusters[S.leaf_clusters[f0]].begin;
        int32_t f1 = f0 + 1;
        const bool alone = next_needs && f0 == p_end;
        while (!alone && f1 < cc.leaf_last && S.clusters[S.leaf_clusters[f1]].end - r0 <= kTprodChunkRows &&
               !(next_needs && f1 == p_end))
          ++f1;
        const int32_t r1 = S.clusters[S.leaf_clusters[f1 - 1]].end;
        STprod t{};
        t.yoff = st.yoff[b] + (r0 - cc.begin);
        t.ldy = cc.size();
        t.col0 = r0;
        t.ncols = r1 - r0;
        t.slot = st.slot[b];
        t.lf0 = f0;
        t.lf1 = f1;
        t.cap = st.cap[b];
        t.toff = toff;
        toff += t.cap;
        const int32_t tp = (int32_t)sc.tprod.size();
        sc.tprod.push_back(t);
        tp_need.push_back(lower ? rc.leaf_first : L - rc.leaf_last);
        if (alone) {
          by_leaf[(lower ? 0 : L) + p_end].push_back(tp);
        } else {
          // forward: ready after the chunk's last leaf; backward: after its
          // first.  The key is the first row leaf that needs it in sweep order.
          if (lower) tp_after[f1 - 1].push_back(tp);
          else tp_after[L + f0].push_back(tp);
        }
        f0 = f1;
      }
      const int32_t ntp = (int32_t)sc.tprod.size() - tp0;
      for (int32_t f = rc.leaf_first; f < rc.leaf_last; ++f) {
        const ClusterNode& lc = S.clusters[S.leaf_clusters[f]];
        SLow w{};
        w.xoff = st.off[b] + (lc.begin - rc.begin);
        w.ldx = rc.size();
        w.tp = tp0;
        w.ntp = ntp;
        // sweep position at which the block's product is complete
        w.pad = lower ? cc.leaf_last : L - cc.leaf_first;
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
    // contributions in the order their products complete (the leaf task
    // accumulates them in this order, waiting only when it reaches one)
    std::stable_sort(ll[s].begin(), ll[s].end(), [](const SLow& x, const SLow& y) { return x.pad < y.pad; });
    for (SLow& w : ll[s]) w.pad = 0;
    lf.l0 = (int32_t)sc.low.size();
    lf.nl = (int32_t)ll[s].size();
    sc.low.insert(sc.low.end(), ll[s].begin(), ll[s].end());
    lf.tq0 = (int32_t)sc.leaf_tq.size();
    lf.ntq = (int32_t)by_leaf[s].size();
    sc.leaf_tq.insert(sc.leaf_tq.end(), by_leaf[s].begin(), by_leaf[s].end());
    sc.max_m = std::max(sc.max_m, lf.m);
  }
  // producers of the dense records: the leaf task of the preceding leaf for
  // the block coupling neighbours, otherwise the push task of the leaf that
  // completes sigma
  std::vector<std::vector<int32_t>> push(2 * L);
  for (int32_t s = 0; s < 2 * L; ++s) sc.leaves[s].next_rec = sc.leaves[s].prev_rec = -1;
  for (int32_t s = 0; s < 2 * L; ++s) {
    const bool fwd = s < L;
    const int32_t j = s % L;
    const SLeaf& lf = sc.leaves[s];
    for (int32_t r = lf.d0; r < lf.d0 + lf.nd; ++r) {
      const SDense& d = sc.dense[r];
      const int32_t prod = fwd ? d.lf1 - 1 : d.lf0;     // leaf that completes sigma
      const bool neighbour = (d.lf1 - d.lf0 == 1) && (fwd ? prod == j - 1 : prod == j + 1);
      const int32_t ps = (fwd ? 0 : L) + prod;
      if (neighbour && sc.leaves[ps].next_rec < 0) {
        sc.leaves[ps].next_rec = r;
        sc.leaves[s].prev_rec = r;
      } else {
        push[ps].push_back(r);
      }
    }
  }
  // Work released by one leaf is queued in the order its consumers come in
  // the sweep (forward: ascending rows, backward: descending), and the
  // records are split into tasks of kPushChunk so that several workgroups
  // form them together.
  // neighbour blocks times the inverse, for leaves up to 64 rows: the
  // neighbour record and, when the rows fit 128 in all, the second
  // neighbour's record of a block whose columns are this leaf alone (taken
  // from the push tasks: on the sweep's critical path, a push after this
  // task's end would delay the leaf after next)
  for (int32_t s = 0; s < 2 * L; ++s) {
    SLeaf& lf = sc.leaves[s];
    lf.nm = -1;
    lf.next_rec2 = -1;
    lf.nm_rows = 0;
    if (lf.next_rec < 0) continue;
    const SDense& d = sc.dense[lf.next_rec];
    if (lf.m > 64 || d.m > 128 || d.ncols != lf.m) continue;
    int32_t rows = d.m;
    const bool fwd = s < L;
    const int32_t j = s % L;
    const int32_t c2 = fwd ? j + 2 : j - 2;   // leaf after next in sweep order
    if (c2 >= 0 && c2 < L) {
      const int32_t row2 = S.clusters[S.leaf_clusters[c2]].begin;
      std::vector<int32_t>& pr = push[s];
      for (size_t q = 0; q < pr.size(); ++q) {
        const SDense& d2 = sc.dense[pr[q]];
        if (d2.row0 == row2 && d2.lf1 - d2.lf0 == 1 && d2.ncols == lf.m && rows + d2.m <= 128) {
          lf.next_rec2 = pr[q];
          rows += d2.m;
          pr.erase(pr.begin() + q);
          break;
        }
      }
    }
    lf.nm = sc.nm_elems;
    lf.nm_rows = rows;
    sc.nm_elems += (int64_t)rows * lf.m;
  }
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
    // the T-products of blocks with the same column rows (several row
    // clusters against one sigma) share a task, at most kTprodGroup of
    // them, in the order of their first consumers: fewer workgroups wait
    // on the same leaf, and each product still sets its own flag
    std::vector<char> used(tl.size(), 0);
    for (size_t i = 0; i < tl.size(); ++i) {
      if (used[i]) continue;
      const int32_t id = (int32_t)sc.tg0.size();
      sc.tg0.push_back((int32_t)sc.tg_list.size());
      const STprod& t0 = sc.tprod[tl[i]];
      int32_t cnt = 0;
      for (size_t q = i; q < tl.size() && cnt < kTprodGroup; ++q) {
        const STprod& t = sc.tprod[tl[q]];
        if (used[q] || t.col0 != t0.col0 || t.ncols != t0.ncols) continue;
        sc.tg_list.push_back(tl[q]);
        used[q] = 1;
        ++cnt;
      }
      sc.tasks.push_back({tp_kind, id});
    }
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
  sc.tg0.push_back((int32_t)sc.tg_list.size());
  // every T-product is formed exactly once: by a T-product task or by the
  // leaf task that completes its rows
  std::vector<int32_t> seen(sc.tprod.size(), 0);
  for (int32_t q : sc.tg_list) ++seen[q];
  for (int32_t q : sc.leaf_tq) ++seen[q];
  for (int32_t c : seen) HLU_REQUIRE(c == 1, HLU_ERR_INVALID_ARG, "solve schedule: T-product not formed once");
  check_solve_waits(sc);
}

// Every flag a task of the persistent solve waits on is set by exactly one
// task that comes earlier in claim order.  Workgroups claim tasks in that
// order, so the earliest unfinished task waits on finished tasks only and
// every claimed task completes, whatever the number of resident workgroups.
void check_solve_waits(const SolveSched& sc) {
  const int32_t L = sc.L;
  const int32_t nt = (int32_t)sc.tasks.size();
  std::vector<int32_t> leaf_at(2 * L, -1), rec_at(sc.dense.size(), -1), tp_at(sc.tprod.size(), -1);
  auto set = [&](std::vector<int32_t>& at, int32_t i, int32_t t) {
    HLU_REQUIRE(i >= 0 && i < (int32_t)at.size() && at[i] < 0, HLU_ERR_INVALID_ARG,
                "solve schedule: a flag is set by two tasks or out of range");
    at[i] = t;
  };
  for (int32_t t = 0; t < nt; ++t) {
    const STask& k = sc.tasks[t];
    if (k.kind == kFwdLeaf || k.kind == kBwdLeaf) {
      const SLeaf& lf = sc.leaves[k.idx];
      set(leaf_at, k.idx, t);
      if (lf.next_rec >= 0) set(rec_at, lf.next_rec, t);
      if (lf.next_rec2 >= 0) set(rec_at, lf.next_rec2, t);
      for (int32_t q = 0; q < lf.ntq; ++q) set(tp_at, sc.leaf_tq[lf.tq0 + q], t);
    } else if (k.kind == kFwdPush || k.kind == kBwdPush) {
      for (int32_t q = sc.push0[k.idx]; q < sc.push0[k.idx + 1]; ++q) set(rec_at, sc.push_recs[q], t);
    } else {
      for (int32_t q = sc.tg0[k.idx]; q < sc.tg0[k.idx + 1]; ++q) set(tp_at, sc.tg_list[q], t);
    }
  }
  auto before = [&](const std::vector<int32_t>& at, int32_t i, int32_t t) {
    HLU_REQUIRE(i >= 0 && i < (int32_t)at.size() && at[i] >= 0 && at[i] < t, HLU_ERR_INVALID_ARG,
                "solve schedule: a task waits on a flag no earlier task sets");
  };
  for (int32_t t = 0; t < nt; ++t) {
    const STask& k = sc.tasks[t];
    const bool fwd = k.kind == kFwdLeaf || k.kind == kFwdPush || k.kind == kFwdTprod;
    HLU_REQUIRE(fwd == (t < sc.n_fwd_tasks), HLU_ERR_INVALID_ARG, "solve schedule: sweeps interleaved");
    const int32_t base = fwd ? 0 : L;
    if (k.kind == kFwdLeaf || k.kind == kBwdLeaf) {
      const SLeaf& lf = sc.leaves[k.idx];
      for (int32_t d = lf.d0; d < lf.d0 + lf.nd; ++d) before(rec_at, d, t);
      for (int32_t l = lf.l0; l < lf.l0 + lf.nl; ++l)
        for (int32_t q = 0; q < sc.low[l].ntp; ++q) before(tp_at, sc.low[l].tp + q, t);
    } else if (k.kind == kFwdPush || k.kind == kBwdPush) {
      for (int32_t q = sc.push0[k.idx]; q < sc.push0[k.idx + 1]; ++q) {
        const SDense& d = sc.dense[sc.push_recs[q]];
        for (int32_t f = d.lf0; f < d.lf1; ++f) before(leaf_at, base + f, t);
      }
    } else {
      for (int32_t q = sc.tg0[k.idx]; q < sc.tg0[k.idx + 1]; ++q) {
        const STprod& p = sc.tprod[sc.tg_list[q]];
        for (int32_t f = p.lf0; f < p.lf1; ++f) before(leaf_at, base + f, t);
      }
    }
  }
  // the backward leaf tasks also wait for the count of finished forward
  // tasks, all of which come first (checked above)
}

}  // namespace hlu
