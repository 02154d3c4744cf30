// Builds the chain schedule of the persistent H-solve (chain_sched.h) from
// the block tree and the arena layout of the factors, merges the schedules
// of a batch, and checks the claim order.
#include "chain_sched.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <string>

#include "common.h"

namespace hlu {

namespace {

struct GatherLists {     // inputs of one gather, in build order
  std::vector<GDense> dense;
  std::vector<GLow> low;
  std::vector<GInline> inl;
  int32_t pmax = -1;
};

}  // namespace

void build_chain_sched(const Structure& S, const StoragePlan& st, ChainSched* out) {
  ChainSched& sc = *out;
  sc = ChainSched{};
  const int32_t L = (int32_t)S.leaf_clusters.size();
  sc.L = L;
  sc.members = 1;
  sc.member_L = {L};
  sc.member_pos0 = {0};
  auto lc = [&](int32_t f) -> const ClusterNode& { return S.clusters[S.leaf_clusters[f]]; };
  auto pos = [&](int32_t s, int32_t f) { return s == 0 ? f : L - 1 - f; };
  std::vector<int32_t> leaf_of_cluster(S.clusters.size(), -1);
  for (int32_t f = 0; f < L; ++f) leaf_of_cluster[S.leaf_clusters[f]] = f;
  std::vector<int64_t> diag(L, -1);
  // per sweep position: near targets (as source) and the gather inputs of
  // classes 1..3 (as target)
  std::vector<std::vector<CTarget>> near(2 * L);
  std::vector<GatherLists> gl(2 * (size_t)L * kGatherClasses);
  auto gather_of = [&](int32_t s, int32_t p, int32_t cls) -> GatherLists& {
    return gl[((size_t)s * L + p) * kGatherClasses + (cls - 1)];
  };
  // distance classes: class c holds win[c] < d <= win[c + 1]; class 0 is
  // the chain's, the last is unbounded
  constexpr int32_t kNC = kGatherClasses + 1;
  int32_t win[kNC + 1];
  win[0] = 0;
  for (int32_t c = 1; c <= kLateWindow - kChainWindow + 1; ++c) win[c] = kChainWindow + c - 1;
  win[kNC - 1] = kMidWindow;
  win[kNC] = 1 << 30;
  const int32_t first_mid = kNC - 2;   // classes from here on use T-product chunks for low-rank blocks
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
    const int32_t s = lower ? 0 : 1;
    const bool dense = B.kind == kDense;
    const int32_t ldr = rc.size(), ldc = cc.size();
    // source leaves of sigma by distance class for the row leaf k:
    // [lo[c], hi[c]) for class c = 0 (near, the chain) .. 3
    auto classify = [&](int32_t k, int32_t* lo, int32_t* hi) {
      const int32_t f0 = cc.leaf_first, f1 = cc.leaf_last;
      for (int32_t c = 0; c < kNC; ++c) {
        if (s == 0) {   // d = k - f: class c holds k - win[c+1] <= f < k - win[c]
          hi[c] = c == 0 ? f1 : std::clamp(k - win[c], f0, f1);
          lo[c] = c == kNC - 1 ? f0 : std::clamp(k - win[c + 1], f0, f1);
        } else {        // d = f - k: class c holds k + win[c] < f <= k + win[c+1]
          lo[c] = c == 0 ? f0 : std::clamp(k + win[c] + 1, f0, f1);
          hi[c] = c == kNC - 1 ? f1 : std::clamp(k + win[c + 1] + 1, f0, f1);
        }
      }
    };
    auto pmax_of = [&](int32_t fa, int32_t fb) { return s == 0 ? pos(0, fb - 1) : pos(1, fa); };
    // low-rank: T-product chunks of the class 2 and 3 parts, shared by the
    // row leaves: boundaries at every row's class limits
    const int32_t tp0 = (int32_t)sc.tprod.size();
    if (!dense) {
      std::vector<int32_t> bounds;
      int32_t used0 = cc.leaf_last, used1 = cc.leaf_first;
      for (int32_t k = rc.leaf_first; k < rc.leaf_last; ++k) {
        int32_t lo[kNC], hi[kNC];
        classify(k, lo, hi);
        for (int32_t c = first_mid; c < kNC; ++c) {
          if (hi[c] <= lo[c]) continue;
          used0 = std::min(used0, lo[c]);
          used1 = std::max(used1, hi[c]);
          bounds.push_back(lo[c]);
          bounds.push_back(hi[c]);
        }
      }
      std::sort(bounds.begin(), bounds.end());
      bounds.erase(std::unique(bounds.begin(), bounds.end()), bounds.end());
      for (size_t i = 0; i + 1 < bounds.size(); ++i) {
        if (bounds[i] < used0 || bounds[i + 1] > used1) continue;
        // rows [bounds[i], bounds[i+1]) in pieces of whole leaves of at most
        // kTprodRows rows, each formed by its own task as soon as its leaves
        // are solved (the consumer sums the pieces)
        for (int32_t fa = bounds[i]; fa < bounds[i + 1];) {
          int32_t fb = fa + 1;
          while (fb < bounds[i + 1] && lc(fb).end - lc(fa).begin <= kTprodRows) ++fb;
          CTprod t{};
          t.yoff = st.yoff[b] + (lc(fa).begin - cc.begin);
          t.ldy = ldc;
          t.col0 = lc(fa).begin;
          t.ncols = lc(fb - 1).end - lc(fa).begin;
          t.slot = st.slot[b];
          t.cap = st.cap[b];
          t.pmax = pmax_of(fa, fb);
          t.sweep = s;
          t.member = 0;
          t.toff = toff;
          toff += t.cap;
          sc.tprod.push_back(t);
          fa = fb;
        }
      }
    }
    const int32_t tp1 = (int32_t)sc.tprod.size();
    for (int32_t k = rc.leaf_first; k < rc.leaf_last; ++k) {
      const ClusterNode& kc = lc(k);
      const int32_t pk = pos(s, k);
      int32_t lo[kNC], hi[kNC];
      classify(k, lo, hi);
      const int64_t row_off = kc.begin - rc.begin;
      // near pieces: one per source leaf
      for (int32_t f = lo[0]; f < hi[0]; ++f) {
        CTarget t{};
        t.dpos = pk - pos(s, f);
        t.m = kc.size();
        t.kind = dense ? 0 : 1;
        t.off = st.off[b] + row_off + (dense ? (int64_t)(lc(f).begin - cc.begin) * ldr : 0);
        t.ld = ldr;
        if (!dense) {
          t.yoff = st.yoff[b] + (lc(f).begin - cc.begin);
          t.ldy = ldc;
          t.slot = st.slot[b];
        }
        near[s * L + pos(s, f)].push_back(t);
      }
      for (int32_t c = 1; c < kNC; ++c) {
        const int32_t fa = lo[c], fb = hi[c];
        if (fb <= fa) continue;
        GatherLists& g = gather_of(s, pk, c);
        const int32_t pm = pmax_of(fa, fb);
        const int32_t col0 = lc(fa).begin, ncols = lc(fb - 1).end - col0;
        if (dense) {
          g.dense.push_back(GDense{st.off[b] + row_off + (int64_t)(col0 - cc.begin) * ldr, ldr, col0, ncols, pm});
        } else if (c < first_mid) {   // one source leaf, needed soon: formed inline
          g.inl.push_back(GInline{st.off[b] + row_off, st.yoff[b] + (col0 - cc.begin), ldr, ldc, st.slot[b], col0,
                                  ncols, pm});
        } else {               // through the T-product chunks covering [fa, fb)
          int32_t q0 = -1, q1 = -1;
          for (int32_t q = tp0; q < tp1; ++q) {
            const CTprod& t = sc.tprod[q];
            if (t.col0 >= col0 && t.col0 + t.ncols <= col0 + ncols) {
              if (q0 < 0) q0 = q;
              q1 = q + 1;
            }
          }
          HLU_REQUIRE(q0 >= 0, HLU_ERR_INVALID_ARG, "solve schedule: low-rank part without chunks");
          int32_t rows = 0;
          for (int32_t q = q0; q < q1; ++q) rows += sc.tprod[q].ncols;
          HLU_REQUIRE(rows == ncols, HLU_ERR_INVALID_ARG, "solve schedule: chunks do not tile a low-rank part");
          g.low.push_back(GLow{st.off[b] + row_off, ldr, q0, q1 - q0, 0});
        }
        g.pmax = std::max(g.pmax, pm);
      }
    }
  }
  sc.tbuf_per_rhs = toff;
  // positions, stacked operators (near targets by distance; rows beyond
  // kMaxStackRows are demoted to the target's late gather)
  sc.leaves.resize(2 * (size_t)L);
  std::vector<int64_t> inv(L);
  for (int32_t f = 0; f < L; ++f) {
    HLU_REQUIRE(diag[f] >= 0, HLU_ERR_INVALID_ARG, "solve schedule: missing diagonal leaf");
    HLU_REQUIRE(lc(f).size() <= 2 * kMaxLeafRows, HLU_ERR_UNSUPPORTED, "solve schedule: leaf cluster above 128 rows");
    inv[f] = sc.inv_elems;
    sc.inv_elems += (int64_t)lc(f).size() * lc(f).size();
    sc.max_m = std::max(sc.max_m, lc(f).size());
  }
  for (int32_t s = 0; s < 2; ++s) {
    for (int32_t p = 0; p < L; ++p) {
      const int32_t f = s == 0 ? p : L - 1 - p;
      CLeaf& lf = sc.leaves[s * L + p];
      lf.row0 = lc(f).begin;
      lf.m = lc(f).size();
      lf.leaf = f;
      lf.inv = inv[f];
      lf.diag = diag[f];
      std::vector<CTarget>& nt = near[s * L + p];
      std::stable_sort(nt.begin(), nt.end(), [](const CTarget& x, const CTarget& y) { return x.dpos < y.dpos; });
      int32_t rows = lf.m;
      lf.t0 = (int32_t)sc.tgt.size();
      for (const CTarget& t0 : nt) {
        if (rows + t0.m <= kMaxStackRows) {
          CTarget t = t0;
          t.srow0 = rows;
          rows += t.m;
          sc.tgt.push_back(t);
        } else {   // demoted: the target's class 1 gather multiplies it itself
          GatherLists& g = gather_of(s, p + t0.dpos, 1);
          const int32_t pm = p;
          if (t0.kind == 0) g.dense.push_back(GDense{t0.off, t0.ld, lf.row0, lf.m, pm});
          else g.inl.push_back(GInline{t0.off, t0.yoff, t0.ld, t0.ldy, t0.slot, lf.row0, lf.m, pm});
          g.pmax = std::max(g.pmax, pm);
        }
      }
      lf.nt = (int32_t)sc.tgt.size() - lf.t0;
      HLU_REQUIRE(lf.nt <= kMaxTargets, HLU_ERR_UNSUPPORTED, "solve schedule: too many near targets");
      lf.srows = rows;
      lf.stack = sc.stack_elems;
      sc.stack_elems += (int64_t)rows * lf.m;
    }
  }
  // gathers and T-product groups, with their claim keys
  struct Keyed {
    int32_t key, kind, idx;
  };
  std::vector<Keyed> order;
  std::vector<std::vector<int32_t>> chain_recs;   // per position (sweep-major): the records its chain reads
  for (int32_t s = 0; s < 2; ++s) {
    for (int32_t p = 0; p < L; ++p) {
      CLeaf& lf = sc.leaves[s * L + p];
      std::vector<int32_t> last_recs;   // the record of each class the chain reads
      for (int32_t c = 1; c < kNC; ++c) {
        GatherLists& g = gather_of(s, p, c);
        // inputs of the class, oldest source first (a gather works while
        // the newest is solved), packed into gathers of bounded work
        struct Item {
          int32_t pmax, kind, idx, cost;
        };
        std::vector<Item> items;
        for (size_t i = 0; i < g.dense.size(); ++i) items.push_back({g.dense[i].pmax, 0, (int32_t)i, g.dense[i].ncols});
        for (size_t i = 0; i < g.inl.size(); ++i) items.push_back({g.inl[i].pmax, 1, (int32_t)i, 16 + g.inl[i].ncols / 2});
        for (size_t i = 0; i < g.low.size(); ++i) {
          int32_t pm = -1;
          for (int32_t q = g.low[i].tp; q < g.low[i].tp + g.low[i].ntp; ++q) pm = std::max(pm, sc.tprod[q].pmax);
          items.push_back({pm, 2, (int32_t)i, 6 + 2 * g.low[i].ntp});
        }
        if (items.empty()) continue;
        std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) { return x.pmax < y.pmax; });
        int32_t prev = -1;
        for (size_t i0 = 0; i0 < items.size();) {
          size_t i1 = i0;
          int32_t cost = 0, pm = -1;
          while (i1 < items.size() && (i1 == i0 || cost + items[i1].cost <= kGatherBudget)) {
            cost += items[i1].cost;
            pm = std::max(pm, items[i1].pmax);
            ++i1;
          }
          CGather G{};
          G.pos = s * L + p;
          G.member = 0;
          G.m = lf.m;
          G.row0 = lf.row0;
          G.d0 = (int32_t)sc.gdense.size();
          G.l0 = (int32_t)sc.glow.size();
          G.i0 = (int32_t)sc.ginl.size();
          for (size_t i = i0; i < i1; ++i) {
            if (items[i].kind == 0) sc.gdense.push_back(g.dense[items[i].idx]);
            else if (items[i].kind == 1) sc.ginl.push_back(g.inl[items[i].idx]);
            else sc.glow.push_back(g.low[items[i].idx]);
          }
          G.nd = (int32_t)sc.gdense.size() - G.d0;
          G.ni = (int32_t)sc.ginl.size() - G.i0;
          G.nl = (int32_t)sc.glow.size() - G.l0;
          G.rec = sc.num_recs++;
          G.prev = prev;
          prev = G.rec;
          HLU_REQUIRE(pm < p - win[c] || (c == 1 && pm < p), HLU_ERR_INVALID_ARG,
                      "solve schedule: gather reads a source inside its window");
          order.push_back({s * L + pm, 1, (int32_t)sc.gathers.size()});
          sc.gathers.push_back(G);
          i0 = i1;
        }
        last_recs.push_back(prev);
      }
      // the records the chain reads, contiguous: moved to the end of the
      // record numbering of this leaf by a renumbering below
      lf.nrec = (int32_t)last_recs.size();
      lf.rec0 = last_recs.empty() ? 0 : last_recs[0];
      chain_recs.push_back(last_recs);
      HLU_REQUIRE(lf.nrec <= kMaxRecords, HLU_ERR_UNSUPPORTED, "solve schedule: too many gather records for a leaf");
    }
  }
  // renumber the records: the ones a chain reads come first, contiguous per
  // position; the inner records of linked classes after them
  {
    std::vector<int32_t> newid(sc.num_recs, -1);
    int32_t next = 0;
    for (size_t q = 0; q < chain_recs.size(); ++q) {
      CLeaf& lf = sc.leaves[q];
      lf.rec0 = next;
      for (int32_t r : chain_recs[q]) newid[r] = next++;
    }
    for (int32_t& id : newid)
      if (id < 0) id = next++;
    for (CGather& G : sc.gathers) {
      G.rec = newid[G.rec];
      if (G.prev >= 0) G.prev = newid[G.prev];
    }
  }
  // T-products of chunks with the same source rows share a task (at most
  // 8), in build order
  {
    std::vector<int32_t> idx(sc.tprod.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int32_t)i;
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) {
      const CTprod& a = sc.tprod[x];
      const CTprod& b = sc.tprod[y];
      if (a.sweep != b.sweep) return a.sweep < b.sweep;
      if (a.pmax != b.pmax) return a.pmax < b.pmax;
      if (a.col0 != b.col0) return a.col0 < b.col0;
      return a.ncols < b.ncols;
    });
    for (size_t i = 0; i < idx.size();) {
      const CTprod& t0 = sc.tprod[idx[i]];
      const int32_t id = (int32_t)sc.tg0.size();
      sc.tg0.push_back((int32_t)sc.tg_list.size());
      size_t j = i;
      int64_t rows = 0;   // a group forms its products one after the other: bound its rows
      while (j < idx.size() && j - i < 8) {
        const CTprod& t = sc.tprod[idx[j]];
        if (t.sweep != t0.sweep || t.col0 != t0.col0 || t.ncols != t0.ncols) break;
        if (j > i && rows + t.ncols > 2 * kTprodRows) break;
        rows += t.ncols;
        sc.tg_list.push_back(idx[j]);
        ++j;
      }
      order.push_back({t0.sweep * L + t0.pmax, 0, id});
      i = j;
    }
    sc.tg0.push_back((int32_t)sc.tg_list.size());
  }
  std::stable_sort(order.begin(), order.end(), [](const Keyed& x, const Keyed& y) {
    return x.key < y.key || (x.key == y.key && x.kind < y.kind);
  });
  for (const Keyed& k : order) sc.tasks.push_back(CTask{k.kind == 0 ? kTaskTprod : kTaskGather, k.idx});
  check_chain_sched(sc);
  // coverage: every (target leaf, source leaf) pair of every off-diagonal
  // block enters the solve exactly once, through the chain or a gather
  std::vector<uint8_t> seen(2 * (size_t)L * L, 0);
  int64_t marked = 0;
  std::vector<int32_t> leaf_at_row(S.N);
  for (int32_t f = 0; f < L; ++f)
    for (int32_t r = lc(f).begin; r < lc(f).end; ++r) leaf_at_row[r] = f;
  auto mark = [&](int32_t s, int32_t k, int32_t f) {
    uint8_t& v = seen[((size_t)s * L + k) * L + f];
    HLU_REQUIRE(v == 0, HLU_ERR_INVALID_ARG, "solve schedule: a block piece enters twice");
    v = 1;
    ++marked;
  };
  auto mark_rows = [&](int32_t s, int32_t k, int32_t col0, int32_t ncols) {
    for (int32_t f = leaf_at_row[col0]; f <= leaf_at_row[col0 + ncols - 1]; ++f) mark(s, k, f);
  };
  for (int32_t s = 0; s < 2; ++s)
    for (int32_t p = 0; p < L; ++p) {
      const CLeaf& lf = sc.leaves[s * L + p];
      for (int32_t j = lf.t0; j < lf.t0 + lf.nt; ++j) mark(s, sc.leaves[s * L + p + sc.tgt[j].dpos].leaf, lf.leaf);
    }
  for (const CGather& g : sc.gathers) {
    const int32_t s = g.pos / L, k = sc.leaves[g.pos].leaf;
    for (int32_t i = g.d0; i < g.d0 + g.nd; ++i) mark_rows(s, k, sc.gdense[i].col0, sc.gdense[i].ncols);
    for (int32_t i = g.i0; i < g.i0 + g.ni; ++i) mark_rows(s, k, sc.ginl[i].col0, sc.ginl[i].ncols);
    for (int32_t i = g.l0; i < g.l0 + g.nl; ++i)
      for (int32_t q = sc.glow[i].tp; q < sc.glow[i].tp + sc.glow[i].ntp; ++q)
        mark_rows(s, k, sc.tprod[q].col0, sc.tprod[q].ncols);
  }
  int64_t expected = 0;
  for (size_t b = 0; b < S.leaves.size(); ++b) {
    const BlockNode& B = S.blocks[S.leaves[b]];
    if (B.row == B.col) continue;
    expected += (int64_t)(S.clusters[B.row].leaf_last - S.clusters[B.row].leaf_first) *
                (S.clusters[B.col].leaf_last - S.clusters[B.col].leaf_first);
  }
  HLU_REQUIRE(marked == expected, HLU_ERR_INVALID_ARG, "solve schedule: block pieces missing from the solve");
  if (getenv("HLU_DEBUG_SCHED")) {   // debug: schedule sizes
    int64_t nt = 0, maxntp = 0;
    for (const GLow& g : sc.glow) { nt += g.ntp; maxntp = std::max<int64_t>(maxntp, g.ntp); }
    fprintf(stderr, "chain schedule: L %d tprod %zu groups %zu gathers %zu dense %zu inline %zu low %zu (chunks %lld, max %lld) "
            "tasks %zu stack %lld\n", L, sc.tprod.size(), sc.tg0.size() - 1, sc.gathers.size(), sc.gdense.size(),
            sc.ginl.size(), sc.glow.size(), (long long)nt, (long long)maxntp, sc.tasks.size(), (long long)sc.stack_elems);
  }
}

void merge_chain_scheds(const std::vector<const ChainSched*>& S, const std::vector<int64_t>& a,
                        const std::vector<int32_t>& d, const std::vector<int32_t>& o, ChainSched* out) {
  ChainSched& M = *out;
  M = ChainSched{};
  const size_t np = S.size();
  M.members = (int32_t)np;
  std::vector<int32_t> LB(np), TGB(np), TPB(np), GB(np), RB(np);
  std::vector<int64_t> SB(np), IB(np), TB(np);
  for (size_t p = 0; p < np; ++p) {
    LB[p] = M.L;
    M.L += S[p]->L;
    M.member_L.push_back(S[p]->L);
    M.member_pos0.push_back(LB[p]);
  }
  M.leaves.resize(2 * (size_t)M.L);
  for (size_t p = 0; p < np; ++p) {
    const ChainSched& s = *S[p];
    SB[p] = M.stack_elems;
    IB[p] = M.inv_elems;
    TB[p] = M.tbuf_per_rhs;
    TPB[p] = (int32_t)M.tprod.size();
    TGB[p] = (int32_t)M.tg0.size();
    GB[p] = (int32_t)M.gathers.size();
    RB[p] = M.num_recs;
    const int32_t T0 = (int32_t)M.tgt.size(), D0 = (int32_t)M.gdense.size(), W0 = (int32_t)M.glow.size(),
                  I0 = (int32_t)M.ginl.size();
    for (CTarget t : s.tgt) {
      t.off += a[p];
      t.yoff += a[p];
      t.slot += d[p];
      M.tgt.push_back(t);
    }
    for (GDense g : s.gdense) {
      g.off += a[p];
      g.col0 += o[p];
      M.gdense.push_back(g);
    }
    for (GLow g : s.glow) {
      g.xoff += a[p];
      g.tp += TPB[p];
      M.glow.push_back(g);
    }
    for (GInline g : s.ginl) {
      g.xoff += a[p];
      g.yoff += a[p];
      g.slot += d[p];
      g.col0 += o[p];
      M.ginl.push_back(g);
    }
    for (CTprod t : s.tprod) {
      t.yoff += a[p];
      t.toff += TB[p];
      t.col0 += o[p];
      t.slot += d[p];
      t.member = (int32_t)p;
      M.tprod.push_back(t);
    }
    for (size_t i = 0; i + 1 < s.tg0.size(); ++i) M.tg0.push_back(s.tg0[i] - s.tg0[0] + (int32_t)M.tg_list.size());
    for (int32_t q : s.tg_list) M.tg_list.push_back(q + TPB[p]);
    for (CGather g : s.gathers) {
      const int32_t sw = g.pos / s.L, pp = g.pos % s.L;
      g.pos = sw * M.L + LB[p] + pp;
      g.member = (int32_t)p;
      g.row0 += o[p];
      g.d0 += D0;
      g.l0 += W0;
      g.i0 += I0;
      g.rec += RB[p];
      if (g.prev >= 0) g.prev += RB[p];
      M.gathers.push_back(g);
    }
    for (int32_t q = 0; q < 2 * s.L; ++q) {
      CLeaf lf = s.leaves[q];
      lf.row0 += o[p];
      lf.stack += SB[p];
      lf.inv += IB[p];
      lf.diag += a[p];
      lf.t0 += T0;
      lf.rec0 += RB[p];
      const int32_t sw = q / s.L, pp = q % s.L;
      M.leaves[(size_t)sw * M.L + LB[p] + pp] = lf;
    }
    M.stack_elems += s.stack_elems;
    M.inv_elems += s.inv_elems;
    M.tbuf_per_rhs += s.tbuf_per_rhs;
    M.num_recs += s.num_recs;
    M.max_m = std::max(M.max_m, s.max_m);
  }
  M.tg0.push_back((int32_t)M.tg_list.size());
  // interleave the members' helper tasks: each advances in proportion to
  // its own sweep length (its own order kept, so every wait still points
  // backwards within the member)
  struct Key {
    double pos;
    int32_t p, i;
  };
  std::vector<Key> keys;
  for (size_t p = 0; p < np; ++p) {
    const ChainSched& s = *S[p];
    const int32_t n = (int32_t)s.tasks.size();
    for (int32_t i = 0; i < n; ++i) keys.push_back({(i + 0.5) / (double)n, (int32_t)p, i});
  }
  std::stable_sort(keys.begin(), keys.end(),
                   [](const Key& x, const Key& y) { return x.pos < y.pos || (x.pos == y.pos && x.p < y.p); });
  for (const Key& k : keys) {
    CTask t = S[k.p]->tasks[k.i];
    t.idx += t.kind == kTaskTprod ? TGB[k.p] : GB[k.p];
    M.tasks.push_back(t);
  }
  check_chain_sched(M);
}

// Claim-order check.  For every member: each helper task reads T-products
// formed by earlier helper tasks only, and the chain progress it waits for
// is at most the latest source position of the helper tasks that any
// chain of the member waits on before it ... in other words: ordering the
// member's helpers by their key (sweep, latest source position), a chain
// at position p waits only on gathers whose keys are below p - kChainWindow
// (late gathers: below p), and all helper tasks claimed before those carry
// keys no larger.  Checked here on the merged task list.
void check_chain_sched(const ChainSched& sc) {
  const size_t nt = sc.tasks.size();
  std::vector<int32_t> tp_at(sc.tprod.size(), -1), rec_at(sc.num_recs, -1);
  std::vector<int32_t> last_key(sc.members, -1);   // keys of a member's tasks never decrease
  auto key_of = [&](const CTask& t, int32_t* member) -> int32_t {
    if (t.kind == kTaskTprod) {
      const CTprod& p = sc.tprod[sc.tg_list[sc.tg0[t.idx]]];
      *member = p.member;
      return p.sweep * sc.member_L[p.member] + p.pmax;
    }
    const CGather& g = sc.gathers[t.idx];
    *member = g.member;
    const int32_t Lm = sc.member_L[g.member];
    const int32_t sw = g.pos / sc.L;
    int32_t pm = -1;
    for (int32_t i = g.d0; i < g.d0 + g.nd; ++i) pm = std::max(pm, sc.gdense[i].pmax);
    for (int32_t i = g.i0; i < g.i0 + g.ni; ++i) pm = std::max(pm, sc.ginl[i].pmax);
    for (int32_t i = g.l0; i < g.l0 + g.nl; ++i)
      for (int32_t q = sc.glow[i].tp; q < sc.glow[i].tp + sc.glow[i].ntp; ++q) pm = std::max(pm, sc.tprod[q].pmax);
    return sw * Lm + pm;
  };
  for (size_t i = 0; i < nt; ++i) {
    const CTask& t = sc.tasks[i];
    int32_t member = 0;
    const int32_t key = key_of(t, &member);
    HLU_REQUIRE(key >= last_key[member], HLU_ERR_INVALID_ARG, "solve schedule: helper keys out of order");
    last_key[member] = key;
    if (t.kind == kTaskTprod) {
      for (int32_t q = sc.tg0[t.idx]; q < sc.tg0[t.idx + 1]; ++q) {
        HLU_REQUIRE(tp_at[sc.tg_list[q]] < 0, HLU_ERR_INVALID_ARG, "solve schedule: T-product formed twice");
        tp_at[sc.tg_list[q]] = (int32_t)i;
      }
    } else {
      const CGather& g = sc.gathers[t.idx];
      for (int32_t w = g.l0; w < g.l0 + g.nl; ++w)
        for (int32_t q = sc.glow[w].tp; q < sc.glow[w].tp + sc.glow[w].ntp; ++q)
          HLU_REQUIRE(tp_at[q] >= 0 && tp_at[q] < (int32_t)i, HLU_ERR_INVALID_ARG,
                      "solve schedule: a gather reads a T-product no earlier task forms");
      HLU_REQUIRE(rec_at[g.rec] < 0, HLU_ERR_INVALID_ARG, "solve schedule: record written twice");
      HLU_REQUIRE(g.prev < 0 || (rec_at[g.prev] >= 0 && rec_at[g.prev] < (int32_t)i), HLU_ERR_INVALID_ARG,
                  "solve schedule: a gather adds a record no earlier task writes");
      rec_at[g.rec] = (int32_t)i;
    }
  }
  for (int32_t q : tp_at) HLU_REQUIRE(q >= 0, HLU_ERR_INVALID_ARG, "solve schedule: T-product never formed");
  // every record a chain waits on is produced, from sources behind the chain
  for (size_t q = 0; q < sc.leaves.size(); ++q) {
    const CLeaf& lf = sc.leaves[q];
    for (int32_t rec = lf.rec0; rec < lf.rec0 + lf.nrec; ++rec)
      HLU_REQUIRE(rec < sc.num_recs && rec_at[rec] >= 0, HLU_ERR_INVALID_ARG,
                  "solve schedule: a chain waits on a record no task writes");
  }
}

}  // namespace hlu
