// C ABI of libhlu (include/hlu.h), single-problem part: handles, workspace
// binding, the factor and solve drivers that launch the planned waves and
// the persistent solve.  Batches are in batch.cpp, GMRES in gmres.cpp.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "handle.h"
#include "mesh.h"
#include "trunc_rounds.h"

namespace hlu {

// ------------------------------------------------------------- errors
namespace {
thread_local std::string g_last_error;
}
void set_error(const std::string& msg) { g_last_error = msg; }
const char* get_error() { return g_last_error.c_str(); }


// ------------------------------------------------------------- layout
WorkLayout work_layout(const PlanSet& ps, int32_t prec) {
  WorkLayout L;
  L.arena_bytes = align256((size_t)ps.store.total_elems * elem_size(prec));
  L.dims_off = L.arena_bytes;
  L.status_off = L.dims_off + align256((size_t)ps.store.num_slots * sizeof(int32_t));
  L.peak_off = L.status_off + align256(kStatusWords * sizeof(int32_t));
  L.total = L.peak_off + (size_t)ps.store.num_slots * sizeof(int32_t);
  return L;
}

int32_t kcap_for(const hlu_factor_opts* o) {
  int32_t k = kDefaultCap;
  if (o->max_rank > 0) k = std::min(o->max_rank, kDefaultCap);
  return k;
}

void check_opts(const hlu_factor_opts* o) {
  HLU_REQUIRE(o != nullptr, HLU_ERR_INVALID_ARG, "factor options are NULL");
  HLU_REQUIRE(o->eps >= 0.0 && std::isfinite(o->eps), HLU_ERR_INVALID_ARG, "eps must be finite and >= 0");
  HLU_REQUIRE(o->max_rank >= 0, HLU_ERR_INVALID_ARG, "max_rank must be >= 0");
  HLU_REQUIRE(o->prec == HLU_FP32 || o->prec == HLU_FP64 || o->prec == HLU_FP32_ACC64, HLU_ERR_INVALID_ARG,
              "prec must be HLU_FP64, HLU_FP32 or HLU_FP32_ACC64");
}

std::shared_ptr<PlanBundle> get_bundle(Shared& sh, int32_t kcap) {
  std::lock_guard<std::mutex> lock(sh.mu);
  auto it = sh.bundles.find(kcap);
  if (it != sh.bundles.end()) return it->second;
  auto pb = std::make_shared<PlanBundle>();
  pb->kcap = kcap;
  build_plans(sh.S, kcap, kMaxRhs, sh.nonzero_admissible, &pb->ps);
  build_chain_sched(sh.S, pb->ps.store, &pb->sc);
  sh.bundles[kcap] = pb;
  return pb;
}

void ensure_device(Shared& sh, PlanBundle& pb) {
  std::lock_guard<std::mutex> lock(sh.mu);
  if (!sh.d_perm) sh.d_perm = sh.mem.keep(upload(sh.S.perm));
  if (pb.on_device) return;
  pb.dfactor.load(pb.ps.factor);
  pb.dsolve.load(pb.ps.fwd_bwd);
  pb.dapply.load(pb.ps.apply);
  pb.dsc.load(pb.sc);
  ensure_targets(sh, pb);
  pb.on_device = true;
}

namespace {
template <class V>
size_t vbytes(const V& v) {
  return v.size() * sizeof(typename V::value_type);
}
size_t plan_device_bytes(const Plan& p) {
  return vbytes(p.getrf) + vbytes(p.tri) + vbytes(p.gemm) + vbytes(p.terms) + vbytes(p.trunc) + vbytes(p.parts) +
         vbytes(p.fill) + vbytes(p.gemm_tile_op) + vbytes(p.gemm_tile_ij);
}
}  // namespace

size_t bundle_device_bytes(const Shared& sh, const PlanBundle& pb) {
  const ChainSched& sc = pb.sc;
  size_t b = plan_device_bytes(pb.ps.factor) + plan_device_bytes(pb.ps.fwd_bwd) + plan_device_bytes(pb.ps.apply);
  b += vbytes(sc.leaves) + vbytes(sc.tgt) + vbytes(sc.gdense) + vbytes(sc.glow) + vbytes(sc.ginl) +
       vbytes(sc.gathers) + vbytes(sc.tprod) + vbytes(sc.tg0) + vbytes(sc.tg_list) + vbytes(sc.tasks) +
       vbytes(sc.member_L) + vbytes(sc.member_pos0);
  b += sh.col.size() * sizeof(int64_t);      // scatter targets
  b += sh.S.perm.size() * sizeof(int32_t);   // permutation
  return b;
}

// The buffers of a persistent solve, carved in this order from one region
// (caller memory bound with hlu_bind_solve_workspace) or each allocated by
// the library; `take(bytes)` hands out the next piece.
template <class Take>
void carve_solve_bufs(SolveBufs& b, const ChainSched& sc, int32_t N, int32_t rhs, Take take) {
  b.max_rhs = rhs;
  b.inv = take((size_t)std::max<int64_t>(1, sc.inv_elems) * sizeof(double));   // sized for FP64
  b.stack = take((size_t)std::max<int64_t>(1, sc.stack_elems) * sizeof(double));
  b.pivots = static_cast<double*>(take((size_t)N * sizeof(double)));
  b.y = static_cast<double*>(take((size_t)N * rhs * sizeof(double)));
  b.tbuf = static_cast<double*>(take((size_t)std::max<int64_t>(1, sc.tbuf_per_rhs) * rhs * sizeof(double)));
  b.rstride = (int64_t)sc.max_m * rhs;
  b.fbuf = static_cast<double*>(take((size_t)std::max(1, sc.num_recs) * (size_t)b.rstride * sizeof(double)));
  const size_t nflags = sc.tprod.size() + (size_t)sc.num_recs + 1;
  b.flags = static_cast<int32_t*>(take(nflags * sizeof(int32_t)));
  b.prog = static_cast<int32_t*>(take(2 * kMaxChains * sizeof(int32_t)));
  b.ctr = static_cast<int32_t*>(take(kSolveCtrWords * sizeof(int32_t)));
  b.kargs = take(kChainArgBytes);
  if (b.flags) {
    HIP_OK(hipMemset(b.flags, 0, nflags * sizeof(int32_t)));
    HIP_OK(hipMemset(b.prog, 0, 2 * kMaxChains * sizeof(int32_t)));
    HIP_OK(hipMemset(b.ctr, 0, kSolveCtrWords * sizeof(int32_t)));
  }
  b.epoch = 0;
}

void SolveBufs::alloc(const ChainSched& sc, int32_t N, int32_t rhs) {
  carve_solve_bufs(*this, sc, N, rhs, [&](size_t bytes) -> void* { return mem.keep(dmalloc<unsigned char>(bytes)); });
  if (getenv("HLU_DEBUG_SOLVE_TRACE"))
    trace = mem.keep(dmalloc<int64_t>(10 * (size_t)std::max(1, sc.L) + 6 * (size_t)std::max(1, sc.num_recs)));
}

void SolveBufs::place(const ChainSched& sc, int32_t N, int32_t rhs, void* base, size_t bytes) {
  size_t used = 0;
  carve_solve_bufs(*this, sc, N, rhs, [&](size_t n) -> void* {
    void* p = static_cast<char*>(base) + used;
    used += align256(n);
    HLU_REQUIRE(used <= bytes, HLU_ERR_OUT_OF_MEMORY, "solve workspace too small");
    return p;
  });
}

size_t solve_buffer_bytes(const ChainSched& sc, int32_t N, int32_t rhs) {
  size_t used = 0;
  SolveBufs probe;
  carve_solve_bufs(probe, sc, N, rhs, [&](size_t n) -> void* {
    used += align256(n);
    return nullptr;
  });
  return used;
}

int64_t solve_wait_ticks() {
  static std::once_flag once;
  static int64_t khz = 100000;   // 100 MHz unless the device says otherwise
  std::call_once(once, [] {
    int dev = 0, r = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&r, hipDeviceAttributeWallClockRate, dev) == hipSuccess &&
        r > 0)
      khz = r;
  });
  double us = 20e6;
  if (const char* e = getenv("HLU_DEBUG_SOLVE_WAIT_US")) us = std::max(0.0, atof(e));
  return (int64_t)(us * (double)khz / 1000.0);
}

bool take_solve_error(int32_t* ctr, hipStream_t s) {
  int32_t e = 0;
  HIP_OK(hipMemcpyAsync(&e, ctr + 3, sizeof(e), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (e == 0) return false;
  HIP_OK(zero_int_launch(ctr + 3, 1, s));
  HIP_OK(hipStreamSynchronize(s));
  return true;
}

ChainDev make_chain_dev(const ChainSched& sc, const DevSched& d, const SolveBufs& b) {
  ChainDev v{};
  v.leaves = d.leaves;
  v.tgt = d.tgt;
  v.gdense = d.gdense;
  v.glow = d.glow;
  v.ginl = d.ginl;
  v.gathers = d.gathers;
  v.tprod = d.tprod;
  v.tg0 = d.tg0;
  v.tg_list = d.tg_list;
  v.tasks = d.tasks;
  v.member_L = d.member_L;
  v.member_pos0 = d.member_pos0;
  v.stack = b.stack;
  v.inv = b.inv;
  v.pivots = b.pivots;
  v.y = b.y;
  v.tbuf = b.tbuf;
  v.fbuf = b.fbuf;
  v.tp_flag = b.flags;
  v.g_flag = b.flags + sc.tprod.size();
  v.prog = b.prog;
  v.ctr = b.ctr;
  v.rstride = b.rstride;
  v.trace = b.trace;
  v.kargs = b.kargs;
  v.wait_ticks = solve_wait_ticks();
  v.ntasks = (int32_t)sc.tasks.size();
  v.L = sc.L;
  v.members = sc.members;
  v.max_m = sc.max_m;
  v.max_rhs = b.max_rhs;
  return v;
}

void ensure_values(hlu_s* h) {
  if (!h->d_val) h->d_val = h->mem.keep(upload(h->val));
}

void ensure_targets(Shared& sh, PlanBundle& pb) {
  if (pb.d_target) return;
  // arena element of every stored entry (dense leaf or staging block)
  const Structure& S = sh.S;
  const StoragePlan& st = pb.ps.store;
  std::vector<int64_t> init_off(S.leaves.size(), -1);
  for (const InitBlock& ib : pb.ps.init_blocks) init_off[ib.leaf] = ib.off;
  std::vector<int32_t> iperm(S.N);
  for (int32_t i = 0; i < S.N; ++i) iperm[S.perm[i]] = i;
  std::vector<int64_t> target(sh.col.size(), -1);
  for (int32_t r = 0; r < S.N; ++r) {
    const int32_t i = iperm[r];
    for (int32_t p = sh.row_ptr[r]; p < sh.row_ptr[r + 1]; ++p) {
      const int32_t j = iperm[sh.col[p]];
      // leaf block containing (i, j): walk down the block tree
      int32_t node = 0;
      while (S.blocks[node].kind == kSub) {
        const BlockNode& b = S.blocks[node];
        const ClusterNode& rc = S.clusters[b.row];
        const ClusterNode& cc = S.clusters[b.col];
        const int32_t qi = i < S.clusters[rc.son[0]].end ? 0 : 1;
        const int32_t qj = j < S.clusters[cc.son[0]].end ? 0 : 1;
        node = b.son[2 * qi + qj];
      }
      const BlockNode& b = S.blocks[node];
      const ClusterNode& rc = S.clusters[b.row];
      const ClusterNode& cc = S.clusters[b.col];
      const int64_t base = b.kind == kDense ? st.off[b.leaf_id] : init_off[b.leaf_id];
      HLU_REQUIRE(base >= 0, HLU_ERR_INVALID_ARG, "internal: entry without storage");
      target[p] = base + (i - rc.begin) + (int64_t)(j - cc.begin) * rc.size();
    }
  }
  pb.d_target = pb.mem.keep(upload(target));
}

void ensure_solve_bufs(hlu_s* h) {
  if (h->sbuf) return;
  auto b = std::make_unique<SolveBufs>();
  if (h->solve_work) b->place(h->pb->sc, h->sh->S.N, kMaxRhs, h->solve_work, h->solve_work_bytes);
  else b->alloc(h->pb->sc, h->sh->S.N, kMaxRhs);
  h->sbuf = std::move(b);
  h->inv_ready = false;
}

// A into a zeroed arena, ranks cleared.
template <class T>
void factor_prepare(hlu_s* h, T* arena, int32_t* dims, hipStream_t s) {
  const StoragePlan& st = h->pb->ps.store;
  ensure_values(h);
  HIP_OK(zero_launch<T>(arena, st.data_elems, s));
  HIP_OK(identity_launch<T>(arena + st.identity_off, st.identity_n, s));
  HIP_OK(scatter_values_launch<T>((int64_t)h->val.size(), h->pb->d_target, h->d_val, arena, s));
  HIP_OK(zero_int_launch(dims, st.num_slots, s));
}
template void factor_prepare<float>(hlu_s*, float*, int32_t*, hipStream_t);
template void factor_prepare<double>(hlu_s*, double*, int32_t*, hipStream_t);

void gather_stats(hlu_s* h, const double* d_pivots) {
  const StoragePlan& st = h->pb->ps.store;
  const Structure& S = h->sh->S;
  std::vector<int32_t> dims(st.num_slots);
  HIP_OK(hipMemcpy(dims.data(), h->dims, dims.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  int32_t maxr = 0;
  double sumr = 0, lr_entries = 0;
  int64_t nlr = 0;
  for (size_t l = 0; l < S.leaves.size(); ++l) {
    if (st.slot[l] < 0) continue;
    const BlockNode& b = S.blocks[S.leaves[l]];
    const int32_t r = dims[st.slot[l]];
    maxr = std::max(maxr, r);
    sumr += r;
    lr_entries += (double)r * (S.clusters[b.row].size() + S.clusters[b.col].size());
    ++nlr;
  }
  h->stats.max_rank = maxr;
  h->stats.mean_rank = nlr ? sumr / nlr : 0.0;
  h->stats.lowrank_entries = lr_entries;
  std::vector<double> piv(S.N);
  HIP_OK(hipMemcpy(piv.data(), d_pivots, piv.size() * sizeof(double), hipMemcpyDeviceToHost));
  double lo = INFINITY, hi = 0.0;
  for (double p : piv) {
    lo = std::min(lo, std::fabs(p));
    hi = std::max(hi, std::fabs(p));
  }
  h->stats.min_abs_pivot = lo;
  h->stats.max_abs_pivot = hi;
}

// Nominal flops of the last factorisation from the status words.
void read_flops(const int32_t* d_status, hlu_stats* st) {
  uint64_t f[kNumFlopKinds * kFlopSpread];
  HIP_OK(hipMemcpy(f, d_status + kFlopWord0, sizeof(f), hipMemcpyDeviceToHost));
  double k[kNumFlopKinds] = {0, 0, 0, 0};
  for (int i = 0; i < kNumFlopKinds * kFlopSpread; ++i) k[i / kFlopSpread] += (double)f[i];
  st->factor_flops_getrf = k[kFlopGetrf];
  st->factor_flops_tri = k[kFlopTri];
  st->factor_flops_gemm = k[kFlopGemm];
  st->factor_flops_trunc = k[kFlopTrunc];
  st->factor_flops = k[0] + k[1] + k[2] + k[3];
}

// Adds the durations of the recorded event pairs to the timing totals.
void harvest_timing(hlu_s* h) {
  for (size_t i = 0; i + 1 < h->tev_used; i += 2) {
    HIP_OK(hipEventSynchronize(h->tev[i + 1]));
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, h->tev[i], h->tev[i + 1]));
    h->stats.solve_launches += 1;
    h->stats.solve_kernel_ms += ms;
  }
  h->tev_used = 0;
}

int64_t* trunc_trace_buffer(size_t* ops);

// Debug: writes the per-op truncation trace of the last factorisation to
// the file named by HLU_DEBUG_TRUNC_TRACE.
void dump_trunc_trace(const Plan& pl) {
  const char* path = getenv("HLU_DEBUG_TRUNC_TRACE");
  size_t cap = 0;
  int64_t* buf = trunc_trace_buffer(&cap);
  if (!path || !buf) return;
  const size_t n = std::min(cap, pl.trunc.size());
  std::vector<int64_t> t((size_t)kTruncTraceFields * n);
  HIP_OK(hipMemcpy(t.data(), buf, t.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
  if (FILE* f = fopen(path, "wb")) {
    fwrite(t.data(), sizeof(int64_t), t.size(), f);
    fclose(f);
  }
  if (FILE* f = fopen((std::string(path) + ".waves").c_str(), "wb")) {
    for (const Wave& w : pl.waves) {
      const int32_t v[2] = {w.begin[kTrunc], w.count[kTrunc]};
      fwrite(v, sizeof(v), 1, f);
    }
    fclose(f);
  }
}

double rank_capacity_entries(const Structure& S, const StoragePlan& st) {
  double e = 0.0;
  for (size_t l = 0; l < S.leaves.size(); ++l) {
    if (st.slot[l] < 0) continue;
    const BlockNode& b = S.blocks[S.leaves[l]];
    e += (double)(S.clusters[b.row].size() + S.clusters[b.col].size()) * st.cap[l];
  }
  return e;
}

void record_factor(hlu_s* h, const hlu_factor_opts* o) {
  h->prec = o->prec;
  h->eps = o->eps;
  h->max_rank = o->max_rank;
  h->factor_compute64 = fp64_tasks(o->prec);
  const PlanSet& ps = h->pb->ps;
  h->stats.workspace_bytes = (int64_t)work_layout(ps, o->prec).total;
  h->stats.rank_capacity_entries = rank_capacity_entries(h->sh->S, ps.store);
  h->stats.factor_waves = (int64_t)ps.factor.waves.size();
  h->stats.factor_tasks = ps.factor.num_tasks;
  h->stats.solve_waves = (int64_t)ps.fwd_bwd.waves.size();
}

namespace {

template <class T>
void run_plan(hlu_s* h, const Plan& pl, const DevArrays& d, bool compute64, hipStream_t s,
              int32_t* peak = nullptr) {
  HIP_OK(run_waves<T>(static_cast<T*>(h->arena), d.P, pl.waves, h->dims, h->status, h->eps, kFloorRel,
                      h->sh->max_leaf, compute64, s, peak, &h->waves));
}

template <class T>
void ensure_inverses(hlu_s* h, hipStream_t s) {
  ensure_solve_bufs(h);
  if (h->inv_ready) return;
  const ChainDev d = make_chain_dev(h->pb->sc, h->pb->dsc, *h->sbuf);
  HIP_OK(chain_prepare_launch<T>(static_cast<const T*>(h->arena), h->dims, d, d.L, s));
  h->inv_ready = true;
}

template <class T>
void factor_impl(hlu_s* h, hipStream_t s) {
  T* arena = static_cast<T*>(h->arena);
  factor_prepare<T>(h, arena, h->dims, s);
  HIP_OK(zero_int_launch(h->status, kStatusWords, s));
  if (h->peak) HIP_OK(zero_int_launch(h->peak, h->pb->ps.store.num_slots, s));   // not for batch members
  run_plan<T>(h, h->pb->ps.factor, h->pb->dfactor, h->factor_compute64, s, h->peak);
  // the persistent solve applies the diagonal leaves through their inverses
  h->inv_ready = false;
  ensure_inverses<T>(h, s);
}

template <class T>
void solve_impl(hlu_s* h, const Plan& pl, const DevArrays& d, const double* b, double* x, int32_t nrhs, int64_t ld,
                hipStream_t s) {
  const StoragePlan& st = h->pb->ps.store;
  T* arena = static_cast<T*>(h->arena);
  const int32_t N = h->sh->S.N;
  for (int32_t c0 = 0; c0 < nrhs; c0 += st.max_rhs) {
    const int32_t nc = std::min(st.max_rhs, nrhs - c0);
    HIP_OK(gather_launch<T>(N, nc, h->sh->d_perm, b + (int64_t)c0 * ld, ld, arena + st.vec_off, N, s));
    HIP_OK(set_int_launch(h->dims + st.nrhs_slot, nc, s));
    // the solves read FP32 factors but accumulate in FP64
    run_plan<T>(h, pl, d, true, s);
    HIP_OK(scatter_perm_launch<T>(N, nc, h->sh->d_perm, arena + st.vec_off, N, x + (int64_t)c0 * ld, ld, s));
  }
}

// x = P^T U^{-1} L^{-1} P b with the persistent solve kernel (FP64 vectors).
template <class T>
void solve_persistent_impl(hlu_s* h, const double* b, double* x, int32_t nrhs, int64_t ld, hipStream_t s) {
  ensure_inverses<T>(h, s);
  SolveBufs& sb = *h->sbuf;
  const ChainSched& sc = h->pb->sc;
  const ChainDev d = make_chain_dev(sc, h->pb->dsc, sb);
  const T* arena = static_cast<const T*>(h->arena);
  const int32_t N = h->sh->S.N;
  for (int32_t c0 = 0; c0 < nrhs; c0 += kMaxRhs) {
    const int32_t nc = std::min(kMaxRhs, nrhs - c0);
    HIP_OK(gather_launch<double>(N, nc, h->sh->d_perm, b + (int64_t)c0 * ld, ld, sb.y, N, s));
    sb.epoch = sb.epoch % 1000000000 + 1;
    if (h->timing) {
      if (h->tev_used + 2 > kMaxTimedEvents) harvest_timing(h);
      while (h->tev.size() < h->tev_used + 2) {
        hipEvent_t e;
        HIP_OK(hipEventCreate(&e));
        h->tev.push_back(e);
      }
      HIP_OK(hipEventRecord(h->tev[h->tev_used], s));
    }
    if (sb.trace) HIP_OK(hipMemsetAsync(sb.trace, 0, 10 * (size_t)sc.L * sizeof(int64_t), s));   // debug
    HIP_OK(chain_solve_launch<T>(arena, h->dims, d, N, nc, sb.epoch, s));
    if (h->timing) {
      HIP_OK(hipEventRecord(h->tev[h->tev_used + 1], s));
      h->tev_used += 2;
      h->stats.solve_columns += nc;
    }
    HIP_OK(scatter_perm_launch<double>(N, nc, h->sh->d_perm, sb.y, N, x + (int64_t)c0 * ld, ld, s));
    if (sb.trace) {   // debug: the chain's clocks of this launch
      HIP_OK(hipStreamSynchronize(s));
      std::vector<int64_t> tr(10 * (size_t)sc.L + 6 * (size_t)sc.num_recs);
      HIP_OK(hipMemcpy(tr.data(), sb.trace, tr.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
      if (FILE* f = fopen(getenv("HLU_DEBUG_SOLVE_TRACE"), "wb")) {
        fwrite(tr.data(), sizeof(int64_t), tr.size(), f);
        fclose(f);
      }
    }
  }
}

void fill_structure_stats(hlu_s* h) {
  const Structure& S = h->sh->S;
  hlu_stats& st = h->stats;
  st = hlu_stats{};
  st.n = S.N;
  st.num_clusters = (int64_t)S.clusters.size();
  st.num_leaf_clusters = (int64_t)S.leaf_clusters.size();
  st.depth = S.depth;
  for (int32_t node : S.leaves) {
    const BlockNode& b = S.blocks[node];
    const int64_t m = S.clusters[b.row].size(), n = S.clusters[b.col].size();
    if (b.kind == kDense) {
      st.num_dense++;
      st.dense_entries += m * n;
    } else {
      st.num_admissible++;
      st.lowrank_rows_plus_cols += m + n;
    }
  }
}

void check_csr(const hlu_csr* A) {
  HLU_REQUIRE(A && A->row_ptr && A->col && A->val, HLU_ERR_INVALID_ARG, "NULL matrix");
  HLU_REQUIRE(A->n > 0 && A->nnz >= 0, HLU_ERR_INVALID_ARG, "need n > 0 and nnz >= 0");
  const int32_t n = A->n;
  HLU_REQUIRE(A->row_ptr[0] == 0 && A->row_ptr[n] == A->nnz, HLU_ERR_INVALID_ARG, "malformed row_ptr");
  for (int32_t r = 0; r < n; ++r) {
    HLU_REQUIRE(A->row_ptr[r + 1] >= A->row_ptr[r], HLU_ERR_INVALID_ARG, "row_ptr not monotone");
    for (int32_t p = A->row_ptr[r]; p < A->row_ptr[r + 1]; ++p) {
      HLU_REQUIRE(A->col[p] >= 0 && A->col[p] < n, HLU_ERR_INVALID_ARG, "column index out of range");
      HLU_REQUIRE(p == A->row_ptr[r] || A->col[p] > A->col[p - 1], HLU_ERR_INVALID_ARG,
                  "columns not strictly increasing");
      HLU_REQUIRE(std::isfinite(A->val[p]), HLU_ERR_INVALID_ARG, "non-finite value");
    }
  }
}

// Where a handle's factor lives for options o: its bound workspace, or the
// batch workspace it belongs to.
void resolve_memory(hlu_s* h, const hlu_factor_opts* o) {
  if (h->batch) {
    HLU_REQUIRE(h->arena && h->prec == o->prec && h->pb->kcap == kcap_for(o), HLU_ERR_STATE,
                "hlu_factor: handle is bound through a batch with other options");
    h->peak = nullptr;
    return;
  }
  const WorkLayout L = work_layout(h->pb->ps, o->prec);
  HLU_REQUIRE(h->work != nullptr, HLU_ERR_STATE, "hlu_factor: no workspace bound");
  HLU_REQUIRE(h->work_bytes >= L.total, HLU_ERR_OUT_OF_MEMORY, "hlu_factor: bound workspace too small");
  h->arena = h->work;
  h->dims = reinterpret_cast<int32_t*>(static_cast<char*>(h->work) + L.dims_off);
  h->status = reinterpret_cast<int32_t*>(static_cast<char*>(h->work) + L.status_off);
  h->peak = reinterpret_cast<int32_t*>(static_cast<char*>(h->work) + L.peak_off);
}

}  // namespace

void use_bundle(hlu_s* h, int32_t kcap) {
  if (h->pb && h->pb->kcap == kcap) return;
  HLU_REQUIRE(!h->batch, HLU_ERR_STATE, "handle is bound through a batch with another rank capacity");
  h->pb = (h->fitted && h->fitted->kcap == kcap) ? h->fitted : get_bundle(*h->sh, kcap);
  h->peak_valid = false;
  h->sbuf.reset();   // solve buffers follow the schedule
  h->factored = false;
}

}  // namespace hlu

using namespace hlu;

hlu_s::~hlu_s() {
  for (hipEvent_t e : tev) (void)hipEventDestroy(e);
}

// =================================================================== C ABI
extern "C" {

const char* hlu_last_error(void) { return get_error(); }

hlu_status hlu_kuhn_domain_sizes(int32_t n, const uint8_t* mask, int32_t* N, int64_t* nnz) {
  return guard([&] {
    HLU_REQUIRE(n >= 1 && n <= 128 && N && nnz, HLU_ERR_INVALID_ARG, "hlu_kuhn_sizes: need 1 <= n <= 128");
    std::vector<int32_t> rp, ci, mid;
    std::vector<double> v;
    int32_t NN;
    kuhn_assemble(n, 1.0, &rp, &ci, &v, &mid, &NN, nullptr, 1.0, mask);
    *N = NN;
    *nnz = (int64_t)ci.size();
  });
}

hlu_status hlu_kuhn_sizes(int32_t n, int32_t* N, int64_t* nnz) { return hlu_kuhn_domain_sizes(n, nullptr, N, nnz); }

hlu_status hlu_kuhn_assemble_domain(int32_t n, double kappa, const uint8_t* mask, const int32_t* beta_box,
                                    double beta_in, int32_t* row_ptr, int32_t* col, double* val, int32_t* mid2) {
  return guard([&] {
    HLU_REQUIRE(n >= 1 && n <= 128 && row_ptr && col && val && mid2, HLU_ERR_INVALID_ARG,
                "hlu_kuhn_assemble: bad arguments");
    HLU_REQUIRE(std::isfinite(kappa), HLU_ERR_INVALID_ARG, "hlu_kuhn_assemble: kappa must be finite");
    HLU_REQUIRE(!beta_box || (std::isfinite(beta_in) && beta_in > 0.0), HLU_ERR_INVALID_ARG,
                "hlu_kuhn_assemble_beta: the coefficient must be finite and positive");
    std::vector<int32_t> rp, ci, mid;
    std::vector<double> v;
    int32_t NN;
    kuhn_assemble(n, kappa, &rp, &ci, &v, &mid, &NN, beta_box, beta_in, mask);
    HLU_REQUIRE(NN > 0, HLU_ERR_INVALID_ARG, "hlu_kuhn_assemble_domain: the domain has no interior edge");
    std::memcpy(row_ptr, rp.data(), rp.size() * sizeof(int32_t));
    std::memcpy(col, ci.data(), ci.size() * sizeof(int32_t));
    std::memcpy(val, v.data(), v.size() * sizeof(double));
    std::memcpy(mid2, mid.data(), mid.size() * sizeof(int32_t));
  });
}

hlu_status hlu_kuhn_assemble_beta(int32_t n, double kappa, const int32_t* beta_box, double beta_in, int32_t* row_ptr,
                                  int32_t* col, double* val, int32_t* mid2) {
  return hlu_kuhn_assemble_domain(n, kappa, nullptr, beta_box, beta_in, row_ptr, col, val, mid2);
}

hlu_status hlu_kuhn_assemble(int32_t n, double kappa, int32_t* row_ptr, int32_t* col, double* val, int32_t* mid2) {
  return hlu_kuhn_assemble_domain(n, kappa, nullptr, nullptr, 1.0, row_ptr, col, val, mid2);
}

hlu_status hlu_kuhn_domain_support_boxes(int32_t n, const uint8_t* mask, int32_t* lo2, int32_t* hi2) {
  return guard([&] {
    HLU_REQUIRE(n >= 1 && n <= 128 && lo2 && hi2, HLU_ERR_INVALID_ARG, "hlu_kuhn_support_boxes: bad arguments");
    std::vector<int32_t> l, h;
    kuhn_support_boxes(n, &l, &h, mask);
    HLU_REQUIRE(!l.empty(), HLU_ERR_INVALID_ARG, "hlu_kuhn_support_boxes: the domain has no interior edge");
    std::memcpy(lo2, l.data(), l.size() * sizeof(int32_t));
    std::memcpy(hi2, h.data(), h.size() * sizeof(int32_t));
  });
}

hlu_status hlu_kuhn_support_boxes(int32_t n, int32_t* lo2, int32_t* hi2) {
  return hlu_kuhn_domain_support_boxes(n, nullptr, lo2, hi2);
}

hlu_status hlu_kuhn_load_domain(int32_t n, const uint8_t* mask, const double* J, double* b) {
  return guard([&] {
    HLU_REQUIRE(n >= 1 && n <= 128 && J && b, HLU_ERR_INVALID_ARG, "hlu_kuhn_load: bad arguments");
    HLU_REQUIRE(std::isfinite(J[0]) && std::isfinite(J[1]) && std::isfinite(J[2]), HLU_ERR_INVALID_ARG,
                "hlu_kuhn_load: J must be finite");
    std::vector<double> v;
    kuhn_load(n, J, &v, mask);
    HLU_REQUIRE(!v.empty(), HLU_ERR_INVALID_ARG, "hlu_kuhn_load: the domain has no interior edge");
    std::memcpy(b, v.data(), v.size() * sizeof(double));
  });
}

hlu_status hlu_kuhn_load(int32_t n, const double* J, double* b) { return hlu_kuhn_load_domain(n, nullptr, J, b); }

hlu_status hlu_spmat_create(int32_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col,
                            const double* d_val, hlu_spmat* out) {
  return guard([&] {
    HLU_REQUIRE(out && n > 0 && nnz >= 0 && d_row_ptr && (nnz == 0 || (d_col && d_val)), HLU_ERR_INVALID_ARG,
                "hlu_spmat_create: bad arguments");
    auto* A = new hlu_spmat_s{n, nnz, d_row_ptr, d_col, d_val};
    *out = A;
  });
}

void hlu_spmat_destroy(hlu_spmat A) { delete A; }

hlu_status hlu_spmv(hlu_spmat A, const double* d_x, double* d_y, int32_t nrhs, int64_t ld, double alpha, double beta,
                    void* stream) {
  return guard([&] {
    HLU_REQUIRE(A && d_x && d_y && nrhs >= 1 && ld >= A->n, HLU_ERR_INVALID_ARG, "hlu_spmv: bad arguments");
    HIP_OK(spmv_launch(A->n, A->rp, A->ci, A->val, d_x, d_y, nrhs, ld, alpha, beta, (hipStream_t)stream));
  });
}

hlu_status hlu_build_boxes(const hlu_csr* A, const int32_t* mid2, const int32_t* box_lo2, const int32_t* box_hi2,
                           double eta, int32_t leaf_size, hlu_handle* out) {
  return guard([&] {
    HLU_REQUIRE(A && mid2 && out, HLU_ERR_INVALID_ARG, "hlu_build: NULL argument");
    HLU_REQUIRE((box_lo2 == nullptr) == (box_hi2 == nullptr), HLU_ERR_INVALID_ARG,
                "hlu_build_boxes: give both box corners or neither");
    HLU_REQUIRE(leaf_size >= 1 && leaf_size <= 128 && eta > 0 && std::isfinite(eta), HLU_ERR_INVALID_ARG,
                "hlu_build: need 1 <= leaf_size <= 128, eta > 0");
    check_csr(A);
    const int32_t n = A->n;
    if (box_lo2)
      for (int64_t e = 0; e < 3 * (int64_t)n; ++e)
        HLU_REQUIRE(box_lo2[e] <= mid2[e] && mid2[e] <= box_hi2[e], HLU_ERR_INVALID_ARG,
                    "hlu_build_boxes: a box does not contain its index's midpoint");
    auto sh = std::make_shared<Shared>();
    sh->S.build(mid2, n, leaf_size, eta, box_lo2, box_hi2);
    sh->row_ptr.assign(A->row_ptr, A->row_ptr + n + 1);
    sh->col.assign(A->col, A->col + A->nnz);
    for (int32_t c : sh->S.leaf_clusters) sh->max_leaf = std::max(sh->max_leaf, sh->S.clusters[c].size());
    // admissible blocks holding entries
    const Structure& S = sh->S;
    std::vector<int32_t> iperm(n);
    for (int32_t i = 0; i < n; ++i) iperm[S.perm[i]] = i;
    std::vector<char> nz(S.leaves.size(), 0);
    for (int32_t r = 0; r < n; ++r) {
      const int32_t i = iperm[r];
      for (int32_t p = sh->row_ptr[r]; p < sh->row_ptr[r + 1]; ++p) {
        const int32_t j = iperm[sh->col[p]];
        int32_t node = 0;
        while (S.blocks[node].kind == kSub) {
          const BlockNode& b = S.blocks[node];
          const int32_t qi = i < S.clusters[S.clusters[b.row].son[0]].end ? 0 : 1;
          const int32_t qj = j < S.clusters[S.clusters[b.col].son[0]].end ? 0 : 1;
          node = b.son[2 * qi + qj];
        }
        if (S.blocks[node].kind == kLowRank) nz[S.blocks[node].leaf_id] = 1;
      }
    }
    for (size_t l = 0; l < nz.size(); ++l)
      if (nz[l]) sh->nonzero_admissible.push_back((int32_t)l);
    auto h = std::make_unique<hlu_s>();
    h->sh = std::move(sh);
    h->val.assign(A->val, A->val + A->nnz);
    fill_structure_stats(h.get());
    *out = h.release();
  });
}

hlu_status hlu_build(const hlu_csr* A, const int32_t* mid2, double eta, int32_t leaf_size, hlu_handle* out) {
  return hlu_build_boxes(A, mid2, nullptr, nullptr, eta, leaf_size, out);
}

hlu_status hlu_build_shared(hlu_handle proto, const hlu_csr* A, hlu_handle* out) {
  return guard([&] {
    HLU_REQUIRE(proto && A && out, HLU_ERR_INVALID_ARG, "hlu_build_shared: NULL argument");
    check_csr(A);
    const Shared& sh = *proto->sh;
    HLU_REQUIRE(A->n == sh.S.N && (size_t)A->nnz == sh.col.size(), HLU_ERR_INVALID_ARG,
                "hlu_build_shared: size differs from the prototype's");
    HLU_REQUIRE(std::equal(sh.row_ptr.begin(), sh.row_ptr.end(), A->row_ptr) &&
                    std::equal(sh.col.begin(), sh.col.end(), A->col),
                HLU_ERR_INVALID_ARG, "hlu_build_shared: sparsity pattern differs from the prototype's");
    auto h = std::make_unique<hlu_s>();
    h->sh = proto->sh;
    h->val.assign(A->val, A->val + A->nnz);
    fill_structure_stats(h.get());
    *out = h.release();
  });
}

void hlu_destroy(hlu_handle h) {
  if (h && h->batch) batch_forget(h->batch, h);
  delete h;
}

hlu_status hlu_workspace_bytes(hlu_handle h, const hlu_factor_opts* o, size_t* bytes) {
  return guard([&] {
    HLU_REQUIRE(h && bytes, HLU_ERR_INVALID_ARG, "hlu_workspace_bytes: NULL argument");
    check_opts(o);
    use_bundle(h, kcap_for(o));
    *bytes = work_layout(h->pb->ps, o->prec).total;
    h->stats.workspace_bytes = (int64_t)*bytes;
    h->stats.rank_capacity_entries = rank_capacity_entries(h->sh->S, h->pb->ps.store);
    h->stats.factor_waves = (int64_t)h->pb->ps.factor.waves.size();
    h->stats.factor_tasks = h->pb->ps.factor.num_tasks;
    h->stats.solve_waves = (int64_t)h->pb->ps.fwd_bwd.waves.size();
  });
}

hlu_status hlu_solve_workspace_bytes(hlu_handle h, const hlu_factor_opts* o, size_t* bytes) {
  return guard([&] {
    HLU_REQUIRE(h && bytes, HLU_ERR_INVALID_ARG, "hlu_solve_workspace_bytes: NULL argument");
    check_opts(o);
    use_bundle(h, kcap_for(o));
    *bytes = solve_buffer_bytes(h->pb->sc, h->sh->S.N, kMaxRhs);
  });
}

hlu_status hlu_bind_solve_workspace(hlu_handle h, void* d_work, size_t bytes) {
  return guard([&] {
    HLU_REQUIRE(h, HLU_ERR_INVALID_ARG, "hlu_bind_solve_workspace: NULL handle");
    HLU_REQUIRE(!h->batch, HLU_ERR_STATE, "hlu_bind_solve_workspace: handle is bound through a batch");
    HLU_REQUIRE((d_work == nullptr) == (bytes == 0), HLU_ERR_INVALID_ARG,
                "hlu_bind_solve_workspace: pointer and size must both be given or both be zero");
    HLU_REQUIRE(((uintptr_t)d_work & 255) == 0, HLU_ERR_INVALID_ARG,
                "hlu_bind_solve_workspace: the workspace must be 256-byte aligned");
    h->solve_work = d_work;
    h->solve_work_bytes = bytes;
    h->sbuf.reset();   // made again, in the new memory, by the next solve
    h->inv_ready = false;
  });
}

hlu_status hlu_plan_device_bytes(hlu_handle h, const hlu_factor_opts* o, size_t* bytes) {
  return guard([&] {
    HLU_REQUIRE(h && bytes, HLU_ERR_INVALID_ARG, "hlu_plan_device_bytes: NULL argument");
    check_opts(o);
    use_bundle(h, kcap_for(o));
    *bytes = bundle_device_bytes(*h->sh, *h->pb);
  });
}

hlu_status hlu_device_bytes(hlu_handle h, const hlu_factor_opts* o, size_t* bytes) {
  return guard([&] {
    HLU_REQUIRE(h && bytes, HLU_ERR_INVALID_ARG, "hlu_device_bytes: NULL argument");
    check_opts(o);
    use_bundle(h, kcap_for(o));
    const size_t ws = work_layout(h->pb->ps, o->prec).total;
    *bytes = ws + solve_buffer_bytes(h->pb->sc, h->sh->S.N, kMaxRhs) + h->val.size() * sizeof(double) +
             bundle_device_bytes(*h->sh, *h->pb);   // a bound solve workspace counts as the solve buffers
  });
}

hlu_status hlu_fit_ranks(hlu_handle h, const hlu_factor_opts* o, int32_t margin, size_t* workspace_bytes) {
  return guard([&] {
    HLU_REQUIRE(h && workspace_bytes, HLU_ERR_INVALID_ARG, "hlu_fit_ranks: NULL argument");
    check_opts(o);
    HLU_REQUIRE(margin <= 4096, HLU_ERR_INVALID_ARG, "hlu_fit_ranks: margin too large");
    HLU_REQUIRE(!h->batch, HLU_ERR_STATE, "hlu_fit_ranks: handle belongs to a batch");
    const int32_t kcap = kcap_for(o);
    if (margin < 0) {   // back to the uniform capacity
      h->fitted.reset();
      h->pb.reset();
      use_bundle(h, kcap);
    } else {
      HLU_REQUIRE(h->peak_valid && h->mode == 0 && h->peak, HLU_ERR_STATE,
                  "hlu_fit_ranks: needs an hlu_factor of this handle with its own workspace first");
      // rank slots of blocks and temporaries come first and depend on the
      // structure only, so they match between capacities
      const int32_t nslot = h->pb->ps.store.nrhs_slot;
      std::vector<int32_t> peak((size_t)nslot);
      HIP_OK(hipMemcpy(peak.data(), h->peak, peak.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
      auto pb = std::make_shared<PlanBundle>();
      pb->kcap = kcap;
      pb->slot_cap.resize((size_t)nslot);
      for (int32_t i = 0; i < nslot; ++i) pb->slot_cap[i] = std::max(1, peak[i] + margin);
      build_plans(h->sh->S, kcap, kMaxRhs, h->sh->nonzero_admissible, &pb->ps, &pb->slot_cap);
      build_chain_sched(h->sh->S, pb->ps.store, &pb->sc);
      h->fitted = pb;
      h->pb = pb;
    }
    h->sbuf.reset();
    h->inv_ready = false;
    h->factored = false;
    h->peak_valid = false;
    *workspace_bytes = work_layout(h->pb->ps, o->prec).total;
    h->stats.workspace_bytes = (int64_t)*workspace_bytes;
    h->stats.rank_capacity_entries = rank_capacity_entries(h->sh->S, h->pb->ps.store);
  });
}

hlu_status hlu_bind_workspace(hlu_handle h, void* d_work, size_t bytes) {
  return guard([&] {
    HLU_REQUIRE(h && d_work, HLU_ERR_INVALID_ARG, "hlu_bind_workspace: NULL argument");
    HLU_REQUIRE(!h->batch, HLU_ERR_STATE, "hlu_bind_workspace: handle belongs to a batch");
    HLU_REQUIRE(((uintptr_t)d_work & 255) == 0, HLU_ERR_INVALID_ARG, "hlu_bind_workspace: need 256-byte alignment");
    h->work = d_work;
    h->work_bytes = bytes;
    h->factored = false;
  });
}

hlu_status hlu_factor(hlu_handle h, const hlu_factor_opts* o, void* stream) {
  hlu_status overflow = HLU_OK;
  hlu_status st = guard([&] {
    HLU_REQUIRE(h, HLU_ERR_INVALID_ARG, "hlu_factor: NULL handle");
    check_opts(o);
    use_bundle(h, kcap_for(o));
    resolve_memory(h, o);
    ensure_device(*h->sh, *h->pb);
    hipStream_t s = (hipStream_t)stream;
    h->factored = false;
    h->mode = 0;
    record_factor(h, o);
    if (fp32_storage(o->prec)) factor_impl<float>(h, s);
    else factor_impl<double>(h, s);
    HIP_OK(hipStreamSynchronize(s));
    int32_t status[3];
    HIP_OK(hipMemcpy(status, h->status, sizeof(status), hipMemcpyDeviceToHost));
    HLU_REQUIRE(status[0] == 0, HLU_ERR_ZERO_PIVOT, "hlu_factor: zero pivot in a diagonal leaf");
    HLU_REQUIRE(status[2] == 0, HLU_ERR_DEVICE, "hlu_factor: a truncation exceeded its round bound");
    h->factored = true;
    gather_stats(h, h->sbuf->pivots);
    read_flops(h->status, &h->stats);
    h->stats.capped_blocks = status[1];
    h->peak_valid = h->peak != nullptr;
    dump_trunc_trace(h->pb->ps.factor);
    if (status[1] > 0 && o->max_rank == 0) {
      set_error("hlu_factor: a truncated rank exceeded the block capacity");
      overflow = HLU_ERR_RANK_OVERFLOW;
    }
  });
  return st != HLU_OK ? st : overflow;
}

hlu_status hlu_solve(hlu_handle h, const double* d_b, double* d_x, int32_t nrhs, int64_t ld, void* stream) {
  return guard([&] {
    HLU_REQUIRE(h && d_b && d_x && nrhs >= 1 && ld >= h->sh->S.N, HLU_ERR_INVALID_ARG, "hlu_solve: bad arguments");
    HLU_REQUIRE(h->factored, HLU_ERR_STATE, "hlu_solve: handle is not factored");
    hipStream_t s = (hipStream_t)stream;
    if (h->mode == 1) {   // the Schulz inverse: x = B_H b
      inverse_apply(h, d_b, d_x, nrhs, ld, s);
      return;
    }
    const char* e = getenv("HLU_DEBUG_WAVE_SOLVE");
    if (e && e[0] == '1') {   // the planned wave form of the same solve, for cross-checks
      if (fp32_storage(h->prec))
        solve_impl<float>(h, h->pb->ps.fwd_bwd, h->pb->dsolve, d_b, d_x, nrhs, ld, s);
      else
        solve_impl<double>(h, h->pb->ps.fwd_bwd, h->pb->dsolve, d_b, d_x, nrhs, ld, s);
    } else if (fp32_storage(h->prec)) {
      solve_persistent_impl<float>(h, d_b, d_x, nrhs, ld, s);
    } else {
      solve_persistent_impl<double>(h, d_b, d_x, nrhs, ld, s);
    }
  });
}

hlu_status hlu_sync_status(hlu_handle h, void* stream) {
  return guard([&] {
    HLU_REQUIRE(h, HLU_ERR_INVALID_ARG, "hlu_sync_status: NULL handle");
    hipStream_t s = (hipStream_t)stream;
    HIP_OK(hipStreamSynchronize(s));
    if (h->sbuf && take_solve_error(h->sbuf->ctr, s))
      fail(HLU_ERR_DEVICE, "hlu_sync_status: a persistent solve gave up waiting for its inputs; its results are invalid");
  });
}

hlu_status hlu_apply_lu(hlu_handle h, const double* d_v, double* d_y, int32_t nrhs, int64_t ld, void* stream) {
  return guard([&] {
    HLU_REQUIRE(h && d_v && d_y && nrhs >= 1 && ld >= h->sh->S.N && d_v != d_y, HLU_ERR_INVALID_ARG,
                "hlu_apply_lu: bad arguments");
    HLU_REQUIRE(h->factored && h->mode == 0, HLU_ERR_STATE, "hlu_apply_lu: handle holds no H-LU factors");
    hipStream_t s = (hipStream_t)stream;
    if (fp32_storage(h->prec))
      solve_impl<float>(h, h->pb->ps.apply, h->pb->dapply, d_v, d_y, nrhs, ld, s);
    else
      solve_impl<double>(h, h->pb->ps.apply, h->pb->dapply, d_v, d_y, nrhs, ld, s);
  });
}

// ------------------------------------------------------------ inspection
hlu_status hlu_structure_sizes(hlu_handle h, int32_t* N, int32_t* num_clusters, int32_t* num_blocks) {
  return guard([&] {
    HLU_REQUIRE(h, HLU_ERR_INVALID_ARG, "hlu_structure_sizes: NULL handle");
    const Structure& S = h->sh->S;
    if (N) *N = S.N;
    if (num_clusters) *num_clusters = (int32_t)S.clusters.size();
    if (num_blocks) *num_blocks = (int32_t)S.leaves.size();
  });
}

hlu_status hlu_export_structure(hlu_handle h, int32_t* perm, int32_t* begin, int32_t* end, int32_t* level,
                                int32_t* son0, int32_t* son1, int32_t* brow, int32_t* bcol, int32_t* bkind) {
  return guard([&] {
    HLU_REQUIRE(h, HLU_ERR_INVALID_ARG, "hlu_export_structure: NULL handle");
    const Structure& S = h->sh->S;
    if (perm) std::memcpy(perm, S.perm.data(), S.perm.size() * sizeof(int32_t));
    for (size_t c = 0; c < S.clusters.size(); ++c) {
      if (begin) begin[c] = S.clusters[c].begin;
      if (end) end[c] = S.clusters[c].end;
      if (level) level[c] = S.clusters[c].level;
      if (son0) son0[c] = S.clusters[c].son[0];
      if (son1) son1[c] = S.clusters[c].son[1];
    }
    for (size_t l = 0; l < S.leaves.size(); ++l) {
      const BlockNode& b = S.blocks[S.leaves[l]];
      if (brow) brow[l] = b.row;
      if (bcol) bcol[l] = b.col;
      if (bkind) bkind[l] = (int32_t)b.kind;
    }
  });
}

hlu_status hlu_get_ranks(hlu_handle h, int32_t* ranks) {
  return guard([&] {
    HLU_REQUIRE(h && ranks, HLU_ERR_INVALID_ARG, "hlu_get_ranks: NULL argument");
    HLU_REQUIRE(h->factored, HLU_ERR_STATE, "hlu_get_ranks: handle is not factored");
    const StoragePlan& st = h->pb->ps.store;
    std::vector<int32_t> dims(st.num_slots);
    HIP_OK(hipMemcpy(dims.data(), h->dims, dims.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    const Structure& S = h->sh->S;
    for (size_t l = 0; l < S.leaves.size(); ++l) ranks[l] = st.slot[l] >= 0 ? dims[st.slot[l]] : -1;
  });
}

hlu_status hlu_check_trunc_rounds(hlu_handle h, const hlu_factor_opts* o, int32_t forced_rank, int64_t* out) {
  return guard([&] {
    HLU_REQUIRE(h && out && forced_rank >= 0, HLU_ERR_INVALID_ARG, "hlu_check_trunc_rounds: bad arguments");
    check_opts(o);
    use_bundle(h, kcap_for(o));
    const Plan& pl = h->pb->ps.factor;
    // every rank of the plan (blocks and temporaries) forced to forced_rank
    const std::vector<int32_t> dims((size_t)std::max(1, h->pb->ps.store.num_slots), forced_rank);
    int64_t rounds = 0, max_rounds = 0, stalled = 0, unfinished = 0;
    for (const TruncOp& op : pl.trunc) {
      const int bound = trunc_max_rounds(op, pl.parts.data(), dims.data());
      int r = std::min(forced_rank, op.cap);
      TruncCursor cur{0, 0};
      int n = 0;
      while (true) {
        bool done = false;
        int absorbed = 0;
        const int K = trunc_round_columns(op, pl.parts.data(), dims.data(), r, kTruncCols, &cur, &done,
                                          [&](int, int p, int) { absorbed += p >= 0; });
        if (K == 0) break;
        ++n;
        stalled += absorbed == 0 && !done;
        // the truncation keeps at most K columns, its eps-rank forced_rank
        // and the round's limit
        r = std::min(std::min(forced_rank, K), trunc_rank_limit(op, done, kTruncCols));
        if (done) break;
        if (n >= bound) {
          ++unfinished;
          break;
        }
      }
      rounds += n;
      max_rounds = std::max<int64_t>(max_rounds, n);
    }
    out[0] = (int64_t)pl.trunc.size();
    out[1] = rounds;
    out[2] = max_rounds;
    out[3] = stalled;
    out[4] = unfinished;
  });
}

hlu_status hlu_get_stats(hlu_handle h, hlu_stats* out) {
  return guard([&] {
    HLU_REQUIRE(h && out, HLU_ERR_INVALID_ARG, "hlu_get_stats: NULL argument");
    harvest_timing(h);
    *out = h->stats;
  });
}

hlu_status hlu_set_timing(hlu_handle h, int32_t enable) {
  return guard([&] {
    HLU_REQUIRE(h, HLU_ERR_INVALID_ARG, "hlu_set_timing: NULL handle");
    harvest_timing(h);
    h->timing = enable != 0;
    h->stats.solve_launches = 0;
    h->stats.solve_columns = 0;
    h->stats.solve_kernel_ms = 0.0;
  });
}

}  // extern "C"
