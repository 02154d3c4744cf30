// C ABI of libhlu (include/hlu.h): handles, workspace binding, the factor
// and solve drivers that launch the planned waves, and the GMRES driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "common.h"
#include "plan.h"
#include "solve_sched.h"
#include "structure.h"

namespace hlu {

// ------------------------------------------------------------- errors
namespace {
thread_local std::string g_last_error;
}
void set_error(const std::string& msg) { g_last_error = msg; }
const char* get_error() { return g_last_error.c_str(); }

void kuhn_assemble(int n, double kappa, std::vector<int32_t>* row_ptr, std::vector<int32_t>* col,
                   std::vector<double>* val, std::vector<int32_t>* mid2, int32_t* N);

// kernels (kernels_hlu.hip / kernels_vec.hip)
template <class T>
hipError_t launch_wave(T* arena, const DevPlan& P, const Wave& w, int32_t* dims, int32_t* status, double eps,
                       double floor_rel, int32_t max_leaf, int32_t tile_base, bool compute64, hipStream_t s);
hipError_t spmv_launch(int32_t n, const int32_t* rp, const int32_t* ci, const double* val, const double* x,
                       double* y, int32_t nrhs, int64_t ld, double alpha, double beta, hipStream_t s);
template <class T>
hipError_t gather_launch(int32_t n, int32_t nrhs, const int32_t* perm, const double* src, int64_t lds, T* dst,
                         int64_t ldd, hipStream_t s);
template <class T>
hipError_t scatter_perm_launch(int32_t n, int32_t nrhs, const int32_t* perm, const T* src, int64_t lds,
                               double* dst, int64_t ldd, hipStream_t s);
template <class T>
hipError_t scatter_values_launch(int64_t nnz, const int64_t* target, const double* val, T* arena, hipStream_t s);
template <class T>
hipError_t zero_launch(T* p, int64_t n, hipStream_t s);
template <class T>
hipError_t identity_launch(T* p, int32_t n, hipStream_t s);
hipError_t set_int_launch(int32_t* p, int32_t v, hipStream_t s);
hipError_t zero_int_launch(int32_t* p, int32_t n, hipStream_t s);
hipError_t multidot_launch(int32_t N, int32_t nrhs, int32_t nv, const double* V, int64_t vstride, const double* w,
                           double* part, double* out, hipStream_t s);
hipError_t orth_update_launch(int32_t N, int32_t nrhs, int32_t nv, const double* V, int64_t vstride,
                              const double* h, double* w, hipStream_t s);
hipError_t scale_cols_launch(int32_t N, int32_t nrhs, const double* src, const double* scale, double* dst,
                             hipStream_t s);
hipError_t combine_launch(int32_t N, int32_t nrhs, int32_t nz, const double* Z, int64_t zstride, const double* y,
                          double* x, int64_t ldx, hipStream_t s);
hipError_t residual_launch(int32_t N, int32_t nrhs, const double* b, int64_t ldb, double* r, hipStream_t s);
hipError_t copy_cols_launch(int32_t N, int32_t nrhs, const double* src, int64_t lds, double* dst, int64_t ldd,
                            hipStream_t s);
namespace {

constexpr int kDefaultCap = 64;
constexpr int kMaxRhs = 32;
constexpr int kDotBlocks = 256;
constexpr size_t kMaxTimedEvents = 4096;   // event pairs kept before they are harvested
// Gram-based truncation resolves singular values down to about
// sqrt(K u) sigma_1; smaller ones are treated as zero.
constexpr double kFloorRel = 1e-7;

template <class F>
hlu_status guard(F&& f) {
  try {
    f();
    return HLU_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return HLU_ERR_OUT_OF_MEMORY;
  } catch (...) {
    set_error("unexpected internal error");
    return HLU_ERR_DEVICE;
  }
}

template <class T>
T* dmalloc(size_t n) {
  if (n == 0) return nullptr;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess) fail(HLU_ERR_OUT_OF_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
  return static_cast<T*>(p);
}

template <class T>
T* upload(const std::vector<T>& v) {
  T* p = dmalloc<T>(v.size());
  if (p) HIP_OK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return p;
}

struct DevArrays {
  std::vector<void*> owned;
  DevPlan P{};
  ~DevArrays() {
    for (void* p : owned)
      if (p) (void)hipFree(p);
  }
  template <class T>
  const T* up(const std::vector<T>& v) {
    T* p = upload(v);
    owned.push_back(p);
    return p;
  }
  void load(const Plan& pl) {
    P.getrf = up(pl.getrf);
    P.tri = up(pl.tri);
    P.gemm = up(pl.gemm);
    P.terms = up(pl.terms);
    P.trunc = up(pl.trunc);
    P.parts = up(pl.parts);
    P.fill = up(pl.fill);
    P.tile_op = up(pl.gemm_tile_op);
    P.tile_ij = up(pl.gemm_tile_ij);
  }
};

}  // namespace
}  // namespace hlu

using namespace hlu;

struct hlu_spmat_s {
  int32_t n;
  int64_t nnz;
  const int32_t* rp;
  const int32_t* ci;
  const double* val;
};

struct hlu_s {
  Structure S;
  std::vector<int32_t> row_ptr, col;
  std::vector<double> val;
  std::vector<int32_t> nonzero_admissible;
  int32_t max_leaf = 0;
  // plans for the current capacity
  std::unique_ptr<PlanSet> plans;
  int32_t plan_kcap = -1;
  std::unique_ptr<DevArrays> dfactor, dsolve, dapply;
  int32_t* d_perm = nullptr;
  int64_t* d_target = nullptr;   // arena element of every stored entry of A
  // persistent solve
  std::unique_ptr<SolveSched> ssched;
  std::vector<void*> sowned;
  SolveDev sdev{};
  int32_t solve_epoch = 0;
  double* d_val = nullptr;
  // workspace
  void* work = nullptr;
  size_t work_bytes = 0;
  // factor state
  bool factored = false;
  int32_t prec = HLU_FP64;
  double eps = 0.0;
  bool factor_compute64 = false;
  hlu_stats stats{};
  // optional timing of the persistent solve launches (event pairs in flight)
  bool timing = false;
  std::vector<hipEvent_t> tev;
  size_t tev_used = 0;
  ~hlu_s() {
    for (hipEvent_t e : tev) (void)hipEventDestroy(e);
    for (void* p : sowned)
      if (p) (void)hipFree(p);
    if (d_perm) (void)hipFree(d_perm);
    if (d_target) (void)hipFree(d_target);
    if (d_val) (void)hipFree(d_val);
  }
};

namespace {

size_t elem_size(int32_t prec) { return prec == HLU_FP32 ? sizeof(float) : sizeof(double); }

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct WorkLayout {
  size_t arena_bytes, dims_off, status_off, total;
};

WorkLayout work_layout(const PlanSet& ps, int32_t prec) {
  WorkLayout L;
  L.arena_bytes = align256((size_t)ps.store.total_elems * elem_size(prec));
  L.dims_off = L.arena_bytes;
  L.status_off = L.dims_off + align256((size_t)ps.store.num_slots * sizeof(int32_t));
  L.total = L.status_off + 256;
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
  HLU_REQUIRE(o->prec == HLU_FP32 || o->prec == HLU_FP64, HLU_ERR_INVALID_ARG, "prec must be HLU_FP32 or HLU_FP64");
}

void ensure_plans(hlu_s* h, int32_t kcap) {
  if (h->plans && h->plan_kcap == kcap) return;
  auto ps = std::make_unique<PlanSet>();
  build_plans(h->S, kcap, kMaxRhs, h->nonzero_admissible, ps.get());
  h->plans = std::move(ps);
  h->plan_kcap = kcap;
  h->dfactor.reset();
  h->dsolve.reset();
  h->dapply.reset();
  for (void* p : h->sowned)
    if (p) (void)hipFree(p);
  h->sowned.clear();
  h->ssched.reset();
  h->factored = false;
  // scatter targets depend on the storage layout
  if (h->d_target) {
    (void)hipFree(h->d_target);
    h->d_target = nullptr;
  }
}

void ensure_device(hlu_s* h) {
  const PlanSet& ps = *h->plans;
  if (!h->dfactor) {
    auto d = std::make_unique<DevArrays>();
    d->load(ps.factor);
    h->dfactor = std::move(d);
  }
  if (!h->dsolve) {
    auto d = std::make_unique<DevArrays>();
    d->load(ps.fwd_bwd);
    h->dsolve = std::move(d);
  }
  if (!h->dapply) {
    auto d = std::make_unique<DevArrays>();
    d->load(ps.apply);
    h->dapply = std::move(d);
  }
  if (!h->ssched) {
    auto sc = std::make_unique<SolveSched>();
    build_solve_sched(h->S, ps.store, sc.get());
    auto keep = [&](void* p) { h->sowned.push_back(p); return p; };
    SolveDev& d = h->sdev;
    d.tasks = static_cast<const STask*>(keep(upload(sc->tasks)));
    d.leaves = static_cast<const SLeaf*>(keep(upload(sc->leaves)));
    d.dense = static_cast<const SDense*>(keep(upload(sc->dense)));
    d.low = static_cast<const SLow*>(keep(upload(sc->low)));
    d.tprod = static_cast<const STprod*>(keep(upload(sc->tprod)));
    d.max_rhs = kMaxRhs;
    // sized for FP64; FP32 factors use the first half
    d.inv = keep(dmalloc<double>((size_t)std::max<int64_t>(1, sc->inv_elems)));
    d.pivots = static_cast<double*>(keep(dmalloc<double>((size_t)h->S.N)));
    d.y = static_cast<double*>(keep(dmalloc<double>((size_t)h->S.N * kMaxRhs)));
    d.tbuf = static_cast<double*>(keep(dmalloc<double>((size_t)std::max<int64_t>(1, sc->tbuf_per_rhs) * kMaxRhs)));
    const size_t nflags = 2 * (size_t)sc->L + sc->tprod.size() + sc->dense.size() + 1;
    int32_t* flags = static_cast<int32_t*>(keep(dmalloc<int32_t>(nflags)));
    HIP_OK(hipMemset(flags, 0, nflags * sizeof(int32_t)));
    d.leaf_flag = flags;
    d.tp_flag = flags + 2 * sc->L;
    d.pflag = flags + 2 * sc->L + sc->tprod.size();
    d.push0 = static_cast<const int32_t*>(keep(upload(sc->push0)));
    d.push_recs = static_cast<const int32_t*>(keep(upload(sc->push_recs)));
    d.pstride = (int64_t)sc->max_m * kMaxRhs;
    d.pbuf = static_cast<double*>(keep(dmalloc<double>(std::max<size_t>(1, sc->dense.size()) * (size_t)d.pstride)));
    d.ctr = static_cast<int32_t*>(keep(dmalloc<int32_t>(4)));
    HIP_OK(hipMemset(d.ctr, 0, 4 * sizeof(int32_t)));
    d.ntasks = (int32_t)sc->tasks.size();
    d.n_fwd = sc->n_fwd_tasks;
    d.trace = nullptr;
    if (const char* tr = getenv("HLU_DEBUG_SOLVE_TRACE")) {   // debug: per-task clocks
      (void)tr;
      d.trace = static_cast<int64_t*>(keep(dmalloc<int64_t>(8 * (size_t)d.ntasks)));
    }
    d.L = sc->L;
    d.max_m = sc->max_m;
    h->solve_epoch = 0;
    h->ssched = std::move(sc);
  }
  if (!h->d_perm) h->d_perm = upload(h->S.perm);
  if (!h->d_val) h->d_val = upload(h->val);
  if (!h->d_target) {
    // arena element of every stored entry (dense leaf or staging block)
    const Structure& S = h->S;
    const StoragePlan& st = ps.store;
    std::vector<int32_t> iperm(S.N);
    for (int32_t i = 0; i < S.N; ++i) iperm[S.perm[i]] = i;
    std::vector<int64_t> init_off(S.leaves.size(), -1);
    for (const InitBlock& ib : ps.init_blocks) init_off[ib.leaf] = ib.off;
    // leaf block containing (i, j): walk down the block tree
    std::vector<int64_t> target(h->col.size(), -1);
    for (int32_t r = 0; r < S.N; ++r) {
      const int32_t i = iperm[r];
      for (int32_t p = h->row_ptr[r]; p < h->row_ptr[r + 1]; ++p) {
        const int32_t j = iperm[h->col[p]];
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
    h->d_target = upload(target);
  }
}

template <class T>
void run_plan(hlu_s* h, const Plan& pl, const DevArrays& d, bool compute64, hipStream_t s) {
  const WorkLayout L = work_layout(*h->plans, h->prec);
  T* arena = static_cast<T*>(h->work);
  int32_t* dims = reinterpret_cast<int32_t*>(static_cast<char*>(h->work) + L.dims_off);
  int32_t* status = reinterpret_cast<int32_t*>(static_cast<char*>(h->work) + L.status_off);
  int32_t tile_base = 0;
  for (const Wave& w : pl.waves) {
    HIP_OK(launch_wave<T>(arena, d.P, w, dims, status, h->eps, kFloorRel, h->max_leaf, tile_base, compute64, s));
    tile_base += w.gemm_tiles;
  }
}

template <class T>
void factor_impl(hlu_s* h, hipStream_t s) {
  const PlanSet& ps = *h->plans;
  const StoragePlan& st = ps.store;
  const WorkLayout L = work_layout(ps, h->prec);
  T* arena = static_cast<T*>(h->work);
  int32_t* dims = reinterpret_cast<int32_t*>(static_cast<char*>(h->work) + L.dims_off);
  int32_t* status = reinterpret_cast<int32_t*>(static_cast<char*>(h->work) + L.status_off);
  HIP_OK(zero_launch<T>(arena, st.data_elems, s));
  HIP_OK(identity_launch<T>(arena + st.identity_off, st.identity_n, s));
  HIP_OK(scatter_values_launch<T>((int64_t)h->col.size(), h->d_target, h->d_val, arena, s));
  HIP_OK(zero_int_launch(dims, st.num_slots, s));
  HIP_OK(zero_int_launch(status, 64, s));
  run_plan<T>(h, ps.factor, *h->dfactor, h->factor_compute64, s);
  // the persistent solve applies the diagonal leaves through their inverses
  HIP_OK(diag_inverse_launch<T>(static_cast<const T*>(h->work), h->sdev, s));
}

template <class T>
void solve_impl(hlu_s* h, const Plan& pl, const DevArrays& d, const double* b, double* x, int32_t nrhs, int64_t ld,
                bool apply, hipStream_t s) {
  const PlanSet& ps = *h->plans;
  const StoragePlan& st = ps.store;
  const WorkLayout L = work_layout(ps, h->prec);
  T* arena = static_cast<T*>(h->work);
  int32_t* dims = reinterpret_cast<int32_t*>(static_cast<char*>(h->work) + L.dims_off);
  const int32_t N = h->S.N;
  for (int32_t c0 = 0; c0 < nrhs; c0 += st.max_rhs) {
    const int32_t nc = std::min(st.max_rhs, nrhs - c0);
    HIP_OK(gather_launch<T>(N, nc, h->d_perm, b + (int64_t)c0 * ld, ld, arena + st.vec_off, N, s));
    HIP_OK(set_int_launch(dims + st.nrhs_slot, nc, s));
    // the solves read FP32 factors but accumulate in FP64
    run_plan<T>(h, pl, d, true, s);
    (void)apply;
    HIP_OK(scatter_perm_launch<T>(N, nc, h->d_perm, arena + st.vec_off, N, x + (int64_t)c0 * ld, ld, s));
  }
}

template <class T>
hipError_t gather_y(hlu_s* h, const double* b, int64_t ld, int32_t nc, hipStream_t s) {
  return gather_launch<double>(h->S.N, nc, h->d_perm, b, ld, h->sdev.y, h->S.N, s);
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

// x = P^T U^{-1} L^{-1} P b with the persistent solve kernel (FP64 vectors).
template <class T>
void solve_persistent_impl(hlu_s* h, const double* b, double* x, int32_t nrhs, int64_t ld, hipStream_t s) {
  const WorkLayout L = work_layout(*h->plans, h->prec);
  const T* arena = static_cast<const T*>(h->work);
  const int32_t* dims = reinterpret_cast<const int32_t*>(static_cast<char*>(h->work) + L.dims_off);
  const int32_t N = h->S.N;
  const int grid = std::max(1, std::min<int>(h->sdev.ntasks, 256));   // one 112 KB-LDS workgroup per CU
  for (int32_t c0 = 0; c0 < nrhs; c0 += kMaxRhs) {
    const int32_t nc = std::min(kMaxRhs, nrhs - c0);
    HIP_OK(gather_y<T>(h, b + (int64_t)c0 * ld, ld, nc, s));
    h->solve_epoch = h->solve_epoch % 1000000000 + 1;
    if (h->timing) {
      if (h->tev_used + 2 > kMaxTimedEvents) harvest_timing(h);
      while (h->tev.size() < h->tev_used + 2) {
        hipEvent_t e;
        HIP_OK(hipEventCreate(&e));
        h->tev.push_back(e);
      }
      HIP_OK(hipEventRecord(h->tev[h->tev_used], s));
    }
    HIP_OK(solve_persistent_launch<T>(arena, dims, h->sdev, N, nc, h->solve_epoch, grid, s));
    if (h->timing) {
      HIP_OK(hipEventRecord(h->tev[h->tev_used + 1], s));
      h->tev_used += 2;
      h->stats.solve_columns += nc;
    }
    HIP_OK(scatter_perm_launch<double>(N, nc, h->d_perm, h->sdev.y, N, x + (int64_t)c0 * ld, ld, s));
    if (h->sdev.trace) {   // debug: dump task clocks and kinds
      HIP_OK(hipStreamSynchronize(s));
      const SolveSched& sc = *h->ssched;
      std::vector<int64_t> tr(8 * (size_t)h->sdev.ntasks);
      HIP_OK(hipMemcpy(tr.data(), h->sdev.trace, tr.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
      if (FILE* f = fopen(getenv("HLU_DEBUG_SOLVE_TRACE"), "wb")) {
        for (int32_t t = 0; t < h->sdev.ntasks; ++t) {
          fwrite(&sc.tasks[t], sizeof(STask), 1, f);   // kind, idx (int32 each)
          fwrite(tr.data() + 8 * t, 8 * sizeof(int64_t), 1, f);
        }
        fclose(f);
      }
    }
  }
}

void gather_stats(hlu_s* h) {
  const PlanSet& ps = *h->plans;
  const StoragePlan& st = ps.store;
  const WorkLayout L = work_layout(ps, h->prec);
  std::vector<int32_t> dims(st.num_slots);
  HIP_OK(hipMemcpy(dims.data(), static_cast<char*>(h->work) + L.dims_off, dims.size() * sizeof(int32_t),
                   hipMemcpyDeviceToHost));
  const Structure& S = h->S;
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
  HIP_OK(hipMemcpy(piv.data(), h->sdev.pivots, piv.size() * sizeof(double), hipMemcpyDeviceToHost));
  double lo = INFINITY, hi = 0.0;
  for (double p : piv) {
    lo = std::min(lo, std::fabs(p));
    hi = std::max(hi, std::fabs(p));
  }
  h->stats.min_abs_pivot = lo;
  h->stats.max_abs_pivot = hi;
}

void fill_structure_stats(hlu_s* h) {
  const Structure& S = h->S;
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

}  // namespace

// =================================================================== C ABI
extern "C" {

const char* hlu_last_error(void) { return get_error(); }

hlu_status hlu_kuhn_sizes(int32_t n, int32_t* N, int64_t* nnz) {
  return guard([&] {
    HLU_REQUIRE(n >= 1 && n <= 128 && N && nnz, HLU_ERR_INVALID_ARG, "hlu_kuhn_sizes: need 1 <= n <= 128");
    std::vector<int32_t> rp, ci, mid;
    std::vector<double> v;
    int32_t NN;
    kuhn_assemble(n, 0.0, &rp, &ci, &v, nullptr, &NN);
    *N = NN;
    *nnz = (int64_t)ci.size();
  });
}

hlu_status hlu_kuhn_assemble(int32_t n, double kappa, int32_t* row_ptr, int32_t* col, double* val, int32_t* mid2) {
  return guard([&] {
    HLU_REQUIRE(n >= 1 && n <= 128 && row_ptr && col && val && mid2, HLU_ERR_INVALID_ARG,
                "hlu_kuhn_assemble: bad arguments");
    HLU_REQUIRE(std::isfinite(kappa), HLU_ERR_INVALID_ARG, "hlu_kuhn_assemble: kappa must be finite");
    std::vector<int32_t> rp, ci, mid;
    std::vector<double> v;
    int32_t NN;
    kuhn_assemble(n, kappa, &rp, &ci, &v, &mid, &NN);
    std::memcpy(row_ptr, rp.data(), rp.size() * sizeof(int32_t));
    std::memcpy(col, ci.data(), ci.size() * sizeof(int32_t));
    std::memcpy(val, v.data(), v.size() * sizeof(double));
    std::memcpy(mid2, mid.data(), mid.size() * sizeof(int32_t));
  });
}

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

hlu_status hlu_build(const hlu_csr* A, const int32_t* mid2, double eta, int32_t leaf_size, hlu_handle* out) {
  return guard([&] {
    HLU_REQUIRE(A && mid2 && out && A->row_ptr && A->col && A->val, HLU_ERR_INVALID_ARG, "hlu_build: NULL argument");
    HLU_REQUIRE(A->n > 0 && A->nnz >= 0 && leaf_size >= 1 && leaf_size <= 128 && eta > 0 && std::isfinite(eta),
                HLU_ERR_INVALID_ARG, "hlu_build: need n > 0, 1 <= leaf_size <= 128, eta > 0");
    const int32_t n = A->n;
    HLU_REQUIRE(A->row_ptr[0] == 0 && A->row_ptr[n] == A->nnz, HLU_ERR_INVALID_ARG, "hlu_build: malformed row_ptr");
    for (int32_t r = 0; r < n; ++r) {
      HLU_REQUIRE(A->row_ptr[r + 1] >= A->row_ptr[r], HLU_ERR_INVALID_ARG, "hlu_build: row_ptr not monotone");
      for (int32_t p = A->row_ptr[r]; p < A->row_ptr[r + 1]; ++p) {
        HLU_REQUIRE(A->col[p] >= 0 && A->col[p] < n, HLU_ERR_INVALID_ARG, "hlu_build: column index out of range");
        HLU_REQUIRE(p == A->row_ptr[r] || A->col[p] > A->col[p - 1], HLU_ERR_INVALID_ARG,
                    "hlu_build: columns not strictly increasing");
        HLU_REQUIRE(std::isfinite(A->val[p]), HLU_ERR_INVALID_ARG, "hlu_build: non-finite value");
      }
    }
    auto h = std::make_unique<hlu_s>();
    h->S.build(mid2, n, leaf_size, eta);
    h->row_ptr.assign(A->row_ptr, A->row_ptr + n + 1);
    h->col.assign(A->col, A->col + A->nnz);
    h->val.assign(A->val, A->val + A->nnz);
    for (int32_t c : h->S.leaf_clusters) h->max_leaf = std::max(h->max_leaf, h->S.clusters[c].size());
    // admissible blocks holding entries
    const Structure& S = h->S;
    std::vector<int32_t> iperm(n);
    for (int32_t i = 0; i < n; ++i) iperm[S.perm[i]] = i;
    std::vector<char> nz(S.leaves.size(), 0);
    for (int32_t r = 0; r < n; ++r) {
      const int32_t i = iperm[r];
      for (int32_t p = h->row_ptr[r]; p < h->row_ptr[r + 1]; ++p) {
        const int32_t j = iperm[h->col[p]];
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
      if (nz[l]) h->nonzero_admissible.push_back((int32_t)l);
    fill_structure_stats(h.get());
    *out = h.release();
  });
}

void hlu_destroy(hlu_handle h) { delete h; }

hlu_status hlu_workspace_bytes(hlu_handle h, const hlu_factor_opts* o, size_t* bytes) {
  return guard([&] {
    HLU_REQUIRE(h && bytes, HLU_ERR_INVALID_ARG, "hlu_workspace_bytes: NULL argument");
    check_opts(o);
    ensure_plans(h, kcap_for(o));
    *bytes = work_layout(*h->plans, o->prec).total;
    h->stats.workspace_bytes = (int64_t)*bytes;
    h->stats.factor_waves = (int64_t)h->plans->factor.waves.size();
    h->stats.factor_tasks = h->plans->factor.num_tasks;
    h->stats.solve_waves = (int64_t)h->plans->fwd_bwd.waves.size();
  });
}

hlu_status hlu_bind_workspace(hlu_handle h, void* d_work, size_t bytes) {
  return guard([&] {
    HLU_REQUIRE(h && d_work, HLU_ERR_INVALID_ARG, "hlu_bind_workspace: NULL argument");
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
    ensure_plans(h, kcap_for(o));
    const WorkLayout L = work_layout(*h->plans, o->prec);
    HLU_REQUIRE(h->work != nullptr, HLU_ERR_STATE, "hlu_factor: no workspace bound");
    HLU_REQUIRE(h->work_bytes >= L.total, HLU_ERR_OUT_OF_MEMORY, "hlu_factor: bound workspace too small");
    ensure_device(h);
    hipStream_t s = (hipStream_t)stream;
    h->factored = false;
    h->prec = o->prec;
    h->eps = o->eps;
    h->factor_compute64 = (o->prec == HLU_FP64);
    if (o->prec == HLU_FP32) factor_impl<float>(h, s);
    else factor_impl<double>(h, s);
    HIP_OK(hipStreamSynchronize(s));
    int32_t status[2];
    HIP_OK(hipMemcpy(status, static_cast<char*>(h->work) + L.status_off, sizeof(status), hipMemcpyDeviceToHost));
    HLU_REQUIRE(status[0] == 0, HLU_ERR_ZERO_PIVOT, "hlu_factor: zero pivot in a diagonal leaf");
    h->factored = true;
    gather_stats(h);
    h->stats.capped_blocks = status[1];
    if (status[1] > 0 && o->max_rank == 0) {
      set_error("hlu_factor: a truncated rank exceeded the block capacity");
      overflow = HLU_ERR_RANK_OVERFLOW;
    }
  });
  return st != HLU_OK ? st : overflow;
}

hlu_status hlu_solve(hlu_handle h, const double* d_b, double* d_x, int32_t nrhs, int64_t ld, void* stream) {
  return guard([&] {
    HLU_REQUIRE(h && d_b && d_x && nrhs >= 1 && ld >= h->S.N, HLU_ERR_INVALID_ARG, "hlu_solve: bad arguments");
    HLU_REQUIRE(h->factored, HLU_ERR_STATE, "hlu_solve: handle is not factored");
    hipStream_t s = (hipStream_t)stream;
    const char* e = getenv("HLU_DEBUG_WAVE_SOLVE");
    if (e && e[0] == '1') {   // the planned wave form of the same solve, for cross-checks
      if (h->prec == HLU_FP32)
        solve_impl<float>(h, h->plans->fwd_bwd, *h->dsolve, d_b, d_x, nrhs, ld, false, s);
      else
        solve_impl<double>(h, h->plans->fwd_bwd, *h->dsolve, d_b, d_x, nrhs, ld, false, s);
    } else if (h->prec == HLU_FP32) {
      solve_persistent_impl<float>(h, d_b, d_x, nrhs, ld, s);
    } else {
      solve_persistent_impl<double>(h, d_b, d_x, nrhs, ld, s);
    }
  });
}

hlu_status hlu_apply_lu(hlu_handle h, const double* d_v, double* d_y, int32_t nrhs, int64_t ld, void* stream) {
  return guard([&] {
    HLU_REQUIRE(h && d_v && d_y && nrhs >= 1 && ld >= h->S.N && d_v != d_y, HLU_ERR_INVALID_ARG,
                "hlu_apply_lu: bad arguments");
    HLU_REQUIRE(h->factored, HLU_ERR_STATE, "hlu_apply_lu: handle is not factored");
    hipStream_t s = (hipStream_t)stream;
    if (h->prec == HLU_FP32)
      solve_impl<float>(h, h->plans->apply, *h->dapply, d_v, d_y, nrhs, ld, true, s);
    else
      solve_impl<double>(h, h->plans->apply, *h->dapply, d_v, d_y, nrhs, ld, true, s);
  });
}

// ------------------------------------------------------------------ GMRES
size_t gmres_workspace_bytes(int32_t n, int32_t nrhs, int32_t restart) {
  if (n <= 0 || nrhs <= 0 || restart <= 0) return 0;
  const size_t blk = align256((size_t)n * nrhs * sizeof(double));
  size_t b = 0;
  b += blk * (size_t)(restart + 1);   // V
  b += blk * (size_t)restart;         // Z
  b += blk;                           // w
  b += align256((size_t)kDotBlocks * (restart + 1) * nrhs * sizeof(double));  // partial dots
  b += align256((size_t)(restart + 1) * nrhs * sizeof(double)) * 3;           // h, h2, y / scale
  return b;
}

hlu_status gmres_solve(hlu_spmat A, const double* d_b, double* d_x, int32_t nrhs, int64_t ld, hlu_handle precond,
                       const hlu_gmres_opts* o, hlu_gmres_info* info, void* d_work, size_t work_bytes,
                       void* stream) {
  bool all_conv = true;
  hlu_status st = guard([&] {
    HLU_REQUIRE(A && d_b && d_x && o && info && d_work && nrhs >= 1 && ld >= A->n, HLU_ERR_INVALID_ARG,
                "gmres_solve: bad arguments");
    HLU_REQUIRE(o->restart >= 1 && o->max_iters >= 1 && o->tol > 0.0, HLU_ERR_INVALID_ARG,
                "gmres_solve: need restart >= 1, max_iters >= 1, tol > 0");
    HLU_REQUIRE(d_b != d_x, HLU_ERR_INVALID_ARG, "gmres_solve: x must not alias b");
    if (precond) {
      HLU_REQUIRE(precond->factored, HLU_ERR_STATE, "gmres_solve: preconditioner not factored");
      HLU_REQUIRE(precond->S.N == A->n, HLU_ERR_INVALID_ARG, "gmres_solve: size mismatch");
    }
    const int32_t N = A->n, m = o->restart;
    HLU_REQUIRE(work_bytes >= gmres_workspace_bytes(N, nrhs, m), HLU_ERR_OUT_OF_MEMORY,
                "gmres_solve: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    char* wp = static_cast<char*>(d_work);
    const size_t blk = align256((size_t)N * nrhs * sizeof(double));
    const int64_t vstride = (int64_t)(blk / sizeof(double));
    double* V = reinterpret_cast<double*>(wp);
    wp += blk * (m + 1);
    double* Z = reinterpret_cast<double*>(wp);
    wp += blk * m;
    double* w = reinterpret_cast<double*>(wp);
    wp += blk;
    double* part = reinterpret_cast<double*>(wp);
    wp += align256((size_t)kDotBlocks * (m + 1) * nrhs * sizeof(double));
    double* dh = reinterpret_cast<double*>(wp);
    wp += align256((size_t)(m + 1) * nrhs * sizeof(double));
    double* dh2 = reinterpret_cast<double*>(wp);
    wp += align256((size_t)(m + 1) * nrhs * sizeof(double));
    double* dy = reinterpret_cast<double*>(wp);

    auto norms = [&](const double* vec, std::vector<double>* out) {
      HIP_OK(multidot_launch(N, nrhs, 1, vec, vstride, vec, part, dh, s));
      std::vector<double> t(nrhs);
      HIP_OK(hipMemcpyAsync(t.data(), dh, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_OK(hipStreamSynchronize(s));
      out->resize(nrhs);
      for (int c = 0; c < nrhs; ++c) (*out)[c] = std::sqrt(std::max(0.0, t[c]));
    };
    // x = 0; residual r = b (in V_0 before scaling)
    HIP_OK(hipMemsetAsync(w, 0, blk, s));
    HIP_OK(copy_cols_launch(N, nrhs, w, N, d_x, ld, s));
    HIP_OK(copy_cols_launch(N, nrhs, d_b, ld, w, N, s));
    std::vector<double> bnorm, rnorm;
    norms(w, &bnorm);
    rnorm = bnorm;
    std::vector<int32_t> iters(nrhs, 0);
    std::vector<char> conv(nrhs, 0);
    for (int c = 0; c < nrhs; ++c)
      if (bnorm[c] == 0.0 || rnorm[c] <= o->tol * bnorm[c]) conv[c] = 1;
    std::vector<double> H((size_t)(m + 1) * m * nrhs), cs(m * nrhs), sn(m * nrhs), g((m + 1) * nrhs);
    std::vector<double> hcol((m + 1) * nrhs), hcol2((m + 1) * nrhs), scale(nrhs), yv((size_t)m * nrhs);
    auto Hc = [&](int i, int j, int c) -> double& { return H[((size_t)c * (m + 1) + i) * m + j]; };
    while (true) {
      bool any = false;
      for (int c = 0; c < nrhs; ++c)
        if (!conv[c] && iters[c] < o->max_iters) any = true;
      if (!any) break;
      // V_0 = r / ||r||  (r in w)
      for (int c = 0; c < nrhs; ++c) scale[c] = (rnorm[c] > 0.0) ? 1.0 / rnorm[c] : 0.0;
      HIP_OK(hipMemcpyAsync(dy, scale.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, s));
      HIP_OK(scale_cols_launch(N, nrhs, w, dy, V, s));
      std::vector<char> active(nrhs, 0);
      std::vector<int> jend(nrhs, 0);
      for (int c = 0; c < nrhs; ++c) {
        active[c] = !conv[c] && iters[c] < o->max_iters;
        for (int i = 0; i <= m; ++i) g[c * (m + 1) + i] = 0.0;
        g[c * (m + 1)] = rnorm[c];
      }
      for (int j = 0; j < m; ++j) {
        bool act = false;
        for (int c = 0; c < nrhs; ++c) act = act || active[c];
        if (!act) break;
        double* Vj = V + (int64_t)j * vstride;
        double* Zj = Z + (int64_t)j * vstride;
        if (precond) {
          hlu_status ps = hlu_solve(precond, Vj, Zj, nrhs, N, s);
          if (ps != HLU_OK) fail(ps, std::string("gmres_solve: preconditioner: ") + get_error());
        } else {
          HIP_OK(copy_cols_launch(N, nrhs, Vj, N, Zj, N, s));
        }
        HIP_OK(spmv_launch(N, A->rp, A->ci, A->val, Zj, w, nrhs, N, 1.0, 0.0, s));
        // classical Gram-Schmidt, twice
        HIP_OK(multidot_launch(N, nrhs, j + 1, V, vstride, w, part, dh, s));
        HIP_OK(orth_update_launch(N, nrhs, j + 1, V, vstride, dh, w, s));
        HIP_OK(multidot_launch(N, nrhs, j + 1, V, vstride, w, part, dh2, s));
        HIP_OK(orth_update_launch(N, nrhs, j + 1, V, vstride, dh2, w, s));
        HIP_OK(hipMemcpyAsync(hcol.data(), dh, (size_t)(j + 1) * nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_OK(hipMemcpyAsync(hcol2.data(), dh2, (size_t)(j + 1) * nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
        std::vector<double> wn;
        norms(w, &wn);
        for (int c = 0; c < nrhs; ++c) {
          scale[c] = 0.0;
          if (!active[c]) continue;
          for (int i = 0; i <= j; ++i) Hc(i, j, c) = hcol[i * nrhs + c] + hcol2[i * nrhs + c];
          Hc(j + 1, j, c) = wn[c];
          scale[c] = wn[c] > 0.0 ? 1.0 / wn[c] : 0.0;
          for (int i = 0; i < j; ++i) {
            const double t = cs[c * m + i] * Hc(i, j, c) + sn[c * m + i] * Hc(i + 1, j, c);
            Hc(i + 1, j, c) = -sn[c * m + i] * Hc(i, j, c) + cs[c * m + i] * Hc(i + 1, j, c);
            Hc(i, j, c) = t;
          }
          const double den = std::hypot(Hc(j, j, c), Hc(j + 1, j, c));
          cs[c * m + j] = den > 0.0 ? Hc(j, j, c) / den : 1.0;
          sn[c * m + j] = den > 0.0 ? Hc(j + 1, j, c) / den : 0.0;
          Hc(j, j, c) = den;
          Hc(j + 1, j, c) = 0.0;
          double* gc = &g[c * (m + 1)];
          gc[j + 1] = -sn[c * m + j] * gc[j];
          gc[j] = cs[c * m + j] * gc[j];
          iters[c]++;
          jend[c] = j + 1;
          if (std::fabs(gc[j + 1]) <= o->tol * bnorm[c] || iters[c] >= o->max_iters || den == 0.0) active[c] = 0;
        }
        HIP_OK(hipMemcpyAsync(dy, scale.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, s));
        HIP_OK(scale_cols_launch(N, nrhs, w, dy, V + (int64_t)(j + 1) * vstride, s));
      }
      // y = H^{-1} g per column, x += Z y
      int jmax = 0;
      for (int c = 0; c < nrhs; ++c) jmax = std::max(jmax, jend[c]);
      std::fill(yv.begin(), yv.end(), 0.0);
      for (int c = 0; c < nrhs; ++c) {
        const int je = jend[c];
        for (int i = je - 1; i >= 0; --i) {
          double t = g[c * (m + 1) + i];
          for (int k = i + 1; k < je; ++k) t -= Hc(i, k, c) * yv[(size_t)k * nrhs + c];
          yv[(size_t)i * nrhs + c] = Hc(i, i, c) != 0.0 ? t / Hc(i, i, c) : 0.0;
        }
      }
      if (jmax > 0) {
        HIP_OK(hipMemcpyAsync(dh, yv.data(), (size_t)jmax * nrhs * sizeof(double), hipMemcpyHostToDevice, s));
        HIP_OK(combine_launch(N, nrhs, jmax, Z, vstride, dh, d_x, ld, s));
      }
      // true residual
      HIP_OK(spmv_launch(N, A->rp, A->ci, A->val, d_x, w, nrhs, ld, 1.0, 0.0, s));
      HIP_OK(residual_launch(N, nrhs, d_b, ld, w, s));
      norms(w, &rnorm);
      for (int c = 0; c < nrhs; ++c)
        if (!conv[c] && rnorm[c] <= o->tol * bnorm[c]) conv[c] = 1;
      if (jmax == 0) break;
    }
    for (int c = 0; c < nrhs; ++c) {
      info[c].iters = iters[c];
      info[c].converged = conv[c];
      info[c].relres = bnorm[c] > 0.0 ? rnorm[c] / bnorm[c] : 0.0;
      info[c].abs_res = rnorm[c];
      if (!conv[c]) all_conv = false;
    }
  });
  if (st != HLU_OK) return st;
  if (!all_conv) {
    set_error("gmres_solve: not converged within max_iters");
    return HLU_ERR_NOT_CONVERGED;
  }
  return HLU_OK;
}

// ------------------------------------------------------------ inspection
hlu_status hlu_structure_sizes(hlu_handle h, int32_t* N, int32_t* num_clusters, int32_t* num_blocks) {
  return guard([&] {
    HLU_REQUIRE(h, HLU_ERR_INVALID_ARG, "hlu_structure_sizes: NULL handle");
    if (N) *N = h->S.N;
    if (num_clusters) *num_clusters = (int32_t)h->S.clusters.size();
    if (num_blocks) *num_blocks = (int32_t)h->S.leaves.size();
  });
}

hlu_status hlu_export_structure(hlu_handle h, int32_t* perm, int32_t* begin, int32_t* end, int32_t* level,
                                int32_t* son0, int32_t* son1, int32_t* brow, int32_t* bcol, int32_t* bkind) {
  return guard([&] {
    HLU_REQUIRE(h, HLU_ERR_INVALID_ARG, "hlu_export_structure: NULL handle");
    const Structure& S = h->S;
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
    const StoragePlan& st = h->plans->store;
    const WorkLayout L = work_layout(*h->plans, h->prec);
    std::vector<int32_t> dims(st.num_slots);
    HIP_OK(hipMemcpy(dims.data(), static_cast<char*>(h->work) + L.dims_off, dims.size() * sizeof(int32_t),
                     hipMemcpyDeviceToHost));
    for (size_t l = 0; l < h->S.leaves.size(); ++l) ranks[l] = st.slot[l] >= 0 ? dims[st.slot[l]] : -1;
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
