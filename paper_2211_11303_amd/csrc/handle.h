// Internal state of libhlu behind the opaque handles of include/hlu.h, and
// the helpers shared by the C entry points (api.cpp), the batch driver
// (batch.cpp) and the GMRES driver (gmres.cpp).
//
// Ownership: everything that depends only on the sparsity pattern and the
// block tree (the tree itself, the task plans, the solve schedule, the
// scatter targets) lives in a Shared object that every handle built on the
// same pattern references, so equal meshes are planned once.  A handle owns
// its matrix values, its factor state and the buffers of its own solves; the
// factor itself lives in caller memory (a bound workspace, or a batch
// workspace).
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "plan.h"
#include "chain_sched.h"
#include "structure.h"
#include "waves.h"

namespace hlu {

constexpr int kDefaultCap = 64;             // rank capacity of a low-rank block
constexpr int kMaxRhs = 32;                 // columns per solve launch
constexpr int kDotBlocks = 256;             // blocks of the partial dot products
constexpr size_t kMaxTimedEvents = 4096;    // event pairs kept before they are harvested
// Gram-based truncation resolves singular values down to about
// sqrt(K u) sigma_1; smaller ones are treated as zero.
constexpr double kFloorRel = 1e-7;

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
// Factor storage in FP32 (HLU_FP32, HLU_FP32_ACC64) or FP64; dense factor
// tasks in FP64 arithmetic (HLU_FP64, HLU_FP32_ACC64) or FP32.
inline bool fp32_storage(int32_t prec) { return prec != HLU_FP64; }
inline bool fp64_tasks(int32_t prec) { return prec != HLU_FP32; }
inline size_t elem_size(int32_t prec) { return fp32_storage(prec) ? sizeof(float) : sizeof(double); }

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

// Device memory freed with the owner.
struct Owned {
  std::vector<void*> ptrs;
  template <class T>
  T* keep(T* p) {
    ptrs.push_back((void*)p);
    return p;
  }
  ~Owned() {
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
  }
};

// Device copy of a plan's task arrays.
struct DevArrays {
  Owned mem;
  DevPlan P{};
  void load(const Plan& pl) {
    P.getrf = mem.keep(upload(pl.getrf));
    P.tri = mem.keep(upload(pl.tri));
    P.gemm = mem.keep(upload(pl.gemm));
    P.terms = mem.keep(upload(pl.terms));
    P.trunc = mem.keep(upload(pl.trunc));
    P.parts = mem.keep(upload(pl.parts));
    P.fill = mem.keep(upload(pl.fill));
    P.tile_op = mem.keep(upload(pl.gemm_tile_op));
    P.tile_ij = mem.keep(upload(pl.gemm_tile_ij));
  }
};

// Read-only device copy of a persistent-solve schedule.
struct DevSched {
  Owned mem;
  const CLeaf* leaves = nullptr;
  const CTarget* tgt = nullptr;
  const GDense* gdense = nullptr;
  const GLow* glow = nullptr;
  const GInline* ginl = nullptr;
  const CGather* gathers = nullptr;
  const CTprod* tprod = nullptr;
  const int32_t* tg0 = nullptr;
  const int32_t* tg_list = nullptr;
  const CTask* tasks = nullptr;
  const int32_t* member_L = nullptr;
  const int32_t* member_pos0 = nullptr;
  void load(const ChainSched& sc) {
    leaves = mem.keep(upload(sc.leaves));
    tgt = mem.keep(upload(sc.tgt));
    gdense = mem.keep(upload(sc.gdense));
    glow = mem.keep(upload(sc.glow));
    ginl = mem.keep(upload(sc.ginl));
    gathers = mem.keep(upload(sc.gathers));
    tprod = mem.keep(upload(sc.tprod));
    tg0 = mem.keep(upload(sc.tg0));
    tg_list = mem.keep(upload(sc.tg_list));
    tasks = mem.keep(upload(sc.tasks));
    member_L = mem.keep(upload(sc.member_L));
    member_pos0 = mem.keep(upload(sc.member_pos0));
  }
};

// Chains of one persistent solve launch at most (a quarter of the grid:
// the rest of the workgroups run the helper tasks, and several persistent
// solves on concurrent streams still find helpers).
constexpr int kMaxChains = 64;

// Mutable buffers of persistent solves with a given schedule (columns per
// launch <= max_rhs).
struct SolveBufs {
  Owned mem;
  void* inv = nullptr;        // triangle inverses (sized for FP64)
  void* stack = nullptr;      // stacked operators of the chains (sized for FP64)
  double* pivots = nullptr;   // U_ii, cluster order
  double* y = nullptr;        // N x max_rhs
  double* tbuf = nullptr;     // T products
  double* fbuf = nullptr;     // gather records
  int32_t* flags = nullptr;   // T-product flags, then record flags
  int32_t* prog = nullptr;    // chain progress words
  int32_t* ctr = nullptr;
  int64_t* trace = nullptr;   // debug clocks of the chain (HLU_DEBUG_SOLVE_TRACE)
  void* kargs = nullptr;      // launch arguments of the persistent solve
  int64_t rstride = 0;
  int32_t max_rhs = 0;
  int32_t epoch = 0;
  void alloc(const ChainSched& sc, int32_t N, int32_t max_rhs);   // library-owned memory
  void place(const ChainSched& sc, int32_t N, int32_t max_rhs, void* base, size_t bytes);   // caller memory
};

// Words of a persistent solve's counter block (kernels_chain.hip: claim
// counter, unused, error of the launch, error since the host last read it,
// workgroups that have left).
constexpr int kSolveCtrWords = 8;
// Longest wait of a persistent-solve task before its launch gives up, in
// device wall-clock ticks: 20 s, or HLU_DEBUG_SOLVE_WAIT_US microseconds
// (the tests force the error path with a tiny limit).
int64_t solve_wait_ticks();
// Reads and clears the error word a persistent launch leaves in ctr[3]
// (synchronises the stream); true if some launch gave up a wait.
bool take_solve_error(int32_t* ctr, hipStream_t s);

// Device bytes SolveBufs::alloc takes for this schedule.
size_t solve_buffer_bytes(const ChainSched& sc, int32_t N, int32_t max_rhs);

// Kernel launch view of a schedule and its buffers.
ChainDev make_chain_dev(const ChainSched& sc, const DevSched& d, const SolveBufs& b);

// Plans of the Schulz inverse for one rank capacity and their device copies.
struct InverseBundle {
  InversePlanSet ip;
  DevArrays dstep[2], dapply[2], damul;
};

// Plans for one rank capacity, shared by the handles of one structure.
// Host part built by get_bundle; device copies made by ensure_device.
struct PlanBundle {
  int32_t kcap = 0;
  std::vector<int32_t> slot_cap;   // fitted capacities per rank slot (empty: uniform kcap)
  PlanSet ps;
  ChainSched sc;
  bool on_device = false;
  DevArrays dfactor, dsolve, dapply;
  DevSched dsc;
  Owned mem;
  int64_t* d_target = nullptr;   // arena element of every stored entry of A
  std::unique_ptr<InverseBundle> inv;   // built by get_inverse_bundle on first use
};

struct Shared {
  Structure S;
  std::vector<int32_t> row_ptr, col;        // sparsity pattern of A (natural order)
  std::vector<int32_t> nonzero_admissible;  // admissible leaves holding entries
  int32_t max_leaf = 0;
  Owned mem;
  int32_t* d_perm = nullptr;
  std::mutex mu;
  std::map<int32_t, std::shared_ptr<PlanBundle>> bundles;
};

// Device bytes of the plan arrays, schedule, scatter targets and
// permutation shared by every handle of the structure (one copy per rank
// capacity).
size_t bundle_device_bytes(const Shared& sh, const PlanBundle& pb);

// Plans for capacity kcap (host work, built on first use; thread-safe).
std::shared_ptr<PlanBundle> get_bundle(Shared& sh, int32_t kcap);
// Device copies of the bundle's plans and schedule, the scatter targets and
// the permutation (first call uploads; thread-safe).
void ensure_device(Shared& sh, PlanBundle& pb);

struct WorkLayout {
  size_t arena_bytes, dims_off, status_off, peak_off, total;
};
WorkLayout work_layout(const PlanSet& ps, int32_t prec);

int32_t kcap_for(const hlu_factor_opts* o);
void check_opts(const hlu_factor_opts* o);

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

// ------------------------------------------------------------ kernels
// launch_wave / run_waves: waves.h
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
hipError_t scatter_values_scaled_launch(int64_t nnz, const int64_t* target, int64_t shift, double scale,
                                        const double* val, T* arena, hipStream_t s);
// {||v - u||^2, ||v||^2} over n elements into the last two of
// diff_norm_scratch_doubles() doubles of scratch (deterministic order)
size_t diff_norm_scratch_doubles();
template <class T>
hipError_t diff_norm_launch(int64_t n, const T* v, const T* u, double* scratch, hipStream_t s);
template <class T>
hipError_t zero_launch(T* p, int64_t n, hipStream_t s);
template <class T>
hipError_t identity_launch(T* p, int32_t n, hipStream_t s);
hipError_t set_int_launch(int32_t* p, int32_t v, hipStream_t s);
hipError_t zero_int_launch(int32_t* p, int32_t n, hipStream_t s);
// segmented vector kernels of GMRES: nseg segments [off[c], off[c] + len[c])
// of every vector block
hipError_t seg_dot_launch(int32_t nseg, const int64_t* off, const int64_t* len, int32_t nv, const double* V,
                          int64_t vstride, const double* w, double* part, double* out, hipStream_t s);
hipError_t seg_orth_launch(int32_t nseg, const int64_t* off, const int64_t* len, int64_t max_len, int32_t nv,
                           const double* V, int64_t vstride, const double* h, double* w, hipStream_t s);
hipError_t seg_scale_launch(int32_t nseg, const int64_t* off, const int64_t* len, int64_t max_len,
                            const double* src, const double* scale, double* dst, hipStream_t s);
hipError_t seg_combine_launch(int32_t nseg, const int64_t* off, const int64_t* len, int64_t max_len, int32_t nz,
                              const double* Z, int64_t zstride, const double* y, double* x, hipStream_t s);
hipError_t sub_launch(int64_t n, const double* b, double* r, hipStream_t s);
hipError_t copy_cols_launch(int32_t N, int32_t nrhs, const double* src, int64_t lds, double* dst, int64_t ldd,
                            hipStream_t s);

}  // namespace hlu

struct hlu_batch_s;

struct hlu_spmat_s {
  int32_t n;
  int64_t nnz;
  const int32_t* rp;
  const int32_t* ci;
  const double* val;
};

struct hlu_s {
  std::shared_ptr<hlu::Shared> sh;
  std::shared_ptr<hlu::PlanBundle> pb;   // plans of the capacity last asked for
  std::shared_ptr<hlu::PlanBundle> fitted;   // plans with capacities fitted to measured ranks (hlu_fit_ranks)
  int32_t* peak = nullptr;               // per rank slot: largest eps-rank asked for by the last factorisation
  hlu::WaveStreams waves;                // second stream of the factorisation's waves
  bool peak_valid = false;
  std::vector<double> val;               // values of A (natural order, pattern of sh)
  hlu::Owned mem;
  double* d_val = nullptr;
  // workspace bound by hlu_bind_workspace
  void* work = nullptr;
  size_t work_bytes = 0;
  // persistent-solve buffers bound by hlu_bind_solve_workspace (null: library-owned)
  void* solve_work = nullptr;
  size_t solve_work_bytes = 0;
  hlu_batch_s* batch = nullptr;          // batch whose workspace holds this factor
  // where the current factor lives (set when it is computed)
  void* arena = nullptr;
  int32_t* dims = nullptr;
  int32_t* status = nullptr;
  // own persistent solves
  std::unique_ptr<hlu::SolveBufs> sbuf;
  bool inv_ready = false;                // sbuf->inv holds this factor's inverses
  // factor state (mode 0: H-LU factors; mode 1: Schulz inverse B_H, held in
  // H-matrix inv_mat of the inverse layout; `factored`: a preconditioner is
  // ready)
  int32_t mode = 0;
  int32_t inv_mat = 1;
  double* red = nullptr;                 // inverse mode: reduction scratch in the workspace
  int32_t symmetric = -1;                // values checked symmetric (1), not (0), unchecked (-1)
  bool factored = false;
  int32_t prec = HLU_FP64;
  double eps = 0.0;
  int32_t max_rank = 0;                  // options of the last factorisation
  bool factor_compute64 = false;
  hlu_stats stats{};
  // optional timing of the persistent solve launches
  bool timing = false;
  std::vector<hipEvent_t> tev;
  size_t tev_used = 0;
  ~hlu_s();
};

namespace hlu {
// Factor-state helpers used by api.cpp and batch.cpp.
void ensure_values(hlu_s* h);                       // d_val
void ensure_targets(Shared& sh, PlanBundle& pb);    // pb.d_target
void ensure_solve_bufs(hlu_s* h);                   // sbuf for pb's schedule
template <class T>
void factor_prepare(hlu_s* h, T* arena, int32_t* dims, hipStream_t s);   // A into the arena
void gather_stats(hlu_s* h, const double* d_pivots);
void read_flops(const int32_t* d_status, hlu_stats* st);
void use_bundle(hlu_s* h, int32_t kcap);
// y = B_H b with the Schulz inverse of the handle (hlu_solve in inverse mode)
void inverse_apply(hlu_s* h, const double* b, double* x, int32_t nrhs, int64_t ld, hipStream_t s);
void harvest_timing(hlu_s* h);
void record_factor(hlu_s* h, const hlu_factor_opts* o);
void batch_forget(hlu_batch_s* b, hlu_s* h);        // a member handle is destroyed
}  // namespace hlu
