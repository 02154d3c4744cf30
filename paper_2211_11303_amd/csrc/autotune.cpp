// Leaf-size selection by measurement for the batched workload: for one
// Kuhn-cube mesh and wavenumber, every candidate leaf size gets its own
// cluster tree, block tree and plans (host), a factorisation and one GMRES
// solve (device); the candidate with the smallest device time wins.  The
// leaf size trades the length of the solve's leaf chain and the number of
// factor waves against the size of the dense leaf tasks, so the best value
// depends on the mesh and is measured rather than modelled.
#include <cmath>
#include <memory>
#include <vector>

#include "gmres.h"
#include "handle.h"
#include "mesh.h"

namespace hlu {
}

using namespace hlu;

namespace {

struct HandleGuard {
  hlu_handle h = nullptr;
  ~HandleGuard() {
    if (h) hlu_destroy(h);
  }
};
struct SpmatGuard {
  hlu_spmat A = nullptr;
  ~SpmatGuard() {
    if (A) hlu_spmat_destroy(A);
  }
};
struct EventGuard {
  hipEvent_t e = nullptr;
  ~EventGuard() {
    if (e) (void)hipEventDestroy(e);
  }
};

void ok(hlu_status st) {
  if (st != HLU_OK) fail(st, get_error());
}

}  // namespace

extern "C" hlu_status hlu_autotune_leaf(int32_t n, double kappa, double eta, const int32_t* leaves, int32_t count,
                                        const hlu_factor_opts* fo, const hlu_gmres_opts* go, int32_t nrhs,
                                        double* seconds, int32_t* best, void* stream) {
  return guard([&] {
    HLU_REQUIRE(n >= 1 && n <= 128 && std::isfinite(kappa) && eta > 0 && leaves && count >= 1 && count <= 16 &&
                    seconds && best && nrhs >= 1 && nrhs <= kMaxRhs,
                HLU_ERR_INVALID_ARG, "hlu_autotune_leaf: bad arguments");
    for (int32_t c = 0; c < count; ++c)
      HLU_REQUIRE(leaves[c] >= 1 && leaves[c] <= 128, HLU_ERR_INVALID_ARG, "hlu_autotune_leaf: leaf outside 1..128");
    check_opts(fo);
    check_gmres_opts(go);
    hipStream_t s = (hipStream_t)stream;
    std::vector<int32_t> rp, ci, mid;
    std::vector<double> val;
    int32_t N = 0;
    kuhn_assemble(n, kappa, &rp, &ci, &val, &mid, &N);
    const int64_t nnz = (int64_t)ci.size();
    Owned common;
    const int32_t* drp = common.keep(upload(rp));
    const int32_t* dci = common.keep(upload(ci));
    const double* dval = common.keep(upload(val));
    SpmatGuard A;
    ok(hlu_spmat_create(N, nnz, drp, dci, dval, &A.A));
    // right-hand sides b = A x with x = 1 in every column
    const double* dx = common.keep(upload(std::vector<double>((size_t)N * nrhs, 1.0)));
    double* db = common.keep(dmalloc<double>((size_t)N * nrhs));
    double* dz = common.keep(dmalloc<double>((size_t)N * nrhs));
    ok(hlu_spmv(A.A, dx, db, nrhs, N, 1.0, 0.0, stream));
    EventGuard e0, e1;
    HIP_OK(hipEventCreate(&e0.e));
    HIP_OK(hipEventCreate(&e1.e));
    const size_t gw = gmres_workspace_bytes(N, nrhs, go->restart);
    void* gwork = common.keep(dmalloc<char>(gw));
    std::vector<hlu_gmres_info> info(nrhs);
    int32_t pick = 0;
    for (int32_t c = 0; c < count; ++c) {
      hlu_csr csr{N, nnz, rp.data(), ci.data(), val.data()};
      HandleGuard h;
      ok(hlu_build(&csr, mid.data(), eta, leaves[c], &h.h));
      size_t ws = 0;
      ok(hlu_workspace_bytes(h.h, fo, &ws));
      Owned mem;
      void* work = mem.keep(dmalloc<char>(ws));
      ok(hlu_bind_workspace(h.h, work, ws));
      auto factor = [&] {
        const hlu_status st = hlu_factor(h.h, fo, stream);
        if (!(st == HLU_ERR_RANK_OVERFLOW && fo->max_rank > 0)) ok(st);
      };
      factor();   // uploads the plans; the second factorisation is timed
      HIP_OK(hipEventRecord(e0.e, s));
      factor();
      const hlu_status g = gmres_solve(A.A, db, dz, nrhs, N, h.h, go, info.data(), gwork, gw, stream);
      if (g != HLU_ERR_NOT_CONVERGED) ok(g);
      HIP_OK(hipEventRecord(e1.e, s));
      HIP_OK(hipEventSynchronize(e1.e));
      float ms = 0.f;
      HIP_OK(hipEventElapsedTime(&ms, e0.e, e1.e));
      bool conv = true;
      for (const hlu_gmres_info& i : info) conv = conv && i.converged;
      seconds[c] = conv ? ms / 1e3 : HUGE_VAL;
      if (seconds[c] < seconds[pick]) pick = c;
    }
    *best = leaves[pick];
  });
}
