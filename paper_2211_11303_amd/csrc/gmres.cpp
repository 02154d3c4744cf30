// Restarted flexible GMRES (Algorithm 1, step III with a Krylov method in
// place of the plain iteration): right preconditioning, x0 = 0, classical
// Gram-Schmidt applied twice, Givens rotations on the host, convergence on
// the true residual at the end of each cycle.
//
// The driver runs nseg independent systems at once.  Every vector block
// holds one segment per system; dot products, norms and updates are
// segment-wise, so each system keeps its own Arnoldi process, while the
// operator and preconditioner are applied to the whole block in one launch
// (the columns of one matrix, or the problems of a batch).
#include <algorithm>
#include <cmath>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "gmres.h"

namespace hlu {

size_t gmres_core_bytes(int64_t total, int32_t nseg, int32_t m) {
  const size_t blk = align256((size_t)total * sizeof(double));
  size_t b = 0;
  b += blk * (size_t)(m + 1);   // V
  b += blk * (size_t)m;         // Z
  b += blk;                     // w
  b += align256((size_t)kDotBlocks * (m + 1) * nseg * sizeof(double));   // partial dots
  b += align256((size_t)(m + 1) * nseg * sizeof(double)) * 3;            // h, h2, y / scale
  b += align256((size_t)nseg * sizeof(int64_t)) * 2;                     // segment offsets, lengths
  return b;
}

void gmres_core(const GmresSystem& sys, const double* b, double* x, const hlu_gmres_opts* o, void* d_work,
                hlu_gmres_info* info, hipStream_t s) {
  const int32_t nseg = sys.nseg, m = o->restart;
  const size_t blk = align256((size_t)sys.total * sizeof(double));
  const int64_t vstride = (int64_t)(blk / sizeof(double));
  char* wp = static_cast<char*>(d_work);
  double* V = reinterpret_cast<double*>(wp);
  wp += blk * (m + 1);
  double* Z = reinterpret_cast<double*>(wp);
  wp += blk * m;
  double* w = reinterpret_cast<double*>(wp);
  wp += blk;
  double* part = reinterpret_cast<double*>(wp);
  wp += align256((size_t)kDotBlocks * (m + 1) * nseg * sizeof(double));
  double* dh = reinterpret_cast<double*>(wp);
  wp += align256((size_t)(m + 1) * nseg * sizeof(double));
  double* dh2 = reinterpret_cast<double*>(wp);
  wp += align256((size_t)(m + 1) * nseg * sizeof(double));
  double* dy = reinterpret_cast<double*>(wp);
  wp += align256((size_t)(m + 1) * nseg * sizeof(double));
  int64_t* doff = reinterpret_cast<int64_t*>(wp);
  wp += align256((size_t)nseg * sizeof(int64_t));
  int64_t* dlen = reinterpret_cast<int64_t*>(wp);
  HIP_OK(hipMemcpyAsync(doff, sys.off.data(), nseg * sizeof(int64_t), hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(dlen, sys.len.data(), nseg * sizeof(int64_t), hipMemcpyHostToDevice, s));
  int64_t max_len = 1;
  for (int64_t l : sys.len) max_len = std::max(max_len, l);

  auto norms = [&](const double* vec, std::vector<double>* out) {
    HIP_OK(seg_dot_launch(nseg, doff, dlen, 1, vec, vstride, vec, part, dh, s));
    std::vector<double> t(nseg);
    int32_t err = 0;
    HIP_OK(hipMemcpyAsync(t.data(), dh, nseg * sizeof(double), hipMemcpyDeviceToHost, s));
    if (sys.d_err) HIP_OK(hipMemcpyAsync(&err, sys.d_err, sizeof(err), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (err != 0) {
      HIP_OK(zero_int_launch(sys.d_err, 1, s));
      HIP_OK(hipStreamSynchronize(s));
      fail(HLU_ERR_DEVICE, "gmres: a preconditioner launch gave up waiting for its inputs");
    }
    out->resize(nseg);
    for (int c = 0; c < nseg; ++c) (*out)[c] = std::sqrt(std::max(0.0, t[c]));
  };
  // x = 0; residual r = b (in w)
  HIP_OK(hipMemsetAsync(x, 0, (size_t)sys.total * sizeof(double), s));
  HIP_OK(hipMemcpyAsync(w, b, (size_t)sys.total * sizeof(double), hipMemcpyDeviceToDevice, s));
  std::vector<double> bnorm, rnorm;
  norms(w, &bnorm);
  rnorm = bnorm;
  std::vector<int32_t> iters(nseg, 0);
  std::vector<char> conv(nseg, 0);
  for (int c = 0; c < nseg; ++c)
    if (bnorm[c] == 0.0 || rnorm[c] <= o->tol * bnorm[c]) conv[c] = 1;
  std::vector<double> H((size_t)(m + 1) * m * nseg), cs((size_t)m * nseg), sn((size_t)m * nseg);
  std::vector<double> g((size_t)(m + 1) * nseg), hcol((size_t)(m + 1) * nseg), hcol2((size_t)(m + 1) * nseg);
  std::vector<double> scale(nseg), yv((size_t)m * nseg);
  auto Hc = [&](int i, int j, int c) -> double& { return H[((size_t)c * (m + 1) + i) * m + j]; };
  while (true) {
    bool any = false;
    for (int c = 0; c < nseg; ++c)
      if (!conv[c] && iters[c] < o->max_iters) any = true;
    if (!any) break;
    // V_0 = r / ||r||  (r in w)
    for (int c = 0; c < nseg; ++c) scale[c] = (rnorm[c] > 0.0) ? 1.0 / rnorm[c] : 0.0;
    HIP_OK(hipMemcpyAsync(dy, scale.data(), nseg * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_OK(seg_scale_launch(nseg, doff, dlen, max_len, w, dy, V, s));
    std::vector<char> active(nseg, 0);
    std::vector<int> jend(nseg, 0);
    for (int c = 0; c < nseg; ++c) {
      active[c] = !conv[c] && iters[c] < o->max_iters;
      for (int i = 0; i <= m; ++i) g[(size_t)c * (m + 1) + i] = 0.0;
      g[(size_t)c * (m + 1)] = rnorm[c];
    }
    for (int j = 0; j < m; ++j) {
      bool act = false;
      for (int c = 0; c < nseg; ++c) act = act || active[c];
      if (!act) break;
      double* Vj = V + (int64_t)j * vstride;
      double* Zj = Z + (int64_t)j * vstride;
      sys.precond(Vj, Zj);
      sys.matvec(Zj, w);
      // classical Gram-Schmidt, twice
      HIP_OK(seg_dot_launch(nseg, doff, dlen, j + 1, V, vstride, w, part, dh, s));
      HIP_OK(seg_orth_launch(nseg, doff, dlen, max_len, j + 1, V, vstride, dh, w, s));
      HIP_OK(seg_dot_launch(nseg, doff, dlen, j + 1, V, vstride, w, part, dh2, s));
      HIP_OK(seg_orth_launch(nseg, doff, dlen, max_len, j + 1, V, vstride, dh2, w, s));
      HIP_OK(hipMemcpyAsync(hcol.data(), dh, (size_t)(j + 1) * nseg * sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_OK(hipMemcpyAsync(hcol2.data(), dh2, (size_t)(j + 1) * nseg * sizeof(double), hipMemcpyDeviceToHost, s));
      std::vector<double> wn;
      norms(w, &wn);
      for (int c = 0; c < nseg; ++c) {
        scale[c] = 0.0;
        if (!active[c]) continue;
        for (int i = 0; i <= j; ++i) Hc(i, j, c) = hcol[(size_t)i * nseg + c] + hcol2[(size_t)i * nseg + c];
        Hc(j + 1, j, c) = wn[c];
        scale[c] = wn[c] > 0.0 ? 1.0 / wn[c] : 0.0;
        for (int i = 0; i < j; ++i) {
          const double t = cs[(size_t)c * m + i] * Hc(i, j, c) + sn[(size_t)c * m + i] * Hc(i + 1, j, c);
          Hc(i + 1, j, c) = -sn[(size_t)c * m + i] * Hc(i, j, c) + cs[(size_t)c * m + i] * Hc(i + 1, j, c);
          Hc(i, j, c) = t;
        }
        const double den = std::hypot(Hc(j, j, c), Hc(j + 1, j, c));
        cs[(size_t)c * m + j] = den > 0.0 ? Hc(j, j, c) / den : 1.0;
        sn[(size_t)c * m + j] = den > 0.0 ? Hc(j + 1, j, c) / den : 0.0;
        Hc(j, j, c) = den;
        Hc(j + 1, j, c) = 0.0;
        double* gc = &g[(size_t)c * (m + 1)];
        gc[j + 1] = -sn[(size_t)c * m + j] * gc[j];
        gc[j] = cs[(size_t)c * m + j] * gc[j];
        iters[c]++;
        jend[c] = j + 1;
        if (std::fabs(gc[j + 1]) <= o->tol * bnorm[c] || iters[c] >= o->max_iters || den == 0.0) active[c] = 0;
      }
      HIP_OK(hipMemcpyAsync(dy, scale.data(), nseg * sizeof(double), hipMemcpyHostToDevice, s));
      HIP_OK(seg_scale_launch(nseg, doff, dlen, max_len, w, dy, V + (int64_t)(j + 1) * vstride, s));
    }
    // y = H^{-1} g per system, x += Z y
    int jmax = 0;
    for (int c = 0; c < nseg; ++c) jmax = std::max(jmax, jend[c]);
    std::fill(yv.begin(), yv.end(), 0.0);
    for (int c = 0; c < nseg; ++c) {
      const int je = jend[c];
      for (int i = je - 1; i >= 0; --i) {
        double t = g[(size_t)c * (m + 1) + i];
        for (int k = i + 1; k < je; ++k) t -= Hc(i, k, c) * yv[(size_t)k * nseg + c];
        yv[(size_t)i * nseg + c] = Hc(i, i, c) != 0.0 ? t / Hc(i, i, c) : 0.0;
      }
    }
    if (jmax > 0) {
      HIP_OK(hipMemcpyAsync(dh, yv.data(), (size_t)jmax * nseg * sizeof(double), hipMemcpyHostToDevice, s));
      HIP_OK(seg_combine_launch(nseg, doff, dlen, max_len, jmax, Z, vstride, dh, x, s));
    }
    // true residual
    sys.matvec(x, w);
    HIP_OK(sub_launch(sys.total, b, w, s));
    norms(w, &rnorm);
    for (int c = 0; c < nseg; ++c)
      if (!conv[c] && rnorm[c] <= o->tol * bnorm[c]) conv[c] = 1;
    if (jmax == 0) break;
  }
  for (int c = 0; c < nseg; ++c) {
    info[c].iters = iters[c];
    info[c].converged = conv[c];
    info[c].relres = bnorm[c] > 0.0 ? rnorm[c] / bnorm[c] : 0.0;
    info[c].abs_res = rnorm[c];
  }
}

void check_gmres_opts(const hlu_gmres_opts* o) {
  HLU_REQUIRE(o != nullptr, HLU_ERR_INVALID_ARG, "gmres options are NULL");
  HLU_REQUIRE(o->restart >= 1 && o->max_iters >= 1 && o->tol > 0.0, HLU_ERR_INVALID_ARG,
              "gmres: need restart >= 1, max_iters >= 1, tol > 0");
}

}  // namespace hlu

using namespace hlu;

namespace hlu {
namespace {

// gmres_solve on a given workspace.  may_allocate = false: fail instead of
// making the preconditioner's solve buffers (the allocation-free entry).
hlu_status gmres_solve_on(hlu_spmat A, const double* d_b, double* d_x, int32_t nrhs, int64_t ld, hlu_handle precond,
                          const hlu_gmres_opts* o, hlu_gmres_info* info, void* d_work, size_t work_bytes,
                          hipStream_t s, bool may_allocate) {
  bool all_conv = true;
  hlu_status st = guard([&] {
    HLU_REQUIRE(A && d_b && d_x && o && info && d_work && nrhs >= 1 && ld >= A->n, HLU_ERR_INVALID_ARG,
                "gmres_solve: bad arguments");
    check_gmres_opts(o);
    HLU_REQUIRE(d_b != d_x, HLU_ERR_INVALID_ARG, "gmres_solve: x must not alias b");
    if (precond) {
      HLU_REQUIRE(precond->factored, HLU_ERR_STATE, "gmres_solve: preconditioner not factored");
      HLU_REQUIRE(precond->sh->S.N == A->n, HLU_ERR_INVALID_ARG, "gmres_solve: size mismatch");
      if (!may_allocate && precond->mode == 0) {
        HLU_REQUIRE(precond->sbuf != nullptr, HLU_ERR_STATE,
                    "gmres_solve_static: the preconditioner's solve buffers are not made yet (one hlu_solve makes "
                    "them)");
        HLU_REQUIRE(!precond->timing, HLU_ERR_STATE, "gmres_solve_static: solve timing creates events; disable it");
      }
    }
    const int32_t N = A->n;
    const int64_t total = (int64_t)N * nrhs;
    HLU_REQUIRE(work_bytes >= gmres_workspace_bytes(N, nrhs, o->restart), HLU_ERR_OUT_OF_MEMORY,
                "gmres_solve: workspace too small");
    char* wp = static_cast<char*>(d_work);
    double* bb = reinterpret_cast<double*>(wp);
    wp += align256((size_t)total * sizeof(double));
    double* xx = reinterpret_cast<double*>(wp);
    wp += align256((size_t)total * sizeof(double));
    HIP_OK(copy_cols_launch(N, nrhs, d_b, ld, bb, N, s));
    GmresSystem sys;
    sys.nseg = nrhs;
    sys.total = total;
    for (int c = 0; c < nrhs; ++c) {
      sys.off.push_back((int64_t)c * N);
      sys.len.push_back(N);
    }
    sys.matvec = [&](const double* in, double* out) {
      HIP_OK(spmv_launch(N, A->rp, A->ci, A->val, in, out, nrhs, N, 1.0, 0.0, s));
    };
    sys.precond = [&](const double* in, double* out) {
      if (precond) {
        hlu_status ps = hlu_solve(precond, in, out, nrhs, N, s);
        if (ps != HLU_OK) fail(ps, std::string("gmres_solve: preconditioner: ") + get_error());
      } else {
        HIP_OK(hipMemcpyAsync(out, in, (size_t)total * sizeof(double), hipMemcpyDeviceToDevice, s));
      }
    };
    if (precond && precond->mode == 0) {   // H-LU factors: the persistent solve's error word
      ensure_solve_bufs(precond);   // made by the first solve otherwise (checked above when not allowed)
      sys.d_err = precond->sbuf->ctr + 3;
    }
    gmres_core(sys, bb, xx, o, wp, info, s);
    HIP_OK(copy_cols_launch(N, nrhs, xx, N, d_x, ld, s));
    HIP_OK(hipStreamSynchronize(s));
    for (int c = 0; c < nrhs; ++c)
      if (!info[c].converged) all_conv = false;
  });
  if (st != HLU_OK) return st;
  if (!all_conv) {
    set_error("gmres_solve: not converged within max_iters");
    return HLU_ERR_NOT_CONVERGED;
  }
  return HLU_OK;
}

// Workspace of gmres_solve_static: a file-scope device array, one copy per
// GPU, located once per device with hipGetSymbolAddress.  In host code the
// array's name is not a device address; only the located pointers are used.
constexpr size_t kStaticGmresBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kStaticGmresBytes];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;   // device ordinal -> address of its copy of `scratch`

void* static_scratch() {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  void* ptr = nullptr;
  HIP_OK(hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)));
  HLU_REQUIRE(ptr != nullptr, HLU_ERR_DEVICE, "gmres_solve_static: no address for the static workspace");
  g_scratch_ptr[dev] = ptr;
  return ptr;
}

}  // namespace
}  // namespace hlu

extern "C" {

size_t gmres_workspace_bytes(int32_t n, int32_t nrhs, int32_t restart) {
  if (n <= 0 || nrhs <= 0 || restart <= 0) return 0;
  const int64_t total = (int64_t)n * nrhs;
  // + the right-hand side and the iterate, contiguous
  return gmres_core_bytes(total, nrhs, restart) + 2 * align256((size_t)total * sizeof(double));
}

hlu_status gmres_solve(hlu_spmat A, const double* d_b, double* d_x, int32_t nrhs, int64_t ld, hlu_handle precond,
                       const hlu_gmres_opts* o, hlu_gmres_info* info, void* d_work, size_t work_bytes,
                       void* stream) {
  return gmres_solve_on(A, d_b, d_x, nrhs, ld, precond, o, info, d_work, work_bytes, (hipStream_t)stream, true);
}

size_t gmres_refined_workspace_bytes(int32_t n, int32_t nrhs, int32_t restart) {
  if (n <= 0 || nrhs <= 0 || restart <= 0) return 0;
  return gmres_workspace_bytes(n, nrhs, restart) + 2 * align256((size_t)n * nrhs * sizeof(double));
}

hlu_status gmres_solve_refined(hlu_spmat A, const double* d_b, double* d_x, int32_t nrhs, int64_t ld, hlu_handle H,
                               const hlu_gmres_opts* o, const hlu_refine_opts* r, hlu_gmres_info* info,
                               int32_t* refines, void* d_work, size_t work_bytes, void* stream) {
  constexpr double kMinRefineEps = 1e-7;   // the truncation's resolution floor
  hipStream_t s = (hipStream_t)stream;
  hlu_status result = HLU_OK;
  const hlu_status st = guard([&] {
    HLU_REQUIRE(A && d_b && d_x && H && o && r && info && refines && d_work && nrhs >= 1 && ld >= A->n && d_b != d_x,
                HLU_ERR_INVALID_ARG, "gmres_solve_refined: bad arguments");
    HLU_REQUIRE(o->restart >= 1 && o->max_iters >= 1 && r->refine_iters >= 1 && r->max_refines >= 0 &&
                    r->eps_factor > 0.0 && r->eps_factor < 1.0,
                HLU_ERR_INVALID_ARG, "gmres_solve_refined: bad options");
    HLU_REQUIRE(H->factored && H->mode == 0 && !H->batch, HLU_ERR_STATE,
                "gmres_solve_refined: needs H-LU factors in the handle's own workspace");
    HLU_REQUIRE(H->sh->S.N == A->n, HLU_ERR_INVALID_ARG, "gmres_solve_refined: size mismatch");
    const int32_t N = A->n;
    HLU_REQUIRE(work_bytes >= gmres_refined_workspace_bytes(N, nrhs, o->restart), HLU_ERR_OUT_OF_MEMORY,
                "gmres_solve_refined: workspace too small");
    const size_t gw = gmres_workspace_bytes(N, nrhs, o->restart);
    double* pb = reinterpret_cast<double*>(static_cast<char*>(d_work) + gw);
    double* px = reinterpret_cast<double*>(static_cast<char*>(d_work) + gw + align256((size_t)N * nrhs * 8));
    *refines = 0;
    auto can_refine = [&] { return *refines < r->max_refines && H->eps > kMinRefineEps; };
    hlu_gmres_opts go = *o;
    bool capped = can_refine() && r->refine_iters < go.max_iters;
    if (capped) go.max_iters = r->refine_iters;
    hlu_status g = gmres_solve(A, d_b, d_x, nrhs, ld, H, &go, info, d_work, gw, stream);
    if (g != HLU_OK && g != HLU_ERR_NOT_CONVERGED) fail(g, get_error());
    while (g == HLU_ERR_NOT_CONVERGED) {
      std::vector<int32_t> open;
      for (int32_t k = 0; k < nrhs; ++k)
        if (!info[k].converged) open.push_back(k);
      if (open.empty()) {
        g = HLU_OK;
        break;
      }
      if (can_refine()) {
        const hlu_factor_opts fo{std::max(H->eps * r->eps_factor, kMinRefineEps), H->max_rank, H->prec};
        const hlu_status f = hlu_factor(H, &fo, stream);
        if (f != HLU_OK && f != HLU_ERR_RANK_OVERFLOW) fail(f, get_error());
        ++*refines;
      } else if (!capped) {
        break;   // the last attempt had the full budget
      }
      go = *o;
      capped = can_refine() && r->refine_iters < go.max_iters;
      if (capped) go.max_iters = r->refine_iters;
      const int32_t no = (int32_t)open.size();
      for (int32_t i = 0; i < no; ++i)
        HIP_OK(hipMemcpyAsync(pb + (size_t)i * N, d_b + (size_t)open[i] * ld, (size_t)N * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
      std::vector<hlu_gmres_info> io((size_t)no);
      g = gmres_solve(A, pb, px, no, N, H, &go, io.data(), d_work, gmres_workspace_bytes(N, no, go.restart), stream);
      if (g != HLU_OK && g != HLU_ERR_NOT_CONVERGED) fail(g, get_error());
      for (int32_t i = 0; i < no; ++i) {
        HIP_OK(hipMemcpyAsync(d_x + (size_t)open[i] * ld, px + (size_t)i * N, (size_t)N * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
        info[open[i]] = io[(size_t)i];
      }
    }
    HIP_OK(hipStreamSynchronize(s));
    if (g == HLU_ERR_NOT_CONVERGED) {
      set_error("gmres_solve_refined: a column missed tol");
      result = HLU_ERR_NOT_CONVERGED;
    }
  });
  return st != HLU_OK ? st : result;
}

size_t hlu_richardson_workspace_bytes(int32_t n, int32_t nrhs) {
  if (n <= 0 || nrhs <= 0) return 0;
  const size_t blk = align256((size_t)n * nrhs * sizeof(double));
  return 4 * blk + align256((size_t)kDotBlocks * nrhs * sizeof(double)) + 2 * align256((size_t)nrhs * sizeof(double)) +
         2 * align256((size_t)nrhs * sizeof(int64_t));
}

// Algorithm 1, steps III-IV, for every column of b: x_0 = 0 and, for
// k = 1, 2, ...: r = b - A x; err = ||r|| / ||b||; x += U^{-1}(L^{-1} r);
// stop once err < tol (the correction is applied before leaving, the order
// the paper gives) or after max_iters corrections; then ||A x - b||_2.
// Columns run together; a column that has stopped gets zero corrections.
hlu_status hlu_richardson(hlu_spmat A, const double* d_b, double* d_x, int32_t nrhs, int64_t ld, hlu_handle precond,
                          double tol, int32_t max_iters, hlu_gmres_info* info, void* d_work, size_t work_bytes,
                          void* stream) {
  hipStream_t s = (hipStream_t)stream;
  return guard([&] {
    HLU_REQUIRE(A && d_b && d_x && precond && info && d_work && nrhs >= 1 && ld >= A->n && d_b != d_x,
                HLU_ERR_INVALID_ARG, "hlu_richardson: bad arguments");
    HLU_REQUIRE(tol >= 0.0 && std::isfinite(tol) && max_iters >= 1, HLU_ERR_INVALID_ARG,
                "hlu_richardson: need a finite tol >= 0 and max_iters >= 1");
    HLU_REQUIRE(precond->factored, HLU_ERR_STATE, "hlu_richardson: preconditioner not factored");
    HLU_REQUIRE(precond->sh->S.N == A->n, HLU_ERR_INVALID_ARG, "hlu_richardson: size mismatch");
    const int32_t N = A->n;
    HLU_REQUIRE(work_bytes >= hlu_richardson_workspace_bytes(N, nrhs), HLU_ERR_OUT_OF_MEMORY,
                "hlu_richardson: workspace too small");
    const int64_t total = (int64_t)N * nrhs;
    const size_t blk = align256((size_t)total * sizeof(double));
    char* wp = static_cast<char*>(d_work);
    double* bb = reinterpret_cast<double*>(wp);
    wp += blk;
    double* xx = reinterpret_cast<double*>(wp);
    wp += blk;
    double* r = reinterpret_cast<double*>(wp);
    wp += blk;
    double* z = reinterpret_cast<double*>(wp);
    wp += blk;
    double* part = reinterpret_cast<double*>(wp);
    wp += align256((size_t)kDotBlocks * nrhs * sizeof(double));
    double* dn = reinterpret_cast<double*>(wp);
    wp += align256((size_t)nrhs * sizeof(double));
    double* dc = reinterpret_cast<double*>(wp);
    wp += align256((size_t)nrhs * sizeof(double));
    int64_t* doff = reinterpret_cast<int64_t*>(wp);
    wp += align256((size_t)nrhs * sizeof(int64_t));
    int64_t* dlen = reinterpret_cast<int64_t*>(wp);
    std::vector<int64_t> off(nrhs), len(nrhs, N);
    for (int c = 0; c < nrhs; ++c) off[c] = (int64_t)c * N;
    HIP_OK(hipMemcpyAsync(doff, off.data(), nrhs * sizeof(int64_t), hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(dlen, len.data(), nrhs * sizeof(int64_t), hipMemcpyHostToDevice, s));
    HIP_OK(copy_cols_launch(N, nrhs, d_b, ld, bb, N, s));
    HIP_OK(hipMemsetAsync(xx, 0, (size_t)total * sizeof(double), s));
    auto sqnorms = [&](const double* v) {
      HIP_OK(seg_dot_launch(nrhs, doff, dlen, 1, v, 0, v, part, dn, s));
      std::vector<double> t(nrhs);
      HIP_OK(hipMemcpyAsync(t.data(), dn, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_OK(hipStreamSynchronize(s));
      return t;
    };
    auto residual = [&] {   // r = b - A x
      HIP_OK(spmv_launch(N, A->rp, A->ci, A->val, xx, r, nrhs, N, 1.0, 0.0, s));
      HIP_OK(sub_launch(total, bb, r, s));
    };
    std::vector<double> bnorm = sqnorms(bb);
    for (double& v : bnorm) v = std::sqrt(std::max(0.0, v));
    std::vector<char> done(nrhs, 0), conv(nrhs, 0);
    std::vector<int32_t> iters(nrhs, 0);
    std::vector<double> coef(nrhs);
    for (int32_t k = 1; k <= max_iters; ++k) {
      residual();
      const std::vector<double> rn = sqnorms(r);
      bool any = false;
      for (int c = 0; c < nrhs; ++c) {
        coef[c] = done[c] ? 0.0 : 1.0;
        any = any || !done[c];
      }
      if (!any) break;
      HIP_OK(hipMemcpyAsync(dc, coef.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, s));
      HIP_OK(seg_scale_launch(nrhs, doff, dlen, N, r, dc, r, s));   // stopped columns: zero correction
      const hlu_status ps = hlu_solve(precond, r, z, nrhs, N, s);
      if (ps != HLU_OK) fail(ps, std::string("hlu_richardson: preconditioner: ") + get_error());
      for (int c = 0; c < nrhs; ++c) coef[c] = -coef[c];
      HIP_OK(hipMemcpyAsync(dc, coef.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, s));
      HIP_OK(seg_orth_launch(nrhs, doff, dlen, N, 1, z, 0, dc, xx, s));   // x += z on running columns
      for (int c = 0; c < nrhs; ++c) {
        if (done[c]) continue;
        iters[c] = k;
        const double err = bnorm[c] > 0.0 ? std::sqrt(std::max(0.0, rn[c])) / bnorm[c] : 0.0;
        if (err < tol) done[c] = conv[c] = 1;
      }
    }
    residual();
    const std::vector<double> rn = sqnorms(r);
    for (int c = 0; c < nrhs; ++c) {
      info[c].iters = iters[c];
      info[c].converged = conv[c];
      info[c].abs_res = std::sqrt(std::max(0.0, rn[c]));
      info[c].relres = bnorm[c] > 0.0 ? info[c].abs_res / bnorm[c] : 0.0;
    }
    HIP_OK(copy_cols_launch(N, nrhs, xx, N, d_x, ld, s));
    HIP_OK(hipStreamSynchronize(s));
  });
}

size_t gmres_static_max_bytes(void) { return kStaticGmresBytes; }

hlu_status gmres_solve_static(hlu_spmat A, const double* d_b, double* d_x, int32_t nrhs, int64_t ld,
                              hlu_handle precond, const hlu_gmres_opts* o, hlu_gmres_info* info, void* stream) {
  void* work = nullptr;
  hlu_status st = guard([&] {
    HLU_REQUIRE(A && o && nrhs >= 1 && o->restart >= 1, HLU_ERR_INVALID_ARG, "gmres_solve_static: bad arguments");
    const size_t need = gmres_workspace_bytes(A->n, nrhs, o->restart);
    HLU_REQUIRE(need <= kStaticGmresBytes, HLU_ERR_OUT_OF_MEMORY,
                "gmres_solve_static: the Krylov workspace (" + std::to_string(need) +
                    " bytes) exceeds the static workspace (" + std::to_string(kStaticGmresBytes) + " bytes)");
    work = static_scratch();
  });
  if (st != HLU_OK) return st;
  return gmres_solve_on(A, d_b, d_x, nrhs, ld, precond, o, info, work, kStaticGmresBytes, (hipStream_t)stream,
                        false);
}

}  // extern "C"
