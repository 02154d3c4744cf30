// Approximate inverse B_H of the H-matrix A_H by the Schulz iteration
// (Sec. 3: the inverse of the H-matrix approximation of the Galerkin matrix
// by the iterative method of Schulz; Sec. 4: truncated SVDs in the
// admissible blocks; Example 2: B_H as the preconditioner):
//
//   X_{k+1} = X_k (2I - A_H X_k),   X_0 = alpha A^T,
//   alpha = 1 / (||A||_1 ||A||_inf),
//
// every product in H-arithmetic on A's block tree with the factor's task
// kernels (products of blocks, truncated low-rank additions).  A is required
// to be symmetric (the Galerkin matrix K - kappa^2 M is), so X_0 = alpha A.
// The iteration stops on the residual rho_k = ||(I - A_H X_k) Omega||_F /
// ||Omega||_F of the caller's probe block Omega, when it reaches tol, when a
// step does not decrease it (the truncation floor; the previous iterate is
// kept) or after max_iters steps.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "handle.h"

namespace hlu {

InverseBundle& get_inverse_bundle(Shared& sh, PlanBundle& pb) {
  std::lock_guard<std::mutex> lock(sh.mu);
  if (!pb.inv) {
    auto ib = std::make_unique<InverseBundle>();
    build_inverse_plans(sh.S, pb.kcap, kMaxRhs, &ib->ip);
    // matrix 0 has the factor's leaf layout, so A's scatter targets apply
    HLU_REQUIRE(ib->ip.store.off == pb.ps.store.off && ib->ip.store.yoff == pb.ps.store.yoff &&
                    ib->ip.store.identity_off == pb.ps.store.identity_off,
                HLU_ERR_INVALID_ARG, "internal: inverse layout differs from the factor layout");
    for (int s = 0; s < 2; ++s) {
      ib->dstep[s].load(ib->ip.step[s]);
      ib->dapply[s].load(ib->ip.apply[s]);
    }
    ib->damul.load(ib->ip.amul);
    pb.inv = std::move(ib);
  }
  return *pb.inv;
}

namespace {

struct InvLayout {
  size_t arena_bytes, dims_off, status_off, red_off, total;
};

InvLayout inv_layout(const InversePlanSet& ip, int32_t prec) {
  InvLayout L;
  L.arena_bytes = align256((size_t)ip.store.total_elems * elem_size(prec));
  L.dims_off = L.arena_bytes;
  L.status_off = L.dims_off + align256((size_t)ip.store.num_slots * sizeof(int32_t));
  L.red_off = L.status_off + align256(kStatusWords * sizeof(int32_t));
  L.total = L.red_off + align256(diff_norm_scratch_doubles() * sizeof(double));
  return L;
}

// A == A^T up to rounding (|a_ij - a_ji| <= 1e-13 max |a|), on the host.
bool values_symmetric(const Shared& sh, const std::vector<double>& val) {
  double amax = 0.0;
  for (double v : val) amax = std::max(amax, std::fabs(v));
  const int32_t N = (int32_t)sh.row_ptr.size() - 1;
  for (int32_t r = 0; r < N; ++r)
    for (int32_t p = sh.row_ptr[r]; p < sh.row_ptr[r + 1]; ++p) {
      const int32_t c = sh.col[p];
      const auto b = sh.col.begin() + sh.row_ptr[c], e = sh.col.begin() + sh.row_ptr[c + 1];
      const auto it = std::lower_bound(b, e, r);
      const double vt = (it != e && *it == r) ? val[it - sh.col.begin()] : 0.0;
      if (std::fabs(val[p] - vt) > 1e-13 * amax) return false;
    }
  return true;
}

// 1 / (||A||_1 ||A||_inf): X_0 = alpha A^T gives X_0 A eigenvalues in (0, 1].
double schulz_alpha(const Shared& sh, const std::vector<double>& val) {
  const int32_t N = (int32_t)sh.row_ptr.size() - 1;
  std::vector<double> colsum(N, 0.0);
  double rowmax = 0.0;
  for (int32_t r = 0; r < N; ++r) {
    double rs = 0.0;
    for (int32_t p = sh.row_ptr[r]; p < sh.row_ptr[r + 1]; ++p) {
      rs += std::fabs(val[p]);
      colsum[sh.col[p]] += std::fabs(val[p]);
    }
    rowmax = std::max(rowmax, rs);
  }
  const double colmax = *std::max_element(colsum.begin(), colsum.end());
  HLU_REQUIRE(colmax > 0.0 && rowmax > 0.0, HLU_ERR_INVALID_ARG, "hlu_inverse: zero matrix");
  return 1.0 / (colmax * rowmax);
}

template <class T>
void run_inv_plan(hlu_s* h, const Plan& pl, const DevArrays& d, bool compute64, hipStream_t s) {
  HIP_OK(run_waves<T>(static_cast<T*>(h->arena), d.P, pl.waves, h->dims, h->status, h->eps, kFloorRel,
                      h->sh->max_leaf, compute64, s, nullptr, &h->waves));
}

// rho = ||V - A_H X V||_F / ||V||_F for the probe block V (nc columns at
// vec_off) and X in matrix 1 + 2 which.
template <class T>
double inv_residual(hlu_s* h, InverseBundle& ib, int which, int32_t nc, hipStream_t s) {
  const InversePlanSet& ip = ib.ip;
  T* arena = static_cast<T*>(h->arena);
  run_inv_plan<T>(h, ip.apply[which], ib.dapply[which], true, s);   // W = X V
  run_inv_plan<T>(h, ip.amul, ib.damul, true, s);                   // U = A_H W
  const int64_t n = (int64_t)h->sh->S.N * nc;
  HIP_OK(diff_norm_launch<T>(n, arena + ip.store.vec_off, arena + ip.vec3_off, h->red, s));
  double r[2];
  HIP_OK(hipMemcpyAsync(r, h->red + diff_norm_scratch_doubles() - 2, sizeof(r), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return r[1] > 0.0 ? std::sqrt(r[0] / r[1]) : 0.0;
}

template <class T>
void inverse_impl(hlu_s* h, InverseBundle& ib, double alpha, const hlu_schulz_opts* so, const double* d_probe,
                  int32_t nprobe, hlu_schulz_info* info, hipStream_t s) {
  const InversePlanSet& ip = ib.ip;
  const StoragePlan& st = ip.store;
  T* arena = static_cast<T*>(h->arena);
  const int32_t N = h->sh->S.N;
  ensure_values(h);
  HIP_OK(zero_launch<T>(arena, st.data_elems, s));
  HIP_OK(identity_launch<T>(arena + st.identity_off, st.identity_n, s));
  const int64_t nnz = (int64_t)h->val.size();
  HIP_OK(scatter_values_launch<T>(nnz, h->pb->d_target, h->d_val, arena, s));   // matrix 0: A_H
  HIP_OK(scatter_values_scaled_launch<T>(nnz, h->pb->d_target, ip.mat_elems, alpha, h->d_val, arena, s));   // X_0
  HIP_OK(zero_int_launch(h->dims, st.num_slots, s));
  HIP_OK(zero_int_launch(h->status, kStatusWords, s));
  HIP_OK(gather_launch<T>(N, nprobe, h->sh->d_perm, d_probe, N, arena + st.vec_off, N, s));
  HIP_OK(set_int_launch(h->dims + st.nrhs_slot, nprobe, s));
  int cur = 0;   // X_k in matrix 1 + 2 cur
  double rho = inv_residual<T>(h, ib, cur, nprobe, s);
  const double rho0 = rho;
  int32_t it = 0;
  const bool c64 = fp64_tasks(h->prec);
  while (it < so->max_iters && rho > so->tol) {
    const int out = 1 - cur;
    // Z (matrix 2), the target iterate and the plans' temporary ranks start at zero
    HIP_OK(zero_launch<T>(arena + ip.mat0_off + 2 * ip.mat_elems, ip.mat_elems, s));
    HIP_OK(zero_launch<T>(arena + ip.mat0_off + (int64_t)(1 + 2 * out) * ip.mat_elems, ip.mat_elems, s));
    HIP_OK(zero_int_launch(h->dims + 2 * ip.mat_slots, ip.mat_slots, s));
    HIP_OK(zero_int_launch(h->dims + (1 + 2 * out) * ip.mat_slots, ip.mat_slots, s));
    HIP_OK(zero_int_launch(h->dims + ip.temp_slot0, st.num_slots - ip.temp_slot0, s));
    run_inv_plan<T>(h, ip.step[cur], ib.dstep[cur], c64, s);
    HIP_OK(set_int_launch(h->dims + st.nrhs_slot, nprobe, s));
    const double rn = inv_residual<T>(h, ib, out, nprobe, s);
    if (!(rn < rho)) break;   // no progress: keep X_k
    cur = out;
    rho = rn;
    ++it;
  }
  h->inv_mat = 1 + 2 * cur;
  info->iters = it;
  info->converged = rho <= so->tol ? 1 : 0;
  info->residual = rho;
  info->residual0 = rho0;
}

// Ranks of B_H and the task counts of one step into the handle's stats.
void inverse_stats(hlu_s* h, InverseBundle& ib) {
  const InversePlanSet& ip = ib.ip;
  const StoragePlan& st = ip.store;
  const Structure& S = h->sh->S;
  std::vector<int32_t> dims(st.num_slots);
  HIP_OK(hipMemcpy(dims.data(), h->dims, dims.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  int32_t maxr = 0;
  double sumr = 0.0, entries = 0.0;
  int64_t nlr = 0;
  for (size_t l = 0; l < S.leaves.size(); ++l) {
    if (st.slot[l] < 0) continue;
    const BlockNode& b = S.blocks[S.leaves[l]];
    const int32_t r = dims[st.slot[l] + h->inv_mat * ip.mat_slots];
    maxr = std::max(maxr, r);
    sumr += r;
    entries += (double)r * (S.clusters[b.row].size() + S.clusters[b.col].size());
    ++nlr;
  }
  h->stats.max_rank = maxr;
  h->stats.mean_rank = nlr ? sumr / nlr : 0.0;
  h->stats.lowrank_entries = entries;
  h->stats.factor_waves = (int64_t)ip.step[0].waves.size();
  h->stats.factor_tasks = ip.step[0].num_tasks;
  h->stats.workspace_bytes = (int64_t)inv_layout(ip, h->prec).total;
}

template <class T>
void inverse_apply_impl(hlu_s* h, const double* b, double* x, int32_t nrhs, int64_t ld, hipStream_t s) {
  InverseBundle& ib = *h->pb->inv;
  const StoragePlan& st = ib.ip.store;
  T* arena = static_cast<T*>(h->arena);
  const int32_t N = h->sh->S.N;
  const int which = h->inv_mat == 1 ? 0 : 1;
  for (int32_t c0 = 0; c0 < nrhs; c0 += st.max_rhs) {
    const int32_t nc = std::min(st.max_rhs, nrhs - c0);
    HIP_OK(gather_launch<T>(N, nc, h->sh->d_perm, b + (int64_t)c0 * ld, ld, arena + st.vec_off, N, s));
    HIP_OK(set_int_launch(h->dims + st.nrhs_slot, nc, s));
    run_inv_plan<T>(h, ib.ip.apply[which], ib.dapply[which], true, s);
    HIP_OK(scatter_perm_launch<T>(N, nc, h->sh->d_perm, arena + st.vec2_off, N, x + (int64_t)c0 * ld, ld, s));
  }
}

}  // namespace

void inverse_apply(hlu_s* h, const double* b, double* x, int32_t nrhs, int64_t ld, hipStream_t s) {
  if (fp32_storage(h->prec)) inverse_apply_impl<float>(h, b, x, nrhs, ld, s);
  else inverse_apply_impl<double>(h, b, x, nrhs, ld, s);
}

}  // namespace hlu

using namespace hlu;

extern "C" {

hlu_status hlu_inverse_workspace_bytes(hlu_handle h, const hlu_factor_opts* o, size_t* bytes) {
  return guard([&] {
    HLU_REQUIRE(h && bytes, HLU_ERR_INVALID_ARG, "hlu_inverse_workspace_bytes: NULL argument");
    check_opts(o);
    HLU_REQUIRE(h->sh->nonzero_admissible.empty(), HLU_ERR_UNSUPPORTED,
                "hlu_inverse: admissible blocks hold matrix entries (leaf size too small for the inverse)");
    use_bundle(h, kcap_for(o));
    InverseBundle& ib = get_inverse_bundle(*h->sh, *h->pb);
    *bytes = inv_layout(ib.ip, o->prec).total;
  });
}

hlu_status hlu_inverse(hlu_handle h, const hlu_factor_opts* o, const hlu_schulz_opts* so, const double* d_probe,
                       int32_t nprobe, hlu_schulz_info* info, void* stream) {
  return guard([&] {
    HLU_REQUIRE(h && so && d_probe && info, HLU_ERR_INVALID_ARG, "hlu_inverse: NULL argument");
    check_opts(o);
    HLU_REQUIRE(so->max_iters >= 0 && so->tol >= 0.0 && std::isfinite(so->tol), HLU_ERR_INVALID_ARG,
                "hlu_inverse: need max_iters >= 0 and a finite tol >= 0");
    HLU_REQUIRE(nprobe >= 1 && nprobe <= kMaxRhs, HLU_ERR_INVALID_ARG, "hlu_inverse: need 1 <= nprobe <= 32");
    HLU_REQUIRE(!h->batch, HLU_ERR_STATE, "hlu_inverse: handle is bound through a batch");
    HLU_REQUIRE(h->sh->nonzero_admissible.empty(), HLU_ERR_UNSUPPORTED,
                "hlu_inverse: admissible blocks hold matrix entries (leaf size too small for the inverse)");
    if (h->symmetric < 0) h->symmetric = values_symmetric(*h->sh, h->val) ? 1 : 0;
    HLU_REQUIRE(h->symmetric == 1, HLU_ERR_UNSUPPORTED, "hlu_inverse: the matrix is not symmetric");
    use_bundle(h, kcap_for(o));
    ensure_device(*h->sh, *h->pb);
    InverseBundle& ib = get_inverse_bundle(*h->sh, *h->pb);
    const InvLayout L = inv_layout(ib.ip, o->prec);
    HLU_REQUIRE(h->work != nullptr, HLU_ERR_STATE, "hlu_inverse: no workspace bound");
    HLU_REQUIRE(h->work_bytes >= L.total, HLU_ERR_OUT_OF_MEMORY, "hlu_inverse: bound workspace too small");
    h->factored = false;
    h->arena = h->work;
    h->dims = reinterpret_cast<int32_t*>(static_cast<char*>(h->work) + L.dims_off);
    h->status = reinterpret_cast<int32_t*>(static_cast<char*>(h->work) + L.status_off);
    h->red = reinterpret_cast<double*>(static_cast<char*>(h->work) + L.red_off);
    h->peak = nullptr;
    h->peak_valid = false;
    h->prec = o->prec;
    h->eps = o->eps;
    h->factor_compute64 = fp64_tasks(o->prec);
    h->mode = 1;
    h->sbuf.reset();   // the persistent LU solve's buffers hold nothing of the inverse
    const double alpha = schulz_alpha(*h->sh, h->val);
    hipStream_t s = (hipStream_t)stream;
    std::memset(info, 0, sizeof(*info));
    if (fp32_storage(o->prec)) inverse_impl<float>(h, ib, alpha, so, d_probe, nprobe, info, s);
    else inverse_impl<double>(h, ib, alpha, so, d_probe, nprobe, info, s);
    HIP_OK(hipStreamSynchronize(s));
    int32_t status[3];
    HIP_OK(hipMemcpy(status, h->status, sizeof(status), hipMemcpyDeviceToHost));
    HLU_REQUIRE(status[2] == 0, HLU_ERR_DEVICE, "hlu_inverse: a truncation exceeded its round bound");
    inverse_stats(h, ib);
    h->stats.capped_blocks = status[1];
    read_flops(h->status, &h->stats);
    h->factored = true;
  });
}

}  // extern "C"
