// Batches of independent problems factored and solved together.
//
// The problems' factors live in one workspace: problem p's arena at a byte
// offset of its own, all rank tables in one region.  Every task of a
// problem's factor plan addresses the arena by element offsets and its
// ranks by table slots, so a batch plan is the union of the problems' plans
// with offsets and slots shifted: wave w of the batch holds wave w of every
// problem, and each launch of the batch runs the getrf / trsm / H-GEMM /
// recompression tasks of all problems that are ready at that depth.  The
// batch needs as many waves as its deepest problem, not their sum.
//
// The persistent solve is merged the same way: every problem keeps its own
// chains, the problems' helper tasks are interleaved (each problem's own
// order is kept, so every wait still points backwards), vectors of all
// problems are stacked into one block, and a single launch runs all sweeps.
#include <algorithm>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "gmres.h"

struct hlu_batch_s {
  std::vector<hlu_s*> hs;
  hlu::WaveStreams waves;   // second stream of the batched factorisation's waves
  hlu_factor_opts opts{};
  int32_t kcap = 0, max_rhs = 0;
  // workspace layout
  std::vector<size_t> arena_off;    // bytes from the workspace start
  std::vector<int32_t> slot_base;   // first rank slot of each problem
  std::vector<int32_t> row_base;    // first row of each problem in stacked vectors
  int32_t N_tot = 0;
  size_t dims_off = 0, status_off = 0, total = 0;
  int32_t max_leaf = 0;
  // merged factor plan and solve schedule
  hlu::Plan plan;
  hlu::DevArrays dplan;
  hlu::ChainSched sc;
  hlu::DevSched dsc;
  hlu::SolveBufs bufs;
  hlu::Owned mem;
  int32_t* d_perm = nullptr;        // stacked permutation (problem p: rows of p only)
  // block-diagonal A of all problems, for the batched GMRES
  int32_t* d_rp = nullptr;
  int32_t* d_ci = nullptr;
  double* d_val = nullptr;
  // bound workspace
  void* work = nullptr;
  size_t work_bytes = 0;
  bool factored = false;
};

namespace hlu {

namespace {

MatRef shift(MatRef r, int64_t a, int32_t d) {
  r.off += a;
  if (r.rows < 0) r.rows -= d;   // -(s+1) -> -(s+d+1)
  if (r.cols < 0) r.cols -= d;
  return r;
}

// Union of the problems' factor plans (see the file comment).
void merge_plans(const std::vector<const Plan*>& P, const std::vector<int64_t>& a, const std::vector<int32_t>& d,
                 Plan* out) {
  Plan& M = *out;
  const size_t np = P.size();
  size_t nw = 0;
  for (const Plan* p : P) {
    nw = std::max(nw, p->waves.size());
    M.num_tasks += p->num_tasks;
  }
  std::vector<int64_t> tile_pos(np, 0);
  std::vector<int32_t> gemm_begin(np, 0);
  M.waves.assign(nw, Wave{});
  for (size_t w = 0; w < nw; ++w) {
    Wave& W = M.waves[w];
    W.gemm_tiles = 0;
    for (int k = 0; k < kNumKinds; ++k) {
      switch (k) {
        case kGetrf: W.begin[k] = (int32_t)M.getrf.size(); break;
        case kTri: W.begin[k] = (int32_t)M.tri.size(); break;
        case kGemm: W.begin[k] = (int32_t)M.gemm.size(); break;
        case kTrunc: W.begin[k] = (int32_t)M.trunc.size(); break;
        default: W.begin[k] = (int32_t)M.fill.size(); break;
      }
      int32_t count = 0;
      for (size_t p = 0; p < np; ++p) {
        if (w >= P[p]->waves.size()) continue;
        const Plan& Q = *P[p];
        const Wave& pw = Q.waves[w];
        if (k == kGemm) gemm_begin[p] = (int32_t)M.gemm.size();
        for (int32_t i = pw.begin[k]; i < pw.begin[k] + pw.count[k]; ++i) {
          switch (k) {
            case kGetrf: {
              GetrfOp g = Q.getrf[i];
              g.off += a[p];
              M.getrf.push_back(g);
              break;
            }
            case kTri: {
              TriOp t = Q.tri[i];
              t.tri += a[p];
              t.V = shift(t.V, a[p], d[p]);
              t.W = shift(t.W, a[p], d[p]);
              M.tri.push_back(t);
              break;
            }
            case kGemm: {
              GemmOp g = Q.gemm[i];
              g.C = shift(g.C, a[p], d[p]);
              const int32_t t0 = (int32_t)M.terms.size();
              for (int32_t t = g.t0; t < g.t0 + g.nt; ++t) {
                GemmTerm tm = Q.terms[t];
                tm.A = shift(tm.A, a[p], d[p]);
                tm.B = shift(tm.B, a[p], d[p]);
                M.terms.push_back(tm);
              }
              g.t0 = t0;
              M.gemm.push_back(g);
              break;
            }
            case kTrunc: {
              TruncOp t = Q.trunc[i];
              t.xoff += a[p];
              t.yoff += a[p];
              t.slot += d[p];
              const int32_t p0 = (int32_t)M.parts.size();
              for (int32_t q = t.p0; q < t.p0 + t.np; ++q) {
                TruncPart part = Q.parts[q];
                part.X = shift(part.X, a[p], d[p]);
                part.Y = shift(part.Y, a[p], d[p]);
                M.parts.push_back(part);
              }
              t.p0 = p0;
              M.trunc.push_back(t);
              break;
            }
            default: {
              FillOp f = Q.fill[i];
              f.M = shift(f.M, a[p], d[p]);
              M.fill.push_back(f);
              break;
            }
          }
        }
        count += pw.count[k];
      }
      W.count[k] = count;
      if (k == kTrunc) std::stable_sort(M.trunc.begin() + W.begin[k], M.trunc.end(), trunc_launch_before);
    }
    // GEMM tiles of the wave, problem by problem, pointing at the merged ops
    for (size_t p = 0; p < np; ++p) {
      if (w >= P[p]->waves.size()) continue;
      const Plan& Q = *P[p];
      const Wave& pw = Q.waves[w];
      for (int32_t t = 0; t < pw.gemm_tiles; ++t) {
        const int64_t q = tile_pos[p] + t;
        M.gemm_tile_op.push_back(Q.gemm_tile_op[q] - pw.begin[kGemm] + gemm_begin[p]);
        M.gemm_tile_ij.push_back(Q.gemm_tile_ij[q]);
      }
      tile_pos[p] += pw.gemm_tiles;
      W.gemm_tiles += pw.gemm_tiles;
    }
  }
}

hlu_batch_s* checked(hlu_batch_s* b, bool need_bound) {
  HLU_REQUIRE(b, HLU_ERR_INVALID_ARG, "NULL batch");
  for (hlu_s* h : b->hs) HLU_REQUIRE(h, HLU_ERR_STATE, "a member handle of the batch was destroyed");
  if (need_bound) HLU_REQUIRE(b->work, HLU_ERR_STATE, "no batch workspace bound");
  return b;
}

template <class T>
void factor_batch_impl(hlu_batch_s* b, hipStream_t s) {
  char* base = static_cast<char*>(b->work);
  int32_t* dims = reinterpret_cast<int32_t*>(base + b->dims_off);
  int32_t* status = reinterpret_cast<int32_t*>(base + b->status_off);
  for (size_t p = 0; p < b->hs.size(); ++p)
    factor_prepare<T>(b->hs[p], reinterpret_cast<T*>(base + b->arena_off[p]), dims + b->slot_base[p], s);
  HIP_OK(zero_int_launch(status, kStatusWords, s));
  const bool compute64 = fp64_tasks(b->opts.prec);
  HIP_OK(run_waves<T>(reinterpret_cast<T*>(base), b->dplan.P, b->plan.waves, dims, status, b->opts.eps, kFloorRel,
                      b->max_leaf, compute64, s, nullptr, &b->waves));
  const ChainDev d = make_chain_dev(b->sc, b->dsc, b->bufs);
  HIP_OK(chain_prepare_launch<T>(reinterpret_cast<const T*>(base), dims, d, d.L, s));
}

template <class T>
void solve_batch_impl(hlu_batch_s* b, const double* x_in, double* x_out, int32_t nrhs, hipStream_t s) {
  char* base = static_cast<char*>(b->work);
  const int32_t* dims = reinterpret_cast<const int32_t*>(base + b->dims_off);
  SolveBufs& sb = b->bufs;
  const ChainDev d = make_chain_dev(b->sc, b->dsc, sb);
  const int32_t N = b->N_tot;
  HIP_OK(gather_launch<double>(N, nrhs, b->d_perm, x_in, N, sb.y, N, s));
  sb.epoch = sb.epoch % 1000000000 + 1;
  HIP_OK(chain_solve_launch<T>(reinterpret_cast<const T*>(base), dims, d, N, nrhs, sb.epoch, s));
  HIP_OK(scatter_perm_launch<double>(N, nrhs, b->d_perm, sb.y, N, x_out, N, s));
}

void solve_batch(hlu_batch_s* b, const double* in, double* out, int32_t nrhs, hipStream_t s) {
  if (fp32_storage(b->opts.prec)) solve_batch_impl<float>(b, in, out, nrhs, s);
  else solve_batch_impl<double>(b, in, out, nrhs, s);
}

}  // namespace

void batch_forget(hlu_batch_s* b, hlu_s* h) {
  for (hlu_s*& m : b->hs)
    if (m == h) m = nullptr;
  b->factored = false;
}

}  // namespace hlu

using namespace hlu;

extern "C" {

hlu_status hlu_batch_create(const hlu_handle* hs, int32_t count, const hlu_factor_opts* o, int32_t max_rhs,
                            hlu_batch* out) {
  return guard([&] {
    HLU_REQUIRE(hs && out && count >= 1, HLU_ERR_INVALID_ARG, "hlu_batch_create: bad arguments");
    HLU_REQUIRE(max_rhs >= 1 && max_rhs <= kMaxRhs, HLU_ERR_INVALID_ARG, "hlu_batch_create: need 1 <= max_rhs <= 32");
    HLU_REQUIRE(count <= kMaxChains, HLU_ERR_UNSUPPORTED,
                "hlu_batch_create: at most 64 problems (each needs a chain workgroup of the solve)");
    check_opts(o);
    for (int32_t i = 0; i < count; ++i) {
      HLU_REQUIRE(hs[i], HLU_ERR_INVALID_ARG, "hlu_batch_create: NULL handle");
      HLU_REQUIRE(!hs[i]->batch, HLU_ERR_STATE, "hlu_batch_create: handle already belongs to a batch");
      for (int32_t j = 0; j < i; ++j)
        HLU_REQUIRE(hs[j] != hs[i], HLU_ERR_INVALID_ARG, "hlu_batch_create: handle listed twice");
    }
    auto b = std::make_unique<hlu_batch_s>();
    b->opts = *o;
    b->kcap = kcap_for(o);
    b->max_rhs = max_rhs;
    b->hs.assign(hs, hs + count);
    std::vector<std::shared_ptr<PlanBundle>> pbs;
    for (hlu_s* h : b->hs) {
      pbs.push_back((h->fitted && h->fitted->kcap == b->kcap) ? h->fitted : get_bundle(*h->sh, b->kcap));
      ensure_device(*h->sh, *pbs.back());
    }
    // layout: arenas, then all rank tables, then the status words
    size_t off = 0;
    int32_t slots = 0, rows = 0;
    for (size_t p = 0; p < pbs.size(); ++p) {
      const PlanSet& ps = pbs[p]->ps;
      b->arena_off.push_back(off);
      off += work_layout(ps, o->prec).arena_bytes;
      b->slot_base.push_back(slots);
      slots += ps.store.num_slots;
      b->row_base.push_back(rows);
      rows += b->hs[p]->sh->S.N;
      b->max_leaf = std::max(b->max_leaf, b->hs[p]->sh->max_leaf);
    }
    b->N_tot = rows;
    b->dims_off = off;
    b->status_off = b->dims_off + align256((size_t)slots * sizeof(int32_t));
    b->total = b->status_off + kStatusWords * sizeof(int32_t);
    // merged plan and schedule
    const size_t es = elem_size(o->prec);
    std::vector<int64_t> a;
    for (size_t x : b->arena_off) a.push_back((int64_t)(x / es));
    std::vector<const Plan*> plans;
    std::vector<const ChainSched*> scheds;
    for (auto& pb : pbs) {
      plans.push_back(&pb->ps.factor);
      scheds.push_back(&pb->sc);
    }
    merge_plans(plans, a, b->slot_base, &b->plan);
    merge_chain_scheds(scheds, a, b->slot_base, b->row_base, &b->sc);
    b->dplan.load(b->plan);
    b->dsc.load(b->sc);
    b->bufs.alloc(b->sc, b->N_tot, max_rhs);
    // stacked permutation and block-diagonal A
    std::vector<int32_t> perm(b->N_tot), rp(1, 0), ci;
    std::vector<double> val;
    for (size_t p = 0; p < b->hs.size(); ++p) {
      const Shared& sh = *b->hs[p]->sh;
      const int32_t o0 = b->row_base[p];
      for (int32_t i = 0; i < sh.S.N; ++i) perm[o0 + i] = o0 + sh.S.perm[i];
      for (int32_t r = 0; r < sh.S.N; ++r) rp.push_back(rp.back() + sh.row_ptr[r + 1] - sh.row_ptr[r]);
      for (int32_t c : sh.col) ci.push_back(c + o0);
      val.insert(val.end(), b->hs[p]->val.begin(), b->hs[p]->val.end());
    }
    b->d_perm = b->mem.keep(upload(perm));
    b->d_rp = b->mem.keep(upload(rp));
    b->d_ci = b->mem.keep(upload(ci));
    b->d_val = b->mem.keep(upload(val));
    for (size_t p = 0; p < b->hs.size(); ++p) {
      hlu_s* h = b->hs[p];
      h->pb = pbs[p];
      h->sbuf.reset();
      h->factored = false;
      h->batch = b.get();
      h->prec = o->prec;
    }
    *out = b.release();
  });
}

hlu_status hlu_batch_workspace_bytes(hlu_batch b, size_t* bytes) {
  return guard([&] {
    checked(b, false);
    HLU_REQUIRE(bytes, HLU_ERR_INVALID_ARG, "hlu_batch_workspace_bytes: NULL argument");
    *bytes = b->total;
  });
}

hlu_status hlu_batch_bind_workspace(hlu_batch b, void* d_work, size_t bytes) {
  return guard([&] {
    checked(b, false);
    HLU_REQUIRE(d_work, HLU_ERR_INVALID_ARG, "hlu_batch_bind_workspace: NULL workspace");
    HLU_REQUIRE(((uintptr_t)d_work & 255) == 0, HLU_ERR_INVALID_ARG,
                "hlu_batch_bind_workspace: need 256-byte alignment");
    HLU_REQUIRE(bytes >= b->total, HLU_ERR_OUT_OF_MEMORY, "hlu_batch_bind_workspace: workspace too small");
    b->work = d_work;
    b->work_bytes = bytes;
    b->factored = false;
    char* base = static_cast<char*>(d_work);
    for (size_t p = 0; p < b->hs.size(); ++p) {
      hlu_s* h = b->hs[p];
      h->arena = base + b->arena_off[p];
      h->dims = reinterpret_cast<int32_t*>(base + b->dims_off) + b->slot_base[p];
      h->status = reinterpret_cast<int32_t*>(base + b->status_off);
      h->peak = nullptr;
      h->peak_valid = false;
      h->factored = false;
    }
  });
}

hlu_status hlu_factor_batch(hlu_batch b, void* stream) {
  hlu_status overflow = HLU_OK;
  hlu_status st = guard([&] {
    checked(b, true);
    hipStream_t s = (hipStream_t)stream;
    b->factored = false;
    for (hlu_s* h : b->hs) {
      h->factored = false;
      record_factor(h, &b->opts);
    }
    if (fp32_storage(b->opts.prec)) factor_batch_impl<float>(b, s);
    else factor_batch_impl<double>(b, s);
    HIP_OK(hipStreamSynchronize(s));
    int32_t status[3];
    HIP_OK(hipMemcpy(status, static_cast<char*>(b->work) + b->status_off, sizeof(status), hipMemcpyDeviceToHost));
    HLU_REQUIRE(status[0] == 0, HLU_ERR_ZERO_PIVOT, "hlu_factor_batch: zero pivot in a diagonal leaf");
    HLU_REQUIRE(status[2] == 0, HLU_ERR_DEVICE, "hlu_factor_batch: a truncation exceeded its round bound");
    for (size_t p = 0; p < b->hs.size(); ++p) {
      hlu_s* h = b->hs[p];
      h->factored = true;
      h->inv_ready = false;   // its own solves form their inverses on first use
      gather_stats(h, b->bufs.pivots + b->row_base[p]);
      h->stats.capped_blocks = status[1];
    }
    b->factored = true;
    if (status[1] > 0 && b->opts.max_rank == 0) {
      set_error("hlu_factor_batch: a truncated rank exceeded the block capacity");
      overflow = HLU_ERR_RANK_OVERFLOW;
    }
  });
  return st != HLU_OK ? st : overflow;
}

hlu_status hlu_batch_sizes(hlu_batch b, int32_t* count, int32_t* n_total, int32_t* row_base, int64_t* factor_waves,
                           int64_t* factor_tasks) {
  return guard([&] {
    checked(b, false);
    if (count) *count = (int32_t)b->hs.size();
    if (n_total) *n_total = b->N_tot;
    if (row_base) std::memcpy(row_base, b->row_base.data(), b->row_base.size() * sizeof(int32_t));
    if (factor_waves) *factor_waves = (int64_t)b->plan.waves.size();
    if (factor_tasks) *factor_tasks = b->plan.num_tasks;
  });
}

hlu_status hlu_solve_batch(hlu_batch b, const double* d_b, double* d_x, int32_t nrhs, void* stream) {
  return guard([&] {
    checked(b, true);
    HLU_REQUIRE(d_b && d_x && nrhs >= 1 && nrhs <= b->max_rhs, HLU_ERR_INVALID_ARG,
                "hlu_solve_batch: need 1 <= nrhs <= the batch's max_rhs");
    HLU_REQUIRE(b->factored, HLU_ERR_STATE, "hlu_solve_batch: batch is not factored");
    solve_batch(b, d_b, d_x, nrhs, (hipStream_t)stream);
  });
}

hlu_status hlu_batch_sync_status(hlu_batch b, void* stream) {
  return guard([&] {
    checked(b, false);
    hipStream_t s = (hipStream_t)stream;
    HIP_OK(hipStreamSynchronize(s));
    if (b->bufs.ctr && take_solve_error(b->bufs.ctr, s))
      fail(HLU_ERR_DEVICE,
           "hlu_batch_sync_status: a persistent solve gave up waiting for its inputs; its results are invalid");
  });
}

size_t gmres_batch_workspace_bytes(hlu_batch b, int32_t nrhs, int32_t restart) {
  if (!b || nrhs <= 0 || restart <= 0) return 0;
  return gmres_core_bytes((int64_t)b->N_tot * nrhs, (int32_t)b->hs.size() * nrhs, restart);
}

hlu_status gmres_solve_batch(hlu_batch b, const double* d_b, double* d_x, int32_t nrhs, const hlu_gmres_opts* o,
                             hlu_gmres_info* info, void* d_work, size_t work_bytes, void* stream) {
  bool all_conv = true;
  hlu_status st = guard([&] {
    checked(b, true);
    HLU_REQUIRE(d_b && d_x && info && d_work && nrhs >= 1 && nrhs <= b->max_rhs && d_b != d_x, HLU_ERR_INVALID_ARG,
                "gmres_solve_batch: bad arguments");
    check_gmres_opts(o);
    HLU_REQUIRE(b->factored, HLU_ERR_STATE, "gmres_solve_batch: batch is not factored");
    HLU_REQUIRE(work_bytes >= gmres_batch_workspace_bytes(b, nrhs, o->restart), HLU_ERR_OUT_OF_MEMORY,
                "gmres_solve_batch: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const int32_t P = (int32_t)b->hs.size(), N = b->N_tot;
    GmresSystem sys;
    sys.nseg = P * nrhs;
    sys.total = (int64_t)N * nrhs;
    for (int32_t c = 0; c < nrhs; ++c)
      for (int32_t p = 0; p < P; ++p) {
        sys.off.push_back((int64_t)c * N + b->row_base[p]);
        sys.len.push_back(b->hs[p]->sh->S.N);
      }
    sys.matvec = [&](const double* in, double* out) {
      HIP_OK(spmv_launch(N, b->d_rp, b->d_ci, b->d_val, in, out, nrhs, N, 1.0, 0.0, s));
    };
    sys.precond = [&](const double* in, double* out) { solve_batch(b, in, out, nrhs, s); };
    sys.d_err = b->bufs.ctr + 3;
    gmres_core(sys, d_b, d_x, o, d_work, info, s);
    for (int32_t c = 0; c < sys.nseg; ++c)
      if (!info[c].converged) all_conv = false;
  });
  if (st != HLU_OK) return st;
  if (!all_conv) {
    set_error("gmres_solve_batch: not converged within max_iters");
    return HLU_ERR_NOT_CONVERGED;
  }
  return HLU_OK;
}

void hlu_batch_destroy(hlu_batch b) {
  if (!b) return;
  for (hlu_s* h : b->hs) {
    if (!h) continue;
    h->batch = nullptr;
    h->arena = nullptr;
    h->dims = nullptr;
    h->status = nullptr;
    h->peak = nullptr;
    h->peak_valid = false;
    h->factored = false;
  }
  delete b;
}

}  // extern "C"
