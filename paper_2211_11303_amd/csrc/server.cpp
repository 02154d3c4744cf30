// Serving runtime: solve requests (mesh size n, kappa, right-hand sides) for
// the Kuhn-cube problem, answered by cached H-LU factorisations with
// continuous batching on one GPU.
//
//  * Factor cache: one factorisation per (n, kappa), kept in device memory
//    while it fits the budget; structures and task plans are shared per n
//    (hlu_build_shared), planned once.
//  * Admission by device bytes: a request is started only if its factor
//    (when not cached) and its GMRES work fit the budget next to everything
//    in use; idle cached factors are evicted least recently used first.
//  * Continuous batching: a free worker takes the oldest admissible request
//    and every other queued request for the same factor (up to max_batch_rhs
//    columns), and answers them with one GMRES call; each column keeps its
//    own Krylov process, so a result does not depend on its companions.
//  * Overlap: each worker owns a HIP stream, so the factorisations and
//    solves of different requests run on the device at the same time.
//  * Refinement: columns that a cached factor does not bring to tol within
//    a first budget of iterations get that factor refactored at a smaller
//    eps and are solved again.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "handle.h"
#include "mesh.h"

namespace hlu {
}

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
  int64_t id = 0;
  int32_t n = 0, nrhs = 0;
  double kappa = 0;
  const double* b = nullptr;
  double* x = nullptr;
  hlu_gmres_info* info = nullptr;
  double t_submit = 0, t_start = 0, t_done = 0;
  hlu_status status = HLU_OK;
  bool done = false;
};

// Structure of one mesh size: host plans + sizes for the admission check.
struct Mesh {
  hlu_handle proto = nullptr;
  int32_t N = 0;
  int64_t nnz = 0;
  size_t factor_bytes = 0;   // workspace + solve buffers + values + device CSR
};

// A cached factorisation.
struct Entry {
  int32_t n = 0;
  double kappa = 0;
  hlu_handle h = nullptr;
  hlu_spmat A = nullptr;
  hlu::Owned mem;            // device CSR and workspace
  size_t bytes = 0;
  double eps = 0;            // truncation tolerance of the current factor
  int32_t refines = 0;       // refactorisations at a smaller eps so far
  bool ready = false, busy = false;
  int64_t last_use = 0;
};

}  // namespace

struct hlu_server_s {
  hlu_server_opts o{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::map<int64_t, std::unique_ptr<Request>> reqs;
  std::map<std::pair<int32_t, double>, std::unique_ptr<Entry>> cache;
  std::map<int32_t, Mesh> meshes;
  std::mutex plan_mu;        // serialises planning of new mesh sizes
  int64_t next_id = 1, tick = 0;
  size_t used = 0;
  hlu_server_stats st{};
  bool stop = false;
  std::vector<std::thread> workers;
};

namespace {

using hlu::fail;

size_t gmres_bytes(const hlu_server_s* S, int32_t N, int32_t k) {
  return gmres_workspace_bytes(N, k, S->o.gmres.restart) + 3 * hlu::align256((size_t)N * k * sizeof(double));
}

// Plans mesh n if new (caller holds plan_mu, not mu).
void ensure_mesh(hlu_server_s* S, int32_t n) {
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->meshes.count(n)) return;
  }
  std::vector<int32_t> rp, ci, mid;
  std::vector<double> val;
  int32_t N;
  hlu::kuhn_assemble(n, 1.0, &rp, &ci, &val, &mid, &N);
  hlu_csr csr{N, (int64_t)ci.size(), rp.data(), ci.data(), val.data()};
  Mesh m;
  hlu_status st = hlu_build(&csr, mid.data(), S->o.eta, S->o.leaf, &m.proto);
  if (st != HLU_OK) fail(st, hlu::get_error());
  size_t dev = 0, plans = 0;
  st = hlu_device_bytes(m.proto, &S->o.factor, &dev);   // plans the structure (host)
  if (st == HLU_OK) st = hlu_plan_device_bytes(m.proto, &S->o.factor, &plans);
  if (st != HLU_OK) {
    hlu_destroy(m.proto);
    fail(st, hlu::get_error());
  }
  m.N = N;
  m.nnz = (int64_t)ci.size();
  // a factor's own bytes; the structure's shared plans are counted once per
  // mesh, for as long as the server lives
  m.factor_bytes = dev - plans + (size_t)(N + 1) * 4 + (size_t)m.nnz * 12;
  std::lock_guard<std::mutex> lk(S->mu);
  S->meshes[n] = m;
  S->used += plans;
  S->st.peak_bytes = std::max(S->st.peak_bytes, S->used);
}

// Under mu: drop least recently used idle factors until `need` more bytes fit.
bool make_room(hlu_server_s* S, size_t need, const Entry* keep) {
  while (S->used + need > S->o.hbm_budget) {
    Entry* victim = nullptr;
    for (auto& kv : S->cache) {
      Entry* e = kv.second.get();
      if (e == keep || e->busy || !e->ready) continue;
      if (!victim || e->last_use < victim->last_use) victim = e;
    }
    if (!victim) return false;
    S->used -= victim->bytes;
    if (victim->A) hlu_spmat_destroy(victim->A);
    if (victim->h) hlu_destroy(victim->h);
    S->st.evictions++;
    S->cache.erase({victim->n, victim->kappa});
  }
  return true;
}

struct Job {
  std::vector<Request*> group;
  Entry* e = nullptr;
  size_t gm = 0;
  int32_t cols = 0;
};

// Under mu: the oldest admissible request and its companions.
bool pick(hlu_server_s* S, Job* job) {
  bool any_in_flight = false;
  for (auto& kv : S->cache) any_in_flight = any_in_flight || kv.second->busy;
  for (auto it = S->queue.begin(); it != S->queue.end();) {
    Request* r = *it;
    const auto key = std::make_pair(r->n, r->kappa);
    auto ce = S->cache.find(key);
    Entry* e = ce == S->cache.end() ? nullptr : ce->second.get();
    if (e && e->busy) {
      ++it;
      continue;
    }
    const Mesh& m = S->meshes[r->n];
    // companions: queued requests for the same factor, oldest first
    std::vector<Request*> group{r};
    int32_t cols = r->nrhs;
    for (auto jt = std::next(it); jt != S->queue.end(); ++jt) {
      Request* q = *jt;
      if (q->n == r->n && q->kappa == r->kappa && cols + q->nrhs <= S->o.max_batch_rhs) {
        group.push_back(q);
        cols += q->nrhs;
      }
    }
    const size_t need = gmres_bytes(S, m.N, cols) + (e ? 0 : m.factor_bytes);
    if (!make_room(S, need, e)) {
      if (!any_in_flight && S->cache.empty()) {
        // can never fit: fail it rather than wait forever
        r->status = HLU_ERR_OUT_OF_MEMORY;
        r->done = true;
        r->t_done = now_s();
        S->st.failed++;
        it = S->queue.erase(it);
        S->cv_done.notify_all();
        continue;
      }
      ++it;
      continue;
    }
    if (!e) {
      auto ne = std::make_unique<Entry>();
      ne->n = r->n;
      ne->kappa = r->kappa;
      ne->bytes = m.factor_bytes;
      ne->eps = S->o.factor.eps;
      e = ne.get();
      S->cache[key] = std::move(ne);
    }
    e->busy = true;
    S->used += need;
    S->st.peak_bytes = std::max(S->st.peak_bytes, S->used);
    for (Request* q : group) S->queue.erase(std::find(S->queue.begin(), S->queue.end(), q));
    job->group = std::move(group);
    job->e = e;
    job->gm = gmres_bytes(S, m.N, cols);
    job->cols = cols;
    return true;
  }
  return false;
}

constexpr double kMinRefineEps = 1e-7;   // the truncation's resolution floor

// (Re)factorisation of a built entry at its eps on stream s (outside mu);
// with a rank cap, blocks at the cap are accepted.
void refactor_entry(hlu_server_s* S, Entry* e, hipStream_t s) {
  hlu_factor_opts fo = S->o.factor;
  fo.eps = e->eps;
  hlu_status st = hlu_factor(e->h, &fo, s);
  if (st == HLU_ERR_RANK_OVERFLOW && fo.max_rank > 0) st = HLU_OK;
  if (st != HLU_OK) fail(st, hlu::get_error());
}

bool can_refine(const hlu_server_s* S, const Entry* e) {
  return S->o.refine_iters > 0 && e->refines < S->o.max_refines && e->eps > kMinRefineEps;
}

// Factorisation of entry e on stream s (outside mu).
void factor_entry(hlu_server_s* S, Entry* e, const Mesh& m, hipStream_t s) {
  std::vector<int32_t> rp, ci, mid;
  std::vector<double> val;
  int32_t N;
  hlu::kuhn_assemble(e->n, e->kappa, &rp, &ci, &val, &mid, &N);
  hlu_csr csr{N, (int64_t)ci.size(), rp.data(), ci.data(), val.data()};
  hlu_status st = hlu_build_shared(m.proto, &csr, &e->h);
  if (st != HLU_OK) fail(st, hlu::get_error());
  int32_t* drp = e->mem.keep(hlu::upload(rp));
  int32_t* dci = e->mem.keep(hlu::upload(ci));
  double* dval = e->mem.keep(hlu::upload(val));
  st = hlu_spmat_create(N, (int64_t)ci.size(), drp, dci, dval, &e->A);
  if (st != HLU_OK) fail(st, hlu::get_error());
  size_t ws = 0;
  st = hlu_workspace_bytes(e->h, &S->o.factor, &ws);
  if (st != HLU_OK) fail(st, hlu::get_error());
  void* work = e->mem.keep(hlu::dmalloc<char>(ws));
  st = hlu_bind_workspace(e->h, work, ws);
  if (st != HLU_OK) fail(st, hlu::get_error());
  refactor_entry(S, e, s);
}

// Device buffers of one worker's GMRES calls, grown on demand and kept (a
// free would synchronise the device and stall the other workers).
struct WorkerBufs {
  std::unique_ptr<hlu::Owned> mem;
  double* db = nullptr;
  double* dx = nullptr;
  double* dt = nullptr;   // results of the columns solved again after a refinement
  void* work = nullptr;
  size_t vec_elems = 0, work_bytes = 0;
  void reserve(size_t elems, size_t wb) {
    if (mem && elems <= vec_elems && wb <= work_bytes) return;
    mem.reset();
    mem = std::make_unique<hlu::Owned>();
    vec_elems = std::max(elems, vec_elems);
    work_bytes = std::max(wb, work_bytes);
    db = mem->keep(hlu::dmalloc<double>(vec_elems));
    dx = mem->keep(hlu::dmalloc<double>(vec_elems));
    dt = mem->keep(hlu::dmalloc<double>(vec_elems));
    work = mem->keep(hlu::dmalloc<char>(work_bytes));
  }
};

void run_job(hlu_server_s* S, Job& job, hipStream_t s, WorkerBufs& wb) {
  Entry* e = job.e;
  const double t0 = now_s();
  for (Request* r : job.group) r->t_start = t0;
  hlu_status status = HLU_OK;
  std::vector<hlu_gmres_info> info(job.cols);
  const Mesh* m;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    m = &S->meshes[e->n];
  }
  const int32_t N = m->N;
  bool factored_now = false;
  int64_t refined = 0;
  status = hlu::guard([&] {
    if (!e->ready) {
      factor_entry(S, e, *m, s);
      factored_now = true;
    }
    const size_t wbytes = gmres_workspace_bytes(N, job.cols, S->o.gmres.restart);
    wb.reserve((size_t)N * job.cols, wbytes);
    double* db = wb.db;
    double* dx = wb.dx;
    int32_t c = 0;
    for (Request* r : job.group) {
      HIP_OK(hipMemcpyAsync(db + (size_t)c * N, r->b, (size_t)N * r->nrhs * sizeof(double), hipMemcpyHostToDevice,
                            s));
      c += r->nrhs;
    }
    // first try: a limited budget if the factor can still be refined
    hlu_gmres_opts go = S->o.gmres;
    bool capped = can_refine(S, e) && S->o.refine_iters < go.max_iters;
    if (capped) go.max_iters = S->o.refine_iters;
    hlu_status g = gmres_solve(e->A, db, dx, job.cols, N, e->h, &go, info.data(), wb.work, wbytes, s);
    if (g != HLU_OK && g != HLU_ERR_NOT_CONVERGED) fail(g, hlu::get_error());
    // columns that missed tol: refactor at a smaller eps (or, when that is
    // no longer allowed, lift the iteration cap) and solve them again
    while (g == HLU_ERR_NOT_CONVERGED) {
      std::vector<int32_t> open;
      for (int32_t k = 0; k < job.cols; ++k)
        if (!info[k].converged) open.push_back(k);
      if (open.empty()) break;
      if (can_refine(S, e)) {
        e->eps = std::max(e->eps * S->o.refine_eps_factor, kMinRefineEps);
        e->refines++;
        refactor_entry(S, e, s);
        refined++;
      } else if (!capped) {
        break;
      }
      go = S->o.gmres;
      capped = can_refine(S, e) && S->o.refine_iters < go.max_iters;
      if (capped) go.max_iters = S->o.refine_iters;
      // right-hand sides of the open columns, packed, from the requests
      std::vector<const double*> src;
      for (Request* r : job.group)
        for (int32_t k = 0; k < r->nrhs; ++k) src.push_back(r->b + (size_t)k * N);
      const int32_t no = (int32_t)open.size();
      for (int32_t i = 0; i < no; ++i)
        HIP_OK(hipMemcpyAsync(db + (size_t)i * N, src[open[i]], (size_t)N * sizeof(double), hipMemcpyHostToDevice,
                              s));
      std::vector<hlu_gmres_info> io(no);
      const size_t wbo = gmres_workspace_bytes(N, no, go.restart);
      g = gmres_solve(e->A, db, wb.dt, no, N, e->h, &go, io.data(), wb.work, wbo, s);
      if (g != HLU_OK && g != HLU_ERR_NOT_CONVERGED) fail(g, hlu::get_error());
      for (int32_t i = 0; i < no; ++i) {
        HIP_OK(hipMemcpyAsync(dx + (size_t)open[i] * N, wb.dt + (size_t)i * N, (size_t)N * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
        info[open[i]] = io[i];
      }
    }
    c = 0;
    for (Request* r : job.group) {
      HIP_OK(hipMemcpyAsync(r->x, dx + (size_t)c * N, (size_t)N * r->nrhs * sizeof(double), hipMemcpyDeviceToHost,
                            s));
      c += r->nrhs;
    }
    HIP_OK(hipStreamSynchronize(s));
  });
  std::lock_guard<std::mutex> lk(S->mu);
  S->used -= job.gm;
  e->busy = false;
  e->last_use = ++S->tick;
  if (factored_now) S->st.factorizations++;
  else S->st.cache_hits++;
  S->st.refinements += refined;
  S->st.gmres_calls++;
  if (job.group.size() > 1) S->st.coalesced_requests += (int64_t)job.group.size();
  if (status != HLU_OK) {
    // drop a factor that failed to build
    if (!e->ready) {
      S->used -= e->bytes;
      if (e->A) hlu_spmat_destroy(e->A);
      if (e->h) hlu_destroy(e->h);
      S->cache.erase({e->n, e->kappa});
    }
  } else {
    e->ready = true;
  }
  const double t1 = now_s();
  int32_t c = 0;
  for (Request* r : job.group) {
    bool conv = true;
    for (int32_t k = 0; k < r->nrhs; ++k) {
      if (status == HLU_OK) {
        r->info[k] = info[c + k];
        conv = conv && info[c + k].converged;
      }
    }
    c += r->nrhs;
    r->status = status != HLU_OK ? status : (conv ? HLU_OK : HLU_ERR_NOT_CONVERGED);
    r->t_done = t1;
    r->done = true;
    if (r->status == HLU_OK) S->st.completed++;
    else S->st.failed++;
  }
  S->st.bytes_in_use = S->used;
  S->cv_done.notify_all();
  S->cv_work.notify_all();
}

void worker_main(hlu_server_s* S) {
  (void)hipSetDevice(S->device);
  // non-blocking: the library's synchronous copies on the null stream do not
  // wait for the other workers' kernels (default priority)
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
  WorkerBufs wb;
  while (true) {
    Job job;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop || pick(S, &job); });
      if (job.group.empty()) {
        if (S->stop) break;
        continue;
      }
    }
    run_job(S, job, s, wb);
  }
  (void)hipStreamSynchronize(s);
  (void)hipStreamDestroy(s);
}

}  // namespace

using namespace hlu;

extern "C" {

hlu_status hlu_server_create(const hlu_server_opts* o, hlu_server* out) {
  return guard([&] {
    HLU_REQUIRE(o && out, HLU_ERR_INVALID_ARG, "hlu_server_create: NULL argument");
    HLU_REQUIRE(o->workers >= 1 && o->workers <= 16, HLU_ERR_INVALID_ARG, "hlu_server_create: need 1..16 workers");
    HLU_REQUIRE(o->max_batch_rhs >= 1 && o->max_batch_rhs <= kMaxRhs, HLU_ERR_INVALID_ARG,
                "hlu_server_create: need 1 <= max_batch_rhs <= 32");
    HLU_REQUIRE(o->hbm_budget > 0, HLU_ERR_INVALID_ARG, "hlu_server_create: need a device budget");
    HLU_REQUIRE(o->leaf >= 1 && o->leaf <= 128 && o->eta > 0, HLU_ERR_INVALID_ARG, "hlu_server_create: bad leaf/eta");
    check_opts(&o->factor);
    HLU_REQUIRE(o->gmres.restart >= 1 && o->gmres.max_iters >= 1 && o->gmres.tol > 0, HLU_ERR_INVALID_ARG,
                "hlu_server_create: bad GMRES options");
    HLU_REQUIRE(o->refine_iters >= 0 && (o->refine_iters == 0 || (o->max_refines >= 0 && o->refine_eps_factor > 0 &&
                                                                   o->refine_eps_factor < 1)),
                HLU_ERR_INVALID_ARG, "hlu_server_create: bad refinement options");
    auto S = std::make_unique<hlu_server_s>();
    S->o = *o;
    HIP_OK(hipGetDevice(&S->device));
    for (int i = 0; i < o->workers; ++i) S->workers.emplace_back(worker_main, S.get());
    *out = S.release();
  });
}

hlu_status hlu_server_prepare(hlu_server S, int32_t n) {
  return guard([&] {
    HLU_REQUIRE(S && n >= 1 && n <= 128, HLU_ERR_INVALID_ARG, "hlu_server_prepare: bad arguments");
    std::lock_guard<std::mutex> lk(S->plan_mu);
    ensure_mesh(S, n);
  });
}

hlu_status hlu_server_submit(hlu_server S, int32_t n, double kappa, int32_t nrhs, const double* b, double* x,
                             hlu_gmres_info* info, int64_t* ticket) {
  return guard([&] {
    HLU_REQUIRE(S && b && x && info && ticket && n >= 1 && n <= 128 && std::isfinite(kappa), HLU_ERR_INVALID_ARG,
                "hlu_server_submit: bad arguments");
    HLU_REQUIRE(nrhs >= 1 && nrhs <= S->o.max_batch_rhs, HLU_ERR_INVALID_ARG,
                "hlu_server_submit: need 1 <= nrhs <= max_batch_rhs");
    {
      std::lock_guard<std::mutex> lk(S->plan_mu);
      ensure_mesh(S, n);
    }
    auto r = std::make_unique<Request>();
    r->n = n;
    r->kappa = kappa;
    r->nrhs = nrhs;
    r->b = b;
    r->x = x;
    r->info = info;
    r->t_submit = now_s();
    std::lock_guard<std::mutex> lk(S->mu);
    HLU_REQUIRE(!S->stop, HLU_ERR_STATE, "hlu_server_submit: server is shutting down");
    r->id = S->next_id++;
    *ticket = r->id;
    S->queue.push_back(r.get());
    S->reqs[r->id] = std::move(r);
    S->st.submitted++;
    S->cv_work.notify_all();
  });
}

hlu_status hlu_server_wait(hlu_server S, int64_t ticket, double timeout_s, double* queued_s, double* latency_s) {
  hlu_status result = HLU_OK;
  hlu_status st = guard([&] {
    HLU_REQUIRE(S, HLU_ERR_INVALID_ARG, "hlu_server_wait: NULL server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    HLU_REQUIRE(it != S->reqs.end(), HLU_ERR_INVALID_ARG, "hlu_server_wait: unknown ticket");
    Request* r = it->second.get();
    auto ready = [&] { return r->done; };
    if (timeout_s < 0) {
      S->cv_done.wait(lk, ready);
    } else if (!S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
      fail(HLU_ERR_STATE, "hlu_server_wait: timed out");
    }
    if (queued_s) *queued_s = r->t_start > 0 ? r->t_start - r->t_submit : r->t_done - r->t_submit;
    if (latency_s) *latency_s = r->t_done - r->t_submit;
    result = r->status;
    S->reqs.erase(it);
  });
  if (st != HLU_OK) return st;
  if (result != HLU_OK) set_error("hlu_server_wait: the request failed or did not converge");
  return result;
}

hlu_status hlu_server_get_stats(hlu_server S, hlu_server_stats* out) {
  return guard([&] {
    HLU_REQUIRE(S && out, HLU_ERR_INVALID_ARG, "hlu_server_get_stats: NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    out->bytes_in_use = S->used;
    out->cached_factors = (int32_t)S->cache.size();
  });
}

void hlu_server_destroy(hlu_server S) {
  if (!S) return;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    // drain: every queued request is answered before the workers stop
    S->cv_done.wait(lk, [&] { return S->queue.empty() && std::none_of(S->cache.begin(), S->cache.end(),
                                                                     [](auto& kv) { return kv.second->busy; }); });
    S->stop = true;
    S->cv_work.notify_all();
  }
  for (std::thread& t : S->workers) t.join();
  for (auto& kv : S->cache) {
    if (kv.second->A) hlu_spmat_destroy(kv.second->A);
    if (kv.second->h) hlu_destroy(kv.second->h);
  }
  for (auto& kv : S->meshes) hlu_destroy(kv.second.proto);
  delete S;
}

}  // extern "C"
