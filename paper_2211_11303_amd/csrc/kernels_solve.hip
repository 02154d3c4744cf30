// Persistent H-triangular solve (Algorithm 1, step III) for gfx950.
//
// One launch runs both sweeps.  Workgroups claim tasks in the schedule's
// order through an atomic counter; a task waits (bounded spin) on the
// completion flags of the tasks it reads, which always come earlier in the
// order, so every claimed task can finish.  Results passed between tasks
// (solution rows, T products) are stored and loaded with agent-scope
// coherent accesses and flags are set after the stores complete, so no
// L2 writeback or invalidation (one L2 per XCD) sits on the critical path.
// Factors are read in their storage type T; arithmetic and vectors are FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "solve_sched.h"

namespace hlu {
namespace dev {

typedef double double4_t __attribute__((ext_vector_type(4)));
constexpr int kRecTilesPerWave = 4;   // neighbour record: (128 / 16) row tiles x 2 column tiles / 4 wavefronts
constexpr int kSolTilesPerWave = 2;   // solution rows: (64 / 16) row tiles x 2 column tiles / 4 wavefronts

constexpr int kSolveThreads = 256;
constexpr int kMaxRhsTile = 8;          // columns per register tile of the triangular solve
// debug trace per task: claim, solve start, end, workgroup, low-rank done,
// triangle done, product done, flags stored, batched low-rank started,
// batched low-rank done, neighbour record published (fused form), (unused)
constexpr int kTraceFields = 12;

struct SolveArgs {
  const STask* tasks;
  const SLeaf* leaves;
  const SDense* dense;
  const SLow* low;
  const STprod* tprod;
  const int32_t* dims;
  double* y;            // N x nrhs, cluster order, leading dimension N
  double* tbuf;         // T products
  int32_t* leaf_flag;   // 2L flags
  int32_t* tp_flag;     // one per T-product
  int32_t* ctr;         // [0] claim counter, [1] finished forward tasks, [2] error of this
                        // launch, [3] error of any launch since the host last read it,
                        // [4] workgroups that have left the task loop
  const int32_t* push0; // push task -> first record in push_recs
  const int32_t* push_recs;
  const int32_t* leaf_tq; // T-product chunks computed by leaf tasks
  const int32_t* tg0;     // T-product task -> first T-product in tg_list
  const int32_t* tg_list;
  double* pbuf;         // partial-sum records, pstride doubles each (m x nrhs, ld m)
  int32_t* pflag;       // one per record
  int64_t pstride;
  int64_t* trace;       // optional (debug): kTraceFields clocks per task
  int64_t wait_ticks;   // longest wait, in wall-clock ticks, before the launch gives up
  int32_t ntasks, n_fwd, N, nrhs, max_rhs, L, epoch;
  int32_t cur_task;     // set per task (trace only)
};

__device__ __forceinline__ void stamp(const SolveArgs& a, int field) {
  if (a.trace && threadIdx.x == 0) a.trace[kTraceFields * a.cur_task + field] = (int64_t)wall_clock64();
}

// Data exchanged between tasks (y, T products) is written and read with
// agent-scope relaxed atomics: such accesses go to the device coherence
// point, so no cache writeback/invalidation is needed between tasks.
__device__ __forceinline__ double cload(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void cstore(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t load_relaxed(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Spin (relaxed loads, no cache maintenance) until *f == want, for at most
// `ticks` of the constant-rate wall clock; returns false on timeout (and
// sets the launch's error word) or if another task already reported one.
// After an error every wait returns at once, so the launch drains.
__device__ bool spin_eq(const int32_t* f, int32_t want, int32_t* err, int64_t ticks) {
  if (load_relaxed(f) == want) return true;
  const int64_t t0 = (int64_t)wall_clock64();
  while (load_relaxed(f) != want) {
    if (load_relaxed(err) != 0) return false;
    __builtin_amdgcn_s_sleep(2);
    if ((int64_t)wall_clock64() - t0 > ticks) {
      __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
  }
  return true;
}

// After flags were observed by some threads: order the workgroup's later
// (coherent) loads after the flag loads.
__device__ void acquire_all() {
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// All threads: wait for flags[lf0..lf1) == epoch, then acquire.
__device__ void wait_leaves(const SolveArgs& a, int base, int lf0, int lf1) {
  for (int f = lf0 + (int)threadIdx.x; f < lf1; f += blockDim.x)
    spin_eq(a.leaf_flag + base + f, a.epoch, a.ctr + 2, a.wait_ticks);
  acquire_all();
}

__device__ void wait_one(const SolveArgs& a, const int32_t* f, int32_t want) {
  if (threadIdx.x == 0) spin_eq(f, want, a.ctr + 2, a.wait_ticks);
  acquire_all();
}

// Publish this task's results: every wave completes its coherent stores
// (workgroup release = wait for outstanding stores), then the flag.
__device__ void publish(int32_t* f, int32_t epoch) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_s_waitcnt(0);
    __hip_atomic_store(f, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__device__ __forceinline__ double bcast(double v, int lane) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// acc (m x nrhs, LDS, row-major with stride ldacc) := tri^{-1} acc with the
// precomputed inverse I of the diagonal leaf's triangle (m x m, column-major):
// forward, the strictly lower part of L^{-1} with its unit diagonal;
// backward, U^{-1} (on and above the diagonal).  A dense product over all
// threads instead of m dependent substitution steps.
template <class P>
__device__ void apply_inverse(const P* I, int m, bool forward, double* acc, int ldacc, int nrhs) {
  constexpr int kPer = 16;
  double out[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int o = threadIdx.x + q * 256;
    out[q] = 0.0;
    if (o < m * nrhs) {
      const int i = o % m, c = o / m;
      double sum = 0.0;
      if (forward) {
        sum = acc[i * ldacc + c];
#pragma unroll 8
        for (int k = 0; k < i; ++k) sum += double(I[i + k * m]) * acc[k * ldacc + c];
      } else {
#pragma unroll 8
        for (int k = i; k < m; ++k) sum += double(I[i + k * m]) * acc[k * ldacc + c];
      }
      out[q] = sum;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int o = threadIdx.x + q * 256;
    if (o < m * nrhs) acc[(o % m) * ldacc + o / m] = out[q];
  }
  __syncthreads();
}

// Staging buffers of a workgroup (LDS): A chunk (max_m x kKC doubles) and
// B chunk (kKC x max_rhs doubles).
constexpr int kKC = 64;

// r[(i, c)] -= sum_k A[i, k] B[k, c] with A (m x K, type T, A[i + k*lda]) and
// B (K x nrhs, FP64, B[k*bs + c*bcs]); both streamed through LDS in chunks of
// kKC so that all loads of a chunk are in flight together.
template <class T, bool kBInLds = false>
__device__ void mm_sub(const T* A, int64_t lda, const double* B, int64_t bs, int64_t bcs, int m, int K,
                       int nrhs, double* r, double* As, double* Bs) {
  for (int k0 = 0; k0 < K; k0 += kKC) {
    const int kc = min(kKC, K - k0);
    for (int e = threadIdx.x; e < m * kc; e += blockDim.x) {
      const int i = e % m, k = e / m;
      As[k * 128 + i] = double(A[i + (int64_t)(k0 + k) * lda]);
    }
    for (int e = threadIdx.x; e < kc * nrhs; e += blockDim.x) {
      const int k = e % kc, c = e / kc;
      const double* bp = B + (int64_t)(k0 + k) * bs + (int64_t)c * bcs;
      Bs[c * kKC + k] = kBInLds ? *bp : cload(bp);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int o = threadIdx.x + q * kSolveThreads;
      if (o < m * nrhs) {
        const int i = o % m, c = o / m;
        double sum = 0.0;
#pragma unroll 8
        for (int k = 0; k < kc; ++k) sum += As[k * 128 + i] * Bs[c * kKC + k];
        r[q] -= sum;
      }
    }
    __syncthreads();
  }
}

template <class T>
__device__ void dense_contrib(const SolveArgs& a, const T* arena, const SDense& D, int m, int nrhs, double* r,
                              double* As, double* Bs) {
  mm_sub<T>(arena + D.off, D.ld, a.y + D.col0, 1, a.N, m, D.ncols, nrhs, r, As, Bs);
}

// r -= X_b[rows of this leaf] T_b with T_b the sum of the block's chunk
// products (summed into the LDS area Ts first when there are several).
template <class T>
__device__ void low_contrib(const SolveArgs& a, const T* arena, const SLow& Lw, int m, int nrhs, double* r,
                            double* As, double* Bs, double* Ts) {
  const STprod tp = a.tprod[Lw.tp];
  const int k = a.dims[tp.slot];
  if (Lw.ntp == 1) {
    const double* Tb = a.tbuf + tp.toff * a.max_rhs;
    mm_sub<T>(arena + Lw.xoff, Lw.ldx, Tb, 1, tp.cap, m, k, nrhs, r, As, Bs);
    return;
  }
  for (int e = threadIdx.x; e < k * nrhs; e += blockDim.x) {
    const int kk = e % k, c = e / k;
    double sum = 0.0;
    for (int q = 0; q < Lw.ntp; ++q) sum += cload(a.tbuf + a.tprod[Lw.tp + q].toff * a.max_rhs + kk + c * tp.cap);
    Ts[kk + c * k] = sum;
  }
  __syncthreads();
  mm_sub<T, true>(arena + Lw.xoff, Lw.ldx, Ts, 1, k, m, k, nrhs, r, As, Bs);
}

// r -= sum over the low-rank contributions t < 256 (of at most kMaxChunks
// chunks) of this leaf of X_t T_t, as one product of the concatenated matrices
// [X_1 .. X_G] [T_1; ..; T_G]: every column kk of every X_t is a "virtual
// column", in schedule order.  Virtual columns go through LDS in fixed
// windows of 64 (so the summation order depends on the ranks only, not on
// timing); before a window the task waits for the T products it reads.
// Each thread issues all of a window's loads before writing LDS, so a
// window costs one memory round trip instead of one per contribution.
// scr: LDS scratch of at least 2816 doubles, free during the call.
constexpr int kVCols = 1024;   // virtual columns per table window
constexpr int kMaxChunks = 4;  // contributions with more chunks go one by one
// Returns true if some contribution was left for the caller (more than 256,
// or more than kMaxChunks chunks).
template <class T>
__device__ bool low_batched(const SolveArgs& a, const T* arena, const SLeaf& lf, int m, int nrhs, double* r,
                            double* As, double* Bs, double* scr) {
  constexpr int kPer = 16;
  int* kpre = reinterpret_cast<int*>(scr);                   // [257] column offsets of the contributions
  int64_t* colX = reinterpret_cast<int64_t*>(scr + 256);     // [kVCols] arena index of X column
  int64_t* colT = reinterpret_cast<int64_t*>(scr + 1280);    // [kVCols] tbuf index of T row
  int* colC = reinterpret_cast<int*>(scr + 2304);            // [kVCols] T column stride
  const int nl = min(lf.nl, 256);
  const int t0 = threadIdx.x;
  int k1 = 0, kt = 0;   // rank; virtual columns (rank x chunks)
  SLow Lw{};
  STprod tp{};
  if (t0 < nl) {
    Lw = a.low[lf.l0 + t0];
    if (Lw.ntp <= kMaxChunks) {
      tp = a.tprod[Lw.tp];
      k1 = a.dims[tp.slot];
      kt = k1 * Lw.ntp;
    }
  }
  kpre[t0 + 1] = kt;
  if (t0 == 0) kpre[0] = 0;
  const bool left = __syncthreads_or(t0 < nl && Lw.ntp > kMaxChunks) || lf.nl > 256;
  for (int d = 1; d < 256; d <<= 1) {   // inclusive scan of 256 entries
    const int v = t0 >= d ? kpre[t0 + 1 - d] : 0;
    __syncthreads();
    kpre[t0 + 1] += v;
    __syncthreads();
  }
  const int vtot = kpre[256];
  const int my0 = kpre[t0], my1 = kpre[t0 + 1];
  for (int w0 = 0; w0 < vtot; w0 += kVCols) {
    // table of this window's virtual columns, written by their contributions
    // (chunk q of a contribution repeats its X columns against T chunk q)
    for (int q = 0; q < Lw.ntp && kt > 0; ++q) {
      const int64_t tb = (q == 0 ? tp.toff : a.tprod[Lw.tp + q].toff) * a.max_rhs;
      for (int kk = 0; kk < k1; ++kk) {
        const int v = my0 + q * k1 + kk - w0;
        if (v >= 0 && v < kVCols) {
          colX[v] = Lw.xoff + (int64_t)kk * Lw.ldx;
          colT[v] = tb + kk;
          colC[v] = tp.cap;
        }
      }
    }
    __syncthreads();
    const int wn = min(kVCols, vtot - w0);
    for (int v0 = 0; v0 < wn; v0 += kKC) {
      const int vc = min(kKC, wn - v0);
      // the T products of the contributions overlapping these columns
      if (kt > 0 && my0 < w0 + v0 + vc && my1 > w0 + v0)
        for (int q = 0; q < Lw.ntp; ++q) spin_eq(a.tp_flag + Lw.tp + q, a.epoch, a.ctr + 2, a.wait_ticks);
      acquire_all();
      // T rows and the first X pass are loaded together, then written
      double tr[8];
      int td[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = threadIdx.x + u * kSolveThreads;
        td[u] = -1;
        tr[u] = 0.0;
        if (e < vc * nrhs) {
          const int vv = e % vc, c = e / vc;
          tr[u] = cload(a.tbuf + colT[v0 + vv] + (int64_t)c * colC[v0 + vv]);
          td[u] = c * kKC + vv;
        }
      }
      for (int b0 = 0; b0 < m * vc; b0 += 16 * kSolveThreads) {
        double xr[16];
        int xd[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int e = b0 + threadIdx.x + u * kSolveThreads;
          xd[u] = -1;
          xr[u] = 0.0;
          if (e < m * vc) {
            const int i = e % m, vv = e / m;
            xr[u] = double(arena[colX[v0 + vv] + i]);
            xd[u] = vv * 128 + i;
          }
        }
        if (b0 == 0) {
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (td[u] >= 0) Bs[td[u]] = tr[u];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (xd[u] >= 0) As[xd[u]] = xr[u];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int o = threadIdx.x + q * kSolveThreads;
        if (o < m * nrhs) {
          const int i = o % m, c = o / m;
          double sum = 0.0;
#pragma unroll 8
          for (int vv = 0; vv < vc; ++vv) sum += As[vv * 128 + i] * Bs[c * kKC + vv];
          r[q] -= sum;
        }
      }
      __syncthreads();
    }
  }
  return left;
}


template <class T>
__device__ void run_leaf(const SolveArgs& a, const T* arena, const T* inv, const T* nm, int s, bool forward,
                         double* acc, double* As, double* Bs, double* Dg) {
  const SLeaf lf = a.leaves[s];
  const int m = lf.m, nrhs = a.nrhs;
  const int ldacc = a.max_rhs;
  const int flag_base = forward ? 0 : a.L;
  if (!forward) {
    // the backward sweep overwrites y in place: wait for every forward task
    wait_one(a, a.ctr + 1, a.n_fwd);
  }
  // outputs (i, c) owned by fixed threads; partial sums in registers
  constexpr int kPer = 16;   // m * nrhs <= 128 * 32 = 16 * 256
  double r[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int o = threadIdx.x + q * kSolveThreads;
    r[q] = (o < m * nrhs) ? cload(a.y + lf.row0 + (o % m) + (int64_t)(o / m) * a.N) : 0.0;
  }
  // low-rank contributions in schedule order (sorted by when their T
  // products complete): the first 256 together, then the others one by one (acc is free until the dense records are
  // summed; the LDS area of the diagonal inverses until they are staged)
  const int nl = lf.nl;
  stamp(a, 8);
  const bool rest = low_batched<T>(a, arena, lf, m, nrhs, r, As, Bs, acc);
  stamp(a, 9);
  for (int t = rest ? 0 : nl; t < nl; ++t) {
    const SLow Lw = a.low[lf.l0 + t];
    if (t < 256 && Lw.ntp <= kMaxChunks) continue;
    for (int q = 0; q < Lw.ntp; ++q) wait_one(a, a.tp_flag + Lw.tp + q, a.epoch);
    low_contrib<T>(a, arena, Lw, m, nrhs, r, As, Bs, Dg);
  }
  stamp(a, 4);
  // stage factor data of the critical section before waiting on the
  // preceding leaf: the triangle inverses of the diagonal leaf and the
  // neighbouring row's block multiplied after the solve
  const bool diag_lds = m * m <= 64 * 64;
  if (diag_lds) {
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) Dg[e] = double(inv[lf.inv + e]);
  }
  SDense Dn{};
  const bool next_lds = lf.next_rec >= 0 && a.dense[lf.next_rec].m <= 128 && a.dense[lf.next_rec].ncols <= kKC;
  if (lf.next_rec >= 0) Dn = a.dense[lf.next_rec];
  const bool fused = lf.nm >= 0;   // record formed from r with (D Inv), see below
  const int rec_rows = lf.nm_rows;   // rows of the neighbour record(s) in the fused form
  if (fused) {
    for (int e = threadIdx.x; e < rec_rows * m; e += blockDim.x) {
      const int i = e % rec_rows, k = e / rec_rows;
      As[k * 128 + i] = double(nm[lf.nm + e]);
    }
  } else if (next_lds) {
    for (int e = threadIdx.x; e < Dn.m * Dn.ncols; e += blockDim.x) {
      const int i = e % Dn.m, k = e / Dn.m;
      As[k * 128 + i] = double(arena[Dn.off + i + (int64_t)k * Dn.ld]);
    }
  }
  __syncthreads();
  // dense contributions: the partial-sum records of this row in record
  // order, except the one the preceding leaf task forms, which comes last
  for (int t = threadIdx.x; t < lf.nd; t += blockDim.x)
    if (lf.d0 + t != lf.prev_rec) spin_eq(a.pflag + lf.d0 + t, a.epoch, a.ctr + 2, a.wait_ticks);
  acquire_all();
  for (int t0 = 0; t0 < lf.nd; t0 += 4) {
    // four records' loads in flight together
    double v[4][kPer];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int rec = lf.d0 + t0 + u;
      const double* P = a.pbuf + (int64_t)rec * a.pstride;
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int o = threadIdx.x + q * kSolveThreads;
        v[u][q] = (t0 + u < lf.nd && rec != lf.prev_rec && o < m * nrhs) ? cload(P + o) : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < kPer; ++q) r[q] -= v[u][q];
  }
  if (lf.prev_rec >= 0) {
    wait_one(a, a.pflag + lf.prev_rec, a.epoch);
    const double* P = a.pbuf + (int64_t)lf.prev_rec * a.pstride;
    double v[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int o = threadIdx.x + q * kSolveThreads;
      v[q] = o < m * nrhs ? cload(P + o) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) r[q] -= v[q];
  }
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int o = threadIdx.x + q * kSolveThreads;
    if (o < m * nrhs) acc[(o % m) * ldacc + o / m] = r[q];
  }
  stamp(a, 1);
  __syncthreads();
  if (fused) {
    // the neighbour record P = (D Inv) r_j (with the second neighbour's
    // record stacked below it) first, then y_j = Inv r_j, both on
    // the FP64 matrix cores (16 x 16 x 4 tiles; columns in 16-column tiles,
    // tiles dealt round robin to the wavefronts).  P is stored and its flag
    // set before y_j is formed: the next leaf task waits for P only, so the
    // solution rows, their stores and the T-product chunks of this task
    // overlap with the next task.
    // Operand lanes: A[i][k] at lane i + 16k, B[k][j] at lane j + 16k;
    // result register r of lane l is D[l/16 + 4r][l%16].
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ct_n = (nrhs + 15) >> 4, ks_n = (m + 3) >> 2;
    // tile t = wave + 4 it: with ct_n in {1, 2} all of a wavefront's tiles
    // share one column tile, so one B operand feeds all its MFMAs per step
    const int ct = wave % ct_n;
    const int j = 16 * ct + (lane & 15), kl = lane >> 4;
    const int col = 16 * ct + (lane & 15);
    {
      const int ntiles = ((rec_rows + 15) >> 4) * ct_n;
      double4_t dacc[kRecTilesPerWave];
#pragma unroll
      for (int it = 0; it < kRecTilesPerWave; ++it) dacc[it] = double4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
      for (int ks = 0; ks < ks_n; ++ks) {
        const int k = 4 * ks + kl;
        const double bv = (k < m && j < nrhs) ? acc[k * ldacc + j] : 0.0;
#pragma unroll
        for (int it = 0; it < kRecTilesPerWave; ++it) {
          const int t = wave + 4 * it;   // uniform within the wavefront
          if (t < ntiles) {
            const int i = 16 * (t / ct_n) + (lane & 15);
            const double av = (k < m && i < rec_rows) ? As[k * 128 + i] : 0.0;
            dacc[it] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, dacc[it], 0, 0, 0);
          }
        }
      }
      // rows [0, Dn.m): the next leaf's record; the rest: the second
      // neighbour's record
      double* P = a.pbuf + (int64_t)lf.next_rec * a.pstride;
      double* P2 = lf.next_rec2 >= 0 ? a.pbuf + (int64_t)lf.next_rec2 * a.pstride : nullptr;
      const int dm2 = rec_rows - Dn.m;
#pragma unroll
      for (int it = 0; it < kRecTilesPerWave; ++it) {
        const int t = wave + 4 * it;
        if (t < ntiles) {
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int row = 16 * (t / ct_n) + (lane >> 4) + 4 * rr;
            if (col < nrhs && row < Dn.m) cstore(P + row + col * Dn.m, dacc[it][rr]);
            else if (col < nrhs && row < rec_rows) cstore(P2 + (row - Dn.m) + col * dm2, dacc[it][rr]);
          }
        }
      }
      // every wave's record stores complete, then the records' flags
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __syncthreads();
      if (threadIdx.x == 0) {
        __builtin_amdgcn_s_waitcnt(0);
        __hip_atomic_store(a.pflag + lf.next_rec, a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (lf.next_rec2 >= 0)
          __hip_atomic_store(a.pflag + lf.next_rec2, a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    stamp(a, 10);
    {
      const int ntiles = ((m + 15) >> 4) * ct_n;
      double4_t dacc[kSolTilesPerWave];
#pragma unroll
      for (int it = 0; it < kSolTilesPerWave; ++it) dacc[it] = double4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
      for (int ks = 0; ks < ks_n; ++ks) {
        const int k = 4 * ks + kl;
        const double bv = (k < m && j < nrhs) ? acc[k * ldacc + j] : 0.0;
#pragma unroll
        for (int it = 0; it < kSolTilesPerWave; ++it) {
          const int t = wave + 4 * it;
          if (t < ntiles) {
            const int i = 16 * (t / ct_n) + (lane & 15);
            double av = 0.0;
            if (k < m && i < m)
              av = forward ? (i > k ? Dg[i + k * m] : (i == k ? 1.0 : 0.0)) : (i <= k ? Dg[i + k * m] : 0.0);
            dacc[it] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, dacc[it], 0, 0, 0);
          }
        }
      }
      __syncthreads();   // every wave has read r_j from acc
#pragma unroll
      for (int it = 0; it < kSolTilesPerWave; ++it) {
        const int t = wave + 4 * it;
        if (t < ntiles) {
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int row = 16 * (t / ct_n) + (lane >> 4) + 4 * rr;
            const double v = dacc[it][rr];
            if (col < nrhs && row < m) {
              acc[row * ldacc + col] = v;
              cstore(a.y + lf.row0 + row + (int64_t)col * a.N, v);
            }
          }
        }
      }
    }
    __syncthreads();
    stamp(a, 5);
  } else {
    if (diag_lds) apply_inverse<double>(Dg, m, forward, acc, ldacc, nrhs);
    else apply_inverse<T>(inv + lf.inv, m, forward, acc, ldacc, nrhs);
    stamp(a, 5);
    for (int o = threadIdx.x; o < m * nrhs; o += blockDim.x)
      cstore(a.y + lf.row0 + (o % m) + (int64_t)(o / m) * a.N, acc[(o % m) * ldacc + o / m]);
  }
  if (lf.next_rec >= 0 && !fused) {
    // the neighbouring row's dense block times this solution row (both in LDS)
    const SDense& D = Dn;
    double pr[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) pr[q] = 0.0;
    if (next_lds) {
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int o = threadIdx.x + q * kSolveThreads;
        if (o < D.m * nrhs) {
          const int i = o % D.m, c = o / D.m;
          double sum = 0.0;
#pragma unroll 8
          for (int k = 0; k < D.ncols; ++k) sum += As[k * 128 + i] * acc[k * ldacc + c];
          pr[q] = sum;
        }
      }
    } else {
      mm_sub<T, true>(arena + D.off, D.ld, acc, ldacc, 1, D.m, D.ncols, nrhs, pr, As, Bs);
#pragma unroll
      for (int q = 0; q < kPer; ++q) pr[q] = -pr[q];
    }
    double* P = a.pbuf + (int64_t)lf.next_rec * a.pstride;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int o = threadIdx.x + q * kSolveThreads;
      if (o < D.m * nrhs) cstore(P + o, pr[q]);
    }
  }
  // T-product chunks of exactly this leaf's rows that the next leaf needs:
  // T = Y[rows of this leaf]^T y_j, Y staged in the (now free) inverse area
  for (int q = 0; q < lf.ntq; ++q) {
    const STprod tp = a.tprod[a.leaf_tq[lf.tq0 + q]];
    const int k = a.dims[tp.slot];
    const T* Y = arena + tp.yoff;
    const bool staged = m * k <= 64 * 64;
    __syncthreads();
    if (staged)
      for (int e = threadIdx.x; e < m * k; e += blockDim.x) {
        const int i = e % m, kk = e / m;
        Dg[i + kk * m] = double(Y[i + (int64_t)kk * tp.ldy]);
      }
    __syncthreads();
    double* Tb = a.tbuf + tp.toff * a.max_rhs;
    for (int o = threadIdx.x; o < k * nrhs; o += blockDim.x) {
      const int kk = o % k, c = o / k;
      double sum = 0.0;
      if (staged) {
#pragma unroll 8
        for (int i = 0; i < m; ++i) sum += Dg[i + kk * m] * acc[i * ldacc + c];
      } else {
        for (int i = 0; i < m; ++i) sum += double(Y[i + (int64_t)kk * tp.ldy]) * acc[i * ldacc + c];
      }
      cstore(Tb + kk + c * tp.cap, sum);
    }
  }
  stamp(a, 6);
  // every wave's stores complete, then the flags of all results of this task
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_s_waitcnt(0);
    if (lf.next_rec >= 0 && !fused)
      __hip_atomic_store(a.pflag + lf.next_rec, a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int q = 0; q < lf.ntq; ++q)
      __hip_atomic_store(a.tp_flag + a.leaf_tq[lf.tq0 + q], a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(a.leaf_flag + s, a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  stamp(a, 7);
}

// Partial-sum records of dense blocks whose column cluster this task's leaf
// completes: P = D y[sigma] (m x nrhs).
template <class T>
__device__ void run_push(const SolveArgs& a, const T* arena, int id, bool forward, double* As, double* Bs) {
  const int flag_base = forward ? 0 : a.L;
  for (int q0 = a.push0[id]; q0 < a.push0[id + 1]; ++q0) {
    const int rec = a.push_recs[q0];
    const SDense D = a.dense[rec];
    wait_leaves(a, flag_base, D.lf0, D.lf1);
    double pr[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) pr[q] = 0.0;
    mm_sub<T>(arena + D.off, D.ld, a.y + D.col0, 1, a.N, D.m, D.ncols, a.nrhs, pr, As, Bs);
    double* P = a.pbuf + (int64_t)rec * a.pstride;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int o = threadIdx.x + q * kSolveThreads;
      if (o < D.m * a.nrhs) cstore(P + o, -pr[q]);
    }
    publish(a.pflag + rec, a.epoch);
  }
}

// T = Y^T y[cols] (k x nrhs): one output per thread for short blocks, a
// row-split reduction through LDS for long ones.
template <class T>
__device__ void run_tprod(const SolveArgs& a, const T* arena, int tpi, bool forward, double* As, double* Bs) {
  const STprod tp = a.tprod[tpi];
  wait_leaves(a, forward ? 0 : a.L, tp.lf0, tp.lf1);
  const int k = a.dims[tp.slot];
  const int nrhs = a.nrhs;
  double* Tb = a.tbuf + tp.toff * a.max_rhs;
  const T* Y = arena + tp.yoff;
  const int nout = k * nrhs;     // <= 64 * 32 = 8 * 256
  // rows per stage: as many as the staging areas hold (Y: As, 128 x kKC
  // doubles; y: Bs and the inverse area behind it, 32 x kKC + 64 x 64), so
  // that each thread has many loads in flight per round trip
  int R = 256;
  while (R > kKC && (R * k > 128 * kKC || R * nrhs > 32 * kKC + 64 * 64)) R >>= 1;
  double s[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) s[q] = 0.0;
  for (int r0 = 0; r0 < tp.ncols; r0 += R) {
    const int rc = min(R, tp.ncols - r0);
    for (int e = threadIdx.x; e < rc * k; e += blockDim.x) {
      const int r = e % rc, kk = e / rc;
      As[kk * R + r] = double(Y[r0 + r + (int64_t)kk * tp.ldy]);
    }
    for (int e = threadIdx.x; e < rc * nrhs; e += blockDim.x) {
      const int r = e % rc, c = e / rc;
      Bs[c * R + r] = cload(a.y + tp.col0 + r0 + r + (int64_t)c * a.N);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int o = threadIdx.x + q * kSolveThreads;
      if (o < nout) {
        const int kk = o % k, c = o / k;
        double sum = 0.0;
#pragma unroll 8
        for (int r = 0; r < rc; ++r) sum += As[kk * R + r] * Bs[c * R + r];
        s[q] += sum;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int o = threadIdx.x + q * kSolveThreads;
    if (o < nout) cstore(Tb + (o % k) + (o / k) * tp.cap, s[q]);
  }
  publish(a.tp_flag + tpi, a.epoch);
}

template <class T>
__global__ void __launch_bounds__(kSolveThreads) solve_persistent_kernel(const T* arena, const T* inv,
                                                                        const T* nm, SolveArgs a0) {
  SolveArgs a = a0;
  // LDS: acc (128 x 32 doubles), A staging (128 x kKC doubles), B staging
  // (32 x kKC doubles), triangle inverses of a leaf up to 64 rows (64 x 64
  // doubles): 144 KB
  extern __shared__ double smem[];
  __shared__ int s_task;
  double* acc = smem;
  double* As = acc + 128 * 32;
  double* Bs = As + 128 * kKC;
  double* Dg = Bs + 32 * kKC;
  while (true) {
    if (threadIdx.x == 0) s_task = atomicAdd(a.ctr, 1);
    __syncthreads();
    const int t = s_task;
    __syncthreads();
    if (t >= a.ntasks) break;
    const STask task = a.tasks[t];
    a.cur_task = t;
    if (a.trace && threadIdx.x == 0) {
      a.trace[kTraceFields * t] = (int64_t)wall_clock64();
      a.trace[kTraceFields * t + 3] = blockIdx.x;
    }
    switch (task.kind) {
      case kFwdLeaf: run_leaf<T>(a, arena, inv, nm, task.idx, true, acc, As, Bs, Dg); break;
      case kFwdTprod:
        for (int q = a.tg0[task.idx]; q < a.tg0[task.idx + 1]; ++q) run_tprod<T>(a, arena, a.tg_list[q], true, As, Bs);
        break;
      case kBwdLeaf: run_leaf<T>(a, arena, inv, nm, task.idx, false, acc, As, Bs, Dg); break;
      case kBwdTprod:
        for (int q = a.tg0[task.idx]; q < a.tg0[task.idx + 1]; ++q) run_tprod<T>(a, arena, a.tg_list[q], false, As, Bs);
        break;
      case kFwdPush: run_push<T>(a, arena, task.idx, true, As, Bs); break;
      case kBwdPush: run_push<T>(a, arena, task.idx, false, As, Bs); break;
    }
    stamp(a, 2);
    if (task.kind == kFwdLeaf || task.kind == kFwdTprod || task.kind == kFwdPush) {
      if (threadIdx.x == 0) __hip_atomic_fetch_add(a.ctr + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
  }
  // the last workgroup to leave folds this launch's error word into the
  // word the host reads (hlu_sync_status, GMRES)
  if (threadIdx.x == 0) {
    const int32_t left = __hip_atomic_fetch_add(a.ctr + 4, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (left == (int32_t)gridDim.x - 1 && load_relaxed(a.ctr + 2) != 0)
      __hip_atomic_store(a.ctr + 3, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Inverses of the two triangles of each diagonal leaf, one workgroup per
// (leaf, triangle): blockIdx.y = 0 forms L^{-1} (unit lower) and writes its
// strictly lower part, blockIdx.y = 1 forms U^{-1} and writes the upper part
// with the diagonal, so both share one m x m block.  Columns of the identity
// are solved in chunks of `cols` in LDS by column-oriented substitution.
template <class T>
__global__ void __launch_bounds__(256) diag_inverse_kernel(const T* arena, const SLeaf* leaves, T* inv,
                                                           double* pivots, int cols) {
  extern __shared__ double sm[];
  const SLeaf lf = leaves[blockIdx.x];
  const int m = lf.m;
  const bool upper = blockIdx.y == 1;
  double* Ts = sm;            // m x m, column-major
  double* Vs = sm + m * m;    // m x cols, row i at Vs[i * cols]
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) Ts[e] = double(arena[lf.diag + e]);
  if (upper)
    for (int q = threadIdx.x; q < m; q += blockDim.x) pivots[lf.row0 + q] = double(arena[lf.diag + q + (int64_t)q * m]);
  for (int c0 = 0; c0 < m; c0 += cols) {
    const int pc = min(cols, m - c0);
    for (int e = threadIdx.x; e < m * pc; e += blockDim.x) {
      const int i = e / pc, j = e % pc;
      Vs[i * cols + j] = (i == c0 + j) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (!upper) {
      // rows above column c0 + j of the result stay zero: start at q = c0
      for (int q = c0; q < m - 1; ++q) {
        const int rows = m - q - 1;
        for (int e = threadIdx.x; e < rows * pc; e += blockDim.x) {
          const int r = q + 1 + e % rows, j = e / rows;
          Vs[r * cols + j] -= Ts[r + q * m] * Vs[q * cols + j];
        }
        __syncthreads();
      }
    } else {
      // rows below column c0 + j stay zero: start at the chunk's last column
      for (int q = c0 + pc - 1; q >= 0; --q) {
        const double d = 1.0 / Ts[q + q * m];
        for (int j = threadIdx.x; j < pc; j += blockDim.x) Vs[q * cols + j] *= d;
        __syncthreads();
        for (int e = threadIdx.x; e < q * pc; e += blockDim.x) {
          const int r = e % q, j = e / q;
          Vs[r * cols + j] -= Ts[r + q * m] * Vs[q * cols + j];
        }
        __syncthreads();
      }
    }
    for (int e = threadIdx.x; e < m * pc; e += blockDim.x) {
      const int i = e % m, j = e / m, col = c0 + j;
      if (upper ? i <= col : i > col) inv[lf.inv + i + (int64_t)col * m] = T(Vs[i * cols + j]);
    }
    __syncthreads();
  }
}

// For every leaf task with a neighbour record (lf.nm >= 0): the records'
// blocks D (rows of the next leaf, then of the second neighbour's record if
// any, x this leaf) times this leaf's triangle inverse (forward: unit lower
// L^{-1}; backward: U^{-1}), in FP64, stored in the factor's type.  One
// workgroup per leaf task; D and the inverse in LDS.
template <class T>
__global__ void __launch_bounds__(256) next_inverse_kernel(const T* arena, const SLeaf* leaves,
                                                           const SDense* dense, const T* inv, T* nm, int L) {
  extern __shared__ double sm[];
  const int s = blockIdx.x;
  const SLeaf lf = leaves[s];
  if (lf.nm < 0) return;
  const bool forward = s < L;
  const SDense d = dense[lf.next_rec];
  const int m = lf.m, dm = lf.nm_rows, dm1 = d.m;
  double* Ds = sm;              // dm x m, leading dimension dm (<= 128 x 64)
  double* Is = sm + 128 * 64;   // m x m (<= 64 x 64)
  for (int e = threadIdx.x; e < dm * m; e += blockDim.x) {
    const int i = e % dm, k = e / dm;
    if (i < dm1) {
      Ds[e] = double(arena[d.off + i + (int64_t)k * d.ld]);
    } else {
      const SDense& d2 = dense[lf.next_rec2];
      Ds[e] = double(arena[d2.off + (i - dm1) + (int64_t)k * d2.ld]);
    }
  }
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
    const int q = e % m, k = e / m;
    const double v = double(inv[lf.inv + e]);
    Is[e] = forward ? (q > k ? v : (q == k ? 1.0 : 0.0)) : (q <= k ? v : 0.0);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < dm * m; e += blockDim.x) {
    const int i = e % dm, k = e / dm;
    double sum = 0.0;
    for (int q = 0; q < m; ++q) sum += Ds[i + q * dm] * Is[q + k * m];
    nm[lf.nm + e] = T(sum);
  }
}

__global__ void solve_reset_kernel(int32_t* ctr) {
  if (threadIdx.x < 3 || threadIdx.x == 4) ctr[threadIdx.x] = 0;
}

}  // namespace dev

template <class T>
hipError_t solve_persistent_launch(const T* arena, const int32_t* dims, const SolveDev& d, int32_t N,
                                   int32_t nrhs, int32_t epoch, int32_t grid, hipStream_t s) {
  dev::solve_reset_kernel<<<1, 64, 0, s>>>(d.ctr);
  dev::SolveArgs a{d.tasks, d.leaves, d.dense, d.low, d.tprod, dims, d.y, d.tbuf, d.leaf_flag, d.tp_flag,
                   d.ctr, d.push0, d.push_recs, d.leaf_tq, d.tg0, d.tg_list, d.pbuf, d.pflag, d.pstride, d.trace,
                   d.wait_ticks, d.ntasks, d.n_fwd, N, nrhs, d.max_rhs, d.L, epoch, 0};
  // acc 128 x 32, A staging 128 x kKC, B staging 32 x kKC, inverses 64 x 64
  const size_t sh = ((size_t)128 * 32 + 128 * dev::kKC + 32 * dev::kKC + 64 * 64) * sizeof(double);
  static std::once_flag attr;
  std::call_once(attr, [sh] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&dev::solve_persistent_kernel<T>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  });
  dev::solve_persistent_kernel<T><<<grid, dev::kSolveThreads, sh, s>>>(arena, static_cast<const T*>(d.inv),
                                                                       static_cast<const T*>(d.nm), a);
  return hipGetLastError();
}

template <class T>
hipError_t diag_inverse_launch(const T* arena, const SolveDev& d, hipStream_t s) {
  constexpr size_t kLds = 160 * 1024;
  const size_t m = (size_t)d.max_m;
  const size_t tri = m * m * sizeof(double);
  int cols = (int)std::min<size_t>(m, (kLds - tri) / (m * sizeof(double)));
  const size_t sh = tri + m * (size_t)cols * sizeof(double);
  static std::once_flag attr;
  std::call_once(attr, [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&dev::diag_inverse_kernel<T>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLds);
  });
  dim3 g(d.L, 2);
  dev::diag_inverse_kernel<T><<<g, 256, sh, s>>>(arena, d.leaves, static_cast<T*>(d.inv), d.pivots, cols);
  // neighbour blocks times the inverses (96 KB of LDS)
  constexpr size_t kNmLds = (128 * 64 + 64 * 64) * sizeof(double);
  static std::once_flag attr2;
  std::call_once(attr2, [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&dev::next_inverse_kernel<T>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kNmLds);
  });
  dev::next_inverse_kernel<T><<<2 * d.L, 256, kNmLds, s>>>(arena, d.leaves, d.dense, static_cast<const T*>(d.inv),
                                                          static_cast<T*>(d.nm), d.L);
  return hipGetLastError();
}

template hipError_t diag_inverse_launch<float>(const float*, const SolveDev&, hipStream_t);
template hipError_t diag_inverse_launch<double>(const double*, const SolveDev&, hipStream_t);

template hipError_t solve_persistent_launch<float>(const float*, const int32_t*, const SolveDev&, int32_t, int32_t,
                                                   int32_t, int32_t, hipStream_t);
template hipError_t solve_persistent_launch<double>(const double*, const int32_t*, const SolveDev&, int32_t,
                                                    int32_t, int32_t, int32_t, hipStream_t);

}  // namespace hlu
