// Persistent H-triangular solve in chain form (Algorithm 1, step III:
// z = U^{-1}(L^{-1} r)) for gfx950; the schedule is described in
// chain_sched.h.
//
// One launch runs both sweeps.  Workgroups claim work through an atomic
// counter: the first claims are the chains (one per member of a batch and
// group of right-hand-side columns), the rest the helper tasks in the
// schedule's order.  Waits are bounded spins on flags and progress words
// stored with agent-scope atomics; data passed between workgroups (solution
// rows, T products, gather records) is stored and loaded with agent-scope
// coherent accesses, and a flag or progress word is stored only after every
// wave of the workgroup has completed its stores, so no cache writeback or
// invalidation sits on the critical path.  Factors are read in their
// storage type T; arithmetic and vectors are FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "chain_sched.h"

namespace hlu {
namespace dev {

constexpr int kThreads = 256;
constexpr int kKC = 64;            // columns per staged chunk of a dense product
constexpr int kRingRows = 2 * kMaxLeafRows;

struct KArgs {   // fits kChainArgBytes
  ChainDev d;
  const int32_t* dims;
  int64_t* trace;   // debug: chain 0 per position: clocks (hop start, inputs ready, product done,
                    // published) and the mask of gather records not ready at the first look
  int64_t* gtrace;  // debug: per gather record: clocks (start, dense done, inline done, end), position, input counts
  int32_t N, nrhs, n_chain, cw, epoch, n_chains_total;
};

__device__ __forceinline__ double cload(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void cstore(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t load_relaxed(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_relaxed(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Spin until *f satisfies the predicate, for at most `ticks` of the
// constant-rate wall clock; on timeout set the launch's error word.  After
// an error every wait returns at once, so the launch drains.
// The error word and the clock are looked at every 32nd poll only: each poll
// is a load from memory (agent scope), and the flag is what is waited for.
template <class Pred>
__device__ bool spin_until(const int32_t* f, Pred ok, int32_t* err, int64_t ticks) {
  if (ok(load_relaxed(f))) return true;
  const int64_t t0 = (int64_t)wall_clock64();
  for (uint32_t it = 1;; ++it) {
    __builtin_amdgcn_s_sleep(2);
    if (ok(load_relaxed(f))) return true;
    if ((it & 31u) == 0) {
      if (load_relaxed(err) != 0) return false;
      if ((int64_t)wall_clock64() - t0 > ticks) {
        store_relaxed(err, 1);
        return false;
      }
    }
  }
}

// After flags were observed by some threads: order the workgroup's later
// loads after the flag loads.
__device__ void acquire_all() {
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Every wave completes its stores, then one thread stores the flag.
__device__ void publish(int32_t* f, int32_t v) {
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __syncthreads();
  if (threadIdx.x == 0) store_relaxed(f, v);
}

// All chains of `member` have finished position pmax of the sweep.
__device__ void wait_progress(const KArgs& a, int member, int sweep, int pmax) {
  for (int c = threadIdx.x; c < a.n_chain; c += blockDim.x)
    spin_until(a.d.prog + 2 * (member * a.n_chain + c) + sweep, [pmax](int32_t v) { return v > pmax; },
               a.d.ctr + 2, a.d.wait_ticks);
  acquire_all();
}

__device__ void wait_flag(const KArgs& a, const int32_t* f) {
  if (threadIdx.x == 0)
    spin_until(f, [e = a.epoch](int32_t v) { return v == e; }, a.d.ctr + 2, a.d.wait_ticks);
  acquire_all();
}

// r[(i, c)] -= sum_k A[i, k] B[k, c] with A (m x K, type T, A[i + k*lda])
// and B (K x nrhs, FP64, B[k*bs + c*bcs]); both staged through LDS in
// chunks of kKC columns so that all loads of a chunk are in flight
// together.  Output (i, c) = o % m, o / m for o = threadIdx.x + 256 q.
template <class T, bool kBInLds = false>
__device__ void mm_sub(const T* A, int64_t lda, const double* B, int64_t bs, int64_t bcs, int m, int K, int nrhs,
                       double* r, double* As, double* Bs) {
  for (int k0 = 0; k0 < K; k0 += kKC) {
    const int kc = min(kKC, K - k0);
    for (int e = threadIdx.x; e < m * kc; e += blockDim.x) {
      const int i = e % m, k = e / m;
      As[k * kRingRows + i] = double(A[i + (int64_t)(k0 + k) * lda]);
    }
    for (int e = threadIdx.x; e < kc * nrhs; e += blockDim.x) {
      const int k = e % kc, c = e / kc;
      const double* bp = B + (int64_t)(k0 + k) * bs + (int64_t)c * bcs;
      Bs[c * kKC + k] = kBInLds ? *bp : cload(bp);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int o = threadIdx.x + q * kThreads;
      if (o < m * nrhs) {
        const int i = o % m, c = o / m;
        double sum = 0.0;
#pragma unroll 8
        for (int k = 0; k < kc; ++k) sum += As[k * kRingRows + i] * Bs[c * kKC + k];
        r[q] -= sum;
      }
    }
    __syncthreads();
  }
}

// T = Y^T y (k x nrhs) for Y (ncols x k, type T, Y[r + kk*ldy]) and the
// rows [col0, col0 + ncols) of y; rows staged through LDS; the result goes
// to out[kk + c*ldo] (global with coherent stores, or LDS).
template <class T, bool kToLds>
__device__ void tprod_block(const KArgs& a, const T* Y, int64_t ldy, int col0, int ncols, int k, double* out, int ldo,
                            double* As, double* Bs) {
  const int nrhs = a.nrhs;
  const int nout = k * nrhs;   // <= 64 * 32 = 8 * 256
  int R = 256;
  while (R > kKC && (R * k > kRingRows * kKC || R * nrhs > 32 * kKC + 64 * 64)) R >>= 1;
  double s[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) s[q] = 0.0;
  for (int r0 = 0; r0 < ncols; r0 += R) {
    const int rc = min(R, ncols - r0);
    for (int e = threadIdx.x; e < rc * k; e += blockDim.x) {
      const int r = e % rc, kk = e / rc;
      As[kk * R + r] = double(Y[r0 + r + (int64_t)kk * ldy]);
    }
    for (int e = threadIdx.x; e < rc * nrhs; e += blockDim.x) {
      const int r = e % rc, c = e / rc;
      Bs[c * R + r] = cload(a.d.y + col0 + r0 + r + (int64_t)c * a.N);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int o = threadIdx.x + q * kThreads;
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
    const int o = threadIdx.x + q * kThreads;
    if (o < nout) {
      double* p = out + (o % k) + (o / k) * ldo;
      if (kToLds) *p = s[q];
      else cstore(p, s[q]);
    }
  }
  __syncthreads();
}

// r -= sum over the low-rank inputs GLow[l0 .. l0 + nl) of X_t T_t, T_t the
// sum of the input's T-product chunks, as one product of the concatenated
// matrices [X_1 .. X_G] [T_1; ..; T_G]: every column kk of every X_t is a
// "virtual column", in schedule order.  Virtual columns go through LDS in
// fixed windows of 64 (the summation order depends on the ranks only, not
// on timing).  Before a window all threads wait, in parallel, for the
// chunk flags of the inputs it touches; then the T rows (summed over the
// chunks) and the X columns of the window are loaded together.
// scr: LDS scratch of at least 1536 doubles.
constexpr int kVCols = 512;   // virtual columns per table pass
template <class T>
__device__ void low_sum(const KArgs& a, const T* arena, int l0, int nl, int m, double* r, double* As, double* Bs,
                        double* scr) {
  const ChainDev& d = a.d;
  const int nrhs = a.nrhs;
  int* kpre = reinterpret_cast<int*>(scr);                   // [nl + 1] virtual column offsets (ints)
  int64_t* colX = reinterpret_cast<int64_t*>(scr + 512);     // [kVCols] arena index of the X column
  int* colW = reinterpret_cast<int*>(scr + 1024);            // [kVCols] input of the column
  int* colK = colW + kVCols;                                 // [kVCols] its column within the input
  for (int c0 = 0; c0 < nl; c0 += 256) {   // inputs in batches of 256
    const int nb = min(256, nl - c0);
    const int t0 = threadIdx.x;
    int k1 = 0;
    if (t0 < nb) k1 = a.dims[d.tprod[d.glow[l0 + c0 + t0].tp].slot];
    kpre[t0 + 1] = t0 < nb ? k1 : 0;
    if (t0 == 0) kpre[0] = 0;
    __syncthreads();
    for (int dd = 1; dd < 256; dd <<= 1) {   // inclusive scan of 256 entries
      const int v = t0 >= dd ? kpre[t0 + 1 - dd] : 0;
      __syncthreads();
      kpre[t0 + 1] += v;
      __syncthreads();
    }
    const int vtot = kpre[256];
    const int my0 = kpre[t0];
    __syncthreads();
    for (int w0 = 0; w0 < vtot; w0 += kVCols) {
      if (t0 < nb) {
        const GLow W = d.glow[l0 + c0 + t0];
        for (int kk = 0; kk < k1; ++kk) {
          const int v = my0 + kk - w0;
          if (v >= 0 && v < kVCols) {
            colX[v] = W.xoff + (int64_t)kk * W.ldx;
            colW[v] = c0 + t0;
            colK[v] = kk;
          }
        }
      }
      __syncthreads();
      const int wn = min(kVCols, vtot - w0);
      for (int v0 = 0; v0 < wn; v0 += kKC) {
        const int vc = min(kKC, wn - v0);
        // chunk flags of the window's inputs: 4 threads per virtual column
        {
          const int vv = threadIdx.x >> 2, sub = threadIdx.x & 3;
          if (vv < vc) {
            const GLow W = d.glow[l0 + colW[v0 + vv]];
            for (int q = sub; q < W.ntp; q += 4)
              spin_until(d.tp_flag + W.tp + q, [e = a.epoch](int32_t v) { return v == e; }, d.ctr + 2, d.wait_ticks);
          }
        }
        acquire_all();
        // T rows of the window (summed over chunks) and its X columns
        double tr[8];
        int td[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = threadIdx.x + u * kThreads;
          td[u] = -1;
          tr[u] = 0.0;
          if (e < vc * nrhs) {
            const int vv = e % vc, c = e / vc;
            const GLow W = d.glow[l0 + colW[v0 + vv]];
            const int kk = colK[v0 + vv];
            double sum = 0.0;
            for (int q = 0; q < W.ntp; ++q) {
              const CTprod tq = d.tprod[W.tp + q];
              sum += cload(d.tbuf + tq.toff * d.max_rhs + kk + (int64_t)c * tq.cap);
            }
            tr[u] = sum;
            td[u] = c * kKC + vv;
          }
        }
        for (int b0 = 0; b0 < m * vc; b0 += 16 * kThreads) {
          double xr[16];
          int xd[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int e = b0 + threadIdx.x + u * kThreads;
            xd[u] = -1;
            xr[u] = 0.0;
            if (e < m * vc) {
              const int i = e % m, vv = e / m;
              xr[u] = double(arena[colX[v0 + vv] + i]);
              xd[u] = vv * kRingRows + i;
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
        for (int q = 0; q < 16; ++q) {
          const int o = threadIdx.x + q * kThreads;
          if (o < m * nrhs) {
            const int i = o % m, c = o / m;
            double sum = 0.0;
#pragma unroll 8
            for (int vv = 0; vv < vc; ++vv) sum += As[vv * kRingRows + i] * Bs[c * kKC + vv];
            r[q] -= sum;
          }
        }
        __syncthreads();
      }
    }
  }
}

// F[rec] = -(sum of the gather's inputs), m x nrhs, leading dimension m.
template <class T>
__device__ void run_gather(const KArgs& a, const T* arena, int gi, double* As, double* Bs, double* scr, double* Ts) {
  const ChainDev& d = a.d;
  const CGather g = d.gathers[gi];
  const int sweep = g.pos >= d.L ? 1 : 0;
  const int m = g.m, nrhs = a.nrhs;
  double r[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) r[q] = 0.0;
  int64_t* tr = a.gtrace ? a.gtrace + 6 * (int64_t)g.rec : nullptr;   // debug clocks
  if (tr && threadIdx.x == 0) {
    tr[0] = (int64_t)wall_clock64();
    tr[4] = g.pos;
    tr[5] = g.nd | (g.ni << 10) | ((int64_t)g.nl << 20);
  }
  for (int t = g.d0; t < g.d0 + g.nd; ++t) {
    const GDense D = d.gdense[t];
    wait_progress(a, g.member, sweep, D.pmax);
    mm_sub<T>(arena + D.off, D.ld, d.y + D.col0, 1, a.N, m, D.ncols, nrhs, r, As, Bs);
  }
  if (tr && threadIdx.x == 0) tr[1] = (int64_t)wall_clock64();
  for (int t = g.i0; t < g.i0 + g.ni; ++t) {
    const GInline I = d.ginl[t];
    const int k = a.dims[I.slot];
    if (k == 0) continue;
    wait_progress(a, g.member, sweep, I.pmax);
    tprod_block<T, true>(a, arena + I.yoff, I.ldy, I.col0, I.ncols, k, Ts, k, As, Bs);
    mm_sub<T, true>(arena + I.xoff, I.ldx, Ts, 1, k, m, k, nrhs, r, As, Bs);
  }
  if (tr && threadIdx.x == 0) tr[2] = (int64_t)wall_clock64();
  if (g.nl > 0) low_sum<T>(a, arena, g.l0, g.nl, m, r, As, Bs, scr);
  if (g.prev >= 0) {   // the previous gather of this class: its record is added in
    wait_flag(a, d.g_flag + g.prev);
    const double* P = d.fbuf + (int64_t)g.prev * d.rstride;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int o = threadIdx.x + q * kThreads;
      if (o < m * nrhs) r[q] += cload(P + o);
    }
  }
  if (tr && threadIdx.x == 0) tr[3] = (int64_t)wall_clock64();
  double* F = d.fbuf + (int64_t)g.rec * d.rstride;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int o = threadIdx.x + q * kThreads;
    if (o < m * nrhs) cstore(F + o, r[q]);
  }
  publish(d.g_flag + g.rec, a.epoch);
}

// T-product chunks of one group: T = Y^T y[chunk rows].
template <class T>
__device__ void run_tprod_group(const KArgs& a, const T* arena, int id, double* As, double* Bs) {
  const ChainDev& d = a.d;
  for (int q = d.tg0[id]; q < d.tg0[id + 1]; ++q) {
    const int tpi = d.tg_list[q];
    const CTprod tp = d.tprod[tpi];
    wait_progress(a, tp.member, tp.sweep, tp.pmax);
    const int k = a.dims[tp.slot];
    if (k > 0)
      tprod_block<T, false>(a, arena + tp.yoff, tp.ldy, tp.col0, tp.ncols, k, d.tbuf + tp.toff * d.max_rhs,
                            tp.cap, As, Bs);
    publish(d.tp_flag + tpi, a.epoch);
  }
}

// One chain: columns [c0, c0 + cw) of one member, both sweeps.  Thread t
// owns row t of each position's stacked operator S_f (<= 256 rows); the
// right-hand side of the position goes through LDS (Rs, m x CW), the near
// contributions of the next kChainWindow positions accumulate in an LDS
// ring of kChainWindow + 1 slots.
template <class T, int CW>
__device__ void run_chain(const KArgs& a, const T* arena, int q, double* smem) {
  const ChainDev& d = a.d;
  const int member = q / a.n_chain, grp = q % a.n_chain;
  const int c0 = grp * a.cw;
  const int cw = min(a.cw, a.nrhs - c0);
  const int Lm = d.member_L[member], pos0 = d.member_pos0[member];
  int32_t* prog = d.prog + 2 * q;
  constexpr int kSlots = kChainWindow + 1;
  const int ringrows = d.max_m;
  double* ring = smem;                                 // [kSlots][ringrows][CW]
  double* Rs = ring + kSlots * ringrows * CW;          // [ringrows][CW]
  int4* tgs = reinterpret_cast<int4*>(Rs + ringrows * CW);   // [kMaxTargets] near targets of the position
  const T* stack = static_cast<const T*>(d.stack);
  const int t = threadIdx.x;
  constexpr int kPerB = (kRingRows * CW + kThreads - 1) / kThreads;
  for (int sweep = 0; sweep < 2; ++sweep) {
    for (int e = t; e < (kSlots + 1) * ringrows * CW; e += kThreads) ring[e] = 0.0;   // ring and Rs
    __syncthreads();
    CLeaf nxt = d.leaves[sweep * d.L + pos0];
    for (int pp = 0; pp < Lm; ++pp) {
      const CLeaf lf = nxt;
      nxt = d.leaves[sweep * d.L + pos0 + (pp + 1 < Lm ? pp + 1 : pp)];   // next position's record, early
      const int m = lf.m, rows = lf.srows;
      if (t < lf.nt) {   // this position's near targets, for the ring updates below
        const CTarget tg = d.tgt[lf.t0 + t];
        tgs[t] = make_int4(tg.dpos, tg.srow0, tg.m, 0);
      }
      // this thread's stacked-operator row (first 64 columns prefetched)
      // (loads issued unconditionally from clamped, in-bounds addresses, so
      // that all of them are in flight together; unused values are masked
      // where they are consumed)
      T ar[kMaxLeafRows];
      const T* srow = stack + lf.stack + (t < rows ? t : 0);
#pragma unroll
      for (int k = 0; k < kMaxLeafRows; ++k) ar[k] = srow[(int64_t)(k < m ? k : m - 1) * rows];
      // right-hand side rows of this chain's columns
      double bv[kPerB];
#pragma unroll
      for (int u = 0; u < kPerB; ++u) {
        const int o = t + u * kThreads;
        const int oc = o < m * cw ? o : 0;
        bv[u] = cload(d.y + lf.row0 + (oc % m) + (int64_t)(c0 + oc / m) * a.N);
      }
      // the gather records of this position
      int64_t* tr = (a.trace && q == 0) ? a.trace + 5 * (sweep * d.L + pos0 + pp) : nullptr;
      if (tr && t == 0) tr[0] = (int64_t)wall_clock64();
      {
        const int32_t rec = t < lf.nrec ? lf.rec0 + t : -1;
        if (rec >= 0) {
          if (tr && load_relaxed(d.g_flag + rec) != a.epoch) atomicOr(reinterpret_cast<unsigned long long*>(tr + 4), 1ull << t);
          spin_until(d.g_flag + rec, [e = a.epoch](int32_t v) { return v == e; }, d.ctr + 2, d.wait_ticks);
        }
      }
      acquire_all();
      if (tr && t == 0) tr[1] = (int64_t)wall_clock64();
      const int slot = pp % kSlots;
      // the records' entries, four records' loads in flight per step
      double fsum[kPerB];
#pragma unroll
      for (int u = 0; u < kPerB; ++u) fsum[u] = 0.0;
      {
        double fv[kPerB][kMaxRecords];
#pragma unroll
        for (int u = 0; u < kPerB; ++u) {
          const int o = t + u * kThreads;
          const int oc = o < m * cw ? o : 0;
#pragma unroll
          for (int g = 0; g < kMaxRecords; ++g) {
            const int64_t rec = lf.rec0 + (g < lf.nrec ? g : 0);
            fv[u][g] = cload(d.fbuf + rec * d.rstride + (oc % m) + (int64_t)(c0 + oc / m) * m);
          }
        }
#pragma unroll
        for (int u = 0; u < kPerB; ++u)
#pragma unroll
          for (int g = 0; g < kMaxRecords; ++g)
            if (g < lf.nrec) fsum[u] += fv[u][g];
      }
#pragma unroll
      for (int u = 0; u < kPerB; ++u) {
        const int o = t + u * kThreads;
        if (o < m * cw) {
          const int i = o % m, cc = o / m;
          Rs[i * CW + cc] = bv[u] + ring[(slot * ringrows + i) * CW + cc] + fsum[u];
        }
      }
      __syncthreads();
      for (int e = t; e < ringrows * CW; e += kThreads) ring[slot * ringrows * CW + e] = 0.0;
      // S_f r: y_f in rows [0, m), near contributions below
      if (t < rows) {
        double acc[CW];
#pragma unroll
        for (int cc = 0; cc < CW; ++cc) acc[cc] = 0.0;
        // fully unrolled in chunks of 8 rows (ar stays in registers); rows
        // k >= m of a chunk have ar[k] = 0 and finite Rs entries (zeroed
        // at the start of the sweep, written with finite values since)
#pragma unroll
        for (int k0 = 0; k0 < kMaxLeafRows; k0 += 8) {
          if (k0 < m) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const double av = (k0 + u < m) ? double(ar[k0 + u]) : 0.0;
              const double* rk = Rs + (k0 + u) * CW;
#pragma unroll
              for (int cc = 0; cc < CW; ++cc) acc[cc] += av * rk[cc];
            }
          }
        }
        for (int k = kMaxLeafRows; k < m; ++k) {
          const double av = double(srow[(int64_t)k * rows]);
#pragma unroll
          for (int cc = 0; cc < CW; ++cc) acc[cc] += av * Rs[k * CW + cc];
        }
        if (t < m) {
#pragma unroll
          for (int cc = 0; cc < CW; ++cc)
            if (cc < cw) cstore(d.y + lf.row0 + t + (int64_t)(c0 + cc) * a.N, acc[cc]);
        } else {
          for (int j = 0; j < lf.nt; ++j) {
            const int4 tg = tgs[j];   // dpos, srow0, m
            if (t >= tg.y && t < tg.y + tg.z) {
              double* rp = ring + (((pp + tg.x) % kSlots) * ringrows + (t - tg.y)) * CW;
#pragma unroll
              for (int cc = 0; cc < CW; ++cc) rp[cc] -= acc[cc];
              break;
            }
          }
        }
      }
      if (tr && t == 0) tr[2] = (int64_t)wall_clock64();
      publish(prog + sweep, pp + 1);
      if (tr && t == 0) tr[3] = (int64_t)wall_clock64();
    }
  }
}

// The launch arguments come from device memory (written by the reset
// kernel): a kernel parameter bound to a reference would be copied to
// private memory, while uniform loads through this pointer stay scalar.
template <class T, int CW>
__global__ void __launch_bounds__(kThreads) chain_solve_kernel(const T* arena, const KArgs* __restrict__ ka) {
  const KArgs& a = *ka;
  extern __shared__ double smem[];
  __shared__ int s_task;
  double* As = smem;                         // kRingRows x kKC
  double* Bs = As + kRingRows * kKC;         // 32 x kKC (+ 64 x 64 for tprod_block's row stages)
  double* Ts = Bs + 32 * kKC + 64 * 64;      // 64 x 32
  double* scr = Ts + 64 * 32;                // 2816
  while (true) {
    if (threadIdx.x == 0) s_task = atomicAdd(a.d.ctr, 1);
    __syncthreads();
    const int t = s_task;
    __syncthreads();
    if (t >= a.n_chains_total + a.d.ntasks) break;
    if (t < a.n_chains_total) {
      run_chain<T, CW>(a, arena, t, smem);
    } else {
      const CTask task = a.d.tasks[t - a.n_chains_total];
      if (task.kind == kTaskTprod) run_tprod_group<T>(a, arena, task.idx, As, Bs);
      else run_gather<T>(a, arena, task.idx, As, Bs, scr, Ts);
    }
    __syncthreads();
  }
  // the last workgroup to leave folds this launch's error word into the
  // word the host reads
  if (threadIdx.x == 0) {
    const int32_t left = __hip_atomic_fetch_add(a.d.ctr + 4, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (left == (int32_t)gridDim.x - 1 && load_relaxed(a.d.ctr + 2) != 0) store_relaxed(a.d.ctr + 3, 1);
  }
}

__global__ void chain_reset_kernel(KArgs a, KArgs* dst) {
  if (threadIdx.x == 0) *dst = a;
  if (threadIdx.x < 3 || threadIdx.x == 4) a.d.ctr[threadIdx.x] = 0;
  for (int i = threadIdx.x; i < 2 * a.n_chains_total; i += blockDim.x) a.d.prog[i] = 0;
}

// Inverses of the two triangles of each diagonal leaf, one workgroup per
// (leaf, triangle): blockIdx.y = 0 forms L^{-1} (unit lower) and writes its
// strictly lower part, blockIdx.y = 1 forms U^{-1} and writes the upper part
// with the diagonal, so both share one m x m block.  Columns of the identity
// are solved in chunks of `cols` in LDS by column-oriented substitution.
template <class T>
__global__ void __launch_bounds__(256) diag_inverse_kernel(const T* arena, const CLeaf* leaves, T* inv,
                                                           double* pivots, int cols) {
  extern __shared__ double sm[];
  const CLeaf lf = leaves[blockIdx.x];   // forward positions = leaves in order
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
      for (int q = c0; q < m - 1; ++q) {
        const int rows = m - q - 1;
        for (int e = threadIdx.x; e < rows * pc; e += blockDim.x) {
          const int r = q + 1 + e % rows, j = e / rows;
          Vs[r * cols + j] -= Ts[r + q * m] * Vs[q * cols + j];
        }
        __syncthreads();
      }
    } else {
      for (int q = c0 + pc - 1; q >= 0; --q) {
        const double dq = 1.0 / Ts[q + q * m];
        for (int j = threadIdx.x; j < pc; j += blockDim.x) Vs[q * cols + j] *= dq;
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

// The stacked operator of every position (one workgroup each): the leaf's
// triangle inverse (forward: unit lower L^{-1}; backward: U^{-1}), then for
// every near target the block from this leaf to the target (dense piece,
// or X_t Y_s^T of a low-rank block) times that inverse; FP64, stored in T.
// LDS: the inverse (m x m) and a 16-row slice of the block.
constexpr int kStackSlice = 16;
template <class T>
__global__ void __launch_bounds__(256) stack_kernel(const T* arena, const int32_t* dims, const CLeaf* leaves,
                                                    const CTarget* tgt, const T* inv, T* stack, int L) {
  extern __shared__ double sm[];
  const int q = blockIdx.x;
  const CLeaf lf = leaves[q];
  const bool forward = q < L;
  const int m = lf.m, rows = lf.srows;
  double* Is = sm;                 // m x m, column-major
  double* Ps = sm + m * m;         // kStackSlice x m, row-major
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
    const int i = e % m, j = e / m;
    const double v = double(inv[lf.inv + e]);
    Is[e] = forward ? (i > j ? v : (i == j ? 1.0 : 0.0)) : (i <= j ? v : 0.0);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < m * m; e += blockDim.x)
    stack[lf.stack + (e % m) + (int64_t)(e / m) * rows] = T(Is[e]);
  for (int j = lf.t0; j < lf.t0 + lf.nt; ++j) {
    const CTarget tg = tgt[j];
    const int k = tg.kind == 1 ? dims[tg.slot] : 0;
    for (int i0 = 0; i0 < tg.m; i0 += kStackSlice) {
      const int ni = min(kStackSlice, tg.m - i0);
      for (int e = threadIdx.x; e < ni * m; e += blockDim.x) {
        const int i = e / m, l = e % m;
        double v = 0.0;
        if (tg.kind == 0) {
          v = double(arena[tg.off + (i0 + i) + (int64_t)l * tg.ld]);
        } else {
          for (int r = 0; r < k; ++r)
            v += double(arena[tg.off + (i0 + i) + (int64_t)r * tg.ld]) * double(arena[tg.yoff + l + (int64_t)r * tg.ldy]);
        }
        Ps[i * m + l] = v;
      }
      __syncthreads();
      for (int e = threadIdx.x; e < ni * m; e += blockDim.x) {
        const int i = e % ni, c = e / ni;
        double v = 0.0;
        for (int l = 0; l < m; ++l) v += Ps[i * m + l] * Is[l + c * m];
        stack[lf.stack + (tg.srow0 + i0 + i) + (int64_t)c * rows] = T(v);
      }
      __syncthreads();
    }
  }
}

}  // namespace dev

static_assert(sizeof(dev::KArgs) <= kChainArgBytes, "launch arguments exceed their device buffer");

namespace {
constexpr size_t kLdsMax = 160 * 1024;

size_t helper_lds() {
  return ((size_t)dev::kRingRows * dev::kKC + 32 * dev::kKC + 64 * 64 + 64 * 32 + 2816) * sizeof(double);
}
size_t chain_lds(int cw, int max_m) {
  return ((size_t)(kChainWindow + 2) * max_m * cw) * sizeof(double) + kMaxTargets * sizeof(int4);
}

template <class T, int CW>
hipError_t launch_cw(const T* arena, const dev::KArgs* a, int grid, size_t sh, hipStream_t s) {
  static std::once_flag attr;   // the kernel's static LDS (claim slot) comes on top
  std::call_once(attr, [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&dev::chain_solve_kernel<T, CW>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kLdsMax - 1024));
  });
  dev::chain_solve_kernel<T, CW><<<grid, dev::kThreads, sh, s>>>(arena, a);
  return hipGetLastError();
}
}  // namespace

template <class T>
hipError_t chain_solve_launch(const T* arena, const int32_t* dims, const ChainDev& d, int32_t N, int32_t nrhs,
                              int32_t epoch, hipStream_t s) {
  constexpr int kGrid = 256;       // one workgroup per CU
  constexpr int kChainBudget = 64; // chains per launch at most (the prog buffer's size)
  // chains: groups of kChainCols columns per member
  const int per_member = std::max(1, kChainBudget / std::max(1, d.members));
  int n_chain = std::min((nrhs + kChainCols - 1) / kChainCols, per_member);
  int cw = (nrhs + n_chain - 1) / n_chain;
  int CW = 1;
  while (CW < cw) CW <<= 1;
  if (CW > 32 || chain_lds(CW, d.max_m) + 1024 > kLdsMax || helper_lds() + 1024 > kLdsMax ||
      d.members > kChainBudget)
    return hipErrorInvalidValue;
  n_chain = (nrhs + cw - 1) / cw;
  dev::KArgs a{d, dims, d.trace, d.trace ? d.trace + 5 * 2 * (int64_t)d.L : nullptr, N, nrhs, n_chain, cw, epoch,
               d.members * n_chain};
  dev::KArgs* ka = reinterpret_cast<dev::KArgs*>(d.kargs);
  dev::chain_reset_kernel<<<1, 256, 0, s>>>(a, ka);
  const size_t sh = std::max(helper_lds(), chain_lds(CW, d.max_m));
  switch (CW) {
    case 1: return launch_cw<T, 1>(arena, ka, kGrid, sh, s);
    case 2: return launch_cw<T, 2>(arena, ka, kGrid, sh, s);
    case 4: return launch_cw<T, 4>(arena, ka, kGrid, sh, s);
    case 8: return launch_cw<T, 8>(arena, ka, kGrid, sh, s);
    case 16: return launch_cw<T, 16>(arena, ka, kGrid, sh, s);
    default: return launch_cw<T, 32>(arena, ka, kGrid, sh, s);
  }
}

template <class T>
hipError_t chain_prepare_launch(const T* arena, const int32_t* dims, const ChainDev& d, int32_t num_leaves,
                                hipStream_t s) {
  const size_t m = (size_t)d.max_m;
  const size_t tri = m * m * sizeof(double);
  int cols = (int)std::min<size_t>(m, (kLdsMax - tri) / (m * sizeof(double)));
  const size_t sh = tri + m * (size_t)cols * sizeof(double);
  static std::once_flag attr;
  std::call_once(attr, [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&dev::diag_inverse_kernel<T>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&dev::stack_kernel<T>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax);
  });
  dim3 g(num_leaves, 2);
  dev::diag_inverse_kernel<T><<<g, 256, sh, s>>>(arena, d.leaves, static_cast<T*>(d.inv), d.pivots, cols);
  const size_t sh2 = (m * m + (size_t)dev::kStackSlice * m) * sizeof(double);
  dev::stack_kernel<T><<<2 * num_leaves, 256, sh2, s>>>(arena, dims, d.leaves, d.tgt, static_cast<const T*>(d.inv),
                                                        static_cast<T*>(d.stack), num_leaves);
  return hipGetLastError();
}

template hipError_t chain_prepare_launch<float>(const float*, const int32_t*, const ChainDev&, int32_t, hipStream_t);
template hipError_t chain_prepare_launch<double>(const double*, const int32_t*, const ChainDev&, int32_t, hipStream_t);
template hipError_t chain_solve_launch<float>(const float*, const int32_t*, const ChainDev&, int32_t, int32_t, int32_t,
                                              hipStream_t);
template hipError_t chain_solve_launch<double>(const double*, const int32_t*, const ChainDev&, int32_t, int32_t,
                                               int32_t, hipStream_t);

}  // namespace hlu
