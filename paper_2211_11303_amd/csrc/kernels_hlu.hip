// Batched task kernels of the H-LU factorisation, H-solves and L U product
// for gfx950.  Each launch runs the tasks of one kind from one wave of a
// plan; tasks of a wave touch disjoint data.  T is the storage and
// arithmetic type of the factors (float or double); the small dense algebra
// inside the truncation is always FP64.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include <cstdint>
#include <mutex>

#include "plan.h"
#include "trunc_rounds.h"
#include "waves.h"

// Row of the 16 x 16 result block held in register r of lane l by
// v_mfma_f32_16x16x4f32 (column l % 16).
#define MFMA_F32_ROW(l, r) (4 * ((l) >> 4) + (r))

namespace hlu {
namespace dev {

__device__ __forceinline__ int dimv(int32_t code, const int32_t* dims) { return dim_of(code, dims); }

template <class T>
__device__ __forceinline__ T& at(T* base, const MatRef& m, int i, int j) {
  return base[m.off + (int64_t)i * m.rs + (int64_t)j * m.cs];
}

// Nominal flops of the factor's tasks, added per workgroup into kFlopSpread
// counters per kind (spread by block index to limit atomic contention).
__device__ __forceinline__ void add_flops(int32_t* status, int kind, double flops) {
  unsigned long long* f = reinterpret_cast<unsigned long long*>(status + kFlopWord0);
  atomicAdd(f + kind * kFlopSpread + (blockIdx.x & (kFlopSpread - 1)), (unsigned long long)flops);
}

// --------------------------------------------------------------- GETRF
// Unpivoted right-looking LU of one dense diagonal leaf per workgroup,
// staged in LDS.  A zero pivot is counted in status[0] (the factor goes on,
// so that every wave finishes); |pivot| extremes are not tracked here.
template <class T, class C>
__global__ void __launch_bounds__(256) getrf_kernel(T* arena, const GetrfOp* ops, int32_t* status) {
  extern __shared__ unsigned char smem_raw[];
  C* D = reinterpret_cast<C*>(smem_raw);
  const GetrfOp op = ops[blockIdx.x];
  const int m = op.m;
  T* g = arena + op.off;
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
    const int i = e % m, j = e / m;
    D[i + j * m] = g[i + (int64_t)j * op.ld];
  }
  __syncthreads();
  for (int p = 0; p < m; ++p) {
    const C piv = D[p + p * m];
    if (piv == C(0)) {
      if (threadIdx.x == 0) atomicAdd(&status[0], 1);
    }
    const C inv = piv == C(0) ? C(0) : C(1) / piv;
    for (int i = p + 1 + threadIdx.x; i < m; i += blockDim.x) D[i + p * m] *= inv;
    __syncthreads();
    const int rem = m - p - 1;
    for (int e = threadIdx.x; e < rem * rem; e += blockDim.x) {
      const int i = p + 1 + e % rem, j = p + 1 + e / rem;
      D[i + j * m] -= D[i + p * m] * D[p + j * m];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
    const int i = e % m, j = e / m;
    g[i + (int64_t)j * op.ld] = T(D[i + j * m]);
  }
  if (threadIdx.x == 0) add_flops(status, kFlopGetrf, 2.0 * m * m * m / 3.0);
}

// ----------------------------------------------------------------- TRI
// Triangular solve / multiply with a dense diagonal leaf (m <= max leaf),
// one workgroup per task.  The leaf and a chunk of up to 64 columns of V
// are staged in LDS; substitutions eliminate one row per step with all
// threads updating the remaining rows (m barriers per chunk).
constexpr int kTriMaxCols = 64;
constexpr size_t kLdsBytes = 160 * 1024;

template <class T, class C>
__global__ void __launch_bounds__(256) tri_kernel(T* arena, const TriOp* ops, const int32_t* dims,
                                                  int tri_cols, int32_t* status) {
  extern __shared__ unsigned char smem_raw[];
  const TriOp op = ops[blockIdx.x];
  const int m = op.m;
  const int kTriCols = tri_cols;                     // columns per chunk (<= 64)
  C* Ts = reinterpret_cast<C*>(smem_raw);          // m x m, column-major (ld m)
  C* Vs = Ts + m * m;                                // m x kTriCols, row i at Vs[i * kTriCols]
  const int p = dimv(op.V.cols, dims);
  const T* Tg = arena + op.tri;
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) Ts[e] = C(Tg[(e % m) + (int64_t)(e / m) * op.ld]);
  const bool mul = op.mode == kMulUpper || op.mode == kMulUnitLower;
  for (int c0 = 0; c0 < p; c0 += kTriCols) {
    const int pc = min(kTriCols, p - c0);
    for (int e = threadIdx.x; e < m * pc; e += blockDim.x) {
      const int i = e % m, j = e / m;
      Vs[i * kTriCols + j] = C(at(arena, op.V, i, c0 + j));
    }
    __syncthreads();
    switch (op.mode) {
      case kSolveUnitLower:     // forward: rows below step q get V[r] -= L[r][q] V[q]
        for (int q = 0; q < m - 1; ++q) {
          const int rows = m - q - 1;
          for (int e = threadIdx.x; e < rows * pc; e += blockDim.x) {
            const int r = q + 1 + e % rows, j = e / rows;
            Vs[r * kTriCols + j] -= Ts[r + q * m] * Vs[q * kTriCols + j];
          }
          __syncthreads();
        }
        break;
      case kSolveUpperT:        // U^T lower, non-unit: scale row q, then update below
        for (int q = 0; q < m; ++q) {
          const C d = C(1) / Ts[q + q * m];
          for (int j = threadIdx.x; j < pc; j += blockDim.x) Vs[q * kTriCols + j] *= d;
          __syncthreads();
          const int rows = m - q - 1;
          for (int e = threadIdx.x; e < rows * pc; e += blockDim.x) {
            const int r = q + 1 + e % rows, j = e / rows;
            Vs[r * kTriCols + j] -= Ts[q + r * m] * Vs[q * kTriCols + j];
          }
          __syncthreads();
        }
        break;
      case kSolveUpper:         // backward: scale row q, then update above
        for (int q = m - 1; q >= 0; --q) {
          const C d = C(1) / Ts[q + q * m];
          for (int j = threadIdx.x; j < pc; j += blockDim.x) Vs[q * kTriCols + j] *= d;
          __syncthreads();
          for (int e = threadIdx.x; e < q * pc; e += blockDim.x) {
            const int r = e % q, j = e / q;
            Vs[r * kTriCols + j] -= Ts[r + q * m] * Vs[q * kTriCols + j];
          }
          __syncthreads();
        }
        break;
      case kMulUpper:
        for (int e = threadIdx.x; e < m * pc; e += blockDim.x) {
          const int i = e % m, j = e / m;
          C s = 0;
          for (int q = i; q < m; ++q) s += Ts[i + q * m] * Vs[q * kTriCols + j];
          at(arena, op.W, i, c0 + j) = T(s);
        }
        break;
      case kMulUnitLower:
        for (int e = threadIdx.x; e < m * pc; e += blockDim.x) {
          const int i = e % m, j = e / m;
          C s = Vs[i * kTriCols + j];
          for (int q = 0; q < i; ++q) s += Ts[i + q * m] * Vs[q * kTriCols + j];
          at(arena, op.W, i, c0 + j) = T(s);
        }
        break;
    }
    __syncthreads();
    if (!mul) {
      for (int e = threadIdx.x; e < m * pc; e += blockDim.x) {
        const int i = e % m, jj = e / m;
        at(arena, op.V, i, c0 + jj) = T(Vs[i * kTriCols + jj]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) add_flops(status, kFlopTri, (double)m * m * p);
}

// ---------------------------------------------------------------- GEMM
// One 64 x 64 output tile per workgroup, C = beta C + sum_t alpha_t A_t B_t
// (operands of any strides), on the matrix cores: k is streamed through LDS
// in chunks of 16 (A scaled by alpha_t when staged), each wavefront owns a
// 32 x 32 quarter of the tile as 2 x 2 blocks of 16 x 16, and each block
// accumulates 16 x 16 x 4 MFMAs in the arithmetic type C (FP32 or FP64).
// Operand lanes: A[i][k] at lane i + 16k, B[k][j] at lane j + 16k; result
// register r of lane l holds D[mfma_row(l, r)][l % 16] (layouts measured on
// the device).  Thread 0 adds the tile's nominal flops (2 m n k per term)
// to the factor's flop counters.
constexpr int kGT = 64, kGK = 16;

typedef float mfma_f4 __attribute__((ext_vector_type(4)));
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

template <class C>
struct Mfma;
template <>
struct Mfma<float> {
  typedef mfma_f4 acc_t;
  __device__ static acc_t step(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int r) { return MFMA_F32_ROW(lane, r); }
};
template <>
struct Mfma<double> {
  typedef mfma_d4 acc_t;
  __device__ static acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <class T, class C>
__global__ void __launch_bounds__(256) gemm_kernel(T* arena, const GemmOp* ops, const GemmTerm* terms,
                                                   const int32_t* tile_op, const int32_t* tile_ij,
                                                   int32_t tile0, const int32_t* dims, int32_t* status) {
  __shared__ C As[kGK][kGT + 1];
  __shared__ C Bs[kGK][kGT + 1];
  typedef typename Mfma<C>::acc_t acc_t;
  const int tile = tile0 + blockIdx.x;
  const GemmOp op = ops[tile_op[tile]];
  const int ti = tile_ij[tile] >> 16, tj = tile_ij[tile] & 0xffff;
  const int M = dimv(op.C.rows, dims), N = dimv(op.C.cols, dims);
  const int i0 = ti * kGT, j0 = tj * kGT;
  if (i0 >= M || j0 >= N) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{C(0), C(0), C(0), C(0)};
  double flops = 0.0;
  for (int t = 0; t < op.nt; ++t) {
    const GemmTerm tm = terms[op.t0 + t];
    const int K = dimv(tm.A.cols, dims);
    const C alpha = C(tm.alpha);
    flops += 2.0 * min(kGT, M - i0) * min(kGT, N - j0) * K;
    for (int k0 = 0; k0 < K; k0 += kGK) {
      for (int e = threadIdx.x; e < kGK * kGT; e += 256) {
        // consecutive threads walk the unit-stride dimension of the operand
        // when it has one
        int r, c;
        if (tm.A.rs == 1) { r = e % kGT; c = e / kGT; } else { c = e % kGK; r = e / kGK; }
        const int gi = i0 + r, gk = k0 + c;
        As[c][r] = (gi < M && gk < K) ? alpha * C(at(arena, tm.A, gi, gk)) : C(0);
        int r2, c2;
        if (tm.B.cs == 1) { c2 = e % kGT; r2 = e / kGT; } else { r2 = e % kGK; c2 = e / kGK; }
        const int bk = k0 + r2, bj = j0 + c2;
        Bs[r2][c2] = (bk < K && bj < N) ? C(at(arena, tm.B, bk, bj)) : C(0);
      }
      __syncthreads();
      const int kc = min(kGK, K - k0);
      for (int ks = 0; ks < kc; ks += 4) {
        const int kk = ks + (lane >> 4);
        C av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = As[kk][wr + 16 * a + (lane & 15)];
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = Bs[kk][wc + 16 * b + (lane & 15)];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<C>::step(av[a], bv[b], acc[a][b]);
      }
      __syncthreads();
    }
  }
  const C beta = C(op.beta);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = i0 + wr + 16 * a + Mfma<C>::row(lane, r);
        const int gj = j0 + wc + 16 * b + (lane & 15);
        if (gi < M && gj < N) {
          T& c = at(arena, op.C, gi, gj);
          c = T((op.beta == 0.0 ? C(0) : beta * C(c)) + acc[a][b][r]);
        }
      }
  if (threadIdx.x == 0) add_flops(status, kFlopGemm, flops);
}

// ---------------------------------------------------------------- FILL
template <class T>
__global__ void fill_kernel(T* arena, const FillOp* ops, const int32_t* dims) {
  const FillOp op = ops[blockIdx.y];
  const int M = dimv(op.M.rows, dims), N = dimv(op.M.cols, dims);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)M * N;
       e += (int64_t)gridDim.x * blockDim.x)
    at(arena, op.M, (int)(e % M), (int)(e / M)) = T(op.value);
}

// --------------------------------------------------------------- TRUNC
// Truncated low-rank addition C <- C + sum_p alpha_p X_p Y_p^T, one
// workgroup per task.  With Xa = [X_C, parts], Ya = [Y_C, parts] (K
// columns), the singular values of Xa Ya^T are found as follows (all FP64):
//   Gx = Xa^T Xa = R^T R        pivoted Cholesky, numerical rank r1
//                               (Xa P_1..r1 = Q R11 with Q orthonormal)
//   S  = R (Ya^T Ya) R^T = W diag(sigma^2) W^T     cyclic Jacobi, LDS
// Keeping the r leading triplets with sigma_i > max(eps, floor) sigma_1
// (r <= capacity) gives the best rank-r approximation Q W_r W_r^T R Ya^T:
//   X_C = Xa T_x,  T_x = P_1..r1 R11^{-1} W_r   (orthonormal columns)
//   Y_C = Ya T_y,  T_y = R^T W_r                (norms sigma_i)
// More than kKMax columns are absorbed in rounds, truncating after each; the
// round structure and its termination bound are in trunc_rounds.h.
constexpr int kKMax = kTruncCols;
constexpr int kLd = kKMax + 1;
// The truncation runs 256 threads; its K x K updates (pivoted Cholesky,
// Jacobi) give thread t the entries (t / 16 + 16 u, t % 16 + 16 v), u, v < 4.
static_assert(kKMax <= 64, "the 16 x 16 thread grid of the truncation covers at most 64 x 64 entries");

struct ColSrc {
  int64_t off;     // column 0 element of the source (already offset by column)
  int32_t rs;      // row stride of the source
  int32_t row_off; // first row of C covered
  int32_t rows;    // rows covered
  double alpha;
};

template <class T>
__device__ void load_tile(const T* arena, const ColSrc* src, int K, int i0, int RT, int mrows, double* tile) {
  // tile[i * kLd + a] = column a, row i0 + i
  for (int e = threadIdx.x; e < RT * K; e += blockDim.x) {
    const int a = e / RT, i = e % RT;
    const int gi = i0 + i;
    double v = 0.0;
    if (gi < mrows) {
      const ColSrc s = src[a];
      const int li = gi - s.row_off;
      if (li >= 0 && li < s.rows) v = s.alpha * double(arena[s.off + (int64_t)li * s.rs]);
    }
    tile[i * kLd + a] = v;
  }
}

// G = A^T A for the K source columns over mrows rows (G: K x K, ld kLd).
// Each thread owns a 4 x 4 block of G (16 x 16 blocks cover K <= 64); row
// tiles of kKMax rows are staged in `stage`.
template <class T>
__device__ void gram(const T* arena, const ColSrc* src, int K, int mrows, double* G, double* stage) {
  const int bi = threadIdx.x / 16, bj = threadIdx.x % 16;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  const bool active = 4 * bi < K && 4 * bj < K;
  for (int i0 = 0; i0 < mrows; i0 += kKMax) {
    load_tile(arena, src, K, i0, kKMax, mrows, stage);
    __syncthreads();
    const int rt = min(kKMax, mrows - i0);
    if (active) {
      for (int i = 0; i < rt; ++i) {
        double x[4], y[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          x[a] = (4 * bi + a < K) ? stage[i * kLd + 4 * bi + a] : 0.0;
          y[a] = (4 * bj + a < K) ? stage[i * kLd + 4 * bj + a] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] += x[a] * y[b];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (4 * bi + a < K && 4 * bj + b < K) G[(4 * bi + a) * kLd + 4 * bj + b] = acc[a][b];
  __syncthreads();
}

// Pivoted Cholesky of the symmetric positive semidefinite G (K x K, ld
// kLd), whose content is overwritten by Schur complements.  Row k < r1 of R
// (ld kLd) receives R[k][:] in the original column order (zero in columns
// chosen earlier), piv[k] the k-th pivot; stops when the largest remaining
// diagonal is <= tol2 times the largest initial one.  Returns r1.
__device__ int pivoted_cholesky(double* G, double* R, int K, double tol2, int* piv, double* d, int* chosen,
                                int* s_int, double* s_dbl) {
  for (int j = threadIdx.x; j < K; j += blockDim.x) {
    d[j] = G[j * kLd + j];
    chosen[j] = 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double dm = 0.0;
    for (int j = 0; j < K; ++j) dm = fmax(dm, d[j]);
    s_dbl[0] = dm;
  }
  __syncthreads();
  const double dmax0 = s_dbl[0];
  int r1 = 0;
  for (int k = 0; k < K; ++k) {
    if (threadIdx.x < 64) {   // argmax of the unchosen diagonal, lowest index on ties
      double best = -1.0;
      int bidx = K;
      for (int j = threadIdx.x; j < K; j += 64)
        if (!chosen[j] && d[j] > best) {
          best = d[j];
          bidx = j;
        }
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bidx, o, 64);
        if (ob > best || (ob == best && oi < bidx)) {
          best = ob;
          bidx = oi;
        }
      }
      if (threadIdx.x == 0) {
        s_int[0] = (bidx < K && best > 0.0 && best > tol2 * dmax0) ? bidx : -1;
        s_dbl[1] = best;
      }
    }
    __syncthreads();
    const int p = s_int[0];
    if (p < 0) break;
    const double rkk = sqrt(s_dbl[1]);
    for (int j = threadIdx.x; j < K; j += blockDim.x) {
      R[k * kLd + j] = (j == p) ? rkk : (chosen[j] ? 0.0 : G[p * kLd + j] / rkk);
      if (j == p) {   // only this thread reads chosen[p] in this step
        chosen[p] = 1;
        piv[k] = p;
      }
    }
    __syncthreads();
    // Schur complement on the unchosen rows and columns (p is chosen now):
    // entry (a, b) = (ty + 16 u, tx + 16 v), no division per entry
    for (int u = 0; u < 4; ++u) {
      const int a = (int)(threadIdx.x >> 4) + 16 * u;
      if (a >= K) break;
      if (chosen[a]) continue;
      const double ra = R[k * kLd + a];
      for (int v4 = 0; v4 < 4; ++v4) {
        const int b = (int)(threadIdx.x & 15) + 16 * v4;
        if (b >= K) break;
        if (!chosen[b]) G[a * kLd + b] -= ra * R[k * kLd + b];
      }
    }
    for (int j = threadIdx.x; j < K; j += blockDim.x)
      if (!chosen[j]) d[j] -= R[k * kLd + j] * R[k * kLd + j];
    __syncthreads();
    r1 = k + 1;
  }
  return r1;
}

// Cyclic Jacobi on the symmetric n x n matrix A (ld kLd; eigenvalues left on
// the diagonal of the returned buffer, eigenvectors accumulated in W), until
// the squared off-diagonal Frobenius norm is at most off_rel times the total.
// Each round pairs the indices round-robin; the rotations of the n/2
// disjoint pairs are computed first, with a table per index of its pair and
// its two coefficients (pk, pfirst, rt), then A' = J^T A J is written to B
// (double buffering) and W <- W J.  Returns the buffer that holds the final A.
__device__ double* jacobi(double* A, double* B, double* W, int n, double* cs, int* pk, int* pfirst,
                          double* red, double off_rel, int* sweeps, double* rt) {
  const int np = n + (n & 1);
  const int npair = np / 2;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) W[(e / n) * kLd + e % n] = (e / n == e % n) ? 1.0 : 0.0;
  __syncthreads();
  if (n <= 1) return A;
  for (int sweep = 0; sweep < 20; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      const double v = A[(e / n) * kLd + e % n];
      tot += v * v;
      if (e / n != e % n) off += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_down(off, o, 64);
      tot += __shfl_down(tot, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      red[threadIdx.x / 64] = off;
      red[4 + threadIdx.x / 64] = tot;
    }
    __syncthreads();
    const double offs = red[0] + red[1] + red[2] + red[3];
    const double tots = red[4] + red[5] + red[6] + red[7];
    __syncthreads();
    if (tots == 0.0 || offs <= off_rel * tots) break;
    ++*sweeps;
    for (int r = 0; r < np - 1; ++r) {
      for (int k = threadIdx.x; k < npair; k += blockDim.x) {
        int p, q;
        if (k == 0) {
          p = np - 1;
          q = r;
        } else {   // (r + k) mod (np - 1) and (r - k) mod (np - 1), both arguments in [0, 2 (np - 1))
          p = r + k;
          if (p >= np - 1) p -= np - 1;
          q = r - k + np - 1;
          if (q >= np - 1) q -= np - 1;
        }
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p * kLd + q];
          const double app = A[p * kLd + p], aqq = A[q * kLd + q];
          if (apq != 0.0 && fabs(apq) > 1e-17 * sqrt(fabs(app * aqq))) {
            const double th = (aqq - app) / (2.0 * apq);
            const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
          // per index i: the pair (pk[i], pfirst[i]) = (p, q) and i's two
          // coefficients on it, (c, -s) for p and (s, c) for q
          pk[p] = p;
          pfirst[p] = q;
          rt[2 * p] = c;
          rt[2 * p + 1] = -s;
          pk[q] = p;
          pfirst[q] = q;
          rt[2 * q] = s;
          rt[2 * q + 1] = c;
          cs[4 * k + 2] = p;
          cs[4 * k + 3] = q;
        } else {
          pk[p] = p;   // unpaired index (odd n): untouched this round
          pfirst[p] = p;
          rt[2 * p] = 1.0;
          rt[2 * p + 1] = 0.0;
        }
        cs[4 * k] = c;
        cs[4 * k + 1] = s;
      }
      __syncthreads();
      // B[i][j] = sum_{a in pair(i)} sum_{b in pair(j)} t_i[a] t_j[b] A[a][b],
      // with t = (c, -s) on (p, q) for the first index of a pair, (s, c) for the second
      // entry (i, j) = (ty + 16 u, tx + 16 v): no division per entry
      for (int u = 0; u < 4; ++u) {
        const int i = (int)(threadIdx.x >> 4) + 16 * u;
        if (i >= n) break;
        const int ia = pk[i], ib = pfirst[i];
        const double ti0 = rt[2 * i], ti1 = rt[2 * i + 1];
        for (int v4 = 0; v4 < 4; ++v4) {
          const int j = (int)(threadIdx.x & 15) + 16 * v4;
          if (j >= n) break;
          const int ja = pk[j], jb = pfirst[j];
          const double tj0 = rt[2 * j], tj1 = rt[2 * j + 1];
          double v = ti0 * (tj0 * A[ia * kLd + ja] + (tj1 != 0.0 ? tj1 * A[ia * kLd + jb] : 0.0));
          if (ti1 != 0.0) v += ti1 * (tj0 * A[ib * kLd + ja] + (tj1 != 0.0 ? tj1 * A[ib * kLd + jb] : 0.0));
          B[i * kLd + j] = v;
        }
      }
      // W <- W J: (row, pair) = (ty + 16 u, tx + 16 v), no division per entry
      for (int v2 = 0; v2 < 2; ++v2) {
        const int k = (int)(threadIdx.x & 15) + 16 * v2;
        if (k >= npair) break;
        if (cs[4 * k] == 1.0 && cs[4 * k + 1] == 0.0) continue;
        const int p = (int)cs[4 * k + 2], q = (int)cs[4 * k + 3];
        const double c = cs[4 * k], s = cs[4 * k + 1];
        for (int u = 0; u < 4; ++u) {
          const int row = (int)(threadIdx.x >> 4) + 16 * u;
          if (row >= n) break;
          const double wp = W[row * kLd + p], wq = W[row * kLd + q];
          W[row * kLd + p] = c * wp - s * wq;
          W[row * kLd + q] = s * wp + c * wq;
        }
      }
      __syncthreads();
      double* t = A;
      A = B;
      B = t;
    }
  }
  return A;
}

constexpr int kCompressMin = 8;         // S larger than this is compressed before the eigensolver
constexpr double kCompressTol = 0.01;   // relative pivot tolerance of that compression, in units of eps

template <class T>
__global__ void __launch_bounds__(256) trunc_kernel(T* arena, const TruncOp* ops, const TruncPart* parts,
                                                    int32_t* dims, double eps, double floor_rel,
                                                    int32_t* status, int64_t* trace, int32_t op_base,
                                                    int round_cols, int32_t* peak) {
  __shared__ double bufG[kKMax * kLd];
  __shared__ double bufR[kKMax * kLd];
  __shared__ double bufS[kKMax * kLd];
  __shared__ double bufW[kKMax * kLd];
  __shared__ ColSrc xs[kKMax], ys[kKMax];
  __shared__ double dvec[kKMax], mu[kKMax], dscale[kKMax], dinv[kKMax];
  __shared__ double cs[4 * (kKMax / 2 + 1)];
  __shared__ double rt[2 * kKMax];   // Jacobi: per index, its two rotation coefficients
  __shared__ double s_dbl[4];
  __shared__ double red[8];
  __shared__ int piv[kKMax], chosen[kKMax], sel[kKMax], pk[kKMax], pfirst[kKMax];
  __shared__ int s_int[4];
  __shared__ int s_K, s_r, s_r1, s_part, s_pcol, s_done, s_maxr;

  const TruncOp op = ops[blockIdx.x];
  const double tol2 = floor_rel * floor_rel;
  // Jacobi stops when the remaining off-diagonal part of the core is far
  // below the truncation threshold: (0.03 eps)^4 relative in squared
  // Frobenius norm (eigenvalues of the core are squared singular values)
  const double te = 0.03 * fmax(eps, floor_rel);
  const double off_rel = fmax(1e-26, te * te * te * te);
  const int64_t t_start = trace ? (int64_t)wall_clock64() : 0;
  int rounds = 0, k_first = -1, r1_first = -1, sweeps = 0;
  double fl = 0.0;   // nominal flops of the op (thread 0)
  // debug: clocks per phase (thread 0, after the phase's closing barrier)
  int64_t ph[6] = {0, 0, 0, 0, 0, 0};
  int64_t t_last = t_start;
  auto mark = [&](int i) {
    if (trace) {
      const int64_t t = (int64_t)wall_clock64();
      ph[i] += t - t_last;
      t_last = t;
    }
  };
  if (threadIdx.x == 0) {
    s_r = dims[op.slot];
    s_part = 0;
    s_pcol = 0;
    s_maxr = trunc_max_rounds(op, parts, dims);
  }
  __syncthreads();
  while (true) {
    // column list: current C columns, then part columns (trunc_rounds.h)
    if (threadIdx.x == 0) {
      TruncCursor cur{s_part, s_pcol};
      bool done = false;
      const int K = trunc_round_columns(op, parts, dims, s_r, round_cols, &cur, &done, [&](int k, int p, int c) {
        if (p < 0) {
          xs[k] = ColSrc{op.xoff + (int64_t)c * op.ldx, 1, 0, op.m, 1.0};
          ys[k] = ColSrc{op.yoff + (int64_t)c * op.ldy, 1, 0, op.n, 1.0};
        } else {
          const TruncPart P = parts[op.p0 + p];
          xs[k] = ColSrc{P.X.off + (int64_t)c * P.X.cs, P.X.rs, P.row_off, dimv(P.X.rows, dims), P.alpha};
          ys[k] = ColSrc{P.Y.off + (int64_t)c * P.Y.cs, P.Y.rs, P.col_off, dimv(P.Y.rows, dims), 1.0};
        }
      });
      s_part = cur.part;
      s_pcol = cur.col;
      s_K = K;
      s_done = done;
    }
    __syncthreads();
    const int K = s_K;
    if (K == 0) {
      if (threadIdx.x == 0) s_r = 0;
      __syncthreads();
      break;
    }
    // (1) Gy -> S buffer, Gx -> G buffer; balance every column pair so that
    // |x_a| = |y_a| (x_a y_a^T unchanged), then pivoted Cholesky of Gx -> R
    gram(arena, ys, K, op.n, bufS, bufG);
    gram(arena, xs, K, op.m, bufG, bufR);
    for (int a = threadIdx.x; a < K; a += blockDim.x) {
      const double gx = bufG[a * kLd + a], gy = bufS[a * kLd + a];
      const bool nz = gx > 0.0 && gy > 0.0;
      dscale[a] = nz ? sqrt(sqrt(gy / gx)) : 0.0;
      dinv[a] = nz ? 1.0 / dscale[a] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
      const int a = e / K, b = e % K;
      bufG[a * kLd + b] *= dscale[a] * dscale[b];
      bufS[a * kLd + b] *= dinv[a] * dinv[b];
    }
    __syncthreads();
    mark(0);
    const int r1c = pivoted_cholesky(bufG, bufR, K, tol2, piv, dvec, chosen, s_int, s_dbl);
    if (threadIdx.x == 0) s_r1 = r1c;
    __syncthreads();
    mark(1);
    if (threadIdx.x == 0) fl += 2.0 * (op.m + op.n) * K * K + (double)K * K * K / 3.0;
    const int r1 = s_r1;
    if (k_first < 0) {
      k_first = K;
      r1_first = r1;
    }
    int rnew = 0;
    if (r1 > 0) {
      // (2) T1 = Gy R^T -> G buffer; S = R T1 -> S buffer
      for (int e = threadIdx.x; e < K * r1; e += blockDim.x) {
        const int a = e / r1, k = e % r1;
        double acc = 0.0;
        for (int b = 0; b < K; ++b) acc += bufS[a * kLd + b] * bufR[k * kLd + b];
        bufG[a * kLd + k] = acc;
      }
      __syncthreads();
      for (int e = threadIdx.x; e < r1 * r1; e += blockDim.x) {
        const int k = e / r1, l = e % r1;
        double acc = 0.0;
        for (int a = 0; a < K; ++a) acc += bufR[k * kLd + a] * bufG[a * kLd + l];
        bufS[k * kLd + l] = acc;
      }
      __syncthreads();
      // symmetrise against rounding
      for (int e = threadIdx.x; e < r1 * r1; e += blockDim.x) {
        const int k = e / r1, l = e % r1;
        if (k < l) {
          const double v = 0.5 * (bufS[k * kLd + l] + bufS[l * kLd + k]);
          bufS[k * kLd + l] = v;
          bufS[l * kLd + k] = v;
        }
      }
      __syncthreads();
      // (3) eigen-decomposition of S.  S is PSD and only eigenpairs above
      // (eps sigma_1)^2 are kept, so S is first compressed by a pivoted
      // Cholesky S ~ R2^T R2 (r2 x r1) whose dropped Schur complement is far
      // below that threshold; the eigenpairs come from the small M = R2 R2^T
      // (r2 x r2): S u = lambda u with u = R2^T v / sqrt(lambda).  When the
      // compression does not pay, S (kept in the W buffer) goes to Jacobi.
      double* Sres;
      double* Free;
      for (int e = threadIdx.x; e < r1 * r1; e += blockDim.x) bufW[(e / r1) * kLd + e % r1] = bufS[(e / r1) * kLd + e % r1];
      __syncthreads();
      int r2 = r1;
      if (r1 > kCompressMin) {
        const double ts = kCompressTol * fmax(eps, floor_rel);
        r2 = pivoted_cholesky(bufS, bufG, r1, ts * ts, sel, dvec, chosen, s_int, s_dbl);
      }
      mark(2);
      if (r2 <= kKMax / 2 && r2 + 2 < r1) {
        // M = R2 R2^T in columns [0, 32) of the S buffer; Jacobi double
        // buffer in columns [32, 64); eigenvectors V -> W buffer
        for (int e = threadIdx.x; e < r2 * r2; e += blockDim.x) {
          const int k = e / r2, l = e % r2;
          double v = 0.0;
          for (int j = 0; j < r1; ++j) v += bufG[k * kLd + j] * bufG[l * kLd + j];
          bufS[k * kLd + l] = v;
        }
        __syncthreads();
        const int sw0 = sweeps;
        const double* Mres = jacobi(bufS, bufS + kKMax / 2, bufW, r2, cs, pk, pfirst, red, off_rel, &sweeps, rt);
        if (threadIdx.x == 0)
          fl += 9.0 * r2 * r2 * r2 * (sweeps - sw0) + 4.0 * r2 * r2 * r1 + (double)r1 * r1 * r1 / 3.0;
        for (int k = threadIdx.x; k < r1; k += blockDim.x) mu[k] = k < r2 ? fmax(Mres[k * kLd + k], 0.0) : 0.0;
        __syncthreads();
        // eigenvectors of S, r1 x r2 -> S buffer, then into the W buffer
        for (int e = threadIdx.x; e < r1 * r2; e += blockDim.x) {
          const int i = e / r2, c = e % r2;
          double v = 0.0;
          if (mu[c] > 0.0) {
            for (int k = 0; k < r2; ++k) v += bufG[k * kLd + i] * bufW[k * kLd + c];
            v /= sqrt(mu[c]);
          }
          bufS[i * kLd + c] = v;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < r1 * r2; e += blockDim.x) bufW[(e / r2) * kLd + e % r2] = bufS[(e / r2) * kLd + e % r2];
        __syncthreads();
        Sres = bufS;
        Free = bufG;
      } else {
        for (int e = threadIdx.x; e < r1 * r1; e += blockDim.x) bufS[(e / r1) * kLd + e % r1] = bufW[(e / r1) * kLd + e % r1];
        __syncthreads();
        const int sw0 = sweeps;
        Sres = jacobi(bufS, bufG, bufW, r1, cs, pk, pfirst, red, off_rel, &sweeps, rt);
        if (threadIdx.x == 0)
          fl += 9.0 * r1 * r1 * r1 * (sweeps - sw0) + (r1 > kCompressMin ? (double)r1 * r1 * r1 / 3.0 : 0.0);
        Free = (Sres == bufS) ? bufG : bufS;
        for (int k = threadIdx.x; k < r1; k += blockDim.x) mu[k] = fmax(Sres[k * kLd + k], 0.0);
        __syncthreads();
      }
      mark(3);
      for (int k = threadIdx.x; k < r1; k += blockDim.x) {
        int rank = 0;
        for (int l = 0; l < r1; ++l)
          if (mu[l] > mu[k] || (mu[l] == mu[k] && l < k)) ++rank;
        sel[rank] = k;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        const double s1 = sqrt(mu[sel[0]]);
        const double thr = fmax(eps, floor_rel) * s1;
        int cnt = 0;
        for (int k = 0; k < r1; ++k)
          if (sqrt(mu[sel[k]]) > thr) ++cnt;
        if (s1 == 0.0) cnt = 0;
        const int lim = trunc_rank_limit(op, s_done != 0, round_cols);
        const int r = cnt < lim ? cnt : lim;
        if (cnt > lim) atomicAdd(&status[1], 1);
        if (peak) atomicMax(&peak[op.slot], cnt);   // the eps-rank asked for, before any cap
        s_r = r;
      }
      __syncthreads();
      rnew = s_r;
      if (threadIdx.x == 0)
        fl += 2.0 * K * K * r1 + 2.0 * r1 * r1 * K + (double)r1 * r1 * rnew + 2.0 * K * r1 * rnew +
              2.0 * op.m * r1 * rnew + 2.0 * op.n * K * rnew;
      // (4) Z = R11^{-1} W_r (r1 x rnew) -> Free ; Ty = R^T W_r (K x rnew) -> Sres.
      // R11 (R's pivot columns, upper triangular) is first copied to Sres,
      // which is free until Ty is written
      for (int e = threadIdx.x; e < r1 * r1; e += blockDim.x) {
        const int k = e / r1, l = e % r1;
        if (l >= k) Sres[k * kLd + l] = bufR[k * kLd + piv[l]];
      }
      __syncthreads();
      for (int c = threadIdx.x; c < rnew; c += blockDim.x) {
        const int ev = sel[c];
        for (int k = r1 - 1; k >= 0; --k) {
          double v = bufW[k * kLd + ev];
          for (int l = k + 1; l < r1; ++l) v -= Sres[k * kLd + l] * Free[l * kLd + c];
          Free[k * kLd + c] = v / Sres[k * kLd + k];
        }
      }
      __syncthreads();
      for (int e = threadIdx.x; e < K * rnew; e += blockDim.x) {
        const int a = e / rnew, c = e % rnew;
        const int ev = sel[c];
        double v = 0.0;
        for (int k = 0; k < r1; ++k) v += bufR[k * kLd + a] * bufW[k * kLd + ev];
        Sres[a * kLd + c] = v;
      }
      __syncthreads();
      mark(4);
      // (5) X_C = Xa[:, piv] Z ; Y_C = Ya Ty (row tiles staged in the R buffer)
      for (int pass = 0; pass < 2; ++pass) {
        const ColSrc* src = pass == 0 ? xs : ys;
        const int mrows = pass == 0 ? op.m : op.n;
        const int64_t out = pass == 0 ? op.xoff : op.yoff;
        const int ldo = pass == 0 ? op.ldx : op.ldy;
        const int nk = pass == 0 ? r1 : K;
        for (int i0 = 0; i0 < mrows; i0 += kKMax) {
          load_tile(arena, src, K, i0, kKMax, mrows, bufR);
          __syncthreads();
          const int rt = min(kKMax, mrows - i0);
          // the tile's columns in product order, scaled: X_a[:, piv[k]] dscale[piv[k]]
          // (pass 0) or Y_a[:, a] dinv[a] (pass 1), into the free W buffer
          for (int e = threadIdx.x; e < rt * nk; e += blockDim.x) {
            const int i = e % rt, k = e / rt;
            bufW[i * kLd + k] = pass == 0 ? bufR[i * kLd + piv[k]] * dscale[piv[k]] : bufR[i * kLd + k] * dinv[k];
          }
          __syncthreads();
          const double* F = pass == 0 ? Free : Sres;
          for (int e = threadIdx.x; e < rt * rnew; e += blockDim.x) {
            const int i = e % rt, c = e / rt;
            double v = 0.0;
            for (int k = 0; k < nk; ++k) v += bufW[i * kLd + k] * F[k * kLd + c];
            arena[out + (i0 + i) + (int64_t)c * ldo] = T(v);
          }
          __syncthreads();
        }
      }
      mark(5);
    } else if (threadIdx.x == 0) {
      s_r = 0;
    }
    __syncthreads();
    ++rounds;
    if (s_done) break;
    if (rounds >= s_maxr) {   // unreachable by the round structure; reported, never spun on
      if (threadIdx.x == 0) atomicAdd(&status[2], 1);
      break;
    }
  }
  if (threadIdx.x == 0) {
    dims[op.slot] = s_r;
    add_flops(status, kFlopTrunc, fl);
  }
  if (trace && threadIdx.x == 0) {   // debug: per-op size and clocks
    int64_t* t = trace + kTruncTraceFields * ((int64_t)op_base + blockIdx.x);
    t[0] = op.m;
    t[1] = op.n;
    t[2] = rounds | ((int64_t)(k_first & 0xfff) << 8) | ((int64_t)(r1_first & 0xfff) << 20);
    t[3] = s_r | ((int64_t)sweeps << 16);
    t[4] = t_start;
    t[5] = (int64_t)wall_clock64();
    for (int i = 0; i < 6; ++i) t[6 + i] = ph[i];
  }
}

}  // namespace dev

// ------------------------------------------------------------ launchers

// Debug (HLU_DEBUG_TRUNC_TRACE): per truncation op of a factor plan, the
// block size, rounds, final rank and clocks.  Allocated on first use.
constexpr int64_t kTruncTraceOps = 12 << 20;
int64_t* trunc_trace_buffer(size_t* ops) {
  static int64_t* buf = nullptr;
  static std::once_flag tried;
  std::call_once(tried, [] {
    if (getenv("HLU_DEBUG_TRUNC_TRACE") &&
        hipMalloc(&buf, (size_t)kTruncTraceOps * kTruncTraceFields * sizeof(int64_t)) != hipSuccess)
      buf = nullptr;
  });
  if (ops) *ops = (size_t)kTruncTraceOps;
  return buf;
}

// Columns of one truncation round: kTruncCols, or fewer with
// HLU_DEBUG_TRUNC_COLS (2..64), which the tests use to force blocks to the
// round's width while parts remain (the rank-overflow path).
int trunc_round_cols() {
  const char* e = getenv("HLU_DEBUG_TRUNC_COLS");
  if (!e) return kTruncCols;
  const int c = atoi(e);
  return c < 2 ? 2 : (c > kTruncCols ? kTruncCols : c);
}

template <class T, class C>
hipError_t launch_wave_c(T* arena, const DevPlan& P, const Wave& w, int32_t* dims, int32_t* status,
                         double eps, double floor_rel, int32_t max_leaf, int32_t tile_base,
                         hipStream_t s, int32_t* peak, int part) {
  static std::once_flag attrs_set;   // launchers run on several server threads
  std::call_once(attrs_set, [] {
    // allow dynamic LDS up to the 160 KB of a gfx950 CU
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&dev::getrf_kernel<T, C>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)dev::kLdsBytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&dev::tri_kernel<T, C>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)dev::kLdsBytes);
  });
  const bool rest = part != kWaveTruncOnly, trunc = part != kWaveNoTrunc;
  if (rest && w.count[kFill] > 0) {
    dim3 g(64, w.count[kFill]);
    dev::fill_kernel<T><<<g, 256, 0, s>>>(arena, P.fill + w.begin[kFill], dims);
  }
  if (rest && w.count[kGetrf] > 0) {
    const size_t sh = (size_t)max_leaf * max_leaf * sizeof(C);
    dev::getrf_kernel<T, C><<<w.count[kGetrf], 256, sh, s>>>(arena, P.getrf + w.begin[kGetrf], status);
  }
  if (rest && w.count[kTri] > 0) {
    const size_t tri_bytes = (size_t)max_leaf * max_leaf * sizeof(C);
    int cols = (int)((dev::kLdsBytes - tri_bytes) / ((size_t)max_leaf * sizeof(C)));
    cols = cols > dev::kTriMaxCols ? dev::kTriMaxCols : cols;
    const size_t sh = tri_bytes + (size_t)max_leaf * cols * sizeof(C);
    dev::tri_kernel<T, C><<<w.count[kTri], 256, sh, s>>>(arena, P.tri + w.begin[kTri], dims, cols, status);
  }
  if (rest && w.gemm_tiles > 0) {
    dev::gemm_kernel<T, C><<<w.gemm_tiles, 256, 0, s>>>(arena, P.gemm, P.terms, P.tile_op, P.tile_ij,
                                                      tile_base, dims, status);
  }
  if (trunc && w.count[kTrunc] > 0) {
    int64_t* tr = trunc_trace_buffer(nullptr);
    if (tr && w.begin[kTrunc] + w.count[kTrunc] > kTruncTraceOps) tr = nullptr;
    dev::trunc_kernel<T><<<w.count[kTrunc], 256, 0, s>>>(arena, P.trunc + w.begin[kTrunc], P.parts, dims,
                                                          eps, floor_rel, status, tr, w.begin[kTrunc],
                                                          trunc_round_cols(), peak);
  }
  return hipGetLastError();
}

// T: storage type of the factors; compute64: do the arithmetic of the dense
// tasks in FP64 (always the case for FP64 storage).
template <class T>
hipError_t launch_wave(T* arena, const DevPlan& P, const Wave& w, int32_t* dims, int32_t* status,
                       double eps, double floor_rel, int32_t max_leaf, int32_t tile_base, bool compute64,
                       hipStream_t s, int32_t* peak, int part) {
  if (compute64)
    return launch_wave_c<T, double>(arena, P, w, dims, status, eps, floor_rel, max_leaf, tile_base, s, peak, part);
  return launch_wave_c<T, T>(arena, P, w, dims, status, eps, floor_rel, max_leaf, tile_base, s, peak, part);
}

template hipError_t launch_wave<float>(float*, const DevPlan&, const Wave&, int32_t*, int32_t*, double,
                                       double, int32_t, int32_t, bool, hipStream_t, int32_t*, int);
template hipError_t launch_wave<double>(double*, const DevPlan&, const Wave&, int32_t*, int32_t*, double,
                                        double, int32_t, int32_t, bool, hipStream_t, int32_t*, int);

WaveStreams::~WaveStreams() {
  if (fork) (void)hipEventDestroy(fork);
  if (join) (void)hipEventDestroy(join);
  if (aux) (void)hipStreamDestroy(aux);
}

template <class T>
hipError_t run_waves(T* arena, const DevPlan& P, const std::vector<Wave>& waves, int32_t* dims, int32_t* status,
                     double eps, double floor_rel, int32_t max_leaf, bool compute64, hipStream_t s, int32_t* peak,
                     WaveStreams* ws) {
  int32_t tile_base = 0;
  for (const Wave& w : waves) {
    const bool has_t = w.count[kTrunc] > 0;
    const bool has_o = w.count[kFill] + w.count[kGetrf] + w.count[kTri] > 0 || w.gemm_tiles > 0;
    hipError_t e;
    if (ws && has_t && has_o) {
      // the tasks of one wave touch disjoint data (the planner's invariant):
      // the truncations run on the second stream beside the other kinds,
      // and both streams meet again before the next wave
      if (!ws->aux) {   // created together, kept only when all three exist
        hipStream_t aux = nullptr;
        hipEvent_t fork = nullptr, join = nullptr;
        e = hipStreamCreateWithFlags(&aux, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
        if (e != hipSuccess) {
          if (join) (void)hipEventDestroy(join);
          if (fork) (void)hipEventDestroy(fork);
          if (aux) (void)hipStreamDestroy(aux);
          return e;
        }
        ws->aux = aux;
        ws->fork = fork;
        ws->join = join;
      }
      if ((e = hipEventRecord(ws->fork, s)) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(ws->aux, ws->fork, 0)) != hipSuccess) return e;
      if ((e = launch_wave<T>(arena, P, w, dims, status, eps, floor_rel, max_leaf, tile_base, compute64, s, peak,
                              kWaveNoTrunc)) != hipSuccess)
        return e;
      if ((e = launch_wave<T>(arena, P, w, dims, status, eps, floor_rel, max_leaf, tile_base, compute64, ws->aux,
                              peak, kWaveTruncOnly)) != hipSuccess)
        return e;
      if ((e = hipEventRecord(ws->join, ws->aux)) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(s, ws->join, 0)) != hipSuccess) return e;
    } else if ((e = launch_wave<T>(arena, P, w, dims, status, eps, floor_rel, max_leaf, tile_base, compute64, s,
                                   peak)) != hipSuccess) {
      return e;
    }
    tile_base += w.gemm_tiles;
  }
  return hipSuccess;
}

template hipError_t run_waves<float>(float*, const DevPlan&, const std::vector<Wave>&, int32_t*, int32_t*, double,
                                     double, int32_t, bool, hipStream_t, int32_t*, WaveStreams*);
template hipError_t run_waves<double>(double*, const DevPlan&, const std::vector<Wave>&, int32_t*, int32_t*, double,
                                      double, int32_t, bool, hipStream_t, int32_t*, WaveStreams*);

}  // namespace hlu
