// Batched task kernels of the H-LU factorisation, H-solves and L U product
// for gfx950.  Each launch runs the tasks of one kind from one wave of a
// plan; tasks of a wave touch disjoint data.  T is the storage and
// arithmetic type of the factors (float or double); the small dense algebra
// inside the truncation is always FP64.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.h"

namespace hlu {
namespace dev {

__device__ __forceinline__ int dimv(int32_t code, const int32_t* dims) {
  return code >= 0 ? code : dims[-code - 1];
}

template <class T>
__device__ __forceinline__ T& at(T* base, const MatRef& m, int i, int j) {
  return base[m.off + (int64_t)i * m.rs + (int64_t)j * m.cs];
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
                                                  int tri_cols) {
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
}

// ---------------------------------------------------------------- GEMM
// One 64 x 64 output tile per workgroup: C = beta C + sum_t alpha_t A_t B_t,
// operands of any strides, k streamed through LDS in chunks of 16; each of
// the 256 threads accumulates a 4 x 4 sub-tile.
constexpr int kGT = 64, kGK = 16;

template <class T, class C>
__global__ void __launch_bounds__(256) gemm_kernel(T* arena, const GemmOp* ops, const GemmTerm* terms,
                                                   const int32_t* tile_op, const int32_t* tile_ij,
                                                   int32_t tile0, const int32_t* dims) {
  __shared__ C As[kGK][kGT + 1];
  __shared__ C Bs[kGK][kGT + 1];
  const int tile = tile0 + blockIdx.x;
  const GemmOp op = ops[tile_op[tile]];
  const int ti = tile_ij[tile] >> 16, tj = tile_ij[tile] & 0xffff;
  const int M = dimv(op.C.rows, dims), N = dimv(op.C.cols, dims);
  const int i0 = ti * kGT, j0 = tj * kGT;
  if (i0 >= M || j0 >= N) return;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  C acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = C(0);
  for (int t = 0; t < op.nt; ++t) {
    const GemmTerm tm = terms[op.t0 + t];
    const int K = dimv(tm.A.cols, dims);
    const C alpha = C(tm.alpha);
    C part[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) part[a][b] = C(0);
    for (int k0 = 0; k0 < K; k0 += kGK) {
      for (int e = threadIdx.x; e < kGK * kGT; e += 256) {
        // A tile: rows i0.., cols k0..; index so that consecutive threads
        // walk the unit-stride dimension of A when possible
        int r, c;
        if (tm.A.rs == 1) { r = e % kGT; c = e / kGT; } else { c = e % kGK; r = e / kGK; }
        const int gi = i0 + r, gk = k0 + c;
        As[c][r] = (gi < M && gk < K) ? C(at(arena, tm.A, gi, gk)) : C(0);
        int r2, c2;
        if (tm.B.cs == 1) { c2 = e % kGT; r2 = e / kGT; } else { r2 = e % kGK; c2 = e / kGK; }
        const int bk = k0 + r2, bj = j0 + c2;
        Bs[r2][c2] = (bk < K && bj < N) ? C(at(arena, tm.B, bk, bj)) : C(0);
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < kGK; ++kk) {
        C av[4], bv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) av[a] = As[kk][ty + 16 * a];
#pragma unroll
        for (int b = 0; b < 4; ++b) bv[b] = Bs[kk][tx + 16 * b];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) part[a][b] += av[a] * bv[b];
      }
      __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] += alpha * part[a][b];
  }
  const C beta = C(op.beta);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int gi = i0 + ty + 16 * a, gj = j0 + tx + 16 * b;
      if (gi < M && gj < N) {
        T& c = at(arena, op.C, gi, gj);
        c = T((op.beta == 0.0 ? C(0) : beta * C(c)) + acc[a][b]);
      }
    }
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
// workgroup per task.  With Xa = [X_C, parts], Ya = [Y_C, parts] (K columns):
//   G = Xa^T Xa = V diag(lambda) V^T                 (Jacobi, LDS)
//   S = diag(s) V^T (Ya^T Ya) V diag(s), s = sqrt(lambda)
//     = W diag(sigma^2) W^T                          (Jacobi, LDS)
// sigma are the singular values of Xa Ya^T.  Keep the r leading ones with
// sigma_i > max(eps, floor) sigma_1, r <= capacity, and write
//   X_C = Xa V diag(1/s) W_r,  Y_C = Ya V diag(s) W_r,
// so X_C Y_C^T is the best rank-r approximation of Xa Ya^T.  More than
// kKMax columns are absorbed in chunks, truncating after each chunk.
constexpr int kKMax = 78;   // three (kKMax x kKMax+1) FP64 buffers fit the 160 KB LDS
constexpr int kLd = kKMax + 1;

struct ColSrc {
  int64_t off;     // column 0 element of the source (already offset by column)
  int32_t rs;      // row stride of the source
  int32_t row_off; // first row of C covered
  int32_t rows;    // rows covered
  double alpha;
};

template <class T>
__device__ void load_tile(const T* arena, const ColSrc* src, int K, int i0, int RT, int mrows,
                          double* tile) {
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

// Gram matrix of the K source columns over mrows rows into G (K x K, ld kLd),
// staging row tiles in stage (at least kKMax * kLd doubles).
template <class T>
__device__ void gram(const T* arena, const ColSrc* src, int K, int mrows, double* G, double* stage) {
  const int RT = kKMax;
  const int npairs = K * (K + 1) / 2;
  // each thread owns pairs e = tid, tid + 256, ...  (at most 13 for K <= 80)
  double acc[14];
#pragma unroll
  for (int q = 0; q < 14; ++q) acc[q] = 0.0;
  for (int i0 = 0; i0 < mrows; i0 += RT) {
    load_tile(arena, src, K, i0, RT, mrows, stage);
    __syncthreads();
    const int rt = min(RT, mrows - i0);
#pragma unroll
    for (int q = 0; q < 14; ++q) {
      const int e = threadIdx.x + q * 256;
      if (e < npairs) {
        // map e -> (a, b), a <= b
        int a = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while ((a + 1) * (a + 2) / 2 <= e) ++a;
        while (a * (a + 1) / 2 > e) --a;
        const int b = e - a * (a + 1) / 2;   // b <= a
        double s = 0.0;
        for (int i = 0; i < rt; ++i) s += stage[i * kLd + a] * stage[i * kLd + b];
        acc[q] += s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 14; ++q) {
    const int e = threadIdx.x + q * 256;
    if (e < npairs) {
      int a = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
      while ((a + 1) * (a + 2) / 2 <= e) ++a;
      while (a * (a + 1) / 2 > e) --a;
      const int b = e - a * (a + 1) / 2;
      G[a * kLd + b] = acc[q];
      G[b * kLd + a] = acc[q];
    }
  }
  __syncthreads();
}

// Cyclic parallel Jacobi on the symmetric K x K matrix A (ld kLd, LDS).
// Rotations are also applied to the columns of U1 (and U2 if not null).
// Round-robin pairing: K is padded to an even Kp with inert indices.
__device__ void jacobi_eig(double* A, int K, double* U1, double* U2, double* cs_buf, double* red) {
  const int Kp = K + (K & 1);
  const int npair = Kp / 2;
  for (int sweep = 0; sweep < 30; ++sweep) {
    // convergence test: off-diagonal vs total Frobenius norm
    double off = 0.0, tot = 0.0;
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
      const int i = e / K, j = e % K;
      const double v = A[i * kLd + j];
      tot += v * v;
      if (i != j) off += v * v;
    }
    // block reduction
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
    if (tots == 0.0 || offs <= 1e-26 * tots) break;
    for (int r = 0; r < Kp - 1; ++r) {
      // rotation parameters for the pairs of this round
      for (int k = threadIdx.x; k < npair; k += blockDim.x) {
        int p, q;
        if (k == 0) {
          p = Kp - 1;
          q = r;
        } else {
          p = (r + k) % (Kp - 1);
          q = (r - k + Kp - 1) % (Kp - 1);
        }
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        double c = 1.0, s = 0.0;
        if (q < K) {
          const double apq = A[p * kLd + q];
          const double app = A[p * kLd + p], aqq = A[q * kLd + q];
          if (fabs(apq) > 1e-17 * sqrt(fabs(app * aqq)) && apq != 0.0) {
            const double th = (A[q * kLd + q] - A[p * kLd + p]) / (2.0 * apq);
            const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        cs_buf[4 * k + 0] = c;
        cs_buf[4 * k + 1] = s;
        cs_buf[4 * k + 2] = p;
        cs_buf[4 * k + 3] = q;
      }
      __syncthreads();
      // columns of A
      for (int e = threadIdx.x; e < npair * K; e += blockDim.x) {
        const int k = e / K, row = e % K;
        const int p = (int)cs_buf[4 * k + 2], q = (int)cs_buf[4 * k + 3];
        if (q >= K) continue;
        const double c = cs_buf[4 * k], s = cs_buf[4 * k + 1];
        const double ap = A[row * kLd + p], aq = A[row * kLd + q];
        A[row * kLd + p] = c * ap - s * aq;
        A[row * kLd + q] = s * ap + c * aq;
      }
      __syncthreads();
      // rows of A, and columns of U1/U2
      for (int e = threadIdx.x; e < npair * K; e += blockDim.x) {
        const int k = e / K, col = e % K;
        const int p = (int)cs_buf[4 * k + 2], q = (int)cs_buf[4 * k + 3];
        if (q >= K) continue;
        const double c = cs_buf[4 * k], s = cs_buf[4 * k + 1];
        const double ap = A[p * kLd + col], aq = A[q * kLd + col];
        A[p * kLd + col] = c * ap - s * aq;
        A[q * kLd + col] = s * ap + c * aq;
        const double u1p = U1[col * kLd + p], u1q = U1[col * kLd + q];
        U1[col * kLd + p] = c * u1p - s * u1q;
        U1[col * kLd + q] = s * u1p + c * u1q;
        if (U2) {
          const double u2p = U2[col * kLd + p], u2q = U2[col * kLd + q];
          U2[col * kLd + p] = c * u2p - s * u2q;
          U2[col * kLd + q] = s * u2p + c * u2q;
        }
      }
      __syncthreads();
    }
  }
}

template <class T>
__global__ void __launch_bounds__(256) trunc_kernel(T* arena, const TruncOp* ops, const TruncPart* parts,
                                                    int32_t* dims, double eps, double floor_rel,
                                                    int32_t* status) {
  __shared__ double bufA[kKMax * kLd];
  __shared__ double bufB[kKMax * kLd];
  __shared__ double bufC[kKMax * kLd];
  __shared__ ColSrc xs[kKMax], ys[kKMax];
  __shared__ double lam[kKMax], sq[kKMax], mu[kKMax];
  __shared__ double cs_buf[4 * (kKMax / 2 + 1)];
  __shared__ double red[8];
  __shared__ int sel[kKMax];
  __shared__ int s_K, s_r, s_part, s_pcol, s_done;

  const TruncOp op = ops[blockIdx.x];
  if (threadIdx.x == 0) {
    s_r = dims[op.slot];
    s_part = 0;
    s_pcol = 0;
  }
  __syncthreads();
  while (true) {
    // assemble the column list: current C columns, then up to kKMax - r part columns
    if (threadIdx.x == 0) {
      int K = 0;
      const int r = s_r;
      for (int a = 0; a < r; ++a) {
        xs[K] = ColSrc{op.xoff + (int64_t)a * op.ldx, 1, 0, op.m, 1.0};
        ys[K] = ColSrc{op.yoff + (int64_t)a * op.ldy, 1, 0, op.n, 1.0};
        ++K;
      }
      int p = s_part, c = s_pcol;
      while (p < op.np && K < kKMax) {
        const TruncPart P = parts[op.p0 + p];
        const int kp = dimv(P.X.cols, dims);
        if (c >= kp) {
          ++p;
          c = 0;
          continue;
        }
        xs[K] = ColSrc{P.X.off + (int64_t)c * P.X.cs, P.X.rs, P.row_off, dimv(P.X.rows, dims), P.alpha};
        ys[K] = ColSrc{P.Y.off + (int64_t)c * P.Y.cs, P.Y.rs, P.col_off, dimv(P.Y.rows, dims), 1.0};
        ++K;
        ++c;
      }
      // skip exhausted parts
      while (p < op.np && c >= dimv(parts[op.p0 + p].X.cols, dims)) {
        ++p;
        c = 0;
      }
      s_part = p;
      s_pcol = c;
      s_K = K;
      s_done = (p >= op.np);
    }
    __syncthreads();
    const int K = s_K;
    if (K == 0) {
      if (threadIdx.x == 0) s_r = 0;
      __syncthreads();
      break;
    }
    // (1) G = Xa^T Xa -> A ; V -> B
    gram(arena, xs, K, op.m, bufA, bufC);
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
      const int i = e / K, j = e % K;
      bufB[i * kLd + j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    jacobi_eig(bufA, K, bufB, nullptr, cs_buf, red);
    if (threadIdx.x == 0) {
      double lmax = 0.0;
      for (int a = 0; a < K; ++a) lmax = fmax(lmax, bufA[a * kLd + a]);
      for (int a = 0; a < K; ++a) {
        const double l = bufA[a * kLd + a];
        lam[a] = l;
        sq[a] = (l > 1e-15 * K * lmax && l > 0.0) ? sqrt(l) : 0.0;
      }
    }
    __syncthreads();
    // (2) Gy -> A, C = Gy V, A = V^T C, scaled by sq
    gram(arena, ys, K, op.n, bufA, bufC);
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
      const int i = e / K, j = e % K;
      double s = 0.0;
      for (int c = 0; c < K; ++c) s += bufA[i * kLd + c] * bufB[c * kLd + j];
      bufC[i * kLd + j] = s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
      const int i = e / K, j = e % K;
      double s = 0.0;
      for (int c = 0; c < K; ++c) s += bufB[c * kLd + i] * bufC[c * kLd + j];
      bufA[i * kLd + j] = sq[i] * s * sq[j];
    }
    __syncthreads();
    // (3) U1 = V diag(1/s) -> C, U2 = V diag(s) -> B (in place)
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
      const int i = e / K, j = e % K;
      const double v = bufB[i * kLd + j];
      bufC[i * kLd + j] = sq[j] > 0.0 ? v / sq[j] : 0.0;
      bufB[i * kLd + j] = v * sq[j];
    }
    __syncthreads();
    jacobi_eig(bufA, K, bufC, bufB, cs_buf, red);
    // (4) order the eigenvalues of S, choose the rank
    for (int a = threadIdx.x; a < K; a += blockDim.x) mu[a] = fmax(bufA[a * kLd + a], 0.0);
    __syncthreads();
    for (int a = threadIdx.x; a < K; a += blockDim.x) {
      int rank = 0;
      for (int b = 0; b < K; ++b)
        if (mu[b] > mu[a] || (mu[b] == mu[a] && b < a)) ++rank;
      sel[rank] = a;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const double s1 = sqrt(mu[sel[0]]);
      const double thr = fmax(eps, floor_rel) * s1;
      int cnt = 0;
      for (int a = 0; a < K; ++a)
        if (sqrt(mu[sel[a]]) > thr) ++cnt;
      if (s1 == 0.0) cnt = 0;
      int r = cnt < op.cap ? cnt : op.cap;
      if (cnt > op.cap) atomicAdd(&status[1], 1);
      s_r = r;
    }
    __syncthreads();
    const int rnew = s_r;
    // (5) X_C = Xa U1[:, sel], Y_C = Ya U2[:, sel], row tiles staged in A
    for (int pass = 0; pass < 2; ++pass) {
      const ColSrc* src = pass == 0 ? xs : ys;
      const int mrows = pass == 0 ? op.m : op.n;
      const double* U = pass == 0 ? bufC : bufB;
      const int64_t out = pass == 0 ? op.xoff : op.yoff;
      const int ldo = pass == 0 ? op.ldx : op.ldy;
      for (int i0 = 0; i0 < mrows; i0 += kKMax) {
        load_tile(arena, src, K, i0, kKMax, mrows, bufA);
        __syncthreads();
        const int rt = min(kKMax, mrows - i0);
        for (int e = threadIdx.x; e < rt * rnew; e += blockDim.x) {
          const int i = e % rt, j = e / rt;
          const int col = sel[j];
          double s = 0.0;
          for (int a = 0; a < K; ++a) s += bufA[i * kLd + a] * U[a * kLd + col];
          arena[out + (i0 + i) + (int64_t)j * ldo] = T(s);
        }
        __syncthreads();
      }
    }
    __syncthreads();
    if (s_done) break;
  }
  if (threadIdx.x == 0) dims[op.slot] = s_r;
}

}  // namespace dev

// ------------------------------------------------------------ launchers

template <class T, class C>
hipError_t launch_wave_c(T* arena, const DevPlan& P, const Wave& w, int32_t* dims, int32_t* status,
                         double eps, double floor_rel, int32_t max_leaf, int32_t tile_base,
                         hipStream_t s) {
  static bool attrs_set = false;
  if (!attrs_set) {
    // allow dynamic LDS up to the 160 KB of a gfx950 CU
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&dev::getrf_kernel<T, C>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)dev::kLdsBytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&dev::tri_kernel<T, C>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)dev::kLdsBytes);
    attrs_set = true;
  }
  if (w.count[kFill] > 0) {
    dim3 g(64, w.count[kFill]);
    dev::fill_kernel<T><<<g, 256, 0, s>>>(arena, P.fill + w.begin[kFill], dims);
  }
  if (w.count[kGetrf] > 0) {
    const size_t sh = (size_t)max_leaf * max_leaf * sizeof(C);
    dev::getrf_kernel<T, C><<<w.count[kGetrf], 256, sh, s>>>(arena, P.getrf + w.begin[kGetrf], status);
  }
  if (w.count[kTri] > 0) {
    const size_t tri_bytes = (size_t)max_leaf * max_leaf * sizeof(C);
    int cols = (int)((dev::kLdsBytes - tri_bytes) / ((size_t)max_leaf * sizeof(C)));
    cols = cols > dev::kTriMaxCols ? dev::kTriMaxCols : cols;
    const size_t sh = tri_bytes + (size_t)max_leaf * cols * sizeof(C);
    dev::tri_kernel<T, C><<<w.count[kTri], 256, sh, s>>>(arena, P.tri + w.begin[kTri], dims, cols);
  }
  if (w.gemm_tiles > 0) {
    dev::gemm_kernel<T, C><<<w.gemm_tiles, 256, 0, s>>>(arena, P.gemm, P.terms, P.tile_op, P.tile_ij,
                                                      tile_base, dims);
  }
  if (w.count[kTrunc] > 0) {
    dev::trunc_kernel<T><<<w.count[kTrunc], 256, 0, s>>>(arena, P.trunc + w.begin[kTrunc], P.parts, dims,
                                                          eps, floor_rel, status);
  }
  return hipGetLastError();
}

// T: storage type of the factors; compute64: do the arithmetic of the dense
// tasks in FP64 (always the case for FP64 storage).
template <class T>
hipError_t launch_wave(T* arena, const DevPlan& P, const Wave& w, int32_t* dims, int32_t* status,
                       double eps, double floor_rel, int32_t max_leaf, int32_t tile_base, bool compute64,
                       hipStream_t s) {
  if (compute64)
    return launch_wave_c<T, double>(arena, P, w, dims, status, eps, floor_rel, max_leaf, tile_base, s);
  return launch_wave_c<T, T>(arena, P, w, dims, status, eps, floor_rel, max_leaf, tile_base, s);
}

template hipError_t launch_wave<float>(float*, const DevPlan&, const Wave&, int32_t*, int32_t*, double,
                                       double, int32_t, int32_t, bool, hipStream_t);
template hipError_t launch_wave<double>(double*, const DevPlan&, const Wave&, int32_t*, int32_t*, double,
                                        double, int32_t, int32_t, bool, hipStream_t);

}  // namespace hlu
