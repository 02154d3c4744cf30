// Vector kernels: CSR SpMV of A (FP64), permutation/cast between the natural
// and the cluster order, scatter of A into the H-matrix arena, and the
// reductions and updates of GMRES (FP64).
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hlu {
namespace dev {

// Y = alpha A X + beta Y, nrhs columns.  One 64-lane wavefront per row
// group: each lane takes one nonzero, the row sum is a wavefront reduction;
// rows with more than 64 entries loop.
template <int RHS>
__global__ void __launch_bounds__(256) spmv_kernel(int32_t n, const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ ci,
                                                   const double* __restrict__ val,
                                                   const double* __restrict__ x, double* __restrict__ y,
                                                   int32_t nrhs, int64_t ld, double alpha, double beta) {
  // 4 rows per wavefront: 16 lanes per row (rows hold 7..27 entries)
  const int lane = threadIdx.x & 15;
  const int row = (blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  if (row >= n) return;
  const int p0 = rp[row], p1 = rp[row + 1];
  for (int c0 = 0; c0 < nrhs; c0 += RHS) {
    double s[RHS];
#pragma unroll
    for (int c = 0; c < RHS; ++c) s[c] = 0.0;
    for (int p = p0 + lane; p < p1; p += 16) {
      const double a = val[p];
      const int j = ci[p];
#pragma unroll
      for (int c = 0; c < RHS; ++c)
        if (c0 + c < nrhs) s[c] += a * x[j + (int64_t)(c0 + c) * ld];
    }
#pragma unroll
    for (int c = 0; c < RHS; ++c) {
      double v = s[c];
      v += __shfl_xor(v, 8, 16);
      v += __shfl_xor(v, 4, 16);
      v += __shfl_xor(v, 2, 16);
      v += __shfl_xor(v, 1, 16);
      s[c] = v;
    }
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < RHS; ++c)
        if (c0 + c < nrhs) {
          double* yy = y + row + (int64_t)(c0 + c) * ld;
          *yy = (beta == 0.0 ? 0.0 : beta * *yy) + alpha * s[c];
        }
    }
  }
}

// dst[i + c*ldd] = T(src[perm[i] + c*lds])  (natural -> cluster order)
template <class T>
__global__ void gather_kernel(int32_t n, int32_t nrhs, const int32_t* __restrict__ perm,
                              const double* __restrict__ src, int64_t lds, T* __restrict__ dst, int64_t ldd) {
  const int64_t total = (int64_t)n * nrhs;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), c = (int)(e / n);
    dst[i + c * ldd] = T(src[perm[i] + c * lds]);
  }
}

// dst[perm[i] + c*ldd] = double(src[i + c*lds])  (cluster -> natural order)
template <class T>
__global__ void scatter_perm_kernel(int32_t n, int32_t nrhs, const int32_t* __restrict__ perm,
                                    const T* __restrict__ src, int64_t lds, double* __restrict__ dst,
                                    int64_t ldd) {
  const int64_t total = (int64_t)n * nrhs;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), c = (int)(e / n);
    dst[perm[i] + c * ldd] = double(src[i + c * lds]);
  }
}

// arena[target[e]] = T(val[e]) for every stored entry of A
template <class T>
__global__ void scatter_values_kernel(int64_t nnz, const int64_t* __restrict__ target,
                                      const double* __restrict__ val, T* __restrict__ arena) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
    arena[target[e]] = T(val[e]);
}

// arena[target[e] + shift] = T(scale * val[e]): a scaled copy of A in
// another H-matrix of the same layout
template <class T>
__global__ void scatter_values_scaled_kernel(int64_t nnz, const int64_t* __restrict__ target, int64_t shift,
                                             double scale, const double* __restrict__ val, T* __restrict__ arena) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
    arena[target[e] + shift] = T(scale * val[e]);
}

// part[2 b], part[2 b + 1] = sum over block b's fixed range of (v - u)^2 and
// v^2 (tree order fixed by the thread index); then one block adds the
// partial sums in order: out = {||v - u||^2, ||v||^2}, deterministic.
constexpr int kNormBlocks = 256;
template <class T>
__global__ void __launch_bounds__(256) diff_norm_kernel(int64_t n, const T* __restrict__ v, const T* __restrict__ u,
                                                        double* __restrict__ part) {
  __shared__ double sd[256], sv[256];
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t e0 = blockIdx.x * chunk, e1 = e0 + chunk < n ? e0 + chunk : n;
  double d = 0.0, w = 0.0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const double a = double(v[e]), b = double(u[e]);
    d += (a - b) * (a - b);
    w += a * a;
  }
  sd[threadIdx.x] = d;
  sv[threadIdx.x] = w;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      sd[threadIdx.x] += sd[threadIdx.x + o];
      sv[threadIdx.x] += sv[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sd[0];
    part[2 * blockIdx.x + 1] = sv[0];
  }
}
__global__ void finish_norm_kernel(int nb, const double* __restrict__ part, double* __restrict__ out) {
  if (threadIdx.x == 0) {
    double d = 0.0, w = 0.0;
    for (int b = 0; b < nb; ++b) {
      d += part[2 * b];
      w += part[2 * b + 1];
    }
    out[0] = d;
    out[1] = w;
  }
}

template <class T>
__global__ void zero_kernel(T* __restrict__ p, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    p[e] = T(0);
}

template <class T>
__global__ void identity_kernel(T* __restrict__ p, int32_t n) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += gridDim.x * blockDim.x)
    p[e] = (e % n == e / n) ? T(1) : T(0);
}

__global__ void set_int_kernel(int32_t* p, int32_t v) { *p = v; }

__global__ void zero_int_kernel(int32_t* p, int32_t n) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) p[e] = 0;
}

// ---------------------------------------------------------------- GMRES
// Every GMRES vector block holds nseg independent segments: segment c is
// [off[c], off[c] + len[c]) (a column of one system, or one problem of a
// batch).  Kernels run a grid (x, c): blockIdx.y picks the segment.
constexpr int kDotBlocks = 256;

// part[blk][i][c] = sum over block blk's share of segment c of V_i w
__global__ void __launch_bounds__(256) seg_dot_kernel(int32_t nseg, const int64_t* __restrict__ off,
                                                      const int64_t* __restrict__ len, int32_t nv,
                                                      const double* __restrict__ V, int64_t vstride,
                                                      const double* __restrict__ w, double* __restrict__ part) {
  __shared__ double red[4];
  const int c = blockIdx.y;
  const int64_t o = off[c], n = len[c];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = blockIdx.x * per, r1 = min(n, r0 + per);
  for (int i = 0; i < nv; ++i) {
    const double* v = V + i * vstride + o;
    const double* ww = w + o;
    double s = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) s += v[r] * ww[r];
    for (int k = 32; k > 0; k >>= 1) s += __shfl_down(s, k, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[((int64_t)blockIdx.x * nv + i) * nseg + c] = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
  }
}

// out[i][c] = sum over blocks of part[blk][i][c], fixed order (deterministic)
__global__ void finish_dot_kernel(int32_t nblk, int32_t nv, int32_t nseg, const double* __restrict__ part,
                                  double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nv * nseg) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * nv * nseg + e];
  out[e] = s;
}

// w -= sum_i h[i][c] V_i on segment c
__global__ void seg_orth_kernel(int32_t nseg, const int64_t* __restrict__ off, const int64_t* __restrict__ len,
                                int32_t nv, const double* __restrict__ V, int64_t vstride,
                                const double* __restrict__ h, double* __restrict__ w) {
  const int c = blockIdx.y;
  const int64_t o = off[c], n = len[c];
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    double s = w[o + r];
    for (int i = 0; i < nv; ++i) s -= h[i * nseg + c] * V[i * vstride + o + r];
    w[o + r] = s;
  }
}

// dst = scale[c] src on segment c (scale read on the device)
__global__ void seg_scale_kernel(int32_t nseg, const int64_t* __restrict__ off, const int64_t* __restrict__ len,
                                 const double* __restrict__ src, const double* __restrict__ scale,
                                 double* __restrict__ dst) {
  const int c = blockIdx.y;
  const int64_t o = off[c], n = len[c];
  const double a = scale[c];
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    dst[o + r] = a * src[o + r];
}

// x += sum_i y[i][c] Z_i on segment c
__global__ void seg_combine_kernel(int32_t nseg, const int64_t* __restrict__ off, const int64_t* __restrict__ len,
                                   int32_t nz, const double* __restrict__ Z, int64_t zstride,
                                   const double* __restrict__ y, double* __restrict__ x) {
  const int c = blockIdx.y;
  const int64_t o = off[c], n = len[c];
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < nz; ++i) s += y[i * nseg + c] * Z[i * zstride + o + r];
    x[o + r] += s;
  }
}

// r = b - r  (r holds A x on entry)
__global__ void sub_kernel(int64_t n, const double* __restrict__ b, double* __restrict__ r) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    r[e] = b[e] - r[e];
}

__global__ void copy_cols_kernel(int32_t N, int32_t nrhs, const double* __restrict__ src, int64_t lds,
                                 double* __restrict__ dst, int64_t ldd) {
  const int64_t total = (int64_t)N * nrhs;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e / N), i = (int)(e % N);
    dst[i + c * ldd] = src[i + c * lds];
  }
}

}  // namespace dev

static inline int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (int)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

hipError_t spmv_launch(int32_t n, const int32_t* rp, const int32_t* ci, const double* val, const double* x,
                       double* y, int32_t nrhs, int64_t ld, double alpha, double beta, hipStream_t s) {
  const int rows_per_block = 256 / 16;
  const int grid = (n + rows_per_block - 1) / rows_per_block;
  if (nrhs >= 4)
    dev::spmv_kernel<4><<<grid, 256, 0, s>>>(n, rp, ci, val, x, y, nrhs, ld, alpha, beta);
  else
    dev::spmv_kernel<1><<<grid, 256, 0, s>>>(n, rp, ci, val, x, y, nrhs, ld, alpha, beta);
  return hipGetLastError();
}

template <class T>
hipError_t gather_launch(int32_t n, int32_t nrhs, const int32_t* perm, const double* src, int64_t lds, T* dst,
                         int64_t ldd, hipStream_t s) {
  dev::gather_kernel<T><<<grid_for((int64_t)n * nrhs), 256, 0, s>>>(n, nrhs, perm, src, lds, dst, ldd);
  return hipGetLastError();
}
template <class T>
hipError_t scatter_perm_launch(int32_t n, int32_t nrhs, const int32_t* perm, const T* src, int64_t lds,
                               double* dst, int64_t ldd, hipStream_t s) {
  dev::scatter_perm_kernel<T><<<grid_for((int64_t)n * nrhs), 256, 0, s>>>(n, nrhs, perm, src, lds, dst, ldd);
  return hipGetLastError();
}
template <class T>
hipError_t scatter_values_launch(int64_t nnz, const int64_t* target, const double* val, T* arena, hipStream_t s) {
  dev::scatter_values_kernel<T><<<grid_for(nnz), 256, 0, s>>>(nnz, target, val, arena);
  return hipGetLastError();
}
template <class T>
hipError_t scatter_values_scaled_launch(int64_t nnz, const int64_t* target, int64_t shift, double scale,
                                        const double* val, T* arena, hipStream_t s) {
  dev::scatter_values_scaled_kernel<T><<<grid_for(nnz), 256, 0, s>>>(nnz, target, shift, scale, val, arena);
  return hipGetLastError();
}
size_t diff_norm_scratch_doubles() { return 2 * dev::kNormBlocks + 2; }
template <class T>
hipError_t diff_norm_launch(int64_t n, const T* v, const T* u, double* scratch, hipStream_t s) {
  dev::diff_norm_kernel<T><<<dev::kNormBlocks, 256, 0, s>>>(n, v, u, scratch);
  dev::finish_norm_kernel<<<1, 64, 0, s>>>(dev::kNormBlocks, scratch, scratch + 2 * dev::kNormBlocks);
  return hipGetLastError();
}
template <class T>
hipError_t zero_launch(T* p, int64_t n, hipStream_t s) {
  dev::zero_kernel<T><<<grid_for(n), 256, 0, s>>>(p, n);
  return hipGetLastError();
}
template <class T>
hipError_t identity_launch(T* p, int32_t n, hipStream_t s) {
  dev::identity_kernel<T><<<grid_for((int64_t)n * n), 256, 0, s>>>(p, n);
  return hipGetLastError();
}
hipError_t set_int_launch(int32_t* p, int32_t v, hipStream_t s) {
  dev::set_int_kernel<<<1, 1, 0, s>>>(p, v);
  return hipGetLastError();
}
hipError_t zero_int_launch(int32_t* p, int32_t n, hipStream_t s) {
  dev::zero_int_kernel<<<grid_for(n), 256, 0, s>>>(p, n);
  return hipGetLastError();
}

#define INST(T)                                                                                          \
  template hipError_t gather_launch<T>(int32_t, int32_t, const int32_t*, const double*, int64_t, T*, int64_t, \
                                       hipStream_t);                                                     \
  template hipError_t scatter_perm_launch<T>(int32_t, int32_t, const int32_t*, const T*, int64_t, double*,  \
                                             int64_t, hipStream_t);                                      \
  template hipError_t scatter_values_launch<T>(int64_t, const int64_t*, const double*, T*, hipStream_t);  \
  template hipError_t scatter_values_scaled_launch<T>(int64_t, const int64_t*, int64_t, double, const double*, \
                                                      T*, hipStream_t);                                  \
  template hipError_t diff_norm_launch<T>(int64_t, const T*, const T*, double*, hipStream_t);            \
  template hipError_t zero_launch<T>(T*, int64_t, hipStream_t);                                          \
  template hipError_t identity_launch<T>(T*, int32_t, hipStream_t);
INST(float)
INST(double)
#undef INST

// GMRES helpers
static inline dim3 seg_grid(int32_t nseg, int64_t max_len) {
  int64_t gx = (max_len + 255) / 256;
  gx = gx < 1 ? 1 : (gx > 1024 ? 1024 : gx);
  return dim3((unsigned)gx, (unsigned)nseg);
}
hipError_t seg_dot_launch(int32_t nseg, const int64_t* off, const int64_t* len, int32_t nv, const double* V,
                          int64_t vstride, const double* w, double* part, double* out, hipStream_t s) {
  dev::seg_dot_kernel<<<dim3(dev::kDotBlocks, nseg), 256, 0, s>>>(nseg, off, len, nv, V, vstride, w, part);
  const int e = nv * nseg;
  dev::finish_dot_kernel<<<(e + 255) / 256, 256, 0, s>>>(dev::kDotBlocks, nv, nseg, part, out);
  return hipGetLastError();
}
hipError_t seg_orth_launch(int32_t nseg, const int64_t* off, const int64_t* len, int64_t max_len, int32_t nv,
                           const double* V, int64_t vstride, const double* h, double* w, hipStream_t s) {
  dev::seg_orth_kernel<<<seg_grid(nseg, max_len), 256, 0, s>>>(nseg, off, len, nv, V, vstride, h, w);
  return hipGetLastError();
}
hipError_t seg_scale_launch(int32_t nseg, const int64_t* off, const int64_t* len, int64_t max_len,
                            const double* src, const double* scale, double* dst, hipStream_t s) {
  dev::seg_scale_kernel<<<seg_grid(nseg, max_len), 256, 0, s>>>(nseg, off, len, src, scale, dst);
  return hipGetLastError();
}
hipError_t seg_combine_launch(int32_t nseg, const int64_t* off, const int64_t* len, int64_t max_len, int32_t nz,
                              const double* Z, int64_t zstride, const double* y, double* x, hipStream_t s) {
  dev::seg_combine_kernel<<<seg_grid(nseg, max_len), 256, 0, s>>>(nseg, off, len, nz, Z, zstride, y, x);
  return hipGetLastError();
}
hipError_t sub_launch(int64_t n, const double* b, double* r, hipStream_t s) {
  dev::sub_kernel<<<grid_for(n), 256, 0, s>>>(n, b, r);
  return hipGetLastError();
}
hipError_t copy_cols_launch(int32_t N, int32_t nrhs, const double* src, int64_t lds, double* dst, int64_t ldd,
                            hipStream_t s) {
  dev::copy_cols_kernel<<<grid_for((int64_t)N * nrhs), 256, 0, s>>>(N, nrhs, src, lds, dst, ldd);
  return hipGetLastError();
}

}  // namespace hlu
