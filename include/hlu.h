/*
 * hlu.h -- C ABI of libhlu: H-LU preconditioned GMRES for the lowest-order
 * Nedelec discretisation of the time-harmonic Maxwell equations on MI355X
 * (gfx950).
 *
 * Method: Parvizi, Khodadadian, Beuchler, Wick, "Hierarchical LU
 * preconditioning for the time-harmonic Maxwell equations" (arXiv 2211.11303).
 *   - Galerkin matrix A = K - kappa^2 M of the Nedelec edge element
 *     (Sec. 2.1, eq. (5) and eq. (8)); the paper's kappa is kappa^2 here.
 *   - H-matrix on an eta-admissible block partition (Sec. 3, Definition 1),
 *     eta = 2 and a geometric cluster tree (Sec. 4).
 *   - H-LU factorisation (Algorithm 1, step II) with truncated SVD
 *     recompression of the low-rank blocks (Sec. 4).
 *   - Preconditioner application U^{-1}(L^{-1} r) (Algorithm 1, step III)
 *     inside restarted GMRES (Sec. 4, Example 1).
 *
 * Conventions for every call:
 *   - Every call returns an hlu_status.  No call aborts, throws or prints.
 *     On failure hlu_last_error() returns a message for the calling thread.
 *   - Pointers named d_* or documented as "device" are HIP device pointers;
 *     all others are host pointers.  Inputs are borrowed: the library copies
 *     what it keeps and never frees caller memory.
 *   - "stream" is a hipStream_t passed as void* (NULL = default stream).
 *     Work is stream-ordered; calls that must report a device-side result
 *     (hlu_factor, gmres_solve) synchronise that stream before returning.
 *   - Dense vectors and blocks of vectors are column-major: nrhs columns of
 *     length N with leading dimension ld >= N, in the natural (mesh) order of
 *     the unknowns.
 *   - On error a handle's state is unchanged.
 */
#ifndef HLU_H
#define HLU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HLU_OK = 0,
  HLU_ERR_INVALID_ARG = -1,    /* a size, pointer or option is invalid        */
  HLU_ERR_OUT_OF_MEMORY = -2,  /* a host or device allocation failed, or the
                                  bound workspace is too small               */
  HLU_ERR_DEVICE = -3,         /* a HIP runtime call failed                   */
  HLU_ERR_ZERO_PIVOT = -4,     /* unpivoted LU met an exact zero pivot        */
  HLU_ERR_NOT_CONVERGED = -5,  /* GMRES stopped at max_iters above tol        */
  HLU_ERR_STATE = -6,          /* call out of order (e.g. solve before factor)*/
  HLU_ERR_RANK_OVERFLOW = -7,  /* a truncated rank exceeded the block's
                                  storage capacity (result kept at capacity)  */
  HLU_ERR_UNSUPPORTED = -8     /* input outside what the library handles     */
} hlu_status;

/* Precision of an H-LU.  HLU_FP64: factors stored and computed in FP64.
 * HLU_FP32: factors stored in FP32 and the dense factor tasks (leaf LU,
 * triangular solves, products) computed in FP32.  HLU_FP32_ACC64: factors
 * stored in FP32, the dense factor tasks computed in FP64 and rounded to
 * FP32 when stored.  In every mode the truncation's small dense algebra is
 * FP64, and the H-solves read the stored factors and accumulate in FP64. */
typedef enum { HLU_FP64 = 0, HLU_FP32 = 1, HLU_FP32_ACC64 = 2 } hlu_precision;

typedef struct hlu_spmat_s* hlu_spmat;  /* device CSR of A, for y = A x      */
typedef struct hlu_s* hlu_handle;       /* structure + H-LU of one problem    */
typedef struct hlu_batch_s* hlu_batch;  /* independent problems run together  */

/* Host CSR, 0-based, columns sorted ascending within each row. */
typedef struct {
  int32_t n;              /* rows = columns                                   */
  int64_t nnz;
  const int32_t* row_ptr; /* n + 1 entries                                    */
  const int32_t* col;     /* nnz entries                                      */
  const double* val;      /* nnz entries                                      */
} hlu_csr;

/* Truncation of every low-rank addition (Sec. 4): keep singular values
 * sigma_i > eps * sigma_1, at most max_rank of them.
 *   eps >= 0; eps == 0 keeps every non-zero triplet (no truncation);
 *   max_rank > 0 caps the rank (the paper's fixed-rank mode) and sizes the
 *   low-rank storage; max_rank == 0 means no cap, storage sized to
 *   min(rows, cols, 64) per block and HLU_ERR_RANK_OVERFLOW if exceeded.
 * prec: arithmetic and storage type of the factors (FP32 or FP64). */
typedef struct {
  double eps;
  int32_t max_rank;
  int32_t prec; /* hlu_precision */
} hlu_factor_opts;

typedef struct {
  int32_t restart;   /* Krylov basis size per cycle, >= 1                    */
  int32_t max_iters; /* total Arnoldi steps per right-hand side, >= 1        */
  double tol;        /* stop when ||b - A x||_2 <= tol ||b||_2               */
} hlu_gmres_opts;

typedef struct {
  int32_t iters;     /* Arnoldi steps (= preconditioner applications)        */
  int32_t converged; /* 1 if the true relative residual reached tol          */
  double relres;     /* ||b - A x||_2 / ||b||_2 at exit (true residual)      */
  double abs_res;    /* ||A x - b||_2, the "error" of Algorithm 1, step IV   */
} hlu_gmres_info;

typedef struct {
  int64_t n;
  int64_t num_clusters, num_leaf_clusters, depth;
  int64_t num_admissible, num_dense;
  int64_t dense_entries;         /* entries stored in dense leaves            */
  int64_t lowrank_rows_plus_cols;/* sum over admissible blocks of (m + n)     */
  int64_t workspace_bytes;       /* bound workspace needed by hlu_factor      */
  int64_t factor_waves;          /* dependency levels of the factor schedule  */
  int64_t factor_tasks;          /* primitive tasks in the factor schedule    */
  int64_t solve_waves;           /* dependency levels of one forward+backward sweep */
  int32_t max_rank;              /* largest rank after the factorisation      */
  int32_t capped_blocks;         /* blocks whose eps-rank exceeded capacity   */
  double mean_rank;              /* mean rank over admissible blocks          */
  double lowrank_entries;        /* sum over admissible blocks of (m+n) rank  */
  double min_abs_pivot, max_abs_pivot; /* |U_ii| over all diagonal leaves     */
  int64_t solve_launches;        /* persistent solve launches timed since hlu_set_timing */
  int64_t solve_columns;         /* right-hand-side columns those launches processed */
  double solve_kernel_ms;        /* their summed durations (HIP events on the launch stream) */
  /* Nominal flops of the last hlu_factor (not filled for batch members):
   * leaf LU 2m^3/3, triangular solves and products m^2 n, products of
   * blocks 2mnk per term, truncation: Gram matrices 2(m+n)K^2, pivoted
   * Cholesky K^3/3, core 2K^2 r + 2r^2 K, Jacobi 9n^3 per sweep, rebuild
   * 2(m r + n K) r_new (K stacked columns, r their numerical rank). */
  double factor_flops;
  double factor_flops_getrf, factor_flops_tri, factor_flops_gemm, factor_flops_trunc;
  /* Rank storage reserved in the workspace: sum over admissible blocks of
   * (m + n) times the block's capacity (min(m, n, 64 or max_rank), or the
   * fitted capacity after hlu_fit_ranks). */
  double rank_capacity_entries;
} hlu_stats;

/* Schulz iteration for the H-matrix inverse (hlu_inverse). */
typedef struct {
  int32_t max_iters;   /* Schulz steps at most, >= 0                          */
  double tol;          /* stop when the probed residual rho <= tol            */
} hlu_schulz_opts;

typedef struct {
  int32_t iters;       /* Schulz steps taken (and kept)                       */
  int32_t converged;   /* 1 if rho <= tol                                     */
  double residual;     /* rho = ||(I - A_H B_H) Omega||_F / ||Omega||_F       */
  double residual0;    /* rho of the start X_0                                */
} hlu_schulz_info;

/* ---------------------------------------------------------------- problem
 * The Kuhn-split unit cube (Example 1, Sec. 4): n^3 cubes, each cut into six
 * tetrahedra; unknowns are the N = 7n^3 - 9n^2 + 3n interior edges
 * (perfect-conductor boundary, Sec. 2.1), ordered lexicographically by
 * (tail vertex id, head vertex id) with vertex (i,j,k) -> i + (n+1)(j + (n+1)k)
 * and edges oriented from the lower to the higher id. */

/* N and nnz(A) for n >= 1. */
hlu_status hlu_kuhn_sizes(int32_t n, int32_t* N, int64_t* nnz);

/* Assemble A = K - kappa^2 M (exact element integrals of the Whitney edge
 * basis) into caller-allocated host arrays: row_ptr[N+1], col[nnz],
 * val[nnz]; and mid2[3N], the doubled lattice coordinates
 * p_tail + p_head of each edge midpoint (row-major N x 3). */
hlu_status hlu_kuhn_assemble(int32_t n, double kappa, int32_t* row_ptr, int32_t* col,
                             double* val, int32_t* mid2);
/* The same with a piecewise constant coefficient of the curl-curl term
 * (the 1/mu of eq. (1); beta of Sec. 2.1, a magnet block of Example 3):
 * tetrahedra of the cubes (i, j, k) with beta_box[0] <= i < beta_box[3],
 * beta_box[1] <= j < beta_box[4], beta_box[2] <= k < beta_box[5] (host, 6
 * cube indices; NULL: none) get K scaled by beta_in > 0, the others by 1. */
hlu_status hlu_kuhn_assemble_beta(int32_t n, double kappa, const int32_t* beta_box, double beta_in,
                                  int32_t* row_ptr, int32_t* col, double* val, int32_t* mid2);
/* Support box of every interior edge's basis function: the bounding box of
 * the tetrahedra containing the edge, in doubled lattice units (those of
 * mid2), lo2 and hi2 host N x 3.  For hlu_build_boxes. */
hlu_status hlu_kuhn_support_boxes(int32_t n, int32_t* lo2, int32_t* hi2);

/* Right-hand side of the weak form (Sec. 2.1) for a constant source field
 * J[3] (Example 1: J_S = (0, 0, 1)): b[j] = <J, Phi_j> over the interior
 * edges, exact, into the caller's host array b[N]. */
hlu_status hlu_kuhn_load(int32_t n, const double* J, double* b);

/* ----------------------------------------------------- lattice domains
 * The same discretisation on a union of cubes of the n^3 lattice (e.g. the
 * two boxes of Example 2): mask[i + n (j + n k)] != 0 (host, n^3 bytes)
 * puts cube (i, j, k) in the domain.  The mesh is the Kuhn split of those
 * cubes; the unknowns are the edges not lying in a boundary face (a square
 * with exactly one of its two cubes in the domain: the perfect-conductor
 * condition of eq. (4) on the domain's boundary), numbered as for the cube.
 * mask = NULL is the whole cube, so these calls generalise the ones above.
 * hlu_kuhn_domain_sizes gives N = 0 for a domain without interior edges;
 * the other calls reject such a domain (HLU_ERR_INVALID_ARG). */
hlu_status hlu_kuhn_domain_sizes(int32_t n, const uint8_t* mask, int32_t* N, int64_t* nnz);
hlu_status hlu_kuhn_assemble_domain(int32_t n, double kappa, const uint8_t* mask, const int32_t* beta_box,
                                    double beta_in, int32_t* row_ptr, int32_t* col, double* val, int32_t* mid2);
hlu_status hlu_kuhn_load_domain(int32_t n, const uint8_t* mask, const double* J, double* b);
hlu_status hlu_kuhn_domain_support_boxes(int32_t n, const uint8_t* mask, int32_t* lo2, int32_t* hi2);

/* ----------------------------------------------------------- sparse matrix
 * Wraps a device CSR (borrowed: the caller keeps d_row_ptr[n+1], d_col[nnz],
 * d_val[nnz] alive until hlu_spmat_destroy). */
hlu_status hlu_spmat_create(int32_t n, int64_t nnz, const int32_t* d_row_ptr,
                            const int32_t* d_col, const double* d_val, hlu_spmat* out);
void hlu_spmat_destroy(hlu_spmat A);

/* Y = alpha A X + beta Y for nrhs device columns (ld >= n).  beta == 0
 * ignores the input content of Y.  X and Y must not overlap. */
hlu_status hlu_spmv(hlu_spmat A, const double* d_x, double* d_y, int32_t nrhs, int64_t ld,
                    double alpha, double beta, void* stream);

/* ------------------------------------------------------------- H-LU handle
 * Algorithm 1, step I + the cluster and block trees of Sec. 3/4 (host work
 * only).  A: host CSR; mid2: host N x 3 doubled midpoint coordinates, from
 * which the geometric cluster tree is built (leaf clusters hold at most
 * leaf_size indices); eta: admissibility parameter (min diam <= eta dist). */
hlu_status hlu_build(const hlu_csr* A, const int32_t* mid2, double eta, int32_t leaf_size,
                     hlu_handle* out);
/* hlu_build with the admissibility test (Sec. 3, Definition 1) on given
 * boxes instead of the midpoint boxes: box_lo2/box_hi2 host N x 3 (doubled
 * lattice units, each containing its index's midpoint), e.g. the supports
 * of the basis functions (hlu_kuhn_support_boxes).  A cluster's box is the
 * union of its indices' boxes; the cluster tree is still split on the
 * midpoints.  With the supports of the basis functions, admissible blocks
 * hold no matrix entry at any leaf size. */
hlu_status hlu_build_boxes(const hlu_csr* A, const int32_t* mid2, const int32_t* box_lo2,
                           const int32_t* box_hi2, double eta, int32_t leaf_size, hlu_handle* out);

/* A new handle for a matrix with exactly the sparsity pattern of proto's
 * (same n, row_ptr and col; values may differ, e.g. another kappa on the
 * same mesh).  It shares proto's cluster tree, block tree and task plans
 * (read-only, reference-counted), so building it costs one pattern check.
 * HLU_ERR_INVALID_ARG if the pattern differs. */
hlu_status hlu_build_shared(hlu_handle proto, const hlu_csr* A, hlu_handle* out);

/* Destroys the handle; its device buffers are freed, caller workspaces are
 * not.  A handle destroyed while in a batch leaves the batch unusable
 * (HLU_ERR_STATE) until hlu_batch_destroy. */
void hlu_destroy(hlu_handle h);

/* Device bytes hlu_factor needs for these options (plans the schedule). */
hlu_status hlu_workspace_bytes(hlu_handle h, const hlu_factor_opts* o, size_t* bytes);

/* Caller-owned memory for the persistent H-solve's buffers (triangle
 * inverses, stacked operators, gather records, T products, flags; Algorithm
 * 1, step III).  Without it the library allocates them on the first solve.
 * hlu_solve_workspace_bytes: bytes for options o (the rank capacity decides
 * the schedule).  hlu_bind_solve_workspace: d_work device memory, 256-byte
 * aligned, at least that many bytes, owned by the caller and used until the
 * handle is destroyed or bound again (NULL, 0 returns to library-owned
 * buffers); the next solve rebuilds its buffers there. */
hlu_status hlu_solve_workspace_bytes(hlu_handle h, const hlu_factor_opts* o, size_t* bytes);
hlu_status hlu_bind_solve_workspace(hlu_handle h, void* d_work, size_t bytes);

/* All device bytes a factored handle holds for these options: the bound
 * workspace, the library-owned buffers of its own solves, its matrix values,
 * and the plan arrays, solve schedule, scatter targets and permutation of
 * its structure (hlu_plan_device_bytes; those are shared by every handle of
 * the structure, so a caller holding several handles of one structure counts
 * them once).  For admission by device-memory budget. */
hlu_status hlu_device_bytes(hlu_handle h, const hlu_factor_opts* o, size_t* bytes);
/* The shared part of hlu_device_bytes: device copies of the structure's
 * task plans, solve schedule, scatter targets and permutation. */
hlu_status hlu_plan_device_bytes(hlu_handle h, const hlu_factor_opts* o, size_t* bytes);

/* Hands the library a caller-owned device buffer of at least the bytes
 * reported above (256-byte aligned).  It stays in use until re-bound or the
 * handle is destroyed. */
/* Fit the rank capacities to the ranks the last hlu_factor of this handle
 * asked for (Sec. 4: each truncation keeps the singular values above
 * eps * sigma_1).  Every admissible block and every temporary low-rank
 * accumulator of the factorisation gets capacity min(m, n, kcap,
 * peak + margin), peak being the largest eps-rank any of its truncations
 * asked for (also when a capacity cut it), instead of min(m, n, kcap) with
 * kcap = 64 (or max_rank).  The plans are rebuilt for the new layout (host
 * work of the same order as hlu_build's first factorisation); the factor is
 * dropped (the handle is no longer factored) and *workspace_bytes receives
 * the workspace hlu_factor with options o now needs: bind a workspace of
 * that size and factor again.  With the same eps and values the new
 * factorisation is the same (bit for bit) as long as no capacity is
 * exceeded; a block that needs more is reported as by hlu_factor
 * (HLU_ERR_RANK_OVERFLOW, or counted in capped_blocks with max_rank > 0),
 * and fitting again after that factorisation raises its capacity.  The
 * peaks may come from a factorisation with a small max_rank (a capped run
 * that needs little memory) and o may then have max_rank = 0.  margin < 0
 * drops the fitted capacities.  Needs the handle's own workspace (not a
 * batch).  Batches built afterwards from the handle use its fitted
 * capacities when their options have the same kcap. */
hlu_status hlu_fit_ranks(hlu_handle h, const hlu_factor_opts* o, int32_t margin, size_t* workspace_bytes);

hlu_status hlu_bind_workspace(hlu_handle h, void* d_work, size_t bytes);

/* Algorithm 1, step II: copies A into the H-matrix and computes L (unit
 * lower) and U in H-arithmetic, in place, on the GPU.  Synchronises the
 * stream and returns HLU_ERR_ZERO_PIVOT / HLU_ERR_RANK_OVERFLOW if the
 * device reported them (after a zero pivot the handle is unfactored). */
hlu_status hlu_factor(hlu_handle h, const hlu_factor_opts* o, void* stream);

/* x = (L U)^{-1} b in the natural order, i.e. x = P^T U^{-1} L^{-1} P b
 * (Algorithm 1, step III).  d_b, d_x: device, nrhs columns, leading
 * dimension ld; d_x may alias d_b.  Stream-ordered, no synchronisation. */
hlu_status hlu_solve(hlu_handle h, const double* d_b, double* d_x, int32_t nrhs, int64_t ld,
                     void* stream);

/* Synchronises the stream and reports what the stream-ordered solves of h
 * left on the device: HLU_ERR_DEVICE if a persistent solve launched on h
 * since the previous report gave up waiting for one of its inputs (each
 * wait is bounded by 20 s of device wall clock; the launch then drains and
 * its result is invalid).  Clears the report.  gmres_solve checks the same
 * word at every synchronisation of its iteration and fails with
 * HLU_ERR_DEVICE. */
hlu_status hlu_sync_status(hlu_handle h, void* stream);

/* y = P^T L U P v (the product of the computed factors), for checking the
 * factor error; same layout rules as hlu_solve (no aliasing). */
hlu_status hlu_apply_lu(hlu_handle h, const double* d_v, double* d_y, int32_t nrhs, int64_t ld,
                        void* stream);

/* Approximate inverse B_H of the H-matrix A_H by the Schulz iteration
 * (Sec. 3: the inverse of the H-matrix approximation of the Galerkin
 * matrix by the iterative method of Schulz; Sec. 4: truncated SVD of rank r
 * in the admissible blocks; Example 2: B_H as the preconditioner):
 *   X_{k+1} = X_k (2I - A_H X_k),  X_0 = A^T / (||A||_1 ||A||_inf),
 * both products in H-arithmetic on the handle's block tree, every addition
 * into a low-rank block truncated with the rule of o (eps, max_rank); o->prec
 * as for hlu_factor.  The iteration stops when rho_k = ||(I - A_H X_k)
 * Omega||_F / ||Omega||_F <= so->tol, when a step does not decrease rho
 * (the truncation floor; the previous iterate is kept), or after
 * so->max_iters steps.  d_probe: Omega, device, N x nprobe column-major in
 * the natural order, 1 <= nprobe <= 32 (borrowed; the caller draws it).
 * Requires a symmetric A (HLU_ERR_UNSUPPORTED otherwise; K - kappa^2 M is
 * symmetric) and no admissible block holding matrix entries (leaf sizes
 * >= 32 on the Kuhn cube; HLU_ERR_UNSUPPORTED otherwise).  Uses the bound
 * workspace, of at least hlu_inverse_workspace_bytes(h, o) bytes (four
 * H-matrices: A_H, two iterates, 2I - A_H X_k).  On success the handle holds
 * B_H instead of H-LU factors: hlu_solve and gmres_solve's preconditioner
 * apply x = B_H b (an H-matrix-vector product), hlu_apply_lu returns
 * HLU_ERR_STATE until the next hlu_factor.  info (host) receives the steps
 * and residuals; hlu_get_stats the ranks of B_H and the flops.  Synchronises
 * the stream. */
hlu_status hlu_inverse_workspace_bytes(hlu_handle h, const hlu_factor_opts* o, size_t* bytes);
hlu_status hlu_inverse(hlu_handle h, const hlu_factor_opts* o, const hlu_schulz_opts* so,
                       const double* d_probe, int32_t nprobe, hlu_schulz_info* info, void* stream);

/* Restarted right-preconditioned flexible GMRES (Sec. 4), x0 = 0,
 * classical Gram-Schmidt applied twice, FP64 throughout; precond may be
 * NULL.  Each of the nrhs columns is solved independently (its own Arnoldi
 * process; operator and preconditioner applied to all columns per launch).
 * info: host array of nrhs entries.  d_work: caller-owned device buffer of
 * gmres_workspace_bytes(n, nrhs, restart) bytes.  Synchronises the stream.
 * Returns HLU_ERR_NOT_CONVERGED if any column missed tol (x then holds the
 * last iterate). */
size_t gmres_workspace_bytes(int32_t n, int32_t nrhs, int32_t restart);
hlu_status gmres_solve(hlu_spmat A, const double* d_b, double* d_x, int32_t nrhs, int64_t ld,
                       hlu_handle precond, const hlu_gmres_opts* o, hlu_gmres_info* info,
                       void* d_work, size_t work_bytes, void* stream);

/* GMRES with refinement of the preconditioner, for wavenumbers close to a
 * cavity resonance, where the H-LU at eps is too coarse (Sec. 4 reports
 * iteration counts growing with kappa; a smaller eps is the paper's remedy
 * of a better H-matrix approximation).  The first gmres_solve gets at most
 * r->refine_iters iterations while a refinement is still allowed; columns
 * that miss tol then make the library refactor H (hlu_factor with
 * eps <- max(eps * r->eps_factor, 1e-7), same precision and rank cap, in
 * H's own workspace) and solve those columns again from x0 = 0, at most
 * r->max_refines times; the last attempt has o->max_iters.  Converged
 * columns keep their result.  H must hold H-LU factors in its own
 * workspace (not a batch).  info: the last solve of each column;
 * *refines: the refactorisations made (H stays refined).  d_work:
 * gmres_refined_workspace_bytes(n, nrhs, restart) bytes (the GMRES
 * workspace and two packed vector blocks).  Synchronises the stream.
 * Returns HLU_ERR_NOT_CONVERGED if a column still misses tol. */
typedef struct {
  int32_t refine_iters; /* first-try iteration budget, >= 1                    */
  int32_t max_refines;  /* refactorisations at most, >= 0                      */
  double eps_factor;    /* eps multiplier per refactorisation, in (0, 1)       */
} hlu_refine_opts;
size_t gmres_refined_workspace_bytes(int32_t n, int32_t nrhs, int32_t restart);
hlu_status gmres_solve_refined(hlu_spmat A, const double* d_b, double* d_x, int32_t nrhs, int64_t ld,
                               hlu_handle H, const hlu_gmres_opts* o, const hlu_refine_opts* r,
                               hlu_gmres_info* info, int32_t* refines, void* d_work, size_t work_bytes,
                               void* stream);

/* gmres_solve without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, semantics and results
 * as gmres_solve; the Krylov workspace is a static device array of
 * gmres_static_max_bytes() bytes (64 MiB), one per GPU, held from the first
 * call on that GPU until the process ends.  Calls no hipMalloc / hipFree:
 * HLU_ERR_OUT_OF_MEMORY if gmres_workspace_bytes(n, nrhs, restart) exceeds
 * that size; HLU_ERR_STATE if precond's solve buffers have not been made
 * yet (one hlu_solve or gmres_solve on it makes them) or its solve timing
 * is on.  Every call on a GPU uses that GPU's one array: calls that overlap
 * on one GPU (several streams or threads) race and must be serialised by
 * the caller. */
size_t gmres_static_max_bytes(void);
hlu_status gmres_solve_static(hlu_spmat A, const double* d_b, double* d_x, int32_t nrhs, int64_t ld,
                              hlu_handle precond, const hlu_gmres_opts* o, hlu_gmres_info* info,
                              void* stream);

/* Preconditioned Richardson iteration of Algorithm 1, steps III-IV, for
 * every column of b (device, N x nrhs, leading dimension ld): x_0 = 0 and
 * for k = 1, 2, ...:  r = b - A x;  err = ||r||_2 / ||b||_2;
 * x += M^{-1} r (the preconditioner of `precond`: its H-LU factors, or its
 * Schulz inverse);  stop once err < tol -- the correction is applied before
 * the loop is left, the order the paper gives -- or after max_iters
 * corrections.  info[c] (host): iters = corrections applied, converged
 * (err < tol reached), abs_res = ||A x - b||_2 at exit (step IV's "error"),
 * relres = abs_res / ||b||_2.  x (device) must not alias b.  d_work: device
 * workspace of at least hlu_richardson_workspace_bytes(N, nrhs) bytes.
 * Returns HLU_OK even when a column did not reach tol (see info).
 * Synchronises the stream. */
size_t hlu_richardson_workspace_bytes(int32_t n, int32_t nrhs);
hlu_status hlu_richardson(hlu_spmat A, const double* d_b, double* d_x, int32_t nrhs, int64_t ld,
                          hlu_handle precond, double tol, int32_t max_iters, hlu_gmres_info* info,
                          void* d_work, size_t work_bytes, void* stream);

/* ------------------------------------------------------------------ batch
 * Independent problems (each an hlu_handle, of any size) factored and solved
 * together: every launch of the batch factorisation runs the ready tasks of
 * all problems, and one persistent launch runs the H-solves of all problems.
 * Results equal those of the problems factored and solved one by one (the
 * same tasks in the same per-problem order).
 *
 * hlu_batch_create: hs[count] distinct handles not in another batch; o: the
 * options of every factorisation; max_rhs (1..32): columns per problem of
 * hlu_solve_batch / gmres_solve_batch.  Plans each distinct structure once
 * (host work); the handles stay owned by the caller and must outlive the
 * batch.  After hlu_factor_batch every member is factored and usable on its
 * own (hlu_solve, gmres_solve), with its factor inside the batch workspace.
 *
 * Stacked vectors: problem p occupies rows [row_base[p], row_base[p] + N_p)
 * of a column of n_total rows (natural order within the problem); a block
 * holds nrhs such columns, leading dimension n_total. */
hlu_status hlu_batch_create(const hlu_handle* hs, int32_t count, const hlu_factor_opts* o,
                            int32_t max_rhs, hlu_batch* out);
void hlu_batch_destroy(hlu_batch b);

/* hlu_sync_status for the batch's own persistent solves (hlu_solve_batch;
 * gmres_solve_batch checks at every synchronisation). */
hlu_status hlu_batch_sync_status(hlu_batch b, void* stream);

/* count, n_total, row_base[count] (host, may be NULL) and the size of the
 * merged factor schedule (waves, tasks). */
hlu_status hlu_batch_sizes(hlu_batch b, int32_t* count, int32_t* n_total, int32_t* row_base,
                           int64_t* factor_waves, int64_t* factor_tasks);

/* Device bytes of the batch workspace (all factors, rank tables, status). */
hlu_status hlu_batch_workspace_bytes(hlu_batch b, size_t* bytes);
/* Caller-owned, 256-byte aligned, at least the bytes above; replaces the
 * members' own workspaces for as long as the batch lives. */
hlu_status hlu_batch_bind_workspace(hlu_batch b, void* d_work, size_t bytes);

/* Algorithm 1, step II for every member, as one merged wave schedule.
 * Synchronises the stream; HLU_ERR_ZERO_PIVOT / HLU_ERR_RANK_OVERFLOW as
 * for hlu_factor (for the batch as a whole). */
hlu_status hlu_factor_batch(hlu_batch b, void* stream);

/* Algorithm 1, step III for every member in one persistent launch: d_b, d_x
 * stacked device blocks of nrhs <= max_rhs columns (leading dimension
 * n_total; must not overlap).  Stream-ordered. */
hlu_status hlu_solve_batch(hlu_batch b, const double* d_b, double* d_x, int32_t nrhs, void* stream);

/* gmres_solve for every member at once: stacked d_b, d_x (nrhs <= max_rhs
 * columns, leading dimension n_total, no overlap); each (problem, column)
 * is an independent system with its own Arnoldi process, preconditioned by
 * the member's H-LU.  info: host array of count * nrhs entries, entry
 * c * count + p for problem p, column c.  d_work: caller-owned device
 * buffer of gmres_batch_workspace_bytes(b, nrhs, restart) bytes. */
size_t gmres_batch_workspace_bytes(hlu_batch b, int32_t nrhs, int32_t restart);
hlu_status gmres_solve_batch(hlu_batch b, const double* d_b, double* d_x, int32_t nrhs,
                             const hlu_gmres_opts* o, hlu_gmres_info* info, void* d_work,
                             size_t work_bytes, void* stream);

/* ---------------------------------------------------------------- serving
 * A request loop on one GPU for the Kuhn-cube problem: each request names a
 * mesh (n) and kappa and brings nrhs right-hand sides; it is answered by
 * FP64 GMRES preconditioned with the H-LU of A = K - kappa^2 M.
 *   - Factorisations are cached per (n, kappa) in device memory; structures
 *     and plans are built once per n.
 *   - Admission by device bytes: a request starts only when its factor (if
 *     not cached) and its GMRES buffers fit hbm_budget next to everything in
 *     use; idle cached factors are evicted least recently used first.  A
 *     request that cannot fit even into an empty cache fails with
 *     HLU_ERR_OUT_OF_MEMORY.
 *   - Continuous batching: a free worker takes the oldest admissible request
 *     together with every queued request for the same factor (up to
 *     max_batch_rhs columns in all) and answers them with one GMRES call;
 *     each column keeps its own Krylov process, so a result is the same
 *     alone and in the mix.
 *   - Overlap: each of the `workers` threads owns a HIP stream (default
 *     priority), so factorisations and solves of different requests run on
 *     the device concurrently.
 *   - Refinement (refine_iters > 0): a GMRES call first runs at most
 *     refine_iters iterations.  Columns that have not converged by then
 *     (near a resonance of the cavity the factor at eps is too coarse a
 *     preconditioner) make the worker refactor the cached factor in place
 *     with eps multiplied by refine_eps_factor (0 < factor < 1), at most
 *     max_refines times per factor and not below 1e-7, and solve those
 *     columns again with the full gmres.max_iters.  Columns that converged
 *     keep their first result, so a result still does not depend on its
 *     companions; it does depend on whether the cached factor was refined
 *     by an earlier request.  The refined factor stays cached.
 * Device memory of the cache and of the workers' GMRES buffers is owned by
 * the server (the workers keep their largest buffers for reuse). */
typedef struct hlu_server_s* hlu_server;
typedef struct {
  int32_t workers;         /* worker threads = requests in flight, 1..16         */
  int32_t max_batch_rhs;   /* columns per GMRES call (and per request), 1..32    */
  size_t hbm_budget;       /* device bytes for cached factors + GMRES buffers    */
  double eta;              /* admissibility parameter                            */
  int32_t leaf;            /* leaf size of the cluster trees                     */
  hlu_factor_opts factor;  /* options of every factorisation                     */
  hlu_gmres_opts gmres;    /* options of every solve                             */
  int32_t refine_iters;    /* 0: no refinement; else iterations of a first try   */
  int32_t max_refines;     /* refactorisations per cached factor, >= 0           */
  double refine_eps_factor;/* eps multiplier per refinement, in (0, 1)          */
} hlu_server_opts;
typedef struct {
  int64_t submitted, completed, failed;
  int64_t factorizations;      /* factors computed (cache misses)                */
  int64_t cache_hits;          /* GMRES calls served by a cached factor          */
  int64_t evictions;
  int64_t gmres_calls;
  int64_t coalesced_requests;  /* requests that shared a GMRES call              */
  size_t bytes_in_use, peak_bytes;  /* admitted device bytes, now and at peak    */
  int32_t cached_factors;
  int64_t refinements;         /* refactorisations at a smaller eps               */
} hlu_server_stats;

hlu_status hlu_server_create(const hlu_server_opts* o, hlu_server* out);
/* Builds and plans the structure of mesh n now (host work that the first
 * request for n would otherwise pay). */
hlu_status hlu_server_prepare(hlu_server s, int32_t n);
/* Queues a request; returns at once with a ticket.  b: host, N x nrhs
 * column-major (leading dimension N = 7n^3 - 9n^2 + 3n, natural order); x:
 * host output of the same shape; info: host output [nrhs].  b, x and info
 * are borrowed until hlu_server_wait returns for the ticket. */
hlu_status hlu_server_submit(hlu_server s, int32_t n, double kappa, int32_t nrhs, const double* b,
                             double* x, hlu_gmres_info* info, int64_t* ticket);
/* Blocks until the request is answered (timeout_s < 0: no limit; on timeout
 * HLU_ERR_STATE and the ticket stays valid).  Returns the request's status
 * (HLU_ERR_NOT_CONVERGED if a column missed tol) and, if non-NULL, the host
 * wall-clock seconds from submission to start of service and to completion.
 * The ticket is released. */
hlu_status hlu_server_wait(hlu_server s, int64_t ticket, double timeout_s, double* queued_s,
                           double* latency_s);
hlu_status hlu_server_get_stats(hlu_server s, hlu_server_stats* out);
/* Answers every queued request, stops the workers, frees the cache. */
void hlu_server_destroy(hlu_server s);

/* ------------------------------------------------------------ autotuning
 * Leaf size of the cluster trees for the Kuhn-cube mesh n at wavenumber
 * kappa, chosen by measurement (for batches of problems of several sizes).
 * For each of the `count` (1..16) candidates in leaves[] (each 1..128):
 * builds and plans the structure (host, not timed), factors A = K -
 * kappa^2 M with fo twice (the first uploads the plans) and solves nrhs
 * (1..32) right-hand sides b = A 1 with GMRES (go); seconds[c] (host out)
 * is the device time of the second factorisation plus the solve, measured
 * with HIP events on `stream`, or HUGE_VAL if a column did not converge.
 * *best (host out) = the candidate with the smallest time (the first on
 * ties).  Allocates and frees its own device memory; synchronous. */
hlu_status hlu_autotune_leaf(int32_t n, double kappa, double eta, const int32_t* leaves, int32_t count,
                             const hlu_factor_opts* fo, const hlu_gmres_opts* go, int32_t nrhs,
                             double* seconds, int32_t* best, void* stream);

/* ------------------------------------------------------------ inspection */
/* Sizes of the structure arrays, then a copy of them into caller-allocated
 * host arrays (any pointer may be NULL to skip it):
 *   perm[N]: natural index of the i-th index in cluster order;
 *   clusters: begin[C], end[C], level[C], son0[C], son1[C] (-1 for leaves),
 *             pre-order;
 *   blocks (leaves of the block tree, pre-order): brow[B], bcol[B] (cluster
 *             ids), bkind[B] (0 dense, 1 low-rank). */
hlu_status hlu_structure_sizes(hlu_handle h, int32_t* N, int32_t* num_clusters,
                               int32_t* num_blocks);
hlu_status hlu_export_structure(hlu_handle h, int32_t* perm, int32_t* begin, int32_t* end,
                                int32_t* level, int32_t* son0, int32_t* son1, int32_t* brow,
                                int32_t* bcol, int32_t* bkind);

/* Ranks of the admissible blocks (in block pre-order, B entries, -1 for
 * dense blocks) after hlu_factor. Synchronous. */
hlu_status hlu_get_ranks(hlu_handle h, int32_t* ranks);
hlu_status hlu_get_stats(hlu_handle h, hlu_stats* out);

/* Host replay of the round structure of every truncation of the factor
 * plan for options o (Sec. 4: truncated SVD after each low-rank addition),
 * with every rank the plan reads forced to forced_rank (>= 0): the rounds
 * the device kernel would run if every truncation kept that rank (at most
 * the block's capacity, the columns of the round and the round's limit).
 * No device work.  out (host, 5 entries): truncation ops, total rounds,
 * largest rounds of one op, rounds that absorbed no part column while parts
 * remained (a block already at the round's 64 columns), ops that did not
 * finish within their bound (0 for a plan the kernel completes). */
hlu_status hlu_check_trunc_rounds(hlu_handle h, const hlu_factor_opts* o, int32_t forced_rank, int64_t* out);

/* enable != 0: from now on bracket every persistent solve launch of hlu_solve
 * (and of gmres_solve's preconditioner) with HIP events on its stream;
 * hlu_get_stats then waits for the recorded events and reports their count
 * and summed duration.  Every call resets both; enable == 0 stops timing. */
hlu_status hlu_set_timing(hlu_handle h, int32_t enable);

/* Message of the last failing call on this thread ("" if none). */
const char* hlu_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HLU_H */
