/*
 * r3mg.h -- C ABI of the MI355X (gfx950) implementation of R3MG-C: conjugate gradients preconditioned by
 * one V-cycle of an algebraic-geometric multilevel hierarchy built from support-point coordinates only.
 *
 * Paper: Polverino, Feder, Heltai, "R3MG-C: a high-order algebraic-geometric multilevel preconditioner for
 * continuous finite element discretizations".
 *   - Section 3 (Definition of an R-tree of order (m,M)) and Section 4 (point-based agglomeration): the
 *     support points are agglomerated by an R-tree of axis-aligned boxes; each box owns its points.
 *   - Section 4: prolongations evaluate the box-local Q^{p'} basis at the owned fine points (first level) or
 *     inject parent-box polynomials into child boxes (agglomerated levels); level operators are inherited,
 *     A_i = P_i^T A P_i.
 *   - Section 6: the smoother is degree-3 Chebyshev-accelerated Jacobi tuned by Lanczos estimates, with
 *     2 pre- and 2 post-smoothing steps; the coarsest problem is solved directly; PCG applies one V-cycle
 *     per iteration.
 *
 * Conventions (all entry points):
 *   - Host arrays passed to set-up are read and copied; the caller keeps ownership.
 *   - Device pointers are HIP device memory owned by the caller (e.g. torch tensors); every operation is
 *     ordered on the given hipStream_t (passed as void*; NULL means the default stream). Functions that
 *     return values to the host synchronise that stream before returning.
 *   - Vectors are float64 in the caller's numbering.  Multi-RHS arguments are nrhs contiguous vectors
 *     (column j at offset j*n).
 *   - A negative status means the call failed and modified nothing it was given (outputs undefined for
 *     R3MG_ERR_HIP).  R3MG_NOT_CONVERGED (positive) means the solve ran to maxit: x holds the last iterate.
 *   - Handles are not thread-safe; one handle serves one stream at a time.  No entry point falls back to the
 *     CPU: without a usable gfx950 device the device entry points return R3MG_ERR_HIP.
 */
#ifndef R3MG_H
#define R3MG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct r3mg_handle_* r3mg_handle;

/* Largest coarsest level, in DoFs, that the dense float64 Cholesky inverse takes: two n x n float64 arrays,
   2 x 34 GB at this size.  The paper's coarsest solve is a sparse direct one (Section 6); this library inverts
   the coarsest operator densely on the device, which fits HBM up to this size.  Up to 10,240 DoFs the inverse's
   upper-triangular 64 x 64 tiles are kept as well (about half its size), and V-cycles over up to 4 right-hand
   sides read those instead of the whole inverse. */
#define R3MG_MAX_COARSEST_DOFS 65536

typedef enum {
  R3MG_OK = 0,
  R3MG_NOT_CONVERGED = 1,
  R3MG_ERR_INVALID = -1,         /* bad argument, size, non-finite value, unsupported option */
  R3MG_ERR_NOT_UNISOLVENT = -2,  /* a box cannot interpolate Q^{p'} from its owned points (Section 4 remarks) */
  R3MG_ERR_DEGENERATE_BOX = -3,  /* a box with zero extent along an axis while p' >= 1 */
  R3MG_ERR_NOT_SPD = -4,         /* non-positive diagonal, asymmetric Galerkin operator or failed Cholesky */
  R3MG_ERR_OOM = -5,             /* device or host allocation failed, or an index exceeds int32 range */
  R3MG_ERR_HIP = -6              /* a HIP runtime call failed */
} r3mg_status;

/* Options.  Defaults (r3mg_default_options) in brackets. */
typedef struct {
  int dim;              /* spatial dimension of the coordinates, 2 or 3 [3] */
  int coarse_degree;    /* p' in 0..3, box polynomial degree per axis (p'=0: Nicolaides) [1] */
  int leaf_size;        /* R-tree M: maximum number of points per leaf box [64] */
  int max_levels;       /* levels including the fine one; 0 = until max_coarse_dofs or the root [0] */
  int max_coarse_dofs;  /* stop coarsening at the first level with at most this many DoFs [2000]; a coarsest
                           level above R3MG_MAX_COARSEST_DOFS (max_levels reached first) is R3MG_ERR_INVALID */
  int skip_leaf_level;  /* 1 = first coarse level at depth t-d instead of the leaf depth t [0] */
  int cheb_degree;      /* Chebyshev polynomial degree K >= 1 [3] */
  int pre_steps;        /* smoothing applications before the coarse correction [2] */
  int post_steps;       /* smoothing applications after the coarse correction [2] */
  int lanczos_steps;    /* Lanczos steps of the eigenvalue estimate [10] */
  double cheb_boost;    /* lambda_hi = boost * lambda_hat [1.1] */
  double cheb_ratio;    /* lambda_lo = lambda_hi / ratio [30] */
  int vcycle_fp32;      /* 0 = float64 V-cycle; 1 = float32 V-cycle inside float64 CG [0] */
  int use_graph;        /* 1 = replay PCG iterations from a captured hipGraph [1] */
  int fine_kernel;      /* row-block kernel of the fine level for one right-hand side: -1 = the fastest of
                           shapes 0..12 timed at r3mg_factor [-1]; 0..12 = that shape.  0..2: CSR row blocks of
                           (2048 nonzeros, 64 rows), (4096, 128), (4096, 64); 3..5: the same blocks in a
                           persistent pipelined kernel; 6..8: local-column blocks (each block's distinct columns
                           staged once; 1-byte positions with 2048 nonzeros, 64 rows, 256 columns; 2-byte with
                           (4096, 64, 1024) and (4096, 128, 1024)); 9: shape 6 with vector loads; 10: the
                           kernel of shape 9 over 1-byte blocks of (3072 nonzeros, 128 rows, 256 columns); 11, 12:
                           the blocks of shapes 9 and 10 taken two per workgroup (more loads in flight).  With
                           the float32 V-cycle, PCG's float64 operator takes the fastest shape in float64, timed
                           separately.  Every shape sums a row in the same order, so results do not depend on this
                           choice when no row has more than 256 nonzeros. */
  int multi_rhs_kernel; /* fine-level kernel for several right-hand sides: -1 = the fastest timed at the first
                           multi-RHS solve [-1]; 0 = lanes-per-row CSR kernel (each lane all columns of its
                           nonzeros); 1 / 2 = row blocks staged in LDS (values, 2-byte column positions and
                           u at the block's distinct columns; each thread sums one row's 16-byte column chunk):
                           one persistent workgroup per compute unit that loads the next block while summing
                           one (1), or one workgroup per block (2), for 16 float or 8 / 16 double right-hand
                           sides (other counts: the lanes kernel); 3 = CSR with the
                           columns split over lanes (each nonzero's u row read as consecutive 16-byte pieces);
                           4 = the same with each
                           nonzero's value and column loaded once per row and shared by shuffles */
  int matrix_cache;     /* how the level kernels read matrix values: -1 = with ordinary loads where a level's
                           matrix stream is at most 128 MiB (it can stay in the caches across a smoothing sweep),
                           with nontemporal loads elsewhere [-1]; 0 = nontemporal loads on every level; 1 =
                           ordinary loads on every level.  The results do not depend on it. */
  int tune_cache;       /* 1 = kernel choices made by timing (the fine level's row-block shape, the multi-RHS
                           kernels) are looked up in and added to the persisted tuning cache, keyed by the device
                           and the handle's level structure (the file named by the R3MG_TUNE_CACHE environment
                           variable, an empty value for none, else $HOME/.cache/r3mg/tune-cache.txt) [1]; 0 = every
                           handle times its kernels.  Choices forced by fine_kernel or multi_rhs_kernel are never
                           cached. */
} r3mg_options;

typedef struct {
  int64_t n;               /* rows of the level operator */
  int64_t nnz;             /* stored entries (coarse levels: all B*B entries of every stored block) */
  int64_t nboxes;          /* boxes that define the level (0 for the fine level) */
  double max_box_extent;   /* largest box diagonal on the level (0 for the fine level) */
  double lambda_hi;        /* Chebyshev interval (0 on the dense coarsest level) */
  double lambda_lo;
  double bytes_per_apply;  /* algorithmic bytes of one smoother operator application in the V-cycle precision */
  char kernel[48];         /* kernel applying the level for one right-hand side in the V-cycle precision, e.g.
                              "k_level_local<float,u8,3072,128,256,vec>" (position bytes, block capacity, rows
                              per block, distinct columns, form: block, vec, or vec2 for two blocks per workgroup) or
                              "k_level_boxrow<float,9>" (rows per box);
                              "dense" on the coarsest level; "" before r3mg_factor */
} r3mg_level_info;

/* Fill *opt with the defaults listed above. */
void r3mg_default_options(r3mg_options* opt);

/* Host-only analysis (no GPU use): constrained rows, R-tree, level selection, DoF permutation, transfer tables,
 * unisolvence check, Galerkin sparsity.  Inputs: coords (host, n x dim row-major float64), CSR of the symmetric
 * fine operator A (host; row_ptr n+1 int64, col_idx nnz int32, vals nnz float64, columns ascending in each
 * row).  Constrained rows are the rows whose stored off-diagonal values are all exactly 0.0 (identity
 * Dirichlet rows).  On success *out is a handle that supports the export and info calls; r3mg_factor completes
 * it for solving.  Errors: INVALID, NOT_UNISOLVENT, DEGENERATE_BOX, NOT_SPD, OOM. */
r3mg_status r3mg_analyze(const double* coords, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                         const double* vals, const r3mg_options* opt, r3mg_handle* out);

/* r3mg_analyze with cell-based agglomeration (Section 4): the R-tree's leaves are the mesh cells (cells: host
 * ncells x nloc support-point indices in the caller's numbering, row-major; ordered in the tree by the centres
 * of their bounding boxes), each agglomerate's box is the bounding box of its cells' support points, and every
 * support point is owned by the first level-1 agglomerate, in array order, holding one of its cells (the
 * paper's unique assignment of shared support points).  leaf_size counts cells.  Errors as r3mg_analyze, and
 * INVALID for a cell index out of range or a support point in no cell. */
r3mg_status r3mg_analyze_cells(const double* coords, int64_t n, const int32_t* cells, int64_t ncells, int nloc,
                               const int64_t* row_ptr, const int32_t* col_idx, const double* vals,
                               const r3mg_options* opt, r3mg_handle* out);

/* Device numeric set-up of an analysed handle on `stream`: upload, Galerkin products A_{l+1} = P_l^T A_l P_l,
 * inverse diagonals, Lanczos estimates, dense coarsest Cholesky factorisation and inverse.  Synchronises. */
r3mg_status r3mg_factor(r3mg_handle h, void* stream);

/* r3mg_analyze followed by r3mg_factor (Section 4 set-up).  On failure *out is left NULL. */
r3mg_status r3mg_setup(const double* coords, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                       const double* vals, const r3mg_options* opt, void* stream, r3mg_handle* out);

/* Numeric re-set-up with new values on the same sparsity pattern (device array, nnz float64, caller's CSR
 * order).  The constrained set, partition and transfers are kept.  A matrix-free fine operator set by
 * r3mg_set_matrix_free is dropped (the solver returns to the CSR matrix).  Synchronises. */
r3mg_status r3mg_update_values(r3mg_handle h, const double* vals_dev, void* stream);

/* Matrix-free fine-level operator (not in the paper; an alternative to streaming the CSR matrix).  Describes the
 * handle's fine matrix as the Q_p Laplace stiffness matrix of the Poisson problem of Section 6: the sum over
 * cells e of kappa_e K_e with (K_e)_ab = integral over the cell of grad phi_a . grad phi_b, computed with
 * Gauss-Legendre quadrature of p + 1 points per axis, the basis phi being the tensor Lagrange polynomials on
 * the p + 1 Gauss-Lobatto nodes per axis mapped by the multilinear map of the cell's 2^d corner support
 * points; constrained rows and columns (the handle's constrained set) are removed and the constrained rows keep
 * their diagonal entry.
 *   cells   host int32 array, ncells x (p+1)^d, row-major: the caller's support-point indices of each cell in
 *           tensor order (local node (i_0, .., i_{d-1}) at position i_0 + (p+1) i_1 + (p+1)^2 i_2, node i_a at
 *           the a-th coordinate's Gauss-Lobatto point), copied; NULL drops a matrix-free operator set before
 *   degree  p in 1..3;   kappa  host float64 per cell, positive, or NULL for 1
 * The operator is applied to y = A v for a fixed pseudo-random v and compared with the CSR matrix; a maximum
 * difference above 1e-10 max|A v| (wrong degree, node order, geometry or quadrature) is R3MG_ERR_INVALID and
 * leaves the CSR matrix in use.  Once set, every application of the fine operator (smoother, residual, PCG's
 * A p; one or several right-hand sides) is matrix-free.  Results then differ from the CSR path by rounding
 * only.  Several right-hand sides need ncells (p+1)^d nrhs < 2^31 and n nrhs < 2^31 (R3MG_ERR_INVALID at the
 * solve otherwise).  Synchronises. */
r3mg_status r3mg_set_matrix_free(r3mg_handle h, const int32_t* cells, int64_t ncells, int degree, const double* kappa,
                                 void* stream);

/* z = B r, one V-cycle (Section 4) in the handle's V-cycle precision, for nrhs right-hand sides. */
r3mg_status r3mg_vcycle(r3mg_handle h, const double* r_dev, double* z_dev, int nrhs, void* stream);

/* Capacity of the device scratch that r3mg_vcycle_noalloc takes its work vectors from (64 MiB, a static device
 * array of the library that every GPU using it holds until the process ends). */
#define R3MG_NOALLOC_SCRATCH_BYTES (64 << 20)

/* r3mg_vcycle for callers that cannot allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation.  The same V-cycle as r3mg_vcycle, with the same kernels and bitwise the same
 * results, for nrhs in {1, 2, 4, 8, 16} right-hand sides, with the level work vectors (5 per level, n_l x nrhs
 * values in the V-cycle precision, each rounded up to 256 bytes) taken from the library's static device scratch
 * of R3MG_NOALLOC_SCRATCH_BYTES instead of the handle's buffers.  For nrhs > 1 the fine-level kernel is the one
 * the handle's timing chose for that many columns (r3mg_vcycle and r3mg_pcg_solve time the candidates at their
 * first call with that many; this call does not time, since timing synchronises), the default lanes kernel
 * before any such call.  The call allocates no device or host memory,
 * does not synchronise and launches kernels only (the carved work vectors are zeroed by a fill kernel), so it
 * may be captured into a graph.  r_dev, z_dev: device float64, nrhs columns of n (caller's numbering; z is
 * written).  The handle's device must be current.  All calls on one GPU share its scratch, which keeps the last
 * call's contents: calls that overlap on one GPU (two streams, two threads, two handles) race.  Errors: INVALID
 * for another nrhs, for work vectors larger than the scratch (the message states both sizes), for a matrix-free
 * fine operator with nrhs > 1 whose cell outputs have not been sized by a call of r3mg_vcycle or r3mg_pcg_solve
 * with at least that many columns, or when the handle's device is not current; nothing is launched then. */
r3mg_status r3mg_vcycle_noalloc(r3mg_handle h, const double* r_dev, double* z_dev, int nrhs, void* stream);

/* y = A_l x on level `level` in float64 (level 0 in the caller's numbering, coarse levels in box * B + q
 * numbering), or, for level == -1, the fine operator as PCG applies it.  Diagnostic/parity entry point. */
r3mg_status r3mg_level_apply(r3mg_handle h, int level, const double* x_dev, double* y_dev, void* stream);

/* PCG preconditioned by r3mg_vcycle (Section 6 solver): x (in: initial guess, out: solution) for nrhs
 * independent right-hand sides solved in lockstep, each frozen once ||r_k||_2 <= rtol ||r_0||_2.
 * iters and relres (host arrays of nrhs, may be NULL) receive the iteration count and final ||r||/||r_0||.
 * Returns R3MG_NOT_CONVERGED if any column reached maxit.  Synchronises. */
r3mg_status r3mg_pcg_solve(r3mg_handle h, const double* b_dev, double* x_dev, int nrhs, double rtol, int maxit,
                           void* stream, int* iters, double* relres);

/* r3mg_pcg_solve with the stop rule of the paper's experiments (Section 6: an absolute residual norm below a
 * threshold or a given reduction): each column stops once ||r_k||_2 <= max(rtol ||r_0||_2, atol).  cond (host
 * array of nrhs, may be NULL) receives the condition estimate of the preconditioned operator from the CG
 * coefficients (largest over smallest eigenvalue of the Lanczos tridiagonal of the iterations taken; the
 * "Cond." column of the paper's tables); 1 when no iteration was taken.  Errors as r3mg_pcg_solve. */
r3mg_status r3mg_pcg_solve_ex(r3mg_handle h, const double* b_dev, double* x_dev, int nrhs, double rtol, double atol,
                              int maxit, void* stream, int* iters, double* relres, double* cond);

/* Several independent problems (each with its own handle, one right-hand side each) solved by PCG in one
 * launch sequence: the iterations of all problems are captured into one hipGraph and replayed together.
 * b[k], x[k] are device vectors of handle k.  iters/relres: host arrays of `count` (may be NULL). */
r3mg_status r3mg_pcg_solve_group(int count, r3mg_handle* hs, const double* const* b, double* const* x,
                                 double rtol, int maxit, void* stream, int* iters, double* relres);

/* Convergence history of the last PCG solve on the handle (r3mg_pcg_solve, r3mg_pcg_solve_ex, or this handle's
 * problem in r3mg_pcg_solve_group): rr[j] = ||r_j||_2, the recursive residual norm after j iterations, for
 * j = 0 .. iters of column `col` (0 <= col < 16) of the last block of at most 16 right-hand sides solved.  *count
 * receives iters + 1 (0 before any solve); min(cap, *count) entries are written (rr may be NULL to query the
 * count).  After a residual-replacement restart (float32 V-cycle) the entries that follow it are the norms of the
 * restarted recursion.  Synchronises.  Errors: INVALID (col or cap out of range, handle not factored). */
r3mg_status r3mg_pcg_history(r3mg_handle h, int col, double* rr, int cap, int* count);

/* Per-level statistics: levels has room for *nlevels entries on input; on output *nlevels = level count
 * (levels may be NULL to query the count). */
r3mg_status r3mg_info(r3mg_handle h, r3mg_level_info* levels, int* nlevels);

/* Ownership of level `level` >= 1: owner_box[i] (host, n entries) = box at that level owning fine point i in
 * the caller's numbering; box_lohi (host, nboxes x 2*dim) = (lo_0..lo_{d-1}, hi_0..hi_{d-1}) per box.  Either
 * pointer may be NULL.  Available after r3mg_analyze. */
r3mg_status r3mg_export_partition(r3mg_handle h, int level, int32_t* owner_box, double* box_lohi);

/* Prolongation from level+1 to level (host CSR): level 0 rows in the caller's numbering, all B entries of
 * every unconstrained row stored; coarse numbering box * B + q.  Pass row_ptr == NULL to query the sizes via
 * *nrows / *nnz (either may be NULL).  Available after r3mg_analyze. */
r3mg_status r3mg_export_P(r3mg_handle h, int level, int64_t* row_ptr, int32_t* col, double* val,
                          int64_t* nrows, int64_t* nnz);

/* Galerkin operator of level >= 1 as host CSR (box * B + q numbering, all entries of stored blocks).  Pass
 * row_ptr == NULL to query sizes.  Requires r3mg_factor. */
r3mg_status r3mg_export_level(r3mg_handle h, int level, int64_t* row_ptr, int32_t* col, double* val,
                              int64_t* nrows, int64_t* nnz);

/* Average device time of one launch of the level-`level` fused smoother kernel (SpMV + Chebyshev update) in
 * the V-cycle precision, timed with hipEvents on `stream`, and the bytes one launch of the level's storage format
 * moves (matrix as stored, row data, 7 vector streams).  flush_bytes = 0: `reps` back-to-back launches, as a
 * smoothing sweep runs them (the caches may keep part of the matrix between launches); flush_bytes > 0: each
 * launch timed alone after a pass that reads and writes flush_bytes of other device memory (allocated for the
 * call), so that its operands come from HBM.  Diagnostic entry point for roofline measurement. */
r3mg_status r3mg_time_smoother_kernel(r3mg_handle h, int level, int reps, int64_t flush_bytes, void* stream,
                                      double* ms_per_launch, double* bytes_per_launch);

/* The same for nrhs right-hand sides (1, 2, 4, 8 or 16; interleaved vectors, as the block V-cycle applies the
 * level): the multi-right-hand-side kernels are tuned for nrhs first if no solve has tuned them, and the bytes are
 * those of the tuned kernel's storage format (fine level with the LDS-staged kernel: values, 2-byte positions,
 * distinct-column lists, block records, row order and row pointers; CSR kernels: values, 4-byte columns and row
 * pointers) plus 7 vector streams of nrhs columns.  R3MG_ERR_INVALID for another nrhs or bad arguments. */
r3mg_status r3mg_time_smoother_kernel_nrhs(r3mg_handle h, int level, int nrhs, int reps, int64_t flush_bytes,
                                           void* stream, double* ms_per_launch, double* bytes_per_launch);

/* Adjoint gradient of a per-cell coefficient (standard adjoint method; not in the paper):
 * g[e] = - sum_{a,b unconstrained} lam[c_ea] Ke_e[a,b] u[c_eb], cells (device, ncells x nloc int32, caller's
 * numbering), Ke (device float64, nloc x nloc per cell at stride ke_stride doubles; 0 = one shared matrix),
 * u, lam, g device float64. */
r3mg_status r3mg_cell_grad(r3mg_handle h, const int32_t* cells_dev, int nloc, const double* Ke_dev,
                           int64_t ke_stride, const double* u_dev, const double* lam_dev, double* g_dev,
                           int64_t ncells, void* stream);

/* Assembler of A(kappa) = sum_e kappa_e Ke_e on the unconstrained DoFs (identity on constrained rows) into
 * the handle's fine CSR pattern in the caller's order: vals_dev[s] = sum over the (cell, a, b) contributions
 * of slot s in a fixed order (deterministic).  cells (host, ncells x nloc int32).  The gather list is built
 * once on the host; every pair (a,b) of a cell must be a stored entry of the pattern or constrained. */
typedef struct r3mg_assembler_* r3mg_assembler;
r3mg_status r3mg_assembler_create(r3mg_handle h, const int32_t* cells, int nloc, int64_t ncells,
                                  r3mg_assembler* out);
r3mg_status r3mg_assemble(r3mg_assembler a, const double* kappa_dev, const double* Ke_dev, int64_t ke_stride,
                          double* vals_dev, void* stream);
void r3mg_assembler_free(r3mg_assembler a);

/* Host-only R-tree partition of points (Section 3 Definition, Section 4 point-based agglomeration): depth t
 * of the bisection tree for `leaf`, and order (host, n int32): leaf-ordered position -> point index.
 * Either output may be NULL. */
r3mg_status r3mg_rtree(const double* coords, int64_t n, int dim, int leaf, int* depth, int32_t* order);

void r3mg_free(r3mg_handle h);
const char* r3mg_status_string(r3mg_status s);
/* Message of the last failed call on the calling thread ("" after a successful call). */
const char* r3mg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* R3MG_H */
