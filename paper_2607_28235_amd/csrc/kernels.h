// Launch wrappers of the R3MG-C HIP kernels (gfx950).  All launches are asynchronous on `s`.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace r3mg {

// flags of the fused level kernel (SpMV + Chebyshev/Jacobi update)
enum : int {
  F_PLAIN = 1,        // y = A u only (written to `rho`)
  F_RHO_FROM_B = 2,   // rho_old := b (x was zero)
  F_RHO_STORE = 4,    // store rho_new = rho_old - A u
  F_X_ASSIGN = 8,     // x := u
  F_X_ADD = 16,       // x += u
  F_D_OUT = 32,       // dout := c1 u + c2 dinv rho_new
  F_KEEP = 64,        // read the matrix with ordinary loads, so that it can stay in the caches between the
                      // back-to-back applications of a smoothing sweep (k_level_local_vec, k_level_boxrow and the
                      // block-row kernels; without it they read it with nontemporal loads)
};
// Largest matrix stream (values and positions) of a level that is read with F_KEEP: the 2D Q3 fine level (73 MB
// in float32, 132 MB in float64) gained, a 3D fine level of ~700 MB lost (its matrix evicted the vectors).
constexpr double kKeepCachedBytes = 128.0 * 1024 * 1024;

constexpr int kMaxNR = 16;

// Device-side PCG state of one block of up to kMaxNR columns.  all_done must stay the first word: every kernel
// of an iteration reads it through the `skip` pointer and returns at once when it is set.
struct PcgState {
  int all_done, nr, flexible, restart;  // restart: set by the true-residual check when a converged column's true
                                        // residual fails the stop rule (float32 V-cycle: residual replacement)
  int iters[kMaxNR];
  int done[kMaxNR];
  double gamma[kMaxNR], alpha[kMaxNR], beta[kMaxNR], rr[kMaxNR], rr_prev[kMaxNR], rr0[kMaxNR], tau2[kMaxNR],
      rr_true[kMaxNR];
  // CG coefficients per iteration j < hist_rows (Lanczos condition estimate): alpha_j of column k at
  // hist[2 j kMaxNR + k], beta_j at hist[(2 j + 1) kMaxNR + k]; squared recursive residual norms ||r_j||^2,
  // j = 0..hist_rows, at rhist[j kMaxNR + k]
  double* hist;
  double* rhist;
  int hist_rows, pad2;
};

// Level operator description for the fused kernel.
template <typename T>
struct LevelOp {
  int n = 0;          // rows
  int blk = 1;        // 1: CSR (ptr = row pointer, idx = columns); > 1: block rows (ptr = bptr, idx = bcol)
  const int* ptr = nullptr;
  const int* idx = nullptr;
  const T* val = nullptr;
  const T* dinv = nullptr;
  int lanes = 8;      // lanes per row (power of two, <= 64)
};

template <typename T>
void launch_level(const LevelOp<T>& op, int nr, const T* u, const T* b, T* rho, T* x, T* dout, double c1,
                  double c2, int flags, const int* skip, hipStream_t s);

// Fine-level row blocks of one kernel shape (device pointers).  A block is a run of consecutive rows.  CSR
// shapes use rb only; local-column shapes also carry, per block, its distinct columns ucol[ubp[b] .. ubp[b+1])
// (ascending) and, per nonzero, the position of its column in that list (lidx: 1 or 2 bytes per nonzero).  A
// block whose distinct columns exceed the shape's staging capacity holds a single row and is read through the
// CSR column array.
struct FineBlocks {
  int nrb = 0;
  const int* rb = nullptr;
  const int* ubp = nullptr;
  const int* ucol = nullptr;
  const void* lidx = nullptr;
  const int* meta = nullptr;  // local-column blocks: per block (first row, first nonzero, first distinct column, 0),
                              // 16-byte records, nrb + 1 of them
};

// Fine-level row-block kernel for one right-hand side.  Shapes:
//   0..2  CSR blocks, one workgroup per block; geometry (staging capacity in nonzeros, rows per block)
//         (2048, 64), (4096, 128), (4096, 64); blocks of several rows hold at most capacity - 3 nonzeros;
//   3..5  the same blocks, persistent and software-pipelined with 16-byte matrix loads (the column and value
//         arrays must carry kFinePad zero entries after the last nonzero);
//   6..8  local-column blocks, one workgroup per block: (1-byte indices, 2048 nonzeros, 64 rows, 256 distinct
//         columns), (2-byte, 4096, 64, 1024), (2-byte, 4096, 128, 1024); blocks of several rows hold at most
//         capacity - 3 nonzeros;
//   9     the blocks of shape 6 with 16-byte value loads and 4-byte loads of four packed positions (values and
//         positions must carry kFinePad padding entries);
//   10    the kernel of shape 9 over 1-byte local-column blocks of (3072 nonzeros, 128 rows, 256 columns)
//         (local geometry 3), which keep half again as many loads in flight per workgroup;
//   11    the blocks of shape 9 taken two per workgroup (k_level_local_vec_nb): both blocks' loads in flight
//         before the first barrier, each block summed as by shape 9;
//   12    the blocks of shape 10 taken two per workgroup;
//   13    the kernel of shape 9 over (3072, 64, 256) blocks (local geometry 4): agglomerated levels only.
// With partials != null (F_PLAIN only; shapes 0..8) the launch writes partial sums of u_i (A u)_i to
// partials[0..np) and returns np (<= fb.nrb).
constexpr int kCsrGeoms = 3;
constexpr int kFineShapes = 13;    // shapes 0..12 serve the fine level
constexpr int kStreamShapes = 14;  // shape 13: the vector kernel over geometry-4 blocks (agglomerated levels)
constexpr int kVecTwoFirst = 11;  // shapes 11, 12: the blocks of shapes 9, 10 taken two per workgroup
constexpr int kAggVecShape = 13;
constexpr int kLocalFirst = 6;
constexpr int kStreamCapOf[kCsrGeoms] = {2048, 4096, 4096};
constexpr int kStreamRowsOf[kCsrGeoms] = {64, 128, 64};
constexpr int kResidentBlocks = 2048;  // workgroups of 256 threads resident at once: 256 CUs x 8
constexpr int kLocalGeoms = 3;     // local geometries of the block kernels (shapes 6..8)
constexpr int kLocalGeomsAll = 5;  // geometries 3 and 4 (1-byte positions, 3072 nonzeros, 256 columns) are read by
                                   // the vector kernel only: 128-row blocks on the fine level (shape 10), 64-row
                                   // blocks on the 2D agglomerated levels, whose rows hold ~70 nonzeros (shape 13)
constexpr int kLocalCap[kLocalGeomsAll] = {2048, 4096, 4096, 3072, 3072};
constexpr int kLocalRows[kLocalGeomsAll] = {64, 64, 128, 128, 64};
constexpr int kLocalUcap[kLocalGeomsAll] = {256, 1024, 1024, 256, 256};
constexpr int kLocalIdxBytes[kLocalGeomsAll] = {1, 2, 2, 1, 1};
constexpr int kFinePad = 4;
template <typename T>
int launch_level_stream(int shape, const FineBlocks& fb, const LevelOp<T>& op, const T* u, const T* b, T* rho, T* x,
                        T* dout, double c1, double c2, int flags, const int* skip, double* partials, hipStream_t s);

// Block-row variant for the agglomerated levels and one right-hand side (one wave per box; maxnb = largest
// number of stored blocks in a block row).  Needs blockrow_lds_bytes(B, maxnb * B, sizeof(T)) <= 64 KiB.
size_t blockrow_lds_bytes(int blk, int maxw, size_t esz);
template <typename T>
void launch_level_blockrow(const LevelOp<T>& op, int maxnb, const T* u, const T* b, T* rho, T* x, T* dout, double c1,
                           double c2, int flags, const int* skip, hipStream_t s);

// Boxes of 4, 9 or 16 rows (2D agglomerated levels, p' = 1, 2, 3) with block rows of at most 64 * kBoxRowMaxNP
// entries: one wave per box, each lane owning positions of the block row in all the box's rows.
constexpr int kBoxRowMaxNP = 3;
bool boxrow_supported(int blk, int maxnb);
// Restriction fused into a box-row launch (2D, four children per parent box, boxes 4 G .. 4 G + 3 the children
// of parent G): the launch's residuals rho = b - A x of each parent's children are restricted with the
// children's 1D factors pt (2 k^2 per child, k = p' + 1) into bnext[G B + a], and dnext = dinv_next bnext
// inv_theta_next when dnext is set; the same sums in the same order as launch_restrict_c.  rho is still stored.
template <typename T>
struct BoxRestrict {
  const T* pt = nullptr;
  T* bnext = nullptr;
  const T* dinv_next = nullptr;
  T* dnext = nullptr;
  T inv_theta_next = 0;
};
template <typename T>
void launch_level_boxrow(const LevelOp<T>& op, int maxnb, const T* u, const T* b, T* rho, T* x, T* dout, double c1,
                         double c2, int flags, const int* skip, hipStream_t s, const BoxRestrict<T>* rs = nullptr);

// Wide block rows (maxnb * blk large): one workgroup per (box, 8-row chunk).
template <typename T>
void launch_level_blockrow_wg(const LevelOp<T>& op, int maxnb, const T* u, const T* b, T* rho, T* x, T* dout,
                              double c1, double c2, int flags, const int* skip, hipStream_t s);

// q = A p (float64, CSR), per-block partial <p, q> -> partials[blk * nr + k]; returns number of blocks
int launch_spmv_dot(const LevelOp<double>& op, int nr, const double* p, double* q, double* partials,
                    const int* skip, hipStream_t s);

// transfers
template <typename T>
void launch_restrict0(int nbox, int64_t n_points, int d, int pc, int nr, const int* leaf_off, const int* owner,
                      const T* xi, const T* src, T* bnext, const T* dinv_next, T* dnext, double inv_theta_next,
                      const int* skip, hipStream_t s);
// (several columns: one workgroup per level-1 box, nbox boxes with points leaf_off[K] .. leaf_off[K+1] - 1)
template <typename T>
void launch_prolong0(int n, int nbox, int d, int pc, int nr, const int* leaf_off, const int* owner, const T* xi,
                     const T* e, const T* epend, T* v, const int* skip, hipStream_t s);
template <typename T>
void launch_restrict_c(int nbox_next, int nbox, int shift, int d, int pc, int nr, const T* pt, const T* src,
                       T* bnext, const T* dinv_next, T* dnext, double inv_theta_next, const int* skip,
                       hipStream_t s);
template <typename T>
void launch_prolong_c(int nbox, int shift, int d, int pc, int nr, const T* pt, const T* e, const T* epend, T* v,
                      const int* skip, hipStream_t s);

// elementwise helpers
template <typename T>
void launch_xupdate(int64_t count, T* x, const T* v, int assign, const int* skip, hipStream_t s);
template <typename T>
void launch_vc_entry(int n, int nr, const int* perm, const double* r_user, int64_t ld_user, T* b0,
                     const T* dinv, T* d0, double inv_theta, hipStream_t s);
template <typename T>
void launch_vc_exit(int n, int nr, const int* perm, const T* x0, const T* dpend, double* z_user, int64_t ld_user,
                    hipStream_t s);
template <typename T>
void launch_dense_apply(int nc, int nr, const double* cinv, const T* b, T* x, const int* skip, hipStream_t s);
// The same product with the symmetric inverse read once: its upper-triangular 64 x 64 tiles (I <= J), listed in
// `tiles` as (I, J) pairs and packed in that order, each row-major and zero beyond nc.  Pass 1 forms every
// tile's row products and, off the diagonal, its transposed products, into part (nt x nt x 64 x nr float64,
// slot (R, S) of row block R); pass 2 sums each row block's nt slots in index order.  nr = 1, 2 or 4.
constexpr int kDenseTile = 64;
constexpr int kDenseSymMaxTiles = 160;  // coarsest sizes up to 10,240: 422 MB of packed tiles at most
constexpr int kDenseSymMaxNR = 4;
// packs the upper tiles of the full inverse, rounded to M (float64, or float32 for the float32 V-cycle)
template <typename M>
void launch_dense_pack_sym(int nc, int ntiles, const double* full, const int* tiles, M* packed, hipStream_t s);
// Prolongation fused into pass 2: the coarsest level's x (box G = rows G*B .. G*B+B-1) goes on to the level above
// as v[C*B+q'] = sum_q P~_C[q'][q] x[G*B+q] for the children C of G (nbox boxes there, child_shift shift), in
// k_prolong_c's order.
template <typename T>
struct DenseProlong {
  int nbox_coarse = 0;  // boxes of the coarsest level
  int nbox = 0, shift = 0, d = 2, pc = 1;
  const T* pt = nullptr;
  T* v = nullptr;
};
template <typename T, typename M>
void launch_dense_apply_sym(int nc, int nt, int nr, const M* packed, const int* tiles, double* part, const T* b,
                            T* x, const DenseProlong<T>* pr, const int* skip, hipStream_t s);
void launch_gather_cols(int n, int nr, int nuser, const int* perm, const double* user, int64_t ld_user,
                        double* out, hipStream_t s);
void launch_scatter_cols(int n, int nr, int nuser, const int* perm, const double* in, double* user,
                         int64_t ld_user, hipStream_t s);
void launch_cast_d2f(int64_t count, const double* a, float* b, hipStream_t s);
void launch_gather_vals(int64_t nnz, const int64_t* src, const double* user_vals, double* out, hipStream_t s);

// set-up kernels
void launch_diag_inv(int n, int blk, const int* ptr, const int* idx, const double* val, double* dinv, double* diag,
                     int* bad, hipStream_t s);
// nup blocks formed: up[t] (K <= K'), whose transpose also fills block mir[t] (-1 on the diagonal)
void launch_galerkin0(int64_t nup, int d, int pc, const int* up, const int* mir, const int* brow, const int* bptr,
                      const int* gal_ptr, const int* gal_ent, const int* owner, const double* xi, const int* col,
                      const double* val, double* out, hipStream_t s);
void launch_galerkin_c(int64_t nblocks, int d, int pc, int shift, int nbox_in, const int* brow, const int* bptr_out,
                       const int* bcol_out, const int* bptr_in, const int* bcol_in, const double* val_in,
                       const double* pt, double* out, hipStream_t s);
void launch_to_dense(int nbox, int B, const int* bptr, const int* bcol, const double* val, double* dense,
                     hipStream_t s);
void launch_lanczos_start(int n, const int* perm, double* v, hipStream_t s);
// Multi-right-hand-side CSR kernel with the columns split over lanes: G lanes per row, NR / GW column groups of
// GW = 16 / sizeof(T) columns each (G a power of two, nr / GW <= G <= 64; CSR operators only).  Same flags and
// epilogue as launch_level.  Returns false (nothing launched) for an unsupported nr or G.
template <typename T>
bool launch_level_split(const LevelOp<T>& op, int nr, int G, const T* u, const T* b, T* rho, T* x, T* dout, double c1,
                        double c2, int flags, const int* skip, hipStream_t s);
// The same product with each nonzero's value and column loaded once per row group and shared by shuffles (the G
// lanes of a row load G consecutive entries at a time).  Same arguments and conditions as launch_level_split.
template <typename T>
bool launch_level_split2(const LevelOp<T>& op, int nr, int G, const T* u, const T* b, T* rho, T* x, T* dout,
                         double c1, double c2, int flags, const int* skip, hipStream_t s);
// Fine-level blocks of the LDS-staged multi-right-hand-side kernel (device pointers), one set per staging class.
// A block is a run of consecutive rows rb[b] .. rb[b+1]; its distinct columns are ucol[ubp[b] .. ubp[b+1])
// (ascending); every nonzero stores the 2-byte position of its column in that list (lidx, kMrPad zero entries
// after the last); ord[rb[b] + i] is the block's i-th row in order of decreasing length.  A block beyond the
// class's staging capacity holds a single row, read through the CSR columns.
struct MrBlocks {
  int nrb = 0;
  int cls = -1;
  const int* rb = nullptr;
  const int* ubp = nullptr;
  const int* ucol = nullptr;
  const uint16_t* lidx = nullptr;
  const int* ord = nullptr;
  const int* meta = nullptr;  // per block (first row, first nonzero, first distinct column, 0), nrb + 1 records
};
// Staging classes (element type, right-hand sides): 0 = (float, 16), 1 = (double, 16), 2 = (double, 8).  Per
// block at most kMrCap nonzeros, kMrUcap distinct columns and kMrRows rows (256 threads / 16-byte chunks per
// column); the LDS of one workgroup (values, positions, u at the distinct columns) stays within 80 KiB, so two
// workgroups share a compute unit.
constexpr int kMrClasses = 3;
constexpr int kMrCap[kMrClasses] = {6144, 3072, 3840};
constexpr int kMrUcap[kMrClasses] = {640, 384, 640};
constexpr int kMrRows[kMrClasses] = {64, 32, 64};
constexpr int kMrPad = 8;
// staging class of nr right-hand sides in element size esz (-1: none)
inline int mr_class(int nr, int esz) {
  if (esz == 4) return nr == 16 ? 0 : -1;
  return nr == 16 ? 1 : nr == 8 ? 2 : -1;
}
// Multi-right-hand-side fine-level kernel over the blocks of staging class mr_class(nr, sizeof(T)): per block,
// values, positions and u at the distinct columns are staged in LDS; each row is summed in ascending entry order by
// the threads of its 16-byte column chunks, rows taking the row slots in order of decreasing length.  pipelined:
// one persistent workgroup per compute unit with two LDS stages, the next block's loads in flight while a block is
// summed; else one workgroup per block.  Same flags and epilogue as launch_level.  Returns false (nothing
// launched) when nr has no staging class or mb belongs to another class.
template <typename T>
bool launch_level_lmr(const MrBlocks& mb, const LevelOp<T>& op, int nr, bool pipelined, const T* u, const T* b,
                      T* rho, T* x, T* dout, double c1, double c2, int flags, const int* skip, hipStream_t s);
// partial sums of w_i x_i y_i (w may be null) -> partials (returns count)
int launch_dot(int64_t n, const double* w, const double* x, const double* y, double* partials, hipStream_t s);
void launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s);   // y = a x + b y
void launch_lanczos_u(int64_t n, const double* dinv, const double* Av, double beta_prev, const double* vprev,
                      double* u, hipStream_t s);  // u = dinv*Av - beta_prev*vprev

// ---- matrix-free fine operator: the Q_p Laplace stiffness action on multilinear cells ----
// 1D tables of the cell kernel: B[q][i] = l_i(g_q) and G[q][i] = l_i'(g_q) for the Lagrange basis l_i on the
// k = p + 1 Gauss-Lobatto nodes of [0, 1] at the k Gauss-Legendre points g_q = X[q], and the Gauss weights W[q].
template <typename T>
struct MfTables {
  T B[4][4];
  T G[4][4];
  T W[4];
  T X[4];
};
// Device description (pointers into the handle's buffers).  conn: ncells x nlocp internal DoFs per cell in
// tensor order (x fastest; -1 for constrained DoFs and padding, nlocp = k^d rounded up to a multiple of 4).
// Geometry, structure of arrays over cells (plane c at geo[c * ncells + e]):
//   affine cells:      C = kappa |det J| J^-1 J^-T (the d(d+1)/2 entries of the upper triangle, row by row);
//   multilinear cells: the coefficients of the map's derivative, x(xi) = sum over subsets S of the axes of
//                      c_S prod_{a in S} xi_a: 2D c_1, c_2, c_12 (2 values each), 3D c_1, c_2, c_3, c_12, c_13,
//                      c_23, c_123 (3 values each), then kappa; C at a Gauss point is kappa adj(J) adj(J)^T / det J.
// inc_ptr / inc: per internal DoF, the positions e * nlocp + a of its cell-local outputs in ascending order
// (empty for constrained DoFs, whose row is cd[i] u_i).
struct MfOp {
  int d = 0, k = 0, n = 0, ncells = 0, nlocp = 0;
  bool affine = false;
  const int* conn = nullptr;
  const int* inc_ptr = nullptr;
  const int* inc = nullptr;
};
// t = A u by two launches (cell-local outputs Y, then per-DoF sums in a fixed order), followed by the epilogue
// of launch_level (one right-hand side).
template <typename T>
void launch_mf_apply(const MfOp& m, const MfTables<T>& tb, const T* geo, const T* cd, T* Y, const T* dinv,
                     const T* u, const T* b, T* rho, T* x, T* dout, double c1, double c2, int flags, const int* skip,
                     hipStream_t s);

// The same for nr in {2, 4, 8, 16} interleaved right-hand sides; Y holds ncells x nlocp x nr entries.
template <typename T>
void launch_mf_apply_mr(const MfOp& m, int nr, const MfTables<T>& tb, const T* geo, const T* cd, T* Y, const T* dinv,
                        const T* u, const T* b, T* rho, T* x, T* dout, double c1, double c2, int flags,
                        const int* skip, hipStream_t s);

// Dense Cholesky factorisation A = L L^T (lower, in place, row-major n x n) and inverse A^{-1} = L^{-T} L^{-1}
// into Inv (full), in 64 x 64 tiles on the FP64 matrix cores; *bad set on a non-positive pivot.  ws: ceil(n/64)
// x 64 x 64 doubles (inverted diagonal tiles); Y: n x n doubles of scratch (L^{-1}).
void dense_cholesky_inverse(int n, double* A, double* Inv, double* ws, double* Y, int* bad, hipStream_t s);

// PCG (float64).  Each reduction is a vector kernel storing per-block partial sums (at most kPcgBlocks blocks,
// a partition that depends only on n and nr, so the iterates do not depend on the kernel that formed A p)
// followed by a one-block kernel that sums them in index order and updates the scalars of `st`.
constexpr int kPcgBlocks = 1024;
// One right-hand side: the scalar steps folded into the vector kernels after their reductions (every block forms
// the total from the per-block partials in the order of the one-block kernels; block 0 records it in the state).
// partials: 4 pcg_blocks(n) entries, area 0 <p, q>, area 1 ||r||^2, area 2 <r, z> and <q, z>.  An iteration is
// q = A p; launch_pcg_dot; launch_pcg_xr1 (alpha, x, r); the V-cycle; launch_pcg_z1 (stop test, z); launch_pcg_p1
// (beta, p).  Enqueued as two halves, the stop test ends the first (launch_pcg_check1) and launch_pcg_z1 runs
// without it.  launch_pcg_z with mode 1 at the start of a solve must write its partials to area 2.
int pcg_blocks(int n);
void launch_pcg_dot(int n, const double* p, const double* q, double* partials, PcgState* st, hipStream_t s);
template <typename T>
void launch_pcg_xr1(int n, PcgState* st, double* x, double* r, const double* p, const double* q, double* partials,
                    T* b0, const T* dinv0, T* d0, double inv_theta0, hipStream_t s);
template <typename T>
void launch_pcg_z1(int n, PcgState* st, bool check, const T* x0, const T* dpend, double* z, const double* r,
                   const double* q, double* partials, hipStream_t s);
void launch_pcg_check1(int n, PcgState* st, const double* partials, hipStream_t s);
void launch_pcg_p1(int n, PcgState* st, const double* z, double* p, const double* partials, hipStream_t s);
// <p, q> per column (n x nr interleaved) and alpha = gamma / <p, q> (0 for converged columns); skips when
// st->all_done.  nr in {1, 2, 4, 8, 16}.
void launch_pcg_dot_alpha(int n, int nr, const double* p, const double* q, double* partials, PcgState* st,
                          hipStream_t s);
// alpha from partials[b * nr + k], b < npart, formed by another kernel (the lanes kernel's fused dot)
void launch_pcg_alpha(int nr, PcgState* st, const double* partials, int npart, hipStream_t s);
// x += alpha p; r -= alpha q; ||r||^2 and the stop test (iteration counts, done flags, all_done, residual
// history); V-cycle entry b0 = (T) r (float32 V-cycle only) and d0 = dinv0 b0 / theta0 when d0 is set
template <typename T>
void launch_pcg_xr(int n, int nr, PcgState* st, double* x, double* r, const double* p, const double* q,
                   double* partials, T* b0, const T* dinv0, T* d0, double inv_theta0, hipStream_t s);
// z = (double)(x0 + dpend) (dpend may be null).  mode 0: nothing else (st may be null); mode 1 (PCG start):
// p = z and gamma = <r, z>; mode 2 (iteration): beta = <r, z> / gamma, or -alpha <q, z> / gamma with q set
// (flexible), and gamma = <r, z>.  Modes 1 and 2 skip when st->all_done.
template <typename T>
void launch_pcg_z(int n, int nr, PcgState* st, int mode, const T* x0, const T* dpend, double* z, const double* r,
                  const double* q, double* p, double* partials, hipStream_t s);
void launch_pcg_p(int n, int nr, PcgState* st, const double* z, double* p, hipStream_t s);
// r = b - q and the initial state: ||r_0||^2, tau^2 = max(rtol^2 ||r_0||^2, atol^2), done flags (columns
// k >= nr_active are done from the start).  restart = 1: a restart from the true residual that keeps tau^2,
// ||r_0||^2 and the iteration counts of every column.
void launch_pcg_residual_init(int n, int nr, const double* b, const double* q, double* r, double* partials,
                              PcgState* st, int restart, double rtol, double atol, int nr_active, int flexible,
                              double* hist, double* rhist, int hist_rows, hipStream_t s);
// ||b - q||^2 per column into st->rr_true; st->restart = 1 if a converged column fails its stop rule with it.
// Never skips (it runs after the iterations).
void launch_pcg_true_residual(int n, int nr, const double* b, const double* q, double* partials, PcgState* st,
                              hipStream_t s);
// copy *st to host-mapped pinned memory (device address of a hipHostMalloc buffer)
void launch_pcg_state_out(const PcgState* st, PcgState* host_mapped, hipStream_t s);
template <typename T>
void launch_vc_prep(int n, int nr, const double* r, T* b0, const T* dinv0, T* d0, double inv_theta0,
                    const int* skip, hipStream_t s);

// FEM helpers (adjoint gradient, kappa assembly)
void launch_cell_grad(int64_t ncells, int nloc, const int* cells, const double* Ke, int64_t ke_stride,
                      const double* u, const double* lam, const unsigned char* constrained_user, double* g,
                      hipStream_t s);
void launch_assemble(int64_t nnz, const int64_t* slot_ptr, const int64_t* contrib, const double* kappa,
                     const double* Ke, int64_t ke_stride, int nloc, const unsigned char* diag_one, double* vals,
                     hipStream_t s);

}  // namespace r3mg
