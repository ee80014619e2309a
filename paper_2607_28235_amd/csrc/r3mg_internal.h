// Internal data structures of the R3MG-C library (host analysis + device hierarchy).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "kernels.h"
#include "r3mg.h"

namespace r3mg {

// ---------------------------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------------------------
struct Error {
  r3mg_status code;
  std::string msg;
};

#define R3MG_HIP_CHECK(expr)                                                          \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      throw ::r3mg::Error{R3MG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)

void set_last_error(const std::string& s);

// ---------------------------------------------------------------------------------------------
// Device buffer (RAII)
// ---------------------------------------------------------------------------------------------
template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n) {
    o.p = nullptr;
    o.n = 0;
  }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      o.p = nullptr;
      o.n = 0;
    }
    return *this;
  }
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    if (count == n && p) return;
    release();
    if (count == 0) return;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();  // the failed allocation must not be reported by a later launch check
      throw Error{R3MG_ERR_OOM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed"};
    }
    n = count;
  }
  void upload(const T* src, size_t count, hipStream_t s) {
    alloc(count);
    if (count) R3MG_HIP_CHECK(hipMemcpyAsync(p, src, count * sizeof(T), hipMemcpyHostToDevice, s));
  }
  void upload(const std::vector<T>& v, hipStream_t s) { upload(v.data(), v.size(), s); }
};

// ---------------------------------------------------------------------------------------------
// Host analysis results
// ---------------------------------------------------------------------------------------------
struct LocalBlocks {  // local-column row blocks of a CSR pattern (device form: FineBlocks)
  std::vector<int32_t> rb, ubp, ucol;
  std::vector<uint8_t> lidx;  // 1 or 2 bytes per nonzero, plus kFinePad padding entries
};

struct MrHost {  // blocks of one staging class of the multi-right-hand-side kernel (device form: MrBlocks)
  LocalBlocks lb;
  std::vector<int32_t> ord;  // per block, its rows in order of decreasing row length
};

struct HostLevel {           // agglomerated level l >= 1 (boxes of the R-tree at `depth`)
  int depth = 0;
  int64_t nbox = 0;
  int64_t n = 0;             // nbox * B
  std::vector<double> lo, hi;  // nbox x d
  std::vector<int64_t> bptr;   // block sparsity of A_l: nbox + 1
  std::vector<int32_t> bcol;   // sorted block columns per block row
  std::vector<double> pt1d;    // l < L: injection into the parent box, nbox x d x (p'+1)^2 [axis][child node][parent node]
  int child_shift = 0;         // l >= 2: boxes of level l-1 per box of level l = 2^child_shift
  double max_extent = 0.0;
  // l < L, when no block row is wider than 256 columns: the level as CSR (row (K, q) starts at
  // B^2 bptr[K] + q nb_K B) and its 1-byte local-column row blocks
  std::vector<int32_t> rowptr;
  LocalBlocks loc;   // local-column blocks of geometry loc_geom (0: 2048 nonzeros, 4: 3072 nonzeros)
  int loc_geom = 0;
};

struct Analysis {
  r3mg_options opt{};
  int d = 0, pc = 0, B = 0;
  int64_t n = 0, nnz = 0;
  int depth = 0;                         // R-tree depth t
  std::vector<int> depths;               // depths of levels 1..L
  std::vector<int32_t> order;            // leaf position -> user point (= perm: internal -> user)
  std::vector<int32_t> iperm;            // user -> internal
  std::vector<int64_t> leaf_off;         // internal offsets of the level-1 boxes (nbox1 + 1)
  bool cell_based = false;               // agglomeration of cells (else of support points)
  // fine-level row blocks: CSR geometries (2048/64, 4096/128, 4096/64 nonzeros/rows) and local-column
  // geometries (block offsets, distinct-column offsets and lists, local column index bytes per nonzero)
  std::vector<int32_t> rb[3];
  LocalBlocks loc[4];
  std::vector<uint8_t> constrained;      // internal order
  std::vector<uint8_t> constrained_user; // caller's order
  std::vector<int32_t> owner;            // internal point -> level-1 box, -1 if constrained
  std::vector<double> xi;                // internal point x d: local coordinates in the level-1 box
  std::vector<double> coords_int;        // internal point x d coordinates
  // fine operator in internal numbering
  std::vector<int32_t> rowptr;           // n + 1
  std::vector<int32_t> col;              // nnz
  std::vector<double> val;               // nnz
  std::vector<int64_t> src;              // internal nnz position -> user nnz position
  std::vector<int32_t> user_col;         // the caller's pattern (for assembly)
  std::vector<int64_t> user_rowptr;
  std::vector<HostLevel> lv;             // lv[0] unused (fine level); lv[l] for l = 1..L
  std::vector<int32_t> gal_ptr;          // level-1 Galerkin work lists: per stored block, entries (row, s, e)
  std::vector<int32_t> gal_ent;
  std::vector<int32_t> gal_up, gal_mir;  // blocks (K, K') with K <= K' that the kernel forms, and the block (K', K)
                                         // each one's transpose fills (-1 on the diagonal)
  int nlevels() const { return (int)depths.size() + 1; }
};

// builds the analysis; throws Error
// cells (optional, host ncells x nloc support-point indices): cell-based agglomeration
std::unique_ptr<Analysis> analyze(const double* coords, int64_t n, const int64_t* row_ptr,
                                  const int32_t* col_idx, const double* vals, const r3mg_options& opt,
                                  const int32_t* cells = nullptr, int64_t ncells = 0, int nloc = 0);

void encode_fine(Analysis& an);
// blocks of staging class cls (kMrCap / kMrRows / kMrUcap) of the multi-right-hand-side kernel over the fine level
void encode_mr_blocks(const Analysis& an, int cls, MrHost& out);

// bisection R-tree (Section 3, Section 4 point-based agglomeration); offsets[k] per depth k
void bisection_rtree(const double* coords, int64_t n, int d, int leaf, int& depth, std::vector<int32_t>& order,
                     std::vector<std::vector<int64_t>>& offsets);

// 1D GLL nodes of the box basis on [0,1]
void box_nodes_1d(int pc, double* t);

// ---------------------------------------------------------------------------------------------
// Matrix-free fine operator (host form; device layout described at MfOp in kernels.h)
// ---------------------------------------------------------------------------------------------
struct MatFreeHost {
  int d = 0, p = 0, k = 0, nloc = 0, nlocp = 0, ncomp = 0, nq = 0;
  int64_t ncells = 0;
  bool affine = false;
  std::vector<int32_t> conn;            // ncells x nlocp internal DoFs (-1: constrained or padding)
  std::vector<double> geo;              // affine: ncomp x ncells; multilinear: map coefficients and kappa
  std::vector<int32_t> inc_ptr, inc;    // per internal DoF: cell-local output positions, ascending
  std::vector<double> cd;               // diagonal of constrained rows (0 elsewhere)
  double B[4][4], G[4][4], W[4], X[4];  // 1D tables (MfTables)
};
// cells: host ncells x (p+1)^d caller indices in tensor order (x fastest); kappa: host ncells or null
MatFreeHost build_matrix_free(const Analysis& an, const int32_t* cells, int64_t ncells, int p, const double* kappa);

// ---------------------------------------------------------------------------------------------
// Device hierarchy
// ---------------------------------------------------------------------------------------------
struct MatFreeDev {
  bool on = false;
  MfOp op;
  bool affine = false;
  int p = 0;
  int64_t nincid = 0;
  DBuf<int32_t> conn, inc_ptr, inc;
  DBuf<double> geo64, cd64, y64, y64mr;
  DBuf<float> geo32, cd32, y32, y32mr;
  int mr_cap = 0;  // columns the multi-right-hand-side cell outputs (y32mr / y64mr) have room for
  MfTables<float> t32;
  MfTables<double> t64;
  double bytes32 = 0, bytes64 = 0;  // algorithmic bytes of one application (7 vector streams included)
};

struct DevLevel {
  int64_t n = 0, nbox = 0;
  int64_t nnz = 0;
  // fine level (l = 0): CSR
  DBuf<int32_t> rowptr, col;
  // coarse levels (l >= 1): block rows
  DBuf<int32_t> bptr, bcol;
  DBuf<double> val64;
  DBuf<float> val32;
  DBuf<double> dinv64;
  DBuf<float> dinv32;
  double lam_hi = 0, lam_lo = 0, lam_hat = 0;
  // Chebyshev coefficients of the level's smoother (set with the interval): first direction scale 1/theta, then
  // (c1, c2) of steps k = 1..K-1
  double cheb_inv_theta = 0;
  std::vector<double> cheb_c1, cheb_c2;
  int lanes = 8;  // lanes per row of the SpMV kernels
  DBuf<int32_t> rb[3];  // l = 0: CSR row blocks of the single-RHS row-block kernels, per geometry
  DBuf<int32_t> lrb[kLocalGeomsAll], lubp[kLocalGeomsAll], lucol[kLocalGeomsAll];  // local-column blocks per geometry
  DBuf<uint8_t> lidx[kLocalGeomsAll];
  DBuf<int32_t> lmeta[kLocalGeomsAll];  // per-block records of the local-column blocks (FineBlocks::meta)
  FineBlocks fb[kStreamShapes];  // l = 0: row blocks of every kernel shape
  // l = 0: blocks of the LDS-staged multi-right-hand-side kernel per staging class, built at the first
  // multi-right-hand-side tuning that needs them
  DBuf<int32_t> mrb[kMrClasses], mubp[kMrClasses], mucol[kMrClasses], mord[kMrClasses], mmeta[kMrClasses];
  DBuf<uint16_t> mlidx[kMrClasses];
  MrBlocks mr[kMrClasses];
  double shape_bytes[kStreamShapes] = {};  // algorithmic bytes of one application with each shape
  int shape = 0;        // l = 0: kernel shape chosen by timing at set-up
  int shape64 = 0;      // l = 0: shape of the float64 operator PCG applies (with a float64 V-cycle: shape)
  bool boxrow = false;  // l >= 1: applied by the box-row kernel (boxes of 4, 9 or 16 rows)
  int keep32 = 0, keep64 = 0;  // F_KEEP for the float32 / float64 applications (matrix stream small enough)
  int maxnb = 0;     // l >= 1: largest number of stored blocks in a block row
  // transfer to the next level
  DBuf<double> xi64;     // l = 0: n x d
  DBuf<float> xi32;
  DBuf<int32_t> owner;   // l = 0: n (level-1 box of each point, -1 if constrained)
  DBuf<int32_t> leaf_off;  // l = 0: nbox1 + 1 internal offsets of the level-1 boxes
  DBuf<int32_t> brow;    // l >= 1 during set-up: block -> block row
  DBuf<int32_t> gal_ptr, gal_ent;  // l = 1: Galerkin work lists
  DBuf<int32_t> gal_up, gal_mir;   // l = 1: the blocks formed and their mirrors
  DBuf<double> pt64;     // l >= 1 (l < L): nbox x d x (p'+1)^2
  DBuf<float> pt32;
  int child_shift = 0;   // level l >= 2: 2^child_shift boxes of level l-1 per box
  // V-cycle work vectors in the V-cycle precision (n x nrhs interleaved)
  DBuf<char> b, x, rho, dA, dB;
  int64_t vec_cap = 0;
  double bytes_apply = 0;
  const MatFreeDev* mf = nullptr;  // l = 0: matrix-free operator in use (null: CSR)
};

struct PcgScalars;  // device-side PCG state (defined in the solver)

// a fresh value for Device::graph_epoch (unique over the process)
uint64_t next_graph_epoch();

struct Device {
  int dev = 0;
  // changes whenever this device's captured graphs are dropped (a buffer they use was reallocated, new values,
  // another operator): graphs captured elsewhere from this handle (a group solve) are valid while it is unchanged
  uint64_t graph_epoch = next_graph_epoch();
  std::string tune_sig;  // tuning-cache key prefix of this handle: device and level structure (set at set-up)
  std::vector<DevLevel> lv;
  // dense coarsest: inverse (nL x nL float64, row-major); for up to kDenseSymMaxTiles tile rows also its upper
  // 64 x 64 tiles packed (csym in float64, or csym32 rounded to float32 for a float32 V-cycle; tile list ctile)
  // and the pass-1 slots for up to 4 columns (cpart)
  DBuf<double> cinv;
  int64_t nc = 0;
  DBuf<double> csym, cpart;
  DBuf<float> csym32;
  DBuf<int32_t> ctile;
  int ct = 0;  // tile rows of csym; 0 = the full inverse only
  // fine-level helpers
  DBuf<int32_t> perm;   // internal -> user
  DBuf<int64_t> src;    // internal nnz -> user nnz
  // PCG work (float64, internal numbering, n x nrhs interleaved)
  DBuf<double> px, pr, pp, pq, pz, pb;
  DBuf<double> partials;  // reduction partials
  DBuf<char> state;       // PcgState
  DBuf<double> hist;      // CG coefficients and squared residual norms per iteration (PcgState::hist, rhist)
  int hist_rows = 0;
  DBuf<int> flag;         // set-up error flag
  int64_t pcg_cap = 0;
  // graph cache: (nrhs) -> exec
  std::map<int, hipGraphExec_t> graphs;
  std::map<int, hipGraph_t> graph_defs;
  hipStream_t cap_stream = nullptr;
  void* pinned = nullptr;      // host pinned buffer: the PcgState read back at the end of a chunk of iterations
  void* pinned_dev = nullptr;  // its device address (written by a kernel, no copy engine involved)
  hipEvent_t ev[2] = {nullptr, nullptr};
  // iterations of the last converged solve per (nr, precision) key: the rtol and atol it ran to, the iterations
  // of its slowest column and their mean squared residual reduction per iteration (the first chunk of the next
  // solve is enqueued from it)
  struct SolveRecord {
    double rtol = 0, atol = 0, q = 0;
    int iters = 0;
  };
  std::map<int, SolveRecord> last_solve;
  int last_restarts = 0;  // residual-replacement restarts of the last solve (float32 V-cycle)
  // autotuned SpMM lanes per (level, nrhs)
  std::map<std::pair<int, int>, int> tuned;
  MatFreeDev mf;
  ~Device();
};

struct HandleImpl {
  std::unique_ptr<Analysis> an;
  std::unique_ptr<Device> dev;
  bool factored = false;
  DBuf<unsigned char> cons_user_dev;  // constrained mask in the caller's order (adjoint gradient)
};

// kernel family that applies a level operator (solver.cpp chooses; r3mg_info reports it)
enum class LevelKernel { Stream, BoxRow, BlockRowWG, BlockRow, Lanes, MatFree };
LevelKernel level_kernel(const Analysis& an, const DevLevel& D, int l, int nr, int esz);
std::string level_kernel_name(const Analysis& an, const DevLevel& D, int l, int esz);

// solver entry points (solver.cpp)
void device_setup(HandleImpl& h, hipStream_t s);
void update_values(HandleImpl& h, const double* vals_dev, hipStream_t s);
void vcycle_api(HandleImpl& h, const double* r, double* z, int nrhs, hipStream_t s);
// the same V-cycle with its work vectors in the static device scratch (no allocation, no synchronisation)
void vcycle_noalloc(HandleImpl& h, const double* r, double* z, int nrhs, hipStream_t s);
void level_apply(HandleImpl& h, int level, const double* x, double* y, hipStream_t s);
r3mg_status pcg_solve(HandleImpl& h, const double* b, double* x, int nrhs, double rtol, double atol, int maxit,
                      hipStream_t s, double* cond,
                      int* iters, double* relres);
r3mg_status pcg_group(int count, HandleImpl** hs, const double* const* b, double* const* x, double rtol, int maxit,
                      hipStream_t s, int* iters, double* relres);
// residual norms ||r_j||_2, j = 0..iters, of column col of the last block solved on the handle (rr may be null);
// returns iters + 1 (0 before any solve)
int residual_history(HandleImpl& h, int col, double* rr, int cap);
void time_smoother_kernel(HandleImpl& h, int level, int nrhs, int reps, int64_t flush_bytes, hipStream_t s,
                          double* ms, double* bytes);
// matrix-free fine operator: upload, check against the CSR operator, switch level 0 to it; detach returns to CSR
void attach_matrix_free(HandleImpl& h, MatFreeHost&& m, hipStream_t s);
void detach_matrix_free(HandleImpl& h);

}  // namespace r3mg

struct r3mg_handle_ {
  r3mg::HandleImpl impl;
};
