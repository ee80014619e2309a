// Device set-up, V-cycle and PCG drivers of the R3MG-C library.
//
// Paper Section 4 (multilevel preconditioner: inherited operators, transfers, one V-cycle per CG iteration),
// Section 5 Remark on the smoother and Section 6 (Chebyshev-Jacobi smoother tuned by Lanczos, direct coarsest
// solve, PCG stopping rule).  The V-cycle is the symmetric multiplicative cycle
//   B_L r = A_L^{-1} r;  B_l r: x = S^nu(r,0); r_c = P^T (r - A x); x += P B_{l+1} r_c; x = S^nu(r, x).
// Each smoothing application is the Chebyshev recurrence on D^{-1}A started from the current iterate.  The
// implementation carries the unscaled residual rho = b - A x through every step, so that every operator
// application of a level is one fused kernel (t = A u; rho -= t; x += u; d = c1 u + c2 D^{-1} rho): the
// residual at the start of an application and the residual that is restricted are obtained from the last
// direction instead of a separate b - A x pass.  In exact arithmetic the iterates equal the textbook ones.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <numeric>
#include <vector>

#include "kernels.h"
#include "tunecache.h"
#include "noalloc.h"
#include "r3mg_internal.h"

namespace r3mg {

uint64_t next_graph_epoch() {
  static std::atomic<uint64_t> epoch{0};
  return ++epoch;
}

namespace {

double sturm_max(const std::vector<double>& a, const std::vector<double>& b) {
  const int m = (int)a.size();
  std::vector<double> off(m, 0.0);
  for (int i = 0; i + 1 < m; ++i) {
    off[i] += std::fabs(b[i]);
    off[i + 1] += std::fabs(b[i]);
  }
  double lo = INFINITY, hi = -INFINITY;
  for (int i = 0; i < m; ++i) {
    lo = std::min(lo, a[i] - off[i]);
    hi = std::max(hi, a[i] + off[i]);
  }
  auto count_below = [&](double x) {
    int cnt = 0;
    double q = a[0] - x;
    if (q < 0) ++cnt;
    for (int k = 1; k < m; ++k) {
      if (q == 0.0) q = 1e-300;
      q = a[k] - x - b[k - 1] * b[k - 1] / q;
      if (q < 0) ++cnt;
    }
    return cnt;
  };
  for (int it = 0; it < 200; ++it) {
    if (hi - lo <= 1e-15 * std::max(1.0, std::fabs(hi))) break;
    double mid = 0.5 * (lo + hi);
    if (count_below(mid) == m)
      hi = mid;
    else
      lo = mid;
  }
  return hi;
}

// smallest eigenvalue of the symmetric tridiagonal (a, b) by Sturm bisection
static double sturm_min(const std::vector<double>& a, const std::vector<double>& b) {
  const int m = (int)a.size();
  std::vector<double> off(m, 0.0);
  for (int i = 0; i + 1 < m; ++i) {
    off[i] += std::fabs(b[i]);
    off[i + 1] += std::fabs(b[i]);
  }
  double lo = INFINITY, hi = -INFINITY;
  for (int i = 0; i < m; ++i) {
    lo = std::min(lo, a[i] - off[i]);
    hi = std::max(hi, a[i] + off[i]);
  }
  auto count_below = [&](double x) {
    int cnt = 0;
    double q = a[0] - x;
    if (q < 0) ++cnt;
    for (int k = 1; k < m; ++k) {
      if (q == 0.0) q = 1e-300;
      q = a[k] - x - b[k - 1] * b[k - 1] / q;
      if (q < 0) ++cnt;
    }
    return cnt;
  };
  for (int it = 0; it < 200; ++it) {
    if (hi - lo <= 1e-15 * std::max(std::fabs(lo), std::fabs(hi))) break;
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) >= 1)
      hi = mid;
    else
      lo = mid;
  }
  return 0.5 * (lo + hi);
}

// Condition estimate of the preconditioned operator from m CG steps (the Lanczos tridiagonal of the CG
// coefficients): T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1}, T_j,j+1 = sqrt(beta_j)/alpha_j; lambda_max / lambda_min.
static double cg_condition(const std::vector<double>& alpha, const std::vector<double>& beta) {
  const int m = (int)alpha.size();
  if (m == 0) return 1.0;
  std::vector<double> a(m), b(m > 1 ? m - 1 : 0);
  for (int j = 0; j < m; ++j) {
    a[j] = 1.0 / alpha[j] + (j > 0 ? beta[j - 1] / alpha[j - 1] : 0.0);
    if (j + 1 < m) b[j] = std::sqrt(beta[j]) / alpha[j];
  }
  return sturm_max(a, b) / sturm_min(a, b);
}

int lanes_for(double avg_row) {
  int g = 2;
  while (g < 64 && g * 4 < avg_row) g <<= 1;
  return g;
}

template <typename T>
T* vbuf(DBuf<char>& b) {
  return reinterpret_cast<T*>(b.p);
}

double host_sum(const double* dev, int cnt, hipStream_t s) {
  std::vector<double> h(cnt);
  R3MG_HIP_CHECK(hipMemcpyAsync(h.data(), dev, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
  R3MG_HIP_CHECK(hipStreamSynchronize(s));
  double acc = 0;
  for (double v : h) acc += v;
  return acc;
}

// every kernel that writes per-block partial sums is checked against the buffer before launch
void need_partials(Device& dv, int64_t count) {
  if (count > (int64_t)dv.partials.n)
    throw Error{R3MG_ERR_INVALID, "internal: reduction buffer too small (" + std::to_string(count) + " > " +
                                      std::to_string(dv.partials.n) + ")"};
}

void drop_graphs(Device& dv) {
  for (auto& kv : dv.graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto& kv : dv.graph_defs) (void)hipGraphDestroy(kv.second);
  dv.graphs.clear();
  dv.graph_defs.clear();
  dv.graph_epoch = next_graph_epoch();
}

}  // namespace

Device::~Device() {
  drop_graphs(*this);
  for (auto e : ev)
    if (e) (void)hipEventDestroy(e);
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  if (pinned) (void)hipHostFree(pinned);
}

struct Ctx {
  Analysis& an;
  Device& dv;
  bool fp32;
  // V-cycle work vectors of this call, kWorkSlots per level (null: the handle's own buffers, DevLevel::b ...)
  char* const* work = nullptr;
};

// V-cycle work vector `slot` of level l: the call's table, else the handle's buffer
enum : int { W_B = 0, W_X, W_RHO, W_DA, W_DB, kWorkSlots };
template <typename T>
T* wv(Ctx& c, int l, int slot) {
  if (c.work) return reinterpret_cast<T*>(c.work[(size_t)l * kWorkSlots + slot]);
  DevLevel& D = c.dv.lv[l];
  DBuf<char>* bufs[kWorkSlots] = {&D.b, &D.x, &D.rho, &D.dA, &D.dB};
  return reinterpret_cast<T*>(bufs[slot]->p);
}

template <typename T>
LevelOp<T> level_op(Ctx& c, int l) {
  DevLevel& D = c.dv.lv[l];
  LevelOp<T> op;
  op.n = (int)D.n;
  op.lanes = D.lanes;
  if (l == 0) {
    op.blk = 1;
    op.ptr = D.rowptr.p;
    op.idx = D.col.p;
  } else {
    op.blk = c.an.B;
    op.ptr = D.bptr.p;
    op.idx = D.bcol.p;
  }
  if constexpr (sizeof(T) == 4) {
    op.val = D.val32.p;
    op.dinv = D.dinv32.p;
  } else {
    op.val = D.val64.p;
    op.dinv = D.dinv64.p;
  }
  return op;
}

// Tuned multi-RHS kernel codes, per (level, nr, precision): G in 1..64 = lanes-per-row CSR/block-row kernel with
// G lanes; kCodeSplit + G = column-split CSR kernel with G lanes; kCodeSplit2 + G = the column-split kernel with
// shared entry loads; -1 / -2 = LDS-staged kernel, pipelined / one workgroup per block.  Level -1 holds PCG's
// float64 q = A p (with its dot products).
constexpr int kCodeSplit = 100;
constexpr int kCodeSplit2 = 200;

// the column-split kernel a code >= kCodeSplit names
template <typename T>
static bool launch_split_code(int code, const LevelOp<T>& op, int nr, const T* u, const T* b, T* rho, T* x, T* dout,
                              double c1, double c2, int flags, const int* skip, hipStream_t s) {
  if (code >= kCodeSplit2)
    return launch_level_split2<T>(op, nr, code - kCodeSplit2, u, b, rho, x, dout, c1, c2, flags, skip, s);
  return launch_level_split<T>(op, nr, code - kCodeSplit, u, b, rho, x, dout, c1, c2, flags, skip, s);
}

// Kernel that applies level l for nr right-hand sides in element size esz: the row-block kernel on the fine
// level for one right-hand side, a block-row kernel on coarse levels whose block rows fit LDS, the
// lanes-per-row kernel otherwise.
LevelKernel level_kernel(const Analysis& an, const DevLevel& D, int l, int nr, int esz) {
  if (l == 0 && D.mf) return LevelKernel::MatFree;
  if (l > 0 && nr == 1 && D.boxrow) return LevelKernel::BoxRow;
  if (nr == 1 && D.fb[D.shape].nrb > 0 && (l == 0 || D.shape >= kLocalFirst + kLocalGeoms)) return LevelKernel::Stream;
  if (l > 0 && nr == 1 && D.maxnb > 0 && an.B >= 8 && (int64_t)D.maxnb * an.B >= 256 &&
      (int64_t)D.maxnb * an.B * esz <= 65536)
    return LevelKernel::BlockRowWG;
  if (l > 0 && nr == 1 && D.maxnb > 0 && an.B <= 64 && blockrow_lds_bytes(an.B, D.maxnb * an.B, esz) <= 65536)
    return LevelKernel::BlockRow;
  return LevelKernel::Lanes;
}

std::string level_kernel_name(const Analysis& an, const DevLevel& D, int l, int esz) {
  const char* t = esz == 4 ? "float" : "double";
  switch (level_kernel(an, D, l, 1, esz)) {
    case LevelKernel::Stream:
      if (D.shape >= kLocalFirst) {
        // shapes 9..13 (vector kernel): geometries 0, 3, 0, 3, 4; shapes 11 and 12 ("vec2") take two blocks per
        // workgroup
        const bool vec = D.shape >= kLocalFirst + kLocalGeoms;
        static const int vec_geom[5] = {0, 3, 0, 3, 4};
        const int g = !vec ? D.shape - kLocalFirst : vec_geom[D.shape - kLocalFirst - kLocalGeoms];
        const bool two = D.shape == kVecTwoFirst || D.shape == kVecTwoFirst + 1;
        return std::string("k_level_local<") + t + ",u" + std::to_string(8 * kLocalIdxBytes[g]) + "," +
               std::to_string(kLocalCap[g]) + "," + std::to_string(kLocalRows[g]) + "," +
               std::to_string(kLocalUcap[g]) + (!vec ? ",block>" : two ? ",vec2>" : ",vec>");
      }
      return std::string("k_level_stream<") + t + "," + std::to_string(kStreamCapOf[D.shape % kCsrGeoms]) + "," +
             std::to_string(kStreamRowsOf[D.shape % kCsrGeoms]) + (D.shape >= kCsrGeoms ? ",pipe16>" : ",block>");
    case LevelKernel::MatFree:
      return std::string("k_mf_cell<") + t + "," + std::to_string(D.mf->op.d) + "D,Q" + std::to_string(D.mf->p) +
             (D.mf->affine ? ",affine>" : ",multilinear>") + "+k_mf_gather<" + t + ">";
    case LevelKernel::BoxRow: return std::string("k_level_boxrow<") + t + "," + std::to_string(an.B) + ">";
    case LevelKernel::BlockRowWG: return std::string("k_level_blockrow_wg<") + t + ">";
    case LevelKernel::BlockRow: return std::string("k_level_blockrow<") + t + ">";
    default: return std::string("k_level<") + t + ">";
  }
}

// Blocks of staging class cls of the LDS-staged multi-RHS kernel over the fine CSR level, encoded on the host and
// uploaded the first time a tuning needs them (false: no staging class, or the fine level is matrix-free)
static bool ensure_mr_blocks(Ctx& c, int cls, hipStream_t s) {
  DevLevel& D = c.dv.lv[0];
  if (cls < 0 || D.mf) return false;
  if (D.mr[cls].nrb > 0) return true;
  MrHost h;
  encode_mr_blocks(c.an, cls, h);
  D.mrb[cls].upload(h.lb.rb, s);
  D.mubp[cls].upload(h.lb.ubp, s);
  h.lb.ucol.push_back(0);  // padding entry: the kernel's clamped staging loads of a block without columns
  D.mucol[cls].upload(h.lb.ucol, s);
  D.mord[cls].upload(h.ord, s);
  {
    std::vector<int32_t> meta(h.lb.rb.size() * 4, 0);
    for (size_t k = 0; k < h.lb.rb.size(); ++k) {
      meta[4 * k] = h.lb.rb[k];
      meta[4 * k + 1] = c.an.rowptr[h.lb.rb[k]];
      meta[4 * k + 2] = h.lb.ubp[k];
    }
    D.mmeta[cls].upload(meta, s);
    R3MG_HIP_CHECK(hipStreamSynchronize(s));
  }
  D.mlidx[cls].upload(reinterpret_cast<const uint16_t*>(h.lb.lidx.data()), h.lb.lidx.size() / 2, s);
  R3MG_HIP_CHECK(hipStreamSynchronize(s));  // the host vectors are released on return
  MrBlocks& m = D.mr[cls];
  m.cls = cls;
  m.rb = D.mrb[cls].p;
  m.ubp = D.mubp[cls].p;
  m.ucol = D.mucol[cls].p;
  m.lidx = D.mlidx[cls].p;
  m.ord = D.mord[cls].p;
  m.meta = D.mmeta[cls].p;
  m.nrb = (int)h.lb.rb.size() - 1;
  return true;
}

// F_KEEP when the level's matrix stream in precision T is small enough to stay in the caches
template <typename T>
static int keep_flag(const DevLevel& D) {
  return sizeof(T) == 4 ? D.keep32 : D.keep64;
}

template <typename T>
void apply_level(Ctx& c, int l, int nr, const T* u, const T* b, T* rho, T* x, T* dout, double c1, double c2, int flags,
                 const int* skip, hipStream_t s, const BoxRestrict<T>* rs = nullptr) {
  LevelOp<T> op = level_op<T>(c, l);
  DevLevel& D = c.dv.lv[l];
  switch (level_kernel(c.an, D, l, nr, (int)sizeof(T))) {
    case LevelKernel::MatFree: {
      const MatFreeDev& F = *D.mf;
      if (nr > 1 && nr > F.mr_cap) throw std::runtime_error("matrix-free operator: multi-RHS outputs not allocated");
      if constexpr (sizeof(T) == 4) {
        if (nr == 1)
          launch_mf_apply<float>(F.op, F.t32, F.geo32.p, F.cd32.p, F.y32.p, op.dinv, u, b, rho, x, dout, c1, c2,
                                 flags, skip, s);
        else
          launch_mf_apply_mr<float>(F.op, nr, F.t32, F.geo32.p, F.cd32.p, F.y32mr.p, op.dinv, u, b, rho, x, dout,
                                    c1, c2, flags, skip, s);
      } else {
        if (nr == 1)
          launch_mf_apply<double>(F.op, F.t64, F.geo64.p, F.cd64.p, F.y64.p, op.dinv, u, b, rho, x, dout, c1, c2,
                                  flags, skip, s);
        else
          launch_mf_apply_mr<double>(F.op, nr, F.t64, F.geo64.p, F.cd64.p, F.y64mr.p, op.dinv, u, b, rho, x, dout,
                                     c1, c2, flags, skip, s);
      }
      break;
    }
    case LevelKernel::Stream: {
      op.ptr = D.rowptr.p;  // CSR row pointers (coarse levels: of the block-row layout)
      op.idx = D.col.p;     // CSR columns (fine level only; coarse rows never take the long-row path)
      const int sh = (l == 0 && sizeof(T) == 8) ? D.shape64 : D.shape;
      launch_level_stream<T>(sh, D.fb[sh], op, u, b, rho, x, dout, c1, c2, flags | keep_flag<T>(D), skip, nullptr,
                             s);
      break;
    }
    case LevelKernel::BoxRow:
      launch_level_boxrow<T>(op, D.maxnb, u, b, rho, x, dout, c1, c2, flags | keep_flag<T>(D), skip, s, rs);
      break;
    case LevelKernel::BlockRowWG:
      launch_level_blockrow_wg<T>(op, D.maxnb, u, b, rho, x, dout, c1, c2, flags | keep_flag<T>(D), skip, s);
      break;
    case LevelKernel::BlockRow:
      launch_level_blockrow<T>(op, D.maxnb, u, b, rho, x, dout, c1, c2, flags | keep_flag<T>(D), skip, s);
      break;
    default: {
      if (nr > 1) {
        auto it = c.dv.tuned.find({l, nr * 2 + (sizeof(T) == 4 ? 1 : 0)});
        if (it != c.dv.tuned.end()) {
          if (it->second < 0) {  // fine level: LDS-staged multi-RHS kernel (-1: pipelined, -2: block per workgroup)
            op.ptr = D.rowptr.p;
            op.idx = D.col.p;
            const int cls = mr_class(nr, (int)sizeof(T));
            if (cls < 0 || !launch_level_lmr<T>(D.mr[cls], op, nr, it->second == -1, u, b, rho, x, dout, c1, c2,
                                                flags | keep_flag<T>(D), skip, s))
              throw std::runtime_error("multi-RHS LDS-staged kernel: no blocks for this shape");
            break;
          }
          if (it->second >= kCodeSplit) {  // fine level: column-split CSR kernel
            op.ptr = D.rowptr.p;
            op.idx = D.col.p;
            if (!launch_split_code<T>(it->second, op, nr, u, b, rho, x, dout, c1, c2, flags, skip, s))
              throw std::runtime_error("multi-RHS column-split kernel: unsupported shape");
            break;
          }
          op.lanes = it->second;
        }
      }
      launch_level<T>(op, nr, u, b, rho, x, dout, c1, c2, flags, skip, s);
    }
  }
}

static void ensure_level_vectors(Ctx& c, int nr) {
  const size_t s = c.fp32 ? sizeof(float) : sizeof(double);
  const int L = c.an.nlevels() - 1;
  MatFreeDev& F = c.dv.mf;
  if (c.dv.lv[0].mf && nr > 1 && F.mr_cap < nr) {
    // cell outputs of the matrix-free operator for nr columns (float64 for PCG's A p, plus the V-cycle precision)
    const int64_t entries = (int64_t)F.op.ncells * F.op.nlocp * nr;
    if (entries >= (int64_t(1) << 31) || (int64_t)F.op.n * nr >= (int64_t(1) << 31))
      throw Error{R3MG_ERR_INVALID, "matrix-free operator: too many cell-local entries for this many right-hand sides"};
    F.y64mr.alloc((size_t)entries);
    if (c.fp32) F.y32mr.alloc((size_t)entries);
    F.mr_cap = nr;
    drop_graphs(c.dv);
  }
  for (int l = 0; l <= L; ++l) {
    DevLevel& D = c.dv.lv[l];
    if (D.vec_cap >= D.n * nr) continue;
    const size_t bytes = (size_t)D.n * nr * s;
    DBuf<char>* bufs[5] = {&D.b, &D.x, &D.rho, &D.dA, &D.dB};
    for (DBuf<char>* bp : bufs) {
      bp->alloc(bytes);
      R3MG_HIP_CHECK(hipMemset(bp->p, 0, bytes));
    }
    D.vec_cap = D.n * nr;
    drop_graphs(c.dv);
  }
}

static void ensure_pcg_vectors(Ctx& c, int nr) {
  Device& dv = c.dv;
  const int64_t n = c.an.n;
  if (dv.pcg_cap < n * nr) {
    DBuf<double>* bufs[6] = {&dv.px, &dv.pr, &dv.pp, &dv.pq, &dv.pz, &dv.pb};
    for (DBuf<double>* bp : bufs) {
      bp->alloc((size_t)n * nr);
      R3MG_HIP_CHECK(hipMemset(bp->p, 0, (size_t)n * nr * sizeof(double)));
    }
    dv.pcg_cap = n * nr;
    // the fine-level SpMV uses 256 / lanes rows per block; vector kernels 256 rows per block
    const int64_t rpb = 256 / std::max(nr > 1 ? 8 : 1, dv.lv[0].lanes);
    const int64_t nlog_spmv = (n + rpb - 1) / rpb;
    const int64_t nlog_vec = (n + 255) / 256;
    size_t nrb_max = 0;
    for (int sh = 0; sh < kStreamShapes; ++sh) nrb_max = std::max(nrb_max, (size_t)dv.lv[0].fb[sh].nrb);
    // (the PCG reductions: two partials per column and block, at most kPcgBlocks blocks)
    dv.partials.alloc(std::max<size_t>({(size_t)4096, (size_t)(nlog_spmv * nr), (size_t)(nlog_vec * 2 * nr), nrb_max,
                                        (size_t)kPcgBlocks * 2 * nr}));
    drop_graphs(dv);
  }
  if (!dv.state.p) {
    dv.state.alloc(sizeof(PcgState));
    R3MG_HIP_CHECK(hipMemset(dv.state.p, 0, sizeof(PcgState)));
  }
  // pinned host memory for the state read back at the end of a chunk of iterations, written by a kernel through
  // its device address
  if (!dv.pinned) {
    R3MG_HIP_CHECK(hipHostMalloc(&dv.pinned, sizeof(PcgState) + 64, hipHostMallocDefault));
    R3MG_HIP_CHECK(hipHostGetDevicePointer(&dv.pinned_dev, dv.pinned, 0));
  }
}

// Multi-RHS SpMM tile autotuner: the lanes-per-row tile of every level kernel (and of PCG's float64 SpMV) is
// chosen per (level, nrhs, precision) by timing each candidate with hipEvents on the level's own work vectors
// (3 warm-up + 5 timed launches), once per handle; the choice is cached and used by every later solve.  Must run
// outside graph capture (it synchronises).
static float time_launches(hipStream_t s, int reps, const std::function<void()>& f) {
  hipEvent_t e0, e1;
  R3MG_HIP_CHECK(hipEventCreate(&e0));
  R3MG_HIP_CHECK(hipEventCreate(&e1));
  for (int r = 0; r < 3; ++r) f();
  R3MG_HIP_CHECK(hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r) f();
  R3MG_HIP_CHECK(hipEventRecord(e1, s));
  R3MG_HIP_CHECK(hipEventSynchronize(e1));
  float ms = 0;
  R3MG_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms / reps;
}

// whether a multi-RHS kernel code read from the tuning cache can apply level l (-1: PCG's float64 operator) for nr
// columns of element size esz (building the LDS-staged kernel's blocks when it names that kernel)
static bool valid_mr_code(Ctx& c, int l, int nr, int esz, int code, hipStream_t s) {
  auto pow2 = [](int g, int hi) { return g >= 1 && g <= hi && (g & (g - 1)) == 0; };
  if (l > 0) return pow2(code, 64);
  if (l < 0 && pow2(code, 8)) return true;
  if (l == 0 && pow2(code, 64)) return true;
  if (code == -1 || code == -2) return ensure_mr_blocks(c, mr_class(nr, esz), s);
  return pow2(code - kCodeSplit, 64) || pow2(code - kCodeSplit2, 64);
}

// tuning-cache key of a multi-RHS choice
static std::string mr_tune_key(const Device& dv, int l, int nr, int esz) {
  return dv.tune_sig + "/mr/" + std::to_string(l) + "/" + std::to_string(nr) + "/" + std::to_string(esz);
}

template <typename T>
static void autotune_spmm(Ctx& c, int nr, hipStream_t s) {
  if (nr <= 1) return;
  Device& dv = c.dv;
  const int L = c.an.nlevels() - 1;
  const int tag = nr * 2 + (sizeof(T) == 4 ? 1 : 0);
  const int forced = c.an.opt.multi_rhs_kernel;  // -1 timed, 0 lanes, 1 / 2 LDS-staged, 3 / 4 column-split
  const bool cache = forced == -1 && c.an.opt.tune_cache != 0 && !dv.tune_sig.empty();
  const int fl = F_RHO_STORE | F_X_ADD | F_D_OUT;
  for (int l = 0; l < L; ++l) {
    if (dv.tuned.count({l, tag})) continue;
    DevLevel& D = dv.lv[l];
    if (l == 0 && D.mf) continue;  // the matrix-free operator applies the fine level
    int cached = 0;
    if (cache && tune_cache_get(mr_tune_key(dv, l, nr, (int)sizeof(T)), &cached) &&
        valid_mr_code(c, l, nr, (int)sizeof(T), cached, s)) {
      dv.tuned[{l, tag}] = cached;
      continue;
    }
    LevelOp<T> op = level_op<T>(c, l);
    float best = 1e30f;
    int bestCode = D.lanes;
    auto consider = [&](int code, float ms, bool ok, bool allowed) {
      if (ok && allowed && ms < best) {
        best = ms;
        bestCode = code;
      }
    };
    const bool fine = l == 0;
    for (int G = 1; G <= 64; G <<= 1) {
      op.lanes = G;
      const float ms = time_launches(s, 5, [&] {
        launch_level<T>(op, nr, vbuf<T>(D.dA), vbuf<T>(D.b), vbuf<T>(D.rho), vbuf<T>(D.x), vbuf<T>(D.dB), 0.0, 0.0, fl,
                        nullptr, s);
      });
      consider(G, ms, true, !fine || forced <= 0);
    }
    if (fine) {
      LevelOp<T> opc = op;
      opc.ptr = D.rowptr.p;
      opc.idx = D.col.p;
      const int cls = mr_class(nr, (int)sizeof(T));
      for (int g = 0; g < 2; ++g) {
        if ((forced != -1 && forced != 1 + g) || !ensure_mr_blocks(c, cls, s)) continue;
        bool ok = true;
        const float ms = time_launches(s, 5, [&] {
          ok = launch_level_lmr<T>(D.mr[cls], opc, nr, g == 0, vbuf<T>(D.dA), vbuf<T>(D.b), vbuf<T>(D.rho),
                                   vbuf<T>(D.x), vbuf<T>(D.dB), 0.0, 0.0, fl | keep_flag<T>(D), nullptr, s);
        });
        consider(-1 - g, ms, ok, true);
      }
      if (forced == -1 || forced == 3)
        for (int G = 1; G <= 64; G <<= 1) {
          bool ok = true;
          const float ms = time_launches(s, 5, [&] {
            ok = launch_level_split<T>(opc, nr, G, vbuf<T>(D.dA), vbuf<T>(D.b), vbuf<T>(D.rho), vbuf<T>(D.x),
                                       vbuf<T>(D.dB), 0.0, 0.0, fl, nullptr, s);
          });
          consider(kCodeSplit + G, ms, ok, true);
        }
      if (forced == -1 || forced == 4)
        for (int G = 1; G <= 64; G <<= 1) {
          bool ok = true;
          const float ms = time_launches(s, 5, [&] {
            ok = launch_level_split2<T>(opc, nr, G, vbuf<T>(D.dA), vbuf<T>(D.b), vbuf<T>(D.rho), vbuf<T>(D.x),
                                        vbuf<T>(D.dB), 0.0, 0.0, fl, nullptr, s);
          });
          consider(kCodeSplit2 + G, ms, ok, true);
        }
    }
    dv.tuned[{l, tag}] = bestCode;
    if (cache) tune_cache_put(mr_tune_key(dv, l, nr, (int)sizeof(T)), bestCode);
    R3MG_HIP_CHECK(hipMemsetAsync(D.x.p, 0, D.x.n, s));
  }
  // PCG's float64 q = A p and <p, q>: lanes kernel with fused partial dots (at most 8 lanes: bounded number of
  // partials), or the local-column / column-split kernel followed by the per-column dot in a fixed partition
  int cached = 0;
  if (!dv.tuned.count({-1, nr * 2}) && !dv.lv[0].mf && cache &&
      tune_cache_get(mr_tune_key(dv, -1, nr, 8), &cached) && valid_mr_code(c, -1, nr, 8, cached, s)) {
    dv.tuned[{-1, nr * 2}] = cached;
    if (cached >= 1 && cached <= 8) need_partials(dv, (int64_t)((c.an.n + 256 / cached - 1) / (256 / cached)) * nr);
    else need_partials(dv, (int64_t)kPcgBlocks * 2 * nr);
  }
  if (!dv.tuned.count({-1, nr * 2}) && !dv.lv[0].mf) {
    LevelOp<double> op = level_op<double>(c, 0);
    DevLevel& D0 = dv.lv[0];
    float best = 1e30f;
    int bestCode = 1;
    // every candidate ends with alpha in the state: time them on a cleared state (not converged, gamma = 0)
    R3MG_HIP_CHECK(hipMemsetAsync(dv.state.p, 0, sizeof(PcgState), s));
    PcgState* st0 = reinterpret_cast<PcgState*>(dv.state.p);
    if (forced <= 0)
      for (int G = 1; G <= 8; G <<= 1) {
        op.lanes = G;
        need_partials(dv, (int64_t)((c.an.n + 256 / G - 1) / (256 / G)) * nr);
        const float ms = time_launches(s, 5, [&] {
          const int np = launch_spmv_dot(op, nr, dv.pp.p, dv.pq.p, dv.partials.p, nullptr, s);
          launch_pcg_alpha(nr, st0, dv.partials.p, np, s);
        });
        if (ms < best) {
          best = ms;
          bestCode = G;
        }
      }
    op.ptr = D0.rowptr.p;
    op.idx = D0.col.p;
    need_partials(dv, (int64_t)kPcgBlocks * 2 * nr);
    const int cls = mr_class(nr, 8);
    for (int g = 0; g < 2; ++g) {
      if ((forced != -1 && forced != 1 + g) || !ensure_mr_blocks(c, cls, s)) continue;
      bool ok = true;
      const float ms = time_launches(s, 5, [&] {
        ok = launch_level_lmr<double>(D0.mr[cls], op, nr, g == 0, dv.pp.p, nullptr, dv.pq.p, nullptr, nullptr, 0.0,
                                      0.0, F_PLAIN | D0.keep64, nullptr, s);
        if (ok) launch_pcg_dot_alpha((int)c.an.n, nr, dv.pp.p, dv.pq.p, dv.partials.p, st0, s);
      });
      if (ok && ms < best) {
        best = ms;
        bestCode = -1 - g;
      }
    }
    if (forced == -1 || forced == 3)
      for (int G = 1; G <= 64; G <<= 1) {
        bool ok = true;
        const float ms = time_launches(s, 5, [&] {
          ok = launch_level_split<double>(op, nr, G, dv.pp.p, nullptr, dv.pq.p, nullptr, nullptr, 0.0, 0.0, F_PLAIN,
                                          nullptr, s);
          if (ok) launch_pcg_dot_alpha((int)c.an.n, nr, dv.pp.p, dv.pq.p, dv.partials.p, st0, s);
        });
        if (ok && ms < best) {
          best = ms;
          bestCode = kCodeSplit + G;
        }
      }
    if (forced == -1 || forced == 4)
      for (int G = 1; G <= 64; G <<= 1) {
        bool ok = true;
        const float ms = time_launches(s, 5, [&] {
          ok = launch_level_split2<double>(op, nr, G, dv.pp.p, nullptr, dv.pq.p, nullptr, nullptr, 0.0, 0.0, F_PLAIN,
                                           nullptr, s);
          if (ok) launch_pcg_dot_alpha((int)c.an.n, nr, dv.pp.p, dv.pq.p, dv.partials.p, st0, s);
        });
        if (ok && ms < best) {
          best = ms;
          bestCode = kCodeSplit2 + G;
        }
      }
    dv.tuned[{-1, nr * 2}] = bestCode;
    if (cache) tune_cache_put(mr_tune_key(dv, -1, nr, 8), bestCode);
  }
  R3MG_HIP_CHECK(hipStreamSynchronize(s));
}

// Chebyshev coefficients of a level: first direction scale 1/theta, then (c1, c2) of steps k = 1..K-1
struct Cheb {
  double inv_theta;
  std::vector<double> c1, c2;
};
static Cheb cheb_coeffs(double lo, double hi, int K) {
  Cheb ch;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  ch.inv_theta = 1.0 / theta;
  for (int k = 1; k < K; ++k) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    ch.c1.push_back(rn * rho);
    ch.c2.push_back(2.0 * rn / delta);
    rho = rn;
  }
  return ch;
}

// Coarsest solve x = A_L^{-1} b: the symmetric inverse's packed tiles (float32 tiles for the float32 V-cycle) for
// up to kDenseSymMaxNR columns, else the full float64 inverse.  With pr, the prolongation to the level above
// follows (fused into the tiled product's last pass, else k_prolong_c).
template <typename T>
static void coarsest_apply(Ctx& c, int nr, const T* b, T* x, const DenseProlong<T>* pr, const int* skip,
                           hipStream_t s) {
  Device& dv = c.dv;
  if (dv.ct > 0 && nr <= kDenseSymMaxNR) {
    if constexpr (sizeof(T) == 4) {
      if (dv.csym32.p) {
        launch_dense_apply_sym<T, float>((int)dv.nc, dv.ct, nr, dv.csym32.p, dv.ctile.p, dv.cpart.p, b, x, pr, skip,
                                         s);
        return;
      }
    }
    if (dv.csym.p) {
      launch_dense_apply_sym<T, double>((int)dv.nc, dv.ct, nr, dv.csym.p, dv.ctile.p, dv.cpart.p, b, x, pr, skip,
                                        s);
      return;
    }
  }
  launch_dense_apply<T>((int)dv.nc, nr, dv.cinv.p, b, x, skip, s);
  if (pr) launch_prolong_c<T>(pr->nbox, pr->shift, c.an.d, c.an.pc, nr, pr->pt, x, nullptr, pr->v, skip, s);
}

// ---------------------------------------------------------------------------------------------
// V-cycle (recursive).  On entry the level's right-hand side is in lv[l].b (or b_override at level 0) and,
// when pre_steps > 0 and l < L, lv[l].dA holds the first Chebyshev direction D^{-1} b / theta.  On return
// x_l holds the committed iterate; the returned pointer (may be null) is a pending direction still to be
// added to x_l by the consumer.
// ---------------------------------------------------------------------------------------------
template <typename T>
T* vcycle_rec(Ctx& c, int l, int nr, const T* b_override, const int* skip, hipStream_t s) {
  Analysis& an = c.an;
  Device& dv = c.dv;
  const int L = an.nlevels() - 1;
  DevLevel& D = dv.lv[l];
  T* b = b_override ? const_cast<T*>(b_override) : wv<T>(c, l, W_B);
  T* x = wv<T>(c, l, W_X);
  if (l == L) {
    coarsest_apply<T>(c, nr, b, x, nullptr, skip, s);
    return nullptr;
  }
  const r3mg_options& o = an.opt;
  const int K = o.cheb_degree;
  LevelOp<T> op = level_op<T>(c, l);
  T* rho = wv<T>(c, l, W_RHO);
  T* buf[2] = {wv<T>(c, l, W_DA), wv<T>(c, l, W_DB)};
  bool x_zero = true, rho_is_b = true;
  const int total_spmv = K * (o.pre_steps + o.post_steps);
  int done_spmv = 0;
  auto F = [&](T* u, T* dout, double c1, double c2, bool dout_on, const BoxRestrict<T>* rs = nullptr) {
    int fl = (rho_is_b ? F_RHO_FROM_B : 0) | (x_zero ? F_X_ASSIGN : F_X_ADD);
    ++done_spmv;
    if (done_spmv < total_spmv) fl |= F_RHO_STORE;  // the level's last residual is never read
    if (dout_on) fl |= F_D_OUT;
    apply_level<T>(c, l, nr, u, b, rho, x, dout, c1, c2, fl, skip, s, rs);
    x_zero = false;
    rho_is_b = false;
  };
  auto other = [&](T* p) { return p == buf[0] ? buf[1] : buf[0]; };

  // pre-smoothing from x = 0
  T* pend = nullptr;
  for (int app = 0; app < o.pre_steps; ++app) {
    T* u;
    if (app == 0) {
      u = buf[0];  // D^{-1} b / theta prepared by the caller
    } else {
      u = other(pend);
      F(pend, u, 0.0, D.cheb_inv_theta, true);
    }
    for (int k = 1; k < K; ++k) {
      T* w = other(u);
      F(u, w, D.cheb_c1[k - 1], D.cheb_c2[k - 1], true);
      u = w;
    }
    pend = u;
  }
  // restriction of the residual, fused with the first direction of the next level
  DevLevel& N = dv.lv[l + 1];
  const bool next_smooth = (l + 1 < L) && o.pre_steps > 0;
  const double next_inv_theta = next_smooth ? 2.0 / (N.lam_hi + N.lam_lo) : 0.0;
  T* dnext = next_smooth ? wv<T>(c, l + 1, W_DA) : nullptr;
  const T* dinv_next = nullptr;
  if constexpr (sizeof(T) == 4) dinv_next = N.dinv32.p; else dinv_next = N.dinv64.p;
  const T* pt = nullptr;
  if (l > 0) {
    if constexpr (sizeof(T) == 4) pt = D.pt32.p; else pt = D.pt64.p;
  }
  // a box-row level whose boxes come in fours per parent restricts inside the launch that forms its residual
  const bool fused = pend && l > 0 && level_kernel(an, D, l, nr, (int)sizeof(T)) == LevelKernel::BoxRow &&
                     N.child_shift == 2 && D.nbox == 4 * N.nbox && an.d == 2;
  BoxRestrict<T> rs;
  if (fused) {
    rs.pt = pt;
    rs.bnext = wv<T>(c, l + 1, W_B);
    rs.dinv_next = dinv_next;
    rs.dnext = dnext;
    rs.inv_theta_next = (T)next_inv_theta;
  }
  if (pend) F(pend, nullptr, 0.0, 0.0, false, fused ? &rs : nullptr);  // commit the last direction: rho = b - A x
  const T* src = rho_is_b ? b : rho;
  if (fused) {
  } else if (l == 0) {
    const T* xi;
    if constexpr (sizeof(T) == 4) xi = D.xi32.p; else xi = D.xi64.p;
    launch_restrict0<T>((int)N.nbox, an.n, an.d, an.pc, nr, D.leaf_off.p, D.owner.p, xi, src, wv<T>(c, l + 1, W_B), dinv_next,
                        dnext, next_inv_theta, skip, s);
  } else {
    launch_restrict_c<T>((int)N.nbox, (int)D.nbox, N.child_shift, an.d, an.pc, nr, pt, src, wv<T>(c, l + 1, W_B),
                         dinv_next, dnext, next_inv_theta, skip, s);
  }

  // coarse correction
  T* v = buf[0];
  if (l + 1 == L && l > 0) {
    // the coarsest solve, with the prolongation to this level fused into its last pass
    DenseProlong<T> pr;
    pr.nbox_coarse = (int)N.nbox;
    pr.nbox = (int)D.nbox;
    pr.shift = N.child_shift;
    pr.d = an.d;
    pr.pc = an.pc;
    pr.pt = pt;
    pr.v = v;
    coarsest_apply<T>(c, nr, wv<T>(c, l + 1, W_B), wv<T>(c, l + 1, W_X), &pr, skip, s);
  } else if (l == 0) {
    T* pend_c = vcycle_rec<T>(c, l + 1, nr, nullptr, skip, s);
    const T* xi;
    if constexpr (sizeof(T) == 4) xi = D.xi32.p; else xi = D.xi64.p;
    launch_prolong0<T>((int)D.n, (int)N.nbox, an.d, an.pc, nr, D.leaf_off.p, D.owner.p, xi, wv<T>(c, l + 1, W_X),
                       pend_c, v, skip, s);
  } else {
    T* pend_c = vcycle_rec<T>(c, l + 1, nr, nullptr, skip, s);
    launch_prolong_c<T>((int)D.nbox, N.child_shift, an.d, an.pc, nr, pt, wv<T>(c, l + 1, W_X), pend_c, v, skip, s);
  }

  // post-smoothing from the corrected iterate
  if (o.post_steps == 0) {
    launch_xupdate<T>(D.n * nr, x, v, x_zero ? 1 : 0, skip, s);
    return nullptr;
  }
  T* u = v;
  for (int app = 0; app < o.post_steps; ++app) {
    T* w = other(u);
    F(u, w, 0.0, D.cheb_inv_theta, true);  // x += u, rho -= A u, first direction
    u = w;
    for (int k = 1; k < K; ++k) {
      T* w2 = other(u);
      F(u, w2, D.cheb_c1[k - 1], D.cheb_c2[k - 1], true);
      u = w2;
    }
  }
  return u;
}

// ---------------------------------------------------------------------------------------------
// Numeric set-up
// ---------------------------------------------------------------------------------------------
static void lanczos_level(Ctx& c, int l, hipStream_t s) {
  Analysis& an = c.an;
  Device& dv = c.dv;
  DevLevel& D = dv.lv[l];
  const int64_t n = D.n;
  DBuf<double> v, vp, u, Av, diag;
  v.alloc(n);
  vp.alloc(n);
  u.alloc(n);
  Av.alloc(n);
  diag.alloc(n);
  // diag = 1 / dinv is recomputed exactly as the diagonal values by the diag kernel
  LevelOp<double> op = level_op<double>(c, l);
  R3MG_HIP_CHECK(hipMemsetAsync(dv.flag.p, 0, sizeof(int), s));
  launch_diag_inv((int)n, op.blk, op.ptr, op.idx, op.val, D.dinv64.p, diag.p, dv.flag.p, s);
  launch_lanczos_start((int)n, l == 0 ? dv.perm.p : nullptr, v.p, s);
  R3MG_HIP_CHECK(hipMemsetAsync(vp.p, 0, n * sizeof(double), s));
  DBuf<double>& part = dv.partials;
  int np = launch_dot(n, diag.p, v.p, v.p, part.p, s);
  double nrm = std::sqrt(host_sum(part.p, np, s));
  launch_axpby(n, 1.0 / nrm, v.p, 0.0, v.p, s);
  std::vector<double> alpha, beta;
  double bprev = 0.0;
  const int steps = an.opt.lanczos_steps;
  for (int it = 0; it < steps; ++it) {
    apply_level<double>(c, l, 1, v.p, nullptr, Av.p, nullptr, nullptr, 0, 0, F_PLAIN, nullptr, s);
    launch_lanczos_u(n, D.dinv64.p, Av.p, bprev, vp.p, u.p, s);
    np = launch_dot(n, diag.p, u.p, v.p, part.p, s);
    const double a = host_sum(part.p, np, s);
    launch_axpby(n, -a, v.p, 1.0, u.p, s);
    np = launch_dot(n, diag.p, u.p, u.p, part.p, s);
    const double bb = std::sqrt(host_sum(part.p, np, s));
    alpha.push_back(a);
    if (!(bb > 0.0) || it + 1 == steps) break;
    beta.push_back(bb);
    std::swap(v.p, vp.p);             // vp <- v
    launch_axpby(n, 1.0 / bb, u.p, 0.0, v.p, s);  // v <- u / b
    bprev = bb;
  }
  D.lam_hat = sturm_max(alpha, beta);
  D.lam_hi = an.opt.cheb_boost * D.lam_hat;
  D.lam_lo = D.lam_hi / an.opt.cheb_ratio;
  const Cheb ch = cheb_coeffs(D.lam_lo, D.lam_hi, an.opt.cheb_degree);
  D.cheb_inv_theta = ch.inv_theta;
  D.cheb_c1 = ch.c1;
  D.cheb_c2 = ch.c2;
}

void numeric_setup(HandleImpl& h, hipStream_t s) {
  Analysis& an = *h.an;
  Device& dv = *h.dev;
  Ctx c{an, dv, an.opt.vcycle_fp32 != 0};
  const int L = an.nlevels() - 1;
  const int B = an.B;
  // Galerkin products level by level (float64)
  for (int l = 1; l <= L; ++l) {
    DevLevel& D = dv.lv[l];
    const HostLevel& H = an.lv[l];
    const int64_t nblk = H.bptr[H.nbox];
    if (l == 1) {
      DevLevel& F0 = dv.lv[0];
      launch_galerkin0((int64_t)an.gal_up.size(), an.d, an.pc, D.gal_up.p, D.gal_mir.p, D.brow.p, D.bptr.p,
                       D.gal_ptr.p, D.gal_ent.p, F0.owner.p, F0.xi64.p, F0.col.p, F0.val64.p, D.val64.p, s);
    } else {
      DevLevel& P = dv.lv[l - 1];
      launch_galerkin_c(nblk, an.d, an.pc, H.child_shift, (int)P.nbox, D.brow.p, D.bptr.p, D.bcol.p, P.bptr.p,
                        P.bcol.p, P.val64.p, P.pt64.p, D.val64.p, s);
    }
  }
  // smoother set-up on levels 0..L-1
  for (int l = 0; l < L; ++l) {
    lanczos_level(c, l, s);
    int bad = 0;
    R3MG_HIP_CHECK(hipMemcpyAsync(&bad, dv.flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    R3MG_HIP_CHECK(hipStreamSynchronize(s));
    if (bad) throw Error{R3MG_ERR_NOT_SPD, "non-positive diagonal on level " + std::to_string(l)};
    DevLevel& D = dv.lv[l];
    if (c.fp32) {
      D.val32.alloc(D.val64.n);
      launch_cast_d2f((int64_t)D.val64.n, D.val64.p, D.val32.p, s);
      D.dinv32.alloc(D.n);
      launch_cast_d2f(D.n, D.dinv64.p, D.dinv32.p, s);
    }
  }
  // dense coarsest
  {
    DevLevel& D = dv.lv[L];
    dv.nc = D.n;
    DBuf<double> dense;
    dense.alloc((size_t)D.n * D.n);
    R3MG_HIP_CHECK(hipMemsetAsync(dense.p, 0, (size_t)D.n * D.n * sizeof(double), s));
    launch_to_dense((int)D.nbox, B, D.bptr.p, D.bcol.p, D.val64.p, dense.p, s);
    dv.cinv.alloc((size_t)D.n * D.n);
    R3MG_HIP_CHECK(hipMemsetAsync(dv.flag.p, 0, sizeof(int), s));
    DBuf<double> tiles, ybuf;
    tiles.alloc((size_t)((D.n + 63) / 64) * 64 * 64);
    ybuf.alloc((size_t)D.n * D.n);
    dense_cholesky_inverse((int)D.n, dense.p, dv.cinv.p, tiles.p, ybuf.p, dv.flag.p, s);
    int bad = 0;
    R3MG_HIP_CHECK(hipMemcpyAsync(&bad, dv.flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    R3MG_HIP_CHECK(hipStreamSynchronize(s));
    if (bad) throw Error{R3MG_ERR_NOT_SPD, "coarsest operator is not positive definite"};
    // the symmetric inverse's upper tiles, read once per product by up to kDenseSymMaxNR columns (the pass-1
    // slots cost nr/16 of the bytes saved, so wider blocks keep the full inverse)
    const int nt = (int)((D.n + kDenseTile - 1) / kDenseTile);
    dv.ct = 0;
    dv.csym.release();
    dv.csym32.release();
    dv.cpart.release();
    dv.ctile.release();
    if (nt <= kDenseSymMaxTiles) {
      std::vector<int32_t> tl;
      tl.reserve((size_t)nt * (nt + 1));
      for (int I = 0; I < nt; ++I)
        for (int J = I; J < nt; ++J) {
          tl.push_back(I);
          tl.push_back(J);
        }
      const int ntiles = nt * (nt + 1) / 2;
      dv.ctile.upload(tl, s);
      // the float32 V-cycle reads the tiles rounded to float32 (half the bytes; products still in float64)
      if (c.fp32) {
        dv.csym32.alloc((size_t)ntiles * kDenseTile * kDenseTile);
        launch_dense_pack_sym<float>((int)D.n, ntiles, dv.cinv.p, dv.ctile.p, dv.csym32.p, s);
      } else {
        dv.csym.alloc((size_t)ntiles * kDenseTile * kDenseTile);
        launch_dense_pack_sym<double>((int)D.n, ntiles, dv.cinv.p, dv.ctile.p, dv.csym.p, s);
      }
      dv.cpart.alloc((size_t)nt * nt * kDenseTile * kDenseSymMaxNR);
      R3MG_HIP_CHECK(hipStreamSynchronize(s));
      dv.ct = nt;
    }
  }
  drop_graphs(dv);
}

// Tuning-cache key prefix of a handle: the device, and a hash of what decides the kernel choices (dimension,
// coarse degree, the fine row pointers and a strided sample of its columns, every level's size and stored
// nonzeros, the V-cycle precision and the matrix-cache mode).  Numeric values do not enter.
static std::string tune_signature(const Analysis& an, const Device& dv) {
  uint64_t hsh = fnv1a(an.rowptr.data(), an.rowptr.size() * sizeof(int32_t));
  const size_t nc = an.col.size(), step = std::max<size_t>(1, nc / 65536);
  for (size_t i = 0; i < nc; i += step) hsh = fnv1a(&an.col[i], sizeof(int32_t), hsh);
  const int64_t meta[] = {an.d, an.pc, an.B, an.n, an.nnz, an.opt.vcycle_fp32, an.opt.matrix_cache,
                          (int64_t)dv.lv.size()};
  hsh = fnv1a(meta, sizeof meta, hsh);
  for (const DevLevel& D : dv.lv) {
    const int64_t v[2] = {D.n, D.nnz};
    hsh = fnv1a(v, sizeof v, hsh);
  }
  char buf[24];
  std::snprintf(buf, sizeof buf, "%016llx", (unsigned long long)hsh);
  return tune_device_key(dv.dev) + "/" + buf;
}

// Fine-level row-block shape: each candidate shape runs the V-cycle-precision smoother step on level 0 (3
// warm-up + 5 timed launches, hipEvents); the fastest is kept for every later single-RHS application.
static void tune_stream_shape(HandleImpl& h, hipStream_t s) {
  Analysis& an = *h.an;
  Device& dv = *h.dev;
  Ctx c{an, dv, an.opt.vcycle_fp32 != 0};
  ensure_level_vectors(c, 1);
  DevLevel& D = dv.lv[0];
  if (an.opt.fine_kernel >= 0) {
    D.shape = D.shape64 = an.opt.fine_kernel;
    D.bytes_apply = D.shape_bytes[D.shape];
    return;
  }
  // the tuning cache holds shape + 100 shape64
  const bool cache = an.opt.tune_cache != 0 && !dv.tune_sig.empty();
  const std::string key = dv.tune_sig + "/fine1/" + (c.fp32 ? "f32" : "f64");
  int cached = 0;
  if (cache && tune_cache_get(key, &cached) && cached >= 0 && cached % 100 < kFineShapes &&
      cached / 100 < kFineShapes && (c.fp32 || cached / 100 == cached % 100)) {
    D.shape = cached % 100;
    D.shape64 = cached / 100;
    D.bytes_apply = D.shape_bytes[D.shape];
    return;
  }
  const int fl = F_RHO_STORE | F_X_ADD | F_D_OUT;
  // two interleaved rounds, best of each shape; another shape replaces the first one only when it is at least
  // 3% faster, so that timing noise does not flip the choice between runs
  float best[kStreamShapes];
  for (int sh = 0; sh < kStreamShapes; ++sh) best[sh] = 1e30f;
  for (int round = 0; round < 2; ++round) {
    for (int sh = 0; sh < kFineShapes; ++sh) {
      float ms;
      if (c.fp32) {
        LevelOp<float> op = level_op<float>(c, 0);
        ms = time_launches(s, 20, [&] {
          launch_level_stream<float>(sh, D.fb[sh], op, vbuf<float>(D.dA), vbuf<float>(D.b),
                                     vbuf<float>(D.rho), vbuf<float>(D.x), vbuf<float>(D.dB), 0.0, 0.0,
                                     fl | D.keep32, nullptr, nullptr, s);
        });
      } else {
        LevelOp<double> op = level_op<double>(c, 0);
        ms = time_launches(s, 20, [&] {
          launch_level_stream<double>(sh, D.fb[sh], op, vbuf<double>(D.dA), vbuf<double>(D.b),
                                      vbuf<double>(D.rho), vbuf<double>(D.x), vbuf<double>(D.dB), 0.0, 0.0,
                                      fl | D.keep64, nullptr, nullptr, s);
        });
      }
      best[sh] = std::min(best[sh], ms);
    }
  }
  int bestS = 0;
  for (int sh = 1; sh < kFineShapes; ++sh)
    if (best[sh] < 0.97f * best[bestS]) bestS = sh;
  D.shape = D.shape64 = bestS;
  D.bytes_apply = D.shape_bytes[D.shape];
  R3MG_HIP_CHECK(hipMemsetAsync(D.x.p, 0, D.x.n, s));
  R3MG_HIP_CHECK(hipMemsetAsync(D.rho.p, 0, D.rho.n, s));
  if (!c.fp32) {
    if (cache) tune_cache_put(key, D.shape + 100 * D.shape64);
    return;
  }
  // float32 V-cycle: PCG's float64 operator y = A p is timed on its own (the float64 values double the LDS
  // staging, so another shape can win); the same two rounds and 3% rule
  DBuf<double> u64, y64;
  u64.alloc((size_t)an.n);
  y64.alloc((size_t)an.n);
  R3MG_HIP_CHECK(hipMemsetAsync(u64.p, 0, u64.n * sizeof(double), s));
  LevelOp<double> op = level_op<double>(c, 0);
  for (int sh = 0; sh < kStreamShapes; ++sh) best[sh] = 1e30f;
  for (int round = 0; round < 2; ++round)
    for (int sh = 0; sh < kFineShapes; ++sh) {
      const float ms = time_launches(s, 20, [&] {
        launch_level_stream<double>(sh, D.fb[sh], op, u64.p, nullptr, y64.p, nullptr, nullptr, 0.0, 0.0,
                                    F_PLAIN | D.keep64, nullptr, nullptr, s);
      });
      best[sh] = std::min(best[sh], ms);
    }
  bestS = 0;
  for (int sh = 1; sh < kFineShapes; ++sh)
    if (best[sh] < 0.97f * best[bestS]) bestS = sh;
  D.shape64 = bestS;
  if (cache) tune_cache_put(key, D.shape + 100 * D.shape64);
  R3MG_HIP_CHECK(hipStreamSynchronize(s));
}

// uploads local-column row blocks into slot g of a level and points the kernel shape kLocalFirst + g at them
static void upload_local(DevLevel& D, int g, const LocalBlocks& lb, const std::vector<int32_t>& rowptr,
                         hipStream_t s, int slot = -1) {
  D.lrb[g].upload(lb.rb, s);
  D.lubp[g].upload(lb.ubp, s);
  D.lucol[g].upload(lb.ucol, s);
  D.lidx[g].upload(lb.lidx, s);
  std::vector<int32_t> meta(lb.rb.size() * 4, 0);
  for (size_t b = 0; b < lb.rb.size(); ++b) {
    meta[4 * b] = lb.rb[b];
    meta[4 * b + 1] = rowptr[lb.rb[b]];
    meta[4 * b + 2] = lb.ubp[b];
  }
  D.lmeta[g].upload(meta, s);
  FineBlocks& f = D.fb[slot >= 0 ? slot : kLocalFirst + g];
  f.nrb = (int)lb.rb.size() - 1;
  f.rb = D.lrb[g].p;
  f.ubp = D.lubp[g].p;
  f.ucol = D.lucol[g].p;
  f.lidx = D.lidx[g].p;
  f.meta = D.lmeta[g].p;
}

// algorithmic bytes of one application with local-column blocks: values and local column positions,
// distinct-column lists and offsets, row pointers, block offsets, 7 vector streams
static double local_bytes(int64_t nnz, int64_t n, int g, const LocalBlocks& lb, double sv) {
  const double nrb = (double)lb.rb.size() - 1;
  return (double)nnz * (sv + kLocalIdxBytes[g]) + 4.0 * lb.ucol.size() + 4.0 * (nrb + 1) + (double)(n + 1) * 4 +
         4.0 * (nrb + 1) + 7.0 * n * sv;
}

// F_KEEP (ordinary matrix loads) for a level whose matrix stream takes `bytes`, per r3mg_options::matrix_cache
static int keep_rule(const r3mg_options& o, double bytes) {
  if (o.matrix_cache == 0) return 0;
  if (o.matrix_cache == 1) return F_KEEP;
  return bytes <= kKeepCachedBytes ? F_KEEP : 0;
}

void device_setup(HandleImpl& h, hipStream_t s) {
  Analysis& an = *h.an;
  h.dev = std::make_unique<Device>();
  Device& dv = *h.dev;
  R3MG_HIP_CHECK(hipGetDevice(&dv.dev));
  const int L = an.nlevels() - 1;
  const int B = an.B;
  const bool fp32 = an.opt.vcycle_fp32 != 0;
  dv.lv.resize(L + 1);
  dv.flag.alloc(1);
  dv.partials.alloc(4096);  // set-up reductions (at most 1024 partials); grown by the solvers
  dv.perm.upload(an.order, s);
  dv.src.upload(an.src, s);
  // fine level
  {
    DevLevel& D = dv.lv[0];
    D.n = an.n;
    D.nnz = an.nnz;
    D.rowptr.upload(an.rowptr, s);
    {
      // kFinePad zero entries after the last nonzero: the 16-byte loads of the row-block kernel may read them
      std::vector<int32_t> colp(an.col);
      colp.resize(colp.size() + kFinePad, 0);
      D.col.upload(colp, s);
      std::vector<double> valp(an.val);
      valp.resize(valp.size() + kFinePad, 0.0);
      D.val64.upload(valp, s);
    }
    D.xi64.upload(an.xi, s);
    D.owner.upload(an.owner, s);
    std::vector<int32_t> lo(an.leaf_off.begin(), an.leaf_off.end());
    D.leaf_off.upload(lo, s);
    D.lanes = lanes_for((double)an.nnz / (double)an.n);
    const double sv0 = fp32 ? 4 : 8;
    for (int g = 0; g < kCsrGeoms; ++g) {
      D.rb[g].upload(an.rb[g], s);
      const int nrb = (int)an.rb[g].size() - 1;
      // values and columns, row pointers, row-block offsets, 7 vector streams
      const double by = (double)an.nnz * (sv0 + 4) + (double)(an.n + 1) * 4 + 4.0 * (nrb + 1) + 7.0 * an.n * sv0;
      for (int sh : {g, g + kCsrGeoms}) {
        D.fb[sh].nrb = nrb;
        D.fb[sh].rb = D.rb[g].p;
        D.shape_bytes[sh] = by;
      }
    }
    for (int g = 0; g < kLocalGeoms; ++g) {
      upload_local(D, g, an.loc[g], an.rowptr, s);
      D.shape_bytes[kLocalFirst + g] = local_bytes(an.nnz, an.n, g, an.loc[g], sv0);
    }
    // matrix read with ordinary loads when its stream (values and 1-byte positions) fits the caches
    D.keep32 = keep_rule(an.opt, (double)an.nnz * (4 + 1));
    D.keep64 = keep_rule(an.opt, (double)an.nnz * (8 + 1));
    // shape 9: the vector-load kernel over the blocks of local geometry 0; shape 10: the same over geometry 3
    D.fb[kLocalFirst + kLocalGeoms] = D.fb[kLocalFirst];
    D.shape_bytes[kLocalFirst + kLocalGeoms] = D.shape_bytes[kLocalFirst];
    upload_local(D, 3, an.loc[3], an.rowptr, s, kLocalFirst + kLocalGeoms + 1);
    D.shape_bytes[kLocalFirst + kLocalGeoms + 1] = local_bytes(an.nnz, an.n, 3, an.loc[3], sv0);
    // shapes 11 and 12: the blocks of shapes 9 and 10, two per workgroup
    for (int sh : {kVecTwoFirst, kVecTwoFirst + 1}) {
      D.fb[sh] = D.fb[sh - 2];
      D.shape_bytes[sh] = D.shape_bytes[sh - 2];
    }
    D.dinv64.alloc(D.n);
    if (fp32) {
      D.xi32.alloc(D.xi64.n);
      launch_cast_d2f((int64_t)D.xi64.n, D.xi64.p, D.xi32.p, s);
    }
    D.bytes_apply = D.shape_bytes[0];  // replaced by the chosen shape's bytes once the shape is timed
  }
  for (int l = 1; l <= L; ++l) {
    DevLevel& D = dv.lv[l];
    const HostLevel& H = an.lv[l];
    D.n = H.n;
    D.nbox = H.nbox;
    const int64_t nblk = H.bptr[H.nbox];
    D.nnz = nblk * B * B;
    std::vector<int32_t> bp(H.bptr.begin(), H.bptr.end());
    D.bptr.upload(bp, s);
    D.bcol.upload(H.bcol, s);
    std::vector<int32_t> br(nblk);
    for (int64_t k = 0; k < H.nbox; ++k)
      for (int64_t j = H.bptr[k]; j < H.bptr[k + 1]; ++j) br[j] = (int32_t)k;
    D.brow.upload(br, s);
    if (l == 1) {
      D.gal_ptr.upload(an.gal_ptr, s);
      D.gal_ent.upload(an.gal_ent, s);
      D.gal_up.upload(an.gal_up, s);
      D.gal_mir.upload(an.gal_mir, s);
    }
    D.val64.alloc((size_t)D.nnz + kFinePad);  // zero padding: the local-column kernel's vector loads
    R3MG_HIP_CHECK(hipMemsetAsync(D.val64.p, 0, D.val64.n * sizeof(double), s));
    D.dinv64.alloc(D.n);
    D.child_shift = H.child_shift;
    for (int64_t k = 0; k < H.nbox; ++k) D.maxnb = std::max<int>(D.maxnb, (int)(H.bptr[k + 1] - H.bptr[k]));
    if (!H.pt1d.empty()) {
      D.pt64.upload(H.pt1d, s);
      if (fp32) {
        D.pt32.alloc(D.pt64.n);
        launch_cast_d2f((int64_t)D.pt64.n, D.pt64.p, D.pt32.p, s);
      }
    }
    D.lanes = lanes_for((double)(D.nnz) / (double)std::max<int64_t>(1, D.n));
    const double sv = fp32 ? 4 : 8;
    D.bytes_apply = (double)D.nnz * sv + (double)nblk * 4 + (double)(H.nbox + 1) * 4 + 7.0 * D.n * sv;
    // boxes of 4, 9 or 16 rows (2D) take the box-row kernel, which reads only the values, block columns and
    // block-row offsets; the local-column blocks remain for wider block rows
    D.boxrow = boxrow_supported(B, D.maxnb);
    // the box-row and block-row kernels stream the values only
    const int ib = (D.boxrow || H.rowptr.empty()) ? 0 : 1;
    D.keep32 = keep_rule(an.opt, (double)D.nnz * (4 + ib));
    D.keep64 = keep_rule(an.opt, (double)D.nnz * (8 + ib));
    if (!D.boxrow && !H.rowptr.empty()) {  // narrow block rows: the level is held as 1-byte local-column blocks
      D.rowptr.upload(H.rowptr, s);
      // the vector kernel: shape 9 over 2048-nonzero blocks, shape 13 over (3072, 64-row) blocks
      D.shape = H.loc_geom == 4 ? kAggVecShape : kLocalFirst + kLocalGeoms;
      upload_local(D, H.loc_geom, H.loc, H.rowptr, s, D.shape);
      D.shape_bytes[D.shape] = local_bytes(D.nnz, D.n, H.loc_geom, H.loc, sv);
      D.bytes_apply = D.shape_bytes[D.shape];
    }
  }
  numeric_setup(h, s);
  dv.tune_sig = tune_signature(an, dv);
  tune_stream_shape(h, s);
  R3MG_HIP_CHECK(hipStreamSynchronize(s));
  // the allocation-free V-cycle's scratch address on this device, looked up once at set-up
  (void)scratch_device_ptr(dv.dev);
}

void update_values(HandleImpl& h, const double* vals_dev, hipStream_t s) {
  detach_matrix_free(h);  // the cell description no longer matches the new values
  Device& dv = *h.dev;
  launch_gather_vals(h.an->nnz, dv.src.p, vals_dev, dv.lv[0].val64.p, s);
  numeric_setup(h, s);
  R3MG_HIP_CHECK(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------------------------
// Public operations
// ---------------------------------------------------------------------------------------------
template <typename T>
static void vcycle_api_t(HandleImpl& h, const double* r, double* z, int nrhs, hipStream_t s) {
  Analysis& an = *h.an;
  Device& dv = *h.dev;
  Ctx c{an, dv, sizeof(T) == 4};
  const int L = an.nlevels() - 1;
  for (int c0 = 0; c0 < nrhs; c0 += kMaxNR) {
    const int nb = std::min(kMaxNR, nrhs - c0);
    int NR = 1;
    while (NR < nb) NR <<= 1;
    ensure_level_vectors(c, NR);
    if (NR > 1) {
      ensure_pcg_vectors(c, NR);
      autotune_spmm<T>(c, NR, s);
    }
    DevLevel& D0 = dv.lv[0];
    T* b0 = vbuf<T>(D0.b);
    const bool smooth0 = (L > 0) && an.opt.pre_steps > 0;
    const T* dinv0;
    if constexpr (sizeof(T) == 4) dinv0 = D0.dinv32.p; else dinv0 = D0.dinv64.p;
    if (NR == nb) {
      launch_vc_entry<T>((int)an.n, NR, dv.perm.p, r + (int64_t)c0 * an.n, an.n, b0, dinv0,
                         smooth0 ? vbuf<T>(D0.dA) : nullptr, 2.0 / (D0.lam_hi + D0.lam_lo), s);
    } else {
      // gather into float64 scratch with zero padding, then convert
      ensure_pcg_vectors(c, NR);
      launch_gather_cols((int)an.n, NR, nb, dv.perm.p, r + (int64_t)c0 * an.n, an.n, dv.pb.p, s);
      launch_vc_prep<T>((int)an.n, NR, dv.pb.p, b0, dinv0, smooth0 ? vbuf<T>(D0.dA) : nullptr,
                        2.0 / (D0.lam_hi + D0.lam_lo), nullptr, s);
    }
    T* pend = (L == 0) ? nullptr : vcycle_rec<T>(c, 0, NR, nullptr, nullptr, s);
    if (NR == nb) {
      launch_vc_exit<T>((int)an.n, NR, dv.perm.p, vbuf<T>(D0.x), pend, z + (int64_t)c0 * an.n, an.n, s);
    } else {
      // x0 + pend -> pz (float64 interleaved) -> scatter the real columns
      ensure_pcg_vectors(c, NR);
      launch_pcg_z<T>((int)an.n, NR, nullptr, 0, vbuf<T>(D0.x), pend, dv.pz.p, nullptr, nullptr, nullptr, dv.partials.p,
                      s);
      launch_scatter_cols((int)an.n, NR, nb, dv.perm.p, dv.pz.p, z + (int64_t)c0 * an.n, an.n, s);
    }
  }
}

void vcycle_api(HandleImpl& h, const double* r, double* z, int nrhs, hipStream_t s) {
  if (h.an->opt.vcycle_fp32)
    vcycle_api_t<float>(h, r, z, nrhs, s);
  else
    vcycle_api_t<double>(h, r, z, nrhs, s);
}

// The V-cycle of vcycle_api_t for one block of nrhs in {1, 2, 4, 8, 16} columns, with the level work vectors
// carved from the static device scratch: kWorkSlots per level, n_l x nrhs values each, every one starting on a
// 256-byte boundary, zeroed by a fill kernel first (every call starts as the first call of vcycle_api_t does, on
// freshly cleared buffers).  Nothing is allocated, on the device or the host, and nothing synchronises.
constexpr int kNoallocMaxLevels = 32;
template <typename T>
static void vcycle_noalloc_t(HandleImpl& h, const double* r, double* z, int nrhs, hipStream_t s) {
  Analysis& an = *h.an;
  Device& dv = *h.dev;
  const int L = an.nlevels() - 1;
  const int NR = nrhs;
  if (NR != 1 && NR != 2 && NR != 4 && NR != 8 && NR != 16)
    throw Error{R3MG_ERR_INVALID, "r3mg_vcycle_noalloc: nrhs must be 1, 2, 4, 8 or 16"};
  if (L + 1 > kNoallocMaxLevels) throw Error{R3MG_ERR_INVALID, "r3mg_vcycle_noalloc: too many levels"};
  int cur = -1;
  R3MG_HIP_CHECK(hipGetDevice(&cur));
  if (cur != dv.dev) throw Error{R3MG_ERR_INVALID, "r3mg_vcycle_noalloc: the handle's device is not current"};
  DevLevel& D0 = dv.lv[0];
  if (D0.mf && NR > 1 && dv.mf.mr_cap < NR)
    throw Error{R3MG_ERR_INVALID,
                "r3mg_vcycle_noalloc: the matrix-free operator's cell outputs are not sized for this many columns"};
  size_t offs[kNoallocMaxLevels * kWorkSlots];
  size_t off = 0;
  for (int l = 0; l <= L; ++l)
    for (int w = 0; w < kWorkSlots; ++w) {
      offs[(size_t)l * kWorkSlots + w] = off;
      off += ((size_t)dv.lv[l].n * NR * sizeof(T) + 255) / 256 * 256;
    }
  if (off > kNoallocScratchBytes)
    throw Error{R3MG_ERR_INVALID, "r3mg_vcycle_noalloc: the work vectors need " + std::to_string(off) +
                                      " bytes, more than the scratch's " + std::to_string(kNoallocScratchBytes)};
  char* base = static_cast<char*>(scratch_device_ptr(dv.dev));
  char* work[kNoallocMaxLevels * kWorkSlots];
  for (int i = 0; i < (L + 1) * kWorkSlots; ++i) work[i] = base + offs[i];
  scratch_zero(base, off, s);
  Ctx c{an, dv, sizeof(T) == 4, work};
  T* b0 = wv<T>(c, 0, W_B);
  const bool smooth0 = (L > 0) && an.opt.pre_steps > 0;
  const T* dinv0;
  if constexpr (sizeof(T) == 4) dinv0 = D0.dinv32.p; else dinv0 = D0.dinv64.p;
  launch_vc_entry<T>((int)an.n, NR, dv.perm.p, r, an.n, b0, dinv0, smooth0 ? wv<T>(c, 0, W_DA) : nullptr,
                     2.0 / (D0.lam_hi + D0.lam_lo), s);
  T* pend = (L == 0) ? nullptr : vcycle_rec<T>(c, 0, NR, nullptr, nullptr, s);
  launch_vc_exit<T>((int)an.n, NR, dv.perm.p, wv<T>(c, 0, W_X), pend, z, an.n, s);
}

void vcycle_noalloc(HandleImpl& h, const double* r, double* z, int nrhs, hipStream_t s) {
  if (h.an->opt.vcycle_fp32)
    vcycle_noalloc_t<float>(h, r, z, nrhs, s);
  else
    vcycle_noalloc_t<double>(h, r, z, nrhs, s);
}

void level_apply(HandleImpl& h, int level, const double* x, double* y, hipStream_t s) {
  Analysis& an = *h.an;
  Device& dv = *h.dev;
  Ctx c{an, dv, false};
  const int l = level < 0 ? 0 : level;
  LevelOp<double> op = level_op<double>(c, l);
  if (l == 0) {
    ensure_pcg_vectors(c, 1);
    launch_gather_cols((int)an.n, 1, 1, dv.perm.p, x, an.n, dv.pb.p, s);
    apply_level<double>(c, 0, 1, dv.pb.p, nullptr, dv.pq.p, nullptr, nullptr, 0, 0, F_PLAIN, nullptr, s);
    launch_scatter_cols((int)an.n, 1, 1, dv.perm.p, dv.pq.p, y, an.n, s);
  } else {
    launch_level<double>(op, 1, x, nullptr, y, nullptr, nullptr, 0, 0, F_PLAIN, nullptr, s);
  }
}

// q = A p in float64 for NR columns with the kernel PCG's operator uses (the matrix-free operator, the fine level's
// single-RHS shape for float64, else the tuned multi-RHS kernel), without a dot product
static void pcg_operator(Ctx& c, int NR, const double* p, double* q, const int* skip, hipStream_t s) {
  Device& dv = c.dv;
  DevLevel& D0 = dv.lv[0];
  LevelOp<double> op64 = level_op<double>(c, 0);
  if (D0.mf) {
    apply_level<double>(c, 0, NR, p, nullptr, q, nullptr, nullptr, 0.0, 0.0, F_PLAIN, skip, s);
    return;
  }
  if (NR == 1 && D0.fb[D0.shape].nrb > 0) {
    launch_level_stream<double>(D0.shape64, D0.fb[D0.shape64], op64, p, nullptr, q, nullptr, nullptr, 0, 0,
                                F_PLAIN | D0.keep64, skip, nullptr, s);
    return;
  }
  auto it = dv.tuned.find({-1, NR * 2});
  if (it != dv.tuned.end() && (it->second < 0 || it->second >= kCodeSplit)) {
    op64.ptr = D0.rowptr.p;
    op64.idx = D0.col.p;
    const int cls = mr_class(NR, 8);
    const bool ok = it->second < 0
                        ? cls >= 0 && launch_level_lmr<double>(D0.mr[cls], op64, NR, it->second == -1, p, nullptr, q,
                                                               nullptr, nullptr, 0.0, 0.0, F_PLAIN | D0.keep64, skip, s)
                        : launch_split_code<double>(it->second, op64, NR, p, nullptr, q, nullptr, nullptr, 0.0, 0.0,
                                                    F_PLAIN, skip, s);
    if (!ok) throw std::runtime_error("multi-RHS fine-level kernel: unsupported shape");
    return;
  }
  if (it != dv.tuned.end()) op64.lanes = it->second;
  launch_level<double>(op64, NR, p, nullptr, q, nullptr, nullptr, 0.0, 0.0, F_PLAIN, skip, s);
}

// One PCG iteration (all launches skip once every column has converged).  part 0: the whole iteration; part 1:
// q = A p, alpha, the x and r updates and the stop test; part 2: the V-cycle, z, beta and the new p.
template <typename T>
static void pcg_iteration(Ctx& c, int NR, bool flexible, hipStream_t s, int part = 0, bool vcycle_skips = false) {
  Analysis& an = c.an;
  Device& dv = c.dv;
  const int L = an.nlevels() - 1;
  PcgState* st = reinterpret_cast<PcgState*>(dv.state.p);
  const int* skip = reinterpret_cast<const int*>(dv.state.p);
  DevLevel& D0 = dv.lv[0];
  LevelOp<double> op64 = level_op<double>(c, 0);
  const int n = (int)an.n;
  need_partials(dv, (int64_t)kPcgBlocks * std::max(2 * NR, 4));
  if (NR == 1) {
    // one column: q = A p, <p, q>, then alpha, the stop test and beta folded into the vector kernels that follow
    // their reductions (4 launches besides the operator and the V-cycle)
    double* P = dv.partials.p;
    const T* dinv0;
    if constexpr (sizeof(T) == 4) dinv0 = D0.dinv32.p; else dinv0 = D0.dinv64.p;
    if (part != 2) {
      pcg_operator(c, 1, dv.pp.p, dv.pq.p, skip, s);
      launch_pcg_dot(n, dv.pp.p, dv.pq.p, P, st, s);
      const bool smooth0 = (L > 0) && an.opt.pre_steps > 0;
      T* b0 = (sizeof(T) == 4) ? vbuf<T>(D0.b) : nullptr;
      launch_pcg_xr1<T>(n, st, dv.px.p, dv.pr.p, dv.pp.p, dv.pq.p, P, b0, dinv0, smooth0 ? vbuf<T>(D0.dA) : nullptr,
                        2.0 / (D0.lam_hi + D0.lam_lo), s);
      if (part == 1) {
        launch_pcg_check1(n, st, P, s);
        return;
      }
    }
    const T* bl0 = (sizeof(T) == 4) ? vbuf<T>(D0.b) : reinterpret_cast<const T*>(dv.pr.p);
    T* pend = nullptr;
    // with vcycle_skips (group solves, where problems converge at different iterations) the V-cycle's kernels
    // return at once after convergence; otherwise they do not read the flag (one memory latency less each)
    if (L > 0) pend = vcycle_rec<T>(c, 0, 1, bl0, vcycle_skips ? skip : nullptr, s);
    const T* x0 = (L > 0) ? vbuf<T>(D0.x) : bl0;
    launch_pcg_z1<T>(n, st, part == 0, x0, pend, dv.pz.p, dv.pr.p, flexible ? dv.pq.p : nullptr, P, s);
    launch_pcg_p1(n, st, dv.pz.p, dv.pp.p, P, s);
    return;
  }
  if (part != 2) {
    // q = A p, then alpha from <p, q> in the fixed partition of the dot kernel (the iterates do not depend on
    // the kernel that formed q), except after the lanes kernel, whose fused dot has its own partition
    if (D0.mf) {
      apply_level<double>(c, 0, NR, dv.pp.p, nullptr, dv.pq.p, nullptr, nullptr, 0.0, 0.0, F_PLAIN, skip, s);
      launch_pcg_dot_alpha(n, NR, dv.pp.p, dv.pq.p, dv.partials.p, st, s);
    } else if (NR == 1 && D0.fb[D0.shape].nrb > 0) {
      launch_level_stream<double>(D0.shape64, D0.fb[D0.shape64], op64, dv.pp.p, nullptr, dv.pq.p, nullptr, nullptr, 0, 0,
                                  F_PLAIN | D0.keep64, skip, nullptr, s);
      launch_pcg_dot_alpha(n, 1, dv.pp.p, dv.pq.p, dv.partials.p, st, s);
    } else {
      auto it = dv.tuned.find({-1, NR * 2});
      if (it != dv.tuned.end() && (it->second < 0 || it->second >= kCodeSplit)) {
        op64.ptr = D0.rowptr.p;
        op64.idx = D0.col.p;
        bool ok;
        if (it->second < 0) {
          const int cls = mr_class(NR, 8);
          ok = cls >= 0 && launch_level_lmr<double>(D0.mr[cls], op64, NR, it->second == -1, dv.pp.p, nullptr, dv.pq.p,
                                                    nullptr, nullptr, 0.0, 0.0, F_PLAIN | D0.keep64, skip, s);
        }
        else
          ok = launch_split_code<double>(it->second, op64, NR, dv.pp.p, nullptr, dv.pq.p, nullptr, nullptr, 0.0, 0.0,
                                         F_PLAIN, skip, s);
        if (!ok) throw std::runtime_error("multi-RHS fine-level kernel: unsupported shape");
        launch_pcg_dot_alpha(n, NR, dv.pp.p, dv.pq.p, dv.partials.p, st, s);
      } else {
        if (it != dv.tuned.end()) op64.lanes = it->second;
        need_partials(dv, (int64_t)((n + 256 / op64.lanes - 1) / (256 / op64.lanes)) * NR);
        const int np = launch_spmv_dot(op64, NR, dv.pp.p, dv.pq.p, dv.partials.p, skip, s);
        launch_pcg_alpha(NR, st, dv.partials.p, np, s);
      }
    }
    const bool smooth0 = (L > 0) && an.opt.pre_steps > 0;
    const T* dinv0;
    if constexpr (sizeof(T) == 4) dinv0 = D0.dinv32.p; else dinv0 = D0.dinv64.p;
    T* b0 = (sizeof(T) == 4) ? vbuf<T>(D0.b) : nullptr;
    launch_pcg_xr<T>(n, NR, st, dv.px.p, dv.pr.p, dv.pp.p, dv.pq.p, dv.partials.p, b0, dinv0,
                     smooth0 ? vbuf<T>(D0.dA) : nullptr, 2.0 / (D0.lam_hi + D0.lam_lo), s);
  }
  if (part == 1) return;
  // The V-cycle does not read the skip flag: it only writes level work vectors and z, so running it after every
  // column has converged changes nothing (converged columns keep alpha = 0, beta and p), and a flag read at the
  // start of each of its ~45 kernels would put one more memory latency on each of them.
  const T* bl0 = (sizeof(T) == 4) ? vbuf<T>(D0.b) : reinterpret_cast<const T*>(dv.pr.p);
  T* pend = nullptr;
  if (L > 0) pend = vcycle_rec<T>(c, 0, NR, bl0, nullptr, s);
  const T* x0 = (L > 0) ? vbuf<T>(D0.x) : bl0;
  launch_pcg_z<T>(n, NR, st, 2, x0, pend, dv.pz.p, dv.pr.p, flexible ? dv.pq.p : nullptr, nullptr, dv.partials.p, s);
  launch_pcg_p(n, NR, st, dv.pz.p, dv.pp.p, s);
}

// room for the CG coefficients and residual norms of maxit iterations (a reallocation invalidates the captured
// graphs)
static void ensure_hist(Device& dv, int maxit) {
  if (dv.hist_rows >= maxit && dv.hist.p) return;
  dv.hist.alloc((size_t)(3 * (size_t)maxit + 1) * kMaxNR);
  dv.hist_rows = maxit;
  drop_graphs(dv);
}
static double* rhist_of(Device& dv) { return dv.hist.p + (size_t)2 * kMaxNR * dv.hist_rows; }

// r = b - A x; z = B r; p = z; gamma = <r, z>.  restart: from the true residual of the current x, keeping the
// stop thresholds and iteration counts (residual replacement).
template <typename T>
static void pcg_start(Ctx& c, int NR, int nb, double rtol, double atol, bool flexible, bool restart, hipStream_t s) {
  Analysis& an = c.an;
  Device& dv = c.dv;
  const int L = an.nlevels() - 1;
  const int n = (int)an.n;
  PcgState* st = reinterpret_cast<PcgState*>(dv.state.p);
  const int* skip = reinterpret_cast<const int*>(dv.state.p);
  DevLevel& D0 = dv.lv[0];
  need_partials(dv, (int64_t)kPcgBlocks * std::max(2 * NR, 4));
  pcg_operator(c, NR, dv.px.p, dv.pq.p, nullptr, s);
  launch_pcg_residual_init(n, NR, dv.pb.p, dv.pq.p, dv.pr.p, dv.partials.p, st, restart ? 1 : 0, rtol, atol, nb,
                           flexible ? 1 : 0, dv.hist.p, rhist_of(dv), dv.hist_rows, s);
  const bool smooth0 = (L > 0) && an.opt.pre_steps > 0;
  const T* dinv0;
  if constexpr (sizeof(T) == 4) dinv0 = D0.dinv32.p; else dinv0 = D0.dinv64.p;
  T* b0 = (sizeof(T) == 4) ? vbuf<T>(D0.b) : nullptr;
  launch_vc_prep<T>(n, NR, dv.pr.p, b0, dinv0, smooth0 ? vbuf<T>(D0.dA) : nullptr, 2.0 / (D0.lam_hi + D0.lam_lo),
                    skip, s);
  const T* bl0 = (sizeof(T) == 4) ? vbuf<T>(D0.b) : reinterpret_cast<const T*>(dv.pr.p);
  T* pend = nullptr;
  if (L > 0) pend = vcycle_rec<T>(c, 0, NR, bl0, nullptr, s);
  const T* x0 = (L > 0) ? vbuf<T>(D0.x) : bl0;
  // one column: <r, z> partials in area 2, where the first iteration's alpha kernel forms gamma from them
  double* zpart = NR == 1 ? dv.partials.p + 2 * pcg_blocks(n) : dv.partials.p;
  launch_pcg_z<T>(n, NR, st, 1, x0, pend, dv.pz.p, dv.pr.p, nullptr, dv.pp.p, zpart, s);
}

template <typename T>
static hipGraphExec_t iteration_graph(Ctx& c, int NR, bool flexible, int part) {
  Device& dv = c.dv;
  const int key = (NR * 2 + (flexible ? 1 : 0)) * 3 + part;
  auto it = dv.graphs.find(key);
  if (it != dv.graphs.end()) return it->second;
  if (!dv.cap_stream) R3MG_HIP_CHECK(hipStreamCreateWithFlags(&dv.cap_stream, hipStreamNonBlocking));
  hipGraph_t g;
  R3MG_HIP_CHECK(hipStreamBeginCapture(dv.cap_stream, hipStreamCaptureModeThreadLocal));
  try {
    pcg_iteration<T>(c, NR, flexible, dv.cap_stream, part);
  } catch (...) {
    (void)hipStreamEndCapture(dv.cap_stream, &g);
    throw;
  }
  R3MG_HIP_CHECK(hipStreamEndCapture(dv.cap_stream, &g));
  hipGraphExec_t ex;
  R3MG_HIP_CHECK(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
  dv.graphs[key] = ex;
  dv.graph_defs[key] = g;
  return ex;
}

// ---------------------------------------------------------------------------------------------
// Host side of the solve.  Convergence is decided on the device: every kernel of an iteration returns at once
// when all columns have converged, so iterations may be enqueued ahead without reading anything back.  The host
// enqueues the whole predicted solve as one chunk (captured iteration graphs back to back) and reads the state
// once at its end; only when the prediction fell short does it enqueue a further chunk.  The iteration predicted
// to converge is enqueued as its first half (part 1), whose stop test needs no V-cycle; the second half follows
// only if that test failed.  The chunk ends on the device with the float32 V-cycle's true-residual check
// (residual replacement), the write-back of the solution and the state copied into pinned host memory, so a
// solve that converges as predicted synchronises once.
// ---------------------------------------------------------------------------------------------
namespace {

int record_key(int NR, bool fp32) { return NR * 2 + (fp32 ? 1 : 0); }

// iterations to enqueue before the first read: those of the last converged solve with the same key and stop
// rule, else the count its mean residual reduction needs for rtol, else 3
int predict_first(const Device& dv, int key, double rtol, double atol, int maxit) {
  int k = 3;
  auto it = dv.last_solve.find(key);
  if (it != dv.last_solve.end()) {
    const Device::SolveRecord& r = it->second;
    if (r.rtol == rtol && r.atol == atol)
      k = r.iters;
    else if (r.q > 0.0 && r.q < 1.0 && rtol > 0.0)
      k = (int)std::ceil(2.0 * std::log(rtol) / std::log(r.q));
  }
  return std::max(0, std::min(maxit, std::max(1, k)));
}

// further iterations the open columns of a state need, assuming each repeats its last residual reduction
int predict_more(const PcgState& st, int nb) {
  int m = 1;
  for (int j = 0; j < nb; ++j) {
    if (st.done[j]) continue;
    const double rr = st.rr[j], rp = st.rr_prev[j], tau = st.tau2[j];
    if (!(rp > 0.0) || !(rr > 0.0) || !(rr < rp) || !(tau > 0.0)) continue;
    const double need = std::ceil(std::log(tau / rr) / std::log(rr / rp));
    if (need > m) m = (int)std::min(need, 1000.0);
  }
  return m;
}

void record_solve(Device& dv, int key, double rtol, double atol, const PcgState& st, int nb) {
  int kmax = 0;
  double q = 0.0;
  for (int j = 0; j < nb; ++j)
    if (st.iters[j] >= kmax && st.iters[j] > 0) {
      kmax = st.iters[j];
      q = (st.rr0[j] > 0.0 && st.rr[j] > 0.0) ? std::pow(st.rr[j] / st.rr0[j], 1.0 / st.iters[j]) : 0.0;
    }
  if (kmax > 0) dv.last_solve[key] = Device::SolveRecord{rtol, atol, q, kmax};
}

}  // namespace

template <typename T>
static r3mg_status pcg_block(HandleImpl& h, const double* b, double* x, int c0, int nb, double rtol, double atol,
                             int maxit, hipStream_t s, int* iters, double* relres, double* cond) {
  Analysis& an = *h.an;
  Device& dv = *h.dev;
  Ctx c{an, dv, sizeof(T) == 4};
  int NR = 1;
  while (NR < nb) NR <<= 1;
  ensure_level_vectors(c, NR);
  ensure_pcg_vectors(c, NR);
  ensure_hist(dv, std::max(maxit, 1));
  autotune_spmm<T>(c, NR, s);
  const int n = (int)an.n;
  const bool flexible = sizeof(T) == 4;
  PcgState* dst = reinterpret_cast<PcgState*>(dv.state.p);
  if (!dv.ev[0]) {
    R3MG_HIP_CHECK(hipEventCreateWithFlags(&dv.ev[0], hipEventDisableTiming));
    R3MG_HIP_CHECK(hipEventCreateWithFlags(&dv.ev[1], hipEventDisableTiming));
  }
  launch_gather_cols(n, NR, nb, dv.perm.p, b + (int64_t)c0 * n, n, dv.pb.p, s);
  launch_gather_cols(n, NR, nb, dv.perm.p, x + (int64_t)c0 * n, n, dv.px.p, s);
  pcg_start<T>(c, NR, nb, rtol, atol, flexible, false, s);
  hipGraphExec_t ex[3] = {nullptr, nullptr, nullptr};
  if (an.opt.use_graph)
    for (int part = 0; part < 3; ++part) ex[part] = iteration_graph<T>(c, NR, flexible, part);
  auto launch_part = [&](int part) {
    if (ex[part])
      R3MG_HIP_CHECK(hipGraphLaunch(ex[part], s));
    else
      pcg_iteration<T>(c, NR, flexible, s, part);
  };
  int k = 0;           // iterations enqueued
  bool split = false;  // the last one enqueued stopped after its stop test
  auto enqueue_to = [&](int target) {
    if (split && k < target) {
      launch_part(2);
      split = false;
    }
    while (k < target) {
      const bool last = k + 1 == target;
      launch_part(last ? 1 : 0);
      ++k;
      split = last;
    }
  };
  PcgState st;
  auto finish_chunk = [&]() {
    if (flexible) {
      // true residual of x (into z, which the next iteration's second half rewrites before reading it)
      pcg_operator(c, NR, dv.px.p, dv.pz.p, nullptr, s);
      launch_pcg_true_residual(n, NR, dv.pb.p, dv.pz.p, dv.partials.p, dst, s);
    }
    launch_scatter_cols(n, NR, nb, dv.perm.p, dv.px.p, x + (int64_t)c0 * n, n, s);
    launch_pcg_state_out(dst, static_cast<PcgState*>(dv.pinned_dev), s);
    R3MG_HIP_CHECK(hipEventRecord(dv.ev[0], s));
    R3MG_HIP_CHECK(hipEventSynchronize(dv.ev[0]));
    std::memcpy(&st, dv.pinned, sizeof(PcgState));
  };
  const int key = record_key(NR, flexible);
  enqueue_to(predict_first(dv, key, rtol, atol, maxit));
  int restarts = 0;
  for (;;) {
    finish_chunk();
    if (st.all_done) {
      // residual replacement (float32 V-cycle): a column whose true residual fails the stop rule restarts from it,
      // at most twice per solve
      if (!(flexible && st.restart && restarts < 2 && k < maxit)) break;
      ++restarts;
      pcg_start<T>(c, NR, nb, rtol, atol, flexible, true, s);
      split = false;
      enqueue_to(std::min(maxit, k + 2));
      continue;
    }
    if (k >= maxit) break;
    enqueue_to(std::min(maxit, k + predict_more(st, nb)));
  }
  dv.last_restarts = restarts;
  bool conv = true;
  for (int j = 0; j < nb; ++j) {
    const double rr = flexible ? st.rr_true[j] : st.rr[j];
    if (iters) iters[c0 + j] = st.iters[j];
    if (relres) relres[c0 + j] = st.rr0[j] > 0 ? std::sqrt(rr / st.rr0[j]) : 0.0;
    // the float32 V-cycle reports convergence only when the true residual passes the stop rule as well
    conv &= st.done[j] != 0 && (!flexible || rr <= st.tau2[j]);
  }
  if (conv && restarts == 0) record_solve(dv, key, rtol, atol, st, nb);
  if (cond) {
    int mmax = 0;
    for (int j = 0; j < nb; ++j) mmax = std::max(mmax, std::min(st.iters[j], dv.hist_rows));
    std::vector<double> hh((size_t)2 * kMaxNR * std::max(1, mmax));
    if (mmax > 0)
      R3MG_HIP_CHECK(hipMemcpy(hh.data(), dv.hist.p, (size_t)2 * kMaxNR * mmax * sizeof(double), hipMemcpyDeviceToHost));
    for (int j = 0; j < nb; ++j) {
      const int m = std::min(st.iters[j], dv.hist_rows);
      std::vector<double> al(m), be(m > 0 ? m - 1 : 0);
      for (int i = 0; i < m; ++i) al[i] = hh[(size_t)2 * i * kMaxNR + j];
      for (int i = 0; i + 1 < m; ++i) be[i] = hh[(size_t)(2 * i + 1) * kMaxNR + j];
      cond[c0 + j] = cg_condition(al, be);
    }
  }
  return conv ? R3MG_OK : R3MG_NOT_CONVERGED;
}

r3mg_status pcg_solve(HandleImpl& h, const double* b, double* x, int nrhs, double rtol, double atol, int maxit,
                      hipStream_t s, double* cond, int* iters, double* relres) {
  r3mg_status res = R3MG_OK;
  for (int c0 = 0; c0 < nrhs; c0 += kMaxNR) {
    const int nb = std::min(kMaxNR, nrhs - c0);
    r3mg_status r = h.an->opt.vcycle_fp32
                        ? pcg_block<float>(h, b, x, c0, nb, rtol, atol, maxit, s, iters, relres, cond)
                        : pcg_block<double>(h, b, x, c0, nb, rtol, atol, maxit, s, iters, relres, cond);
    if (r != R3MG_OK) res = r;
  }
  return res;
}

int residual_history(HandleImpl& h, int col, double* rr, int cap) {
  Device& dv = *h.dev;
  if (!dv.hist.p || col < 0 || col >= kMaxNR) return 0;
  PcgState st;
  R3MG_HIP_CHECK(hipMemcpy(&st, dv.state.p, sizeof(PcgState), hipMemcpyDeviceToHost));
  const int m = std::min(st.iters[col], dv.hist_rows) + 1;
  if (rr && cap > 0) {
    std::vector<double> v((size_t)m * kMaxNR);
    R3MG_HIP_CHECK(hipMemcpy(v.data(), rhist_of(dv), v.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int j = 0; j < std::min(m, cap); ++j) rr[j] = std::sqrt(v[(size_t)j * kMaxNR + col]);
  }
  return m;
}

// Several problems in one launch sequence: one iteration of every problem (its two halves, so that the stop test
// comes before the V-cycle, whose kernels return at once for a converged problem) is captured into one hipGraph
// with one branch per problem, and the graph is replayed
// in chunks as in pcg_block (whole iterations only: a problem
// restarted by residual replacement must not receive the second half of an iteration); at the end of a chunk
// every problem's state lands in one pinned array, read after one synchronisation.  Problems with a float32
// V-cycle get the same true-residual check and restart.
namespace {
struct BranchStreams {
  std::vector<hipStream_t> s;
  ~BranchStreams() {
    for (auto q : s) (void)hipStreamDestroy(q);
  }
};
// capture-only streams, created once per thread and device and reused by every group solve
std::vector<hipStream_t>& branch_streams(int dev, int count) {
  static thread_local std::map<int, BranchStreams> pool;
  BranchStreams& b = pool[dev];
  while ((int)b.s.size() < count + 1) {
    hipStream_t q;
    R3MG_HIP_CHECK(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
    b.s.push_back(q);
  }
  return b.s;
}

// The instantiated group graphs, by device and (handle, graph epoch, V-cycle precision) of every problem in order:
// a later group solve of the same handles, none of whose graphs was dropped since, replays it without capturing
// again.  A key never matches a freed or changed handle (epochs are unique), and at most kGroupGraphs are kept.
struct GroupGraph {
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
  std::vector<hipEvent_t> evs;  // the capture's fork and join events, kept with the graph
  uint64_t used = 0;
};
constexpr size_t kGroupGraphs = 16;
std::mutex g_group_mu;
std::map<std::vector<uint64_t>, GroupGraph> g_group_graphs;
uint64_t g_group_clock = 0;

void destroy_group_graph(GroupGraph& gg) {
  if (gg.ex) (void)hipGraphExecDestroy(gg.ex);
  if (gg.g) (void)hipGraphDestroy(gg.g);
  for (auto e : gg.evs) (void)hipEventDestroy(e);
  gg = GroupGraph{};
}
}  // namespace

r3mg_status pcg_group(int count, HandleImpl** hs, const double* const* b, double* const* x, double rtol, int maxit,
                      hipStream_t s, int* iters, double* relres) {
  int dev = 0;
  R3MG_HIP_CHECK(hipGetDevice(&dev));
  std::vector<hipStream_t>& br = branch_streams(dev, count);
  hipStream_t cap = br[count];
  GroupGraph fresh;       // a graph captured by this call, until it is cached
  hipGraphExec_t ex = nullptr;
  std::vector<hipEvent_t> evs;
  void* pin = nullptr;
  std::unique_lock<std::mutex> lk(g_group_mu, std::defer_lock);
  auto cleanup = [&]() {
    destroy_group_graph(fresh);
    for (auto e : evs) (void)hipEventDestroy(e);
    if (pin) (void)hipHostFree(pin);
  };
  auto is32 = [&](int k) { return hs[k]->an->opt.vcycle_fp32 != 0; };
  try {
    R3MG_HIP_CHECK(hipHostMalloc(&pin, (size_t)count * sizeof(PcgState) + 64, hipHostMallocDefault));
    void* pin_dev = nullptr;
    R3MG_HIP_CHECK(hipHostGetDevicePointer(&pin_dev, pin, 0));
    // set-up of every problem (plain launches on s)
    for (int k = 0; k < count; ++k) {
      HandleImpl& h = *hs[k];
      Ctx c{*h.an, *h.dev, is32(k)};
      ensure_level_vectors(c, 1);
      ensure_pcg_vectors(c, 1);
      ensure_hist(*h.dev, std::max(maxit, 1));
      const int n = (int)h.an->n;
      launch_gather_cols(n, 1, 1, h.dev->perm.p, b[k], n, h.dev->pb.p, s);
      launch_gather_cols(n, 1, 1, h.dev->perm.p, x[k], n, h.dev->px.p, s);
      if (c.fp32)
        pcg_start<float>(c, 1, 1, rtol, 0.0, true, false, s);
      else
        pcg_start<double>(c, 1, 1, rtol, 0.0, false, false, s);
    }
    // one iteration of every problem, each on its own branch: the cached graph of these handles, else captured now
    std::vector<uint64_t> key{(uint64_t)dev};
    for (int k = 0; k < count; ++k) {
      key.push_back((uint64_t)(uintptr_t)hs[k]);
      key.push_back(hs[k]->dev->graph_epoch);
      key.push_back(is32(k) ? 1 : 0);
    }
    lk.lock();  // held until the solve ends: the cached graph is not evicted or replayed by another call meanwhile
    auto hit = g_group_graphs.find(key);
    if (hit != g_group_graphs.end()) {
      hit->second.used = ++g_group_clock;
      ex = hit->second.ex;
    } else {
      hipEvent_t fork;
      R3MG_HIP_CHECK(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
      fresh.evs.push_back(fork);
      R3MG_HIP_CHECK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
      try {
        R3MG_HIP_CHECK(hipEventRecord(fork, cap));
        for (int k = 0; k < count; ++k) {
          HandleImpl& h = *hs[k];
          Ctx c{*h.an, *h.dev, is32(k)};
          R3MG_HIP_CHECK(hipStreamWaitEvent(br[k], fork, 0));
          // the iteration in its two halves: the stop test precedes the V-cycle, whose kernels then return at
          // once in the iteration where the problem converges (problems converge at different iterations)
          for (int part = 1; part <= 2; ++part) {
            if (c.fp32)
              pcg_iteration<float>(c, 1, true, br[k], part, true);
            else
              pcg_iteration<double>(c, 1, false, br[k], part, true);
          }
          hipEvent_t j;
          R3MG_HIP_CHECK(hipEventCreateWithFlags(&j, hipEventDisableTiming));
          fresh.evs.push_back(j);
          R3MG_HIP_CHECK(hipEventRecord(j, br[k]));
          R3MG_HIP_CHECK(hipStreamWaitEvent(cap, j, 0));
        }
      } catch (...) {
        hipGraph_t dead;
        (void)hipStreamEndCapture(cap, &dead);
        if (dead) (void)hipGraphDestroy(dead);
        throw;
      }
      R3MG_HIP_CHECK(hipStreamEndCapture(cap, &fresh.g));
      R3MG_HIP_CHECK(hipGraphInstantiate(&fresh.ex, fresh.g, nullptr, nullptr, 0));
      ex = fresh.ex;
      if (g_group_graphs.size() >= kGroupGraphs) {  // evict the least recently used
        auto old = g_group_graphs.begin();
        for (auto it = g_group_graphs.begin(); it != g_group_graphs.end(); ++it)
          if (it->second.used < old->second.used) old = it;
        destroy_group_graph(old->second);
        g_group_graphs.erase(old);
      }
      fresh.used = ++g_group_clock;
      g_group_graphs[key] = fresh;
      fresh = GroupGraph{};  // owned by the cache now
    }
    hipEvent_t done_ev;
    R3MG_HIP_CHECK(hipEventCreateWithFlags(&done_ev, hipEventDisableTiming));
    evs.push_back(done_ev);
    std::vector<PcgState> st(count);
    const PcgState* hst = static_cast<const PcgState*>(pin);
    int k = 0;
    auto enqueue_to = [&](int target) {
      for (; k < target; ++k) R3MG_HIP_CHECK(hipGraphLaunch(ex, s));
    };
    auto finish_chunk = [&]() {
      for (int q = 0; q < count; ++q) {
        HandleImpl& h = *hs[q];
        Device& dv = *h.dev;
        PcgState* dst = reinterpret_cast<PcgState*>(dv.state.p);
        if (is32(q)) {
          Ctx c{*h.an, dv, true};
          apply_level<double>(c, 0, 1, dv.px.p, nullptr, dv.pz.p, nullptr, nullptr, 0, 0, F_PLAIN, nullptr, s);
          launch_pcg_true_residual((int)h.an->n, 1, dv.pb.p, dv.pz.p, dv.partials.p, dst, s);
        }
        launch_scatter_cols((int)h.an->n, 1, 1, dv.perm.p, dv.px.p, x[q], h.an->n, s);
        launch_pcg_state_out(dst, static_cast<PcgState*>(pin_dev) + q, s);
      }
      R3MG_HIP_CHECK(hipEventRecord(done_ev, s));
      R3MG_HIP_CHECK(hipEventSynchronize(done_ev));
      std::memcpy(st.data(), hst, (size_t)count * sizeof(PcgState));
    };
    int first = 0;
    for (int q = 0; q < count; ++q)
      first = std::max(first, predict_first(*hs[q]->dev, record_key(1, is32(q)), rtol, 0.0, maxit));
    enqueue_to(first);
    std::vector<int> restarts(count, 0);
    for (;;) {
      finish_chunk();
      bool all = true, restarted = false;
      int more = 1;
      for (int q = 0; q < count; ++q) {
        if (!st[q].all_done) {
          all = false;
          more = std::max(more, predict_more(st[q], 1));
        } else if (is32(q) && st[q].restart && restarts[q] < 2 && k < maxit) {
          ++restarts[q];
          Ctx c{*hs[q]->an, *hs[q]->dev, true};
          pcg_start<float>(c, 1, 1, rtol, 0.0, true, true, s);
          restarted = true;
          all = false;
        }
      }
      if (all || k >= maxit) break;
      if (restarted) more = std::max(more, 2);
      enqueue_to(std::min(maxit, k + more));
    }
    r3mg_status res = R3MG_OK;
    for (int q = 0; q < count; ++q) {
      const bool f32 = is32(q);
      const double rr = f32 ? st[q].rr_true[0] : st[q].rr[0];
      if (iters) iters[q] = st[q].iters[0];
      if (relres) relres[q] = st[q].rr0[0] > 0 ? std::sqrt(rr / st[q].rr0[0]) : 0.0;
      const bool conv = st[q].done[0] && (!f32 || rr <= st[q].tau2[0]);
      if (!conv) res = R3MG_NOT_CONVERGED;
      if (conv && restarts[q] == 0) record_solve(*hs[q]->dev, record_key(1, f32), rtol, 0.0, st[q], 1);
    }
    cleanup();
    return res;
  } catch (...) {
    cleanup();
    throw;
  }
}

// ---------------------------------------------------------------------------------------------
// Matrix-free fine operator
// ---------------------------------------------------------------------------------------------
void detach_matrix_free(HandleImpl& h) {
  if (!h.dev) return;
  Device& dv = *h.dev;
  DevLevel& D0 = dv.lv[0];
  const bool was_on = D0.mf != nullptr;
  D0.mf = nullptr;
  D0.bytes_apply = D0.shape_bytes[D0.shape];
  MatFreeDev& F = dv.mf;
  F.on = false;
  F.conn.release();
  F.inc_ptr.release();
  F.inc.release();
  F.geo64.release();
  F.cd64.release();
  F.y64.release();
  F.geo32.release();
  F.cd32.release();
  F.y32.release();
  F.y64mr.release();
  F.y32mr.release();
  F.mr_cap = 0;
  if (was_on) drop_graphs(dv);
}

void attach_matrix_free(HandleImpl& h, MatFreeHost&& m, hipStream_t s) {
  detach_matrix_free(h);
  Analysis& an = *h.an;
  Device& dv = *h.dev;
  Ctx c{an, dv, an.opt.vcycle_fp32 != 0};
  MatFreeDev& F = dv.mf;
  const int64_t n = an.n;
  try {
    F.conn.upload(m.conn, s);
    F.inc_ptr.upload(m.inc_ptr, s);
    F.inc.upload(m.inc, s);
    F.geo64.upload(m.geo, s);
    F.cd64.upload(m.cd, s);
    F.y64.alloc((size_t)m.ncells * m.nlocp);
    if (c.fp32) {
      F.geo32.alloc(m.geo.size());
      launch_cast_d2f((int64_t)m.geo.size(), F.geo64.p, F.geo32.p, s);
      F.cd32.alloc(n);
      launch_cast_d2f(n, F.cd64.p, F.cd32.p, s);
      F.y32.alloc((size_t)m.ncells * m.nlocp);
    }
    F.affine = m.affine;
    F.p = m.p;
    F.nincid = (int64_t)m.inc.size();
    F.op.d = m.d;
    F.op.k = m.k;
    F.op.n = (int)n;
    F.op.ncells = (int)m.ncells;
    F.op.nlocp = m.nlocp;
    F.op.affine = m.affine;
    F.op.conn = F.conn.p;
    F.op.inc_ptr = F.inc_ptr.p;
    F.op.inc = F.inc.p;
    for (int q = 0; q < 4; ++q) {
      F.t64.W[q] = m.W[q];
      F.t32.W[q] = (float)m.W[q];
      F.t64.X[q] = m.X[q];
      F.t32.X[q] = (float)m.X[q];
      for (int i = 0; i < 4; ++i) {
        F.t64.B[q][i] = m.B[q][i];
        F.t64.G[q][i] = m.G[q][i];
        F.t32.B[q][i] = (float)m.B[q][i];
        F.t32.G[q][i] = (float)m.G[q][i];
      }
    }
    // algorithmic bytes: connectivity, geometry, cell-local outputs written and read back, incidence lists,
    // 7 vector streams (as for the CSR kernels)
    for (int sv = 4; sv <= 8; sv += 4) {
      const double by = (double)m.ncells * m.nloc * 4 + (double)m.geo.size() * sv +
                        (double)m.ncells * m.nloc * sv + (double)(n + 1) * 4 + (double)F.nincid * (4 + sv) +
                        7.0 * n * sv;
      (sv == 4 ? F.bytes32 : F.bytes64) = by;
    }
    // the operator must reproduce the caller's matrix: y = A v for a fixed pseudo-random v, both ways
    ensure_pcg_vectors(c, 1);
    std::vector<double> v(n), y1(n), y2(n);
    for (int64_t i = 0; i < n; ++i) v[i] = (double)((uint32_t)((uint64_t)i * 2654435761u)) / 4294967296.0 - 0.5;
    R3MG_HIP_CHECK(hipMemcpyAsync(dv.pb.p, v.data(), n * sizeof(double), hipMemcpyHostToDevice, s));
    launch_level<double>(level_op<double>(c, 0), 1, dv.pb.p, nullptr, dv.pq.p, nullptr, nullptr, 0.0, 0.0, F_PLAIN,
                         nullptr, s);
    launch_mf_apply<double>(F.op, F.t64, F.geo64.p, F.cd64.p, F.y64.p, dv.lv[0].dinv64.p, dv.pb.p, nullptr,
                            dv.pz.p, nullptr, nullptr, 0.0, 0.0, F_PLAIN, nullptr, s);
    R3MG_HIP_CHECK(hipMemcpyAsync(y1.data(), dv.pq.p, n * sizeof(double), hipMemcpyDeviceToHost, s));
    R3MG_HIP_CHECK(hipMemcpyAsync(y2.data(), dv.pz.p, n * sizeof(double), hipMemcpyDeviceToHost, s));
    R3MG_HIP_CHECK(hipStreamSynchronize(s));
    double ymax = 0.0, dmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      ymax = std::max(ymax, std::fabs(y1[i]));
      dmax = std::max(dmax, std::fabs(y1[i] - y2[i]));
    }
    if (!(dmax <= 1e-10 * ymax)) {
      char msg[160];
      snprintf(msg, sizeof msg,
               "matrix-free operator does not reproduce the matrix (max |difference| %.3e, max |A v| %.3e)", dmax,
               ymax);
      throw Error{R3MG_ERR_INVALID, msg};
    }
  } catch (...) {
    detach_matrix_free(h);
    throw;
  }
  F.on = true;
  DevLevel& D0 = dv.lv[0];
  D0.mf = &F;
  D0.bytes_apply = c.fp32 ? F.bytes32 : F.bytes64;
  drop_graphs(dv);
}

// bytes one application of level l for nr right-hand sides moves in the storage format of the kernel that applies
// it (fine level with several right-hand sides: the tuned kernel's format), 7 vector streams included
static double level_bytes(Ctx& c, int l, int nr, int esz) {
  DevLevel& D = c.dv.lv[l];
  const double vec = 7.0 * (double)D.n * esz;
  if (nr == 1) return D.bytes_apply;
  if (l == 0 && !D.mf) {
    auto it = c.dv.tuned.find({0, nr * 2 + (esz == 4 ? 1 : 0)});
    const double nnz = (double)D.nnz, n = (double)D.n;
    const int cls = mr_class(nr, esz);
    if (it != c.dv.tuned.end() && it->second < 0 && cls >= 0) {
      // values, 2-byte positions, distinct-column lists, block records, row order and row pointers
      const double nuc = (double)D.mucol[cls].n - 1, nrb = (double)D.mr[cls].nrb;
      return nnz * (esz + 2) + 4.0 * nuc + 16.0 * (nrb + 1) + 4.0 * n + 4.0 * (n + 1) + vec * nr;
    }
    return nnz * (esz + 4) + 4.0 * (n + 1) + vec * nr;  // CSR kernels
  }
  return D.bytes_apply + vec * (nr - 1);
}

void time_smoother_kernel(HandleImpl& h, int level, int nrhs, int reps, int64_t flush_bytes, hipStream_t s,
                          double* ms, double* bytes) {
  Analysis& an = *h.an;
  Device& dv = *h.dev;
  Ctx c{an, dv, an.opt.vcycle_fp32 != 0};
  ensure_level_vectors(c, nrhs);
  if (nrhs > 1) {
    ensure_pcg_vectors(c, nrhs);
    if (c.fp32)
      autotune_spmm<float>(c, nrhs, s);
    else
      autotune_spmm<double>(c, nrhs, s);
  }
  DevLevel& D = dv.lv[level];
  hipEvent_t e0, e1;
  R3MG_HIP_CHECK(hipEventCreate(&e0));
  R3MG_HIP_CHECK(hipEventCreate(&e1));
  const int fl = F_RHO_STORE | F_X_ADD | F_D_OUT;
  auto launch_on = [&](int r, hipStream_t st) {
    if (c.fp32) {
      float* u = vbuf<float>((r & 1) ? D.dB : D.dA);
      float* w = vbuf<float>((r & 1) ? D.dA : D.dB);
      apply_level<float>(c, level, nrhs, u, vbuf<float>(D.b), vbuf<float>(D.rho), vbuf<float>(D.x), w, 0.0, 0.0, fl,
                         nullptr, st);
    } else {
      double* u = vbuf<double>((r & 1) ? D.dB : D.dA);
      double* w = vbuf<double>((r & 1) ? D.dA : D.dB);
      apply_level<double>(c, level, nrhs, u, vbuf<double>(D.b), vbuf<double>(D.rho), vbuf<double>(D.x), w, 0.0, 0.0,
                          fl, nullptr, st);
    }
  };
  auto launch = [&](int r) { launch_on(r, s); };
  float t = 0;
  try {
    for (int r = 0; r < 3; ++r) launch(r);
    if (flush_bytes <= 0) {
      // back to back from a captured graph, as a smoothing sweep runs inside the V-cycle's graph (eager launches
      // would time the host's launch rate on the small levels); the graph is replayed once untimed
      if (!dv.cap_stream) R3MG_HIP_CHECK(hipStreamCreateWithFlags(&dv.cap_stream, hipStreamNonBlocking));
      R3MG_HIP_CHECK(hipStreamSynchronize(s));
      hipGraph_t g = nullptr;
      hipGraphExec_t ex = nullptr;
      R3MG_HIP_CHECK(hipStreamBeginCapture(dv.cap_stream, hipStreamCaptureModeThreadLocal));
      try {
        for (int r = 0; r < reps; ++r) launch_on(r, dv.cap_stream);
      } catch (...) {
        (void)hipStreamEndCapture(dv.cap_stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      R3MG_HIP_CHECK(hipStreamEndCapture(dv.cap_stream, &g));
      hipError_t err = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      if (err == hipSuccess) err = hipGraphLaunch(ex, s);
      if (err == hipSuccess) err = hipEventRecord(e0, s);
      if (err == hipSuccess) err = hipGraphLaunch(ex, s);
      if (err == hipSuccess) err = hipEventRecord(e1, s);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
      if (ex) (void)hipGraphExecDestroy(ex);
      (void)hipGraphDestroy(g);
      R3MG_HIP_CHECK(err);
    } else {
      // each launch alone, after a pass that reads and writes flush_bytes of other memory (more than the caches
      // hold), so that the matrix and vectors come from HBM
      DBuf<double> fb;
      const int64_t nf = std::max<int64_t>(1, flush_bytes / 8);
      fb.alloc((size_t)nf);
      R3MG_HIP_CHECK(hipMemsetAsync(fb.p, 0, (size_t)nf * 8, s));
      for (int r = 0; r < reps; ++r) {
        launch_axpby(nf, 1.0, fb.p, 1.0, fb.p, s);
        R3MG_HIP_CHECK(hipEventRecord(e0, s));
        launch(r);
        R3MG_HIP_CHECK(hipEventRecord(e1, s));
        R3MG_HIP_CHECK(hipEventSynchronize(e1));
        float tr = 0;
        R3MG_HIP_CHECK(hipEventElapsedTime(&tr, e0, e1));
        t += tr;
      }
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = (double)t / reps;
  *bytes = level_bytes(c, level, nrhs, c.fp32 ? 4 : 8);
}

}  // namespace r3mg
