// Host analysis of R3MG-C: constrained set, bisection R-tree, level selection, DoF permutation, transfer
// tables, unisolvence check and Galerkin block sparsity.  Pure C++ (no HIP calls).
//
// Paper: Section 3 (Definition of an R-tree of order (m,M)), Section 4 (point-based agglomeration, transfer
// construction, Remarks on parameters and heuristics), Section 6 (level choice).  Readings where the paper is
// silent (the Boost R*-tree is replaced by a deterministic bisection bulk load):
//   depth t = smallest t with 2^t * leaf >= n; a split orders its points lexicographically by
//   (x_{a*}, x_{a*+1 mod d}, ..., point index) with a* the first axis of largest extent and keeps the first
//   ceil(|S|/2) points on the left; level l+1 sits d tree levels above level l; coarsening stops at the first
//   level with at most max_coarse_dofs DoFs, at max_levels, or at the root.
// All floating-point decisions (extents, comparisons, unisolvence pivots) are taken in float64; this file is
// compiled without floating-point contraction so that the transfer values are reproducible.
#include <algorithm>
#include <array>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include "kernels.h"
#include "r3mg_internal.h"

namespace r3mg {

namespace {

template <typename F>
void parallel_for(int64_t count, F&& f) {
  unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (count < 64 || hw == 1) {
    for (int64_t i = 0; i < count; ++i) f(i);
    return;
  }
  std::atomic<int64_t> next{0};
  std::vector<std::thread> th;
  for (unsigned t = 0; t < hw; ++t)
    th.emplace_back([&] {
      for (;;) {
        int64_t i = next.fetch_add(1);
        if (i >= count) break;
        f(i);
      }
    });
  for (auto& t : th) t.join();
}

int tree_depth(int64_t n, int64_t leaf) {
  int t = 0;
  while ((leaf << t) < n) ++t;
  return t;
}

Error err(r3mg_status c, const std::string& m) { return Error{c, m}; }

// l_j(s) = prod_{m != j} (s - t_m) / (t_j - t_m), evaluated in the order m = 0, 1, ...
inline double lagrange(const double* t, int k, int j, double s) {
  double v = 1.0;
  for (int m = 0; m < k; ++m)
    if (m != j) v *= (s - t[m]) / (t[j] - t[m]);
  return v;
}

}  // namespace

void box_nodes_1d(int pc, double* t) {
  switch (pc) {
    case 0: t[0] = 0.5; break;
    case 1: t[0] = 0.0; t[1] = 1.0; break;
    case 2: t[0] = 0.0; t[1] = 0.5; t[2] = 1.0; break;
    default: {
      double s = 1.0 / std::sqrt(5.0);
      t[0] = 0.0; t[1] = 0.5 * (1.0 - s); t[2] = 0.5 * (1.0 + s); t[3] = 1.0;
    }
  }
}

void bisection_rtree(const double* x, int64_t n, int d, int leaf, int& depth, std::vector<int32_t>& order,
                     std::vector<std::vector<int64_t>>& offsets) {
  depth = tree_depth(n, leaf);
  order.resize(n);
  std::iota(order.begin(), order.end(), 0);
  offsets.assign(depth + 1, {});
  offsets[0] = {0, n};
  for (int k = 0; k < depth; ++k) {
    const std::vector<int64_t>& off = offsets[k];
    int64_t nseg = (int64_t)off.size() - 1;
    parallel_for(nseg, [&](int64_t s) {
      int64_t a = off[s], b = off[s + 1];
      if (b - a < 2) return;
      double mn[3], mx[3];
      for (int c = 0; c < d; ++c) { mn[c] = INFINITY; mx[c] = -INFINITY; }
      for (int64_t i = a; i < b; ++i) {
        const double* p = x + (int64_t)order[i] * d;
        for (int c = 0; c < d; ++c) { mn[c] = std::min(mn[c], p[c]); mx[c] = std::max(mx[c], p[c]); }
      }
      int astar = 0;
      double best = mx[0] - mn[0];
      for (int c = 1; c < d; ++c)
        if (mx[c] - mn[c] > best) { best = mx[c] - mn[c]; astar = c; }
      std::sort(order.begin() + a, order.begin() + b, [&](int32_t i, int32_t j) {
        const double* pi = x + (int64_t)i * d;
        const double* pj = x + (int64_t)j * d;
        for (int m = 0; m < d; ++m) {
          int c = (astar + m) % d;
          if (pi[c] < pj[c]) return true;
          if (pj[c] < pi[c]) return false;
        }
        return i < j;
      });
    });
    std::vector<int64_t> nxt(2 * nseg + 1);
    nxt[0] = 0;
    for (int64_t s = 0; s < nseg; ++s) {
      int64_t len = off[s + 1] - off[s];
      nxt[2 * s + 1] = off[s] + (len + 1) / 2;
      nxt[2 * s + 2] = off[s + 1];
    }
    offsets[k + 1] = std::move(nxt);
  }
}

std::unique_ptr<Analysis> analyze(const double* coords, int64_t n, const int64_t* row_ptr,
                                  const int32_t* col_idx, const double* vals, const r3mg_options& opt,
                                  const int32_t* cells, int64_t ncells, int nloc) {
  auto an = std::make_unique<Analysis>();
  an->opt = opt;
  const int d = opt.dim;
  const int pc = opt.coarse_degree;
  if (d != 2 && d != 3) throw err(R3MG_ERR_INVALID, "dim must be 2 or 3");
  if (pc < 0 || pc > 3) throw err(R3MG_ERR_INVALID, "coarse_degree must be in 0..3");
  if (opt.leaf_size < 1 || opt.max_levels < 0 || opt.max_levels == 1 || opt.max_coarse_dofs < 1 ||
      opt.cheb_degree < 1 || opt.pre_steps < 0 || opt.post_steps < 0 || opt.lanczos_steps < 1 ||
      !(opt.cheb_boost > 0.0) || !(opt.cheb_ratio > 1.0) || opt.fine_kernel < -1 ||
      opt.fine_kernel >= kFineShapes || opt.multi_rhs_kernel < -1 || opt.multi_rhs_kernel > 4 ||
      opt.matrix_cache < -1 || opt.matrix_cache > 1 || opt.tune_cache < 0 || opt.tune_cache > 1)
    throw err(R3MG_ERR_INVALID, "invalid option value");
  if (n < 1 || n >= (int64_t(1) << 31)) throw err(R3MG_ERR_INVALID, "n out of range");
  if (!coords || !row_ptr || !col_idx || !vals) throw err(R3MG_ERR_INVALID, "null input");
  int B = 1;
  for (int a = 0; a < d; ++a) B *= (pc + 1);
  an->d = d;
  an->pc = pc;
  an->B = B;
  an->n = n;
  if (row_ptr[0] != 0) throw err(R3MG_ERR_INVALID, "row_ptr[0] != 0");
  for (int64_t i = 0; i < n; ++i)
    if (row_ptr[i + 1] < row_ptr[i]) throw err(R3MG_ERR_INVALID, "row_ptr not monotone");
  const int64_t nnz = row_ptr[n];
  if (nnz >= (int64_t(1) << 31)) throw err(R3MG_ERR_OOM, "nnz exceeds int32 range");
  an->nnz = nnz;
  for (int64_t i = 0; i < n * d; ++i)
    if (!std::isfinite(coords[i])) throw err(R3MG_ERR_INVALID, "non-finite coordinate");
  for (int64_t i = 0; i < n; ++i)
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
      if (col_idx[p] < 0 || col_idx[p] >= n) throw err(R3MG_ERR_INVALID, "column index out of range");
      if (p > row_ptr[i] && col_idx[p] <= col_idx[p - 1])
        throw err(R3MG_ERR_INVALID, "columns must be strictly ascending within a row");
      if (!std::isfinite(vals[p])) throw err(R3MG_ERR_INVALID, "non-finite matrix value");
    }
  // the Jacobi smoother divides by the diagonal: every row, constrained ones included (their identity rows),
  // must store a positive diagonal entry (Section 6 smoother; the coarse levels are checked at r3mg_factor)
  for (int64_t i = 0; i < n; ++i) {
    double dg = 0.0;
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
      if (col_idx[p] == i) dg = vals[p];
    if (!(dg > 0.0))
      throw err(R3MG_ERR_NOT_SPD, "non-positive or missing diagonal entry in row " + std::to_string((long long)i));
  }
  an->user_rowptr.assign(row_ptr, row_ptr + n + 1);
  an->user_col.assign(col_idx, col_idx + nnz);

  // O1: constrained rows (all stored off-diagonal values exactly zero)
  std::vector<uint8_t>& cons_user = an->constrained_user;
  cons_user.assign(n, 1);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
      if (col_idx[p] != i && vals[p] != 0.0) { cons_user[i] = 0; break; }

  // R-tree and levels.  Point-based agglomeration (Section 4): the tree's leaves are the support points.
  // Cell-based agglomeration (Section 4): the tree's leaves are the cells (ordered by the centres of their
  // bounding boxes), a box is the bounding box of its cells' support points, and every support point belongs to
  // the first level-1 agglomerate, in array order, that holds one of its cells.
  std::vector<std::vector<int64_t>> offsets;  // per tree depth: point offsets of the nodes in the internal order
  std::vector<int32_t> cag;                    // cell-based: level-1 agglomerate of every cell
  std::vector<int32_t> corder;
  std::vector<std::vector<int64_t>> coff;
  an->cell_based = cells != nullptr;
  if (!an->cell_based) {
    bisection_rtree(coords, n, d, opt.leaf_size, an->depth, an->order, offsets);
  } else {
    if (ncells < 1 || nloc < 1 || ncells >= (int64_t(1) << 31)) throw err(R3MG_ERR_INVALID, "bad cell array");
    std::vector<double> cen((size_t)ncells * d);
    for (int64_t c = 0; c < ncells; ++c) {
      double lo3[3] = {INFINITY, INFINITY, INFINITY}, hi3[3] = {-INFINITY, -INFINITY, -INFINITY};
      for (int j = 0; j < nloc; ++j) {
        const int32_t v = cells[c * nloc + j];
        if (v < 0 || v >= n) throw err(R3MG_ERR_INVALID, "cell node index out of range");
        for (int a = 0; a < d; ++a) {
          lo3[a] = std::min(lo3[a], coords[(int64_t)v * d + a]);
          hi3[a] = std::max(hi3[a], coords[(int64_t)v * d + a]);
        }
      }
      for (int a = 0; a < d; ++a) cen[c * d + a] = 0.5 * (lo3[a] + hi3[a]);
    }
    bisection_rtree(cen.data(), ncells, d, opt.leaf_size, an->depth, corder, coff);
  }
  {
    int depth = opt.skip_leaf_level ? std::max(an->depth - d, 0) : an->depth;
    an->depths.push_back(depth);
    for (;;) {
      int nlev = (int)an->depths.size() + 1;
      int64_t nboxes = int64_t(1) << an->depths.back();
      if (nboxes * B <= opt.max_coarse_dofs) break;
      if (opt.max_levels && nlev >= opt.max_levels) break;
      if (an->depths.back() == 0) break;
      an->depths.push_back(std::max(an->depths.back() - d, 0));
    }
    const int64_t ncoarse = (int64_t(1) << an->depths.back()) * B;
    if (ncoarse > R3MG_MAX_COARSEST_DOFS)
      throw err(R3MG_ERR_INVALID, "coarsest level would have " + std::to_string(ncoarse) +
                                      " DoFs, more than the dense coarsest solve takes (" +
                                      std::to_string(R3MG_MAX_COARSEST_DOFS) + "): allow more levels");
  }
  if (an->cell_based) {
    for (auto& off : coff)
      for (size_t s = 0; s + 1 < off.size(); ++s)
        if (off[s + 1] == off[s]) throw err(R3MG_ERR_NOT_UNISOLVENT, "empty R-tree node (leaf_size too small)");
    // first-come ownership: agglomerates are visited in array order, so a point goes to the smallest agglomerate
    // index among its cells
    const int d1 = an->depths[0];
    cag.assign(ncells, 0);
    for (size_t k = 0; k + 1 < coff[d1].size(); ++k)
      for (int64_t p = coff[d1][k]; p < coff[d1][k + 1]; ++p) cag[corder[p]] = (int32_t)k;
    std::vector<int32_t> pown(n, INT32_MAX);
    for (int64_t c = 0; c < ncells; ++c)
      for (int j = 0; j < nloc; ++j) {
        int32_t& o = pown[cells[c * nloc + j]];
        o = std::min(o, cag[c]);
      }
    const int64_t nb1 = int64_t(1) << d1;
    std::vector<int64_t> cnt(nb1 + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
      if (pown[i] == INT32_MAX) throw err(R3MG_ERR_INVALID, "support point in no cell");
      ++cnt[pown[i] + 1];
    }
    for (int64_t k = 0; k < nb1; ++k) cnt[k + 1] += cnt[k];
    // internal order: by owner, then by caller index
    an->order.assign(n, 0);
    {
      std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
      for (int64_t i = 0; i < n; ++i) an->order[pos[pown[i]]++] = (int32_t)i;
    }
    // point offsets of the nodes at every depth up to d1 (ancestors of the level-1 agglomerates)
    offsets.assign(d1 + 1, {});
    for (int k = 0; k <= d1; ++k) {
      const int sh = d1 - k;
      std::vector<int64_t>& off = offsets[k];
      off.assign((int64_t(1) << k) + 1, 0);
      for (int64_t b = 0; b < nb1; ++b) off[(b >> sh) + 1] += cnt[b + 1] - cnt[b];
      for (size_t b = 0; b + 1 < off.size(); ++b) off[b + 1] += off[b];
    }
  } else {
    for (auto& off : offsets)
      for (size_t s = 0; s + 1 < off.size(); ++s)
        if (off[s + 1] == off[s]) throw err(R3MG_ERR_NOT_UNISOLVENT, "empty R-tree node (leaf_size too small)");
  }
  const int L = an->nlevels() - 1;
  an->lv.resize(L + 1);
  an->iperm.assign(n, 0);
  for (int64_t p = 0; p < n; ++p) an->iperm[an->order[p]] = (int32_t)p;
  an->coords_int.resize(n * d);
  for (int64_t p = 0; p < n; ++p)
    for (int a = 0; a < d; ++a) an->coords_int[p * d + a] = coords[(int64_t)an->order[p] * d + a];

  // boxes per level
  for (int l = 1; l <= L; ++l) {
    HostLevel& H = an->lv[l];
    H.depth = an->depths[l - 1];
    const std::vector<int64_t>& off = offsets[H.depth];
    H.nbox = (int64_t)off.size() - 1;
    H.n = H.nbox * B;
    H.lo.assign(H.nbox * d, INFINITY);
    H.hi.assign(H.nbox * d, -INFINITY);
    if (an->cell_based) {  // bounding box of the node's cells
      const int sh = an->depths[0] - H.depth;
      for (int64_t c = 0; c < ncells; ++c) {
        const int64_t k = cag[c] >> sh;
        for (int j = 0; j < nloc; ++j)
          for (int a = 0; a < d; ++a) {
            const double v = coords[(int64_t)cells[c * nloc + j] * d + a];
            H.lo[k * d + a] = std::min(H.lo[k * d + a], v);
            H.hi[k * d + a] = std::max(H.hi[k * d + a], v);
          }
      }
    }
    for (int64_t k = 0; k < H.nbox; ++k) {
      if (!an->cell_based)
        for (int64_t p = off[k]; p < off[k + 1]; ++p)
          for (int a = 0; a < d; ++a) {
            double v = an->coords_int[p * d + a];
            H.lo[k * d + a] = std::min(H.lo[k * d + a], v);
            H.hi[k * d + a] = std::max(H.hi[k * d + a], v);
          }
      double e2 = 0;
      for (int a = 0; a < d; ++a) e2 += (H.hi[k * d + a] - H.lo[k * d + a]) * (H.hi[k * d + a] - H.lo[k * d + a]);
      H.max_extent = std::max(H.max_extent, std::sqrt(e2));
    }
    if (l >= 2) H.child_shift = an->depths[l - 2] - an->depths[l - 1];
  }
  auto check_degenerate = [&](int l) {
    if (pc < 1) return;
    const HostLevel& H = an->lv[l];
    for (int64_t k = 0; k < H.nbox * d; ++k)
      if (!(H.hi[k] > H.lo[k])) throw err(R3MG_ERR_DEGENERATE_BOX, "box with zero extent on level " + std::to_string(l));
  };
  check_degenerate(1);

  // level-1 ownership, local coordinates, unisolvence
  an->leaf_off = offsets[an->depths[0]];
  an->constrained.resize(n);
  an->owner.resize(n);
  an->xi.assign(n * d, 0.0);
  double t[4];
  box_nodes_1d(pc, t);
  const HostLevel& H1 = an->lv[1];
  for (int64_t k = 0; k < H1.nbox; ++k)
    for (int64_t p = an->leaf_off[k]; p < an->leaf_off[k + 1]; ++p) {
      an->constrained[p] = cons_user[an->order[p]];
      an->owner[p] = an->constrained[p] ? -1 : (int32_t)k;
      if (pc >= 1)
        for (int a = 0; a < d; ++a)
          an->xi[p * d + a] = (an->coords_int[p * d + a] - H1.lo[k * d + a]) / (H1.hi[k * d + a] - H1.lo[k * d + a]);
    }
  {
    // The box reported does not depend on the order in which the threads reach the boxes: the lowest box that
    // owns fewer than B points if there is one, else the lowest box among those whose Cholesky fails at the
    // earliest column (stage 0: too few points, stage j + 1: pivot j).
    const int64_t nbox1 = H1.nbox;
    std::atomic<int64_t> bad{-1};  // stage * nbox1 + box, the least over the failing boxes
    auto note_bad = [&](int64_t stage, int64_t k) {
      const int64_t key = stage * nbox1 + k;
      int64_t cur = bad.load();
      while ((cur < 0 || key < cur) && !bad.compare_exchange_weak(cur, key)) {
      }
    };
    const int k1 = pc + 1;
    parallel_for(H1.nbox, [&](int64_t k) {
      std::vector<double> G(B * B, 0.0), L(B * B, 0.0), phi(B);
      int64_t cnt = 0;
      for (int64_t p = an->leaf_off[k]; p < an->leaf_off[k + 1]; ++p) {
        if (an->constrained[p]) continue;
        ++cnt;
        double l1[3][4];
        for (int a = 0; a < d; ++a)
          for (int j = 0; j < k1; ++j) l1[a][j] = (pc == 0) ? 1.0 : lagrange(t, k1, j, an->xi[p * d + a]);
        for (int q = 0; q < B; ++q) {
          double v = 1.0;
          int qq = q;
          for (int a = 0; a < d; ++a) { v *= l1[a][qq % k1]; qq /= k1; }
          phi[q] = v;
        }
        for (int i = 0; i < B; ++i)
          for (int j = 0; j < B; ++j) G[i * B + j] += phi[i] * phi[j];
      }
      if (cnt < B) {
        note_bad(0, k);
        return;
      }
      double dmax = 0;
      for (int i = 0; i < B; ++i) dmax = std::max(dmax, G[i * B + i]);
      double tol = 1e-12 * dmax;
      for (int j = 0; j < B; ++j) {
        double piv = G[j * B + j];
        for (int c = 0; c < j; ++c) piv -= L[j * B + c] * L[j * B + c];
        if (!(piv > tol)) {
          note_bad(1 + j, k);
          return;
        }
        L[j * B + j] = std::sqrt(piv);
        for (int i = j + 1; i < B; ++i) {
          double s = G[i * B + j];
          for (int c = 0; c < j; ++c) s -= L[i * B + c] * L[j * B + c];
          L[i * B + j] = s / L[j * B + j];
        }
      }
    });
    if (bad >= 0) throw err(R3MG_ERR_NOT_UNISOLVENT, "box " + std::to_string((long long)(bad.load() % nbox1)) +
                                                    " cannot interpolate Q^p' from its owned points");
  }
  for (int l = 2; l <= L; ++l) check_degenerate(l);

  // fine operator in the internal numbering
  an->rowptr.resize(n + 1);
  an->col.resize(nnz);
  an->val.resize(nnz);
  an->src.resize(nnz);
  an->rowptr[0] = 0;
  for (int64_t p = 0; p < n; ++p) {
    int64_t u = an->order[p];
    an->rowptr[p + 1] = an->rowptr[p] + (int32_t)(row_ptr[u + 1] - row_ptr[u]);
  }
  parallel_for(n, [&](int64_t p) {
    int64_t u = an->order[p];
    int64_t base = an->rowptr[p];
    int64_t len = row_ptr[u + 1] - row_ptr[u];
    std::vector<std::pair<int32_t, int64_t>> e(len);
    for (int64_t q = 0; q < len; ++q) e[q] = {an->iperm[col_idx[row_ptr[u] + q]], row_ptr[u] + q};
    std::sort(e.begin(), e.end());
    for (int64_t q = 0; q < len; ++q) {
      an->col[base + q] = e[q].first;
      an->src[base + q] = e[q].second;
      an->val[base + q] = vals[e[q].second];
    }
  });

  // Galerkin block sparsity, level 1: boxes linked by a stored entry between unconstrained points
  {
    HostLevel& H = an->lv[1];
    std::vector<std::vector<int32_t>> rows(H.nbox);
    parallel_for(H.nbox, [&](int64_t k) {
      std::vector<int32_t>& r = rows[k];
      for (int64_t p = an->leaf_off[k]; p < an->leaf_off[k + 1]; ++p) {
        if (an->constrained[p]) continue;
        for (int32_t q = an->rowptr[p]; q < an->rowptr[p + 1]; ++q) {
          int32_t c = an->col[q];
          if (an->constrained[c]) continue;
          r.push_back(an->owner[c]);
        }
      }
      std::sort(r.begin(), r.end());
      r.erase(std::unique(r.begin(), r.end()), r.end());
    });
    H.bptr.assign(H.nbox + 1, 0);
    for (int64_t k = 0; k < H.nbox; ++k) H.bptr[k + 1] = H.bptr[k] + (int64_t)rows[k].size();
    H.bcol.resize(H.bptr[H.nbox]);
    for (int64_t k = 0; k < H.nbox; ++k) std::copy(rows[k].begin(), rows[k].end(), H.bcol.begin() + H.bptr[k]);
  }
  // Galerkin work lists of level 1: for every stored block (K, K') the rows i of K (unconstrained) whose
  // columns meet box K', with the contiguous run [s, e) of those columns (columns are sorted and boxes are
  // contiguous in the internal numbering); the kernel visits only these runs.
  {
    HostLevel& H = an->lv[1];
    const int64_t nblk = H.bptr[H.nbox];
    std::vector<int32_t> box_all(n);
    for (int64_t k = 0; k < H.nbox; ++k)
      for (int64_t p = an->leaf_off[k]; p < an->leaf_off[k + 1]; ++p) box_all[p] = (int32_t)k;
    std::vector<std::vector<std::array<int32_t, 4>>> per(H.nbox);  // (slot, row, s, e)
    parallel_for(H.nbox, [&](int64_t k) {
      auto& v = per[k];
      const int32_t* bc = H.bcol.data() + H.bptr[k];
      const int64_t nb = H.bptr[k + 1] - H.bptr[k];
      for (int64_t p = an->leaf_off[k]; p < an->leaf_off[k + 1]; ++p) {
        if (an->constrained[p]) continue;
        int32_t q = an->rowptr[p];
        const int32_t qe = an->rowptr[p + 1];
        while (q < qe) {
          const int32_t kb = box_all[an->col[q]];
          int32_t r = q;
          bool any = false;
          while (r < qe && box_all[an->col[r]] == kb) {
            any |= !an->constrained[an->col[r]];
            ++r;
          }
          if (any) {
            const int32_t slot = (int32_t)(std::lower_bound(bc, bc + nb, kb) - bc);
            v.push_back({slot, (int32_t)p, q, r});
          }
          q = r;
        }
      }
      std::stable_sort(v.begin(), v.end(), [](const std::array<int32_t, 4>& x, const std::array<int32_t, 4>& y) {
        return x[0] < y[0];
      });
    });
    an->gal_ptr.assign(nblk + 1, 0);
    for (int64_t k = 0; k < H.nbox; ++k)
      for (auto& e : per[k]) an->gal_ptr[H.bptr[k] + e[0] + 1] += 1;
    for (int64_t b = 0; b < nblk; ++b) an->gal_ptr[b + 1] += an->gal_ptr[b];
    an->gal_ent.resize((size_t)an->gal_ptr[nblk] * 3);
    for (int64_t k = 0; k < H.nbox; ++k) {
      int64_t prev_slot = -1, w = 0;
      for (auto& e : per[k]) {
        if (e[0] != prev_slot) {
          prev_slot = e[0];
          w = an->gal_ptr[H.bptr[k] + e[0]];
        }
        an->gal_ent[w * 3 + 0] = e[1];
        an->gal_ent[w * 3 + 1] = e[2];
        an->gal_ent[w * 3 + 2] = e[3];
        ++w;
      }
    }
    // A1 is symmetric (Galerkin product of a symmetric A): only the blocks on and above the block diagonal are
    // formed, and the transpose of each off-diagonal one fills its mirror (K', K)
    an->gal_up.clear();
    an->gal_mir.clear();
    for (int64_t k = 0; k < H.nbox; ++k)
      for (int64_t b = H.bptr[k]; b < H.bptr[k + 1]; ++b) {
        const int32_t kp = H.bcol[b];
        if (kp < k) continue;
        int32_t m = -1;
        if (kp != k) {
          const int32_t* bc = H.bcol.data() + H.bptr[kp];
          const int32_t* be = H.bcol.data() + H.bptr[kp + 1];
          const int32_t* f = std::lower_bound(bc, be, (int32_t)k);
          if (f == be || *f != k)
            throw err(R3MG_ERR_NOT_SPD, "the operator's sparsity pattern is not symmetric (coarse block pattern)");
          m = (int32_t)(H.bptr[kp] + (f - bc));
        }
        an->gal_up.push_back((int32_t)b);
        an->gal_mir.push_back(m);
      }
  }
  for (int l = 2; l <= L; ++l) {
    HostLevel& P = an->lv[l - 1];
    HostLevel& H = an->lv[l];
    const int s = H.child_shift;
    std::vector<std::vector<int32_t>> rows(H.nbox);
    for (int64_t c = 0; c < P.nbox; ++c) {
      int64_t g = c >> s;
      for (int64_t q = P.bptr[c]; q < P.bptr[c + 1]; ++q) rows[g].push_back(P.bcol[q] >> s);
    }
    H.bptr.assign(H.nbox + 1, 0);
    for (int64_t g = 0; g < H.nbox; ++g) {
      std::sort(rows[g].begin(), rows[g].end());
      rows[g].erase(std::unique(rows[g].begin(), rows[g].end()), rows[g].end());
      H.bptr[g + 1] = H.bptr[g] + (int64_t)rows[g].size();
    }
    H.bcol.resize(H.bptr[H.nbox]);
    for (int64_t g = 0; g < H.nbox; ++g) std::copy(rows[g].begin(), rows[g].end(), H.bcol.begin() + H.bptr[g]);
  }
  for (int l = 1; l <= L; ++l)
    if (an->lv[l].bptr[an->lv[l].nbox] * (int64_t)B * B >= (int64_t(1) << 31) * 8)
      throw err(R3MG_ERR_OOM, "coarse operator too large");

  // injections between agglomerated levels: 1D factors M[a][child node i][parent node j]
  const int k1 = pc + 1;
  for (int l = 1; l < L; ++l) {
    HostLevel& C = an->lv[l];
    const HostLevel& G = an->lv[l + 1];
    const int s = G.child_shift;
    C.pt1d.assign(C.nbox * d * k1 * k1, 0.0);
    for (int64_t c = 0; c < C.nbox; ++c) {
      int64_t g = c >> s;
      for (int a = 0; a < d; ++a)
        for (int i = 0; i < k1; ++i) {
          double y = C.lo[c * d + a] + t[i] * (C.hi[c * d + a] - C.lo[c * d + a]);
          double xi = (pc == 0) ? 0.0 : (y - G.lo[g * d + a]) / (G.hi[g * d + a] - G.lo[g * d + a]);
          for (int j = 0; j < k1; ++j)
            C.pt1d[((c * d + a) * k1 + i) * k1 + j] = (pc == 0) ? 1.0 : lagrange(t, k1, j, xi);
        }
    }
  }
  encode_fine(*an);
  return an;
}

// Row blocks of the fine-level CSR row-block kernels, one set per geometry: consecutive rows, at most `rows` rows
// and `cap` - 3 nonzeros per block (the 16-byte loads start up to 3 entries before the block); a longer row forms
// a block of its own.
static void encode_csr_blocks(Analysis& an) {
  const int64_t n = an.n;
  for (int g = 0; g < kCsrGeoms; ++g) {
    const int cap = kStreamCapOf[g] - 3, rows = kStreamRowsOf[g];
    std::vector<int32_t>& rb = an.rb[g];
    rb.assign(1, 0);
    for (int64_t r = 0; r < n;) {
      int64_t r1 = r + 1;
      while (r1 < n && r1 - r < rows && (int64_t)an.rowptr[r1 + 1] - an.rowptr[r] <= cap) ++r1;
      rb.push_back((int32_t)r1);
      r = r1;
    }
  }
}

// Local-column row blocks over a CSR pattern: rows are taken greedily (within independent row segments) while
// the block stays within `rows` rows, `cap` nonzeros and `ucap` distinct columns; the
// distinct columns are listed in ascending order and every nonzero stores the position of its column in the
// list.  A single row beyond the limits forms a block of its own with its full column list (the kernel reads
// such a block through the CSR columns).  Positions take `ib` bytes; `pad` zero entries follow the last one.
static void encode_local_blocks(const int32_t* rowptr, const int32_t* col, int64_t n, int64_t ncol, int cap,
                                int rows, int ucap, int ib, int pad, LocalBlocks& out) {
  const int64_t nnz = rowptr[n];
  const int64_t nseg = std::max<int64_t>(1, std::min<int64_t>(256, n / 4096));
  struct Seg {
    std::vector<int32_t> ends, ucnt, ucol;
  };
  std::vector<Seg> segs((size_t)nseg);
  std::vector<uint8_t>& lidx = out.lidx;
  lidx.assign((size_t)(nnz + pad) * ib, 0);  // padding: the vector kernels' wide loads
  parallel_for(nseg, [&](int64_t sg) {
    static thread_local std::vector<uint8_t> mark;
    static thread_local std::vector<int32_t> pos;
    if ((int64_t)mark.size() < ncol) {
      mark.assign((size_t)ncol, 0);
      pos.assign((size_t)ncol, 0);
    }
    Seg& S = segs[(size_t)sg];
    const int64_t ra = sg * n / nseg, rz = (sg + 1) * n / nseg;
    std::vector<int32_t> uq;
    for (int64_t r = ra; r < rz;) {
      uq.clear();
      int64_t r1 = r, nz = 0;
      while (r1 < rz && r1 - r < rows) {
        const int32_t a = rowptr[r1], b = rowptr[r1 + 1];
        int64_t add = 0;
        for (int32_t e = a; e < b; ++e) add += mark[col[e]] ? 0 : 1;
        if (r1 > r && (nz + (b - a) > cap || (int64_t)uq.size() + add > ucap)) break;
        for (int32_t e = a; e < b; ++e)
          if (!mark[col[e]]) {
            mark[col[e]] = 1;
            uq.push_back(col[e]);
          }
        nz += b - a;
        ++r1;
      }
      std::sort(uq.begin(), uq.end());
      for (size_t i = 0; i < uq.size(); ++i) {
        pos[uq[i]] = (int32_t)i;
        mark[uq[i]] = 0;
      }
      if ((int64_t)uq.size() <= ucap)
        for (int32_t e = rowptr[r]; e < rowptr[r1]; ++e) {
          const int32_t li = pos[col[e]];
          if (ib == 1)
            lidx[(size_t)e] = (uint8_t)li;
          else
            std::memcpy(&lidx[(size_t)e * 2], &li, 2);  // little-endian low half
        }
      S.ends.push_back((int32_t)r1);
      S.ucnt.push_back((int32_t)uq.size());
      S.ucol.insert(S.ucol.end(), uq.begin(), uq.end());
      r = r1;
    }
  });
  out.rb.assign(1, 0);
  out.ubp.assign(1, 0);
  out.ucol.clear();
  for (const Seg& S : segs) {
    for (size_t k = 0; k < S.ends.size(); ++k) {
      out.rb.push_back(S.ends[k]);
      out.ubp.push_back(out.ubp.back() + S.ucnt[k]);
    }
    out.ucol.insert(out.ucol.end(), S.ucol.begin(), S.ucol.end());
  }
}

// the blocks of local geometry g (the 16-byte loads of the block kernels start up to 3 entries before a block)
static void encode_local_geom(const int32_t* rowptr, const int32_t* col, int64_t n, int g, LocalBlocks& out) {
  encode_local_blocks(rowptr, col, n, n, kLocalCap[g] - 3, kLocalRows[g], kLocalUcap[g], kLocalIdxBytes[g], kFinePad,
                      out);
}

void encode_mr_blocks(const Analysis& an, int cls, MrHost& out) {
  encode_local_blocks(an.rowptr.data(), an.col.data(), an.n, an.n, kMrCap[cls], kMrRows[cls], kMrUcap[cls], 2, kMrPad,
                      out.lb);
  const int64_t nrb = (int64_t)out.lb.rb.size() - 1;
  out.ord.assign((size_t)an.n, 0);
  parallel_for(nrb, [&](int64_t k) {
    const int32_t r0 = out.lb.rb[k], r1 = out.lb.rb[k + 1];
    for (int32_t r = r0; r < r1; ++r) out.ord[r] = r;
    std::stable_sort(out.ord.begin() + r0, out.ord.begin() + r1, [&](int32_t a, int32_t b) {
      return an.rowptr[a + 1] - an.rowptr[a] > an.rowptr[b + 1] - an.rowptr[b];
    });
  });
}

void encode_fine(Analysis& an) {
  encode_csr_blocks(an);
  for (int g = 0; g <= kLocalGeoms; ++g) encode_local_geom(an.rowptr.data(), an.col.data(), an.n, g, an.loc[g]);
  // agglomerated levels with narrow block rows (the 2D hierarchies): CSR row pointers and 1-byte local blocks
  const int L = an.nlevels() - 1;
  const int B = an.B;
  for (int l = 1; l < L; ++l) {
    HostLevel& H = an.lv[l];
    int64_t maxw = 0;
    for (int64_t K = 0; K < H.nbox; ++K) maxw = std::max<int64_t>(maxw, (H.bptr[K + 1] - H.bptr[K]) * B);
    const int64_t nnz = H.bptr[H.nbox] * (int64_t)B * B;
    if (maxw > kLocalUcap[0] || nnz >= (int64_t(1) << 31) - kFinePad) continue;
    H.rowptr.assign(H.n + 1, 0);
    std::vector<int32_t> col((size_t)nnz);
    parallel_for(H.nbox, [&](int64_t K) {
      const int64_t nb = H.bptr[K + 1] - H.bptr[K];
      const int64_t w = nb * B;
      for (int q = 0; q < B; ++q) {
        const int64_t r0 = (int64_t)B * B * H.bptr[K] + q * w;
        H.rowptr[K * B + q] = (int32_t)r0;
        for (int64_t j = 0; j < nb; ++j)
          for (int c = 0; c < B; ++c) col[(size_t)(r0 + j * B + c)] = (int32_t)(H.bcol[H.bptr[K] + j] * B + c);
      }
    });
    H.rowptr[H.n] = (int32_t)nnz;
    encode_local_geom(H.rowptr.data(), col.data(), H.n, 0, H.loc);
    // FP32 V-cycle: where the 2048-nonzero blocks need a second, mostly idle round of resident workgroups and
    // 3072-nonzero blocks fit in one, the level takes the larger blocks (the same row sums in the same order)
    if (an.opt.vcycle_fp32 && (int64_t)H.loc.rb.size() - 1 > kResidentBlocks) {
      LocalBlocks l4;
      encode_local_geom(H.rowptr.data(), col.data(), H.n, 4, l4);
      if ((int64_t)l4.rb.size() - 1 <= kResidentBlocks) {
        H.loc = std::move(l4);
        H.loc_geom = 4;
      }
    }
  }
}

}  // namespace r3mg
