// C ABI of the R3MG-C library: argument checking, error mapping, exports and the kappa assembler.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "kernels.h"
#include "r3mg_internal.h"

namespace r3mg {
static thread_local std::string g_last_error;
void set_last_error(const std::string& s) { g_last_error = s; }
}  // namespace r3mg

using namespace r3mg;

namespace {

template <typename F>
r3mg_status guard(F&& f) {
  try {
    r3mg_status s = f();
    if (s == R3MG_OK) g_last_error.clear();
    return s;
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return R3MG_ERR_OOM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return R3MG_ERR_HIP;
  }
}

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

void require_factored(r3mg_handle h) {
  if (!h) throw Error{R3MG_ERR_INVALID, "null handle"};
  if (!h->impl.factored) throw Error{R3MG_ERR_INVALID, "handle is analysed but not factored"};
}

inline double lag(const double* t, int k, int j, double s) {
  double v = 1.0;
  for (int m = 0; m < k; ++m)
    if (m != j) v *= (s - t[m]) / (t[j] - t[m]);
  return v;
}

}  // namespace

struct r3mg_assembler_ {
  r3mg_handle h = nullptr;
  int nloc = 0;
  int64_t ncells = 0;
  DBuf<int64_t> slot_ptr, contrib;
  DBuf<unsigned char> diag_one;
};

extern "C" {

const char* r3mg_last_error(void) { return g_last_error.c_str(); }

void r3mg_default_options(r3mg_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->dim = 3;
  o->coarse_degree = 1;
  o->leaf_size = 64;
  o->max_levels = 0;
  o->max_coarse_dofs = 2000;
  o->skip_leaf_level = 0;
  o->cheb_degree = 3;
  o->pre_steps = 2;
  o->post_steps = 2;
  o->lanczos_steps = 10;
  o->cheb_boost = 1.1;
  o->cheb_ratio = 30.0;
  o->vcycle_fp32 = 0;
  o->use_graph = 1;
  o->fine_kernel = -1;
  o->multi_rhs_kernel = -1;
  o->matrix_cache = -1;
  o->tune_cache = 1;
}

r3mg_status r3mg_analyze(const double* coords, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                         const double* vals, const r3mg_options* opt, r3mg_handle* out) {
  return guard([&] {
    if (!out || !opt) throw Error{R3MG_ERR_INVALID, "null argument"};
    *out = nullptr;
    auto an = analyze(coords, n, row_ptr, col_idx, vals, *opt);
    r3mg_handle h = new r3mg_handle_();
    h->impl.an = std::move(an);
    *out = h;
    return R3MG_OK;
  });
}

r3mg_status r3mg_analyze_cells(const double* coords, int64_t n, const int32_t* cells, int64_t ncells, int nloc,
                               const int64_t* row_ptr, const int32_t* col_idx, const double* vals,
                               const r3mg_options* opt, r3mg_handle* out) {
  return guard([&] {
    if (!out || !opt || !cells) throw Error{R3MG_ERR_INVALID, "null argument"};
    *out = nullptr;
    auto an = analyze(coords, n, row_ptr, col_idx, vals, *opt, cells, ncells, nloc);
    r3mg_handle h = new r3mg_handle_();
    h->impl.an = std::move(an);
    *out = h;
    return R3MG_OK;
  });
}

r3mg_status r3mg_factor(r3mg_handle h, void* stream) {
  return guard([&] {
    if (!h) throw Error{R3MG_ERR_INVALID, "null handle"};
    h->impl.factored = false;
    h->impl.dev.reset();
    device_setup(h->impl, S(stream));
    h->impl.factored = true;
    return R3MG_OK;
  });
}

r3mg_status r3mg_setup(const double* coords, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                       const double* vals, const r3mg_options* opt, void* stream, r3mg_handle* out) {
  if (!out) return R3MG_ERR_INVALID;
  *out = nullptr;
  r3mg_handle h = nullptr;
  r3mg_status s = r3mg_analyze(coords, n, row_ptr, col_idx, vals, opt, &h);
  if (s != R3MG_OK) return s;
  s = r3mg_factor(h, stream);
  if (s != R3MG_OK) {
    std::string keep = g_last_error;
    r3mg_free(h);
    set_last_error(keep);
    return s;
  }
  *out = h;
  return R3MG_OK;
}

r3mg_status r3mg_update_values(r3mg_handle h, const double* vals_dev, void* stream) {
  return guard([&] {
    require_factored(h);
    if (!vals_dev) throw Error{R3MG_ERR_INVALID, "null values"};
    h->impl.factored = false;
    update_values(h->impl, vals_dev, S(stream));
    h->impl.factored = true;
    return R3MG_OK;
  });
}

r3mg_status r3mg_set_matrix_free(r3mg_handle h, const int32_t* cells, int64_t ncells, int degree, const double* kappa,
                                 void* stream) {
  return guard([&] {
    require_factored(h);
    if (!cells) {
      detach_matrix_free(h->impl);
      return R3MG_OK;
    }
    MatFreeHost m = build_matrix_free(*h->impl.an, cells, ncells, degree, kappa);
    attach_matrix_free(h->impl, std::move(m), S(stream));
    return R3MG_OK;
  });
}

r3mg_status r3mg_vcycle(r3mg_handle h, const double* r_dev, double* z_dev, int nrhs, void* stream) {
  return guard([&] {
    require_factored(h);
    if (!r_dev || !z_dev || nrhs < 1) throw Error{R3MG_ERR_INVALID, "bad vcycle arguments"};
    vcycle_api(h->impl, r_dev, z_dev, nrhs, S(stream));
    return R3MG_OK;
  });
}

r3mg_status r3mg_vcycle_noalloc(r3mg_handle h, const double* r_dev, double* z_dev, int nrhs, void* stream) {
  return guard([&] {
    require_factored(h);
    if (!r_dev || !z_dev) throw Error{R3MG_ERR_INVALID, "bad vcycle arguments"};
    vcycle_noalloc(h->impl, r_dev, z_dev, nrhs, S(stream));
    return R3MG_OK;
  });
}

r3mg_status r3mg_level_apply(r3mg_handle h, int level, const double* x_dev, double* y_dev, void* stream) {
  return guard([&] {
    require_factored(h);
    const int L = h->impl.an->nlevels() - 1;
    if (!x_dev || !y_dev || level < -1 || level > L) throw Error{R3MG_ERR_INVALID, "bad level_apply arguments"};
    level_apply(h->impl, level, x_dev, y_dev, S(stream));
    return R3MG_OK;
  });
}

r3mg_status r3mg_pcg_solve(r3mg_handle h, const double* b_dev, double* x_dev, int nrhs, double rtol, int maxit,
                           void* stream, int* iters, double* relres) {
  return r3mg_pcg_solve_ex(h, b_dev, x_dev, nrhs, rtol, 0.0, maxit, stream, iters, relres, nullptr);
}

r3mg_status r3mg_pcg_solve_ex(r3mg_handle h, const double* b_dev, double* x_dev, int nrhs, double rtol, double atol,
                              int maxit, void* stream, int* iters, double* relres, double* cond) {
  return guard([&] {
    require_factored(h);
    if (!b_dev || !x_dev || nrhs < 1 || !(rtol >= 0.0) || !(atol >= 0.0) || maxit < 0)
      throw Error{R3MG_ERR_INVALID, "bad pcg arguments"};
    return pcg_solve(h->impl, b_dev, x_dev, nrhs, rtol, atol, maxit, S(stream), cond, iters, relres);
  });
}

r3mg_status r3mg_pcg_solve_group(int count, r3mg_handle* hs, const double* const* b, double* const* x, double rtol,
                                 int maxit, void* stream, int* iters, double* relres) {
  return guard([&] {
    if (count < 1 || !hs || !b || !x || !(rtol >= 0.0) || maxit < 0) throw Error{R3MG_ERR_INVALID, "bad group arguments"};
    std::vector<HandleImpl*> v(count);
    for (int k = 0; k < count; ++k) {
      require_factored(hs[k]);
      for (int j = 0; j < k; ++j)
        if (hs[j] == hs[k]) throw Error{R3MG_ERR_INVALID, "a handle appears twice in the group"};
      v[k] = &hs[k]->impl;
      if (!b[k] || !x[k]) throw Error{R3MG_ERR_INVALID, "null vector in group"};
    }
    return pcg_group(count, v.data(), b, x, rtol, maxit, S(stream), iters, relres);
  });
}

r3mg_status r3mg_pcg_history(r3mg_handle h, int col, double* rr, int cap, int* count) {
  return guard([&] {
    require_factored(h);
    if (!count || col < 0 || col >= kMaxNR || cap < 0) throw Error{R3MG_ERR_INVALID, "bad history arguments"};
    *count = residual_history(h->impl, col, rr, cap);
    return R3MG_OK;
  });
}

r3mg_status r3mg_info(r3mg_handle h, r3mg_level_info* levels, int* nlevels) {
  return guard([&] {
    if (!h || !nlevels) throw Error{R3MG_ERR_INVALID, "null argument"};
    const Analysis& an = *h->impl.an;
    const int nl = an.nlevels();
    if (levels) {
      if (*nlevels < nl) throw Error{R3MG_ERR_INVALID, "levels array too small"};
      for (int l = 0; l < nl; ++l) {
        r3mg_level_info& I = levels[l];
        std::memset(&I, 0, sizeof(I));
        if (l == 0) {
          I.n = an.n;
          I.nnz = an.nnz;
        } else {
          const HostLevel& H = an.lv[l];
          I.n = H.n;
          I.nnz = H.bptr[H.nbox] * (int64_t)an.B * an.B;
          I.nboxes = H.nbox;
          I.max_box_extent = H.max_extent;
        }
        if (h->impl.factored) {
          const DevLevel& D = h->impl.dev->lv[l];
          std::string kn;
          if (l < nl - 1) {
            I.lambda_hi = D.lam_hi;
            I.lambda_lo = D.lam_lo;
            I.bytes_per_apply = D.bytes_apply;
            kn = level_kernel_name(an, D, l, an.opt.vcycle_fp32 ? 4 : 8);
          } else {
            I.bytes_per_apply = (double)D.n * D.n * 8.0;
            kn = "dense";
          }
          std::snprintf(I.kernel, sizeof(I.kernel), "%s", kn.c_str());
        }
      }
    }
    *nlevels = nl;
    return R3MG_OK;
  });
}

r3mg_status r3mg_export_partition(r3mg_handle h, int level, int32_t* owner_box, double* box_lohi) {
  return guard([&] {
    if (!h) throw Error{R3MG_ERR_INVALID, "null handle"};
    const Analysis& an = *h->impl.an;
    if (level < 1 || level >= an.nlevels()) throw Error{R3MG_ERR_INVALID, "level out of range"};
    const HostLevel& H = an.lv[level];
    const int shift = an.depths[0] - an.depths[level - 1];
    if (owner_box) {
      const int64_t nb1 = (int64_t)an.leaf_off.size() - 1;
      for (int64_t k = 0; k < nb1; ++k)
        for (int64_t p = an.leaf_off[k]; p < an.leaf_off[k + 1]; ++p) owner_box[an.order[p]] = (int32_t)(k >> shift);
    }
    if (box_lohi) {
      const int d = an.d;
      for (int64_t k = 0; k < H.nbox; ++k)
        for (int a = 0; a < d; ++a) {
          box_lohi[k * 2 * d + a] = H.lo[k * d + a];
          box_lohi[k * 2 * d + d + a] = H.hi[k * d + a];
        }
    }
    return R3MG_OK;
  });
}

r3mg_status r3mg_export_P(r3mg_handle h, int level, int64_t* row_ptr, int32_t* col, double* val, int64_t* nrows,
                          int64_t* nnz) {
  return guard([&] {
    if (!h) throw Error{R3MG_ERR_INVALID, "null handle"};
    const Analysis& an = *h->impl.an;
    const int L = an.nlevels() - 1;
    if (level < 0 || level >= L) throw Error{R3MG_ERR_INVALID, "level out of range"};
    const int d = an.d, pc = an.pc, B = an.B, k1 = pc + 1;
    double t[4];
    box_nodes_1d(pc, t);
    if (level == 0) {
      int64_t nfree = 0;
      for (int64_t i = 0; i < an.n; ++i) nfree += an.constrained_user[i] ? 0 : 1;
      if (nrows) *nrows = an.n;
      if (nnz) *nnz = nfree * B;
      if (!row_ptr) return R3MG_OK;
      row_ptr[0] = 0;
      for (int64_t i = 0; i < an.n; ++i) row_ptr[i + 1] = row_ptr[i] + (an.constrained_user[i] ? 0 : B);
      for (int64_t i = 0; i < an.n; ++i) {
        if (an.constrained_user[i]) continue;
        const int64_t p = an.iperm[i];
        const int32_t K = an.owner[p];
        double l1[3][4];
        for (int a = 0; a < d; ++a)
          for (int j = 0; j < k1; ++j) l1[a][j] = (pc == 0) ? 1.0 : lag(t, k1, j, an.xi[p * d + a]);
        for (int q = 0; q < B; ++q) {
          double v = 1.0;
          int qq = q;
          for (int a = 0; a < d; ++a) {
            v *= l1[a][qq % k1];
            qq /= k1;
          }
          col[row_ptr[i] + q] = K * B + q;
          val[row_ptr[i] + q] = v;
        }
      }
      return R3MG_OK;
    }
    const HostLevel& C = an.lv[level];
    const int s = an.lv[level + 1].child_shift;
    if (nrows) *nrows = C.n;
    if (nnz) *nnz = C.n * B;
    if (!row_ptr) return R3MG_OK;
    for (int64_t r = 0; r <= C.n; ++r) row_ptr[r] = r * B;
    for (int64_t c = 0; c < C.nbox; ++c) {
      const int64_t g = c >> s;
      const double* M = C.pt1d.data() + c * d * k1 * k1;
      for (int qc = 0; qc < B; ++qc)
        for (int q = 0; q < B; ++q) {
          double v = 1.0;
          int a1 = qc, a2 = q;
          for (int a = 0; a < d; ++a) {
            v *= M[(a * k1 + a1 % k1) * k1 + a2 % k1];
            a1 /= k1;
            a2 /= k1;
          }
          const int64_t o = (c * B + qc) * B + q;
          col[o] = (int32_t)(g * B + q);
          val[o] = v;
        }
    }
    return R3MG_OK;
  });
}

r3mg_status r3mg_export_level(r3mg_handle h, int level, int64_t* row_ptr, int32_t* col, double* val,
                              int64_t* nrows, int64_t* nnz) {
  return guard([&] {
    require_factored(h);
    const Analysis& an = *h->impl.an;
    if (level < 1 || level >= an.nlevels()) throw Error{R3MG_ERR_INVALID, "level out of range"};
    const HostLevel& H = an.lv[level];
    const int B = an.B;
    const int64_t tot = H.bptr[H.nbox] * (int64_t)B * B;
    if (nrows) *nrows = H.n;
    if (nnz) *nnz = tot;
    if (!row_ptr) return R3MG_OK;
    std::vector<double> v(tot);
    const DevLevel& D = h->impl.dev->lv[level];
    R3MG_HIP_CHECK(hipMemcpy(v.data(), D.val64.p, tot * sizeof(double), hipMemcpyDeviceToHost));
    row_ptr[0] = 0;
    for (int64_t K = 0; K < H.nbox; ++K) {
      const int64_t j0 = H.bptr[K], nb = H.bptr[K + 1] - j0;
      for (int q = 0; q < B; ++q) {
        const int64_t r = K * B + q;
        const int64_t base = (int64_t)B * B * j0 + (int64_t)q * nb * B;
        row_ptr[r + 1] = row_ptr[r] + nb * B;
        for (int64_t p = 0; p < nb * B; ++p) {
          col[row_ptr[r] + p] = (int32_t)(H.bcol[j0 + p / B] * B + p % B);
          val[row_ptr[r] + p] = v[base + p];
        }
      }
    }
    return R3MG_OK;
  });
}

r3mg_status r3mg_time_smoother_kernel_nrhs(r3mg_handle h, int level, int nrhs, int reps, int64_t flush_bytes,
                                           void* stream, double* ms_per_launch, double* bytes_per_launch) {
  return guard([&] {
    require_factored(h);
    const int L = h->impl.an->nlevels() - 1;
    if (level < 0 || level >= L || reps < 1 || flush_bytes < 0 || !ms_per_launch || !bytes_per_launch)
      throw Error{R3MG_ERR_INVALID, "bad timing arguments"};
    if (nrhs < 1 || nrhs > 16 || (nrhs & (nrhs - 1)) != 0)
      throw Error{R3MG_ERR_INVALID, "nrhs must be 1, 2, 4, 8 or 16"};
    time_smoother_kernel(h->impl, level, nrhs, reps, flush_bytes, S(stream), ms_per_launch, bytes_per_launch);
    return R3MG_OK;
  });
}

r3mg_status r3mg_time_smoother_kernel(r3mg_handle h, int level, int reps, int64_t flush_bytes, void* stream,
                                      double* ms_per_launch, double* bytes_per_launch) {
  return r3mg_time_smoother_kernel_nrhs(h, level, 1, reps, flush_bytes, stream, ms_per_launch, bytes_per_launch);
}

r3mg_status r3mg_cell_grad(r3mg_handle h, const int32_t* cells_dev, int nloc, const double* Ke_dev, int64_t ke_stride,
                           const double* u_dev, const double* lam_dev, double* g_dev, int64_t ncells, void* stream) {
  return guard([&] {
    require_factored(h);
    if (!cells_dev || !Ke_dev || !u_dev || !lam_dev || !g_dev || nloc < 1 || ncells < 0 || ke_stride < 0)
      throw Error{R3MG_ERR_INVALID, "bad cell_grad arguments"};
    HandleImpl& H = h->impl;
    if (!H.cons_user_dev.p) H.cons_user_dev.upload(H.an->constrained_user, S(stream));
    launch_cell_grad(ncells, nloc, cells_dev, Ke_dev, ke_stride, u_dev, lam_dev, H.cons_user_dev.p, g_dev,
                     S(stream));
    return R3MG_OK;
  });
}

r3mg_status r3mg_assembler_create(r3mg_handle h, const int32_t* cells, int nloc, int64_t ncells,
                                  r3mg_assembler* out) {
  return guard([&] {
    if (!h || !cells || !out || nloc < 1 || ncells < 0) throw Error{R3MG_ERR_INVALID, "bad assembler arguments"};
    *out = nullptr;
    const Analysis& an = *h->impl.an;
    const int64_t n = an.n, nnz = an.nnz;
    const std::vector<int64_t>& rp = an.user_rowptr;
    const std::vector<int32_t>& cl = an.user_col;
    const std::vector<uint8_t>& cons = an.constrained_user;
    std::vector<int64_t> cnt(nnz + 1, 0);
    std::vector<int64_t> slot_of((size_t)ncells * nloc * nloc, -1);
    for (int64_t e = 0; e < ncells; ++e)
      for (int a = 0; a < nloc; ++a) {
        const int32_t i = cells[e * nloc + a];
        if (i < 0 || i >= n) throw Error{R3MG_ERR_INVALID, "cell index out of range"};
        if (cons[i]) continue;
        for (int b = 0; b < nloc; ++b) {
          const int32_t j = cells[e * nloc + b];
          if (j < 0 || j >= n) throw Error{R3MG_ERR_INVALID, "cell index out of range"};
          if (cons[j]) continue;
          auto it = std::lower_bound(cl.begin() + rp[i], cl.begin() + rp[i + 1], j);
          if (it == cl.begin() + rp[i + 1] || *it != j) throw Error{R3MG_ERR_INVALID, "pattern misses a coupled pair"};
          const int64_t sidx = it - cl.begin();
          slot_of[(e * nloc + a) * nloc + b] = sidx;
          cnt[sidx + 1] += 1;
        }
      }
    for (int64_t s2 = 0; s2 < nnz; ++s2) cnt[s2 + 1] += cnt[s2];
    std::vector<int64_t> contrib(cnt[nnz]);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    const int64_t nl2 = (int64_t)nloc * nloc;
    for (int64_t e = 0; e < ncells; ++e)
      for (int64_t pr = 0; pr < nl2; ++pr) {
        const int64_t sidx = slot_of[e * nl2 + pr];
        if (sidx >= 0) contrib[fill[sidx]++] = e * nl2 + pr;
      }
    std::vector<unsigned char> d1(nnz, 0);
    for (int64_t i = 0; i < n; ++i)
      if (cons[i])
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
          if (cl[p] == i) d1[p] = 1;
    auto* A = new r3mg_assembler_();
    try {
      A->h = h;
      A->nloc = nloc;
      A->ncells = ncells;
      A->slot_ptr.upload(cnt, nullptr);
      A->contrib.upload(contrib, nullptr);
      A->diag_one.upload(d1, nullptr);
      R3MG_HIP_CHECK(hipStreamSynchronize(nullptr));
    } catch (...) {
      delete A;
      throw;
    }
    *out = A;
    return R3MG_OK;
  });
}

r3mg_status r3mg_assemble(r3mg_assembler a, const double* kappa_dev, const double* Ke_dev, int64_t ke_stride,
                          double* vals_dev, void* stream) {
  return guard([&] {
    if (!a || !kappa_dev || !Ke_dev || !vals_dev || ke_stride < 0) throw Error{R3MG_ERR_INVALID, "bad assemble arguments"};
    launch_assemble(a->h->impl.an->nnz, a->slot_ptr.p, a->contrib.p, kappa_dev, Ke_dev, ke_stride, a->nloc,
                    a->diag_one.p, vals_dev, S(stream));
    return R3MG_OK;
  });
}

void r3mg_assembler_free(r3mg_assembler a) { delete a; }

r3mg_status r3mg_rtree(const double* coords, int64_t n, int dim, int leaf, int* depth, int32_t* order) {
  return guard([&] {
    if (!coords || n < 1 || n >= (int64_t(1) << 31) || (dim != 2 && dim != 3) || leaf < 1)
      throw Error{R3MG_ERR_INVALID, "bad rtree arguments"};
    for (int64_t i = 0; i < n * dim; ++i)
      if (!std::isfinite(coords[i])) throw Error{R3MG_ERR_INVALID, "non-finite coordinate"};
    int t = 0;
    std::vector<int32_t> ord;
    std::vector<std::vector<int64_t>> offs;
    bisection_rtree(coords, n, dim, leaf, t, ord, offs);
    if (depth) *depth = t;
    if (order) std::copy(ord.begin(), ord.end(), order);
    return R3MG_OK;
  });
}

void r3mg_free(r3mg_handle h) {
  if (!h) return;
  delete h;
}

const char* r3mg_status_string(r3mg_status s) {
  switch (s) {
    case R3MG_OK: return "ok";
    case R3MG_NOT_CONVERGED: return "not converged";
    case R3MG_ERR_INVALID: return "invalid argument";
    case R3MG_ERR_NOT_UNISOLVENT: return "agglomerate not unisolvent";
    case R3MG_ERR_DEGENERATE_BOX: return "degenerate box";
    case R3MG_ERR_NOT_SPD: return "operator not SPD";
    case R3MG_ERR_OOM: return "out of memory";
    case R3MG_ERR_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

}  // extern "C"
