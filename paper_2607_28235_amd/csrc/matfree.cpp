// Host set-up of the matrix-free fine operator: cell connectivity in internal numbering, geometric factors at
// the Gauss points of each multilinear cell, and the per-DoF incidence lists that the deterministic per-DoF sum
// reads.  The operator it describes is the Q_p Laplace stiffness matrix (optionally scaled by a coefficient per
// cell) assembled with Gauss quadrature of p + 1 points per axis, the discretisation of the paper's experiments
// (Section 6); the caller's CSR matrix remains the definition, and the device set-up checks the two against
// each other before the operator is used.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "r3mg_internal.h"

namespace r3mg {

namespace {

Error invalid(const std::string& m) { return Error{R3MG_ERR_INVALID, m}; }

// Gauss-Legendre points and weights on [0, 1], k = 2..4 (closed forms)
void gauss_01(int k, double* g, double* w) {
  double x[4] = {0, 0, 0, 0}, wt[4] = {0, 0, 0, 0};
  switch (k) {
    case 2: {
      const double a = 1.0 / std::sqrt(3.0);
      x[0] = -a; x[1] = a;
      wt[0] = wt[1] = 1.0;
      break;
    }
    case 3: {
      const double a = std::sqrt(0.6);
      x[0] = -a; x[1] = 0.0; x[2] = a;
      wt[0] = wt[2] = 5.0 / 9.0;
      wt[1] = 8.0 / 9.0;
      break;
    }
    default: {
      const double r = 2.0 / 7.0 * std::sqrt(6.0 / 5.0);
      const double a = std::sqrt(3.0 / 7.0 - r), b = std::sqrt(3.0 / 7.0 + r);
      const double wa = (18.0 + std::sqrt(30.0)) / 36.0, wb = (18.0 - std::sqrt(30.0)) / 36.0;
      x[0] = -b; x[1] = -a; x[2] = a; x[3] = b;
      wt[0] = wb; wt[1] = wa; wt[2] = wa; wt[3] = wb;
    }
  }
  for (int q = 0; q < k; ++q) {
    g[q] = 0.5 * (1.0 + x[q]);
    w[q] = 0.5 * wt[q];
  }
}

// Lagrange basis on nodes t[0..k) and its derivative at s
void lagrange(int k, const double* t, double s, double* l, double* dl) {
  for (int i = 0; i < k; ++i) {
    double v = 1.0, dv = 0.0;
    for (int m = 0; m < k; ++m) {
      if (m == i) continue;
      const double f = (s - t[m]) / (t[i] - t[m]);
      dv = dv * f + v / (t[i] - t[m]);
      v *= f;
    }
    l[i] = v;
    dl[i] = dv;
  }
}

}  // namespace

MatFreeHost build_matrix_free(const Analysis& an, const int32_t* cells, int64_t ncells, int p, const double* kappa) {
  const int d = an.d;
  if (p < 1 || p > 3) throw invalid("matrix-free operator: degree p must be 1, 2 or 3");
  if (ncells < 1 || ncells >= (int64_t(1) << 31)) throw invalid("matrix-free operator: bad cell count");
  MatFreeHost m;
  m.d = d;
  m.p = p;
  m.k = p + 1;
  m.nloc = d == 2 ? m.k * m.k : m.k * m.k * m.k;
  m.nlocp = (m.nloc + 3) / 4 * 4;
  m.ncomp = d == 2 ? 3 : 6;
  m.nq = m.nloc;
  m.ncells = ncells;
  if (ncells * m.nlocp >= (int64_t(1) << 31)) throw invalid("matrix-free operator: too many cell-local entries");
  const int64_t n = an.n;
  const int k = m.k, nl = m.nloc;
  for (int64_t e = 0; e < ncells; ++e)
    for (int a = 0; a < nl; ++a) {
      const int32_t j = cells[e * nl + a];
      if (j < 0 || j >= n) throw invalid("matrix-free operator: cell index out of range");
    }
  if (kappa)
    for (int64_t e = 0; e < ncells; ++e)
      if (!std::isfinite(kappa[e]) || kappa[e] <= 0.0) throw invalid("matrix-free operator: kappa must be positive");

  // 1D tables
  double t[4], g[4], w[4];
  box_nodes_1d(p, t);
  gauss_01(k, g, w);
  for (int q = 0; q < 4; ++q) {
    m.W[q] = q < k ? w[q] : 0.0;
    m.X[q] = q < k ? g[q] : 0.0;
    for (int i = 0; i < 4; ++i) m.B[q][i] = m.G[q][i] = 0.0;
  }
  for (int q = 0; q < k; ++q) lagrange(k, t, g[q], m.B[q], m.G[q]);

  // cells in internal numbering, ordered by their smallest internal DoF (cells of one box become neighbours)
  std::vector<int32_t> key(ncells);
  for (int64_t e = 0; e < ncells; ++e) {
    int32_t mn = INT32_MAX;
    for (int a = 0; a < nl; ++a) mn = std::min(mn, an.iperm[cells[e * nl + a]]);
    key[e] = mn;
  }
  std::vector<int64_t> ord(ncells);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return key[a] < key[b]; });

  // every unconstrained DoF must lie in a cell
  std::vector<int32_t> cnt(n, 0);
  for (int64_t e = 0; e < ncells; ++e)
    for (int a = 0; a < nl; ++a) {
      const int32_t i = an.iperm[cells[e * nl + a]];
      if (!an.constrained[i]) ++cnt[i];
    }
  for (int64_t i = 0; i < n; ++i)
    if (!an.constrained[i] && cnt[i] == 0) throw invalid("matrix-free operator: an unconstrained DoF is in no cell");

  // geometry at the Gauss points: J = sum_v X_v (grad psi_v)^T over the 2^d corner nodes.  Affine cells keep
  // C = kappa |det J| J^-1 J^-T; multilinear cells keep the coefficients c_S of x(xi) = sum_S c_S prod_{a in S}
  // xi_a for the non-empty subsets S (c_S = sum over corners v inside S of (-1)^{|S| - |v|} X_v) and kappa.
  const int nv = 1 << d;
  const int ncoef = d == 2 ? 7 : 22;
  std::vector<double> Jq((size_t)m.nq * 9);
  std::vector<double> geo_c((size_t)ncells * ncoef), geo_a((size_t)ncells * m.ncomp);
  bool affine = true;
  for (int64_t s = 0; s < ncells; ++s) {
    const int64_t e = ord[s];
    double X[8][3];
    for (int v = 0; v < nv; ++v) {
      int a = 0, stride = 1;
      for (int ax = 0; ax < d; ++ax) {
        a += ((v >> ax) & 1) * p * stride;
        stride *= k;
      }
      const int32_t i = an.iperm[cells[e * nl + a]];
      for (int ax = 0; ax < d; ++ax) X[v][ax] = an.coords_int[(int64_t)i * d + ax];
    }
    const double kap = kappa ? kappa[e] : 1.0;
    {
      // subsets in the order 1, 2, (3,) 12, (13, 23, 123) of the axes, as bit masks over the corner index bits
      static const int sub2[3] = {1, 2, 3};
      static const int sub3[7] = {1, 2, 4, 3, 5, 6, 7};
      const int* sub = d == 2 ? sub2 : sub3;
      const int nsub = d == 2 ? 3 : 7;
      for (int t2 = 0; t2 < nsub; ++t2) {
        const int S = sub[t2];
        for (int ax = 0; ax < d; ++ax) {
          double acc = 0.0;
          for (int v = 0; v < nv; ++v) {
            if ((v & ~S) != 0) continue;
            const int sgn = (__builtin_popcount(S) - __builtin_popcount(v)) & 1 ? -1 : 1;
            acc += sgn * X[v][ax];
          }
          geo_c[((size_t)t2 * d + ax) * ncells + s] = acc;
        }
      }
      geo_c[(size_t)(ncoef - 1) * ncells + s] = kap;
    }
    double jmax = 0.0, jdiff = 0.0;
    for (int q = 0; q < m.nq; ++q) {
      double xi[3] = {g[q % k], g[(q / k) % k], d == 3 ? g[q / (k * k)] : 0.0};
      double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // J[i][c] = dx_i / dxi_c
      for (int v = 0; v < nv; ++v)
        for (int c = 0; c < d; ++c) {
          double dp = 1.0;
          for (int ax = 0; ax < d; ++ax) {
            const int bit = (v >> ax) & 1;
            if (ax == c)
              dp *= bit ? 1.0 : -1.0;
            else
              dp *= bit ? xi[ax] : 1.0 - xi[ax];
          }
          for (int i = 0; i < d; ++i) J[i][c] += X[v][i] * dp;
        }
      double inv[3][3], det;
      if (d == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        inv[0][0] = J[1][1] / det; inv[0][1] = -J[0][1] / det;
        inv[1][0] = -J[1][0] / det; inv[1][1] = J[0][0] / det;
      } else {
        det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
              J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
        inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
        inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
        inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
      }
      if (!(det > 0.0)) throw invalid("matrix-free operator: inverted or degenerate cell");
      for (int i = 0; i < d; ++i)
        for (int c = 0; c < d; ++c) {
          if (q == 0) Jq[i * 3 + c] = J[i][c];
          jmax = std::max(jmax, std::fabs(J[i][c]));
          jdiff = std::max(jdiff, std::fabs(J[i][c] - Jq[i * 3 + c]));
        }
      // C = kappa |det J| J^-1 J^-T (upper triangle, row by row); C_q adds the Gauss weight
      int c = 0;
      for (int r = 0; r < d; ++r)
        for (int s2 = r; s2 < d; ++s2) {
          double acc = 0.0;
          for (int i = 0; i < d; ++i) acc += inv[r][i] * inv[s2][i];
          if (q == 0) geo_a[(size_t)c * ncells + s] = kap * det * acc;
          ++c;
        }
    }
    if (jdiff > 1e-12 * jmax) affine = false;
  }
  m.affine = affine;
  m.geo = affine ? std::move(geo_a) : std::move(geo_c);

  // connectivity (constrained DoFs -> -1) and incidence lists in ascending (cell, node) order
  m.conn.assign((size_t)ncells * m.nlocp, -1);
  m.inc_ptr.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) m.inc_ptr[i + 1] = m.inc_ptr[i] + cnt[i];
  m.inc.resize(m.inc_ptr[n]);
  std::vector<int32_t> fill(m.inc_ptr.begin(), m.inc_ptr.end() - 1);
  for (int64_t s = 0; s < ncells; ++s) {
    const int64_t e = ord[s];
    for (int a = 0; a < nl; ++a) {
      const int32_t i = an.iperm[cells[e * nl + a]];
      if (an.constrained[i]) continue;
      m.conn[(size_t)s * m.nlocp + a] = i;
      m.inc[fill[i]++] = (int32_t)(s * m.nlocp + a);
    }
  }
  // constrained rows: their diagonal entry of the caller's matrix
  m.cd.assign(n, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    if (!an.constrained[i]) continue;
    for (int32_t q = an.rowptr[i]; q < an.rowptr[i + 1]; ++q)
      if (an.col[q] == i) m.cd[i] = an.val[q];
  }
  return m;
}

}  // namespace r3mg
