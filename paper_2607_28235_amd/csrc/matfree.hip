// Matrix-free application of the fine-level operator for Q_p Lagrange elements on multilinear cells (the
// Poisson stiffness matrix of the paper's experiments, Section 6, assembled with Gauss quadrature of p + 1
// points per axis).  The operator is A = D (sum_e K_e) D + diag(cd): D removes the constrained DoFs (their
// columns and rows) and cd holds the diagonal of the constrained rows.
//
// Two launches, both deterministic (no floating-point atomics):
//   k_mf_cell    one thread per cell: gather u_e, y_e = K_e u_e by sum factorisation (one Gauss-point slice at
//                a time along the last axis, which bounds the registers), store y_e to the cell-local buffer Y;
//   k_mf_gather  one thread per DoF: t_i = sum of its cell-local outputs in ascending (cell, node) order, then
//                the smoother epilogue of the CSR level kernels.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hip_util.h"
#include "kernels.h"

namespace r3mg {

namespace {

using hiputil::check_launch;
using hiputil::xcd_block;
using hiputil::xcd_grid;

// geometry entry c of Gauss point q (pre-scaled by the Gauss weight on general cells)
template <typename T, int NC, bool AFF>
__device__ inline T geo_at(const T* __restrict__ geo, const T* ca, int ncells, int e, int q, int c, T w) {
  if constexpr (AFF)
    return w * ca[c];
  else
    return geo[(int64_t)(q * NC + c) * ncells + e];
}

template <typename T, int D, int K, bool AFF>
__global__ __launch_bounds__(256) void k_mf_cell(int ncells, int nlocp, const int* __restrict__ conn,
                                                 const T* __restrict__ geo, MfTables<T> tb,
                                                 const T* __restrict__ u, T* __restrict__ Y,
                                                 const int* __restrict__ skip, int nlog) {
  if (skip && *skip) return;
  const int lb = xcd_block(nlog);
  if (lb < 0) return;
  const int e = lb * 256 + (int)threadIdx.x;
  if (e >= ncells) return;
  constexpr int NL = D == 2 ? K * K : K * K * K;
  constexpr int NP = (NL + 3) / 4 * 4;
  constexpr int NC = D == 2 ? 3 : 6;
  // gather u_e (constrained DoFs and padding read as zero)
  T ue[NL];
  const int* cp = conn + (int64_t)e * nlocp;
#pragma unroll
  for (int a4 = 0; a4 < NP / 4; ++a4) {
    const int4 c4 = *reinterpret_cast<const int4*>(cp + 4 * a4);
    const int cc[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
    for (int m = 0; m < 4; ++m)
      if (4 * a4 + m < NL) ue[4 * a4 + m] = cc[m] >= 0 ? u[cc[m]] : (T)0;
  }
  T ca[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) ca[c] = AFF ? geo[(int64_t)c * ncells + e] : (T)0;
  T v[NL];
#pragma unroll
  for (int a = 0; a < NL; ++a) v[a] = 0;

  if constexpr (D == 2) {
#pragma unroll
    for (int qy = 0; qy < K; ++qy) {
      // contract y at Gauss row qy: z0 = B_y u, z1 = G_y u (per x node)
      T z0[K], z1[K];
#pragma unroll
      for (int ix = 0; ix < K; ++ix) {
        T s0 = 0, s1 = 0;
#pragma unroll
        for (int iy = 0; iy < K; ++iy) {
          s0 += tb.B[qy][iy] * ue[ix + K * iy];
          s1 += tb.G[qy][iy] * ue[ix + K * iy];
        }
        z0[ix] = s0;
        z1[ix] = s1;
      }
      T fx[K], fy[K];
#pragma unroll
      for (int qx = 0; qx < K; ++qx) {
        T gx = 0, gy = 0;
#pragma unroll
        for (int ix = 0; ix < K; ++ix) {
          gx += tb.G[qx][ix] * z0[ix];
          gy += tb.B[qx][ix] * z1[ix];
        }
        const int q = qx + K * qy;
        const T w = AFF ? tb.W[qx] * tb.W[qy] : (T)1;
        const T c00 = geo_at<T, NC, AFF>(geo, ca, ncells, e, q, 0, w);
        const T c01 = geo_at<T, NC, AFF>(geo, ca, ncells, e, q, 1, w);
        const T c11 = geo_at<T, NC, AFF>(geo, ca, ncells, e, q, 2, w);
        fx[qx] = c00 * gx + c01 * gy;
        fy[qx] = c01 * gx + c11 * gy;
      }
      // transposed contractions back to the nodes
#pragma unroll
      for (int ix = 0; ix < K; ++ix) {
        T px = 0, py = 0;
#pragma unroll
        for (int qx = 0; qx < K; ++qx) {
          px += tb.G[qx][ix] * fx[qx];
          py += tb.B[qx][ix] * fy[qx];
        }
#pragma unroll
        for (int iy = 0; iy < K; ++iy) v[ix + K * iy] += tb.B[qy][iy] * px + tb.G[qy][iy] * py;
      }
    }
  } else {
#pragma unroll
    for (int qz = 0; qz < K; ++qz) {
      // contract z at Gauss slice qz
      T z0[K * K], z1[K * K];
#pragma unroll
      for (int j = 0; j < K * K; ++j) {
        T s0 = 0, s1 = 0;
#pragma unroll
        for (int iz = 0; iz < K; ++iz) {
          s0 += tb.B[qz][iz] * ue[j + K * K * iz];
          s1 += tb.G[qz][iz] * ue[j + K * K * iz];
        }
        z0[j] = s0;
        z1[j] = s1;
      }
      T h0[K * K], h1[K * K];  // slice accumulators of the transposed y contraction
#pragma unroll
      for (int j = 0; j < K * K; ++j) h0[j] = h1[j] = 0;
#pragma unroll
      for (int qy = 0; qy < K; ++qy) {
        T y00[K], y01[K], y10[K];
#pragma unroll
        for (int ix = 0; ix < K; ++ix) {
          T a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
          for (int iy = 0; iy < K; ++iy) {
            a0 += tb.B[qy][iy] * z0[ix + K * iy];
            a1 += tb.G[qy][iy] * z0[ix + K * iy];
            a2 += tb.B[qy][iy] * z1[ix + K * iy];
          }
          y00[ix] = a0;
          y01[ix] = a1;
          y10[ix] = a2;
        }
        T fx[K], fy[K], fz[K];
#pragma unroll
        for (int qx = 0; qx < K; ++qx) {
          T gx = 0, gy = 0, gz = 0;
#pragma unroll
          for (int ix = 0; ix < K; ++ix) {
            gx += tb.G[qx][ix] * y00[ix];
            gy += tb.B[qx][ix] * y01[ix];
            gz += tb.B[qx][ix] * y10[ix];
          }
          const int q = qx + K * qy + K * K * qz;
          const T w = AFF ? tb.W[qx] * tb.W[qy] * tb.W[qz] : (T)1;
          const T c00 = geo_at<T, NC, AFF>(geo, ca, ncells, e, q, 0, w);
          const T c01 = geo_at<T, NC, AFF>(geo, ca, ncells, e, q, 1, w);
          const T c02 = geo_at<T, NC, AFF>(geo, ca, ncells, e, q, 2, w);
          const T c11 = geo_at<T, NC, AFF>(geo, ca, ncells, e, q, 3, w);
          const T c12 = geo_at<T, NC, AFF>(geo, ca, ncells, e, q, 4, w);
          const T c22 = geo_at<T, NC, AFF>(geo, ca, ncells, e, q, 5, w);
          fx[qx] = c00 * gx + c01 * gy + c02 * gz;
          fy[qx] = c01 * gx + c11 * gy + c12 * gz;
          fz[qx] = c02 * gx + c12 * gy + c22 * gz;
        }
#pragma unroll
        for (int ix = 0; ix < K; ++ix) {
          T px = 0, py = 0, pz = 0;
#pragma unroll
          for (int qx = 0; qx < K; ++qx) {
            px += tb.G[qx][ix] * fx[qx];
            py += tb.B[qx][ix] * fy[qx];
            pz += tb.B[qx][ix] * fz[qx];
          }
#pragma unroll
          for (int iy = 0; iy < K; ++iy) {
            h0[ix + K * iy] += tb.B[qy][iy] * px + tb.G[qy][iy] * py;
            h1[ix + K * iy] += tb.B[qy][iy] * pz;
          }
        }
      }
#pragma unroll
      for (int iz = 0; iz < K; ++iz)
#pragma unroll
        for (int j = 0; j < K * K; ++j) v[j + K * K * iz] += tb.B[qz][iz] * h0[j] + tb.G[qz][iz] * h1[j];
    }
  }

  // store y_e (16-byte stores; padding entries are written as zero)
  constexpr int VW = 16 / (int)sizeof(T);
  typedef T V16 __attribute__((ext_vector_type(VW)));
  T* yp = Y + (int64_t)e * nlocp;
#pragma unroll
  for (int a0 = 0; a0 < NP; a0 += VW) {
    V16 t;
#pragma unroll
    for (int m = 0; m < VW; ++m) t[m] = (a0 + m < NL) ? v[a0 + m] : (T)0;
    *reinterpret_cast<V16*>(yp + a0) = t;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_mf_gather(int n, const int* __restrict__ inc_ptr, const int* __restrict__ inc,
                                                   const T* __restrict__ Y, const T* __restrict__ cd,
                                                   const T* __restrict__ u, const T* __restrict__ b, T* rho, T* x,
                                                   const T* __restrict__ dinv, T* dout, T c1, T c2, int flags,
                                                   const int* __restrict__ skip, int nlog) {
  if (skip && *skip) return;
  const int lb = xcd_block(nlog);
  if (lb < 0) return;
  const int i = lb * 256 + (int)threadIdx.x;
  if (i >= n) return;
  const int s0 = inc_ptr[i], s1 = inc_ptr[i + 1];
  T t = 0;
  if (s0 == s1) {
    t = cd[i] * u[i];
  } else {
    // up to 8 outputs in flight, summed in ascending order
    int k = s0;
    for (; k + 8 <= s1; k += 8) {
      T yv[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) yv[m] = Y[inc[k + m]];
#pragma unroll
      for (int m = 0; m < 8; ++m) t += yv[m];
    }
    for (; k < s1; ++k) t += Y[inc[k]];
  }
  if (flags & F_PLAIN) {
    rho[i] = t;
    return;
  }
  const T r = ((flags & F_RHO_FROM_B) ? b[i] : rho[i]) - t;
  if (flags & F_RHO_STORE) rho[i] = r;
  const T ui = u[i];
  if (flags & F_X_ASSIGN)
    x[i] = ui;
  else if (flags & F_X_ADD)
    x[i] += ui;
  if (flags & F_D_OUT) dout[i] = c1 * ui + c2 * dinv[i] * r;
}

template <typename T, int D, int K>
void launch_cell(const MfOp& m, const MfTables<T>& tb, const T* geo, const T* u, T* Y, const int* skip,
                 hipStream_t s) {
  const int nlog = (m.ncells + 255) / 256;
  if (m.affine)
    hipLaunchKernelGGL((k_mf_cell<T, D, K, true>), dim3(xcd_grid(nlog)), dim3(256), 0, s, m.ncells, m.nlocp, m.conn,
                       geo, tb, u, Y, skip, nlog);
  else
    hipLaunchKernelGGL((k_mf_cell<T, D, K, false>), dim3(xcd_grid(nlog)), dim3(256), 0, s, m.ncells, m.nlocp,
                       m.conn, geo, tb, u, Y, skip, nlog);
}

}  // namespace

template <typename T>
void launch_mf_apply(const MfOp& m, const MfTables<T>& tb, const T* geo, const T* cd, T* Y, const T* dinv,
                     const T* u, const T* b, T* rho, T* x, T* dout, double c1, double c2, int flags, const int* skip,
                     hipStream_t s) {
  if (m.n <= 0) return;
  if (m.ncells > 0) {
    const int key = m.d * 10 + m.k;
    switch (key) {
      case 22: launch_cell<T, 2, 2>(m, tb, geo, u, Y, skip, s); break;
      case 23: launch_cell<T, 2, 3>(m, tb, geo, u, Y, skip, s); break;
      case 24: launch_cell<T, 2, 4>(m, tb, geo, u, Y, skip, s); break;
      case 32: launch_cell<T, 3, 2>(m, tb, geo, u, Y, skip, s); break;
      case 33: launch_cell<T, 3, 3>(m, tb, geo, u, Y, skip, s); break;
      case 34: launch_cell<T, 3, 4>(m, tb, geo, u, Y, skip, s); break;
      default: throw std::runtime_error("matrix-free operator: unsupported dimension or degree");
    }
    check_launch("k_mf_cell");
  }
  const int nlog = (m.n + 255) / 256;
  hipLaunchKernelGGL((k_mf_gather<T>), dim3(xcd_grid(nlog)), dim3(256), 0, s, m.n, m.inc_ptr, m.inc, Y, cd, u, b,
                     rho, x, dinv, dout, (T)c1, (T)c2, flags, skip, nlog);
  check_launch("k_mf_gather");
}
template void launch_mf_apply<float>(const MfOp&, const MfTables<float>&, const float*, const float*, float*,
                                     const float*, const float*, const float*, float*, float*, float*, double, double,
                                     int, const int*, hipStream_t);
template void launch_mf_apply<double>(const MfOp&, const MfTables<double>&, const double*, const double*, double*,
                                      const double*, const double*, const double*, double*, double*, double*, double,
                                      double, int, const int*, hipStream_t);

}  // namespace r3mg
