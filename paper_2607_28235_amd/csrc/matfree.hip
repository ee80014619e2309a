// Matrix-free application of the fine-level operator for Q_p Lagrange elements on multilinear cells (the
// Poisson stiffness matrix of the paper's experiments, Section 6, assembled with Gauss quadrature of p + 1
// points per axis).  The operator is A = D (sum_e K_e) D + diag(cd): D removes the constrained DoFs (their
// columns and rows) and cd holds the diagonal of the constrained rows.
//
// Two launches, both deterministic (no floating-point atomics):
//   k_mf_cell    one thread per cell: gather u_e, y_e = K_e u_e by sum factorisation (one Gauss-point slice at
//                a time along the last axis, which bounds the registers; the geometric factors of multilinear
//                cells evaluated at each Gauss point from the map's coefficients), store y_e to the cell-local
//                buffer Y;
//   k_mf_gather  one thread per DoF: t_i = sum of its cell-local outputs in ascending (cell, node) order, then
//                the smoother epilogue of the CSR level kernels.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>

#include "hip_util.h"
#include "kernels.h"

namespace r3mg {

namespace {

using hiputil::check_launch;
using hiputil::xcd_block;
using hiputil::xcd_grid;

// Geometry at one Gauss point: the upper triangle of C = w kappa adj(J) adj(J)^T / det J.  Affine cells store
// kappa |det J| J^-1 J^-T per cell; multilinear cells store the map's derivative coefficients.
template <typename T, int D, bool AFF>
__device__ inline void geo_point(const T* gm, T w, T x1, T x2, T x3, T* c) {
  if constexpr (AFF) {
#pragma unroll
    for (int k = 0; k < (D == 2 ? 3 : 6); ++k) c[k] = w * gm[k];
  } else if constexpr (D == 2) {
    // columns of J: dx/dxi1 = c_1 + xi2 c_12, dx/dxi2 = c_2 + xi1 c_12
    const T a = gm[0] + x2 * gm[4], cc = gm[1] + x2 * gm[5];
    const T b = gm[2] + x1 * gm[4], d = gm[3] + x1 * gm[5];
    const T s = w * gm[6] / (a * d - b * cc);
    c[0] = s * (b * b + d * d);
    c[1] = -s * (a * b + cc * d);
    c[2] = s * (a * a + cc * cc);
  } else {
    T j0[3], j1[3], j2[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      j0[i] = gm[i] + x2 * gm[9 + i] + x3 * (gm[12 + i] + x2 * gm[18 + i]);
      j1[i] = gm[3 + i] + x1 * gm[9 + i] + x3 * (gm[15 + i] + x1 * gm[18 + i]);
      j2[i] = gm[6 + i] + x1 * gm[12 + i] + x2 * (gm[15 + i] + x1 * gm[18 + i]);
    }
    // rows of adj(J) = det J^-1: j1 x j2, j2 x j0, j0 x j1
    T m[3][3];
    m[0][0] = j1[1] * j2[2] - j1[2] * j2[1];
    m[0][1] = j1[2] * j2[0] - j1[0] * j2[2];
    m[0][2] = j1[0] * j2[1] - j1[1] * j2[0];
    m[1][0] = j2[1] * j0[2] - j2[2] * j0[1];
    m[1][1] = j2[2] * j0[0] - j2[0] * j0[2];
    m[1][2] = j2[0] * j0[1] - j2[1] * j0[0];
    m[2][0] = j0[1] * j1[2] - j0[2] * j1[1];
    m[2][1] = j0[2] * j1[0] - j0[0] * j1[2];
    m[2][2] = j0[0] * j1[1] - j0[1] * j1[0];
    const T det = j0[0] * m[0][0] + j0[1] * m[0][1] + j0[2] * m[0][2];
    const T s = w * gm[21] / det;
    int k = 0;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int t = r; t < 3; ++t) c[k++] = s * (m[r][0] * m[t][0] + m[r][1] * m[t][1] + m[r][2] * m[t][2]);
  }
}

// y_e = K_e u_e for one cell by sum factorisation, one Gauss-point slice at a time along the last axis (which
// bounds the registers); gm holds the cell's geometry record (affine C or the map's coefficients).
template <typename T, int D, int K, bool AFF>
__device__ __forceinline__ void cell_action(const T* ue, const T* gm, const MfTables<T>& tb, T* v) {
  constexpr int NL = D == 2 ? K * K : K * K * K;
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
        T c[3];
        geo_point<T, 2, AFF>(gm, tb.W[qx] * tb.W[qy], tb.X[qx], tb.X[qy], (T)0, c);
        fx[qx] = c[0] * gx + c[1] * gy;
        fy[qx] = c[1] * gx + c[2] * gy;
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
          T c[6];
          geo_point<T, 3, AFF>(gm, tb.W[qx] * tb.W[qy] * tb.W[qz], tb.X[qx], tb.X[qy], tb.X[qz], c);
          fx[qx] = c[0] * gx + c[1] * gy + c[2] * gz;
          fy[qx] = c[1] * gx + c[3] * gy + c[4] * gz;
          fz[qx] = c[2] * gx + c[4] * gy + c[5] * gz;
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

}

// geometry record of cell e (a harmless unit square / cube for the idle lanes past the last cell)
template <typename T, int D, bool AFF>
__device__ __forceinline__ void load_geometry(const T* __restrict__ geo, int ncells, int e, bool valid, T* gm) {
  constexpr int NC = D == 2 ? 3 : 6;
  constexpr int NG = AFF ? NC : (D == 2 ? 7 : 22);
#pragma unroll
  for (int c = 0; c < NG; ++c) gm[c] = valid ? geo[(int64_t)c * ncells + e] : (T)(c == NG - 1 ? 1 : 0);
  if constexpr (!AFF) {
    if (!valid) {
#pragma unroll
      for (int c = 0; c < NG; ++c) gm[c] = 0;
      if constexpr (D == 2) { gm[0] = 1; gm[3] = 1; gm[6] = 1; }
      else { gm[0] = 1; gm[4] = 1; gm[8] = 1; gm[21] = 1; }
    }
  }
}

// One thread per cell.  When a wave's connectivity and outputs fit LDS (256 cells x nlocp entries <= 64 KiB),
// both are staged through it so that the global loads and stores are contiguous 16-byte accesses.
template <typename T, int D, int K, bool AFF>
__global__ __launch_bounds__(256) void k_mf_cell(int ncells, const int* __restrict__ conn, const T* __restrict__ geo,
                                                 MfTables<T> tb, const T* __restrict__ u, T* __restrict__ Y,
                                                 const int* __restrict__ skip, int nlog) {
  constexpr int NL = D == 2 ? K * K : K * K * K;
  constexpr int NP = (NL + 3) / 4 * 4;
  constexpr int NC = D == 2 ? 3 : 6;
  constexpr int NG = AFF ? NC : (D == 2 ? 7 : 22);
  constexpr int ES = sizeof(T) > 4 ? (int)sizeof(T) : 4;
  constexpr bool STAGE = 256 * NP * ES <= 65536;
  constexpr int VW = 16 / (int)sizeof(T);
  typedef T V16 __attribute__((ext_vector_type(VW)));
  __shared__ __attribute__((aligned(16))) char lds[STAGE ? 256 * NP * ES : 16];
  if (skip && *skip) return;
  const int lb = xcd_block(nlog);
  if (lb < 0) return;
  const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
  const int e = lb * 256 + (int)threadIdx.x;
  const bool valid = e < ncells;
  const int64_t total = (int64_t)ncells * NP;
  const int64_t wbase = (int64_t)(lb * 256 + wv * 64) * NP;  // first entry of this wave's cells
  char* wlds = lds + wv * 64 * NP * ES;

  int cidx[NP];
  if constexpr (STAGE) {
    int* li = reinterpret_cast<int*>(wlds);
#pragma unroll
    for (int j = 0; j < NP / 4; ++j) {
      const int q = j * 64 + lane;
      const int64_t off = wbase + 4 * (int64_t)q;
      int4 c4 = make_int4(-1, -1, -1, -1);
      if (off < total) c4 = *reinterpret_cast<const int4*>(conn + off);
      *reinterpret_cast<int4*>(li + 4 * q) = c4;
    }
    __syncthreads();
#pragma unroll
    for (int a4 = 0; a4 < NP / 4; ++a4) {
      const int4 c4 = *reinterpret_cast<const int4*>(li + lane * NP + 4 * a4);
      cidx[4 * a4] = c4.x;
      cidx[4 * a4 + 1] = c4.y;
      cidx[4 * a4 + 2] = c4.z;
      cidx[4 * a4 + 3] = c4.w;
    }
  } else {
#pragma unroll
    for (int a4 = 0; a4 < NP / 4; ++a4) {
      int4 c4 = make_int4(-1, -1, -1, -1);
      if (valid) c4 = *reinterpret_cast<const int4*>(conn + (int64_t)e * NP + 4 * a4);
      cidx[4 * a4] = c4.x;
      cidx[4 * a4 + 1] = c4.y;
      cidx[4 * a4 + 2] = c4.z;
      cidx[4 * a4 + 3] = c4.w;
    }
  }
  // gather u_e (constrained DoFs, padding and cells past the end read as zero)
  T ue[NL];
#pragma unroll
  for (int a = 0; a < NL; ++a) ue[a] = cidx[a] >= 0 ? u[cidx[a]] : (T)0;
  T gm[NG];
  load_geometry<T, D, AFF>(geo, ncells, e, valid, gm);
  T v[NL];
  cell_action<T, D, K, AFF>(ue, gm, tb, v);

  // store y_e (padding entries are written as zero)
  if constexpr (STAGE) {
    T* lt = reinterpret_cast<T*>(wlds);
    __syncthreads();  // every lane has read its connectivity: the tile now holds outputs
#pragma unroll
    for (int a0 = 0; a0 < NP; a0 += VW) {
      V16 t;
#pragma unroll
      for (int m = 0; m < VW; ++m) t[m] = (a0 + m < NL) ? v[a0 + m] : (T)0;
      *reinterpret_cast<V16*>(lt + lane * NP + a0) = t;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NP / VW; ++j) {
      const int q = j * 64 + lane;
      const int64_t off = wbase + (int64_t)VW * q;
      if (off < total) *reinterpret_cast<V16*>(Y + off) = *reinterpret_cast<const V16*>(lt + VW * q);
    }
  } else {
    if (!valid) return;
    T* yp = Y + (int64_t)e * NP;
#pragma unroll
    for (int a0 = 0; a0 < NP; a0 += VW) {
      V16 t;
#pragma unroll
      for (int m = 0; m < VW; ++m) t[m] = (a0 + m < NL) ? v[a0 + m] : (T)0;
      *reinterpret_cast<V16*>(yp + a0) = t;
    }
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

// Several right-hand sides (nr columns, n x nr interleaved vectors): each thread applies its cell to the columns
// in turn, reusing its connectivity and the geometry held in registers.  Y holds one plane of cell outputs per
// column, Y[k * ncells * nlocp + e * nlocp + a], written through LDS as contiguous 16-byte stores (as for one
// right-hand side).
template <typename T, int D, int K, bool AFF>
__global__ __launch_bounds__(256) void k_mf_cell_mr(int ncells, int nr, const int* __restrict__ conn,
                                                    const T* __restrict__ geo, MfTables<T> tb,
                                                    const T* __restrict__ u, T* __restrict__ Y,
                                                    const int* __restrict__ skip, int nlog) {
  constexpr int NL = D == 2 ? K * K : K * K * K;
  constexpr int NP = (NL + 3) / 4 * 4;
  constexpr int NC = D == 2 ? 3 : 6;
  constexpr int NG = AFF ? NC : (D == 2 ? 7 : 22);
  constexpr int ES = sizeof(T) > 4 ? (int)sizeof(T) : 4;
  constexpr bool STAGE = 256 * NP * ES <= 65536;
  constexpr int VW = 16 / (int)sizeof(T);
  typedef T V16 __attribute__((ext_vector_type(VW)));
  __shared__ __attribute__((aligned(16))) char lds[STAGE ? 256 * NP * ES : 16];
  if (skip && *skip) return;
  const int lb = xcd_block(nlog);
  if (lb < 0) return;
  const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
  const int e = lb * 256 + (int)threadIdx.x;
  const bool valid = e < ncells;
  const int64_t total = (int64_t)ncells * NP;
  const int64_t wbase = (int64_t)(lb * 256 + wv * 64) * NP;
  char* wlds = lds + wv * 64 * NP * ES;
  int cidx[NP];
  if constexpr (STAGE) {
    int* li = reinterpret_cast<int*>(wlds);
#pragma unroll
    for (int j = 0; j < NP / 4; ++j) {
      const int q = j * 64 + lane;
      const int64_t off = wbase + 4 * (int64_t)q;
      int4 c4 = make_int4(-1, -1, -1, -1);
      if (off < total) c4 = *reinterpret_cast<const int4*>(conn + off);
      *reinterpret_cast<int4*>(li + 4 * q) = c4;
    }
    __syncthreads();
#pragma unroll
    for (int a4 = 0; a4 < NP / 4; ++a4) {
      const int4 c4 = *reinterpret_cast<const int4*>(li + lane * NP + 4 * a4);
      cidx[4 * a4] = c4.x;
      cidx[4 * a4 + 1] = c4.y;
      cidx[4 * a4 + 2] = c4.z;
      cidx[4 * a4 + 3] = c4.w;
    }
  } else {
#pragma unroll
    for (int a4 = 0; a4 < NP / 4; ++a4) {
      int4 c4 = make_int4(-1, -1, -1, -1);
      if (valid) c4 = *reinterpret_cast<const int4*>(conn + (int64_t)e * NP + 4 * a4);
      cidx[4 * a4] = c4.x;
      cidx[4 * a4 + 1] = c4.y;
      cidx[4 * a4 + 2] = c4.z;
      cidx[4 * a4 + 3] = c4.w;
    }
  }
  T gm[NG];
  load_geometry<T, D, AFF>(geo, ncells, e, valid, gm);
  // 32-bit element offsets (n * nr < 2^31 is checked at set-up) keep the per-node addresses to one register each
#pragma unroll
  for (int a = 0; a < NL; ++a) cidx[a] = cidx[a] >= 0 ? cidx[a] * nr : -1;
#pragma unroll 1
  for (int k = 0; k < nr; ++k) {
    // the geometric factors at the Gauss points do not depend on the column; without this (empty) register
    // constraint the compiler keeps all of them live across the loop, which exhausts the registers in 3D
#pragma unroll
    for (int c = 0; c < NG; ++c) asm volatile("" : "+v"(gm[c]));
    T ue[NL];
#pragma unroll
    for (int a = 0; a < NL; ++a) ue[a] = cidx[a] >= 0 ? u[cidx[a] + k] : (T)0;
    T v[NL];
    cell_action<T, D, K, AFF>(ue, gm, tb, v);
    T* plane = Y + (int64_t)k * total;
    if constexpr (STAGE) {
      T* lt = reinterpret_cast<T*>(wlds);
      __syncthreads();  // the tile is free: connectivity read (first column) or previous column stored
#pragma unroll
      for (int a0 = 0; a0 < NP; a0 += VW) {
        V16 t;
#pragma unroll
        for (int m = 0; m < VW; ++m) t[m] = (a0 + m < NL) ? v[a0 + m] : (T)0;
        *reinterpret_cast<V16*>(lt + lane * NP + a0) = t;
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < NP / VW; ++j) {
        const int q = j * 64 + lane;
        const int64_t off = wbase + (int64_t)VW * q;
        if (off < total) *reinterpret_cast<V16*>(plane + off) = *reinterpret_cast<const V16*>(lt + VW * q);
      }
    } else if (valid) {
#pragma unroll
      for (int a0 = 0; a0 < NP; a0 += VW) {
        V16 t;
#pragma unroll
        for (int m = 0; m < VW; ++m) t[m] = (a0 + m < NL) ? v[a0 + m] : (T)0;
        *reinterpret_cast<V16*>(plane + (int64_t)e * NP + a0) = t;
      }
    }
  }
}

// One thread per (DoF, column), columns fastest: the column's sum over the DoF's cell outputs in ascending (cell,
// node) order, then the epilogue of the multi-RHS level kernels for that entry.
template <typename T>
__global__ __launch_bounds__(256) void k_mf_gather_mr(int n, int nr, int64_t plane, const int* __restrict__ inc_ptr,
                                                      const int* __restrict__ inc, const T* __restrict__ Y,
                                                      const T* __restrict__ cd, const T* __restrict__ u,
                                                      const T* __restrict__ b, T* rho, T* x,
                                                      const T* __restrict__ dinv, T* dout, T c1, T c2, int flags,
                                                      const int* __restrict__ skip, int nlog) {
  if (skip && *skip) return;
  const int lb = xcd_block(nlog);
  if (lb < 0) return;
  const int64_t t = (int64_t)lb * 256 + threadIdx.x;
  const int64_t i = t / nr;
  const int k = (int)(t - i * nr);
  if (i >= n) return;
  const int s0 = inc_ptr[i], s1 = inc_ptr[i + 1];
  const T* yk = Y + (int64_t)k * plane;
  T acc = 0;
  if (s0 == s1) {
    acc = cd[i] * u[t];
  } else {
    int j = s0;
    for (; j + 8 <= s1; j += 8) {
      T yv[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) yv[m] = yk[inc[j + m]];
#pragma unroll
      for (int m = 0; m < 8; ++m) acc += yv[m];
    }
    for (; j < s1; ++j) acc += yk[inc[j]];
  }
  if (flags & F_PLAIN) {
    rho[t] = acc;
    return;
  }
  const T r = ((flags & F_RHO_FROM_B) ? b[t] : rho[t]) - acc;
  if (flags & F_RHO_STORE) rho[t] = r;
  const T ui = u[t];
  if (flags & F_X_ASSIGN)
    x[t] = ui;
  else if (flags & F_X_ADD)
    x[t] += ui;
  if (flags & F_D_OUT) dout[t] = c1 * ui + c2 * dinv[i] * r;
}

template <typename T, int D, int K>
void launch_cell_mr(const MfOp& m, int nr, const MfTables<T>& tb, const T* geo, const T* u, T* Y, const int* skip,
                    hipStream_t s) {
  const int nlog = (m.ncells + 255) / 256;
  constexpr int NL = D == 2 ? K * K : K * K * K;
  if (m.nlocp != (NL + 3) / 4 * 4) throw std::runtime_error("matrix-free operator: connectivity stride mismatch");
  if (m.affine)
    hipLaunchKernelGGL((k_mf_cell_mr<T, D, K, true>), dim3(xcd_grid(nlog)), dim3(256), 0, s, m.ncells, nr, m.conn,
                       geo, tb, u, Y, skip, nlog);
  else
    hipLaunchKernelGGL((k_mf_cell_mr<T, D, K, false>), dim3(xcd_grid(nlog)), dim3(256), 0, s, m.ncells, nr, m.conn,
                       geo, tb, u, Y, skip, nlog);
}

template <typename T>
void launch_gather_mr(const MfOp& m, int nr, const T* Y, const T* cd, const T* dinv, const T* u, const T* b, T* rho,
                      T* x, T* dout, double c1, double c2, int flags, const int* skip, hipStream_t s) {
  const int64_t threads = (int64_t)m.n * nr;
  const int nlog = (int)((threads + 255) / 256);
  const int64_t plane = (int64_t)m.ncells * m.nlocp;
  hipLaunchKernelGGL((k_mf_gather_mr<T>), dim3(xcd_grid(nlog)), dim3(256), 0, s, m.n, nr, plane, m.inc_ptr, m.inc,
                     Y, cd, u, b, rho, x, dinv, dout, (T)c1, (T)c2, flags, skip, nlog);
}

template <typename T, int D, int K>
void launch_cell(const MfOp& m, const MfTables<T>& tb, const T* geo, const T* u, T* Y, const int* skip,
                 hipStream_t s) {
  const int nlog = (m.ncells + 255) / 256;
  constexpr int NL = D == 2 ? K * K : K * K * K;
  if (m.nlocp != (NL + 3) / 4 * 4) throw std::runtime_error("matrix-free operator: connectivity stride mismatch");
  if (m.affine)
    hipLaunchKernelGGL((k_mf_cell<T, D, K, true>), dim3(xcd_grid(nlog)), dim3(256), 0, s, m.ncells, m.conn, geo, tb,
                       u, Y, skip, nlog);
  else
    hipLaunchKernelGGL((k_mf_cell<T, D, K, false>), dim3(xcd_grid(nlog)), dim3(256), 0, s, m.ncells, m.conn, geo,
                       tb, u, Y, skip, nlog);
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
template <typename T>
void launch_mf_apply_mr(const MfOp& m, int nr, const MfTables<T>& tb, const T* geo, const T* cd, T* Y, const T* dinv,
                        const T* u, const T* b, T* rho, T* x, T* dout, double c1, double c2, int flags,
                        const int* skip, hipStream_t s) {
  if (m.n <= 0) return;
  if (nr != 2 && nr != 4 && nr != 8 && nr != 16) throw std::runtime_error("matrix-free operator: unsupported nrhs");
  switch (m.d * 10 + m.k) {
    case 22: launch_cell_mr<T, 2, 2>(m, nr, tb, geo, u, Y, skip, s); break;
    case 23: launch_cell_mr<T, 2, 3>(m, nr, tb, geo, u, Y, skip, s); break;
    case 24: launch_cell_mr<T, 2, 4>(m, nr, tb, geo, u, Y, skip, s); break;
    case 32: launch_cell_mr<T, 3, 2>(m, nr, tb, geo, u, Y, skip, s); break;
    case 33: launch_cell_mr<T, 3, 3>(m, nr, tb, geo, u, Y, skip, s); break;
    case 34: launch_cell_mr<T, 3, 4>(m, nr, tb, geo, u, Y, skip, s); break;
    default: throw std::runtime_error("matrix-free operator: unsupported dimension or degree");
  }
  check_launch("k_mf_cell_mr");
  launch_gather_mr<T>(m, nr, Y, cd, dinv, u, b, rho, x, dout, c1, c2, flags, skip, s);
  check_launch("k_mf_gather_mr");
}
template void launch_mf_apply_mr<float>(const MfOp&, int, const MfTables<float>&, const float*, const float*, float*,
                                        const float*, const float*, const float*, float*, float*, float*, double,
                                        double, int, const int*, hipStream_t);
template void launch_mf_apply_mr<double>(const MfOp&, int, const MfTables<double>&, const double*, const double*,
                                         double*, const double*, const double*, const double*, double*, double*,
                                         double*, double, double, int, const int*, hipStream_t);
template void launch_mf_apply<float>(const MfOp&, const MfTables<float>&, const float*, const float*, float*,
                                     const float*, const float*, const float*, float*, float*, float*, double, double,
                                     int, const int*, hipStream_t);
template void launch_mf_apply<double>(const MfOp&, const MfTables<double>&, const double*, const double*, double*,
                                      const double*, const double*, const double*, double*, double*, double*, double,
                                      double, int, const int*, hipStream_t);

}  // namespace r3mg
