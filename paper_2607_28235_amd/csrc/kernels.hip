// HIP kernels of the R3MG-C hot path for gfx950 (CDNA4, wave64).
//
// Level operators (paper Section 4: inherited operators A_i = P_i^T A P_i) are applied by one fused kernel
// that also performs the Chebyshev-accelerated Jacobi update of the smoother (Section 5 Remark on the
// smoother, Section 6): t = A u; rho -= t; x += u; d = c1 u + c2 D^{-1} rho.  The fine level is CSR; the
// agglomerated levels store dense B x B blocks (B = (p'+1)^d) with one column index per block, laid out so
// that every row's values are contiguous ("block rows": row (K,q) holds blocks j = 0..nb-1, columns c).
// Transfers (Section 4 construction of P_{M-1} and P~) evaluate the box basis on the fly from per-point
// local coordinates; they never store P.
//
// All reductions are deterministic: fixed per-thread order, fixed shuffle trees, fixed LDS trees, and
// per-block partials summed in index order by a single block.  No floating-point atomics.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <algorithm>
#include <stdexcept>
#include <string>

#include "hip_util.h"
#include "kernels.h"

namespace r3mg {

namespace {

using hiputil::check_launch;
using hiputil::xcd_block;
using hiputil::xcd_grid;

template <typename T>
struct Basis1D {
  T t[4];
  T w[4];
  int k;
};

template <typename T>
Basis1D<T> make_basis(int pc) {
  double t[4] = {0, 0, 0, 0};
  switch (pc) {
    case 0: t[0] = 0.5; break;
    case 1: t[0] = 0.0; t[1] = 1.0; break;
    case 2: t[0] = 0.0; t[1] = 0.5; t[2] = 1.0; break;
    default: {
      double s = 1.0 / std::sqrt(5.0);
      t[0] = 0.0; t[1] = 0.5 * (1.0 - s); t[2] = 0.5 * (1.0 + s); t[3] = 1.0;
    }
  }
  Basis1D<T> b;
  b.k = pc + 1;
  for (int j = 0; j < 4; ++j) {
    double w = 1.0;
    for (int m = 0; m < b.k; ++m)
      if (m != j && j < b.k) w /= (t[j] - t[m]);
    b.t[j] = (T)t[j];
    b.w[j] = (T)w;
  }
  return b;
}

// l_j(s) = w_j prod_{m != j} (s - t_m)
template <typename T>
__device__ inline void lag1d(const Basis1D<T>& bs, T s, T* l) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (j < bs.k) {
      T v = bs.w[j];
#pragma unroll
      for (int m = 0; m < 4; ++m)
        if (m < bs.k && m != j) v *= (s - bs.t[m]);
      l[j] = v;
    }
  }
}

// compile-time forms of lag1d / phi_q (same operations in the same order)
template <typename T, int KB>
__device__ inline void lag1d_k(const Basis1D<T>& bs, T s, T* l) {
#pragma unroll
  for (int j = 0; j < KB; ++j) {
    T v = bs.w[j];
#pragma unroll
    for (int m = 0; m < KB; ++m)
      if (m != j) v *= (s - bs.t[m]);
    l[j] = v;
  }
}
// calls f(q, phi_q) for q = 0 .. KB^D - 1 in ascending order
template <typename T, int D, int KB, typename F>
__device__ inline void for_each_phi(const T (*l)[4], F&& f) {
  int q = 0;
#pragma unroll
  for (int q2 = 0; q2 < (D == 3 ? KB : 1); ++q2)
#pragma unroll
    for (int q1 = 0; q1 < KB; ++q1)
#pragma unroll
      for (int q0 = 0; q0 < KB; ++q0) {
        T v = l[0][q0] * l[1][q1];
        if (D == 3) v *= l[2][q2];
        f(q++, v);
      }
}

// phi_q of multi-index q = q0 + k q1 + k^2 q2 from 1D tables l[a][.]
template <typename T>
__device__ inline T phi_q(const T (*l)[4], int d, int k, int q) {
  T v = l[0][q % k];
  q /= k;
  v *= l[1][q % k];
  if (d == 3) {
    q /= k;
    v *= l[2][q % k];
  }
  return v;
}

template <typename T>
__device__ inline T wave_sum(T v, int width) {
  for (int off = width >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// deterministic block sum (blockDim.x = 256): returns the total in thread 0
__device__ inline double block_sum256(double v, double* sh) {
  v = wave_sum(v, 64);
  int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

}  // namespace

// =============================================================================================
// Fused level kernel: t = A u (CSR or block rows), then the smoother update epilogue.
// G lanes per row (power of two), 256 threads per block, NR right-hand sides interleaved.
// =============================================================================================
template <typename T, int NR, bool BLOCKED>
__device__ inline void row_product(int row, int lane, int G, int blk, const int* __restrict__ ptr,
                                   const int* __restrict__ idx, const T* __restrict__ val,
                                   const T* __restrict__ u, T* acc) {
  if (!BLOCKED) {
    // UNR steps per batch: their column, value and u loads are all in flight before the products (each lane
    // still accumulates its entries in ascending order)
    constexpr int UNR = NR >= 16 ? 2 : 32 / NR;
    const int s = ptr[row], e = ptr[row + 1];
    for (int p0 = s + lane; p0 < e; p0 += UNR * G) {
      T a[UNR];
      int64_t c[UNR];
#pragma unroll
      for (int m = 0; m < UNR; ++m) {
        const int p = p0 + m * G;
        a[m] = p < e ? val[p] : (T)0;
        c[m] = p < e ? (int64_t)idx[p] * NR : 0;
      }
      T uv[UNR][NR];
      constexpr int VW = 16 / (int)sizeof(T);  // entries per 16-byte load (u rows are NR-aligned)
      if constexpr (NR % VW == 0) {
        typedef T V16 __attribute__((ext_vector_type(VW)));
#pragma unroll
        for (int m = 0; m < UNR; ++m)
#pragma unroll
          for (int k = 0; k < NR; k += VW) {
            const V16 t = *reinterpret_cast<const V16*>(u + c[m] + k);
#pragma unroll
            for (int w = 0; w < VW; ++w) uv[m][k + w] = t[w];
          }
      } else {
#pragma unroll
        for (int m = 0; m < UNR; ++m)
#pragma unroll
          for (int k = 0; k < NR; ++k) uv[m][k] = u[c[m] + k];
      }
#pragma unroll
      for (int m = 0; m < UNR; ++m)
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[k] += a[m] * uv[m][k];
    }
  } else {
    const int K = row / blk;
    const int q = row - K * blk;
    const int j0 = ptr[K];
    const int nb = ptr[K + 1] - j0;
    const int64_t vbase = (int64_t)blk * blk * j0 + (int64_t)q * nb * blk;
    const int len = nb * blk;
    int j = lane / blk, c = lane - j * blk;
    const int sj = G / blk, sc = G - sj * blk;
    for (int p = lane; p < len; p += G) {
      const int64_t cc = ((int64_t)idx[j0 + j] * blk + c) * NR;
      const T a = val[vbase + p];
#pragma unroll
      for (int k = 0; k < NR; ++k) acc[k] += a * u[cc + k];
      j += sj;
      c += sc;
      if (c >= blk) { c -= blk; ++j; }
    }
  }
}

template <typename T, int NR, bool BLOCKED>
__global__ __launch_bounds__(256) void k_level(int n, int G, int blk, const int* __restrict__ ptr,
                                               const int* __restrict__ idx, const T* __restrict__ val,
                                               const T* __restrict__ u, const T* __restrict__ b, T* rho, T* x,
                                               const T* __restrict__ dinv, T* dout, T c1, T c2, int flags,
                                               const int* __restrict__ skip, int nlog) {
  if (skip && *skip) return;
  const int lb = xcd_block(nlog);
  if (lb < 0) return;
  const int rpb = 256 / G;
  const int lane = threadIdx.x & (G - 1);
  const int row = lb * rpb + threadIdx.x / G;
  const bool active = row < n;
  T acc[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = 0;
  if (active) row_product<T, NR, BLOCKED>(row, lane, G, blk, ptr, idx, val, u, acc);
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = wave_sum(acc[k], G);
  if (!active) return;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    if ((k & (G - 1)) != lane) continue;
    const int64_t i = (int64_t)row * NR + k;
    const T t = acc[k];
    if (flags & F_PLAIN) {
      rho[i] = t;
      continue;
    }
    const T r = ((flags & F_RHO_FROM_B) ? b[i] : rho[i]) - t;
    if (flags & F_RHO_STORE) rho[i] = r;
    const T ui = u[i];
    if (flags & F_X_ASSIGN)
      x[i] = ui;
    else if (flags & F_X_ADD)
      x[i] += ui;
    if (flags & F_D_OUT) dout[i] = c1 * ui + c2 * dinv[row] * r;
  }
}

template <typename T, int NR>
static void launch_level_nr(const LevelOp<T>& op, const T* u, const T* b, T* rho, T* x, T* dout, double c1,
                            double c2, int flags, const int* skip, hipStream_t s) {
  const int G = op.lanes;
  const int rpb = 256 / G;
  const int nlog = (op.n + rpb - 1) / rpb;
  if (nlog == 0) return;
  if (op.blk == 1)
    hipLaunchKernelGGL((k_level<T, NR, false>), dim3(xcd_grid(nlog)), dim3(256), 0, s, op.n, G, 1, op.ptr, op.idx,
                       op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2, flags, skip, nlog);
  else
    hipLaunchKernelGGL((k_level<T, NR, true>), dim3(xcd_grid(nlog)), dim3(256), 0, s, op.n, G, op.blk, op.ptr,
                       op.idx, op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2, flags, skip, nlog);
  check_launch("k_level");
}

template <typename T>
void launch_level(const LevelOp<T>& op, int nr, const T* u, const T* b, T* rho, T* x, T* dout, double c1,
                  double c2, int flags, const int* skip, hipStream_t s) {
  switch (nr) {
    case 1: launch_level_nr<T, 1>(op, u, b, rho, x, dout, c1, c2, flags, skip, s); break;
    case 2: launch_level_nr<T, 2>(op, u, b, rho, x, dout, c1, c2, flags, skip, s); break;
    case 4: launch_level_nr<T, 4>(op, u, b, rho, x, dout, c1, c2, flags, skip, s); break;
    case 8: launch_level_nr<T, 8>(op, u, b, rho, x, dout, c1, c2, flags, skip, s); break;
    case 16: launch_level_nr<T, 16>(op, u, b, rho, x, dout, c1, c2, flags, skip, s); break;
    default: throw std::runtime_error("unsupported nrhs block");
  }
}
template void launch_level<float>(const LevelOp<float>&, int, const float*, const float*, float*, float*, float*,
                                  double, double, int, const int*, hipStream_t);
template void launch_level<double>(const LevelOp<double>&, int, const double*, const double*, double*, double*,
                                   double*, double, double, int, const int*, hipStream_t);

// ==== fine-level row-block kernels ====

// Sum of the staged products prod[s..e) of one row by TPR consecutive lanes (TPR = 4 or 2) in one canonical
// order, the same for every row-block shape: a_v = prod[s+v] + prod[s+v+4] + ... (v = 0..3, in increasing
// position), row sum = (a_0 + a_2) + (a_1 + a_3).  With TPR = 2 each lane carries two of the four partial sums.
// Lane sub = 0 of the group holds the result.
// Matrix load of the fused level kernels: ordinary with KEEP (the level's matrix fits the caches and is applied
// again right away), nontemporal otherwise.  A compile-time choice: a run-time select between the two would be
// folded into one ordinary load.
template <bool KEEP, typename P>
__device__ inline P ld_matrix(const P* ptr) {
  if constexpr (KEEP)
    return *ptr;
  else
    return __builtin_nontemporal_load(ptr);
}

template <typename T, int TPR>
__device__ inline T row_sum_canonical(const T* prod, int s, int e, int sub) {
  static_assert(TPR == 4 || TPR == 2, "lanes per row");
  if constexpr (TPR == 4) {
    T a = 0;
    for (int k = s + sub; k < e; k += 4) a += prod[k];
    a += __shfl_xor(a, 2, 64);
    a += __shfl_xor(a, 1, 64);
    return a;
  } else {
    T a = 0, c = 0;
    for (int k = s + sub; k < e; k += 4) a += prod[k];
    for (int k = s + sub + 2; k < e; k += 4) c += prod[k];
    T t = a + c;
    t += __shfl_xor(t, 1, 64);
    return t;
  }
}

// Row-block ("stream") variant of the fused kernel for the CSR fine level, one right-hand side.  Each
// workgroup owns a host-computed block of <= RPB consecutive rows holding <= CAP - 3 nonzeros: phase 1 streams
// the block's values and column indices with fully coalesced loads (all issued before any gather) and stages
// val * u[col] in LDS, phase 2 sums each row with 256/RPB lanes and applies the same epilogue as k_level.  A row
// longer than CAP forms a block of its own and is summed by the whole workgroup.  With DOT the block also writes
// the partial sum of u_i (A u)_i (PCG's <p, A p>).  The (CAP, RPB) shape and the kernel form are chosen per
// matrix by timing.
template <typename T, bool DOT, int CAP, int RPB>
__global__ __launch_bounds__(256) void k_level_stream(int nrb, const int* __restrict__ rb, const int* __restrict__ ptr,
                                                      const int* __restrict__ idx, const T* __restrict__ val,
                                                      const T* __restrict__ u, const T* __restrict__ b, T* rho, T* x,
                                                      const T* __restrict__ dinv, T* dout, T c1, T c2, int flags,
                                                      const int* __restrict__ skip, double* partials) {
  constexpr int TPR = 256 / RPB;   // lanes per row in phase 2
  constexpr int EPT = CAP / 256;   // elements per thread in phase 1
  if (skip && *skip) return;
  const int lb = xcd_block(nrb);
  if (lb < 0) return;
  __shared__ T prod[CAP];
  __shared__ double sh[4];
  const int r0 = rb[lb], r1 = rb[lb + 1];
  const int e0 = ptr[r0], e1 = ptr[r1];
  const int nz = e1 - e0;
  // epilogue operands of the row this thread may finalise, fetched before the matrix stream
  const int prow = r0 + (threadIdx.x / TPR);
  const bool pre = (threadIdx.x % TPR) == 0 && prow < r1 && nz <= CAP && !(flags & F_PLAIN);
  T p_old = 0, p_x = 0, p_u = 0, p_di = 0;
  if (pre) {
    p_old = (flags & F_RHO_FROM_B) ? b[prow] : rho[prow];
    p_u = u[prow];
    if (flags & F_X_ADD) p_x = x[prow];
    if (flags & F_D_OUT) p_di = dinv[prow];
  }
  T t = 0;
  int row = -1;
  if (nz <= CAP) {
    // the matrix is streamed once per application: non-temporal loads keep u resident in the caches
    int ci[EPT];
    T vv[EPT];
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const int e = threadIdx.x + m * 256;
      if (e < nz) {
        ci[m] = __builtin_nontemporal_load(idx + e0 + e);
        vv[m] = __builtin_nontemporal_load(val + e0 + e);
      }
    }
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const int e = threadIdx.x + m * 256;
      if (e < nz) prod[e] = vv[m] * u[ci[m]];
    }
    __syncthreads();
    const int rl = threadIdx.x / TPR, sub = threadIdx.x % TPR;
    int s = 0, e = 0;
    if (r0 + rl < r1) {
      s = ptr[r0 + rl] - e0;
      e = ptr[r0 + rl + 1] - e0;
    }
    const T acc = row_sum_canonical<T, TPR>(prod, s, e, sub);
    if (sub == 0 && r0 + rl < r1) {
      row = r0 + rl;
      t = acc;
    }
  } else {  // one long row
    T acc = 0;
    for (int e = e0 + threadIdx.x; e < e1; e += 256) acc += val[e] * u[idx[e]];
    acc = wave_sum(acc, 64);
    __shared__ T shr[4];
    if ((threadIdx.x & 63) == 0) shr[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      row = r0;
      t = (shr[0] + shr[1]) + (shr[2] + shr[3]);
    }
  }
  double contrib = 0.0;
  if (row >= 0) {
    if (flags & F_PLAIN) {
      rho[row] = t;
      if (DOT) contrib = (double)t * (double)u[row];
    } else {
      if (!pre) {  // the long-row path did not prefetch
        p_old = (flags & F_RHO_FROM_B) ? b[row] : rho[row];
        p_u = u[row];
        if (flags & F_X_ADD) p_x = x[row];
        if (flags & F_D_OUT) p_di = dinv[row];
      }
      const T r = p_old - t;
      if (flags & F_RHO_STORE) rho[row] = r;
      if (flags & F_X_ASSIGN)
        x[row] = p_u;
      else if (flags & F_X_ADD)
        x[row] = p_x + p_u;
      if (flags & F_D_OUT) dout[row] = c1 * p_u + c2 * p_di * r;
    }
  }
  if (DOT) {
    const double s = block_sum256(contrib, sh);
    if (threadIdx.x == 0) partials[lb] = s;
  }
}

// Persistent, software-pipelined row-block kernel with 16-byte matrix loads.  Workgroup w owns the contiguous
// row blocks [w nrb / nwg, (w + 1) nrb / nwg) and, while it sums block i, has the matrix stream of block i + 1 in
// flight: per block the gathers of u and the per-row operands are issued before the next block's stream, so
// waiting for them (memory counters retire in order) never waits for the prefetch.  Products are staged in two
// alternating LDS buffers, so one barrier per block suffices.  (i) Each thread streams four consecutive entries per step, starting from the
// block's first entry rounded down to a multiple of four (entries outside the block are masked; the column and
// value arrays carry four padding entries at the end), and stages the four products with one aligned LDS write
// at their offset from that rounded start; (ii) each wave loads the row pointers of its rows once and spreads
// them with lane shuffles; (iii) the row sums go to LDS and the epilogue of a block runs one iteration later in
// wave 0, one row per lane with coalesced loads and stores (its operands are fetched before the next stream).
// Same summation order as the other row-block kernels.
template <typename T>
struct Vec4 {
  typedef T type __attribute__((ext_vector_type(4)));
};
typedef int i4v __attribute__((ext_vector_type(4)));

template <typename T, bool DOT, int CAP, int RPB>
__global__ __launch_bounds__(256) void k_level_stream_pv(int nrb, int nwg, const int* __restrict__ rb,
                                                         const int* __restrict__ ptr, const int* __restrict__ idx,
                                                         const T* __restrict__ val, const T* __restrict__ u,
                                                         const T* __restrict__ b, T* rho, T* x,
                                                         const T* __restrict__ dinv, T* dout, T c1, T c2, int flags,
                                                         const int* __restrict__ skip, double* partials) {
  using V4 = typename Vec4<T>::type;
  constexpr int TPR = 256 / RPB;  // lanes per row
  constexpr int RPW = 64 / TPR;   // rows per wave
  constexpr int NCH = CAP / 1024; // four-entry chunks per thread
  constexpr int EPL = RPB / 64;   // epilogue rows per lane of wave 0
  static_assert(RPB % 64 == 0 && CAP % 1024 == 0, "row-block shape");
  if (skip && *skip) return;
  const int w = xcd_block(nwg);
  if (w < 0) return;
  const int lbA = (int)((int64_t)w * nrb / nwg), lbB = (int)((int64_t)(w + 1) * nrb / nwg);
  __shared__ __align__(32) T prod[2][CAP];
  __shared__ T rsum[2][RPB];
  __shared__ T shr[2][4];
  __shared__ double sh[4];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rl = threadIdx.x / TPR, sub = threadIdx.x % TPR;
  double contrib = 0.0;
  int r0 = 0, r1 = 0, e0 = 0, e1 = 0;
  i4v ci[NCH];
  V4 vv[NCH];
  if (lbA < lbB) {
    r0 = rb[lbA];
    r1 = rb[lbA + 1];
    e0 = ptr[r0];
    e1 = ptr[r1];
    const int a0 = e0 & ~3;
    if (e1 - a0 <= CAP) {
#pragma unroll
      for (int m = 0; m < NCH; ++m) {
        const int e = a0 + 4 * (threadIdx.x + m * 256);
        if (e < e1) {
          ci[m] = __builtin_nontemporal_load(reinterpret_cast<const i4v*>(idx + e));
          vv[m] = __builtin_nontemporal_load(reinterpret_cast<const V4*>(val + e));
        }
      }
    }
  }
  int pr0 = 0, pr1 = 0;  // rows of the block whose epilogue is pending
  int it = 0;
  for (int lb = lbA; lb < lbB; ++lb, it ^= 1) {
    const int a0 = e0 & ~3;
    const bool staged = e1 - a0 <= CAP;
    // (a) everything this block and the pending epilogue still read
    V4 g[NCH];
    if (staged) {
#pragma unroll
      for (int m = 0; m < NCH; ++m) {
        const int e = a0 + 4 * (threadIdx.x + m * 256);
#pragma unroll
        for (int q = 0; q < 4; ++q) g[m][q] = (e + q >= e0 && e + q < e1) ? u[ci[m][q]] : (T)0;
      }
    }
    int rp = e1;
    if (lane <= RPW) {
      const int rr = r0 + wv * RPW + lane;
      rp = ptr[rr < r1 ? rr : r1];
    }
    T eo[EPL], eu[EPL], ex[EPL], ed[EPL];
#pragma unroll
    for (int q = 0; q < EPL; ++q) {
      eo[q] = eu[q] = ex[q] = ed[q] = 0;
      const int row = pr0 + lane + 64 * q;
      if (wv == 0 && row < pr1) {
        eu[q] = u[row];
        if (!(flags & F_PLAIN)) {
          eo[q] = (flags & F_RHO_FROM_B) ? b[row] : rho[row];
          if (flags & F_X_ADD) ex[q] = x[row];
          if (flags & F_D_OUT) ed[q] = dinv[row];
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    // (b) the next block's matrix stream
    int nr0 = 0, nr1 = 0, ne0 = 0, ne1 = 0;
    i4v nci[NCH];
    V4 nvv[NCH];
    if (lb + 1 < lbB) {
      nr0 = r1;
      nr1 = rb[lb + 2];
      ne0 = e1;
      ne1 = ptr[nr1];
      const int na0 = ne0 & ~3;
      if (ne1 - na0 <= CAP) {
#pragma unroll
        for (int m = 0; m < NCH; ++m) {
          const int e = na0 + 4 * (threadIdx.x + m * 256);
          if (e < ne1) {
            nci[m] = __builtin_nontemporal_load(reinterpret_cast<const i4v*>(idx + e));
            nvv[m] = __builtin_nontemporal_load(reinterpret_cast<const V4*>(val + e));
          }
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    // (c) row sums of this block into rsum[it]
    if (staged) {
#pragma unroll
      for (int m = 0; m < NCH; ++m) {
        const int e = a0 + 4 * (threadIdx.x + m * 256);
        if (e < e1) *reinterpret_cast<V4*>(&prod[it][e - a0]) = vv[m] * g[m];
      }
      const int rs = __shfl(rp, lane / TPR, 64), re = __shfl(rp, lane / TPR + 1, 64);
      __syncthreads();
      const T acc = row_sum_canonical<T, TPR>(prod[it], rs - a0, re - a0, sub);
      if (sub == 0) rsum[it][rl] = acc;
    } else {  // one long row
      T acc = 0;
      for (int e = e0 + threadIdx.x; e < e1; e += 256) acc += val[e] * u[idx[e]];
      acc = wave_sum(acc, 64);
      if (lane == 0) shr[it][wv] = acc;
      __syncthreads();
      if (threadIdx.x == 0) rsum[it][0] = (shr[it][0] + shr[it][1]) + (shr[it][2] + shr[it][3]);
    }
    // (d) epilogue of the previous block (its row sums were published by the barrier above)
    if (wv == 0) {
#pragma unroll
      for (int q = 0; q < EPL; ++q) {
        const int row = pr0 + lane + 64 * q;
        if (row < pr1) {
          const T t = rsum[it ^ 1][lane + 64 * q];
          if (flags & F_PLAIN) {
            rho[row] = t;
            if (DOT) contrib += (double)t * (double)eu[q];
          } else {
            const T r = eo[q] - t;
            if (flags & F_RHO_STORE) rho[row] = r;
            if (flags & F_X_ASSIGN)
              x[row] = eu[q];
            else if (flags & F_X_ADD)
              x[row] = ex[q] + eu[q];
            if (flags & F_D_OUT) dout[row] = c1 * eu[q] + c2 * ed[q] * r;
          }
        }
      }
    }
    pr0 = r0;
    pr1 = r1;
    r0 = nr0;
    r1 = nr1;
    e0 = ne0;
    e1 = ne1;
#pragma unroll
    for (int m = 0; m < NCH; ++m) {
      ci[m] = nci[m];
      vv[m] = nvv[m];
    }
  }
  // epilogue of the last block
  __syncthreads();
  if (wv == 0) {
#pragma unroll
    for (int q = 0; q < EPL; ++q) {
      const int row = pr0 + lane + 64 * q;
      if (row < pr1) {
        const T t = rsum[it ^ 1][lane + 64 * q];
        const T uu = u[row];
        if (flags & F_PLAIN) {
          rho[row] = t;
          if (DOT) contrib += (double)t * (double)uu;
        } else {
          const T r = ((flags & F_RHO_FROM_B) ? b[row] : rho[row]) - t;
          if (flags & F_RHO_STORE) rho[row] = r;
          if (flags & F_X_ASSIGN)
            x[row] = uu;
          else if (flags & F_X_ADD)
            x[row] = x[row] + uu;
          if (flags & F_D_OUT) dout[row] = c1 * uu + c2 * dinv[row] * r;
        }
      }
    }
  }
  if (DOT) {
    const double s = block_sum256(contrib, sh);
    if (threadIdx.x == 0) partials[w] = s;
  }
}

// Local-column row-block kernel (one workgroup per block).  The block's distinct columns are gathered once into
// LDS (us); the matrix stream then carries the values and 1- or 2-byte positions into that list instead of 4-byte
// column indices, and each product reads its u entry from LDS.  Phase 2 and the epilogue are those of
// k_level_stream, with the same summation order.  A block with more than UCAP distinct columns is a single row,
// summed by the whole workgroup through the CSR columns.
template <typename T, typename IX, bool DOT, int CAP, int RPB, int UCAP>
__global__ __launch_bounds__(256) void k_level_local(int nrb, const int* __restrict__ rb, const int* __restrict__ ubp,
                                                     const int* __restrict__ ucol, const IX* __restrict__ lidx,
                                                     const int* __restrict__ ptr, const int* __restrict__ idx,
                                                     const T* __restrict__ val, const T* __restrict__ u,
                                                     const T* __restrict__ b, T* rho, T* x,
                                                     const T* __restrict__ dinv, T* dout, T c1, T c2, int flags,
                                                     const int* __restrict__ skip, double* partials) {
  constexpr int TPR = 256 / RPB;
  constexpr int EPT = CAP / 256;
  constexpr int UPT = (UCAP + 255) / 256;
  if (skip && *skip) return;
  const int lb = xcd_block(nrb);
  if (lb < 0) return;
  __shared__ T us[UCAP];
  __shared__ T prod[CAP];
  __shared__ double sh[4];
  const int r0 = rb[lb], r1 = rb[lb + 1];
  const int e0 = ptr[r0], e1 = ptr[r1];
  const int nz = e1 - e0;
  const int u0 = ubp[lb], nu = ubp[lb + 1] - u0;
  const bool staged = nu <= UCAP;
  const int prow = r0 + (threadIdx.x / TPR);
  const bool pre = (threadIdx.x % TPR) == 0 && prow < r1 && staged && !(flags & F_PLAIN);
  T p_old = 0, p_x = 0, p_u = 0, p_di = 0;
  if (pre) {
    p_old = (flags & F_RHO_FROM_B) ? b[prow] : rho[prow];
    p_u = u[prow];
    if (flags & F_X_ADD) p_x = x[prow];
    if (flags & F_D_OUT) p_di = dinv[prow];
  }
  T t = 0;
  int row = -1;
  if (staged) {
    T ug[UPT];
#pragma unroll
    for (int m = 0; m < UPT; ++m) {
      const int c = threadIdx.x + m * 256;
      if (c < nu) ug[m] = u[ucol[u0 + c]];
    }
    IX li[EPT];
    T vv[EPT];
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const int e = threadIdx.x + m * 256;
      if (e < nz) {
        li[m] = __builtin_nontemporal_load(lidx + e0 + e);
        vv[m] = __builtin_nontemporal_load(val + e0 + e);
      }
    }
#pragma unroll
    for (int m = 0; m < UPT; ++m) {
      const int c = threadIdx.x + m * 256;
      if (c < nu) us[c] = ug[m];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const int e = threadIdx.x + m * 256;
      if (e < nz) prod[e] = vv[m] * us[li[m]];
    }
    __syncthreads();
    const int rl = threadIdx.x / TPR, sub = threadIdx.x % TPR;
    int s = 0, e = 0;
    if (r0 + rl < r1) {
      s = ptr[r0 + rl] - e0;
      e = ptr[r0 + rl + 1] - e0;
    }
    const T acc = row_sum_canonical<T, TPR>(prod, s, e, sub);
    if (sub == 0 && r0 + rl < r1) {
      row = r0 + rl;
      t = acc;
    }
  } else {  // one long row
    T acc = 0;
    for (int e = e0 + threadIdx.x; e < e1; e += 256) acc += val[e] * u[idx[e]];
    acc = wave_sum(acc, 64);
    __shared__ T shr[4];
    if ((threadIdx.x & 63) == 0) shr[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      row = r0;
      t = (shr[0] + shr[1]) + (shr[2] + shr[3]);
    }
  }
  double contrib = 0.0;
  if (row >= 0) {
    if (flags & F_PLAIN) {
      rho[row] = t;
      if (DOT) contrib = (double)t * (double)u[row];
    } else {
      if (!pre) {
        p_old = (flags & F_RHO_FROM_B) ? b[row] : rho[row];
        p_u = u[row];
        if (flags & F_X_ADD) p_x = x[row];
        if (flags & F_D_OUT) p_di = dinv[row];
      }
      const T r = p_old - t;
      if (flags & F_RHO_STORE) rho[row] = r;
      if (flags & F_X_ASSIGN)
        x[row] = p_u;
      else if (flags & F_X_ADD)
        x[row] = p_x + p_u;
      if (flags & F_D_OUT) dout[row] = c1 * p_u + c2 * p_di * r;
    }
  }
  if (DOT) {
    const double s = block_sum256(contrib, sh);
    if (threadIdx.x == 0) partials[lb] = s;
  }
}

// Local-column kernel with vector loads (1-byte column positions, one workgroup per block).  As k_level_local,
// but each thread streams four consecutive entries per step (16-byte value loads, 4-byte loads of four packed
// positions) from the block's first entry rounded down to a multiple of four (outside entries masked; values and
// positions carry kFinePad padding entries), stages the four products with one aligned LDS write, and each wave
// loads its rows' row pointers once and spreads them with lane shuffles.
template <typename T, int CAP, int RPB, int UCAP, bool KEEP>
__global__ __launch_bounds__(256) void k_level_local_vec(int nrb, const int4* __restrict__ meta,
                                                         const int* __restrict__ ucol,
                                                         const uint8_t* __restrict__ lidx, const int* __restrict__ ptr,
                                                         const int* __restrict__ idx, const T* __restrict__ val,
                                                         const T* __restrict__ u, const T* __restrict__ b, T* rho,
                                                         T* x, const T* __restrict__ dinv, T* dout, T c1, T c2,
                                                         int flags, const int* __restrict__ skip) {
  using V4 = typename Vec4<T>::type;
  constexpr int TPR = 256 / RPB;
  constexpr int RPW = 64 / TPR;
  constexpr int NCH = CAP / 1024;
  constexpr int UPT = UCAP / 256;
  static_assert(CAP % 1024 == 0 && UCAP % 256 == 0, "local block shape");
  if (skip && *skip) return;
  const int lb = xcd_block(nrb);
  if (lb < 0) return;
  __shared__ T us[UCAP];
  __shared__ __align__(32) T prod[CAP];
  __shared__ T shr[4];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // first row, first nonzero and first distinct column of this block and of the next (one round trip)
  const int4 m0 = meta[lb], m1 = meta[lb + 1];
  const int r0 = m0.x, r1 = m1.x;
  const int e0 = m0.y, e1 = m1.y;
  const int u0 = m0.z, nu = m1.z - u0;
  const bool staged = nu <= UCAP;
  const int rl = threadIdx.x / TPR, sub = threadIdx.x % TPR;
  const int prow = r0 + rl;
  // The loads below are unconditional per thread (clamped addresses; out-of-range values are never used): loads
  // under lane-dependent branches are waited for at the branch's end, which put the block's value stream behind
  // its column list.  Here the column list, values, positions and row pointers are in flight together, and only
  // the gather of u waits for the column list.
  const int prc = min(prow, r1 - 1);  // blocks hold at least one row
  T p_old = 0, p_x = 0, p_u = 0, p_di = 0;
  if (!(flags & F_PLAIN)) {
    p_old = (flags & F_RHO_FROM_B) ? b[prc] : rho[prc];
    p_u = u[prc];
    if (flags & F_X_ADD) p_x = x[prc];
    if (flags & F_D_OUT) p_di = dinv[prc];
  }
  T t = 0;
  if (staged) {
    int uc[UPT];
#pragma unroll
    for (int m = 0; m < UPT; ++m) uc[m] = ucol[u0 + min((int)threadIdx.x + m * 256, nu - 1)];  // nu >= 1
    const int a0 = e0 & ~3;
    uint32_t li[NCH];
    V4 vv[NCH];
#pragma unroll
    for (int m = 0; m < NCH; ++m) {
      const int e = a0 + 4 * (threadIdx.x + m * 256);
      const int ec = e < e1 ? e : a0;
      li[m] = ld_matrix<KEEP>(reinterpret_cast<const uint32_t*>(lidx + ec));
      vv[m] = ld_matrix<KEEP>(reinterpret_cast<const V4*>(val + ec));
    }
    const int rp = ptr[min(r0 + wv * RPW + min(lane, RPW), r1)];  // lanes 0..RPW: this wave's row pointers
    // slots nu .. UCAP-1 take copies and are never read (positions are below nu); no branch lets the gather sink
#pragma unroll
    for (int m = 0; m < UPT; ++m) us[threadIdx.x + m * 256] = u[uc[m]];
    // keep the streamed entries ahead of the barrier (the compiler would otherwise sink some loads past it)
#pragma unroll
    for (int m = 0; m < NCH; ++m) {
      asm volatile("" ::"v"(li[m]));
#pragma unroll
      for (int q = 0; q < 4; ++q) asm volatile("" ::"v"(vv[m][q]));
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NCH; ++m) {
      const int e = a0 + 4 * (threadIdx.x + m * 256);
      if (e < e1) {
        V4 g;
#pragma unroll
        for (int q = 0; q < 4; ++q) g[q] = (e + q >= e0 && e + q < e1) ? us[(li[m] >> (8 * q)) & 0xff] : (T)0;
        *reinterpret_cast<V4*>(&prod[e - a0]) = vv[m] * g;
      }
    }
    const int rs = __shfl(rp, lane / TPR, 64), re = __shfl(rp, lane / TPR + 1, 64);
    __syncthreads();
    t = row_sum_canonical<T, TPR>(prod, rs - a0, re - a0, sub);
  } else {  // one long row
    T acc = 0;
    for (int e = e0 + threadIdx.x; e < e1; e += 256) acc += val[e] * u[idx[e]];
    acc = wave_sum(acc, 64);
    if (lane == 0) shr[wv] = acc;
    __syncthreads();
    t = (shr[0] + shr[1]) + (shr[2] + shr[3]);
  }
  if (sub == 0 && prow < r1 && (staged || rl == 0)) {
    const int row = prow;
    if (flags & F_PLAIN) {
      rho[row] = t;
    } else {
      const T r = p_old - t;
      if (flags & F_RHO_STORE) rho[row] = r;
      if (flags & F_X_ASSIGN)
        x[row] = p_u;
      else if (flags & F_X_ADD)
        x[row] = p_x + p_u;
      if (flags & F_D_OUT) dout[row] = c1 * p_u + c2 * p_di * r;
    }
  }
}

// The same over pairs of blocks: a workgroup takes NB = 2 consecutive blocks and issues the loads of both before
// the first barrier, so that two blocks' streams are in flight per workgroup; each block is summed exactly as by
// k_level_local_vec.
template <typename T, int CAP, int RPB, int UCAP, bool KEEP, int NB>
__global__ __launch_bounds__(256) void k_level_local_vec_nb(int nrb, const int4* __restrict__ meta,
                                                         const int* __restrict__ ucol,
                                                         const uint8_t* __restrict__ lidx, const int* __restrict__ ptr,
                                                         const int* __restrict__ idx, const T* __restrict__ val,
                                                         const T* __restrict__ u, const T* __restrict__ b, T* rho,
                                                         T* x, const T* __restrict__ dinv, T* dout, T c1, T c2,
                                                         int flags, const int* __restrict__ skip) {
  using V4 = typename Vec4<T>::type;
  constexpr int TPR = 256 / RPB;
  constexpr int RPW = 64 / TPR;
  constexpr int NCH = CAP / 1024;
  constexpr int UPT = UCAP / 256;
  static_assert(CAP % 1024 == 0 && UCAP % 256 == 0 && (NB == 1 || NB == 2), "local block shape");
  if (skip && *skip) return;
  const int lg = xcd_block((nrb + NB - 1) / NB);
  if (lg < 0) return;
  __shared__ T us[NB][UCAP];
  __shared__ __align__(32) T prod[NB][CAP];
  __shared__ T shr[NB][4];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rl = threadIdx.x / TPR, sub = threadIdx.x % TPR;
  // per block: first row, first nonzero and first distinct column of it and of the next (one round trip); a
  // missing second block (odd nrb) repeats the last one and stores nothing
  int r0[NB], r1[NB], e0[NB], e1[NB], u0[NB], nu[NB];
  bool live[NB];
#pragma unroll
  for (int h = 0; h < NB; ++h) {
    live[h] = lg * NB + h < nrb;
    const int lb = min(lg * NB + h, nrb - 1);
    const int4 m0 = meta[lb], m1 = meta[lb + 1];
    r0[h] = m0.x;
    r1[h] = m1.x;
    e0[h] = m0.y;
    e1[h] = m1.y;
    u0[h] = m0.z;
    nu[h] = m1.z - m0.z;
  }
  // The loads below are unconditional per thread (clamped addresses; out-of-range values are never used): loads
  // under lane-dependent branches are waited for at the branch's end, which put the block's value stream behind
  // its column list.  Here the column list, values, positions and row pointers are in flight together, and only
  // the gather of u waits for the column list.
  T p_old[NB], p_x[NB], p_u[NB], p_di[NB];
#pragma unroll
  for (int h = 0; h < NB; ++h) {
    const int prc = min(r0[h] + rl, r1[h] - 1);  // blocks hold at least one row
    p_old[h] = p_x[h] = p_u[h] = p_di[h] = 0;
    if (!(flags & F_PLAIN)) {
      p_old[h] = (flags & F_RHO_FROM_B) ? b[prc] : rho[prc];
      p_u[h] = u[prc];
      if (flags & F_X_ADD) p_x[h] = x[prc];
      if (flags & F_D_OUT) p_di[h] = dinv[prc];
    }
  }
  int uc[NB][UPT];
  uint32_t li[NB][NCH];
  V4 vv[NB][NCH];
  int rp[NB];
#pragma unroll
  for (int h = 0; h < NB; ++h) {
    if (nu[h] > UCAP) continue;  // one long row, summed below (uniform over the workgroup)
#pragma unroll
    for (int m = 0; m < UPT; ++m) uc[h][m] = ucol[u0[h] + min((int)threadIdx.x + m * 256, nu[h] - 1)];  // nu >= 1
    const int a0 = e0[h] & ~3;
#pragma unroll
    for (int m = 0; m < NCH; ++m) {
      const int e = a0 + 4 * (threadIdx.x + m * 256);
      const int ec = e < e1[h] ? e : a0;
      li[h][m] = ld_matrix<KEEP>(reinterpret_cast<const uint32_t*>(lidx + ec));
      vv[h][m] = ld_matrix<KEEP>(reinterpret_cast<const V4*>(val + ec));
    }
    rp[h] = ptr[min(r0[h] + wv * RPW + min(lane, RPW), r1[h])];  // lanes 0..RPW: this wave's row pointers
  }
  // slots nu .. UCAP-1 take copies and are never read (positions are below nu); no branch lets the gather sink
#pragma unroll
  for (int h = 0; h < NB; ++h) {
    if (nu[h] > UCAP) continue;
#pragma unroll
    for (int m = 0; m < UPT; ++m) us[h][threadIdx.x + m * 256] = u[uc[h][m]];
  }
  // keep the streamed entries ahead of the barrier (the compiler would otherwise sink some loads past it)
#pragma unroll
  for (int h = 0; h < NB; ++h) {
    if (nu[h] > UCAP) continue;
#pragma unroll
    for (int m = 0; m < NCH; ++m) {
      asm volatile("" ::"v"(li[h][m]));
#pragma unroll
      for (int q = 0; q < 4; ++q) asm volatile("" ::"v"(vv[h][m][q]));
    }
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < NB; ++h) {
    if (nu[h] > UCAP) continue;
    const int a0 = e0[h] & ~3;
#pragma unroll
    for (int m = 0; m < NCH; ++m) {
      const int e = a0 + 4 * (threadIdx.x + m * 256);
      if (e < e1[h]) {
        V4 g;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          g[q] = (e + q >= e0[h] && e + q < e1[h]) ? us[h][(li[h][m] >> (8 * q)) & 0xff] : (T)0;
        *reinterpret_cast<V4*>(&prod[h][e - a0]) = vv[h][m] * g;
      }
    }
  }
  __syncthreads();
  T t[NB];
#pragma unroll
  for (int h = 0; h < NB; ++h) {
    if (nu[h] <= UCAP) {
      const int a0 = e0[h] & ~3;
      const int rs = __shfl(rp[h], lane / TPR, 64), re = __shfl(rp[h], lane / TPR + 1, 64);
      t[h] = row_sum_canonical<T, TPR>(prod[h], rs - a0, re - a0, sub);
    } else {  // one long row
      T acc = 0;
      for (int e = e0[h] + threadIdx.x; e < e1[h]; e += 256) acc += val[e] * u[idx[e]];
      acc = wave_sum(acc, 64);
      if (lane == 0) shr[h][wv] = acc;
      __syncthreads();
      t[h] = (shr[h][0] + shr[h][1]) + (shr[h][2] + shr[h][3]);
    }
  }
#pragma unroll
  for (int h = 0; h < NB; ++h) {
    const bool staged = nu[h] <= UCAP;
    const int row = r0[h] + rl;
    if (!live[h] || sub != 0 || row >= r1[h] || !(staged || rl == 0)) continue;
    if (flags & F_PLAIN) {
      rho[row] = t[h];
    } else {
      const T r = p_old[h] - t[h];
      if (flags & F_RHO_STORE) rho[row] = r;
      if (flags & F_X_ASSIGN)
        x[row] = p_u[h];
      else if (flags & F_X_ADD)
        x[row] = p_x[h] + p_u[h];
      if (flags & F_D_OUT) dout[row] = c1 * p_u[h] + c2 * p_di[h] * r;
    }
  }
}

template <typename T, int CAP, int RPB>
static int launch_stream_block(const FineBlocks& fb, const LevelOp<T>& op, const T* u, const T* b, T* rho, T* x,
                               T* dout, double c1, double c2, int flags, const int* skip, double* partials,
                               hipStream_t s) {
  const int nrb = fb.nrb;
  if (partials)
    hipLaunchKernelGGL((k_level_stream<T, true, CAP, RPB>), dim3(xcd_grid(nrb)), dim3(256), 0, s, nrb, fb.rb, op.ptr,
                       op.idx, op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2, flags, skip, partials);
  else
    hipLaunchKernelGGL((k_level_stream<T, false, CAP, RPB>), dim3(xcd_grid(nrb)), dim3(256), 0, s, nrb, fb.rb, op.ptr,
                       op.idx, op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2, flags, skip, partials);
  return nrb;
}

// workgroups of a persistent kernel: as many as are resident at once on the device (capped by the work)
template <typename K>
static int resident_groups(K kernel) {
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess ||
      hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    throw std::runtime_error("occupancy query of the pipelined row-block kernel failed");
  return std::max(1, per_cu) * std::max(1, cus);
}

template <typename T, bool DOT, int CAP, int RPB>
static int pipe_groups(int nrb) {
  static const int g = resident_groups(k_level_stream_pv<T, DOT, CAP, RPB>);
  return std::min(nrb, g);
}

template <typename T, int CAP, int RPB>
static int launch_stream_pipe(const FineBlocks& fb, const LevelOp<T>& op, const T* u, const T* b, T* rho, T* x,
                              T* dout, double c1, double c2, int flags, const int* skip, double* partials,
                              hipStream_t s) {
  const int nrb = fb.nrb;
  const int nwg = partials ? pipe_groups<T, true, CAP, RPB>(nrb) : pipe_groups<T, false, CAP, RPB>(nrb);
  const dim3 grid(xcd_grid(nwg));
  if (partials)
    hipLaunchKernelGGL((k_level_stream_pv<T, true, CAP, RPB>), grid, dim3(256), 0, s, nrb, nwg, fb.rb, op.ptr, op.idx,
                       op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2, flags, skip, partials);
  else
    hipLaunchKernelGGL((k_level_stream_pv<T, false, CAP, RPB>), grid, dim3(256), 0, s, nrb, nwg, fb.rb, op.ptr,
                       op.idx, op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2, flags, skip, partials);
  return nwg;
}

template <typename T, typename IX, int CAP, int RPB, int UCAP>
static int launch_stream_local(const FineBlocks& fb, const LevelOp<T>& op, const T* u, const T* b, T* rho, T* x,
                               T* dout, double c1, double c2, int flags, const int* skip, double* partials,
                               hipStream_t s) {
  const int nrb = fb.nrb;
  const IX* li = static_cast<const IX*>(fb.lidx);
  if (partials)
    hipLaunchKernelGGL((k_level_local<T, IX, true, CAP, RPB, UCAP>), dim3(xcd_grid(nrb)), dim3(256), 0, s, nrb, fb.rb,
                       fb.ubp, fb.ucol, li, op.ptr, op.idx, op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2, flags,
                       skip, partials);
  else
    hipLaunchKernelGGL((k_level_local<T, IX, false, CAP, RPB, UCAP>), dim3(xcd_grid(nrb)), dim3(256), 0, s, nrb,
                       fb.rb, fb.ubp, fb.ucol, li, op.ptr, op.idx, op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2,
                       flags, skip, partials);
  return nrb;
}

template <typename T, int CAP, int RPB, int UCAP, int NB>
static int launch_stream_local_vec(const FineBlocks& fb, const LevelOp<T>& op, const T* u, const T* b, T* rho, T* x,
                                   T* dout, double c1, double c2, int flags, const int* skip, double* partials,
                                   hipStream_t s) {
  if (partials) throw std::runtime_error("local-column vector kernel: no partial sums");
  const int nrb = fb.nrb;
  if (!fb.meta) throw std::runtime_error("local-column vector kernel: block records missing");
  const int4* meta = reinterpret_cast<const int4*>(fb.meta);
  const uint8_t* lidx = static_cast<const uint8_t*>(fb.lidx);
  if constexpr (NB == 1) {
    if (flags & F_KEEP)
      hipLaunchKernelGGL((k_level_local_vec<T, CAP, RPB, UCAP, true>), dim3(xcd_grid(nrb)), dim3(256), 0, s, nrb, meta,
                         fb.ucol, lidx, op.ptr, op.idx, op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2, flags, skip);
    else
      hipLaunchKernelGGL((k_level_local_vec<T, CAP, RPB, UCAP, false>), dim3(xcd_grid(nrb)), dim3(256), 0, s, nrb,
                         meta, fb.ucol, lidx, op.ptr, op.idx, op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2, flags,
                         skip);
  } else {
    const dim3 grid(xcd_grid((nrb + NB - 1) / NB));
    if (flags & F_KEEP)
      hipLaunchKernelGGL((k_level_local_vec_nb<T, CAP, RPB, UCAP, true, NB>), grid, dim3(256), 0, s, nrb, meta, fb.ucol,
                         lidx, op.ptr, op.idx, op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2, flags, skip);
    else
      hipLaunchKernelGGL((k_level_local_vec_nb<T, CAP, RPB, UCAP, false, NB>), grid, dim3(256), 0, s, nrb, meta,
                         fb.ucol, lidx, op.ptr, op.idx, op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2, flags, skip);
  }
  return nrb;
}

template <typename T>
int launch_level_stream(int shape, const FineBlocks& fb, const LevelOp<T>& op, const T* u, const T* b, T* rho, T* x,
                        T* dout, double c1, double c2, int flags, const int* skip, double* partials, hipStream_t s) {
  if (fb.nrb == 0) return 0;
  int np = 0;
#define R3MG_ARGS fb, op, u, b, rho, x, dout, c1, c2, flags, skip, partials, s
  switch (shape) {
    case 0: np = launch_stream_block<T, 2048, 64>(R3MG_ARGS); break;
    case 1: np = launch_stream_block<T, 4096, 128>(R3MG_ARGS); break;
    case 2: np = launch_stream_block<T, 4096, 64>(R3MG_ARGS); break;
    case 3: np = launch_stream_pipe<T, 2048, 64>(R3MG_ARGS); break;
    case 4: np = launch_stream_pipe<T, 4096, 128>(R3MG_ARGS); break;
    case 5: np = launch_stream_pipe<T, 4096, 64>(R3MG_ARGS); break;
    case 6: np = launch_stream_local<T, uint8_t, 2048, 64, 256>(R3MG_ARGS); break;
    case 7: np = launch_stream_local<T, uint16_t, 4096, 64, 1024>(R3MG_ARGS); break;
    case 8: np = launch_stream_local<T, uint16_t, 4096, 128, 1024>(R3MG_ARGS); break;
    case 9: np = launch_stream_local_vec<T, 2048, 64, 256, 1>(R3MG_ARGS); break;
    case 10: np = launch_stream_local_vec<T, 3072, 128, 256, 1>(R3MG_ARGS); break;
    case 11: np = launch_stream_local_vec<T, 2048, 64, 256, 2>(R3MG_ARGS); break;
    case 12: np = launch_stream_local_vec<T, 3072, 128, 256, 2>(R3MG_ARGS); break;
    case 13: np = launch_stream_local_vec<T, 3072, 64, 256, 1>(R3MG_ARGS); break;
    default: throw std::runtime_error("unknown row-block shape");
  }
#undef R3MG_ARGS
  check_launch("k_level_stream");
  return np;
}
template int launch_level_stream<float>(int, const FineBlocks&, const LevelOp<float>&, const float*, const float*,
                                        float*, float*, float*, double, double, int, const int*, double*, hipStream_t);
template int launch_level_stream<double>(int, const FineBlocks&, const LevelOp<double>&, const double*,
                                         const double*, double*, double*, double*, double, double, int, const int*,
                                         double*, hipStream_t);
// ==== end of fine-level row-block kernels ====

// Multi-right-hand-side CSR kernel with the columns split over lanes (NR columns, interleaved n x NR vectors).
// G lanes per row (G a power of two, NG <= G <= 64, NG = NR / GW, GW = 16 / sizeof(T)): lane (j, s) owns the
// column group j (GW consecutive columns, one 16-byte load per nonzero) and the row's entries s, s + G/NG, ...;
// so the NG lanes of one nonzero read its u row as consecutive 16-byte pieces.  The G/NG entry lanes of a group
// are combined by a butterfly and lane s = 0 applies the epilogue of k_level to its GW columns.
template <typename T, int NR>
__global__ __launch_bounds__(256) void k_level_split(int n, int G, const int* __restrict__ ptr,
                                                     const int* __restrict__ idx, const T* __restrict__ val,
                                                     const T* __restrict__ u, const T* __restrict__ b, T* rho, T* x,
                                                     const T* __restrict__ dinv, T* dout, T c1, T c2, int flags,
                                                     const int* __restrict__ skip, int nlog) {
  constexpr int GW = 16 / (int)sizeof(T);
  constexpr int NG = NR / GW;
  constexpr int UNR = 4;
  static_assert(NR % GW == 0, "column groups");
  typedef T VG __attribute__((ext_vector_type(GW)));
  if (skip && *skip) return;
  const int lb = xcd_block(nlog);
  if (lb < 0) return;
  const int rpb = 256 / G;
  const int li = threadIdx.x % G;
  const int j = li % NG, sv = li / NG, S = G / NG;
  const int row = lb * rpb + threadIdx.x / G;
  VG acc = (VG)0;
  if (row < n) {
    const int s = ptr[row], e = ptr[row + 1];
    for (int p0 = s + sv; p0 < e; p0 += UNR * S) {
      T a[UNR];
      int64_t c[UNR];
#pragma unroll
      for (int m = 0; m < UNR; ++m) {
        const int p = p0 + m * S;
        a[m] = p < e ? val[p] : (T)0;
        c[m] = p < e ? (int64_t)idx[p] * NR + j * GW : j * GW;
      }
      VG uv[UNR];
#pragma unroll
      for (int m = 0; m < UNR; ++m) uv[m] = *reinterpret_cast<const VG*>(u + c[m]);
#pragma unroll
      for (int m = 0; m < UNR; ++m) acc += a[m] * uv[m];
    }
  }
  for (int off = NG; off < G; off <<= 1)
#pragma unroll
    for (int w = 0; w < GW; ++w) acc[w] += __shfl_xor(acc[w], off, 64);
  if (sv == 0 && row < n) {
    const int64_t o = (int64_t)row * NR + j * GW;
    if (flags & F_PLAIN) {
      *reinterpret_cast<VG*>(rho + o) = acc;
    } else {
      const VG old = (flags & F_RHO_FROM_B) ? *reinterpret_cast<const VG*>(b + o) : *reinterpret_cast<VG*>(rho + o);
      const VG r = old - acc;
      if (flags & F_RHO_STORE) *reinterpret_cast<VG*>(rho + o) = r;
      const VG ui = *reinterpret_cast<const VG*>(u + o);
      if (flags & F_X_ASSIGN)
        *reinterpret_cast<VG*>(x + o) = ui;
      else if (flags & F_X_ADD)
        *reinterpret_cast<VG*>(x + o) = *reinterpret_cast<VG*>(x + o) + ui;
      if (flags & F_D_OUT) *reinterpret_cast<VG*>(dout + o) = c1 * ui + (c2 * dinv[row]) * r;
    }
  }
}

// The same product with each nonzero's value and column read once: the G lanes of a row load G consecutive
// entries of the row at a time (one value and one column each, coalesced), then NG steps follow in which lane
// (s, j) takes entry t S + s of that chunk from its owner lane by a shuffle and reads column group j of the
// entry's u row (16 bytes).  Per G entries a lane issues 2 + NG loads instead of 3 per entry it owns, which
// halves the address work of the gathers' texture-address unit.  Same epilogue as k_level_split.
template <typename T, int NR>
__global__ __launch_bounds__(256) void k_level_split2(int n, int G, const int* __restrict__ ptr,
                                                      const int* __restrict__ idx, const T* __restrict__ val,
                                                      const T* __restrict__ u, const T* __restrict__ b, T* rho, T* x,
                                                      const T* __restrict__ dinv, T* dout, T c1, T c2, int flags,
                                                      const int* __restrict__ skip, int nlog) {
  constexpr int GW = 16 / (int)sizeof(T);
  constexpr int NG = NR / GW;
  static_assert(NR % GW == 0, "column groups");
  typedef T VG __attribute__((ext_vector_type(GW)));
  if (skip && *skip) return;
  const int lb = xcd_block(nlog);
  if (lb < 0) return;
  const int rpb = 256 / G;
  const int li = threadIdx.x % G;
  const int gbase = (int)(threadIdx.x & 63) - li;  // the row group's first lane in the wave
  const int j = li % NG, sv = li / NG, S = G / NG;
  const int row = lb * rpb + threadIdx.x / G;
  VG acc = (VG)0;
  int s = 0, e = 0;
  if (row < n) {
    s = ptr[row];
    e = ptr[row + 1];
  }
  // every lane of a row group runs the same chunks, so a shuffle only ever reads an active lane of its group
  for (int c0 = s; c0 < e; c0 += G) {
    const int p = c0 + li;
    const T a_l = p < e ? val[p] : (T)0;
    const int i_l = p < e ? idx[p] : 0;
#pragma unroll
    for (int t = 0; t < NG; ++t) {
      const int src = gbase + t * S + sv;
      const T a = __shfl(a_l, src, 64);
      const int64_t ci = (int64_t)__shfl(i_l, src, 64);
      const VG uv = *reinterpret_cast<const VG*>(u + ci * NR + j * GW);
      acc += a * uv;
    }
  }
  for (int off = NG; off < G; off <<= 1)
#pragma unroll
    for (int w = 0; w < GW; ++w) acc[w] += __shfl_xor(acc[w], off, 64);
  if (sv == 0 && row < n) {
    const int64_t o = (int64_t)row * NR + j * GW;
    if (flags & F_PLAIN) {
      *reinterpret_cast<VG*>(rho + o) = acc;
    } else {
      const VG old = (flags & F_RHO_FROM_B) ? *reinterpret_cast<const VG*>(b + o) : *reinterpret_cast<VG*>(rho + o);
      const VG r = old - acc;
      if (flags & F_RHO_STORE) *reinterpret_cast<VG*>(rho + o) = r;
      const VG ui = *reinterpret_cast<const VG*>(u + o);
      if (flags & F_X_ASSIGN)
        *reinterpret_cast<VG*>(x + o) = ui;
      else if (flags & F_X_ADD)
        *reinterpret_cast<VG*>(x + o) = *reinterpret_cast<VG*>(x + o) + ui;
      if (flags & F_D_OUT) *reinterpret_cast<VG*>(dout + o) = c1 * ui + (c2 * dinv[row]) * r;
    }
  }
}

template <typename T>
bool launch_level_split2(const LevelOp<T>& op, int nr, int G, const T* u, const T* b, T* rho, T* x, T* dout,
                         double c1, double c2, int flags, const int* skip, hipStream_t s) {
  constexpr int GW = 16 / (int)sizeof(T);
  if (nr % GW != 0 || G < nr / GW || G > 64 || (G & (G - 1)) != 0 || op.blk != 1) return false;
  const int rpb = 256 / G;
  const int nlog = (op.n + rpb - 1) / rpb;
  if (nlog == 0) return true;
#define R3MG_SPLIT2(NRV)                                                                                          \
  hipLaunchKernelGGL((k_level_split2<T, NRV>), dim3(xcd_grid(nlog)), dim3(256), 0, s, op.n, G, op.ptr, op.idx,   \
                     op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2, flags, skip, nlog)
  switch (nr) {
    case 4: R3MG_SPLIT2(4); break;
    case 8: R3MG_SPLIT2(8); break;
    case 16: R3MG_SPLIT2(16); break;
    default: return false;
  }
#undef R3MG_SPLIT2
  check_launch("k_level_split2");
  return true;
}
template bool launch_level_split2<float>(const LevelOp<float>&, int, int, const float*, const float*, float*, float*,
                                         float*, double, double, int, const int*, hipStream_t);
template bool launch_level_split2<double>(const LevelOp<double>&, int, int, const double*, const double*, double*,
                                          double*, double*, double, double, int, const int*, hipStream_t);

template <typename T>
bool launch_level_split(const LevelOp<T>& op, int nr, int G, const T* u, const T* b, T* rho, T* x, T* dout, double c1,
                        double c2, int flags, const int* skip, hipStream_t s) {
  constexpr int GW = 16 / (int)sizeof(T);
  if (nr % GW != 0 || G < nr / GW || G > 64 || (G & (G - 1)) != 0 || op.blk != 1) return false;
  const int rpb = 256 / G;
  const int nlog = (op.n + rpb - 1) / rpb;
  if (nlog == 0) return true;
#define R3MG_SPLIT(NRV)                                                                                             \
  hipLaunchKernelGGL((k_level_split<T, (NRV < GW ? GW : NRV)>), dim3(xcd_grid(nlog)), dim3(256), 0, s, op.n, G, op.ptr, \
                     op.idx, op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2, flags, skip, nlog)
  switch (nr) {
    case 2: R3MG_SPLIT(2); break;
    case 4: R3MG_SPLIT(4); break;
    case 8: R3MG_SPLIT(8); break;
    case 16: R3MG_SPLIT(16); break;
    default: return false;
  }
#undef R3MG_SPLIT
  check_launch("k_level_split");
  return true;
}
template bool launch_level_split<float>(const LevelOp<float>&, int, int, const float*, const float*, float*, float*,
                                        float*, double, double, int, const int*, hipStream_t);
template bool launch_level_split<double>(const LevelOp<double>&, int, int, const double*, const double*, double*,
                                         double*, double*, double, double, int, const int*, hipStream_t);

// Sum over the entries [k, z) of one row from LDS: values svs[k], column positions sps[k] into the staged u rows
// usq[p * CH] (16-byte chunks).  Single entries up to a multiple of 4 from vb (the block's aligned start); then
// groups of 8 (two aligned LDS words of 4 values and of 4 positions each), the next group's values and positions
// read together with the current group's u rows, so that one LDS round trip serves 8 entries; then 4-entry groups
// and single entries.  The entries are added in ascending order.
template <typename T, typename VT, int CH>
__device__ __forceinline__ VT lmr_row_sum(const T* svs, const uint16_t* sps, const VT* usq, int vb, int k, int z) {
  typedef T T4 __attribute__((ext_vector_type(4)));
  typedef unsigned short S4 __attribute__((ext_vector_type(4)));
  VT t = (VT)0;
  for (; k < z && ((k - vb) & 3); ++k) t += svs[k] * usq[sps[k] * CH];
  if (k + 8 <= z) {
    T4 a0 = *reinterpret_cast<const T4*>(svs + k), a1 = *reinterpret_cast<const T4*>(svs + k + 4);
    S4 p0 = *reinterpret_cast<const S4*>(sps + k), p1 = *reinterpret_cast<const S4*>(sps + k + 4);
    for (;;) {
      const VT w0 = usq[p0.x * CH], w1 = usq[p0.y * CH], w2 = usq[p0.z * CH], w3 = usq[p0.w * CH];
      const VT w4 = usq[p1.x * CH], w5 = usq[p1.y * CH], w6 = usq[p1.z * CH], w7 = usq[p1.w * CH];
      const T4 c0 = a0, c1 = a1;
      k += 8;
      const bool more = k + 8 <= z;
      if (more) {
        a0 = *reinterpret_cast<const T4*>(svs + k);
        a1 = *reinterpret_cast<const T4*>(svs + k + 4);
        p0 = *reinterpret_cast<const S4*>(sps + k);
        p1 = *reinterpret_cast<const S4*>(sps + k + 4);
      }
      t += c0.x * w0;
      t += c0.y * w1;
      t += c0.z * w2;
      t += c0.w * w3;
      t += c1.x * w4;
      t += c1.y * w5;
      t += c1.z * w6;
      t += c1.w * w7;
      if (!more) break;
    }
  }
  for (; k + 4 <= z; k += 4) {
    const T4 a = *reinterpret_cast<const T4*>(svs + k);
    const S4 p = *reinterpret_cast<const S4*>(sps + k);
    const VT w0 = usq[p.x * CH], w1 = usq[p.y * CH], w2 = usq[p.z * CH], w3 = usq[p.w * CH];
    t += a.x * w0;
    t += a.y * w1;
    t += a.z * w2;
    t += a.w * w3;
  }
  for (; k < z; ++k) t += svs[k] * usq[sps[k] * CH];
  return t;
}

// j-th of the SPLIT cut points of a row's entries [ka, kz) (j = 0: ka, j = SPLIT: kz): the j / SPLIT point rounded
// down to a multiple of 4 entries from vb, so that every part but the first starts aligned
template <int SPLIT>
__device__ __forceinline__ int lmr_cut(int vb, int ka, int kz, int j) {
  if (j <= 0) return ka;
  if (j >= SPLIT) return kz;
  const int c = ka + (int)((int64_t)(kz - ka) * j / SPLIT);
  return min(max(vb + ((c - vb) & ~3), ka), kz);
}

// Epilogue of the fused level kernel for one 16-byte chunk (offset o) of one row, in two parts: the operands it
// reads (loaded before the row sum, so that their latency overlaps it), then, from the row sum t, the values it
// writes: rn (-> rho), xn (-> x), dn (-> dout).
template <typename T, typename VT>
__device__ __forceinline__ void lmr_epi_load(int row, int64_t o, const T* __restrict__ u, const T* __restrict__ b,
                                             const T* rho, const T* x, const T* __restrict__ dinv, int flags, VT& old,
                                             VT& ui, VT& xo, T& di) {
  if (flags & F_PLAIN) return;
  // no branch around the loads (a load under one is waited for at its end, and with it every older load, such as
  // the next block's staging): x and dinv are read whether or not the flags use them
  const T* ob = (flags & F_RHO_FROM_B) ? b : rho;
  old = *reinterpret_cast<const VT*>(ob + o);
  ui = *reinterpret_cast<const VT*>(u + o);
  xo = *reinterpret_cast<const VT*>(x + o);
  di = dinv[row];
}
template <typename T, typename VT>
__device__ __forceinline__ void lmr_epi_store(int64_t o, VT t, VT old, VT ui, VT xo, T di, T c1, T c2, T* rho, T* x,
                                              T* dout, int flags) {
  if (flags & F_PLAIN) {
    *reinterpret_cast<VT*>(rho + o) = t;
    return;
  }
  const VT r = old - t;
  if (flags & F_RHO_STORE) *reinterpret_cast<VT*>(rho + o) = r;
  if (flags & F_X_ASSIGN)
    *reinterpret_cast<VT*>(x + o) = ui;
  else if (flags & F_X_ADD)
    *reinterpret_cast<VT*>(x + o) = xo + ui;
  if (flags & F_D_OUT) *reinterpret_cast<VT*>(dout + o) = c1 * ui + (c2 * di) * r;
}

// Multi-right-hand-side fine-level kernel with LDS staging (NR columns, interleaved n x NR vectors).  One
// workgroup of TPB = 512 threads per block of consecutive rows (MrBlocks); with at most 80 KiB of LDS, two share
// a compute unit (16 waves).  The block's values and 2-byte column positions and u at its distinct columns
// (CH = NR sizeof(T) / 16 chunks of 16 bytes per column) are staged in LDS with 16-byte loads (nontemporal for the
// matrix), all issued before the first LDS store, so that a workgroup keeps ~60 KB of loads in flight; the column
// list carries one padding entry after its last (read by a block without columns).  Thread t then owns chunk
// q = t % CH of half h = (t / CH) % 2 of row slot t / (2 CH): half 0 sums the row's entries below an aligned
// midpoint, half 1 the rest (each in ascending order, from LDS), the two half sums are added across lanes, and
// half 0 applies the epilogue of k_level to its chunk.  With ord, rows take the slots in order of decreasing
// length, so that the rows of a wave have similar lengths.  A block beyond the staging capacity holds one row,
// which the workgroup sums from global memory: phase j takes the entries j, j + TPB / CH, ..., and the phase sums
// are added in phase order.
template <typename T, int NR, int CAP, int UCAP>
__global__ __launch_bounds__(512) void k_level_lmr(int nrb, const int4* __restrict__ meta,
                                                   const int* __restrict__ ucol, const uint16_t* __restrict__ lidx,
                                                   const int* __restrict__ ord, const int* __restrict__ ptr,
                                                   const int* __restrict__ idx, const T* __restrict__ val,
                                                   const T* __restrict__ u, const T* __restrict__ b, T* rho, T* x,
                                                   const T* __restrict__ dinv, T* dout, T c1, T c2, int flags,
                                                   const int* __restrict__ skip) {
  constexpr int TPB = 512;
  constexpr int VW = 16 / (int)sizeof(T);  // elements per 16-byte chunk
  constexpr int CH = NR / VW;              // chunks per column
  constexpr int RMAX = 256 / CH;           // row slots
  constexpr int NPH = TPB / CH;            // phases of the single-row path
  constexpr int NVC = CAP / VW + 2;        // value chunks of CAP entries from a 16-byte aligned start
  constexpr int NPC = CAP / 8 + 2;         // position chunks (8 per 16 bytes)
  constexpr int NV = (NVC + TPB - 1) / TPB, NP = (NPC + TPB - 1) / TPB, NU = (UCAP * CH + TPB - 1) / TPB;
  static_assert(NR % VW == 0 && 64 % (2 * CH) == 0 && CAP % 8 == 0 && UCAP * CH >= TPB, "staging geometry");
  typedef T VT __attribute__((ext_vector_type(VW)));
  typedef unsigned int U4 __attribute__((ext_vector_type(4)));
  if (skip && *skip) return;
  const int lb = xcd_block(nrb);
  if (lb < 0) return;
  __shared__ VT sv[NVC + 1];  // the last entry of each array takes the stores of threads beyond the block
  __shared__ U4 sp[NPC + 1];
  __shared__ VT us[UCAP * CH + 1];
  const int tid = threadIdx.x;
  const int q = tid % CH, h = (tid / CH) & 1, slot = tid / (2 * CH);
  // first row, first nonzero and first distinct column of this block and of the next: one round trip, after
  // which the value and position streams can be issued
  const int4 m0 = meta[lb], m1 = meta[lb + 1];
  const int r0 = m0.x, r1 = m1.x;
  const int e0 = m0.y, e1 = m1.y;
  const int u0 = m0.z, nu = m1.z - u0;
  const int vb = e0 & ~(VW - 1), pb = e0 & ~7;
  const int nvc = (e1 - vb + VW - 1) / VW, npc = (e1 - pb + 7) / 8;
  VT t = (VT)0;
  int row = -1;
  VT eold = (VT)0, eui = (VT)0, exo = (VT)0;
  T edi = 0;
  if (nu <= UCAP && nvc <= NVC && npc <= NPC) {  // uniform over the workgroup
    // the row of this thread's slot, its entry range and the epilogue's operands, loaded first so that they
    // overlap the staging
    const int nrow = r1 - r0;
    const int rr = ord ? ord[r0 + min(slot, nrow - 1)] : r0 + min(slot, nrow - 1);
    const int ka = ptr[rr], kz = ptr[rr + 1];
    lmr_epi_load<T, VT>(rr, (int64_t)rr * NR + q * VW, u, b, rho, x, dinv, flags, eold, eui, exo, edi);
    // every thread issues all its loads before the first LDS store, with no divergent branch around them (a load
    // under one is waited for at the branch's end): indices beyond the block are clamped to its last chunk, and
    // threads beyond it store into a spare LDS entry
    VT vv[NV];
    U4 pv[NP];
    int uc[NU];
    VT uv[NU];
    const int vlast = max(nvc - 1, 0), plast = max(npc - 1, 0), ulast = max(nu * CH - 1, 0);
#pragma unroll
    for (int m = 0; m < NV; ++m)
      vv[m] = __builtin_nontemporal_load(reinterpret_cast<const VT*>(val + vb) + min(tid + TPB * m, vlast));
#pragma unroll
    for (int m = 0; m < NP; ++m)
      pv[m] = __builtin_nontemporal_load(reinterpret_cast<const U4*>(lidx + pb) + min(tid + TPB * m, plast));
#pragma unroll
    for (int m = 0; m < NU; ++m) uc[m] = ucol[u0 + min(tid + TPB * m, ulast) / CH];
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      const int i = min(tid + TPB * m, ulast);
      uv[m] = *reinterpret_cast<const VT*>(u + (int64_t)uc[m] * NR + (i % CH) * VW);
    }
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      const int i = tid + TPB * m;
      sv[i < nvc ? i : NVC] = vv[m];
    }
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      const int i = tid + TPB * m;
      sp[i < npc ? i : NPC] = pv[m];
    }
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      const int i = tid + TPB * m;
      us[i < nu * CH ? i : UCAP * CH] = uv[m];
    }
    if (slot < nrow) row = rr;
    asm volatile("" ::"v"(ka), "v"(kz));  // keeps the entry-range loads ahead of the barrier
    __syncthreads();
    if (row >= 0) {
      t = lmr_row_sum<T, VT, CH>(reinterpret_cast<const T*>(sv) - vb, reinterpret_cast<const uint16_t*>(sp) - pb,
                                 us + q, vb, lmr_cut<2>(vb, ka, kz, h), lmr_cut<2>(vb, ka, kz, h + 1));
    }
#pragma unroll
    for (int w = 0; w < VW; ++w) t[w] += __shfl_xor(t[w], CH, 64);  // half sums of the row (same on both halves)
  } else {  // one row beyond the staging capacity (r1 == r0 + 1)
    const int ph = tid / CH;
    VT acc = (VT)0;
    for (int e = e0 + ph; e < e1; e += NPH)
      acc += val[e] * *reinterpret_cast<const VT*>(u + (int64_t)idx[e] * NR + q * VW);
    us[tid] = acc;
    __syncthreads();
    if (ph == 0) {
      for (int j = 0; j < NPH; ++j) t += us[j * CH + q];
      row = r0;
      lmr_epi_load<T, VT>(row, (int64_t)row * NR + q * VW, u, b, rho, x, dinv, flags, eold, eui, exo, edi);
    }
  }
  if (row >= 0 && h == 0)
    lmr_epi_store<T, VT>((int64_t)row * NR + q * VW, t, eold, eui, exo, edi, c1, c2, rho, x, dout, flags);
}

// Pipelined form of k_level_lmr: one persistent workgroup of 1024 threads per compute unit walks a contiguous run of blocks (runs
// of neighbouring blocks stay on one XCD, whose L2 then serves the columns they share) with two LDS stages.  While
// block i is summed from one stage, block i+1's values, positions, row-pointer and row-order slices and u at its
// distinct columns arrive in the other by direct global-to-LDS loads (no registers held; the loads of a wave fill
// 64 consecutive 16-byte or 4-byte LDS slots), so the HBM stream never waits for the sums.  Block records
// (first row, first nonzero, first distinct column) are read two blocks ahead and the distinct-column indices one
// block ahead.  The two stages alternate in a loop unrolled by two, so that each LDS access names a fixed stage.
// Row order and epilogue are those of k_level_lmr; each row is summed in four aligned parts (16 waves per compute
// unit), added across lanes.  A block's epilogue operands are loaded before its row sums, and its stores are
// issued at the start of the next step.
template <typename T, int NR, int CAP, int UCAP>
struct LmrStage {
  static constexpr int VW = 16 / (int)sizeof(T), CH = NR / VW, RMAX = 256 / CH;
  static constexpr int NVC = CAP / VW + 2, NPC = CAP / 8 + 2, NUC = UCAP * CH;
  typedef T VT __attribute__((ext_vector_type(VW)));
  typedef unsigned int U4 __attribute__((ext_vector_type(4)));
  VT sv[NVC];
  U4 sp[NPC];
  VT us[NUC];
  int rp[RMAX + 1];
  int ord[RMAX];
};

__device__ __forceinline__ void lds_dma16(const void* g, void* l) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)g,
                                   (__attribute__((address_space(3))) void*)l, 16, 0, 0);
}
__device__ __forceinline__ void lds_dma4(const void* g, void* l) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)g,
                                   (__attribute__((address_space(3))) void*)l, 4, 0, 0);
}

template <typename T, int NR, int CAP, int UCAP>
__global__ __launch_bounds__(1024) void k_level_lmr_pipe(int nrb, int nwg, const int4* __restrict__ meta,
                                                         const int* __restrict__ ucol, const uint16_t* __restrict__ lidx,
                                                         const int* __restrict__ ord, const int* __restrict__ ptr,
                                                         const int* __restrict__ idx, const T* __restrict__ val,
                                                         const T* __restrict__ u, const T* __restrict__ b, T* rho,
                                                         T* x, const T* __restrict__ dinv, T* dout, T c1, T c2,
                                                         int flags, const int* __restrict__ skip) {
  typedef LmrStage<T, NR, CAP, UCAP> S;
  typedef typename S::VT VT;
  constexpr int TPB = 1024, SPLIT = 4;
  constexpr int VW = S::VW, CH = S::CH, RMAX = S::RMAX, NVC = S::NVC, NPC = S::NPC, NUC = S::NUC;
  constexpr int NU = (NUC + TPB - 1) / TPB, NPH = TPB / CH;
  static_assert(RMAX <= 64 && RMAX * CH * SPLIT == TPB && NUC >= TPB, "stage geometry");
  if (skip && *skip) return;
  const int lw = xcd_block(nwg);
  if (lw < 0) return;
  const int bb = (int)((int64_t)lw * nrb / nwg), be = (int)((int64_t)(lw + 1) * nrb / nwg);
  if (bb >= be) return;
  // two LDS objects (not one array), so that the compiler sees that the loads into one stage never write the other
  __shared__ S st0, st1;
  const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
  const int q = tid % CH, h = (tid / CH) % SPLIT, slot = tid / (CH * SPLIT);
  // float: epilogue operands loaded before the row sums and stores issued one step later (double: both after the
  // row sums; its registers allow neither)
  constexpr bool DEFER = sizeof(T) == 4;
  VT eold = (VT)0, eui = (VT)0, exo = (VT)0, et = (VT)0;
  T edi = 0;
  int prow = -1;  // DEFER: row of the stores still to issue (-1: none)

  auto staged = [&](int4 m0, int4 m1) {
    const int vb = m0.y & ~(VW - 1), pb = m0.y & ~7;
    return m1.z - m0.z <= UCAP && (m1.y - vb + VW - 1) / VW <= NVC && (m1.y - pb + 7) / 8 <= NPC;
  };
  auto load_uc = [&](int4 m0, int4 m1, int* uc) {
    const int last = max((m1.z - m0.z) * CH - 1, 0);
#pragma unroll
    for (int m = 0; m < NU; ++m) uc[m] = ucol[m0.z + min(tid + TPB * m, last) / CH];
  };
  // direct loads of block (m0, m1) into stage D
  auto issue = [&](S& D, int4 m0, int4 m1, const int* uc) {
    if (!staged(m0, m1)) return;
    const int vb = m0.y & ~(VW - 1), pb = m0.y & ~7;
    const int nvc = (m1.y - vb + VW - 1) / VW, npc = (m1.y - pb + 7) / 8, nuc = (m1.z - m0.z) * CH;
    const int nrow = m1.x - m0.x;
    for (int base = wv * 64; base < nvc; base += TPB)
      if (base + ln < nvc) lds_dma16(val + vb + (int64_t)(base + ln) * VW, &D.sv[base]);
    for (int base = wv * 64; base < npc; base += TPB)
      if (base + ln < npc) lds_dma16(lidx + pb + (int64_t)(base + ln) * 8, &D.sp[base]);
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      const int base = m * TPB + wv * 64;
      if (base < nuc && base + ln < nuc)
        lds_dma16(u + (int64_t)uc[m] * NR + ((base + ln) % CH) * VW, &D.us[base]);
    }
    if (wv < 2 && wv * 64 + ln <= nrow) lds_dma4(ptr + m0.x + wv * 64 + ln, &D.rp[wv * 64]);
    if (ord && wv == 2 && ln < nrow) lds_dma4(ord + m0.x + ln, &D.ord[0]);
  };
  // row sums of block (m0, m1) from stage D (part h of SPLIT per thread, parts added across lanes), then the
  // epilogue
  auto compute = [&](S& D, int4 m0, int4 m1) {
    VT t = (VT)0;
    if (staged(m0, m1)) {
      const int nrow = m1.x - m0.x;
      int row = -1;
      if (slot < nrow) {
        const int lr = ord ? D.ord[slot] - m0.x : slot;
        row = m0.x + lr;
        if (DEFER && h == 0)
          lmr_epi_load<T, VT>(row, (int64_t)row * NR + q * VW, u, b, rho, x, dinv, flags, eold, eui, exo, edi);
        const int vb = m0.y & ~(VW - 1), pb = m0.y & ~7;
        const int ka = D.rp[lr], kz = D.rp[lr + 1];
        t = lmr_row_sum<T, VT, CH>(reinterpret_cast<const T*>(D.sv) - vb,
                                   reinterpret_cast<const uint16_t*>(D.sp) - pb, D.us + q, vb,
                                   lmr_cut<SPLIT>(vb, ka, kz, h), lmr_cut<SPLIT>(vb, ka, kz, h + 1));
      }
#pragma unroll
      for (int w = 0; w < VW; ++w) {
        t[w] += __shfl_xor(t[w], CH, 64);
        t[w] += __shfl_xor(t[w], 2 * CH, 64);
      }
      if (row >= 0 && h == 0) {
        if (DEFER) {
          prow = row;
          et = t;
        } else {
          VT lo = (VT)0, lu = (VT)0, lx = (VT)0;
          T ld = 0;
          lmr_epi_load<T, VT>(row, (int64_t)row * NR + q * VW, u, b, rho, x, dinv, flags, lo, lu, lx, ld);
          lmr_epi_store<T, VT>((int64_t)row * NR + q * VW, t, lo, lu, lx, ld, c1, c2, rho, x, dout, flags);
        }
      }
    } else {  // one row beyond the stage capacity: summed from global memory, phase sums added in phase order, and
              // its epilogue applied at once (no load of this path is left in flight)
      const int ph = tid / CH;
      VT acc = (VT)0;
      for (int e = m0.y + ph; e < m1.y; e += NPH)
        acc += val[e] * *reinterpret_cast<const VT*>(u + (int64_t)idx[e] * NR + q * VW);
      D.us[tid] = acc;
      __syncthreads();
      if (ph == 0) {  // the next step's barrier precedes any reuse of the stage
        for (int j = 0; j < NPH; ++j) t += D.us[j * CH + q];
        const int row = m0.x;
        VT lo = (VT)0, lu = (VT)0, lx = (VT)0;
        T ld = 0;
        lmr_epi_load<T, VT>(row, (int64_t)row * NR + q * VW, u, b, rho, x, dinv, flags, lo, lu, lx, ld);
        lmr_epi_store<T, VT>((int64_t)row * NR + q * VW, t, lo, lu, lx, ld, c1, c2, rho, x, dout, flags);
      }
    }
  };
  // DEFER: the stores of the previous block's rows, issued at the start of the next step (their operands are then
  // known to be loaded), so that they are acknowledged while a block is summed rather than at the next wait
  auto flush = [&] {
    if (DEFER && prow >= 0)
      lmr_epi_store<T, VT>((int64_t)prow * NR + q * VW, et, eold, eui, exo, edi, c1, c2, rho, x, dout, flags);
    prow = -1;
  };

  int uc[NU];
  int4 m0 = meta[bb], m1 = meta[bb + 1];
  load_uc(m0, m1, uc);
  issue(st0, m0, m1, uc);
  int4 m2 = bb + 2 <= nrb ? meta[bb + 2] : m1;
  if (bb + 1 < be) load_uc(m1, m2, uc);
  // block bi in stage A: wait for its loads, start block bi + 1's into stage B, prefetch for bi + 2, sum bi
  // (the stages come in as restrict pointers: the compiler then knows that the loads into B never write A and does
  // not wait for them before reading A)
  auto step = [&](S* __restrict__ A, S* __restrict__ B, int bi) {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0) (expcnt, lgkmcnt unconstrained), visible to the compiler
    __syncthreads();
    flush();
    if (bi + 1 < be) issue(*B, m1, m2, uc);
    const int4 m3 = bi + 3 <= nrb ? meta[bi + 3] : m2;
    if (bi + 2 < be) load_uc(m2, m3, uc);
    compute(*A, m0, m1);
    m0 = m1;
    m1 = m2;
    m2 = m3;
  };
  for (int bi = bb; bi < be; bi += 2) {
    step(&st0, &st1, bi);
    if (bi + 1 < be) step(&st1, &st0, bi + 1);
  }
  flush();
}

template <typename T, int NR, int CLS>
static void launch_lmr_t(const MrBlocks& mb, const LevelOp<T>& op, const int* ord, const T* u, const T* b, T* rho,
                         T* x, T* dout, double c1, double c2, int flags, const int* skip, hipStream_t s) {
  if (!mb.meta) throw std::runtime_error("LDS-staged multi-RHS kernel: block records missing");
  hipLaunchKernelGGL((k_level_lmr<T, NR, kMrCap[CLS], kMrUcap[CLS]>), dim3(xcd_grid(mb.nrb)), dim3(512), 0, s, mb.nrb,
                     reinterpret_cast<const int4*>(mb.meta), mb.ucol, mb.lidx, ord, op.ptr, op.idx, op.val, u, b,
                     rho, x, op.dinv, dout, (T)c1, (T)c2, flags, skip);
}

template <typename T, int NR, int CLS>
static void launch_lmr_pipe_t(const MrBlocks& mb, const LevelOp<T>& op, const T* u, const T* b, T* rho, T* x,
                              T* dout, double c1, double c2, int flags, const int* skip, hipStream_t s) {
  static const int cus = [] {
    int d = 0, v = 0;
    if (hipGetDevice(&d) != hipSuccess || hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, d) != hipSuccess)
      v = 256;
    return std::max(v, 1);
  }();
  const int nwg = std::min(mb.nrb, cus);
  hipLaunchKernelGGL((k_level_lmr_pipe<T, NR, kMrCap[CLS], kMrUcap[CLS]>), dim3(xcd_grid(nwg)), dim3(1024), 0, s,
                     mb.nrb, nwg, reinterpret_cast<const int4*>(mb.meta), mb.ucol, mb.lidx, mb.ord, op.ptr, op.idx,
                     op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2, flags, skip);
}

template <typename T>
bool launch_level_lmr(const MrBlocks& mb, const LevelOp<T>& op, int nr, bool pipelined, const T* u, const T* b,
                      T* rho, T* x, T* dout, double c1, double c2, int flags, const int* skip, hipStream_t s) {
  const int cls = mr_class(nr, (int)sizeof(T));
  if (cls < 0 || mb.cls != cls || mb.nrb <= 0 || op.blk != 1) return false;
  if constexpr (sizeof(T) == 4) {
    if (pipelined)
      launch_lmr_pipe_t<float, 16, 0>(mb, op, u, b, rho, x, dout, c1, c2, flags, skip, s);
    else
      launch_lmr_t<float, 16, 0>(mb, op, mb.ord, u, b, rho, x, dout, c1, c2, flags, skip, s);
  } else {
    if (cls == 1) {
      if (pipelined)
        launch_lmr_pipe_t<double, 16, 1>(mb, op, u, b, rho, x, dout, c1, c2, flags, skip, s);
      else
        launch_lmr_t<double, 16, 1>(mb, op, mb.ord, u, b, rho, x, dout, c1, c2, flags, skip, s);
    } else {
      if (pipelined)
        launch_lmr_pipe_t<double, 8, 2>(mb, op, u, b, rho, x, dout, c1, c2, flags, skip, s);
      else
        launch_lmr_t<double, 8, 2>(mb, op, mb.ord, u, b, rho, x, dout, c1, c2, flags, skip, s);
    }
  }
  check_launch(pipelined ? "k_level_lmr_pipe" : "k_level_lmr");
  return true;
}
template bool launch_level_lmr<float>(const MrBlocks&, const LevelOp<float>&, int, bool, const float*, const float*,
                                      float*, float*, float*, double, double, int, const int*, hipStream_t);
template bool launch_level_lmr<double>(const MrBlocks&, const LevelOp<double>&, int, bool, const double*,
                                       const double*, double*, double*, double*, double, double, int, const int*,
                                       hipStream_t);



// Block-row variant of the fused kernel for the agglomerated levels, one right-hand side.  One wave per box K,
// L = floor(64 / B) lanes per row: lane (q, s) owns the columns p = s, s + L, ... of row (K, q) (w = nb*B values,
// one contiguous run per row).  Every memory access of the box is put in flight at once: the row's first KMAX
// values per lane (registers), the epilogue operands, and the w entries of u the block row touches (nb stored
// blocks of B consecutive columns, staged in LDS once and shared by the B rows).  Each lane then sums its
// columns in ascending order, the L lane sums of a row are added in lane order through LDS, and lane q applies
// the epilogue of row (K, q).  Dynamic LDS: 4 waves x (maxw + 64) entries, maxw = max_K nb_K * B.
template <typename T, int KMAX, bool KEEP>
__global__ __launch_bounds__(256) void k_level_blockrow(int nbox, int blk, int maxw, const int* __restrict__ bptr,
                                                        const int* __restrict__ bcol, const T* __restrict__ val,
                                                        const T* __restrict__ u, const T* __restrict__ b, T* rho, T* x,
                                                        const T* __restrict__ dinv, T* dout, T c1, T c2, int flags,
                                                        const int* __restrict__ skip, int nlog) {
  if (skip && *skip) return;
  extern __shared__ unsigned char smem_raw[];
  const int lb = xcd_block(nlog);
  if (lb < 0) return;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int K = lb * 4 + wv;
  if (K >= nbox) return;  // whole wave leaves; no block-wide barrier follows
  T* xs = reinterpret_cast<T*>(smem_raw) + (size_t)wv * (maxw + 64);
  T* part = xs + maxw;
  const int L = 64 / blk;
  const int q = lane / L, sv = lane - q * L;
  const bool active = q < blk;
  const int j0 = bptr[K], nb = bptr[K + 1] - j0;
  const int w = nb * blk;
  const T* vrow = val + (int64_t)blk * blk * j0 + (int64_t)q * w;
  T v[KMAX];
#pragma unroll
  for (int m = 0; m < KMAX; ++m) {
    const int p = sv + L * m;
    v[m] = (active && p < w) ? ld_matrix<KEEP>(vrow + p) : (T)0;
  }
  const int row = K * blk + lane;
  T p_old = 0, p_u = 0, p_x = 0, p_di = 0;
  if (lane < blk && !(flags & F_PLAIN)) {
    p_old = (flags & F_RHO_FROM_B) ? b[row] : rho[row];
    p_u = u[row];
    if (flags & F_X_ADD) p_x = x[row];
    if (flags & F_D_OUT) p_di = dinv[row];
  }
  for (int p = lane; p < w; p += 64) {
    const int j = p / blk, c = p - j * blk;
    xs[p] = u[(int64_t)bcol[j0 + j] * blk + c];
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  T acc = 0;
  if (active) {
#pragma unroll
    for (int m = 0; m < KMAX; ++m) {
      const int p = sv + L * m;
      if (p < w) acc += v[m] * xs[p];
    }
    for (int p = sv + L * KMAX; p < w; p += L) acc += vrow[p] * xs[p];  // rows longer than L * KMAX
  }
  part[lane] = acc;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (lane < blk) {
    T t = 0;
    for (int s2 = 0; s2 < L; ++s2) t += part[lane * L + s2];
    if (flags & F_PLAIN) {
      rho[row] = t;
    } else {
      const T r = p_old - t;
      if (flags & F_RHO_STORE) rho[row] = r;
      if (flags & F_X_ASSIGN)
        x[row] = p_u;
      else if (flags & F_X_ADD)
        x[row] = p_x + p_u;
      if (flags & F_D_OUT) dout[row] = c1 * p_u + c2 * p_di * r;
    }
  }
}

// LDS bytes of k_level_blockrow for block rows of at most maxw entries
size_t blockrow_lds_bytes(int blk, int maxw, size_t esz) {
  (void)blk;
  return esz * (size_t)4 * (maxw + 64);
}

template <typename T>
void launch_level_blockrow(const LevelOp<T>& op, int maxnb, const T* u, const T* b, T* rho, T* x, T* dout, double c1,
                           double c2, int flags, const int* skip, hipStream_t s) {
  const int nbox = op.n / op.blk;
  const int nlog = (nbox + 3) / 4;
  if (nlog == 0) return;
  const int maxw = maxnb * op.blk;
  const size_t shm = blockrow_lds_bytes(op.blk, maxw, sizeof(T));
  if (shm > 65536) throw std::runtime_error("block-row kernel: block row too wide for LDS");
  if (op.blk > 64) throw std::runtime_error("block-row kernel: more than 64 rows per box");
  if (flags & F_KEEP)
    hipLaunchKernelGGL((k_level_blockrow<T, 16, true>), dim3(xcd_grid(nlog)), dim3(256), shm, s, nbox, op.blk, maxw,
                       op.ptr, op.idx, op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2, flags, skip, nlog);
  else
    hipLaunchKernelGGL((k_level_blockrow<T, 16, false>), dim3(xcd_grid(nlog)), dim3(256), shm, s, nbox, op.blk, maxw,
                       op.ptr, op.idx, op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2, flags, skip, nlog);
  check_launch("k_level_blockrow");
}
template void launch_level_blockrow<float>(const LevelOp<float>&, int, const float*, const float*, float*, float*,
                                           float*, double, double, int, const int*, hipStream_t);
template void launch_level_blockrow<double>(const LevelOp<double>&, int, const double*, const double*, double*,
                                            double*, double*, double, double, int, const int*, hipStream_t);

// Residual staging of the fused restriction: wave w's rows at [w BLK, (w + 1) BLK) of one LDS array.
template <typename T, int BLK>
__device__ inline T* rsh_data() {
  __shared__ T rsh[4 * BLK];
  return rsh;
}
template <typename T, int BLK>
__device__ inline void rsh_store(int wv, int row, T r) {
  rsh_data<T, BLK>()[wv * BLK + row] = r;
}

// Box-row kernel (2D agglomerated levels: boxes of BLK = 4, 9 or 16 rows): one wave per box K.  Lane p owns the
// positions p + 64 m (m < NP) of the box's block row (w = nb BLK entries; position j BLK + c is column
// bcol[j0 + j] BLK + c): it gathers u there once and multiplies it with that position's value in each of the
// BLK rows, so every value load is a coalesced 256-byte row segment and no column list or LDS staging is
// needed.  The BLK row sums over the 64 lanes come out of a transposing butterfly over 16 slots (each step halves
// the rows a lane keeps and doubles the lanes summed), in a fixed order; lane l then holds row
// 8 b5 + 4 b4 + 2 b3 + b2 (b = bits of l) and the lanes with l % 4 == 0 apply the epilogue of k_level.
// With RESTRICT (nbox a multiple of 4, workgroup G = the four children of parent box G) the workgroup then
// restricts its residuals into the parent's entries of the next level (BoxRestrict).
template <typename T, int BLK, int NP, bool KEEP, bool RESTRICT>
__global__ __launch_bounds__(256) void k_level_boxrow(int nbox, const int* __restrict__ bptr,
                                                      const int* __restrict__ bcol, const T* __restrict__ val,
                                                      const T* __restrict__ u, const T* __restrict__ b, T* rho, T* x,
                                                      const T* __restrict__ dinv, T* dout, T c1, T c2, int flags,
                                                      const int* __restrict__ skip, int nlog, BoxRestrict<T> rs) {
  static_assert(BLK <= 16, "rows per box");
  if (skip && *skip) return;
  const int lb = xcd_block(nlog);
  if (lb < 0) return;
  // the wave index is uniform: the box's block-row record then comes through scalar loads
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int K = lb * 4 + wv;
  if (K >= nbox) return;  // whole wave leaves; no barrier follows
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4;
  const int myrow = (b5 ? 8 : 0) + (b4 ? 4 : 0) + (b3 ? 2 : 0) + (b2 ? 1 : 0);
  const bool owner = (lane & 3) == 0 && myrow < BLK;
  const int row = K * BLK + min(myrow, BLK - 1);  // clamped: every lane loads, only owners use the values
  // All loads below are unconditional per lane (clamped addresses, masked values): a load under a lane-dependent
  // branch would be waited for at the branch's end, which serialised the box's round trips.
  T p_old = 0, p_u = 0, p_x = 0, p_di = 0;
  if (!(flags & F_PLAIN)) {
    p_old = (flags & F_RHO_FROM_B) ? b[row] : rho[row];
    p_u = u[row];
    if (flags & F_X_ADD) p_x = x[row];
    if (flags & F_D_OUT) p_di = dinv[row];
  }
  const int j0 = bptr[K], w = (bptr[K + 1] - j0) * BLK;  // w >= BLK: every box holds its diagonal block
  const T* vb = val + (int64_t)BLK * BLK * j0;  // row q of the box at vb + q w
  T acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0;
  int pc[NP];
  int cj[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    pc[m] = min(lane + 64 * m, w - 1);
    cj[m] = bcol[j0 + pc[m] / BLK];
  }
  T v[NP][BLK];
#pragma unroll
  for (int m = 0; m < NP; ++m)
#pragma unroll
    for (int q = 0; q < BLK; ++q) v[m][q] = ld_matrix<KEEP>(vb + (int64_t)q * w + pc[m]);
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    const int c = pc[m] - (pc[m] / BLK) * BLK;
    const T ug = u[(int64_t)cj[m] * BLK + c];
    const T uv = lane + 64 * m < w ? ug : (T)0;
#pragma unroll
    for (int q = 0; q < BLK; ++q) acc[q] += v[m][q] * uv;
  }
  T h8[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) h8[q] = (b5 ? acc[8 + q] : acc[q]) + __shfl_xor(b5 ? acc[q] : acc[8 + q], 32, 64);
  T h4[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) h4[q] = (b4 ? h8[4 + q] : h8[q]) + __shfl_xor(b4 ? h8[q] : h8[4 + q], 16, 64);
  T h2[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) h2[q] = (b3 ? h4[2 + q] : h4[q]) + __shfl_xor(b3 ? h4[q] : h4[2 + q], 8, 64);
  T t = (b2 ? h2[1] : h2[0]) + __shfl_xor(b2 ? h2[0] : h2[1], 4, 64);
  t += __shfl_xor(t, 2, 64);
  t += __shfl_xor(t, 1, 64);
  if (owner) {
    if (flags & F_PLAIN) {
      rho[row] = t;
    } else {
      const T r = p_old - t;
      if (flags & F_RHO_STORE) rho[row] = r;
      if (flags & F_X_ASSIGN)
        x[row] = p_u;
      else if (flags & F_X_ADD)
        x[row] = p_x + p_u;
      if (flags & F_D_OUT) dout[row] = c1 * p_u + c2 * p_di * r;
      if constexpr (RESTRICT) rsh_store<T, BLK>(wv, myrow, r);
    }
  }
  if constexpr (RESTRICT) {
    __syncthreads();  // every wave is present: nbox is a multiple of 4
    if (wv == 0 && lane < BLK) {
      constexpr int k = BLK == 4 ? 2 : BLK == 9 ? 3 : 4, kk = k * k;
      const int q0 = lane % k, q1 = lane / k;
      const T* src = rsh_data<T, BLK>();
      T sum = 0;
      for (int C = 0; C < 4; ++C) {
        const T* m = rs.pt + (int64_t)(lb * 4 + C) * 2 * kk;
        const T* sc = src + C * BLK;
        int qc = 0;
        for (int a1 = 0; a1 < k; ++a1)
          for (int a0 = 0; a0 < k; ++a0, ++qc) sum += (m[a0 * k + q0] * m[kk + a1 * k + q1]) * sc[qc];
      }
      const int64_t tq = (int64_t)lb * BLK + lane;
      rs.bnext[tq] = sum;
      if (rs.dnext) rs.dnext[tq] = rs.dinv_next[tq] * sum * rs.inv_theta_next;
    }
  }
}

bool boxrow_supported(int blk, int maxnb) {
  return (blk == 4 || blk == 9 || blk == 16) && maxnb > 0 && (int64_t)maxnb * blk <= 64 * kBoxRowMaxNP;
}

template <typename T>
void launch_level_boxrow(const LevelOp<T>& op, int maxnb, const T* u, const T* b, T* rho, T* x, T* dout, double c1,
                         double c2, int flags, const int* skip, hipStream_t s, const BoxRestrict<T>* rs) {
  if (!boxrow_supported(op.blk, maxnb)) throw std::runtime_error("box-row kernel: unsupported box shape");
  const int nbox = op.n / op.blk;
  const int nlog = (nbox + 3) / 4;
  if (nlog == 0) return;
  if (rs && (nbox % 4 != 0 || (flags & F_PLAIN) || !rs->pt || !rs->bnext))
    throw std::runtime_error("box-row kernel: fused restriction needs four boxes per parent and a residual");
  const int np = (maxnb * op.blk + 63) / 64;
  const BoxRestrict<T> ra = rs ? *rs : BoxRestrict<T>{};
#define R3_BR(B, N)                                                                                               \
  do {                                                                                                            \
    if (rs) {                                                                                                     \
      if (flags & F_KEEP)                                                                                         \
        hipLaunchKernelGGL((k_level_boxrow<T, B, N, true, true>), dim3(xcd_grid(nlog)), dim3(256), 0, s, nbox,   \
                           op.ptr, op.idx, op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2, flags, skip, nlog,  \
                           ra);                                                                                   \
      else                                                                                                        \
        hipLaunchKernelGGL((k_level_boxrow<T, B, N, false, true>), dim3(xcd_grid(nlog)), dim3(256), 0, s, nbox,  \
                           op.ptr, op.idx, op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2, flags, skip, nlog,  \
                           ra);                                                                                   \
    } else if (flags & F_KEEP) {                                                                                  \
      hipLaunchKernelGGL((k_level_boxrow<T, B, N, true, false>), dim3(xcd_grid(nlog)), dim3(256), 0, s, nbox,    \
                         op.ptr, op.idx, op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2, flags, skip, nlog, ra); \
    } else {                                                                                                      \
      hipLaunchKernelGGL((k_level_boxrow<T, B, N, false, false>), dim3(xcd_grid(nlog)), dim3(256), 0, s, nbox,   \
                         op.ptr, op.idx, op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2, flags, skip, nlog, ra); \
    }                                                                                                             \
  } while (0)
  if (op.blk == 4) {
    if (np == 1) R3_BR(4, 1); else if (np == 2) R3_BR(4, 2); else R3_BR(4, 3);
  } else if (op.blk == 9) {
    if (np == 1) R3_BR(9, 1); else if (np == 2) R3_BR(9, 2); else R3_BR(9, 3);
  } else {
    if (np == 1) R3_BR(16, 1); else if (np == 2) R3_BR(16, 2); else R3_BR(16, 3);
  }
#undef R3_BR
  check_launch("k_level_boxrow");
}
template void launch_level_boxrow<float>(const LevelOp<float>&, int, const float*, const float*, float*, float*,
                                         float*, double, double, int, const int*, hipStream_t,
                                         const BoxRestrict<float>*);
template void launch_level_boxrow<double>(const LevelOp<double>&, int, const double*, const double*, double*,
                                          double*, double*, double, double, int, const int*, hipStream_t,
                                          const BoxRestrict<double>*);

// Wide block rows (3D agglomerated levels): one 256-thread workgroup per (box K, chunk of 8 of its B rows),
// grid = nbox * ceil(B/8).  The workgroup stages the nb*B entries of u touched by box K in LDS, then each wave
// computes two rows against the LDS copy with coalesced value loads; threads 0..7 apply the epilogue.
template <typename T, bool KEEP>
__global__ __launch_bounds__(256) void k_level_blockrow_wg(int nbox, int blk, int nchunk, const int* __restrict__ bptr,
                                                           const int* __restrict__ bcol, const T* __restrict__ val,
                                                           const T* __restrict__ u, const T* __restrict__ b, T* rho,
                                                           T* x, const T* __restrict__ dinv, T* dout, T c1, T c2,
                                                           int flags, const int* __restrict__ skip, int nlog) {
  if (skip && *skip) return;
  extern __shared__ unsigned char smem_raw[];
  const int lb = xcd_block(nlog);
  if (lb < 0) return;
  const int K = lb / nchunk;
  const int q0 = (lb - K * nchunk) * 8;
  T* xs = reinterpret_cast<T*>(smem_raw);
  __shared__ T rs[8];
  const int j0 = bptr[K], nb = bptr[K + 1] - j0;
  const int w = nb * blk;
  for (int p = threadIdx.x; p < w; p += 256) {
    const int j = p / blk, c = p - j * blk;
    xs[p] = u[(int64_t)bcol[j0 + j] * blk + c];
  }
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int qa = q0 + 2 * wv, qb = qa + 1;
  const int64_t vb = (int64_t)blk * blk * j0;
  T a0 = 0, a1 = 0;
  if (qa < blk) {
    // 8 steps of both rows in flight per batch; each lane still sums in ascending column order
    const T* va = val + vb + (int64_t)qa * w;
    const bool hb = qb < blk;
    for (int p0 = 0; p0 < w; p0 += 8 * 64) {
      T ta[8], tb[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int p = p0 + lane + 64 * m;
        ta[m] = p < w ? ld_matrix<KEEP>(va + p) : (T)0;
        tb[m] = (hb && p < w) ? ld_matrix<KEEP>(va + w + p) : (T)0;
      }
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int p = p0 + lane + 64 * m;
        if (p < w) {
          const T xp = xs[p];
          a0 += ta[m] * xp;
          if (hb) a1 += tb[m] * xp;
        }
      }
    }
  }
  a0 = wave_sum(a0, 64);
  a1 = wave_sum(a1, 64);
  if (lane == 0) {
    rs[2 * wv] = a0;
    rs[2 * wv + 1] = a1;
  }
  __syncthreads();
  if (threadIdx.x < 8 && q0 + (int)threadIdx.x < blk) {
    const int row = K * blk + q0 + threadIdx.x;
    const T t = rs[threadIdx.x];
    if (flags & F_PLAIN) {
      rho[row] = t;
    } else {
      const T r = ((flags & F_RHO_FROM_B) ? b[row] : rho[row]) - t;
      if (flags & F_RHO_STORE) rho[row] = r;
      const T ui = u[row];
      if (flags & F_X_ASSIGN)
        x[row] = ui;
      else if (flags & F_X_ADD)
        x[row] += ui;
      if (flags & F_D_OUT) dout[row] = c1 * ui + c2 * dinv[row] * r;
    }
  }
}

template <typename T>
void launch_level_blockrow_wg(const LevelOp<T>& op, int maxnb, const T* u, const T* b, T* rho, T* x, T* dout,
                              double c1, double c2, int flags, const int* skip, hipStream_t s) {
  const int nbox = op.n / op.blk;
  const int nchunk = (op.blk + 7) / 8;
  const int nlog = nbox * nchunk;
  if (nlog == 0) return;
  const size_t shm = sizeof(T) * (size_t)maxnb * op.blk;
  if (shm > 65536) throw std::runtime_error("block-row kernel: block row too wide for LDS");
  if (flags & F_KEEP)
    hipLaunchKernelGGL((k_level_blockrow_wg<T, true>), dim3(xcd_grid(nlog)), dim3(256), shm, s, nbox, op.blk, nchunk,
                       op.ptr, op.idx, op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2, flags, skip, nlog);
  else
    hipLaunchKernelGGL((k_level_blockrow_wg<T, false>), dim3(xcd_grid(nlog)), dim3(256), shm, s, nbox, op.blk, nchunk,
                       op.ptr, op.idx, op.val, u, b, rho, x, op.dinv, dout, (T)c1, (T)c2, flags, skip, nlog);
  check_launch("k_level_blockrow_wg");
}
template void launch_level_blockrow_wg<float>(const LevelOp<float>&, int, const float*, const float*, float*, float*,
                                              float*, double, double, int, const int*, hipStream_t);
template void launch_level_blockrow_wg<double>(const LevelOp<double>&, int, const double*, const double*, double*,
                                               double*, double*, double, double, int, const int*, hipStream_t);

// q = A p with per-block partial sums of p.q (float64 CSR)
template <int NR>
__global__ __launch_bounds__(256) void k_spmv_dot(int n, int G, const int* __restrict__ ptr,
                                                  const int* __restrict__ idx, const double* __restrict__ val,
                                                  const double* __restrict__ p, double* q, double* partials,
                                                  const int* __restrict__ skip, int nlog) {
  if (skip && *skip) return;
  const int lb = xcd_block(nlog);
  if (lb < 0) return;
  __shared__ double sh[4 * NR];
  const int rpb = 256 / G;
  const int lane = threadIdx.x & (G - 1);
  const int row = lb * rpb + threadIdx.x / G;
  const bool active = row < n;
  double acc[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = 0;
  if (active) row_product<double, NR, false>(row, lane, G, 1, ptr, idx, val, p, acc);
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = wave_sum(acc[k], G);
  double contrib[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    contrib[k] = 0;
    if (active && lane == 0) {
      const int64_t i = (int64_t)row * NR + k;
      q[i] = acc[k];
      contrib[k] = acc[k] * p[i];
    }
  }
  // block reduction (fixed order)
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    double v = wave_sum(contrib[k], 64);
    if ((threadIdx.x & 63) == 0) sh[(threadIdx.x >> 6) * NR + k] = v;
  }
  __syncthreads();
  if (threadIdx.x < NR) {
    const int k = threadIdx.x;
    partials[(int64_t)lb * NR + k] = (sh[k] + sh[NR + k]) + (sh[2 * NR + k] + sh[3 * NR + k]);
  }
}

int launch_spmv_dot(const LevelOp<double>& op, int nr, const double* p, double* q, double* partials,
                    const int* skip, hipStream_t s) {
  const int G = op.lanes;
  const int rpb = 256 / G;
  const int nlog = (op.n + rpb - 1) / rpb;
  dim3 grid(xcd_grid(nlog));
#define R3_SD(NRV) \
  hipLaunchKernelGGL((k_spmv_dot<NRV>), grid, dim3(256), 0, s, op.n, G, op.ptr, op.idx, op.val, p, q, partials, skip, nlog)
  switch (nr) {
    case 1: R3_SD(1); break;
    case 2: R3_SD(2); break;
    case 4: R3_SD(4); break;
    case 8: R3_SD(8); break;
    case 16: R3_SD(16); break;
    default: throw std::runtime_error("unsupported nrhs block");
  }
#undef R3_SD
  check_launch("k_spmv_dot");
  return nlog;
}

// =============================================================================================
// Transfers
// =============================================================================================
// Several right-hand sides (nr > 1, interleaved: entry i of column c at i * nr + c): the transfer kernels below
// give each thread a chunk of VW = min(nr, 16 bytes / sizeof(T)) adjacent columns, loaded and stored as one
// vector, so the basis functions and transfer entries are formed once per chunk instead of once per column.
// Each column is summed in the same order as the one-column kernel, except k_restrict0_mr (points in index order).
template <typename T, int W>
struct ColVec {
  typedef T type __attribute__((ext_vector_type(W)));
};
template <typename T>
constexpr int col_vw() {
  return 16 / (int)sizeof(T);
}
// the vector path needs 16-byte aligned vectors (always so for the library's buffers)
static inline bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

// Restriction to the first agglomerated level: b1[K*B+q] = sum_{i in K, i free} phi^K_q(xi_i) src_i.
// One workgroup of W waves per box (W = 1, 2 or 4: about one per 128-point chunk of an average box).  Wave w takes the box's points in chunks of 128
// (chunk w, w + W, ...), two points per lane: the lane's two products per q go to LDS ([q][lane]), then
// L = floor(64 / B) lanes sum each q-row of the chunk (lane s takes columns s, s + L, ...) and lane q adds the L
// sums in lane order to its running total.  Finally wave 0 adds the W wave totals in wave order (deterministic).
// Optionally fuses the first Chebyshev direction of the next level: dnext = dinv_next * b1 * inv_theta_next.
template <typename T, int D, int KB>
__global__ __launch_bounds__(256) void k_restrict0(Basis1D<T> bs, int nr, const int* __restrict__ leaf_off,
                                                   const int* __restrict__ owner, const T* __restrict__ xi,
                                                   const T* __restrict__ src, T* bnext, const T* __restrict__ dinv_next,
                                                   T* dnext, T inv_theta_next, const int* __restrict__ skip) {
  constexpr int B = D == 3 ? KB * KB * KB : KB * KB;
  constexpr int L = 64 / B;
  if (skip && *skip) return;
  extern __shared__ unsigned char smem_raw[];
  const int W = blockDim.x >> 6;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  T* sh = reinterpret_cast<T*>(smem_raw) + (size_t)wv * (B * 65 + 64);  // [B][65] products, then [64] sums
  T* part = sh + B * 65;
  T* wtot = reinterpret_cast<T*>(smem_raw) + (size_t)W * (B * 65 + 64);  // [W][64]
  const int K = blockIdx.x;
  const int i0 = leaf_off[K], i1 = leaf_off[K + 1];
  const int q = lane / L, sv = lane - q * L;
  for (int c = 0; c < nr; ++c) {
    T tot = 0;  // lane q's running sum (q = lane < B)
    for (int base = i0 + wv * 128; base < i1; base += W * 128) {
      // both points' loads are unconditional (clamped to the box's last point) and masked afterwards, so that
      // they are in flight together
      const int ia = base + lane, ib = base + 64 + lane;
      const int iac = min(ia, i1 - 1), ibc = min(ib, i1 - 1);
      const int owa = owner[iac], owb = owner[ibc];
      T ra = src[(int64_t)iac * nr + c], rb = src[(int64_t)ibc * nr + c];
      T xa[3], xb[3];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        xa[a] = xi[(int64_t)iac * D + a];
        xb[a] = xi[(int64_t)ibc * D + a];
      }
      const bool oka = ia < i1 && owa >= 0, okb = ib < i1 && owb >= 0;
      ra = oka ? ra : (T)0;
      rb = okb ? rb : (T)0;
      T la[3][4], lbv[3][4];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        lag1d_k<T, KB>(bs, xa[a], la[a]);
        lag1d_k<T, KB>(bs, xb[a], lbv[a]);
      }
      for_each_phi<T, D, KB>(la, [&](int qq, T ph) { sh[qq * 65 + lane] = ph * ra; });
      for_each_phi<T, D, KB>(lbv, [&](int qq, T ph) { sh[qq * 65 + lane] += ph * rb; });
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      T a = 0;
      if (q < B)
        for (int m = sv; m < 64; m += L) a += sh[q * 65 + m];
      part[lane] = a;
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (lane < B) {
        T t = 0;
#pragma unroll
        for (int s2 = 0; s2 < L; ++s2) t += part[lane * L + s2];
        tot += t;
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    wtot[wv * 64 + lane] = tot;
    __syncthreads();
    if (wv == 0 && lane < B) {
      T t = 0;
      for (int w2 = 0; w2 < W; ++w2) t += wtot[w2 * 64 + lane];
      const int64_t o = ((int64_t)K * B + lane) * nr + c;
      bnext[o] = t;
      if (dnext) dnext[o] = dinv_next[(int64_t)K * B + lane] * t * inv_theta_next;
    }
    __syncthreads();
  }
}

// Restriction to the first agglomerated level for nr > 1 columns: one workgroup per box K, in teams of tsize
// threads.  Thread (g, j) of a team takes the KB consecutive coarse functions q = KB g .. KB g + KB - 1 (same q1,
// q2) and column chunk j.  Team t takes the box's points in chunks of 32 (chunks t, t + nteam, ...) through its own
// LDS: the chunk's 1D basis values (one thread per point) and nr entries of src (zero at constrained points); each
// thread adds phi_q(xi_i) src_i over the chunk's points in index order, phi_q formed as l0[q0] (l1[q1] l2[q2]).
// The team sums are then added in team order.  A team is one wave when its threads fit one (four teams, synchronised
// per wave), else the whole workgroup (one team).
template <typename T, int D, int KB, int VW>
__global__ __launch_bounds__(512) void k_restrict0_mr(Basis1D<T> bs, int nr, int tsize, const int* __restrict__ leaf_off,
                                                      const int* __restrict__ owner, const T* __restrict__ xi,
                                                      const T* __restrict__ src, T* bnext,
                                                      const T* __restrict__ dinv_next, T* dnext, T inv_theta_next,
                                                      const int* __restrict__ skip) {
  using VT = typename ColVec<T, VW>::type;
  constexpr int B = D == 3 ? KB * KB * KB : KB * KB;
  constexpr int P = 32;
  constexpr int LW = D * KB;  // 1D values per point
  if (skip && *skip) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nch = nr / VW;
  const int nteam = blockDim.x / tsize, team = threadIdx.x / tsize, tt = threadIdx.x - team * tsize;
  const bool wave_teams = nteam > 1;  // then tsize == 64
  const size_t region = ((size_t)P * nch * sizeof(VT) + (size_t)P * LW * sizeof(T) + 15) / 16 * 16;
  VT* ss = reinterpret_cast<VT*>(smem_raw + team * region);  // [P][nch] entries of src
  T* lt = reinterpret_cast<T*>(ss + P * nch);                  // [P][LW] 1D values
  auto team_sync = [&]() {
    if (wave_teams) {
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
      __syncthreads();
    }
  };
  const int K = blockIdx.x;
  const int i0 = leaf_off[K], i1 = leaf_off[K + 1];
  const int g = tt / nch, j = tt - g * nch;
  const bool active = g < B / KB;
  const int q1 = g % KB, q2 = g / KB;
  VT acc[KB];
#pragma unroll
  for (int a = 0; a < KB; ++a) acc[a] = (VT)0;
  for (int base = i0 + team * P; base < i1; base += nteam * P) {
    const int np = min(P, i1 - base);
    for (int t = tt; t < np * nch; t += tsize) {
      const int pp = t / nch, jj = t - pp * nch;
      const int i = base + pp;
      const VT sv = *reinterpret_cast<const VT*>(src + (int64_t)i * nr + jj * VW);
      ss[t] = owner[i] >= 0 ? sv : (VT)0;
    }
    if (tt < np) {
      const int i = base + tt;
      T l[3][4];
#pragma unroll
      for (int a = 0; a < D; ++a) lag1d_k<T, KB>(bs, xi[(int64_t)i * D + a], l[a]);
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int m = 0; m < KB; ++m) lt[tt * LW + a * KB + m] = l[a][m];
    }
    team_sync();
    if (active) {
      for (int pp = 0; pp < np; ++pp) {
        const T* lp = lt + pp * LW;
        T l12 = lp[KB + q1];
        if (D == 3) l12 *= lp[2 * KB + q2];
        const VT sv = ss[pp * nch + j];
#pragma unroll
        for (int a = 0; a < KB; ++a) acc[a] += (lp[a] * l12) * sv;
      }
    }
    team_sync();
  }
  if (wave_teams) {  // team sums through LDS, added in team order by team 0
    VT* comb = reinterpret_cast<VT*>(smem_raw + nteam * region);  // [nteam][KB][64]
#pragma unroll
    for (int a = 0; a < KB; ++a) comb[(team * KB + a) * 64 + tt] = acc[a];
    __syncthreads();
    if (team != 0) return;
#pragma unroll
    for (int a = 0; a < KB; ++a) {
      VT t = comb[a * 64 + tt];
      for (int u = 1; u < nteam; ++u) t += comb[(u * KB + a) * 64 + tt];
      acc[a] = t;
    }
  }
  if (active) {
#pragma unroll
    for (int a = 0; a < KB; ++a) {
      const int64_t row = (int64_t)K * B + g * KB + a;
      *reinterpret_cast<VT*>(bnext + row * nr + j * VW) = acc[a];
      if (dnext) *reinterpret_cast<VT*>(dnext + row * nr + j * VW) = (dinv_next[row] * acc[a]) * inv_theta_next;
    }
  }
}

template <typename T>
void launch_restrict0(int nbox, int64_t n_points, int d, int pc, int nr, const int* leaf_off, const int* owner,
                      const T* xi, const T* src, T* bnext, const T* dinv_next, T* dnext, double inv_theta_next,
                      const int* skip, hipStream_t s) {
  const int k = pc + 1;
  const int B = (d == 3) ? k * k * k : k * k;
  if (nbox == 0) return;
  // waves per box: one per 128-point chunk of an average box, at most 4
  int W = 1;
  while (W < 4 && (int64_t)W * 128 * nbox < n_points) W <<= 1;
  auto lds = [&](int w) { return sizeof(T) * ((size_t)w * (B * 65 + 64) + (size_t)w * 64); };
  while (W > 1 && lds(W) > 65536) W >>= 1;
  const Basis1D<T> bs = make_basis<T>(pc);
  constexpr int VW = col_vw<T>();
  if (nr > 1 && nr % std::min(nr, VW) == 0 && aligned16(src) && aligned16(bnext) && (!dnext || aligned16(dnext))) {
    const int vw = std::min(nr, VW), nch = nr / vw;
    const int tsize = ((B / k) * nch + 63) / 64 * 64;  // threads of a team
    if (tsize > 512) throw std::runtime_error("restriction: too many columns");
    const int nteam = tsize == 64 ? 4 : 1, thr = tsize * nteam;
    const size_t esz = vw * sizeof(T);  // bytes of one column chunk
    const size_t region = ((size_t)32 * nch * esz + (size_t)32 * d * k * sizeof(T) + 15) / 16 * 16;
    const size_t shm = nteam * region + (nteam > 1 ? (size_t)nteam * k * 64 * esz : 0);
#define R3MG_R0M(DD, KK)                                                                                           \
  do {                                                                                                             \
    if (vw == 2)                                                                                                   \
      hipLaunchKernelGGL((k_restrict0_mr<T, DD, KK, 2>), dim3(nbox), dim3(thr), shm, s, bs, nr, tsize, leaf_off,    \
                         owner, xi, src, bnext, dinv_next, dnext, (T)inv_theta_next, skip);                          \
    else                                                                                                           \
      hipLaunchKernelGGL((k_restrict0_mr<T, DD, KK, VW>), dim3(nbox), dim3(thr), shm, s, bs, nr, tsize, leaf_off,   \
                         owner, xi, src, bnext, dinv_next, dnext, (T)inv_theta_next, skip);                          \
  } while (0)
    switch (d * 8 + k) {
      case 17: R3MG_R0M(2, 1); break;
      case 18: R3MG_R0M(2, 2); break;
      case 19: R3MG_R0M(2, 3); break;
      case 20: R3MG_R0M(2, 4); break;
      case 25: R3MG_R0M(3, 1); break;
      case 26: R3MG_R0M(3, 2); break;
      case 27: R3MG_R0M(3, 3); break;
      case 28: R3MG_R0M(3, 4); break;
      default: throw std::runtime_error("restriction: unsupported dimension or degree");
    }
#undef R3MG_R0M
    check_launch("k_restrict0_mr");
    return;
  }
#define R3MG_R0(DD, KK)                                                                                           \
  hipLaunchKernelGGL((k_restrict0<T, DD, KK>), dim3(nbox), dim3(64 * W), lds(W), s, bs, nr, leaf_off, owner, xi, src, \
                     bnext, dinv_next, dnext, (T)inv_theta_next, skip)
  switch (d * 8 + k) {
    case 17: R3MG_R0(2, 1); break;
    case 18: R3MG_R0(2, 2); break;
    case 19: R3MG_R0(2, 3); break;
    case 20: R3MG_R0(2, 4); break;
    case 25: R3MG_R0(3, 1); break;
    case 26: R3MG_R0(3, 2); break;
    case 27: R3MG_R0(3, 3); break;
    case 28: R3MG_R0(3, 4); break;
    default: throw std::runtime_error("restriction: unsupported dimension or degree");
  }
#undef R3MG_R0
  check_launch("k_restrict0");
}
template void launch_restrict0<float>(int, int64_t, int, int, int, const int*, const int*, const float*,
                                      const float*, float*, const float*, float*, double, const int*, hipStream_t);
template void launch_restrict0<double>(int, int64_t, int, int, int, const int*, const int*, const double*,
                                       const double*, double*, const double*, double*, double, const int*,
                                       hipStream_t);

// Prolongation from the first agglomerated level: v_i = sum_q phi^K_q(xi_i) (e + epend)[K*B+q] (0 if i is
// constrained).  One thread per fine point.
template <typename T, int D, int KB>
__global__ __launch_bounds__(256) void k_prolong0(int n, Basis1D<T> bs, int nr, const int* __restrict__ owner,
                                                  const T* __restrict__ xi, const T* __restrict__ e,
                                                  const T* __restrict__ epend, T* v, const int* __restrict__ skip,
                                                  int nlog) {
  constexpr int B = D == 3 ? KB * KB * KB : KB * KB;
  if (skip && *skip) return;
  const int lb = xcd_block(nlog);
  if (lb < 0) return;
  const int i = lb * 256 + threadIdx.x;
  if (i >= n) return;
  const int K = owner[i];
  if (K < 0) {
    for (int c = 0; c < nr; ++c) v[(int64_t)i * nr + c] = 0;
    return;
  }
  T l[3][4];
#pragma unroll
  for (int a = 0; a < D; ++a) lag1d_k<T, KB>(bs, xi[(int64_t)i * D + a], l[a]);
  for (int c = 0; c < nr; ++c) {
    T s = 0;
    for_each_phi<T, D, KB>(l, [&](int q, T ph) {
      const int64_t o = ((int64_t)K * B + q) * nr + c;
      T ev = e[o];
      if (epend) ev += epend[o];
      s += ph * ev;
    });
    v[(int64_t)i * nr + c] = s;
  }
}

// The same for nr > 1 columns: one workgroup per level-1 box K (its points are leaf_off[K] .. leaf_off[K+1] - 1,
// owned by K or constrained).  The box's B coarse entries of e + epend (all columns) are formed once in LDS; thread
// (i, j) of the box then takes fine point i and column chunk j (chunks of one point adjacent), in k_prolong0's
// order.  Reading the entries from LDS instead of L2 for every point and chunk was what bounded the kernel.
template <typename T, int D, int KB, int VW>
__global__ __launch_bounds__(256) void k_prolong0_mr(Basis1D<T> bs, int nr, const int* __restrict__ leaf_off,
                                                     const int* __restrict__ owner, const T* __restrict__ xi,
                                                     const T* __restrict__ e, const T* __restrict__ epend, T* v,
                                                     const int* __restrict__ skip) {
  using VT = typename ColVec<T, VW>::type;
  constexpr int B = D == 3 ? KB * KB * KB : KB * KB;
  if (skip && *skip) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  VT* es = reinterpret_cast<VT*>(smem_raw);  // [B][nch]
  const int nch = nr / VW;
  const int K = blockIdx.x;
  const int i0 = leaf_off[K], i1 = leaf_off[K + 1];
  for (int t = threadIdx.x; t < B * nch; t += blockDim.x) {
    const int64_t o = (int64_t)K * B * nr + (int64_t)t * VW;  // entry (K B + t / nch), chunk t % nch
    VT ev = *reinterpret_cast<const VT*>(e + o);
    if (epend) ev += *reinterpret_cast<const VT*>(epend + o);
    es[t] = ev;
  }
  __syncthreads();
  const int total = (i1 - i0) * nch;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int i = i0 + idx / nch, j = idx - (idx / nch) * nch;
    const int ow = owner[i];  // unconditional loads; a constrained point's value is replaced by zero
    T l[3][4];
#pragma unroll
    for (int a = 0; a < D; ++a) lag1d_k<T, KB>(bs, xi[(int64_t)i * D + a], l[a]);
    VT sum = (VT)0;
    for_each_phi<T, D, KB>(l, [&](int q, T ph) { sum += ph * es[q * nch + j]; });
    *reinterpret_cast<VT*>(v + (int64_t)i * nr + j * VW) = ow < 0 ? (VT)0 : sum;
  }
}

template <typename T>
void launch_prolong0(int n, int nbox, int d, int pc, int nr, const int* leaf_off, const int* owner, const T* xi,
                     const T* e, const T* epend, T* v, const int* skip, hipStream_t s) {
  const Basis1D<T> bs = make_basis<T>(pc);
  constexpr int VW = col_vw<T>();
  if (nr > 1 && nr % std::min(nr, VW) == 0 && aligned16(e) && (!epend || aligned16(epend)) && aligned16(v)) {
    const int vw = std::min(nr, VW), nch = nr / vw;
    const int k = pc + 1, B = (d == 3) ? k * k * k : k * k;
    if (nbox == 0) return;
    const size_t shm = (size_t)16 * B * nch;
#define R3MG_P0M(DD, KK)                                                                                           \
  do {                                                                                                             \
    if (vw == 2)                                                                                                   \
      hipLaunchKernelGGL((k_prolong0_mr<T, DD, KK, 2>), dim3(nbox), dim3(256), shm, s, bs, nr, leaf_off, owner, xi, \
                         e, epend, v, skip);                                                                         \
    else                                                                                                           \
      hipLaunchKernelGGL((k_prolong0_mr<T, DD, KK, VW>), dim3(nbox), dim3(256), shm, s, bs, nr, leaf_off, owner,    \
                         xi, e, epend, v, skip);                                                                     \
  } while (0)
    switch (d * 8 + pc + 1) {
      case 17: R3MG_P0M(2, 1); break;
      case 18: R3MG_P0M(2, 2); break;
      case 19: R3MG_P0M(2, 3); break;
      case 20: R3MG_P0M(2, 4); break;
      case 25: R3MG_P0M(3, 1); break;
      case 26: R3MG_P0M(3, 2); break;
      case 27: R3MG_P0M(3, 3); break;
      case 28: R3MG_P0M(3, 4); break;
      default: throw std::runtime_error("prolongation: unsupported dimension or degree");
    }
#undef R3MG_P0M
    check_launch("k_prolong0_mr");
    return;
  }
  const int nlog = (n + 255) / 256;
  if (nlog == 0) return;
#define R3MG_P0(DD, KK)                                                                                            \
  hipLaunchKernelGGL((k_prolong0<T, DD, KK>), dim3(xcd_grid(nlog)), dim3(256), 0, s, n, bs, nr, owner, xi, e, epend, v, \
                     skip, nlog)
  switch (d * 8 + pc + 1) {
    case 17: R3MG_P0(2, 1); break;
    case 18: R3MG_P0(2, 2); break;
    case 19: R3MG_P0(2, 3); break;
    case 20: R3MG_P0(2, 4); break;
    case 25: R3MG_P0(3, 1); break;
    case 26: R3MG_P0(3, 2); break;
    case 27: R3MG_P0(3, 3); break;
    case 28: R3MG_P0(3, 4); break;
    default: throw std::runtime_error("prolongation: unsupported dimension or degree");
  }
#undef R3MG_P0
  check_launch("k_prolong0");
}
template void launch_prolong0<float>(int, int, int, int, int, const int*, const int*, const float*, const float*,
                                     const float*, float*, const int*, hipStream_t);
template void launch_prolong0<double>(int, int, int, int, int, const int*, const int*, const double*,
                                      const double*, const double*, double*, const int*, hipStream_t);

// P~ entry [q'][q] of child box c: prod_a M_c[a][q'_a][q_a]
template <typename T>
__device__ inline T pt_entry(const T* __restrict__ pt, int64_t c, int d, int k, int qc, int qp) {
  const T* m = pt + (int64_t)c * d * k * k;
  T v = m[(0 * k + qc % k) * k + qp % k];
  qc /= k;
  qp /= k;
  v *= m[(1 * k + qc % k) * k + qp % k];
  if (d == 3) {
    qc /= k;
    qp /= k;
    v *= m[(2 * k + qc % k) * k + qp % k];
  }
  return v;
}

// Restriction between agglomerated levels: b[G*B+q] = sum_{C child of G} sum_q' P~_C[q'][q] src[C*B+q'].
// One wave per parent box G (4 per workgroup): the children's entries and 1D injection factors are staged in
// LDS, then lane q sums over the children in order and over q' in ascending order, each P~ entry formed as the
// product of its 1D factors in axis order.
template <typename T>
__global__ __launch_bounds__(256) void k_restrict_c(int nbox_next, int nbox, int shift, int d, int k, int nr,
                                                    const T* __restrict__ pt, const T* __restrict__ src, T* bnext,
                                                    const T* __restrict__ dinv_next, T* dnext, T inv_theta_next,
                                                    const int* __restrict__ skip) {
  if (skip && *skip) return;
  extern __shared__ unsigned char smem_raw[];
  const int B = (d == 3) ? k * k * k : k * k;
  const int kk = k * k;
  const int nch = 1 << shift;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int G = blockIdx.x * 4 + wv;
  if (G >= nbox_next) return;  // whole wave leaves; only wave-level barriers follow
  T* srcs = reinterpret_cast<T*>(smem_raw) + (size_t)wv * nch * (B + d * kk);
  T* pts = srcs + nch * B;
  const int c0 = G << shift;
  const int c1 = min(nbox, (G + 1) << shift);
  const int nc = c1 - c0;
  for (int t = lane; t < nc * d * kk; t += 64) pts[t] = pt[(int64_t)c0 * d * kk + t];
  int q0 = 0, q1 = 0, q2 = 0;
  if (lane < B) {
    q0 = lane % k;
    q1 = (lane / k) % k;
    q2 = lane / kk;
  }
  for (int c = 0; c < nr; ++c) {
    for (int t = lane; t < nc * B; t += 64) srcs[t] = src[((int64_t)c0 * B + t) * nr + c];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < B) {
      T s = 0;
      for (int C = 0; C < nc; ++C) {
        const T* m = pts + C * d * kk;
        const T* sc = srcs + C * B;
        int qc = 0;
        for (int a2 = 0; a2 < (d == 3 ? k : 1); ++a2)
          for (int a1 = 0; a1 < k; ++a1)
            for (int a0 = 0; a0 < k; ++a0, ++qc) {
              T v = m[a0 * k + q0] * m[kk + a1 * k + q1];
              if (d == 3) v *= m[2 * kk + a2 * k + q2];
              s += v * sc[qc];
            }
      }
      const int64_t t = (int64_t)G * B + lane;
      bnext[t * nr + c] = s;
      if (dnext) dnext[t * nr + c] = dinv_next[t] * s * inv_theta_next;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// The same for nr > 1 columns: one workgroup per parent box G, thread (q, j) takes coarse function q and column
// chunk j.  The children's 1D injection factors are staged in LDS once, each child's B x nr entries (contiguous in
// src) one child at a time.
template <typename T, int VW>
__global__ __launch_bounds__(512) void k_restrict_c_mr(int nbox_next, int nbox, int shift, int d, int k, int nr,
                                                       const T* __restrict__ pt, const T* __restrict__ src, T* bnext,
                                                       const T* __restrict__ dinv_next, T* dnext, T inv_theta_next,
                                                       const int* __restrict__ skip) {
  using VT = typename ColVec<T, VW>::type;
  if (skip && *skip) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int B = (d == 3) ? k * k * k : k * k;
  const int kk = k * k;
  const int nch = nr / VW;
  VT* srcs = reinterpret_cast<VT*>(smem_raw);  // [B][nch] of the current child
  T* pts = reinterpret_cast<T*>(srcs + B * nch);
  const int G = blockIdx.x;
  const int c0 = G << shift;
  const int nc = min(nbox, (G + 1) << shift) - c0;
  for (int t = threadIdx.x; t < nc * d * kk; t += blockDim.x) pts[t] = pt[(int64_t)c0 * d * kk + t];
  const int q = threadIdx.x / nch, j = threadIdx.x - q * nch;
  const bool active = q < B;
  const int q0 = q % k, q1 = (q / k) % k, q2 = q / kk;
  VT acc = (VT)0;
  for (int C = 0; C < nc; ++C) {
    __syncthreads();
    const VT* sg = reinterpret_cast<const VT*>(src + (int64_t)(c0 + C) * B * nr);
    for (int t = threadIdx.x; t < B * nch; t += blockDim.x) srcs[t] = sg[t];
    __syncthreads();
    if (active) {
      const T* m = pts + C * d * kk;
      int qc = 0;
      for (int a2 = 0; a2 < (d == 3 ? k : 1); ++a2)
        for (int a1 = 0; a1 < k; ++a1)
          for (int a0 = 0; a0 < k; ++a0, ++qc) {
            T w = m[a0 * k + q0] * m[kk + a1 * k + q1];
            if (d == 3) w *= m[2 * kk + a2 * k + q2];
            acc += w * srcs[qc * nch + j];
          }
    }
  }
  if (active) {
    const int64_t row = (int64_t)G * B + q;
    *reinterpret_cast<VT*>(bnext + row * nr + j * VW) = acc;
    if (dnext) *reinterpret_cast<VT*>(dnext + row * nr + j * VW) = (dinv_next[row] * acc) * inv_theta_next;
  }
}

template <typename T>
void launch_restrict_c(int nbox_next, int nbox, int shift, int d, int pc, int nr, const T* pt, const T* src,
                       T* bnext, const T* dinv_next, T* dnext, double inv_theta_next, const int* skip,
                       hipStream_t s) {
  const int k = pc + 1;
  const int B = (d == 3) ? k * k * k : k * k;
  if (nbox_next == 0) return;
  if (B > 64) throw std::runtime_error("restriction: more than 64 coarse functions per box");
  constexpr int VW = col_vw<T>();
  if (nr > 1 && nr % std::min(nr, VW) == 0 && aligned16(src) && aligned16(bnext) && (!dnext || aligned16(dnext))) {
    const int vw = std::min(nr, VW), nch = nr / vw;
    const int thr = (B * nch + 63) / 64 * 64;
    if (thr > 512) throw std::runtime_error("restriction: too many columns");
    const size_t shmm = sizeof(T) * ((size_t)B * nr + (size_t)(1 << shift) * d * k * k);
    if (vw == 2)
      hipLaunchKernelGGL((k_restrict_c_mr<T, 2>), dim3(nbox_next), dim3(thr), shmm, s, nbox_next, nbox, shift, d, k, nr,
                         pt, src, bnext, dinv_next, dnext, (T)inv_theta_next, skip);
    else
      hipLaunchKernelGGL((k_restrict_c_mr<T, VW>), dim3(nbox_next), dim3(thr), shmm, s, nbox_next, nbox, shift, d, k,
                         nr, pt, src, bnext, dinv_next, dnext, (T)inv_theta_next, skip);
    check_launch("k_restrict_c_mr");
    return;
  }
  const size_t shm = sizeof(T) * (size_t)4 * (1 << shift) * (B + d * k * k);
  hipLaunchKernelGGL((k_restrict_c<T>), dim3((unsigned)((nbox_next + 3) / 4)), dim3(256), shm, s, nbox_next, nbox, shift,
                     d, k, nr, pt, src, bnext, dinv_next, dnext, (T)inv_theta_next, skip);
  check_launch("k_restrict_c");
}
template void launch_restrict_c<float>(int, int, int, int, int, int, const float*, const float*, float*,
                                       const float*, float*, double, const int*, hipStream_t);
template void launch_restrict_c<double>(int, int, int, int, int, int, const double*, const double*, double*,
                                        const double*, double*, double, const int*, hipStream_t);

// Prolongation between agglomerated levels: v[C*B+q'] = sum_q P~_C[q'][q] (e + epend)[G*B+q], G = C >> shift.
template <typename T>
__global__ __launch_bounds__(256) void k_prolong_c(int nbox, int shift, int d, int k, int nr, const T* __restrict__ pt,
                                                   const T* __restrict__ e, const T* __restrict__ epend, T* v,
                                                   const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int B = (d == 3) ? k * k * k : k * k;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)nbox * B) return;
  const int C = (int)(t / B), qc = (int)(t - (int64_t)C * B);
  const int G = C >> shift;
  for (int c = 0; c < nr; ++c) {
    T s = 0;
    for (int q = 0; q < B; ++q) {
      const int64_t o = ((int64_t)G * B + q) * nr + c;
      T ev = e[o];
      if (epend) ev += epend[o];
      s += pt_entry(pt, C, d, k, qc, q) * ev;
    }
    v[t * nr + c] = s;
  }
}

// The same for nr > 1 columns: thread (C B + q', j) takes one fine entry and column chunk j.
template <typename T, int VW>
__global__ __launch_bounds__(256) void k_prolong_c_mr(int nbox, int shift, int d, int k, int nr,
                                                      const T* __restrict__ pt, const T* __restrict__ e,
                                                      const T* __restrict__ epend, T* v, const int* __restrict__ skip) {
  using VT = typename ColVec<T, VW>::type;
  if (skip && *skip) return;
  const int B = (d == 3) ? k * k * k : k * k;
  const int nch = nr / VW;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)nbox * B * nch) return;
  const int64_t row = t / nch;
  const int j = (int)(t - row * nch);
  const int C = (int)(row / B), qc = (int)(row - (int64_t)C * B);
  const int G = C >> shift;
  VT sum = (VT)0;
  for (int q = 0; q < B; ++q) {
    const int64_t o = ((int64_t)G * B + q) * nr + j * VW;
    VT ev = *reinterpret_cast<const VT*>(e + o);
    if (epend) ev += *reinterpret_cast<const VT*>(epend + o);
    sum += pt_entry(pt, C, d, k, qc, q) * ev;
  }
  *reinterpret_cast<VT*>(v + row * nr + j * VW) = sum;
}

template <typename T>
void launch_prolong_c(int nbox, int shift, int d, int pc, int nr, const T* pt, const T* e, const T* epend, T* v,
                      const int* skip, hipStream_t s) {
  const int k = pc + 1;
  const int B = (d == 3) ? k * k * k : k * k;
  constexpr int VW = col_vw<T>();
  if (nr > 1 && nr % std::min(nr, VW) == 0 && aligned16(e) && (!epend || aligned16(epend)) && aligned16(v)) {
    const int vw = std::min(nr, VW);
    const int64_t totm = (int64_t)nbox * B * (nr / vw);
    if (totm == 0) return;
    if (vw == 2)
      hipLaunchKernelGGL((k_prolong_c_mr<T, 2>), dim3((unsigned)((totm + 255) / 256)), dim3(256), 0, s, nbox, shift, d,
                         k, nr, pt, e, epend, v, skip);
    else
      hipLaunchKernelGGL((k_prolong_c_mr<T, VW>), dim3((unsigned)((totm + 255) / 256)), dim3(256), 0, s, nbox, shift,
                         d, k, nr, pt, e, epend, v, skip);
    check_launch("k_prolong_c_mr");
    return;
  }
  const int64_t tot = (int64_t)nbox * B;
  hipLaunchKernelGGL((k_prolong_c<T>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, nbox, shift, d, k, nr, pt,
                     e, epend, v, skip);
  check_launch("k_prolong_c");
}
template void launch_prolong_c<float>(int, int, int, int, int, const float*, const float*, const float*, float*,
                                      const int*, hipStream_t);
template void launch_prolong_c<double>(int, int, int, int, int, const double*, const double*, const double*,
                                       double*, const int*, hipStream_t);

// =============================================================================================
// Elementwise helpers
// =============================================================================================
template <typename T>
__global__ void k_xupdate(int64_t count, T* x, const T* __restrict__ v, int assign, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  x[i] = assign ? v[i] : x[i] + v[i];
}
template <typename T>
void launch_xupdate(int64_t count, T* x, const T* v, int assign, const int* skip, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL((k_xupdate<T>), dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count, x, v, assign, skip);
  check_launch("k_xupdate");
}
template void launch_xupdate<float>(int64_t, float*, const float*, int, const int*, hipStream_t);
template void launch_xupdate<double>(int64_t, double*, const double*, int, const int*, hipStream_t);

// V-cycle entry: b0[i] = r_user[perm[i]] (column c at r_user + c*ld), d0 = dinv * b0 * inv_theta
template <typename T>
__global__ void k_vc_entry(int n, int nr, const int* __restrict__ perm, const double* __restrict__ r, int64_t ld,
                           T* b0, const T* __restrict__ dinv, T* d0, T inv_theta) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)n * nr) return;
  const int i = (int)(t / nr), c = (int)(t - (int64_t)i * nr);
  const T v = (T)r[(int64_t)c * ld + perm[i]];
  b0[t] = v;
  if (d0) d0[t] = dinv[i] * v * inv_theta;
}
template <typename T>
void launch_vc_entry(int n, int nr, const int* perm, const double* r_user, int64_t ld_user, T* b0, const T* dinv,
                     T* d0, double inv_theta, hipStream_t s) {
  const int64_t tot = (int64_t)n * nr;
  hipLaunchKernelGGL((k_vc_entry<T>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, nr, perm, r_user, ld_user,
                     b0, dinv, d0, (T)inv_theta);
  check_launch("k_vc_entry");
}
template void launch_vc_entry<float>(int, int, const int*, const double*, int64_t, float*, const float*, float*,
                                     double, hipStream_t);
template void launch_vc_entry<double>(int, int, const int*, const double*, int64_t, double*, const double*,
                                      double*, double, hipStream_t);

template <typename T>
__global__ void k_vc_exit(int n, int nr, const int* __restrict__ perm, const T* __restrict__ x0,
                          const T* __restrict__ dp, double* z, int64_t ld) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)n * nr) return;
  const int i = (int)(t / nr), c = (int)(t - (int64_t)i * nr);
  T v = x0[t];
  if (dp) v += dp[t];
  z[(int64_t)c * ld + perm[i]] = (double)v;
}
template <typename T>
void launch_vc_exit(int n, int nr, const int* perm, const T* x0, const T* dpend, double* z_user, int64_t ld_user,
                    hipStream_t s) {
  const int64_t tot = (int64_t)n * nr;
  hipLaunchKernelGGL((k_vc_exit<T>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, nr, perm, x0, dpend,
                     z_user, ld_user);
  check_launch("k_vc_exit");
}
template void launch_vc_exit<float>(int, int, const int*, const float*, const float*, double*, int64_t, hipStream_t);
template void launch_vc_exit<double>(int, int, const int*, const double*, const double*, double*, int64_t,
                                     hipStream_t);

// Dense coarsest solve x = A_L^{-1} b with the float64 explicit inverse (one wave per row).
template <typename T, int NR>
__global__ __launch_bounds__(256) void k_dense_apply(int nc, const double* __restrict__ cinv, const T* __restrict__ b,
                                                     T* x, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= nc) return;
  double acc[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = 0;
  const double* a = cinv + (int64_t)row * nc;
  int c = lane;
  for (; c + 192 < nc; c += 256) {  // four independent loads in flight per lane
    const double m0 = a[c], m1 = a[c + 64], m2 = a[c + 128], m3 = a[c + 192];
#pragma unroll
    for (int k = 0; k < NR; ++k)
      acc[k] += (m0 * (double)b[(int64_t)c * NR + k] + m1 * (double)b[(int64_t)(c + 64) * NR + k]) +
                (m2 * (double)b[(int64_t)(c + 128) * NR + k] + m3 * (double)b[(int64_t)(c + 192) * NR + k]);
  }
  for (; c < nc; c += 64) {
    const double m = a[c];
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k] += m * (double)b[(int64_t)c * NR + k];
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    acc[k] = wave_sum(acc[k], 64);
    if (lane == k) x[(int64_t)row * NR + k] = (T)acc[k];
  }
}
template <typename T>
void launch_dense_apply(int nc, int nr, const double* cinv, const T* b, T* x, const int* skip, hipStream_t s) {
  dim3 g((nc + 3) / 4);
  switch (nr) {
    case 1: hipLaunchKernelGGL((k_dense_apply<T, 1>), g, dim3(256), 0, s, nc, cinv, b, x, skip); break;
    case 2: hipLaunchKernelGGL((k_dense_apply<T, 2>), g, dim3(256), 0, s, nc, cinv, b, x, skip); break;
    case 4: hipLaunchKernelGGL((k_dense_apply<T, 4>), g, dim3(256), 0, s, nc, cinv, b, x, skip); break;
    case 8: hipLaunchKernelGGL((k_dense_apply<T, 8>), g, dim3(256), 0, s, nc, cinv, b, x, skip); break;
    case 16: hipLaunchKernelGGL((k_dense_apply<T, 16>), g, dim3(256), 0, s, nc, cinv, b, x, skip); break;
    default: throw std::runtime_error("unsupported nrhs block");
  }
  check_launch("k_dense_apply");
}
template void launch_dense_apply<float>(int, int, const double*, const float*, float*, const int*, hipStream_t);
template void launch_dense_apply<double>(int, int, const double*, const double*, double*, const int*, hipStream_t);

// Symmetric dense coarsest product.  Pass 1: one workgroup per upper tile (I, J); wave w holds the tile's rows
// 16 w .. 16 w + 15 in registers (stored as M = float64, or float32 for the float32 V-cycle, and widened to
// float64 where used: the products and partial sums are float64 either way), lane = column.  The row products
// are summed over the 64 lanes by a transposing butterfly (each step halves the rows a lane keeps and doubles
// the columns summed), which leaves lane l with row 8 b5 + 4 b4 + 2 b3 + b2 of its wave (b = bits of l).  The
// transposed products of an off-diagonal tile take the wave's 16 rows of b from LDS and are summed over the four
// waves in order.
template <typename T, typename M, int NR>
__global__ __launch_bounds__(256) void k_dense_sym_tiles(int nc, int nt, const M* __restrict__ packed,
                                                         const int2* __restrict__ tiles, const T* __restrict__ b,
                                                         double* part, const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double sh[4][64];
  __shared__ T sbr[4][16 * NR];  // wave w's 16 rows of b (0 past the last row), read at use (fewer registers)
  const int t = blockIdx.x;
  const int2 ij = tiles[t];
  const int I = ij.x, J = ij.y;
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const M* a = packed + (int64_t)t * (kDenseTile * kDenseTile) + (16 * w) * kDenseTile + lane;
  M m[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) m[k] = a[k * kDenseTile];
  const int cj = J * kDenseTile + lane;
  const int ri = I * kDenseTile + 16 * w;
  // the entries of b are loaded up front from clamped addresses and masked (loads under a lane-dependent
  // condition would each be waited for)
  T bj[NR];
#pragma unroll
  for (int c = 0; c < NR; ++c) bj[c] = b[(int64_t)min(cj, nc - 1) * NR + c];
  if (I != J) {  // uniform over the workgroup
    if (lane < 16) {
      const T* bp = b + (int64_t)min(ri + lane, nc - 1) * NR;
#pragma unroll
      for (int c = 0; c < NR; ++c) sbr[w][lane * NR + c] = ri + lane < nc ? bp[c] : (T)0;
    }
    __syncthreads();
  }
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4;
  const int myrow = (b5 ? 8 : 0) + (b4 ? 4 : 0) + (b3 ? 2 : 0) + (b2 ? 1 : 0);
  for (int c = 0; c < NR; ++c) {
    const double xj = cj < nc ? (double)bj[c] : 0.0;
    double h8[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double lo = (double)m[q] * xj, hi = (double)m[8 + q] * xj;
      h8[q] = (b5 ? hi : lo) + __shfl_xor(b5 ? lo : hi, 32, 64);
    }
    double h4[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) h4[q] = (b4 ? h8[4 + q] : h8[q]) + __shfl_xor(b4 ? h8[q] : h8[4 + q], 16, 64);
    double h2[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) h2[q] = (b3 ? h4[2 + q] : h4[q]) + __shfl_xor(b3 ? h4[q] : h4[2 + q], 8, 64);
    double h1 = (b2 ? h2[1] : h2[0]) + __shfl_xor(b2 ? h2[0] : h2[1], 4, 64);
    h1 += __shfl_xor(h1, 2, 64);
    h1 += __shfl_xor(h1, 1, 64);
    if ((lane & 3) == 0)
      part[(((int64_t)I * nt + J) * kDenseTile + 16 * w + myrow) * NR + c] = h1;
    if (I != J) {  // uniform over the workgroup
      double cs = 0;
#pragma unroll
      for (int k = 0; k < 16; ++k) cs += (double)m[k] * (double)sbr[w][k * NR + c];
      sh[w][lane] = cs;
      __syncthreads();
      if (w == 0)
        part[(((int64_t)J * nt + I) * kDenseTile + lane) * NR + c] = (sh[0][lane] + sh[1][lane]) +
                                                                      (sh[2][lane] + sh[3][lane]);
      __syncthreads();
    }
  }
}

// Pass 2: the sum of row `row`'s nt slots, as taken by thread (g, i) of a 16 x 16 group (g = slot group, i =
// row): slot S is taken by group S % 16 in index order, the group sums go to sh[g][i], and sum16 adds the 16 groups
// in order.
__device__ inline double dense_slot_sum(int nt, const double* __restrict__ part, int row, int g, int nr, int c) {
  const int R = row / kDenseTile, i = row - R * kDenseTile;
  double acc = 0;
#pragma unroll 4
  for (int S = g; S < nt; S += 16) acc += part[(((int64_t)R * nt + S) * kDenseTile + i) * nr + c];
  return acc;
}
__device__ inline double dense_sum16(const double (*sh)[17], int i) {
  double t = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) t += sh[k][i];
  return t;
}

// Pass 2 alone: rows 16 Q .. 16 Q + 15 of row block R = blockIdx.x / 4 (Q = blockIdx.x % 4).
template <typename T, int NR>
__global__ __launch_bounds__(256) void k_dense_sym_reduce(int nc, int nt, const double* __restrict__ part, T* x,
                                                          const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double sh[16][17];
  const int R = blockIdx.x >> 2, i = 16 * (blockIdx.x & 3) + (threadIdx.x & 15), g = threadIdx.x >> 4;
  const int row = R * kDenseTile + i;
  for (int c = 0; c < NR; ++c) {
    sh[g][threadIdx.x & 15] = dense_slot_sum(nt, part, row, g, NR, c);
    __syncthreads();
    if (g == 0 && row < nc) x[(int64_t)row * NR + c] = (T)dense_sum16(sh, threadIdx.x & 15);
    __syncthreads();
  }
}

// Pass 2 fused with the prolongation to the level above (k_prolong_c with no pending direction): one workgroup
// per parent box G of that level (= box G of the coarsest level, B rows).  Its B rows of x are summed from the
// slots as in k_dense_sym_reduce (16 rows at a time), stored, and kept in LDS; then thread (C, q') of G's
// children forms v[C*B+q'] = sum_q P~_C[q'][q] x[G*B+q] in ascending q.
template <typename T, int NR>
__global__ __launch_bounds__(256) void k_dense_sym_reduce_prolong(int nbox, int shift, int d, int k, int nt,
                                                                  const double* __restrict__ part, T* x,
                                                                  const T* __restrict__ pt, T* v,
                                                                  const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double sh[16][17];
  __shared__ T xs[64 * NR];
  const int B = (d == 3) ? k * k * k : k * k;
  const int G = blockIdx.x;
  const int g = threadIdx.x >> 4, i = threadIdx.x & 15;
  for (int r0 = 0; r0 < B; r0 += 16) {
    const int r = r0 + i;
    for (int c = 0; c < NR; ++c) {
      if (r < B) sh[g][i] = dense_slot_sum(nt, part, G * B + r, g, NR, c);
      __syncthreads();
      if (g == 0 && r < B) {
        const T t = (T)dense_sum16(sh, i);
        x[((int64_t)G * B + r) * NR + c] = t;
        xs[r * NR + c] = t;
      }
      __syncthreads();
    }
  }
  const int c0 = G << shift;
  const int nch = min(nbox, (G + 1) << shift) - c0;
  for (int t = threadIdx.x; t < nch * B; t += blockDim.x) {
    const int C = c0 + t / B, qc = t % B;
    for (int c = 0; c < NR; ++c) {
      T s = 0;
      for (int q = 0; q < B; ++q) s += pt_entry(pt, C, d, k, qc, q) * xs[q * NR + c];
      v[((int64_t)C * B + qc) * NR + c] = s;
    }
  }
}

template <typename M>
__global__ __launch_bounds__(256) void k_dense_pack_sym(int nc, const double* __restrict__ full,
                                                        const int2* __restrict__ tiles, M* packed) {
  const int t = blockIdx.x;
  const int2 ij = tiles[t];
  for (int e = threadIdx.x; e < kDenseTile * kDenseTile; e += 256) {
    const int i = ij.x * kDenseTile + e / kDenseTile, j = ij.y * kDenseTile + e % kDenseTile;
    packed[(int64_t)t * (kDenseTile * kDenseTile) + e] = (i < nc && j < nc) ? (M)full[(int64_t)i * nc + j] : (M)0;
  }
}
template <typename M>
void launch_dense_pack_sym(int nc, int ntiles, const double* full, const int* tiles, M* packed, hipStream_t s) {
  hipLaunchKernelGGL((k_dense_pack_sym<M>), dim3(ntiles), dim3(256), 0, s, nc, full,
                     reinterpret_cast<const int2*>(tiles), packed);
  check_launch("k_dense_pack_sym");
}
template void launch_dense_pack_sym<double>(int, int, const double*, const int*, double*, hipStream_t);
template void launch_dense_pack_sym<float>(int, int, const double*, const int*, float*, hipStream_t);

template <typename T, typename M>
void launch_dense_apply_sym(int nc, int nt, int nr, const M* packed, const int* tiles, double* part, const T* b,
                            T* x, const DenseProlong<T>* pr, const int* skip, hipStream_t s) {
  const int ntiles = nt * (nt + 1) / 2;
  const int2* tl = reinterpret_cast<const int2*>(tiles);
  int B = 0;
  if (pr) {
    B = pr->d == 3 ? (pr->pc + 1) * (pr->pc + 1) * (pr->pc + 1) : (pr->pc + 1) * (pr->pc + 1);
    if (B > 64 || (int64_t)B * pr->nbox_coarse != nc)
      throw std::runtime_error("dense coarsest product: prolongation boxes do not match the coarsest level");
  }
  switch (nr) {
#define R3_DS(NRV)                                                                                                  \
  hipLaunchKernelGGL((k_dense_sym_tiles<T, M, NRV>), dim3(ntiles), dim3(256), 0, s, nc, nt, packed, tl, b, part,   \
                     skip);                                                                                         \
  if (pr)                                                                                                           \
    hipLaunchKernelGGL((k_dense_sym_reduce_prolong<T, NRV>), dim3(pr->nbox_coarse), dim3(256), 0, s, pr->nbox,     \
                       pr->shift, pr->d, pr->pc + 1, nt, part, x, pr->pt, pr->v, skip);                             \
  else                                                                                                              \
    hipLaunchKernelGGL((k_dense_sym_reduce<T, NRV>), dim3(4 * nt), dim3(256), 0, s, nc, nt, part, x, skip);        \
  break;
    case 1: R3_DS(1)
    case 2: R3_DS(2)
    case 4: R3_DS(4)
#undef R3_DS
    default: throw std::runtime_error("symmetric dense coarsest product: unsupported nrhs block");
  }
  check_launch("k_dense_sym");
}
template void launch_dense_apply_sym<float, float>(int, int, int, const float*, const int*, double*, const float*,
                                                   float*, const DenseProlong<float>*, const int*, hipStream_t);
template void launch_dense_apply_sym<float, double>(int, int, int, const double*, const int*, double*,
                                                    const float*, float*, const DenseProlong<float>*, const int*,
                                                    hipStream_t);
template void launch_dense_apply_sym<double, double>(int, int, int, const double*, const int*, double*,
                                                     const double*, double*, const DenseProlong<double>*,
                                                     const int*, hipStream_t);

__global__ void k_gather_cols(int n, int nr, int nuser, const int* __restrict__ perm,
                              const double* __restrict__ user, int64_t ld, double* out) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)n * nr) return;
  const int i = (int)(t / nr), c = (int)(t - (int64_t)i * nr);
  out[t] = c < nuser ? user[(int64_t)c * ld + perm[i]] : 0.0;
}
void launch_gather_cols(int n, int nr, int nuser, const int* perm, const double* user, int64_t ld_user,
                        double* out, hipStream_t s) {
  const int64_t tot = (int64_t)n * nr;
  hipLaunchKernelGGL(k_gather_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, nr, nuser, perm, user,
                     ld_user, out);
  check_launch("k_gather_cols");
}
__global__ void k_scatter_cols(int n, int nr, int nuser, const int* __restrict__ perm,
                               const double* __restrict__ in, double* user, int64_t ld) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)n * nr) return;
  const int i = (int)(t / nr), c = (int)(t - (int64_t)i * nr);
  if (c < nuser) user[(int64_t)c * ld + perm[i]] = in[t];
}
void launch_scatter_cols(int n, int nr, int nuser, const int* perm, const double* in, double* user,
                         int64_t ld_user, hipStream_t s) {
  const int64_t tot = (int64_t)n * nr;
  hipLaunchKernelGGL(k_scatter_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, nr, nuser, perm, in,
                     user, ld_user);
  check_launch("k_scatter_cols");
}

__global__ void k_cast_d2f(int64_t count, const double* __restrict__ a, float* b) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) b[i] = (float)a[i];
}
void launch_cast_d2f(int64_t count, const double* a, float* b, hipStream_t s) {
  if (count == 0) return;
  int64_t g = (count + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_cast_d2f, dim3((unsigned)g), dim3(256), 0, s, count, a, b);
  check_launch("k_cast_d2f");
}

__global__ void k_gather_vals(int64_t nnz, const int64_t* __restrict__ src, const double* __restrict__ uv,
                              double* out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * 256) out[i] = uv[src[i]];
}
void launch_gather_vals(int64_t nnz, const int64_t* src, const double* user_vals, double* out, hipStream_t s) {
  if (nnz == 0) return;
  int64_t g = (nnz + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_gather_vals, dim3((unsigned)g), dim3(256), 0, s, nnz, src, user_vals, out);
  check_launch("k_gather_vals");
}

// =============================================================================================
// Set-up kernels
// =============================================================================================
// inverse diagonal of a level operator; *bad = 1 if any diagonal entry is not > 0
__global__ void k_diag_inv(int n, int blk, const int* __restrict__ ptr, const int* __restrict__ idx,
                           const double* __restrict__ val, double* dinv, double* diag, int* bad) {
  const int row = blockIdx.x * 256 + threadIdx.x;
  if (row >= n) return;
  double dv = 0.0;
  if (blk == 1) {
    int lo = ptr[row], hi = ptr[row + 1];
    while (lo < hi) {  // lower bound of `row`
      int mid = (lo + hi) >> 1;
      if (idx[mid] < row) lo = mid + 1; else hi = mid;
    }
    if (lo < ptr[row + 1] && idx[lo] == row) dv = val[lo];
  } else {
    const int K = row / blk, q = row - K * blk;
    const int j0 = ptr[K], nb = ptr[K + 1] - j0;
    int lo = j0, hi = j0 + nb;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (idx[mid] < K) lo = mid + 1; else hi = mid;
    }
    if (lo < j0 + nb && idx[lo] == K)
      dv = val[(int64_t)blk * blk * j0 + (int64_t)q * nb * blk + (int64_t)(lo - j0) * blk + q];
  }
  if (diag) diag[row] = dv;
  if (!(dv > 0.0)) {
    *bad = 1;
    dinv[row] = 0.0;
  } else {
    dinv[row] = 1.0 / dv;
  }
}
void launch_diag_inv(int n, int blk, const int* ptr, const int* idx, const double* val, double* dinv, double* diag,
                     int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_inv, dim3((n + 255) / 256), dim3(256), 0, s, n, blk, ptr, idx, val, dinv, diag, bad);
  check_launch("k_diag_inv");
}

// Galerkin product, fine -> first agglomerated level (Section 4, inherited operators):
// A1[K,K'] = sum_{i in K free} phi^K(x_i) T_i^T,  T_i[q'] = sum_{j in K' free} A_ij phi^K'_q'(x_j).
// One 256-thread workgroup per stored output block.  The host lists, per block, the rows i of K whose sorted
// columns meet box K' with the column run [s, e).  Eight 32-lane groups take eight entries at a time: group g
// evaluates phi^K(x_i) and T_i into LDS; then every thread adds sum_g phi_g[q] T_g[q'] to the entries (q, q') it
// owns.  For T_i the group's 32 lanes take 32 entries of the run at a time: each loads its entry's column, value,
// owner and coordinates (all 32 chains in flight together) and puts the 1D tables of x_j into LDS; then lane q'
// adds the products of those entries in the run's order.  The summation order is fixed (deterministic).  A1 is
// symmetric, so only the blocks with K <= K' are formed (workgroup t: block up[t]) and each off-diagonal one is
// also stored transposed as block mir[t] = (K', K).
template <int D, int KB>
__global__ __launch_bounds__(256) void k_galerkin0(Basis1D<double> bs, const int* __restrict__ up,
                                                   const int* __restrict__ mir, const int* __restrict__ brow,
                                                   const int* __restrict__ bptr, const int* __restrict__ gal_ptr,
                                                   const int* __restrict__ gal_ent, const int* __restrict__ owner,
                                                   const double* __restrict__ xi, const int* __restrict__ col,
                                                   const double* __restrict__ val, double* out) {
  __shared__ double spi[8][64];
  __shared__ double sT[8][64];
  __shared__ double sl[8][32][12];  // per group: the 1D tables l[a][j] (at 4 a + j) of 32 entries' x_j
  __shared__ double sv[8][32];      // their values A_ij
  __shared__ int sf[8][32];         // their column is free (owner >= 0)
  const int64_t blkid = up[blockIdx.x];
  const int K = brow[blkid];
  const int slot = (int)(blkid - bptr[K]);
  const int nbK = bptr[K + 1] - bptr[K];
  // dimension and degree are compile-time (lag1d_k and the digit arithmetic below unroll), with the same
  // operations in the same order as the run-time forms
  constexpr int d = D, k = KB;
  constexpr int B = D == 3 ? KB * KB * KB : KB * KB;
  constexpr int EMAX = (B * B + 255) / 256;
  int qi[EMAX], qj[EMAX];
  double acc[EMAX];
#pragma unroll
  for (int m = 0; m < EMAX; ++m) {
    const int e = threadIdx.x + m * 256;
    qi[m] = e < B * B ? e / B : -1;
    qj[m] = e < B * B ? e % B : 0;
    acc[m] = 0;
  }
  const int g = threadIdx.x >> 5, lt = threadIdx.x & 31;
  const int en0 = gal_ptr[blkid], en1 = gal_ptr[blkid + 1];
  for (int base = en0; base < en1; base += 8) {
    const int ent = base + g;
    if (ent < en1) {
      const int i = gal_ent[3 * ent], s = gal_ent[3 * ent + 1], e = gal_ent[3 * ent + 2];
      double li[3][4];
#pragma unroll
      for (int a = 0; a < d; ++a) lag1d_k<double, KB>(bs, xi[(int64_t)i * d + a], li[a]);
      for (int q = lt; q < B; q += 32) spi[g][q] = phi_q<double>(li, d, k, q);
      // lane lt owns q' = lt and lt + 32 (B <= 64); the digits of q' in base k pick the 1D tables
      int qd[2][3];
      double t[2] = {0.0, 0.0};
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const int q = lt + 32 * m;
        qd[m][0] = q % k;
        qd[m][1] = 4 + (q / k) % k;
        qd[m][2] = 8 + (q / k / k) % k;
      }
      for (int p0 = s; p0 < e; p0 += 32) {
        const int p = min(p0 + lt, e - 1);  // clamped: every lane loads, the lanes past the run store nothing
        const int j = col[p];
        const double v = val[p];
        const int own = owner[j];
        double lj[3][4] = {};
#pragma unroll
        for (int a = 0; a < d; ++a) lag1d_k<double, KB>(bs, xi[(int64_t)j * d + a], lj[a]);
        if (p0 + lt < e) {
          sv[g][lt] = v;
          sf[g][lt] = own >= 0;
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) sl[g][lt][4 * a + jj] = lj[a][jj];
        }
        // the group is half a wave: its LDS writes and reads stay in program order within the wave
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int cnt = min(32, e - p0);
        for (int u = 0; u < cnt; ++u) {
          if (!sf[g][u]) continue;  // the same for all lanes of the group
          const double vu = sv[g][u];
          const double* L = sl[g][u];
#pragma unroll
          for (int m = 0; m < 2; ++m)
            if (lt + 32 * m < B) {
              double ph = L[qd[m][0]];  // phi_q' = l0[q0] l1[q1] (l2[q2]), in phi_q's order
              ph *= L[qd[m][1]];
              if (d == 3) ph *= L[qd[m][2]];
              t[m] += vu * ph;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
#pragma unroll
      for (int m = 0; m < 2; ++m)
        if (lt + 32 * m < B) sT[g][lt + 32 * m] = t[m];
    } else {
      for (int q = lt; q < B; q += 32) {
        spi[g][q] = 0.0;
        sT[g][q] = 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < EMAX; ++m) {
      if (qi[m] >= 0) {
        double sacc = 0;
#pragma unroll
        for (int gg = 0; gg < 8; ++gg) sacc += spi[gg][qi[m]] * sT[gg][qj[m]];
        acc[m] += sacc;
      }
    }
    __syncthreads();
  }
  const int64_t obase = (int64_t)B * B * bptr[K];
#pragma unroll
  for (int m = 0; m < EMAX; ++m)
    if (qi[m] >= 0) out[obase + (int64_t)qi[m] * nbK * B + (int64_t)slot * B + qj[m]] = acc[m];
  const int mb = mir[blockIdx.x];
  if (mb >= 0) {  // uniform over the workgroup
    const int Km = brow[mb], slm = mb - bptr[Km], nbm = bptr[Km + 1] - bptr[Km];
    const int64_t mbase = (int64_t)B * B * bptr[Km];
#pragma unroll
    for (int m = 0; m < EMAX; ++m)
      if (qi[m] >= 0) out[mbase + (int64_t)qj[m] * nbm * B + (int64_t)slm * B + qi[m]] = acc[m];
  }
}

void launch_galerkin0(int64_t nup, int d, int pc, const int* up, const int* mir, const int* brow, const int* bptr,
                      const int* gal_ptr, const int* gal_ent, const int* owner, const double* xi, const int* col,
                      const double* val, double* out, hipStream_t s) {
  Basis1D<double> bs = make_basis<double>(pc);
  if (nup == 0) return;
#define R3MG_G0(DD, KK)                                                                                             \
  hipLaunchKernelGGL((k_galerkin0<DD, KK>), dim3((unsigned)nup), dim3(256), 0, s, bs, up, mir, brow, bptr, gal_ptr,  \
                     gal_ent, owner, xi, col, val, out)
  switch (d * 8 + pc + 1) {
    case 17: R3MG_G0(2, 1); break;
    case 18: R3MG_G0(2, 2); break;
    case 19: R3MG_G0(2, 3); break;
    case 20: R3MG_G0(2, 4); break;
    case 25: R3MG_G0(3, 1); break;
    case 26: R3MG_G0(3, 2); break;
    case 27: R3MG_G0(3, 3); break;
    case 28: R3MG_G0(3, 4); break;
    default: throw std::runtime_error("Galerkin product: unsupported dimension or degree");
  }
#undef R3MG_G0
  check_launch("k_galerkin0");
}

// Galerkin product between agglomerated levels: A_{l+1}[G,G'] = sum_{C in G, C' in G'} P~_C^T A_l[C,C'] P~_C'.
// One workgroup per output block; A_l blocks and P~ blocks are staged in LDS (dynamic, 4 B^2 doubles).
template <int D, int KB>
__global__ __launch_bounds__(256) void k_galerkin_c(int shift, int nbox_in, const int* __restrict__ brow,
                                                    const int* __restrict__ bptr_out, const int* __restrict__ bcol_out,
                                                    const int* __restrict__ bptr_in, const int* __restrict__ bcol_in,
                                                    const double* __restrict__ val_in, const double* __restrict__ pt,
                                                    double* out) {
  extern __shared__ unsigned char smem_raw[];
  // dimension and degree are compile-time: the B-long loops and the index divisions below unroll or fold, with the
  // same operations in the same order
  constexpr int d = D, k = KB;
  constexpr int B = D == 3 ? KB * KB * KB : KB * KB;
  constexpr int bb = B * B;
  constexpr int EMAX = (bb + 255) / 256;
  double* sA = reinterpret_cast<double*>(smem_raw);
  double* sPc = sA + bb;
  double* sPp = sPc + bb;
  double* sT = sPp + bb;
  const int64_t blkid = blockIdx.x;
  const int G = brow[blkid];
  const int slot = (int)(blkid - bptr_out[G]);
  const int nbG = bptr_out[G + 1] - bptr_out[G];
  const int Gp = bcol_out[blkid];
  double acc[EMAX];
#pragma unroll
  for (int m = 0; m < EMAX; ++m) acc[m] = 0;
  const int c0 = G << shift, c1 = min(nbox_in, (G + 1) << shift);
  const int tlo = Gp << shift, thi = (Gp + 1) << shift;
  for (int C = c0; C < c1; ++C) {
    for (int e = threadIdx.x; e < bb; e += blockDim.x) sPc[e] = pt_entry(pt, C, d, k, e / B, e % B);
    const int j0 = bptr_in[C], nbC = bptr_in[C + 1] - j0;
    int lo = j0, hi = j0 + nbC;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (bcol_in[mid] < tlo) lo = mid + 1; else hi = mid;
    }
    for (int jb = lo; jb < j0 + nbC && bcol_in[jb] < thi; ++jb) {
      const int Cp = bcol_in[jb];
      const int64_t vb = (int64_t)bb * j0 + (int64_t)(jb - j0) * B;
      __syncthreads();
      for (int e = threadIdx.x; e < bb; e += blockDim.x) {
        const int r = e / B, c = e % B;
        sA[e] = val_in[vb + (int64_t)r * nbC * B + c];
        sPp[e] = pt_entry(pt, Cp, d, k, r, c);
      }
      __syncthreads();
      for (int e = threadIdx.x; e < bb; e += blockDim.x) {  // T = A P~_C'
        const int r = e / B, c = e % B;
        double s = 0;
        for (int m = 0; m < B; ++m) s += sA[r * B + m] * sPp[m * B + c];
        sT[e] = s;
      }
      __syncthreads();
#pragma unroll
      for (int m = 0; m < EMAX; ++m) {  // acc += P~_C^T T
        const int e = threadIdx.x + m * blockDim.x;
        if (e < bb) {
          const int q = e / B, qq = e % B;
          double s = 0;
          for (int r = 0; r < B; ++r) s += sPc[r * B + q] * sT[r * B + qq];
          acc[m] += s;
        }
      }
    }
    __syncthreads();
  }
  const int64_t base = (int64_t)bb * bptr_out[G];
#pragma unroll
  for (int m = 0; m < EMAX; ++m) {
    const int e = threadIdx.x + m * blockDim.x;
    if (e < bb) out[base + (int64_t)(e / B) * nbG * B + (int64_t)slot * B + (e % B)] = acc[m];
  }
}

void launch_galerkin_c(int64_t nblocks, int d, int pc, int shift, int nbox_in, const int* brow, const int* bptr_out,
                       const int* bcol_out, const int* bptr_in, const int* bcol_in, const double* val_in,
                       const double* pt, double* out, hipStream_t s) {
  const int k = pc + 1;
  const int B = (d == 3) ? k * k * k : k * k;
  const int bb = B * B;
  const size_t shm = sizeof(double) * 4 * bb;
  if (nblocks == 0) return;
  if (shm > 65536) {  // only B = 64 (3D, degree 3)
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_galerkin_c<3, 4>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) throw std::runtime_error("coarse Galerkin: LDS request too large for this device");
  }
  const int threads = bb <= 256 ? ((bb + 63) / 64) * 64 : 256;
#define R3MG_GC(DD, KK)                                                                                             \
  hipLaunchKernelGGL((k_galerkin_c<DD, KK>), dim3((unsigned)nblocks), dim3(threads), shm, s, shift, nbox_in, brow,  \
                     bptr_out, bcol_out, bptr_in, bcol_in, val_in, pt, out)
  switch (d * 8 + pc + 1) {
    case 17: R3MG_GC(2, 1); break;
    case 18: R3MG_GC(2, 2); break;
    case 19: R3MG_GC(2, 3); break;
    case 20: R3MG_GC(2, 4); break;
    case 25: R3MG_GC(3, 1); break;
    case 26: R3MG_GC(3, 2); break;
    case 27: R3MG_GC(3, 3); break;
    case 28: R3MG_GC(3, 4); break;
    default: throw std::runtime_error("coarse Galerkin product: unsupported dimension or degree");
  }
#undef R3MG_GC
  check_launch("k_galerkin_c");
}

// scatter the block rows of the coarsest level into a dense row-major matrix
__global__ void k_to_dense(int nbox, int B, const int* __restrict__ bptr, const int* __restrict__ bcol,
                           const double* __restrict__ val, double* dense) {
  const int row = blockIdx.x;  // one block per row
  const int K = row / B, q = row - K * B;
  const int j0 = bptr[K], nb = bptr[K + 1] - j0;
  const int nc = nbox * B;
  const int64_t vb = (int64_t)B * B * j0 + (int64_t)q * nb * B;
  for (int p = threadIdx.x; p < nb * B; p += blockDim.x) {
    const int j = p / B, c = p % B;
    dense[(int64_t)row * nc + (int64_t)bcol[j0 + j] * B + c] = val[vb + p];
  }
}
void launch_to_dense(int nbox, int B, const int* bptr, const int* bcol, const double* val, double* dense,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_to_dense, dim3(nbox * B), dim3(256), 0, s, nbox, B, bptr, bcol, val, dense);
  check_launch("k_to_dense");
}

// Lanczos start vector v_i = ((u_i * 2654435761) mod 2^32) / 2^32 - 1/2, u_i = perm[i] (or i)
__global__ void k_lanczos_start(int n, const int* __restrict__ perm, double* v) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint64_t u = perm ? (uint64_t)perm[i] : (uint64_t)i;
  const uint64_t h = (u * 2654435761ull) & 0xffffffffull;
  v[i] = (double)h / 4294967296.0 - 0.5;
}
void launch_lanczos_start(int n, const int* perm, double* v, hipStream_t s) {
  hipLaunchKernelGGL(k_lanczos_start, dim3((n + 255) / 256), dim3(256), 0, s, n, perm, v);
  check_launch("k_lanczos_start");
}

// per-block partial sums of w_i x_i y_i (fixed grid of at most 1024 blocks, grid-stride)
__global__ __launch_bounds__(256) void k_dot(int64_t n, const double* __restrict__ w, const double* __restrict__ x,
                                             const double* __restrict__ y, double* partials) {
  __shared__ double sh[4];
  double acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    acc += (w ? w[i] : 1.0) * x[i] * y[i];
  double t = block_sum256(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}
int launch_dot(int64_t n, const double* w, const double* x, const double* y, double* partials, hipStream_t s) {
  int64_t g = (n + 255) / 256;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_dot, dim3((unsigned)g), dim3(256), 0, s, n, w, x, y, partials);
  check_launch("k_dot");
  return (int)g;
}
__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, double* y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}
void launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, a, x, b, y);
  check_launch("k_axpby");
}
__global__ void k_lanczos_u(int64_t n, const double* __restrict__ dinv, const double* __restrict__ Av, double bp,
                            const double* __restrict__ vp, double* u) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) u[i] = dinv[i] * Av[i] - bp * vp[i];
}
void launch_lanczos_u(int64_t n, const double* dinv, const double* Av, double beta_prev, const double* vprev,
                      double* u, hipStream_t s) {
  hipLaunchKernelGGL(k_lanczos_u, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, dinv, Av, beta_prev, vprev, u);
  check_launch("k_lanczos_u");
}

// =============================================================================================
// Dense Cholesky factorisation and explicit inverse of the coarsest operator (float64, row-major, n x n).
// Blocked in 64 x 64 tiles; every tile product runs on the FP64 matrix cores (v_mfma_f64_16x16x4f64):
//   1. A = L L^T, right-looking by block columns k: the diagonal tile is factored in LDS and inverted
//      (D_k = L_kk^{-1}); the panel below becomes A[i,k] D_k^T; the trailing lower tiles lose A[i,k] A[j,k]^T.
//   2. Y = L^{-1}, forward by block rows k: Y[k, 0..k] <- D_k Y[k, 0..k] (Y starts at zero; Y[k,k] = D_k),
//      then Y[r, 0..k] -= L[r,k] Y[k, 0..k] for r > k.
//   3. A^{-1} = Y^T Y: upper tile (I, J), I <= J, sums Y[M,I]^T Y[M,J] over M >= J and is stored with its
//      mirror (L^{-T} L^{-1} = (L L^T)^{-1}).
// About n^3 / 3 flops in each step (the triangular structure is skipped), against n^3 / 3 + 2 n^3 for two full
// triangular solves on the identity.  Tiles reaching past n are padded with the identity on a diagonal tile
// and zeros elsewhere.  A non-positive pivot sets *bad (the factorisation then continues with pivot 1).
// =============================================================================================
constexpr int DT = 64;
typedef double v4d __attribute__((ext_vector_type(4)));

// X[i][j] = M[(R + i) n + C + j] inside the matrix, outside it 1 on the diagonal of a diagonal tile (diag_pad)
// and 0 elsewhere; stored s[i][j], or s[j][i] with trans.  The tile product reads its operands as s[k][index]
// with the index running across the lanes, so an operand whose index is its row is loaded transposed.
// element (i, j) = (threadIdx.x / 64 + 4 q, threadIdx.x % 64) of tile (R, C), q < 16, from clamped addresses (all
// 16 loads issued before the first is used; entries outside the matrix are masked by dt_put)
constexpr int kDtK = DT * DT / 256;
__device__ inline void dt_fetch(double (&v)[kDtK], const double* __restrict__ M, int n, int R, int C) {
  const int j = threadIdx.x & 63, i0 = threadIdx.x >> 6;
  const int64_t cj = min(C + j, n - 1);
#pragma unroll
  for (int q = 0; q < kDtK; ++q) v[q] = M[(int64_t)min(R + i0 + 4 * q, n - 1) * n + cj];
}
// the fetched elements into LDS (transposed if trans); entries outside the matrix read as 0, or 1 on the diagonal
// (diag_pad)
__device__ inline void dt_put(double (*s)[DT + 1], const double (&v)[kDtK], int n, int R, int C, bool trans,
                              bool diag_pad) {
  const int j = threadIdx.x & 63, i0 = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kDtK; ++q) {
    const int i = i0 + 4 * q;
    const double x = (R + i < n && C + j < n) ? v[q] : (diag_pad && i == j) ? 1.0 : 0.0;
    if (trans)
      s[j][i] = x;
    else
      s[i][j] = x;
  }
}
// tile (R, C) into LDS: the loads come from clamped addresses and are all issued before the first is used, and
// entries outside the matrix are masked afterwards (a load under a lane-dependent condition would be waited for
// on its own)
__device__ inline void dt_load(double (*s)[DT + 1], const double* __restrict__ M, int n, int R, int C, bool trans,
                               bool diag_pad) {
  double v[kDtK];
  dt_fetch(v, M, n, R, C);
  dt_put(s, v, n, R, C, trans, diag_pad);
}

// a 64 x 64 tile of 64 x 64 values stored contiguously (row-major) into LDS, transposed: s[e % 64][e / 64] = T[e]
// (all loads issued before the first store)
__device__ inline void dt_load_packed_t(double (*s)[DT + 1], const double* __restrict__ T) {
  constexpr int K = DT * DT / 256;
  double v[K];
#pragma unroll
  for (int q = 0; q < K; ++q) v[q] = T[threadIdx.x + 256 * q];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const int e = threadIdx.x + 256 * q;
    s[e & 63][e >> 6] = v[q];
  }
}

// acc += sum over k < 64 of Aop(i, k) Bop(k, j), Aop(i, k) = sa[k][i], Bop(k, j) = sb[k][j].  Wave w owns the
// output rows 32 (w / 2) .. + 31 and columns 32 (w % 2) .. + 31 as 2 x 2 subtiles of 16 x 16.  Lane l supplies
// A[l % 16][l / 16] of each 16 x 4 left operand and B[l / 16][l % 16] of each 4 x 16 right operand, and element r
// of its result is C[4 r + l / 16][l % 16] (the instruction's layout, checked on gfx950).
__device__ inline void dt_mfma(const double (*sa)[DT + 1], const double (*sb)[DT + 1], v4d acc[2][2]) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
  const int li = l & 15, lk = l >> 4;
#pragma unroll 4
  for (int k = 0; k < DT; k += 4) {
    const double a0 = sa[k + lk][r0 + li], a1 = sa[k + lk][r0 + 16 + li];
    const double b0 = sb[k + lk][c0 + li], b1 = sb[k + lk][c0 + 16 + li];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
}

__device__ inline void dt_zero(v4d acc[2][2]) {
  for (int s = 0; s < 2; ++s)
    for (int t = 0; t < 2; ++t) acc[s][t] = v4d{0.0, 0.0, 0.0, 0.0};
}

// f(row, col, value) for every element of the wave's part of the tile
template <typename F>
__device__ inline void dt_each(const v4d acc[2][2], F f) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
  for (int s = 0; s < 2; ++s)
    for (int t = 0; t < 2; ++t)
      for (int r = 0; r < 4; ++r) f(r0 + 16 * s + 4 * r + (l >> 4), c0 + 16 * t + (l & 15), acc[s][t][r]);
}

// the elements of tile (R, C) of M in the accumulator's layout (as dt_each visits them), from clamped addresses,
// all loads issued before the first is used
__device__ inline void dt_fetch_acc(double (&old)[2][2][4], const double* M, int n, int R, int C) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = r0 + 16 * s + 4 * r + (l >> 4), j = c0 + 16 * t + (l & 15);
        old[s][t][r] = M[(int64_t)min(R + i, n - 1) * n + min(C + j, n - 1)];
      }
}

// M tile (R, C) = old - acc (sub) or = acc, inside the matrix
__device__ inline void dt_put_acc(const v4d acc[2][2], const double (&old)[2][2][4], double* M, int n, int R, int C,
                                  bool sub) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = r0 + 16 * s + 4 * r + (l >> 4), j = c0 + 16 * t + (l & 15);
        if (R + i < n && C + j < n) M[(int64_t)(R + i) * n + C + j] = sub ? old[s][t][r] - acc[s][t][r] : acc[s][t][r];
      }
}

// M tile (R, C) = acc, inside the matrix
__device__ inline void dt_store(const v4d acc[2][2], double* M, int n, int R, int C) {
  const double none[2][2][4] = {};
  dt_put_acc(acc, none, M, n, R, C, false);
}

// keeps fetched values ahead of a barrier (the compiler would otherwise sink their loads past it)
__device__ inline void dt_pin(const double (&old)[2][2][4]) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) asm volatile("" ::"v"(old[s][t][r]));
}

// sum over m in [m0, m1) of x[m sx] y[m sy] from LDS, in eight interleaved partial sums combined in a fixed
// order, so that the loads of eight terms are in flight together
__device__ inline double dt_dot8(const double* x, int sx, const double* y, int sy, int m0, int m1) {
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int m = m0;
  for (; m + 8 <= m1; m += 8)
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += x[(m + u) * sx] * y[(m + u) * sy];
  for (int u = 0; m < m1; ++m, ++u) a[u] += x[m * sx] * y[m * sy];
  return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// 1. Diagonal tile k0, by two waves.  Wave 0: Cholesky by columns (left-looking): lane l keeps row l of the tile
// in registers, and the rows of L go to LDS as they become final (zero elsewhere), so that step j reads row j of L
// as 16-byte broadcasts and each lane forms its dot product with its own registers; segments of eight entries that
// are still zero are not read.  Wave 1: the inverse D = L^{-1} by rows of D: lane l keeps column l of D in
// registers (zero above the diagonal), so that row i of D needs row i of L only, which is final once column i is;
// so wave 1 forms row j - 1 of D while wave 0 forms column j of L.  L goes back to A (zero above the diagonal), D
// to Dk (64 x 64, zero above the diagonal).  The steps are generated by template recursion, so every register
// index is a constant; the pivots' square roots are broadcast with a lane shuffle, and one barrier per step orders
// the LDS rows.  (Forming row J of D in the same step as column J of L in one wave needed 387 registers and ran
// slower.)
constexpr int kDiagLD = DT + 2;  // LDS row stride: 16-byte aligned rows, 4-way conflicts at most for row-per-lane reads

// sum over m < 8 ceil(J / 8) of x[m] w[m] (w: an LDS row whose entries from J on are zero), in two interleaved
// partial sums (four ran slower)
template <int J, bool XW>
__device__ __forceinline__ double diag_dot(const double (&x)[DT], const double* w) {
  double a0 = 0.0, a1 = 0.0;
#pragma unroll
  for (int c = 0; c < (J + 7) / 8; ++c)
#pragma unroll
    for (int t = 0; t < 8; t += 2) {
      const double2 v = *reinterpret_cast<const double2*>(w + 8 * c + t);
      if (XW) {
        a0 += x[8 * c + t] * v.x;
        a1 += x[8 * c + t + 1] * v.y;
      } else {
        a0 += v.x * x[8 * c + t];
        a1 += v.y * x[8 * c + t + 1];
      }
    }
  return a0 + a1;
}

// column J of L (left-looking): lane l >= J finishes L[l][J] and puts it in LDS
template <int J>
__device__ __forceinline__ void diag_chol_col(double (&r)[DT], double* s, int l, int* bad) {
  const double acc = diag_dot<J, true>(r, s + J * kDiagLD);  // sum over m < J of L[l][m] L[J][m]
  double piv = r[J] - acc;  // left-looking: r[J] still holds the tile's entry
  if (l == J && !(piv > 0.0)) {
    *bad = 1;
    piv = 1.0;
  }
  const double ljj = __shfl(sqrt(piv), J, 64);
  if (l >= J) {
    const double v = (l == J) ? ljj : (r[J] - acc) / ljj;
    s[l * kDiagLD + J] = v;
    r[J] = v;
  }
}

// row I of D = L^{-1} (column l of D in lane l): d[I][l] = -(sum over l <= m < I of L[I][m] d[m][l]) / L[I][I]
// (I > l), 1 / L[I][I] (I = l), 0 (I < l); d[m][l] = 0 for m < l, so the sum may run over m < I.  It needs row I
// of L only.
template <int I>
__device__ __forceinline__ void diag_inv_row(double (&d)[DT], const double* s, int l) {
  const double* ri = s + I * kDiagLD;
  const double acc = diag_dot<I, false>(d, ri);
  const double lii = ri[I];
  d[I] = (I < l) ? 0.0 : (I == l) ? 1.0 / lii : -acc / lii;
}

// Step J of the two waves: wave 0 forms column J of L, wave 1 row J - 1 of D (row J - 1 of L is final after
// column J - 1); one barrier per step orders the LDS rows.
template <int J>
struct DiagSteps {
  static __device__ __forceinline__ void run(double (&r)[DT], double (&d)[DT], double* s, int l, bool w0, int* bad) {
    if constexpr (J <= DT) {
      if (w0) {
        if constexpr (J < DT) diag_chol_col<J>(r, s, l, bad);
      } else {
        if constexpr (J > 0) diag_inv_row<J - 1>(d, s, l);
      }
      if constexpr (J < DT) __syncthreads();
      DiagSteps<J + 1>::run(r, d, s, l, w0, bad);
    }
  }
};

__global__ __launch_bounds__(128) void k_dchol_diag(int n, int k0, double* A, double* Dk, int* bad) {
  __shared__ __align__(16) double s[DT * kDiagLD];
  const int l = threadIdx.x & 63;
  const bool w0 = threadIdx.x < 64;
  {
    // rows 2 q + w, column l of the tile: all 32 loads of a lane from clamped addresses first, entries outside
    // the matrix masked afterwards (identity there)
    const int w = threadIdx.x >> 6;
    double v[DT / 2];
    const int64_t cl = min(k0 + l, n - 1);
#pragma unroll
    for (int q = 0; q < DT / 2; ++q) v[q] = A[(int64_t)min(k0 + 2 * q + w, n - 1) * n + cl];
#pragma unroll
    for (int q = 0; q < DT / 2; ++q) {
      const int i = 2 * q + w;
      s[i * kDiagLD + l] = (k0 + i < n && k0 + l < n) ? v[q] : (i == l) ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  double r[DT];
#pragma unroll
  for (int m = 0; m < DT; ++m) r[m] = s[l * kDiagLD + m];
  __syncthreads();
  for (int e = threadIdx.x; e < DT * kDiagLD; e += 128) s[e] = 0.0;
  __syncthreads();
  double d[DT];
#pragma unroll
  for (int m = 0; m < DT; ++m) d[m] = 0.0;
  DiagSteps<0>::run(r, d, s, l, w0, bad);
  if (!w0) {
#pragma unroll
    for (int i = 0; i < DT; ++i) Dk[i * DT + l] = d[i];
  }
  for (int e = threadIdx.x; e < DT * DT; e += 128) {
    const int i = e >> 6, j = e & 63;
    if (k0 + i < n && k0 + j < n) A[(int64_t)(k0 + i) * n + k0 + j] = s[i * kDiagLD + j];
  }
}

// 1. Panel: tile (k0 + 64 (1 + blockIdx.x), k0) of A becomes A_ik D_k^T (each workgroup owns its tile's rows).
__global__ __launch_bounds__(256) void k_dchol_panel(int n, int k0, double* A, const double* __restrict__ Dk) {
  __shared__ double sa[DT][DT + 1];
  __shared__ double sb[DT][DT + 1];
  const int R = k0 + DT * (1 + blockIdx.x);
  dt_load(sa, A, n, R, k0, true, false);   // Aop(i, k) = A_ik[i][k]
  // Bop(k, j) = D_k[j][k]
  dt_load_packed_t(sb, Dk);
  __syncthreads();
  v4d acc[2][2];
  dt_zero(acc);
  dt_mfma(sa, sb, acc);
  dt_store(acc, A, n, R, k0);
}

// 1. Trailing update of the lower tiles (I, J), k0 < J <= I: A_IJ -= A_Ik A_Jk^T, with I = k0/64 + 1 + a and
// J = k0/64 + 1 + b.  part 0: every pair (b <= a), enumerated row by row; part 1: the next column only (b = 0,
// a = blockIdx.x); part 2: the other columns (1 <= b <= a), enumerated row by row.
__global__ __launch_bounds__(256) void k_dchol_update(int n, int k0, double* A, int part) {
  __shared__ double sa[DT][DT + 1];
  __shared__ double sb[DT][DT + 1];
  int a, b;
  if (part == 1) {
    a = (int)blockIdx.x;
    b = 0;
  } else {
    a = (int)((sqrt(8.0 * blockIdx.x + 1.0) - 1.0) * 0.5);
    while ((a + 1) * (a + 2) / 2 <= (int)blockIdx.x) ++a;
    while (a * (a + 1) / 2 > (int)blockIdx.x) --a;
    b = (int)blockIdx.x - a * (a + 1) / 2;
    if (part == 2) {  // pairs of the triangle without column 0
      ++a;
      ++b;
    }
  }
  const int RI = k0 + DT * (1 + a), RJ = k0 + DT * (1 + b);
  double old[2][2][4];
  dt_fetch_acc(old, A, n, RI, RJ);           // the tile updated, in flight with the operands
  dt_load(sa, A, n, RI, k0, true, false);    // Aop(i, k) = A_Ik[i][k]
  dt_load(sb, A, n, RJ, k0, true, false);    // Bop(k, j) = A_Jk[j][k]
  dt_pin(old);
  __syncthreads();
  v4d acc[2][2];
  dt_zero(acc);
  dt_mfma(sa, sb, acc);
  dt_put_acc(acc, old, A, n, RI, RJ, true);
}

// 2. Block row k of Y: tile (k, j) for j = blockIdx.x <= k: Y_kj <- D_k Y_kj, except Y_kk = D_k.
__global__ __launch_bounds__(256) void k_dinv_row(int n, int kb, const double* __restrict__ Dk, double* Y) {
  __shared__ double sa[DT][DT + 1];
  __shared__ double sb[DT][DT + 1];
  const int j = blockIdx.x, R = DT * kb, C = DT * j;
  if (j == kb) {
    constexpr int K = DT * DT / 256;
    double v[K];
#pragma unroll
    for (int q = 0; q < K; ++q) v[q] = Dk[threadIdx.x + 256 * q];
#pragma unroll
    for (int q = 0; q < K; ++q) {
      const int e = threadIdx.x + 256 * q, r = e >> 6, c = e & 63;
      if (R + r < n && C + c < n) Y[(int64_t)(R + r) * n + C + c] = v[q];
    }
    return;
  }
  dt_load_packed_t(sa, Dk);   // Aop(i, k) = D_k[i][k]
  dt_load(sb, Y, n, R, C, false, false);                                         // Bop(k, j) = Y_kj[k][j]
  __syncthreads();
  v4d acc[2][2];
  dt_zero(acc);
  dt_mfma(sa, sb, acc);
  __syncthreads();
  dt_store(acc, Y, n, R, C);
}

// 2. Rows below block row k: tile (r, j), r = kb + 1 + blockIdx.x / (kb + 1), j = blockIdx.x % (kb + 1):
// Y_rj -= L_rk Y_kj.
__global__ __launch_bounds__(256) void k_dinv_update(int n, int kb, const double* __restrict__ L, double* Y) {
  __shared__ double sa[DT][DT + 1];
  __shared__ double sb[DT][DT + 1];
  const int r = kb + 1 + (int)blockIdx.x / (kb + 1), j = (int)blockIdx.x % (kb + 1);
  double old[2][2][4];
  dt_fetch_acc(old, Y, n, DT * r, DT * j);           // the tile updated, in flight with the operands
  dt_load(sa, L, n, DT * r, DT * kb, true, false);   // Aop(i, k) = L_rk[i][k]
  dt_load(sb, Y, n, DT * kb, DT * j, false, false);  // Bop(k, j) = Y_kj[k][j]
  dt_pin(old);
  __syncthreads();
  v4d acc[2][2];
  dt_zero(acc);
  dt_mfma(sa, sb, acc);
  dt_put_acc(acc, old, Y, n, DT * r, DT * j, true);
}

// 3. Upper tile (I, J) of A^{-1} = Y^T Y and its mirror; blockIdx.x enumerates the pairs I <= J row by row.
__global__ __launch_bounds__(256) void k_dinv_gram(int n, int nt, const double* __restrict__ Y, double* Inv) {
  __shared__ double sa[DT][DT + 1];
  __shared__ double sb[DT][DT + 1];
  int rem = (int)blockIdx.x, I = 0;
  while (rem >= nt - I) {
    rem -= nt - I;
    ++I;
  }
  const int J = I + rem;
  v4d acc[2][2];
  dt_zero(acc);
  // the tiles of step M + 1 are fetched into registers while step M's product runs from LDS
  double va[kDtK], vb[kDtK];
  dt_fetch(va, Y, n, DT * J, DT * I);
  dt_fetch(vb, Y, n, DT * J, DT * J);
  for (int M = J; M < nt; ++M) {
    dt_put(sa, va, n, DT * M, DT * I, false, false);   // Aop(i, k) = Y_MI[k][i]
    dt_put(sb, vb, n, DT * M, DT * J, false, false);   // Bop(k, j) = Y_MJ[k][j]
    __syncthreads();
    if (M + 1 < nt) {  // uniform over the workgroup
      dt_fetch(va, Y, n, DT * (M + 1), DT * I);
      dt_fetch(vb, Y, n, DT * (M + 1), DT * J);
    }
    dt_mfma(sa, sb, acc);
    __syncthreads();
  }
  dt_store(acc, Inv, n, DT * I, DT * J);
  if (I != J) {  // the mirror tile, staged in LDS so that its rows are written contiguously
    dt_each(acc, [&](int i, int j, double v) { sa[i][j] = v; });
    __syncthreads();
    for (int e = threadIdx.x; e < DT * DT; e += 256) {
      const int r = e >> 6, c = e & 63;  // mirror row r = tile column r
      if (DT * J + r < n && DT * I + c < n) Inv[(int64_t)(DT * J + r) * n + DT * I + c] = sa[c][r];
    }
  }
}

// ws: nt * 64 * 64 doubles (the inverted diagonal tiles); Y: n * n doubles of scratch
// The factorisation looks one step ahead: step kb's update of the next column (part 1) stays on s, while the
// update of the other columns (part 2) runs on a second stream from the end of panel kb on, so that part 1,
// diagonal tile and panel kb + 1, which touch column kb + 1 only, overlap it.  Part 1 of step kb + 1 writes column
// kb + 2, which part 2 of step kb also writes, so it waits for that; parts 2 follow one another on the second
// stream.
namespace {
struct LookAhead {
  hipStream_t s2 = nullptr;
  std::vector<hipEvent_t> ev;
  size_t next = 0;
  ~LookAhead() {
    for (auto e : ev) (void)hipEventDestroy(e);
    if (s2) (void)hipStreamDestroy(s2);
  }
  // all events are created before the first launch, so that the host enqueues the steps ahead of the device
  void create(size_t count) {
    ev.reserve(count);
    for (size_t i = 0; i < count; ++i) {
      hipEvent_t e;
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
        throw std::runtime_error("dense Cholesky: event creation failed");
      ev.push_back(e);
    }
  }
  hipEvent_t event() {
    if (next == ev.size()) throw std::runtime_error("dense Cholesky: events exhausted");
    return ev[next++];
  }
};
}  // namespace

void dense_cholesky_inverse(int n, double* A, double* Inv, double* ws, double* Y, int* bad, hipStream_t s) {
  const int nt = (n + DT - 1) / DT;
  LookAhead la;
  if (hipStreamCreateWithFlags(&la.s2, hipStreamNonBlocking) != hipSuccess)
    throw std::runtime_error("dense Cholesky: stream creation failed");
  la.create(2 * (size_t)nt);
  hipEvent_t prev2 = nullptr;  // part 2 of the previous step done
  for (int kb = 0; kb < nt; ++kb) {
    const int k0 = kb * DT;
    double* Dk = ws + (size_t)kb * DT * DT;
    hipLaunchKernelGGL(k_dchol_diag, dim3(1), dim3(128), 0, s, n, k0, A, Dk, bad);
    const int below = nt - kb - 1;
    if (below > 0) {
      hipLaunchKernelGGL(k_dchol_panel, dim3(below), dim3(256), 0, s, n, k0, A, Dk);
      hipEvent_t done2 = nullptr;  // part 2 of this step done
      if (below > 1) {
        // part 2 needs this step's panel only (part 1 writes another column), so it is forked right after the
        // panel: no event then sits between part 1 and the next diagonal tile on s
        hipEvent_t main = la.event();
        if (hipEventRecord(main, s) != hipSuccess || hipStreamWaitEvent(la.s2, main, 0) != hipSuccess)
          throw std::runtime_error("dense Cholesky: event record failed");
        hipLaunchKernelGGL(k_dchol_update, dim3((below - 1) * below / 2), dim3(256), 0, la.s2, n, k0, A, 2);
        done2 = la.event();
        if (hipEventRecord(done2, la.s2) != hipSuccess) throw std::runtime_error("dense Cholesky: event record failed");
      }
      // part 1 writes the next column, which part 2 of the previous step also writes
      if (prev2 && hipStreamWaitEvent(s, prev2, 0) != hipSuccess)
        throw std::runtime_error("dense Cholesky: stream wait failed");
      hipLaunchKernelGGL(k_dchol_update, dim3(below), dim3(256), 0, s, n, k0, A, 1);
      if (done2) prev2 = done2;
    }
  }
  if (prev2 && hipStreamWaitEvent(s, prev2, 0) != hipSuccess)
    throw std::runtime_error("dense Cholesky: stream wait failed");
  check_launch("dense Cholesky");
  hipMemsetAsync(Y, 0, (size_t)n * n * sizeof(double), s);
  for (int kb = 0; kb < nt; ++kb) {
    hipLaunchKernelGGL(k_dinv_row, dim3(kb + 1), dim3(256), 0, s, n, kb, ws + (size_t)kb * DT * DT, Y);
    const int below = nt - kb - 1;
    if (below > 0) hipLaunchKernelGGL(k_dinv_update, dim3(below * (kb + 1)), dim3(256), 0, s, n, kb, A, Y);
  }
  hipLaunchKernelGGL(k_dinv_gram, dim3(nt * (nt + 1) / 2), dim3(256), 0, s, n, nt, Y, Inv);
  check_launch("dense inverse");
}

// =============================================================================================
// PCG (float64 outer iteration; scalars live on the device)
// =============================================================================================
// Every reduction is a vector kernel that stores per-block partial sums, followed by a one-block kernel that sums
// them in index order and updates the scalars in PcgState.  Vector kernels are grid-stride with at most
// kPcgBlocks blocks, so the partition of every reduction depends only on n and NR and a reduction's result never
// depends on the kernel that formed its operands.  (Finishing a reduction inside the vector kernel, in the block
// that arrives last, was measured slower: the device-scope release each block must issue before taking its
// ticket writes back its die's L2, and 1024 of them cost 60-80 us per kernel against ~4 us for the extra
// launch.)  Vectors are n x NR interleaved; thread t of a block always handles column t % NR of 256-row chunks
// (256 % NR == 0), so consecutive threads touch consecutive elements.

// Per-column block sums: butterfly over the lanes of one column, then the four waves in order; thread k < NR
// writes out[k].
template <int NR>
__device__ inline void column_partials(double acc, double* sh, double* out) {
#pragma unroll
  for (int off = 32; off >= NR; off >>= 1) acc += __shfl_xor(acc, off, 64);
  const int lane = threadIdx.x & 63;
  if (lane < NR) sh[(threadIdx.x >> 6) * NR + lane] = acc;
  __syncthreads();
  if (threadIdx.x < NR) {
    const int k = threadIdx.x;
    out[k] = (sh[k] + sh[NR + k]) + (sh[2 * NR + k] + sh[3 * NR + k]);
  }
}

// Column totals of part[b * stride + k] (k < NR, b < nb) by one 256-thread block: thread t sums blocks t / NR,
// t / NR + 256 / NR, ... of column t % NR in index order, then column_partials.  tot (shared) is valid in every
// thread on return.
template <int NR>
__device__ inline void column_totals(const double* __restrict__ part, int nb, int stride, double* sh, double* tot) {
  const int k = threadIdx.x % NR;
  constexpr int S = 256 / NR;
  double acc = 0;
  // four of the thread's partials at a time: loads issued together (clamped), added in index order
  for (int b0 = threadIdx.x / NR; b0 < nb; b0 += 4 * S) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = part[(int64_t)min(b0 + u * S, nb - 1) * stride + k];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (b0 + u * S < nb) acc += v[u];
  }
  column_partials<NR>(acc, sh, tot);
  __syncthreads();
}

// Two one-column totals at once, each exactly as column_totals<1> forms it (pa[b * sa] and pb[b * sb], b < nb):
// the loads of both are in flight together.  ta, tb (shared) are valid in every thread on return.
__device__ inline void column_totals2(const double* __restrict__ pa, int sa, const double* __restrict__ pb, int sb,
                                      int nb, double* sh, double* ta, double* tb) {
  double acca = 0, accb = 0;
  for (int b0 = threadIdx.x; b0 < nb; b0 += 4 * 256) {
    double va[4], vb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t b = min(b0 + u * 256, nb - 1);
      va[u] = pa[b * sa];
      vb[u] = pb[b * sb];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (b0 + u * 256 < nb) {
        acca += va[u];
        accb += vb[u];
      }
  }
  column_partials<1>(acca, sh, ta);
  __syncthreads();
  column_partials<1>(accb, sh, tb);
  __syncthreads();
}

// grid-stride steps of the one-column PCG vector kernels whose loads are issued together
constexpr int kPcgU = 4;
inline int pcg_grid(int n) {
  const int g = (n + 255) / 256;
  return std::max(1, std::min(g, kPcgBlocks));
}

#define R3_NR_SWITCH(nr, MACRO)                                   \
  switch (nr) {                                                   \
    case 1: MACRO(1); break;                                      \
    case 2: MACRO(2); break;                                      \
    case 4: MACRO(4); break;                                      \
    case 8: MACRO(8); break;                                      \
    case 16: MACRO(16); break;                                    \
    default: throw std::runtime_error("unsupported nrhs block");  \
  }

__device__ inline void pcg_set_alpha(PcgState* st, int k, double pq) {
  st->alpha[k] = st->done[k] ? 0.0 : st->gamma[k] / pq;
  const int j = st->iters[k];
  if (!st->done[k] && st->hist && j < st->hist_rows) st->hist[(int64_t)2 * j * kMaxNR + k] = st->alpha[k];
}

// <p, q> per column: partials[b * NR + k]
template <int NR>
__global__ __launch_bounds__(256) void k_pcg_dot(int n, const double* __restrict__ p, const double* __restrict__ q,
                                                 double* partials, const PcgState* __restrict__ st) {
  __shared__ double sh[4 * NR];
  if (st->all_done) return;
  double acc = 0;
  const int64_t tn = (int64_t)n * NR;
  // U grid-stride steps at a time: their loads are issued together (clamped addresses), then summed in the
  // element order of one step after another
  constexpr int U = NR >= 4 ? 1 : 4 / NR;
  const int64_t step = (int64_t)gridDim.x * 256 * NR;
  for (int64_t base = (int64_t)blockIdx.x * 256 * NR; base < tn; base += U * step) {
    double pv[U][NR], qv[U][NR];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int m = 0; m < NR; ++m) {
        const int64_t o = min(base + u * step + threadIdx.x + 256 * m, tn - 1);
        pv[u][m] = p[o];
        qv[u][m] = q[o];
      }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int m = 0; m < NR; ++m)
        if (base + u * step + threadIdx.x + 256 * m < tn) acc += pv[u][m] * qv[u][m];
  }
  column_partials<NR>(acc, sh, partials + (int64_t)blockIdx.x * NR);
}
template <int NR>
__global__ __launch_bounds__(256) void k_pcg_alpha_nr(PcgState* st, const double* __restrict__ partials, int nb) {
  __shared__ double sh[4 * NR];
  __shared__ double tot[NR];
  if (st->all_done) return;
  column_totals<NR>(partials, nb, NR, sh, tot);
  if (threadIdx.x < NR) pcg_set_alpha(st, threadIdx.x, tot[threadIdx.x]);
}
void launch_pcg_dot_alpha(int n, int nr, const double* p, const double* q, double* partials, PcgState* st,
                          hipStream_t s) {
  const int g = pcg_grid(n);
#define R3_DA(NRV)                                                                                 \
  hipLaunchKernelGGL((k_pcg_dot<NRV>), dim3(g), dim3(256), 0, s, n, p, q, partials, st);           \
  hipLaunchKernelGGL((k_pcg_alpha_nr<NRV>), dim3(1), dim3(256), 0, s, st, partials, g)
  R3_NR_SWITCH(nr, R3_DA)
#undef R3_DA
  check_launch("k_pcg_dot / k_pcg_alpha");
}

// alpha from partials formed by another kernel (the lanes kernel's fused dot: up to one partial per 32 rows),
// one 1024-thread block summing each column in a fixed order
__global__ __launch_bounds__(1024) void k_pcg_alpha(int nr, PcgState* st, const double* __restrict__ partials, int npart) {
  __shared__ double sh[16];
  if (st->all_done) return;
  for (int k = 0; k < nr; ++k) {
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    int b = threadIdx.x;
    for (; b + 3 * 1024 < npart; b += 4 * 1024) {
      a0 += partials[(int64_t)b * nr + k];
      a1 += partials[(int64_t)(b + 1024) * nr + k];
      a2 += partials[(int64_t)(b + 2048) * nr + k];
      a3 += partials[(int64_t)(b + 3072) * nr + k];
    }
    for (; b < npart; b += 1024) a0 += partials[(int64_t)b * nr + k];
    const double v = wave_sum((a0 + a1) + (a2 + a3), 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double pq = 0;
      for (int i = 0; i < 16; ++i) pq += sh[i];
      pcg_set_alpha(st, k, pq);
    }
    __syncthreads();
  }
}
void launch_pcg_alpha(int nr, PcgState* st, const double* partials, int npart, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_alpha, dim3(1), dim3(1024), 0, s, nr, st, partials, npart);
  check_launch("k_pcg_alpha");
}

// x += alpha p; r -= alpha q; ||r||^2 partials; V-cycle entry b0 = (T) r, d0 = dinv0 b0 / theta0
template <typename T, int NR>
__global__ __launch_bounds__(256) void k_pcg_xr(int n, const PcgState* __restrict__ st, double* x, double* r,
                                                const double* __restrict__ p, const double* __restrict__ q,
                                                double* partials, T* b0, const T* __restrict__ dinv0, T* d0,
                                                T inv_theta0) {
  __shared__ double sh[4 * NR];
  if (st->all_done) return;
  const int k = threadIdx.x % NR;
  const double al = st->alpha[k];
  const int64_t tn = (int64_t)n * NR;
  double acc = 0;
  for (int64_t base = (int64_t)blockIdx.x * 256 * NR; base < tn; base += (int64_t)gridDim.x * 256 * NR)
#pragma unroll
    for (int m = 0; m < NR; ++m) {
      const int64_t o = base + threadIdx.x + 256 * m;
      if (o < tn) {
        x[o] += al * p[o];
        const double rv = r[o] - al * q[o];
        r[o] = rv;
        acc += rv * rv;
        if (b0) {
          const T bv = (T)rv;
          b0[o] = bv;
          if (d0) d0[o] = dinv0[o / NR] * bv * inv_theta0;
        } else if (d0) {
          d0[o] = dinv0[o / NR] * (T)rv * inv_theta0;
        }
      }
    }
  column_partials<NR>(acc, sh, partials + (int64_t)blockIdx.x * NR);
}
// the stop test of every open column (iteration count, squared residual and its history, done flag), all_done
template <int NR>
__global__ __launch_bounds__(256) void k_pcg_check(PcgState* st, const double* __restrict__ partials, int nb) {
  __shared__ double sh[4 * NR];
  __shared__ double tot[NR];
  if (st->all_done) return;
  column_totals<NR>(partials, nb, NR, sh, tot);
  if (threadIdx.x == 0) {
    int all = 1;
    for (int c = 0; c < NR; ++c) {
      if (!st->done[c]) {
        const double rr = tot[c];
        st->rr_prev[c] = st->rr[c];
        st->rr[c] = rr;
        const int j = st->iters[c] + 1;
        st->iters[c] = j;
        if (st->rhist && j <= st->hist_rows) st->rhist[(int64_t)j * kMaxNR + c] = rr;
        if (rr <= st->tau2[c]) st->done[c] = 1;
      }
      all &= st->done[c];
    }
    st->all_done = all;
  }
}
template <typename T>
void launch_pcg_xr(int n, int nr, PcgState* st, double* x, double* r, const double* p, const double* q,
                   double* partials, T* b0, const T* dinv0, T* d0, double inv_theta0, hipStream_t s) {
  const int g = pcg_grid(n);
#define R3_XR(NRV)                                                                                              \
  hipLaunchKernelGGL((k_pcg_xr<T, NRV>), dim3(g), dim3(256), 0, s, n, st, x, r, p, q, partials, b0, dinv0, d0, \
                     (T)inv_theta0);                                                                           \
  hipLaunchKernelGGL((k_pcg_check<NRV>), dim3(1), dim3(256), 0, s, st, partials, g)
  R3_NR_SWITCH(nr, R3_XR)
#undef R3_XR
  check_launch("k_pcg_xr / k_pcg_check");
}
template void launch_pcg_xr<float>(int, int, PcgState*, double*, double*, const double*, const double*, double*,
                                   float*, const float*, float*, double, hipStream_t);
template void launch_pcg_xr<double>(int, int, PcgState*, double*, double*, const double*, const double*, double*,
                                    double*, const double*, double*, double, hipStream_t);

// z = x0 + dpend (in float64); mode 1: p = z; modes 1, 2: partials of <r, z> and (q set) <q, z>
template <typename T, int NR>
__global__ __launch_bounds__(256) void k_pcg_z(int n, const PcgState* __restrict__ st, int mode,
                                               const T* __restrict__ x0, const T* __restrict__ dp, double* z,
                                               const double* __restrict__ r, const double* __restrict__ q,
                                               double* pvec, double* partials) {
  __shared__ double sh[4 * NR];
  if (mode != 0 && st->all_done) return;
  const int64_t tn = (int64_t)n * NR;
  double a1 = 0, a2 = 0;
  for (int64_t base = (int64_t)blockIdx.x * 256 * NR; base < tn; base += (int64_t)gridDim.x * 256 * NR)
#pragma unroll
    for (int m = 0; m < NR; ++m) {
      const int64_t o = base + threadIdx.x + 256 * m;
      if (o < tn) {
        T v = x0[o];
        if (dp) v += dp[o];
        const double zv = (double)v;
        z[o] = zv;
        if (mode == 1) pvec[o] = zv;
        if (mode != 0) {
          a1 += r[o] * zv;
          if (q) a2 += q[o] * zv;
        }
      }
    }
  if (mode == 0) return;
  double* out = partials + (int64_t)blockIdx.x * 2 * NR;
  column_partials<NR>(a1, sh, out);
  __syncthreads();
  column_partials<NR>(a2, sh, out + NR);
}
// mode 1: gamma = <r, z>; mode 2: beta (standard gamma'/gamma, or flexible -alpha <q, z> / gamma) and gamma
template <int NR>
__global__ __launch_bounds__(256) void k_pcg_beta(PcgState* st, int mode, const double* __restrict__ partials,
                                                  int nb) {
  __shared__ double sh[4 * NR];
  __shared__ double rz[NR], qz[NR];
  if (st->all_done) return;
  column_totals<NR>(partials, nb, 2 * NR, sh, rz);
  column_totals<NR>(partials + NR, nb, 2 * NR, sh, qz);
  if (threadIdx.x < NR) {
    const int c = threadIdx.x;
    if (mode == 1) {
      st->gamma[c] = rz[c];
    } else if (!st->done[c]) {
      const double g = st->gamma[c];
      st->beta[c] = st->flexible ? (-st->alpha[c] * qz[c]) / g : rz[c] / g;
      st->gamma[c] = rz[c];
      const int j = st->iters[c] - 1;  // the stop test of iteration j has counted it
      if (st->hist && j >= 0 && j < st->hist_rows) st->hist[(int64_t)(2 * j + 1) * kMaxNR + c] = st->beta[c];
    }
  }
}
template <typename T>
void launch_pcg_z(int n, int nr, PcgState* st, int mode, const T* x0, const T* dpend, double* z, const double* r,
                  const double* q, double* p, double* partials, hipStream_t s) {
  const int g = pcg_grid(n);
#define R3_Z(NRV)                                                                                                  \
  hipLaunchKernelGGL((k_pcg_z<T, NRV>), dim3(g), dim3(256), 0, s, n, st, mode, x0, dpend, z, r, q, p, partials); \
  if (mode != 0) hipLaunchKernelGGL((k_pcg_beta<NRV>), dim3(1), dim3(256), 0, s, st, mode, partials, g)
  R3_NR_SWITCH(nr, R3_Z)
#undef R3_Z
  check_launch("k_pcg_z / k_pcg_beta");
}
template void launch_pcg_z<float>(int, int, PcgState*, int, const float*, const float*, double*, const double*,
                                  const double*, double*, double*, hipStream_t);
template void launch_pcg_z<double>(int, int, PcgState*, int, const double*, const double*, double*, const double*,
                                   const double*, double*, double*, hipStream_t);

__global__ void k_pcg_p(int n, int nr, const PcgState* __restrict__ st, const double* __restrict__ z, double* p) {
  if (st->all_done) return;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)n * nr) return;
  const int k = (int)(t % nr);
  if (st->done[k]) return;
  p[t] = z[t] + st->beta[k] * p[t];
}
void launch_pcg_p(int n, int nr, PcgState* st, const double* z, double* p, hipStream_t s) {
  const int64_t tot = (int64_t)n * nr;
  hipLaunchKernelGGL(k_pcg_p, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, nr, st, z, p);
  check_launch("k_pcg_p");
}

// One right-hand side: the scalar steps folded into the vector kernels that follow their reductions.  Every block of
// the next kernel forms the reduction's total itself from the per-block partials (column_totals<1>: the same sums in
// the same order as the one-block kernels above, so the same bits in every block) and block 0 records it in the
// state; each reduction has its own partials area, so that no block overwrites partials another block still reads:
// area 0 (g entries) <p, q>, area 1 (g) ||r||^2, area 2 (2 g) <r, z> and <q, z>, g = pcg_grid(n).  gamma is formed
// from area 2 by the kernel that needs it, so no kernel writes a state scalar that another block of it reads.
int pcg_blocks(int n) { return pcg_grid(n); }

void launch_pcg_dot(int n, const double* p, const double* q, double* partials, PcgState* st, hipStream_t s) {
  hipLaunchKernelGGL((k_pcg_dot<1>), dim3(pcg_grid(n)), dim3(256), 0, s, n, p, q, partials, st);
  check_launch("k_pcg_dot");
}

// alpha = gamma / <p, q> (gamma = <r, z> from area 2); x += alpha p; r -= alpha q; ||r||^2 partials to area 1;
// V-cycle entry b0 = (T) r, d0 = dinv0 b0 / theta0
template <typename T>
__global__ __launch_bounds__(256) void k_pcg_xr1(int n, PcgState* st, double* x, double* r,
                                                 const double* __restrict__ p, const double* __restrict__ q,
                                                 double* partials, int g, T* b0, const T* __restrict__ dinv0, T* d0,
                                                 T inv_theta0) {
  __shared__ double sh[4];
  __shared__ double gam[1], pq[1];
  if (st->all_done) return;
  column_totals2(partials + 2 * g, 2, partials, 1, g, sh, gam, pq);
  const double al = st->done[0] ? 0.0 : gam[0] / pq[0];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->gamma[0] = gam[0];
    pcg_set_alpha(st, 0, pq[0]);
  }
  double acc = 0;
  // kPcgU grid-stride steps at a time, loads issued together (clamped addresses), in the element order of the
  // steps one after another
  const int64_t step = (int64_t)gridDim.x * 256;
  for (int64_t o0 = (int64_t)blockIdx.x * 256 + threadIdx.x; o0 < n; o0 += kPcgU * step) {
    double xv[kPcgU], pv[kPcgU], rv[kPcgU], qv[kPcgU];
    T dv[kPcgU];
#pragma unroll
    for (int u = 0; u < kPcgU; ++u) {
      const int64_t o = min(o0 + u * step, (int64_t)n - 1);
      xv[u] = x[o];
      pv[u] = p[o];
      rv[u] = r[o];
      qv[u] = q[o];
      dv[u] = d0 ? dinv0[o] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < kPcgU; ++u) {
      const int64_t o = o0 + u * step;
      if (o < n) {
        x[o] = xv[u] + al * pv[u];
        const double r1 = rv[u] - al * qv[u];
        r[o] = r1;
        acc += r1 * r1;
        if (b0) {
          const T bv = (T)r1;
          b0[o] = bv;
          if (d0) d0[o] = dv[u] * bv * inv_theta0;
        } else if (d0) {
          d0[o] = dv[u] * (T)r1 * inv_theta0;
        }
      }
    }
  }
  column_partials<1>(acc, sh, partials + g + blockIdx.x);
}
template <typename T>
void launch_pcg_xr1(int n, PcgState* st, double* x, double* r, const double* p, const double* q, double* partials,
                    T* b0, const T* dinv0, T* d0, double inv_theta0, hipStream_t s) {
  const int g = pcg_grid(n);
  hipLaunchKernelGGL((k_pcg_xr1<T>), dim3(g), dim3(256), 0, s, n, st, x, r, p, q, partials, g, b0, dinv0, d0,
                     (T)inv_theta0);
  check_launch("k_pcg_xr1");
}
template void launch_pcg_xr1<float>(int, PcgState*, double*, double*, const double*, const double*, double*, float*,
                                    const float*, float*, double, hipStream_t);
template void launch_pcg_xr1<double>(int, PcgState*, double*, double*, const double*, const double*, double*,
                                     double*, const double*, double*, double, hipStream_t);

// check set: the stop test of the column (from the ||r||^2 partials of area 1, block 0 records it); z = x0 + dpend;
// <r, z> and (q set) <q, z> partials to area 2
template <typename T>
__global__ __launch_bounds__(256) void k_pcg_z1(int n, PcgState* st, int check, const T* __restrict__ x0,
                                                const T* __restrict__ dp, double* z, const double* __restrict__ r,
                                                const double* __restrict__ q, double* partials, int g) {
  __shared__ double sh[4];
  __shared__ double rr[1];
  if (st->all_done) return;
  // only block 0 records the stop test; the vector work below does not depend on it
  if (check && blockIdx.x == 0) column_totals<1>(partials + g, g, 1, sh, rr);
  if (check && blockIdx.x == 0 && threadIdx.x == 0 && !st->done[0]) {
    st->rr_prev[0] = st->rr[0];
    st->rr[0] = rr[0];
    const int j = st->iters[0] + 1;
    st->iters[0] = j;
    if (st->rhist && j <= st->hist_rows) st->rhist[(int64_t)j * kMaxNR] = rr[0];
    if (rr[0] <= st->tau2[0]) st->done[0] = 1;
    st->all_done = st->done[0];
  }
  double a1 = 0, a2 = 0;
  const int64_t step = (int64_t)gridDim.x * 256;
  for (int64_t o0 = (int64_t)blockIdx.x * 256 + threadIdx.x; o0 < n; o0 += kPcgU * step) {
    T xv[kPcgU], dv[kPcgU];
    double rv[kPcgU], qv[kPcgU];
#pragma unroll
    for (int u = 0; u < kPcgU; ++u) {
      const int64_t o = min(o0 + u * step, (int64_t)n - 1);
      xv[u] = x0[o];
      dv[u] = dp ? dp[o] : (T)0;
      rv[u] = r[o];
      qv[u] = q ? q[o] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kPcgU; ++u) {
      const int64_t o = o0 + u * step;
      if (o < n) {
        T v = xv[u];
        if (dp) v += dv[u];
        const double zv = (double)v;
        z[o] = zv;
        a1 += rv[u] * zv;
        if (q) a2 += qv[u] * zv;
      }
    }
  }
  double* out = partials + 2 * g + (int64_t)blockIdx.x * 2;
  column_partials<1>(a1, sh, out);
  __syncthreads();
  column_partials<1>(a2, sh, out + 1);
}
template <typename T>
void launch_pcg_z1(int n, PcgState* st, bool check, const T* x0, const T* dpend, double* z, const double* r,
                   const double* q, double* partials, hipStream_t s) {
  const int g = pcg_grid(n);
  hipLaunchKernelGGL((k_pcg_z1<T>), dim3(g), dim3(256), 0, s, n, st, check ? 1 : 0, x0, dpend, z, r, q, partials,
                     g);
  check_launch("k_pcg_z1");
}
template void launch_pcg_z1<float>(int, PcgState*, bool, const float*, const float*, double*, const double*,
                                   const double*, double*, hipStream_t);
template void launch_pcg_z1<double>(int, PcgState*, bool, const double*, const double*, double*, const double*,
                                    const double*, double*, hipStream_t);

// the stop test alone (from area 1), for an iteration enqueued as two halves
void launch_pcg_check1(int n, PcgState* st, const double* partials, hipStream_t s) {
  const int g = pcg_grid(n);
  hipLaunchKernelGGL((k_pcg_check<1>), dim3(1), dim3(256), 0, s, st, partials + g, g);
  check_launch("k_pcg_check");
}

// beta (standard <r, z> / gamma or flexible -alpha <q, z> / gamma, from area 2; block 0 records it); p = z + beta p
__global__ __launch_bounds__(256) void k_pcg_p1(int n, PcgState* st, const double* __restrict__ z, double* p,
                                                const double* __restrict__ partials, int g) {
  __shared__ double sh[4];
  __shared__ double rz[1], qz[1];
  if (st->all_done || st->done[0]) return;
  column_totals2(partials + 2 * g, 2, partials + 2 * g + 1, 2, g, sh, rz, qz);
  const double gold = st->gamma[0];
  const double be = st->flexible ? (-st->alpha[0] * qz[0]) / gold : rz[0] / gold;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->beta[0] = be;
    const int j = st->iters[0] - 1;  // the stop test of iteration j has counted it
    if (st->hist && j >= 0 && j < st->hist_rows) st->hist[(int64_t)(2 * j + 1) * kMaxNR] = be;
  }
  const int64_t step = (int64_t)gridDim.x * 256;
  for (int64_t o0 = (int64_t)blockIdx.x * 256 + threadIdx.x; o0 < n; o0 += kPcgU * step) {
    double zv[kPcgU], pv[kPcgU];
#pragma unroll
    for (int u = 0; u < kPcgU; ++u) {
      const int64_t o = min(o0 + u * step, (int64_t)n - 1);
      zv[u] = z[o];
      pv[u] = p[o];
    }
#pragma unroll
    for (int u = 0; u < kPcgU; ++u) {
      const int64_t o = o0 + u * step;
      if (o < n) p[o] = zv[u] + be * pv[u];
    }
  }
}
void launch_pcg_p1(int n, PcgState* st, const double* z, double* p, const double* partials, hipStream_t s) {
  const int g = pcg_grid(n);
  hipLaunchKernelGGL(k_pcg_p1, dim3(g), dim3(256), 0, s, n, st, z, p, partials, g);
  check_launch("k_pcg_p1");
}

// ||b - q||^2 partials per column; with r set, r = b - q as well
template <int NR>
__global__ __launch_bounds__(256) void k_pcg_residual(int n, const double* __restrict__ b, const double* __restrict__ q,
                                                      double* r, double* partials) {
  __shared__ double sh[4 * NR];
  const int64_t tn = (int64_t)n * NR;
  double acc = 0;
  for (int64_t base = (int64_t)blockIdx.x * 256 * NR; base < tn; base += (int64_t)gridDim.x * 256 * NR)
#pragma unroll
    for (int m = 0; m < NR; ++m) {
      const int64_t o = base + threadIdx.x + 256 * m;
      if (o < tn) {
        const double v = b[o] - q[o];
        if (r) r[o] = v;
        acc += v * v;
      }
    }
  column_partials<NR>(acc, sh, partials + (int64_t)blockIdx.x * NR);
}
// the initial state (fresh solve, or a restart from the true residual that keeps tau^2, ||r_0||^2 and the
// iteration counts)
template <int NR>
__global__ __launch_bounds__(256) void k_pcg_init(PcgState* st, const double* __restrict__ partials, int nb,
                                                  int restart, double rtol, double atol, int nr_active, int flexible,
                                                  double* hist, double* rhist, int hist_rows) {
  __shared__ double sh[4 * NR];
  __shared__ double tot[NR];
  column_totals<NR>(partials, nb, NR, sh, tot);
  if (threadIdx.x == 0) {
    int all = 1;
    for (int c = 0; c < NR; ++c) {
      const double rr = tot[c];
      if (!restart) {
        st->rr0[c] = rr;
        st->tau2[c] = fmax(rtol * rtol * rr, atol * atol);  // ||r|| <= max(rtol ||r0||, atol)
        st->iters[c] = 0;
        if (rhist && hist_rows >= 0) rhist[c] = rr;
      }
      st->rr[c] = rr;
      st->rr_prev[c] = rr;
      st->rr_true[c] = rr;
      st->alpha[c] = 0;
      st->beta[c] = 0;
      st->done[c] = (c >= nr_active) || (rr <= st->tau2[c]);
      all &= st->done[c];
    }
    st->all_done = all;
    st->nr = NR;
    st->flexible = flexible;
    st->restart = 0;
    st->hist = hist;
    st->rhist = rhist;
    st->hist_rows = hist_rows;
  }
}
void launch_pcg_residual_init(int n, int nr, const double* b, const double* q, double* r, double* partials,
                              PcgState* st, int restart, double rtol, double atol, int nr_active, int flexible,
                              double* hist, double* rhist, int hist_rows, hipStream_t s) {
  const int g = pcg_grid(n);
#define R3_RI(NRV)                                                                                               \
  hipLaunchKernelGGL((k_pcg_residual<NRV>), dim3(g), dim3(256), 0, s, n, b, q, r, partials);                    \
  hipLaunchKernelGGL((k_pcg_init<NRV>), dim3(1), dim3(256), 0, s, st, partials, g, restart, rtol, atol, nr_active, \
                     flexible, hist, rhist, hist_rows)
  R3_NR_SWITCH(nr, R3_RI)
#undef R3_RI
  check_launch("k_pcg_residual / k_pcg_init");
}

// the true residual recorded, and a restart flagged when a column the recursive residual declared converged fails
// the stop rule with it
template <int NR>
__global__ __launch_bounds__(256) void k_pcg_true_check(PcgState* st, const double* __restrict__ partials, int nb) {
  __shared__ double sh[4 * NR];
  __shared__ double tot[NR];
  column_totals<NR>(partials, nb, NR, sh, tot);
  if (threadIdx.x == 0) {
    int rs = 0;
    for (int c = 0; c < NR; ++c) {
      st->rr_true[c] = tot[c];
      if (st->done[c] && tot[c] > st->tau2[c]) rs = 1;
    }
    st->restart = rs;
  }
}
void launch_pcg_true_residual(int n, int nr, const double* b, const double* q, double* partials, PcgState* st,
                              hipStream_t s) {
  const int g = pcg_grid(n);
#define R3_TR(NRV)                                                                                           \
  hipLaunchKernelGGL((k_pcg_residual<NRV>), dim3(g), dim3(256), 0, s, n, b, q, nullptr, partials);          \
  hipLaunchKernelGGL((k_pcg_true_check<NRV>), dim3(1), dim3(256), 0, s, st, partials, g)
  R3_NR_SWITCH(nr, R3_TR)
#undef R3_TR
  check_launch("k_pcg_residual / k_pcg_true_check");
}

// the state, word by word, into host-mapped pinned memory
__global__ void k_pcg_state_out(const uint64_t* __restrict__ src, uint64_t* dst, int words) {
  for (int i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
}
void launch_pcg_state_out(const PcgState* st, PcgState* host_mapped, hipStream_t s) {
  static_assert(sizeof(PcgState) % 8 == 0, "PcgState is copied in 8-byte words");
  hipLaunchKernelGGL(k_pcg_state_out, dim3(1), dim3(256), 0, s, reinterpret_cast<const uint64_t*>(st),
                     reinterpret_cast<uint64_t*>(host_mapped), (int)(sizeof(PcgState) / 8));
  check_launch("k_pcg_state_out");
}

template <typename T>
__global__ void k_vc_prep(int64_t count, int nr, const double* __restrict__ r, T* b0, const T* __restrict__ dinv0,
                          T* d0, T inv_theta0, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= count) return;
  const T v = (T)r[t];
  if (b0) b0[t] = v;
  if (d0) d0[t] = dinv0[t / nr] * v * inv_theta0;
}
template <typename T>
void launch_vc_prep(int n, int nr, const double* r, T* b0, const T* dinv0, T* d0, double inv_theta0,
                    const int* skip, hipStream_t s) {
  const int64_t tot = (int64_t)n * nr;
  hipLaunchKernelGGL((k_vc_prep<T>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, tot, nr, r, b0, dinv0, d0,
                     (T)inv_theta0, skip);
  check_launch("k_vc_prep");
}
template void launch_vc_prep<float>(int, int, const double*, float*, const float*, float*, double, const int*,
                                    hipStream_t);
template void launch_vc_prep<double>(int, int, const double*, double*, const double*, double*, double, const int*,
                                     hipStream_t);

// =============================================================================================
// FEM helpers for the differentiable solve
// =============================================================================================
// g_e = - sum_{a,b free} lam[c_ea] Ke[a,b] u[c_eb]; one wave per cell
__global__ __launch_bounds__(256) void k_cell_grad(int64_t ncells, int nloc, const int* __restrict__ cells,
                                                   const double* __restrict__ Ke, int64_t ke_stride,
                                                   const double* __restrict__ u, const double* __restrict__ lam,
                                                   const unsigned char* __restrict__ cons, double* g) {
  const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (e >= ncells) return;
  const int* c = cells + e * nloc;
  const double* K = Ke + e * ke_stride;
  double acc = 0;
  for (int a = 0; a < nloc; ++a) {
    const int ia = c[a];
    if (cons[ia]) continue;
    const double la = lam[ia];
    double s = 0;
    for (int b = lane; b < nloc; b += 64) {
      const int ib = c[b];
      if (!cons[ib]) s += K[(int64_t)a * nloc + b] * u[ib];
    }
    acc += la * s;
  }
  acc = wave_sum(acc, 64);
  if (lane == 0) g[e] = -acc;
}
void launch_cell_grad(int64_t ncells, int nloc, const int* cells, const double* Ke, int64_t ke_stride,
                      const double* u, const double* lam, const unsigned char* constrained_user, double* g,
                      hipStream_t s) {
  if (ncells == 0) return;
  hipLaunchKernelGGL(k_cell_grad, dim3((unsigned)((ncells + 3) / 4)), dim3(256), 0, s, ncells, nloc, cells, Ke,
                     ke_stride, u, lam, constrained_user, g);
  check_launch("k_cell_grad");
}

// vals[s] = sum over the contributions of slot s (cell e, local pair a*nloc+b, encoded e*nloc^2 + pair) of
// kappa_e Ke_e[a,b]; constrained diagonal slots get 1.0
__global__ void k_assemble(int64_t nnz, const int64_t* __restrict__ sp, const int64_t* __restrict__ contrib,
                           const double* __restrict__ kappa, const double* __restrict__ Ke, int64_t ke_stride,
                           int nloc, const unsigned char* __restrict__ diag_one, double* vals) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= nnz) return;
  const bool one = diag_one[s];
  const int64_t m0 = sp[s], m1 = sp[s + 1];
  const int64_t nl2 = (int64_t)nloc * nloc;
  double acc = 0;
  // four contributions at a time, their loads issued together from clamped indices, summed in order
  for (int64_t m = m0; m < m1; m += 4) {
    int64_t code[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) code[u] = contrib[min(m + u, m1 - 1)];
    double kv[4], kev[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t e = code[u] / nl2, pr = code[u] - e * nl2;
      kv[u] = kappa[e];
      kev[u] = Ke[e * ke_stride + pr];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (m + u < m1) acc += kv[u] * kev[u];
  }
  vals[s] = one ? 1.0 : acc;
}
void launch_assemble(int64_t nnz, const int64_t* slot_ptr, const int64_t* contrib, const double* kappa,
                     const double* Ke, int64_t ke_stride, int nloc, const unsigned char* diag_one, double* vals,
                     hipStream_t s) {
  if (nnz == 0) return;
  hipLaunchKernelGGL(k_assemble, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, nnz, slot_ptr, contrib, kappa,
                     Ke, ke_stride, nloc, diag_one, vals);
  check_launch("k_assemble");
}

}  // namespace r3mg
