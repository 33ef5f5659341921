// rgf_engine.hpp -- workgroup-level dense complex kernels of the half-slice
// recursion: in-register Gauss-Jordan inversion with partial pivoting and a
// register-output GEMM staged through LDS.
//
// Register layout ("column layout"): a workgroup of NW waves holds an
// NP x NP complex matrix (NP = NW*C); lane l owns rows l + 64 s (s < S) and
// wave w owns the C columns w*C .. w*C + C - 1, so a thread holds S x C
// entries. A matrix of size n < NP is padded with the identity, which the
// elimination leaves untouched.

#pragma once

#include "rgf_device.hpp"

namespace rgf {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Returns p unchanged but opaque to the optimiser, so address arithmetic
// derived from a loop-invariant, wave-uniform pointer is not hoisted out of
// the slice loop (hoisted per-lane addresses would occupy dozens of VGPRs
// for the whole sweep).
// The pointer must be wave-uniform; it is moved to SGPRs first.
template <typename P>
__device__ __forceinline__ P* opaque_uniform(P* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  asm volatile("" : "+s"(lo), "+s"(hi));
  return reinterpret_cast<P*>(((uint64_t)hi << 32) | lo);
}

template <typename T, int S, int C>
__device__ __forceinline__ void zero_regs(cx<T> (&A)[S][C]) {
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int j = 0; j < C; ++j) A[s][j] = mk<T>(T(0), T(0));
}

// ----------------------------------------------------------------------------
// Gauss-Jordan inversion in place, partial pivoting without row exchanges.
//
// Step k picks the pivot row p_k = argmax |A[r][k]| over rows not used yet
// (|re| + |im|, ties to the lowest row), scales row p_k by 1/A[p_k][k] and
// eliminates column k from every other row, storing the inverse's column in
// place of the eliminated one. Without exchanges the array ends as
// X = P^T A^{-1} P^T for the row permutation P that maps step k to row p_k:
// A^{-1}[i][j] = X[p_i][q_j] with q the inverse permutation (q_{p_k} = k).
//
// The step is written as one update with no per-element selection:
//   A[r][c] -= m'_r * v_c,   v_c = A[p][c] (c != k), v_k = 1,
//   m'_r = A[r][k] / A[p][k] (r != p),  m'_p = 1 - 1/A[p][k],
// after column k is reset to the unit vector e_p. This yields the scaled
// pivot row in row p, the eliminated rows elsewhere, and the inverse's column
// (-A[r][k]/piv, 1/piv at p) in column k.
//
// One barrier per step: the wave owning column k+1 selects its pivot right
// after updating, computes 1/pivot, and publishes the column, the pivot row
// index and 1/pivot through double-buffered LDS. The raw pivot row of each
// wave's columns is broadcast inside the wave through its LDS scratch.
//
// LDS: colbuf[2][NP] (T), ipivbuf[2] (T), wbuf[NW][NP] (T), pivrow[NP],
// pinv[NP] (int), flag (int; set to 1 on an exact zero pivot).
// ----------------------------------------------------------------------------
template <typename T, int NW, int S, int C, int J>
__device__ __forceinline__ void gj_pivot_publish(const cx<T> (&A)[S][C], int kc, int n,
                                                 uint32_t used, cx<T>* colbuf, cx<T>* ipivbuf,
                                                 int* pivrow, int* flag) {
  constexpr int NP = NW * C;
  const int lane = lane_id();
  T best = T(-1);
  int bidx = 0x7fffffff;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int r = lane + 64 * s;
    // NaN magnitudes count as 0 so an unused row always wins over -1 and
    // the pivot index stays inside [0, n)
    T mag = T(-1);
    if (r < n && !((used >> s) & 1u)) {
      mag = cabs1(A[s][J]);
      if (!(mag >= T(0))) mag = T(0);
    }
    if (mag > best) {
      best = mag;
      bidx = r;
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    T ob = __shfl_xor(best, off);
    int oi = __shfl_xor(bidx, off);
    if (ob > best || (ob == best && oi < bidx)) {
      best = ob;
      bidx = oi;
    }
  }
  cx<T>* cb = colbuf + (kc & 1) * NP;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int r = lane + 64 * s;
    if (r < NP) cb[r] = A[s][J];
  }
  // the pivot value is read back from the published column (LDS requests of
  // one wave complete in order)
  wave_sync_lds();
  if (lane == 0) {
    pivrow[kc] = bidx;
    ipivbuf[kc & 1] = crcp(cb[min(bidx, NP - 1)]);
    if (!(best > T(0))) *flag = 1;
  }
}

// Calls gj_pivot_publish for the register column that holds column kc.
template <typename T, int NW, int S, int C, int J = 0>
__device__ __forceinline__ void gj_pivot_dispatch(const cx<T> (&A)[S][C], int kc, int n,
                                                  uint32_t used, cx<T>* colbuf,
                                                  cx<T>* ipivbuf, int* pivrow, int* flag) {
  if constexpr (J < C) {
    if (wave_id() * C + J == kc)
      gj_pivot_publish<T, NW, S, C, J>(A, kc, n, used, colbuf, ipivbuf, pivrow, flag);
    else
      gj_pivot_dispatch<T, NW, S, C, J + 1>(A, kc, n, used, colbuf, ipivbuf, pivrow, flag);
  }
}

// Column k := e_p in the register column that holds it (if this wave owns it).
template <typename T, int NW, int S, int C, int J = 0>
__device__ __forceinline__ void gj_unit_column(cx<T> (&A)[S][C], int k, int pk) {
  if constexpr (J < C) {
    if (wave_id() * C + J == k) {
      const int lane = lane_id();
#pragma unroll
      for (int s = 0; s < S; ++s)
        A[s][J] = mk<T>((lane + 64 * s == pk) ? T(1) : T(0), T(0));
    } else {
      gj_unit_column<T, NW, S, C, J + 1>(A, k, pk);
    }
  }
}

template <typename T, int NW, int S, int C>
__device__ __forceinline__ void gj_invert(cx<T> (&A)[S][C], int n, cx<T>* colbuf,
                                          cx<T>* wbuf_all, int* pivrow, int* pinv,
                                          int* flag) {
  constexpr int NP = NW * C;
  constexpr int NT = NW * 64;
  const int lane = lane_id(), w = wave_id();
  cx<T>* wbuf = wbuf_all + w * NP;
  cx<T>* ipivbuf = colbuf + 2 * NP;
  uint32_t used = 0;
  if (n > 0 && w == 0)
    gj_pivot_dispatch<T, NW, S, C>(A, 0, n, used, colbuf, ipivbuf, pivrow, flag);
  for (int k = 0; k < n; ++k) {
    __syncthreads();
    const cx<T>* cb = colbuf + (k & 1) * NP;
    const int pk = min(max(pivrow[k], 0), NP - 1);
    const int pl = pk & 63, ps = pk >> 6;
    const cx<T> ipiv = ipivbuf[k & 1];
    cx<T> m[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int r = lane + 64 * s;
      const cx<T> a = (r < NP) ? cb[r] : mk<T>(T(0), T(0));
      m[s] = (r == pk) ? mk<T>(T(1) - ipiv.re, -ipiv.im) : cmul(a, ipiv);
    }
    // raw pivot row of this wave's columns, with 1 in column k: the pivot
    // lane writes all S of its rows (constant register indices keep the tile
    // in registers); the readers pick slot ps by LDS address
    if (lane == pl) {
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int j = 0; j < C; ++j) wbuf[s * C + j] = A[s][j];
      used |= 1u << ps;
    }
    if (lane == 0 && w == k / C) wbuf[ps * C + k - w * C] = mk<T>(T(1), T(0));
    wave_sync_lds();
    gj_unit_column<T, NW, S, C>(A, k, pk);
    const cx<T>* prow = wbuf + ps * C;
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const cx<T> v = prow[j];
#pragma unroll
      for (int s = 0; s < S; ++s) A[s][j] = cfms(m[s], v, A[s][j]);
    }
    if (k + 1 < n && w == (k + 1) / C)
      gj_pivot_dispatch<T, NW, S, C>(A, k + 1, n, used, colbuf, ipivbuf, pivrow, flag);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += NT) pinv[pivrow[i]] = i;
  __syncthreads();
}

// Write the inverse held (permuted) in registers to a column-major global
// buffer K with leading dimension NP: K[i][j] = X[p_i][q_j]. Each wave takes
// its columns c (target column p_c), un-permutes the rows through its LDS
// scratch and stores whole columns coalesced. Columns/rows >= n are skipped.
// If K2 is non-null the same matrix is also written there.
template <typename T, typename TG, int NW, int S, int C>
__device__ __forceinline__ void store_unpermuted(const cx<T> (&X)[S][C], int n,
                                                 cx<T>* wbuf_all, const int* pivrow,
                                                 const int* pinv, cx<TG>* K,
                                                 cx<TG>* K2) {
  constexpr int NP = NW * C;
  const int lane = lane_id(), w = wave_id();
  cx<T>* wbuf = wbuf_all + w * NP;
  K = opaque_uniform(K);
  if (K2) K2 = opaque_uniform(K2);
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int c = w * C + j;
    if (c >= n) break;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int r = lane + 64 * s;
      if (r < n) wbuf[pinv[r]] = X[s][j];
    }
    wave_sync_lds();
    const int col = pivrow[c];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int r = lane + 64 * s;
      if (r < n) {
        cx<T> v = wbuf[r];
        cx<TG> g = mk<TG>((TG)v.re, (TG)v.im);
        stg(K + (size_t)col * NP + r, g);
        if (K2) stg(K2 + (size_t)col * NP + r, g);
      }
    }
    wave_sync_lds();
  }
}

// Store registers (natural order) to a column-major buffer, ld = NP, rows and
// columns below nr x nc.
template <typename T, typename TG, int NW, int S, int C>
__device__ __forceinline__ void store_regs(const cx<T> (&X)[S][C], int nr, int nc,
                                           cx<TG>* K) {
  constexpr int NP = NW * C;
  const int lane = lane_id(), w = wave_id();
  K = opaque_uniform(K);
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int c = w * C + j;
    if (c >= nc) break;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int r = lane + 64 * s;
      if (r < nr) stg(K + (size_t)c * NP + r, mk<TG>((TG)X[s][j].re, (TG)X[s][j].im));
    }
  }
}

// ----------------------------------------------------------------------------
// acc[r][c] = sum_{k < nk} fa(r, k) * fb(k, c) for the NP x NP register tile.
// The accessors return zero outside the operand shapes. Operands are staged
// KC columns of fa / KC rows of fb at a time through LDS (As[KC][NP],
// Bs[KC][NP]); each lane reads its S rows of As and the wave's C columns of Bs
// (a broadcast read), then issues S*C complex FMAs.
// ----------------------------------------------------------------------------
template <typename TA, int NW, int S, int C, int KC, class FA, class FB>
__device__ __forceinline__ void gemm_regs(cx<TA> (&acc)[S][C], int nk, FA fa, FB fb,
                                          cx<TA>* As, cx<TA>* Bs) {
  constexpr int NP = NW * C;
  constexpr int NT = NW * 64;
  const int lane = lane_id(), w = wave_id();
  zero_regs(acc);
  for (int k0 = 0; k0 < nk; k0 += KC) {
    for (int idx = threadIdx.x; idx < KC * NP; idx += NT) {
      const int kk = idx / NP, r = idx - kk * NP;
      As[idx] = (k0 + kk < nk) ? fa(r, k0 + kk) : mk<TA>(TA(0), TA(0));
    }
    for (int idx = threadIdx.x; idx < KC * NP; idx += NT) {
      const int c = idx / KC, kk = idx - c * KC;
      Bs[kk * NP + c] = (k0 + kk < nk) ? fb(k0 + kk, c) : mk<TA>(TA(0), TA(0));
    }
    __syncthreads();
#pragma unroll 1
    for (int kk = 0; kk < KC; ++kk) {
      cx<TA> a[S];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int r = lane + 64 * s;
        a[s] = (r < NP) ? As[kk * NP + r] : mk<TA>(TA(0), TA(0));
      }
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const cx<TA> b = Bs[kk * NP + w * C + j];
#pragma unroll
        for (int s = 0; s < S; ++s) acc[s][j] = cfma(a[s], b, acc[s][j]);
      }
    }
    __syncthreads();
  }
}

// Block-wide sum of one double per thread (result valid in every thread).
template <int NW>
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if (lane_id() == 0) red[wave_id()] = v;
  __syncthreads();
  double tot = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) tot += red[i];
  __syncthreads();
  return tot;
}

// Block-wide max of one double per thread (NaN propagates as the max).
template <int NW>
__device__ __forceinline__ double block_max(double v, double* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double o = __shfl_xor(v, off);
    v = (o > v || o != o) ? o : v;
  }
  __syncthreads();
  if (lane_id() == 0) red[wave_id()] = v;
  __syncthreads();
  double m = red[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) m = (red[i] > m || red[i] != red[i]) ? red[i] : m;
  __syncthreads();
  return m;
}

}  // namespace rgf
