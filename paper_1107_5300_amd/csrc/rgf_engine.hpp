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
__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: lets the compiler branch on it
}

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
//   A[r][c] -= m'_r * v_c,   v_c = A[p][c] (c != k),  v_k = A[p][k] + 1,
//   m'_r = A[r][k] / A[p][k] (r != p),  m'_p = 1 - 1/A[p][k].
// For c != k this is the elimination (rows r != p) and the scaling of the
// pivot row (row p). For column k it yields -A[r][k]/A[p][k] in rows r != p
// and 1/A[p][k] in row p, the inverse's column, so column k needs no reset.
// The constant 1 in m'_p and v_k makes the rounding error grow with |pivot|
// (relative to the result); the caller scales the matrix to entries of
// magnitude below 1 (an exact power of two) to keep the error at the level
// of the elimination itself.
//
// The k loop runs as a runtime loop over wave blocks (k = kb*C + J) around
// compile-time steps J, so every register access has a constant index. One
// barrier per step; the wave that owns column k+1 updates that column first,
// then selects its pivot (a packed 32-bit key reduced across the wave by
// DPP, no LDS round trip), publishes the column, the pivot row and 1/pivot
// through double-buffered LDS, and updates its other columns while the
// other waves do theirs. Inside each wave the pivot row's entries of the
// wave's columns (pivot + 1 in column k) go from the pivot lane to all lanes
// through scalar registers.
//
// LDS: colbuf[2][NP + 1] (T: the column, then 1/pivot), pivrow[NP],
// pinv[NP] (int), flag (int; set to 1 on an exact zero pivot).
// ----------------------------------------------------------------------------
// Wave-wide maximum of a 32-bit key by DPP (no LDS traffic); every lane
// gets the result.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));  // quad [1,0,3,2]
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));  // quad [2,3,0,1]
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false)); // row_half_mirror
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false)); // row_mirror
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false)); // row_bcast:15
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false)); // row_bcast:31
  return __builtin_amdgcn_readlane(v, 63);
}

// Pivot key of row r: the magnitude |re|+|im| rounded to float with its
// low 8 bits replaced by 255 - r, so the largest key is the largest
// magnitude (to a relative 2^-15, ample for partial pivoting) and, among
// equal magnitudes, the lowest row. Unusable rows get 0; usable rows with a
// zero (or NaN) magnitude still get 255 - r > 0, so the choice stays a valid,
// unused row.
template <typename T>
__device__ __forceinline__ uint32_t pivot_key(cx<T> v, int r, bool usable) {
  if (!usable) return 0u;
  float m = (float)cabs1(v);
  if (!(m >= 0.0f)) m = 0.0f;
  return (__float_as_uint(m) & 0xFFFFFF00u) | (uint32_t)(255 - r);
}

// Register column J of slot s (s uniform or not; a chain of selects over the
// S slots, with constant register indices).
template <typename T, int S, int C, int J>
__device__ __forceinline__ cx<T> pick_slot(const cx<T> (&A)[S][C], int s) {
  cx<T> v = A[0][J];
#pragma unroll
  for (int i = 1; i < S; ++i)
    if (s == i) v = A[i][J];
  return v;
}

// A[s][J] -= m[s] * v  for one register column.
template <typename T, int S, int C, int J>
__device__ __forceinline__ void gj_update_column(cx<T> (&A)[S][C], const cx<T> (&m)[S],
                                                 cx<T> v) {
#pragma unroll
  for (int s = 0; s < S; ++s) A[s][J] = cfms(m[s], v, A[s][J]);
}

template <typename T, int S, int C, int J, int SKIP>
__device__ __forceinline__ void gj_update_rest(cx<T> (&A)[S][C], const cx<T> (&m)[S],
                                               const cx<T> (&v)[C]) {
  if constexpr (J < C) {
    if constexpr (J != SKIP) gj_update_column<T, S, C, J>(A, m, v[J]);
    gj_update_rest<T, S, C, J + 1, SKIP>(A, m, v);
  }
}

// Pivot selection for column kc, held in register column J of the calling
// (owner) wave: publishes the column, the pivot row and 1/pivot.
template <typename T, int NW, int S, int C, int J>
__device__ __forceinline__ void gj_select_pivot(const cx<T> (&A)[S][C], int kc, int n,
                                                uint32_t used, cx<T>* colbuf, int* pivrow,
                                                int* flag) {
  constexpr int NP = NW * C;
  const int lane = lane_id();
  cx<T>* cb = colbuf + (kc & 1) * (NP + 1);
  uint32_t key = 0u;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int r = lane + 64 * s;
    if (r < NP) cb[r] = A[s][J];
    key = max(key, pivot_key(A[s][J], r, r < n && !((used >> s) & 1u)));
  }
  key = wave_max_u32(key);
  const int pk = min(255 - (int)(key & 0xFFu), NP - 1);
  if (lane == (pk & 63)) {
    const cx<T> pv = pick_slot<T, S, C, J>(A, pk >> 6);
    pivrow[kc] = pk;
    cb[NP] = crcp_scaled(pv);
    if (!(cabs1(pv) > T(0))) *flag = 1;
  }
}

// Wave broadcast of lane l's value through a scalar register (l uniform).
__device__ __forceinline__ double lane_bcast(double x, int l) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)v, l);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane_bcast(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// v[g] = A[ps][J0 + g] of lane pl, for g < G except column SKIP (ps and pl
// uniform). One branch per register slot keeps the register indices
// constant; the empty asm statement, distinct per slot, keeps the optimiser
// from merging the branches into a dynamically indexed (scratch) access.
template <typename T, int S, int C, int J0, int G, int SKIP, int SS>
__device__ __forceinline__ void gj_row_chunk(const cx<T> (&A)[S][C], int ps, int pl,
                                             cx<T> (&v)[G]) {
  if constexpr (SS < S) {
    if (ps == SS) {
#pragma unroll
      for (int g = 0; g < G; ++g)
        if (J0 + g != SKIP) v[g] = mk<T>(lane_bcast(A[SS][J0 + g].re, pl),
                                         lane_bcast(A[SS][J0 + g].im, pl));
      asm volatile("; gj row chunk slot %0" ::"n"(SS));
    } else {
      gj_row_chunk<T, S, C, J0, G, SKIP, SS + 1>(A, ps, pl, v);
    }
  }
}

// Update of the register columns J0.. except SKIP, in chunks of up to 5
// columns (broadcast the chunk's pivot-row entries, then update it); column
// J (the pivot column k, owner wave only) takes pivot + 1.
template <typename T, int S, int C, int J, int SKIP, int J0>
__device__ __forceinline__ void gj_update_chunks(cx<T> (&A)[S][C], const cx<T> (&m)[S], int ps,
                                                 int pl, bool own) {
  if constexpr (J0 < C) {
    constexpr int G = (C - J0 < 5) ? C - J0 : 5;
    cx<T> v[G];
    gj_row_chunk<T, S, C, J0, G, SKIP, 0>(A, ps, pl, v);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (J0 + g == SKIP) continue;
      cx<T> x = v[g];
      if (J0 + g == J && own) x.re += T(1);
#pragma unroll
      for (int s = 0; s < S; ++s) A[s][J0 + g] = cfms(m[s], x, A[s][J0 + g]);
    }
    gj_update_chunks<T, S, C, J, SKIP, J0 + G>(A, m, ps, pl, own);
  }
}

// Elimination step k = kb*C + J (J compile-time). The pivot row's entries
// of this wave's columns go from the pivot lane to the whole wave through
// scalar registers (readlane), with no LDS traffic.
template <typename T, int NW, int S, int C, int J>
__device__ __forceinline__ void gj_step(cx<T> (&A)[S][C], int kb, int n, uint32_t& used,
                                        cx<T>* colbuf, int* pivrow, int* flag) {
  constexpr int NP = NW * C;
  constexpr int JN = (J + 1) % C;  // register column of k + 1
  const int lane = lane_id(), w = wave_id();
  const int k = kb * C + J;
  const int kbn = (J + 1 == C) ? kb + 1 : kb;  // owner wave of k + 1
  __syncthreads();
  // all LDS reads of the step's column in one round trip
  const cx<T>* cb = colbuf + (k & 1) * (NP + 1);
  const int pkr = pivrow[k];
  const cx<T> ipiv = cb[NP];
  cx<T> a[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int r = lane + 64 * s;
    a[s] = (r < NP) ? cb[r] : mk<T>(T(0), T(0));
  }
  __builtin_amdgcn_sched_barrier(0);
  const int pk = __builtin_amdgcn_readfirstlane(min(max(pkr, 0), NP - 1));
  const int pl = pk & 63, ps = pk >> 6;
  cx<T> m[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int r = lane + 64 * s;
    m[s] = (r == pk) ? mk<T>(T(1) - ipiv.re, -ipiv.im) : cmul(a[s], ipiv);
  }
  if (lane == pl) used |= 1u << ps;
  const bool own = (w == kb);
  // the look-ahead wave's chain (column k+1, pivot, publication) is what the
  // next barrier waits for: it issues ahead of the other wave on its SIMD
  const bool la = (w == kbn && k + 1 < n);
  if (la) __builtin_amdgcn_s_setprio(2);
  {
    cx<T> v1[1];
    gj_row_chunk<T, S, C, JN, 1, -1, 0>(A, ps, pl, v1);
    gj_update_column<T, S, C, JN>(A, m, v1[0]);
  }
  if (la) {
    gj_select_pivot<T, NW, S, C, JN>(A, k + 1, n, used, colbuf, pivrow, flag);
    __builtin_amdgcn_s_setprio(0);
  }
  gj_update_chunks<T, S, C, J, JN, 0>(A, m, ps, pl, own);
}

template <typename T, int NW, int S, int C, int J>
__device__ __forceinline__ void gj_block(cx<T> (&A)[S][C], int kb, int n, uint32_t& used,
                                         cx<T>* colbuf, int* pivrow, int* flag) {
  if constexpr (J < C) {
    if (kb * C + J >= n) return;
    gj_step<T, NW, S, C, J>(A, kb, n, used, colbuf, pivrow, flag);
    gj_block<T, NW, S, C, J + 1>(A, kb, n, used, colbuf, pivrow, flag);
  }
}

template <typename T, int NW, int S, int C>
__device__ __forceinline__ void gj_invert(cx<T> (&A)[S][C], int n, cx<T>* colbuf, int* pivrow,
                                          int* pinv, int* flag) {
  constexpr int NT = NW * 64;
  const int w = wave_id();
  uint32_t used = 0;
  if (n > 0 && w == 0) gj_select_pivot<T, NW, S, C, 0>(A, 0, n, used, colbuf, pivrow, flag);
  for (int kb = 0; kb < NW; ++kb) {
    if (kb * C >= n) break;
    gj_block<T, NW, S, C, 0>(A, kb, n, used, colbuf, pivrow, flag);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += NT) pinv[pivrow[i]] = i;
  __syncthreads();
}

// Scale factor for the inversion: 2^-e with the largest |re| + |im| of the
// tile in [2^(e-1), 2^e), so the scaled entries lie below 1 (1 if the tile
// holds a NaN or an infinity; a zero tile is left as it is). The maximum is
// taken on the high 32 bits of the magnitudes (monotone for non-negative
// floating-point numbers). Costs one barrier, which also orders the previous
// users of the shared buffers before the inversion.
__device__ __forceinline__ uint32_t mag_hi(double v) {
  return (uint32_t)((uint64_t)__double_as_longlong(v) >> 32);
}
__device__ __forceinline__ uint32_t mag_hi(float v) { return __float_as_uint(v); }

template <typename T, int NW, int S, int C>
__device__ __forceinline__ T tile_scale(const cx<T> (&A)[S][C], uint32_t* red) {
  constexpr bool F64 = sizeof(T) == sizeof(double);
  constexpr int MB = F64 ? 20 : 23;           // mantissa bits in the high word
  constexpr uint32_t EMAX = F64 ? 0x7FFu : 0xFFu;
  constexpr int BIAS = F64 ? 1023 : 127, EMIN = F64 ? -1022 : -126;
  uint32_t b = 0u;
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int j = 0; j < C; ++j) b = max(b, mag_hi(cabs1(A[s][j])));
  b = wave_max_u32(b);
  if (lane_id() == 0) red[wave_id()] = b;
  __syncthreads();
  uint32_t m = red[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) m = max(m, red[i]);
  const int ex = (int)((m >> MB) & EMAX);
  if (m == 0u || ex == (int)EMAX) return T(1);
  // max in [2^(ex-BIAS), 2^(ex-BIAS+1)) -> multiply by 2^(BIAS-1-ex)
  // (a subnormal maximum, ex = 0, scales by 2^(BIAS-1))
  return (T)ldexp(1.0, max(BIAS - 1 - ex, EMIN));
}

template <typename T, int S, int C>
__device__ __forceinline__ void scale_regs(cx<T> (&A)[S][C], T f) {
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int j = 0; j < C; ++j) A[s][j] = cscale(A[s][j], f);
}

// Write the inverse held (permuted) in registers to a column-major global
// buffer K with leading dimension NP: K[i][j] = X[p_i][q_j]. Each wave takes
// its columns c (target column p_c), un-permutes the rows through its LDS
// scratch and stores whole columns coalesced. Columns/rows >= n are skipped.
// Every entry is multiplied by f (the scale of the inversion; a power of
// two). If K2 is non-null the same matrix is also written there.
// veps (optional): on-site energies of the matrix's rows, row a at
// veps[2 a + e]; the diagonal entry of a vacancy (+inf, whose row and column
// of the inverted matrix were the identity's) is stored as 0.
template <typename T, typename TG, int NW, int S, int C>
__device__ __forceinline__ void store_unpermuted(const cx<T> (&X)[S][C], int n, T f,
                                                 cx<T>* wbuf_all, const int* pivrow,
                                                 const int* pinv, cx<TG>* K,
                                                 cx<TG>* K2, const double* veps = nullptr,
                                                 int e = 0) {
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
    const bool vcol = veps && is_vacancy(veps[half_row(col, e)]);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int r = lane + 64 * s;
      if (r < n) {
        cx<T> v = wbuf[r];
        cx<TG> g = mk<TG>((TG)(v.re * f), (TG)(v.im * f));
        if (vcol && r == col) g = mk<TG>(TG(0), TG(0));
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

// Store registers (natural order) to a row-major buffer, ld = NP: K[r*NP + c]
// for r < nr, c < nc.
template <typename T, typename TG, int NW, int S, int C>
__device__ __forceinline__ void store_regs_rowmajor(const cx<T> (&X)[S][C], int nr, int nc,
                                                    cx<TG>* K) {
  const int lane = lane_id(), w = wave_id();
  K = opaque_uniform(K);
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int c = w * C + j;
    if (c >= nc) break;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int r = lane + 64 * s;
      if (r < nr) stg(K + (size_t)r * NW * C + c, mk<TG>((TG)X[s][j].re, (TG)X[s][j].im));
    }
  }
}

// ----------------------------------------------------------------------------
// acc[r][c] = sum_{k < nk} fa(r, k) * fb(k, c) for the NP x NP register tile.
// The accessors return zero outside the operand shapes. KC columns of fa and
// KC rows of fb are staged through double-buffered LDS (As[2][KC][NP],
// Bs[2][KC][NP]): the global loads of chunk c+1 are issued before the FMAs
// of chunk c and written to the other buffer afterwards, so one barrier per
// chunk suffices. Each lane reads its S rows of As and the wave's C columns
// of Bs (a broadcast read), then issues S*C complex FMAs.
// ----------------------------------------------------------------------------
template <typename TA, int NW, int S, int C, int KC, class FA, class FB>
__device__ __forceinline__ void gemm_regs(cx<TA> (&acc)[S][C], int nk, FA fa, FB fb,
                                          cx<TA>* As, cx<TA>* Bs) {
  constexpr int NP = NW * C;
  constexpr int NT = NW * 64;
  constexpr int CH = KC * NP;
  constexpr int PER = (CH + NT - 1) / NT;
  const int lane = lane_id(), w = wave_id();
  zero_regs(acc);
  const int nch = (nk + KC - 1) / KC;
  cx<TA> ra[PER], rb[PER];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = threadIdx.x + i * NT;
      ra[i] = mk<TA>(TA(0), TA(0));
      rb[i] = mk<TA>(TA(0), TA(0));
      if (idx < CH) {
        const int kk = idx / NP, r = idx - kk * NP;
        if (k0 + kk < nk) ra[i] = fa(r, k0 + kk);
        const int c = idx / KC, kb = idx - c * KC;
        if (k0 + kb < nk) rb[i] = fb(k0 + kb, c);
      }
    }
  };
  auto put = [&](int buf) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = threadIdx.x + i * NT;
      if (idx < CH) {
        As[buf * CH + idx] = ra[i];
        const int c = idx / KC, kb = idx - c * KC;
        Bs[buf * CH + kb * NP + c] = rb[i];
      }
    }
  };
  if (nch > 0) {
    fetch(0);
    put(0);
  }
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const bool more = ch + 1 < nch;
    if (more) fetch((ch + 1) * KC);
    const cx<TA>* Ab = As + (ch & 1) * CH;
    const cx<TA>* Bb = Bs + (ch & 1) * CH;
#pragma unroll 1
    for (int kk = 0; kk < KC; ++kk) {
      cx<TA> a[S];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int r = lane + 64 * s;
        a[s] = (r < NP) ? Ab[kk * NP + r] : mk<TA>(TA(0), TA(0));
      }
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const cx<TA> b = Bb[kk * NP + w * C + j];
#pragma unroll
        for (int s = 0; s < S; ++s) acc[s][j] = cfma(a[s], b, acc[s][j]);
        // bound the broadcast loads in flight (register pressure)
        if ((j & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
    }
    if (more) put((ch + 1) & 1);
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
