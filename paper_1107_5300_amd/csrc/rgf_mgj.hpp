// rgf_mgj.hpp -- blocked Gauss-Jordan inversion of one half-slice matrix
// (n <= 128, complex, FP64 or FP32) on the matrix cores.
//
// The 8 waves of the workgroup hold the 128 x 128 tile in the accumulator
// layout of the 16 x 16 x 4 MFMA: wave w owns tile column w (columns
// 16 w .. 16 w + 15), as eight 16 x 16 tiles, i.e. 32 complex entries per
// lane. Column panel p (16 columns) is tile column p. Gauss-Jordan with
// partial pivoting over the rows not yet used, without row exchanges, is
// done panel by panel:
//
//   * the owner wave of panel p copies its tiles to LDS, reads them back one
//     row pair per lane and eliminates the panel's (up to) 16 columns with
//     the select-free step of rgf_engine.hpp, pivots chosen by a wave
//     reduction and the pivot row broadcast through scalar registers: no
//     workgroup barrier inside a panel;
//   * the panel's steps act on every other column v as one linear map,
//     v <- v + (Z - E_P) v_P (Z the eliminated panel, E_P the unit columns of
//     its pivot rows P, v_P the entries of v in those rows), so every other
//     wave applies a rank-16 update to its tile column on the matrix cores,
//     reading Z from LDS as the A operand and its own pivot-row entries,
//     staged through LDS, as the B operand;
//   * look-ahead: the owner of panel p + 1 updates its own tiles first and
//     eliminates panel p + 1 while the others apply panel p, so one barrier
//     per panel orders the whole inversion (Z double-buffered in LDS).
//
// After the last panel the tiles hold the inverse with rows and columns
// permuted by the pivot order (A^{-1}[i][j] = X[p_i][q_j], q the inverse
// permutation), as in the register version; it is written out un-permuted.
// Rows and columns >= n are the identity and stay untouched.
//
// Accumulator layout (lane l, element v of a 16 x 16 tile; measured on
// gfx950): FP64 row 4 v + l / 16, FP32 row 4 (l / 16) + v; column l % 16
// for both. Operands: A lane l holds A[l % 16][l / 16], B lane l holds
// B[l / 16][l % 16].

#pragma once

#include "rgf_engine.hpp"

namespace rgf {

constexpr int MG_NP = 128;  // tile rows and columns
constexpr int MG_NW = 8;    // waves; wave w owns tile column w
constexpr int MG_TI = 8;    // 16-row tiles per tile column
constexpr int MG_ZLD = MG_NP + 4;  // LDS leading dimension of a panel column

template <typename T>
struct MgjVec;
template <>
struct MgjVec<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
};
template <>
struct MgjVec<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
};

__device__ __forceinline__ MgjVec<double>::v4 mgj_mfma(double a, double b, MgjVec<double>::v4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ MgjVec<float>::v4 mgj_mfma(float a, float b, MgjVec<float>::v4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row within a 16 x 16 tile of accumulator element v of a lane with l / 16 = lk.
template <typename T>
__device__ __forceinline__ int mgj_row(int v, int lk) {
  if constexpr (sizeof(T) == sizeof(double))
    return 4 * v + lk;
  else
    return 4 * lk + v;
}

template <typename T>
struct MgjTile {
  typename MgjVec<T>::v4 re[MG_TI], im[MG_TI];
};

template <typename T>
struct MgjSmem {
  cx<T> zbuf[2][16][MG_ZLD];  // panels, column-major (column j of the panel, row r)
  cx<T> vp[MG_NW][16][16];    // per wave: entries of its columns in the panel's pivot rows
  short pidx[2][MG_NP];       // panel-local pivot index of each row, -1 if none
  int pivrow[MG_NP];          // pivot row of each elimination step
  int pinv[MG_NP];
  unsigned char used[MG_NP];  // row already chosen as a pivot
  uint32_t red[MG_NW];
  cx<T> prow[16];             // pivot row of the current step (owner wave)
};

// Lane index opaque to the optimiser: offsets derived from it are then
// recomputed where they are used instead of being hoisted out of the slice
// loop, where dozens of them would stay live next to the 32-entry tile.
__device__ __forceinline__ int mgj_lane() {
  int lane = lane_id();
  asm volatile("" : "+v"(lane));
  return lane;
}

template <typename T>
__device__ __forceinline__ cx<T> mgj_get(const MgjTile<T>& D, int I, int v) {
  return mk<T>(D.re[I][v], D.im[I][v]);
}
template <typename T>
__device__ __forceinline__ void mgj_set(MgjTile<T>& D, int I, int v, cx<T> x) {
  D.re[I][v] = x.re;
  D.im[I][v] = x.im;
}

// Entries J0 .. J0 + G - 1 of the pivot row, from lane pl, slot ps (0 or 1,
// uniform): one branch per slot, kept apart by distinct empty asm
// statements so that the panel is never indexed dynamically.
template <typename T, int J0, int G>
__device__ __forceinline__ void mgj_pivot_row(const cx<T> (&Pc)[2][16], int ps, int pl,
                                              cx<T> (&v)[G]) {
  if (ps == 0) {
#pragma unroll
    for (int g = 0; g < G; ++g)
      v[g] = mk<T>(lane_bcast(Pc[0][J0 + g].re, pl), lane_bcast(Pc[0][J0 + g].im, pl));
    asm volatile("; mgj pivot row slot 0");
  } else {
#pragma unroll
    for (int g = 0; g < G; ++g)
      v[g] = mk<T>(lane_bcast(Pc[1][J0 + g].re, pl), lane_bcast(Pc[1][J0 + g].im, pl));
    asm volatile("; mgj pivot row slot 1");
  }
}

// Pivot of panel column J among the rows not used yet (largest |re|+|im|,
// ties to the lowest row), wave-uniform.
template <typename T, int J>
__device__ __forceinline__ int mgj_pivot(const cx<T> (&Pc)[2][16], int n, uint32_t used) {
  const int lane = lane_id();
  uint32_t key = 0u;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int r = lane + 64 * s;
    key = max(key, pivot_key(Pc[s][J], r, r < n && !((used >> s) & 1u)));
  }
  key = wave_max_u32(key);
  return __builtin_amdgcn_readfirstlane(min(255 - (int)(key & 0xFFu), MG_NP - 1));
}

// Elimination step K of panel p (K compile-time) with pivot row pk: the
// owner wave's panel in column layout (lane l: rows l and l + 64). The pivot
// row goes from the pivot lane to the whole wave through LDS; column K + 1
// is updated first and its pivot chosen while the other columns are
// updated (look-ahead inside the panel).
template <typename T, int K>
__device__ __forceinline__ void mgj_step(cx<T> (&Pc)[2][16], int p, int ks, int n, int pk,
                                         uint32_t& used, MgjSmem<T>& ms, int* flag) {
  if constexpr (K < 16) {
    if (K >= ks) return;
    const int lane = lane_id();
    const int pl = pk & 63, ps = pk >> 6;
    // one guarded store per slot, kept apart by distinct empty asm
    // statements (a select between the slots would index the panel
    // dynamically, which moves it to scratch memory)
    if (lane == pl && ps == 0) {
#pragma unroll
      for (int j = 0; j < 16; ++j) ms.prow[j] = Pc[0][j];
    }
    asm volatile("; mgj prow slot 0");
    if (lane == pl && ps == 1) {
#pragma unroll
      for (int j = 0; j < 16; ++j) ms.prow[j] = Pc[1][j];
    }
    asm volatile("; mgj prow slot 1");
    if (lane == pl) {
      ms.pivrow[16 * p + K] = pk;
      ms.pidx[p & 1][pk] = (short)K;
      ms.used[pk] = 1;
      used |= 1u << ps;
    }
    wave_sync_lds();
    const cx<T> piv = ms.prow[K];
    if (lane == 0 && !(cabs1(piv) > T(0))) *flag = 1;
    const cx<T> ipiv = crcp_scaled(piv);
    cx<T> m[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int r = lane + 64 * s;
      m[s] = (r == pk) ? mk<T>(T(1) - ipiv.re, -ipiv.im) : cmul(Pc[s][K], ipiv);
    }
    constexpr int KN = K + 1;
    int pkn = 0;
    if constexpr (KN < 16) {
      const cx<T> vn = ms.prow[KN];
#pragma unroll
      for (int s = 0; s < 2; ++s) Pc[s][KN] = cfms(m[s], vn, Pc[s][KN]);
      if (KN < ks) pkn = mgj_pivot<T, KN>(Pc, n, used);
    }
    // the other columns in chunks of four pivot-row entries (read from LDS
    // per chunk: register pressure)
#pragma unroll
    for (int j0 = 0; j0 < 16; j0 += 4) {
      cx<T> v[4];
#pragma unroll
      for (int g = 0; g < 4; ++g) v[g] = ms.prow[j0 + g];
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int j = j0 + g;
        if (j == KN) continue;
        cx<T> x = v[g];
        if (j == K) x.re += T(1);
#pragma unroll
        for (int s = 0; s < 2; ++s) Pc[s][j] = cfms(m[s], x, Pc[s][j]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    wave_sync_lds();  // prow is rewritten by the next step
    mgj_step<T, KN>(Pc, p, ks, n, pkn, used, ms, flag);
  }
}

// Owner wave of panel p: eliminate the panel (its tile column, up to date
// with every earlier panel), publish Z, the pivot rows and their panel
// index, and keep Z as its tiles.
template <typename T>
__device__ __forceinline__ void mgj_factor(MgjTile<T>& D, int p, int n, MgjSmem<T>& ms,
                                           int* flag) {
  const int lane = mgj_lane(), li = lane & 15, lk = lane >> 4;
  const int buf = p & 1;
  const int ks = min(16, n - 16 * p);
  cx<T>(*zb)[MG_ZLD] = ms.zbuf[buf];
#pragma unroll
  for (int I = 0; I < MG_TI; ++I)
#pragma unroll
    for (int v = 0; v < 4; ++v) zb[li][16 * I + mgj_row<T>(v, lk)] = mgj_get(D, I, v);
  ms.pidx[buf][lane] = -1;
  ms.pidx[buf][lane + 64] = -1;
  wave_sync_lds();
  cx<T> Pc[2][16];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int j = 0; j < 16; ++j) Pc[s][j] = zb[j][lane + 64 * s];
  uint32_t used = (ms.used[lane] ? 1u : 0u) | (ms.used[lane + 64] ? 2u : 0u);
  wave_sync_lds();
  const int pk0 = (ks > 0) ? mgj_pivot<T, 0>(Pc, n, used) : 0;
  mgj_step<T, 0>(Pc, p, ks, n, pk0, used, ms, flag);
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int j = 0; j < 16; ++j) zb[j][lane + 64 * s] = Pc[s][j];
  wave_sync_lds();
#pragma unroll
  for (int I = 0; I < MG_TI; ++I)
#pragma unroll
    for (int v = 0; v < 4; ++v) mgj_set(D, I, v, zb[li][16 * I + mgj_row<T>(v, lk)]);
}

// Every other wave: v <- v + (Z - E_P) v_P for its tile column, on the
// matrix cores (k = the panel's up to 16 steps).
template <typename T>
__device__ __forceinline__ void mgj_update(MgjTile<T>& D, int p, int n, MgjSmem<T>& ms) {
  const int lane = mgj_lane(), w = wave_id(), li = lane & 15, lk = lane >> 4;
  const int buf = p & 1;
  const int ks = min(16, n - 16 * p);
  cx<T>(*vp)[16] = ms.vp[w];
  // this wave's entries in the panel's pivot rows (read before the update)
#pragma unroll
  for (int I = 0; I < MG_TI; ++I)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = ms.pidx[buf][16 * I + mgj_row<T>(v, lk)];
      if (j >= 0) vp[j][li] = mgj_get(D, I, v);
    }
  wave_sync_lds();
  const cx<T>(*zb)[MG_ZLD] = ms.zbuf[buf];
  const int* piv = ms.pivrow + 16 * p;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (4 * q >= ks) break;
    const int k = 4 * q + lk;
    const bool kok = k < ks;
    const cx<T> b = kok ? vp[k][li] : mk<T>(T(0), T(0));
    const int pr = kok ? piv[k] : -1;
#pragma unroll
    for (int I = 0; I < MG_TI; ++I) {
      cx<T> a = kok ? zb[k][16 * I + li] : mk<T>(T(0), T(0));
      if (16 * I + li == pr) a.re -= T(1);
      D.re[I] = mgj_mfma(a.re, b.re, D.re[I]);
      D.im[I] = mgj_mfma(a.re, b.im, D.im[I]);
      D.re[I] = mgj_mfma(-a.im, b.im, D.re[I]);
      D.im[I] = mgj_mfma(a.im, b.re, D.im[I]);
    }
    // bound the operand loads in flight to one k-step (register pressure:
    // the tile itself takes 32 complex entries per lane)
    __builtin_amdgcn_sched_barrier(0);
  }
  wave_sync_lds();  // vp is rewritten by this wave's next update
}

// Invert the n x n matrix held in D (padded to 128 with the identity,
// scaled to entries below 1). Leaves the permuted inverse in D and the
// pivot order in ms.pivrow / ms.pinv; sets *flag (LDS) to 1 on an exact zero
// pivot (the caller clears it per tuple). Ends on a workgroup barrier.
template <typename T>
__device__ __forceinline__ void mgj_invert(MgjTile<T>& D, int n, MgjSmem<T>& ms, int* flag) {
  const int w = wave_id();
  const int npan = (n + 15) >> 4;
  for (int i = threadIdx.x; i < MG_NP; i += MG_NW * 64) ms.used[i] = 0;
  __syncthreads();
  if (w == 0 && npan > 0) mgj_factor(D, 0, n, ms, flag);
  __syncthreads();
  for (int p = 0; p < npan; ++p) {
    // the owner of the next panel is on the critical path: its own update
    // and its elimination run at raised wave priority
    const bool ahead = (w == p + 1 && w < npan);
    if (ahead) __builtin_amdgcn_s_setprio(3);
    if (w != p && 16 * w < n) mgj_update(D, p, n, ms);
    if (ahead) {
      mgj_factor(D, p + 1, n, ms, flag);
      __builtin_amdgcn_s_setprio(0);
    }
    __syncthreads();
  }
  // identity first, so that every entry of pinv stays a valid row index
  for (int i = threadIdx.x; i < MG_NP; i += MG_NW * 64) ms.pinv[i] = i;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += MG_NW * 64) ms.pinv[ms.pivrow[i]] = i;
  __syncthreads();
}

// Largest |re| + |im| of the tile over the workgroup (one barrier); every
// thread gets it.
template <typename T>
__device__ __forceinline__ double mgj_absmax(const MgjTile<T>& D, MgjSmem<T>& ms) {
  uint32_t b = 0u;
#pragma unroll
  for (int I = 0; I < MG_TI; ++I)
#pragma unroll
    for (int v = 0; v < 4; ++v) b = max(b, mag_hi(cabs1(mgj_get(D, I, v))));
  b = wave_max_u32(b);
  if (lane_id() == 0) ms.red[wave_id()] = b;
  __syncthreads();
  uint32_t m = ms.red[0];
#pragma unroll
  for (int i = 1; i < MG_NW; ++i) m = max(m, ms.red[i]);
  __syncthreads();  // red is reused by the next call
  if constexpr (sizeof(T) == sizeof(double))
    return __longlong_as_double((long long)((uint64_t)m << 32));
  else
    return (double)__uint_as_float(m);
}

// 2^-e with the largest |re| + |im| in [2^(e-1), 2^e), so the scaled
// entries lie below 1 (1 for a zero or non-finite maximum).
__device__ __forceinline__ double mgj_pow2_scale(double mx, int emin) {
  if (!(mx > 0.0) || !isfinite(mx)) return 1.0;
  int ex = 0;
  (void)frexp(mx, &ex);
  return ldexp(1.0, max(-ex, emin));
}

template <typename T>
__device__ __forceinline__ void mgj_scale(MgjTile<T>& D, T f) {
#pragma unroll
  for (int I = 0; I < MG_TI; ++I) {
    D.re[I] *= f;
    D.im[I] *= f;
  }
}

// K[i][j] = f X[p_i][q_j] for i, j < n (column-major, leading dimension
// MG_NP; K2 as well if non-null): entry (r, c) of the tile goes to row
// pinv[r], column pivrow[c].
template <typename T, typename TG>
__device__ __forceinline__ void mgj_store(const MgjTile<T>& D, int n, double f,
                                          const MgjSmem<T>& ms, cx<TG>* K, cx<TG>* K2) {
  const int lane = mgj_lane(), w = wave_id(), li = lane & 15, lk = lane >> 4;
  const int c = 16 * w + li;
  if (c >= n) return;
  K = opaque_uniform(K);
  if (K2) K2 = opaque_uniform(K2);
  const size_t col = (size_t)ms.pivrow[c] * MG_NP;
#pragma unroll
  for (int I = 0; I < MG_TI; ++I)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * I + mgj_row<T>(v, lk);
      if (r < n) {
        const cx<T> x = mgj_get(D, I, v);
        const cx<TG> g = mk<TG>((TG)(x.re * f), (TG)(x.im * f));
        const size_t o = col + ms.pinv[r];
        stg(K + o, g);
        if (K2) stg(K2 + o, g);
      }
    }
}

}  // namespace rgf
