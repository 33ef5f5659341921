// rgf_large.hip -- the forward sweep for half-slices wider than one
// workgroup's register tile: 128 < n <= 256 (256 < N <= 512), FP64.
//
// The recursion is the one of rgf_sweep.hpp (Eqs. (4)-(5) on the half-slice
// chain); only the inversion of M_h changes. An n = 240 complex128 matrix
// (921 KB) exceeds one compute unit's registers and LDS, so M_h lives in the
// workspace and is inverted by Gauss-Jordan in column panels of width
// b = 64, keeping partial pivoting over the full height:
//
//   * the panel (all n rows x b columns, already transformed by the earlier
//     panels) is loaded into registers (lane l: rows l + 64 s, s < 4; wave
//     w: columns 8 w .. 8 w + 7) and eliminated in place there, the pivot of
//     each column chosen among all rows not yet used by any panel;
//   * the b steps act on every other column v as one linear map,
//     v <- v + W v_P, with P the panel's pivot rows and W = Z - E_P (Z the
//     panel after elimination, E_P the unit columns of its pivot rows), so
//     the other n - b columns take one rank-b update on the matrix cores
//     (the pivot rows are staged first: the update rewrites them);
//   * after the last panel the array holds the inverse with its rows and
//     columns permuted by the pivot order, as in the in-register version,
//     and is written out un-permuted.
//
// Pivoting across the whole height matters: a 2 x 2 block (Schur
// complement) inversion without it is unstable here. The principal blocks
// of M_h are nonsingular (Im M_h is positive definite) but can be
// arbitrarily ill-conditioned when eta is small, e.g. for evanescent modes
// inside a subband gap.
//
// Workspace per persistent workgroup, complex128, leading dimension LD = 256
// (column-major): K (g_h), G1 ping-pong x 2, X (the matrix being inverted),
// Y (trace scratch), and Xp (the staged pivot rows, b x LD row-major); the
// gradient kernel adds a second K, S, and Z, Q ping-pong pairs, plus the
// restart states and the segment buffer. g_h is complex symmetric, so it is
// read in whichever order is contiguous.

#include <string.h>

#include "rgf_sweep.hpp"

namespace rgf {

namespace {

constexpr int LD = kLargeLd;               // leading dimension of the full matrices
constexpr int BW = 8, BS = 4, BC = 8;      // panel register tile: 256 rows x 64 columns
constexpr int NR = 64 * BS, PB = BW * BC;  // rows held, panel width
constexpr int BP = kTileMaxRows;           // output block of the GEMM calls
static_assert(NR == LD && 2 * BP == LD, "panel height and GEMM blocks");
constexpr size_t FULL = (size_t)LD * LD;   // complex elements of one full matrix
constexpr int kSlotBlocks = 5 * 4 + 1;     // K, G1 x 2, X, Y (4 blocks each); Xp
constexpr int kGradSlotBlocks = 11 * 4 + 1;  // K x 2, G1 x 2, X, Y, S, Z x 2, Q x 2; Xp
static_assert(PB * LD <= BP * BP, "the staged pivot rows fit one block");
// Whole-slice matrices (the accuracy fallback) of up to NRMAX rows: panels
// of 512 rows x 32 columns for N > 256.
constexpr int NRMAX = 2 * LD;
constexpr int WS = 8, WC = 4;              // panel register tile for 512 rows
static_assert(64 * WS == NRMAX && BW * WC * NRMAX <= BP * BP, "whole-slice panel tile");

struct LargeSmem {
  cx<double> colbuf[2 * (NRMAX + 1)];  // pivot column and 1/pivot, double-buffered
  int pivrow[NRMAX];                   // pivot row of each elimination step
  int pinv[NRMAX];
  double red[2 * BW];
  double rowacc[NR];                // gradient row sums of the reverse sweep
  double ksum;                      // sum of the inversions' kappa over the forward sweep
  double ksum_c;                    // the same over the sublattice-symmetric half-slices
  int flag;
};

// ---------------------------------------------------------------- panel GJ
// The elimination step of rgf_engine.hpp on a tall panel: RS slots of 64
// rows (NRT = 64 RS rows held), BW*RC columns, steps 0..nsteps-1 of the
// panel (the caller passes the panel's slice of the pivot list), pivot
// candidates the rows r < n not yet used.

// Pivot key for up to NRT rows: the magnitude as a float with its low bits
// replaced by NRT - 1 - r (8 bits for 256 rows, 9 for 512), so the largest
// key is the largest magnitude (to 2^-15 or 2^-14 relative) and ties go to
// the lowest row; unusable rows get 0.
template <int NRT>
__device__ __forceinline__ uint32_t pivot_key_rows(cx<double> v, int r, bool usable) {
  constexpr uint32_t MASK = NRT <= 256 ? 0xFFu : 0x1FFu;
  static_assert(NRT <= 512, "row index field");
  if (!usable) return 0u;
  float m = (float)cabs1(v);
  if (!(m >= 0.0f)) m = 0.0f;
  return (__float_as_uint(m) & ~MASK) | (uint32_t)(NRT - 1 - r);
}

// A[s][J] for a uniform-per-lane slot s: one branch per slot, kept apart
// by a distinct empty asm statement, so the tile is never indexed
// dynamically (a select chain over four slots is folded into a dynamic
// index, which moves the whole tile to scratch memory).
template <int RS, int RC, int J, int SS = 0>
__device__ __forceinline__ cx<double> pick_slot_br(const cx<double> (&A)[RS][RC], int s) {
  if constexpr (SS + 1 < RS) {
    if (s == SS) {
      asm volatile("; pick slot %0" ::"n"(SS));
      return A[SS][J];
    }
    return pick_slot_br<RS, RC, J, SS + 1>(A, s);
  } else {
    return A[SS][J];
  }
}

template <int RS, int RC, int J>
__device__ __forceinline__ void pgj_select_pivot(const cx<double> (&A)[RS][RC], int kc, int n,
                                                 uint32_t used, cx<double>* colbuf, int* pivrow,
                                                 int* flag) {
  constexpr int NRT = 64 * RS;
  constexpr uint32_t MASK = NRT <= 256 ? 0xFFu : 0x1FFu;
  const int lane = lane_id();
  cx<double>* cb = colbuf + (kc & 1) * (NRT + 1);
  uint32_t key = 0u;
#pragma unroll
  for (int s = 0; s < RS; ++s) {
    const int r = lane + 64 * s;
    cb[r] = A[s][J];
    key = max(key, pivot_key_rows<NRT>(A[s][J], r, r < n && !((used >> s) & 1u)));
  }
  key = wave_max_u32(key);
  const int pk = NRT - 1 - (int)(key & MASK);
  if (lane == (pk & 63)) {
    const cx<double> pv = pick_slot_br<RS, RC, J>(A, pk >> 6);
    pivrow[kc] = pk;
    cb[NRT] = crcp_scaled(pv);
    if (!(cabs1(pv) > 0.0)) *flag = 1;
  }
}

template <int RS, int RC, int J>
__device__ __forceinline__ void pgj_step(cx<double> (&A)[RS][RC], int kb, int nsteps, int n,
                                         uint32_t& used, cx<double>* colbuf, int* pivrow,
                                         int* flag) {
  constexpr int NRT = 64 * RS;
  constexpr int JN = (J + 1) % RC;
  const int lane = lane_id(), w = wave_id();
  const int k = kb * RC + J;
  const int kbn = (J + 1 == RC) ? kb + 1 : kb;
  __syncthreads();
  const cx<double>* cb = colbuf + (k & 1) * (NRT + 1);
  const int pkr = pivrow[k];
  const cx<double> ipiv = cb[NRT];
  cx<double> a[RS];
#pragma unroll
  for (int s = 0; s < RS; ++s) a[s] = cb[lane + 64 * s];
  __builtin_amdgcn_sched_barrier(0);
  const int pk = __builtin_amdgcn_readfirstlane(min(max(pkr, 0), NRT - 1));
  const int pl = pk & 63, ps = pk >> 6;
  cx<double> m[RS];
#pragma unroll
  for (int s = 0; s < RS; ++s) {
    const int r = lane + 64 * s;
    m[s] = (r == pk) ? mk(1.0 - ipiv.re, -ipiv.im) : cmul(a[s], ipiv);
  }
  if (lane == pl) used |= 1u << ps;
  const bool own = (w == kb);
  const bool la = (w == kbn && k + 1 < nsteps);  // the look-ahead wave issues first
  if (la) __builtin_amdgcn_s_setprio(2);
  {
    cx<double> v1[1];
    gj_row_chunk<double, RS, RC, JN, 1, -1, 0>(A, ps, pl, v1);
    gj_update_column<double, RS, RC, JN>(A, m, v1[0]);
  }
  if (la) {
    pgj_select_pivot<RS, RC, JN>(A, k + 1, n, used, colbuf, pivrow, flag);
    __builtin_amdgcn_s_setprio(0);
  }
  gj_update_chunks<double, RS, RC, J, JN, 0>(A, m, ps, pl, own);
}

template <int RS, int RC, int J>
__device__ __forceinline__ void pgj_block(cx<double> (&A)[RS][RC], int kb, int nsteps, int n,
                                          uint32_t& used, cx<double>* colbuf, int* pivrow,
                                          int* flag) {
  if constexpr (J < RC) {
    if (kb * RC + J >= nsteps) return;
    pgj_step<RS, RC, J>(A, kb, nsteps, n, used, colbuf, pivrow, flag);
    pgj_block<RS, RC, J + 1>(A, kb, nsteps, n, used, colbuf, pivrow, flag);
  }
}

template <int RS, int RC>
__device__ __forceinline__ void pgj_panel(cx<double> (&A)[RS][RC], int nsteps, int n,
                                          uint32_t& used, LargeSmem& sm, int c0) {
  int* pivrow = sm.pivrow + c0;
  if (nsteps > 0 && wave_id() == 0)
    pgj_select_pivot<RS, RC, 0>(A, 0, n, used, sm.colbuf, pivrow, &sm.flag);
  for (int kb = 0; kb < BW; ++kb) {
    if (kb * RC >= nsteps) break;
    pgj_block<RS, RC, 0>(A, kb, nsteps, n, used, sm.colbuf, pivrow, &sm.flag);
  }
  __syncthreads();
}

// ---------------------------------------------------------------- sweep

// M_h (n x n) into X, column-major; returns the largest |re| + |im| of the
// thread's entries (NaN if any is NaN) and, in dmax, the largest
// |E - eps_{h,k}| of the thread's diagonal entries (for the accuracy guard;
// vacancies left out).
__device__ __forceinline__ double build_M_large(const SweepArgs& a, const Tuple& q, int h,
                                                const cx<double>* K, cx<double>* X,
                                                double& dmax) {
  const int e = half_parity(h, a.parity);
  const int n = half_size(a.N, e);
  const int nL = half_size(a.N, e ^ 1);
  const bool rhalf = (h & 1) != 0;
  const double mt2 = -(a.t * a.t);
  const double* eps = q.eps_r ? q.eps_r + (int64_t)(h >> 1) * a.N : nullptr;
  const double* ph = (h == 0) ? a.phi : (h == 2 * a.L - 1) ? a.phi + (size_t)a.P * LD : nullptr;
  double mx = 0.0;
  dmax = 0.0;
  for (int i = threadIdx.x; i < n * n; i += BW * 64) {
    const int c = i / n, r = i - c * n;
    cx<double> v = mk(0.0, 0.0);
    if (h > 0) {
      if (!rhalf) {
        v = cscale(ldg(K + (size_t)c * LD + r), mt2);
      } else {
        const int r0 = nb_lo(r, e), r1 = nb_hi(r, e), c0 = nb_lo(c, e), c1 = nb_hi(c, e);
        cx<double> acc = mk(0.0, 0.0);
        if (c0 >= 0) {
          if (r0 >= 0) acc = cadd(acc, ldg(K + (size_t)c0 * LD + r0));
          if (r1 < nL) acc = cadd(acc, ldg(K + (size_t)c0 * LD + r1));
        }
        if (c1 < nL) {
          if (r0 >= 0) acc = cadd(acc, ldg(K + (size_t)c1 * LD + r0));
          if (r1 < nL) acc = cadd(acc, ldg(K + (size_t)c1 * LD + r1));
        }
        v = cscale(acc, mt2);
      }
    }
    if (r == c) {
      const double d = q.z.re - (eps ? eps[half_row(r, e)] : 0.0);
      if (!isinf(d)) dmax = fmax(dmax, fabs(d));  // vacancies left out
      v = cadd(v, mk(d, q.z.im));
    }
    if (ph) {  // lead self-energy on the first and the last half-slice
      for (int p = 0; p < a.P; ++p) {
        const double f = ph[(size_t)p * LD + r] * ph[(size_t)p * LD + c];
        v.re = fma(-f, q.sig[p].re, v.re);
        v.im = fma(-f, q.sig[p].im, v.im);
      }
    }
    // a vacancy's row and column are the identity's
    if (eps && (is_vacancy(eps[half_row(r, e)]) || is_vacancy(eps[half_row(c, e)])))
      v = mk((r == c) ? 1.0 : 0.0, 0.0);
    const double m1 = cabs1(v);
    mx = (m1 > mx || m1 != m1) ? m1 : mx;
    stg(X + (size_t)c * LD + r, v);
  }
  return mx;
}

// 2^-e with mx in [2^(e-1), 2^e) (1 for a zero or non-finite maximum).
__device__ __forceinline__ double pow2_scale(double mx) {
  if (!(mx > 0.0) || !isfinite(mx)) return 1.0;
  int ex = 0;
  (void)frexp(mx, &ex);
  return ldexp(1.0, min(-ex, 1022));
}

// g = M^{-1} (M in X, n x n, n <= 64 RS, leading dimension LDX) into K
// (same leading dimension) by the panel Gauss-Jordan; f is the power-of-two
// scale applied to M for the elimination. Returns (in every thread) kappa =
// max |(f M)^{-1}|, the condition estimate of the accuracy guard.
// veps (optional): on-site energies of the rows, row r at veps[vstride r +
// voff]; the diagonal entry of g at a vacancy (whose row and column of M are
// the identity's) is stored as 0, the removed site's Green's function.
template <int RS, int RC, int LDX>
__device__ __forceinline__ double invert_panels(int n, double f, cx<double>* X, cx<double>* Xp,
                                                cx<double>* K, cx<double> (&A)[RS][RC],
                                                LargeSmem& sm, const double* veps = nullptr,
                                                int vstride = 1, int voff = 0) {
  constexpr int PBT = BW * RC;
  static_assert(64 * RS <= LDX && PBT * LDX <= BP * BP, "panel tile and staging buffer");
  const int lane = lane_id(), w = wave_id();
  uint32_t used = 0u;
  for (int c0 = 0; c0 < n; c0 += PBT) {
    const int bw = min(PBT, n - c0);
    const double fs = (c0 == 0) ? f : 1.0;  // the first panel applies the scale
    // load the panel (rows >= n and columns >= bw stay zero)
#pragma unroll
    for (int j = 0; j < RC; ++j) {
      const int c = w * RC + j;
#pragma unroll
      for (int s = 0; s < RS; ++s) {
        const int r = lane + 64 * s;
        A[s][j] = (r < n && c < bw) ? cscale(ldg(X + (size_t)(c0 + c) * LDX + r), fs)
                                    : mk(0.0, 0.0);
      }
    }
    pgj_panel<RS, RC>(A, bw, n, used, sm, c0);
    // the panel after elimination back to X
#pragma unroll
    for (int j = 0; j < RC; ++j) {
      const int c = w * RC + j;
      if (c >= bw) break;
#pragma unroll
      for (int s = 0; s < RS; ++s) {
        const int r = lane + 64 * s;
        if (r < n) stg(X + (size_t)(c0 + c) * LDX + r, A[s][j]);
      }
    }
    const int nother = n - bw;
    if (nother > 0) {
      // stage the pivot rows of the other columns: Xp[j][c] = fs * X[P_j][c]
      for (int i = threadIdx.x; i < bw * n; i += BW * 64) {
        const int j = i / n, c = i - j * n;
        if (c >= c0 && c < c0 + bw) continue;
        stg(Xp + (size_t)j * LDX + c, cscale(ldg(X + (size_t)c * LDX + sm.pivrow[c0 + j]), fs));
      }
      __syncthreads();
      // X[:, c] = fs * X[:, c] + (Z - E_P) Xp[:, c] for the columns outside the panel
      for (int q0 = 0; q0 < nother; q0 += BP) {
        const int nc = min(BP, nother - q0);
        for (int r0 = 0; r0 < n; r0 += BP) {
          const int nr = min(BP, n - r0);
          auto col = [&](int cc) {
            const int x = q0 + cc;
            return x < c0 ? x : x + bw;
          };
          auto fa = [&](int r, int j) -> cx<double> {
            cx<double> z = ldg(X + (size_t)(c0 + j) * LDX + r0 + r);
            if (r0 + r == sm.pivrow[c0 + j]) z.re -= 1.0;
            return z;
          };
          auto fb = [&](int j, int cc) -> cx<double> {
            return ldg(Xp + (size_t)j * LDX + col(cc));
          };
          auto epi = [&](int r, int cc, cx<double> v, bool ok) {
            if (!ok) return;
            cx<double>* p = X + (size_t)col(cc) * LDX + r0 + r;
            stg(p, cadd(cscale(ldg(p), fs), v));
          };
          gemm_mfma<BW, BP>(nr, nc, bw, fa, fb, epi);
        }
      }
    }
    __syncthreads();
  }
  // un-permute: g[i][j] = f * X[p_i][q_j]
  for (int i = threadIdx.x; i < n; i += BW * 64) sm.pinv[sm.pivrow[i]] = i;
  __syncthreads();
  double kap = 0.0;
  for (int i = threadIdx.x; i < n * n; i += BW * 64) {
    const int j = i / n, r = i - j * n;
    const cx<double> x = ldg(X + (size_t)sm.pinv[j] * LDX + sm.pivrow[r]);
    const double m1 = cabs1(x);
    kap = (m1 > kap || m1 != m1) ? m1 : kap;
    const bool vz = veps && r == j && is_vacancy(veps[(size_t)vstride * r + voff]);
    stg(K + (size_t)j * LDX + r, vz ? mk(0.0, 0.0) : cscale(x, f));
  }
  return block_max<BW>(kap, sm.red);
}

// One half-slice step: g_h from g_{h-1} (Kprev) into Kout and G1_h from
// G1_{h-1} (G1prev) into G1out (G1 buffers must differ, K may be the same
// buffer; at h = 0 neither input is read). X and Xp are the inversion's
// scratch.
__device__ __forceinline__ void large_step(const SweepArgs& a, const Tuple& q, int h,
                                           const cx<double>* Kprev, cx<double>* Kout,
                                           const cx<double>* G1prev, cx<double>* G1out,
                                           cx<double>* X, cx<double>* Xp,
                                           cx<double> (&A)[BS][BC], LargeSmem& sm) {
  const int e = half_parity(h, a.parity);
  const int n = half_size(a.N, e);
  const int n1 = half_size(a.N, half_parity(0, a.parity));
  double dmax;
  const double mx = block_max<BW>(build_M_large(a, q, h, Kprev, X, dmax), sm.red);
  dmax = block_max<BW>(dmax, sm.red);
  const double* veps = q.eps_r ? q.eps_r + (int64_t)(h >> 1) * a.N : nullptr;
  const double kap = invert_panels<BS, BC, LD>(n, pow2_scale(mx), X, Xp, Kout, A, sm, veps, 2, e);
  if (threadIdx.x == 0) {  // read after the next barrier
    sm.ksum += kap;
    if (dmax < kChiralWindow * fabs(a.t)) sm.ksum_c += kap;
  }
  if (h == 0) {
    for (int i = threadIdx.x; i < n * n; i += BW * 64) {
      const int c = i / n, r = i - c * n;
      stg(G1out + (size_t)c * LD + r, ldg(Kout + (size_t)c * LD + r));
    }
    __syncthreads();
    return;
  }
  // G1_h = (G1_{h-1} C_{h-1}) g_h in 128 x 128 output blocks
  const int nL = half_size(a.N, e ^ 1);
  const bool rhalf = (h & 1) != 0;
  const double t = a.t;
  for (int r0 = 0; r0 < n1; r0 += BP) {
    for (int c0 = 0; c0 < n; c0 += BP) {
      auto fa = [&](int r, int k) -> cx<double> {
        if (!rhalf) return cscale(ldg(G1prev + (size_t)k * LD + r0 + r), t);
        const int k0 = nb_lo(k, e), k1 = nb_hi(k, e);
        cx<double> acc = mk(0.0, 0.0);
        if (k0 >= 0) acc = ldg(G1prev + (size_t)k0 * LD + r0 + r);
        if (k1 < nL) acc = cadd(acc, ldg(G1prev + (size_t)k1 * LD + r0 + r));
        return cscale(acc, t);
      };
      auto fb = [&](int k, int c) -> cx<double> {
        return ldg(Kout + (size_t)k * LD + c0 + c);  // g[c0 + c][k] = g[k][c0 + c]
      };
      auto epi = [&](int r, int c, cx<double> v, bool ok) {
        if (ok) stg(G1out + (size_t)(c0 + c) * LD + r0 + r, v);
      };
      gemm_mfma<BW, BP>(min(BP, n1 - r0), min(BP, n - c0), n, fa, fb, epi);
    }
  }
  __syncthreads();
}

// T = sum_{p,q} d_p d_q |S_pq|^2 with S = Phi_L^T G Phi_R (G = G_{1L}, n1 x
// nlast), through Y = G Phi_R; S is also stored (column-major) when Sout is
// non-null, and the channel sums sum_q d_q |S_pq|^2 are left in
// sm.rowacc[p] when chan is set. Every thread returns T.
__device__ __forceinline__ double large_trace(const SweepArgs& a, const Tuple& q,
                                              const cx<double>* G, cx<double>* Y,
                                              cx<double>* Sout, LargeSmem& sm,
                                              bool chan = false) {
  const int H = 2 * a.L;
  const int n1 = half_size(a.N, half_parity(0, a.parity));
  const int nlast = half_size(a.N, half_parity(H - 1, a.parity));
  const int pld = a.phi_ld;
  const double* phiL = a.phi;
  const double* phiR = a.phi + (size_t)a.P * pld;
  for (int r0 = 0; r0 < n1; r0 += BP)
    for (int c0 = 0; c0 < a.P; c0 += BP) {
      auto fa = [&](int r, int k) -> cx<double> { return ldg(G + (size_t)k * LD + r0 + r); };
      auto fb = [&](int k, int c) -> cx<double> {
        return mk(phiR[(size_t)(c0 + c) * pld + k], 0.0);
      };
      auto epi = [&](int r, int c, cx<double> v, bool ok) {
        if (ok) stg(Y + (size_t)(c0 + c) * LD + r0 + r, v);
      };
      gemm_mfma<BW, BP>(min(BP, n1 - r0), min(BP, a.P - c0), nlast, fa, fb, epi);
    }
  if (chan)
    for (int i = threadIdx.x; i < NR; i += BW * 64) sm.rowacc[i] = 0.0;
  __syncthreads();
  double part = 0.0;
  for (int r0 = 0; r0 < a.P; r0 += BP)
    for (int c0 = 0; c0 < a.P; c0 += BP) {
      auto fa = [&](int r, int k) -> cx<double> {
        return mk(phiL[(size_t)(r0 + r) * pld + k], 0.0);
      };
      auto fb = [&](int k, int c) -> cx<double> { return ldg(Y + (size_t)(c0 + c) * LD + k); };
      auto epi = [&](int r, int c, cx<double> v, bool ok) {
        if (!ok) return;
        const double dp = -2.0 * q.sig[r0 + r].im, dq = -2.0 * q.sig[c0 + c].im;
        part += dp * dq * (v.re * v.re + v.im * v.im);
        if (Sout) stg(Sout + (size_t)(c0 + c) * LD + r0 + r, v);
        if (chan) atomicAdd(&sm.rowacc[r0 + r], dq * (v.re * v.re + v.im * v.im));
      };
      gemm_mfma<BW, BP>(min(BP, a.P - r0), min(BP, a.P - c0), n1, fa, fb, epi);
    }
  return block_sum<BW>(part, sm.red);
}

__device__ __forceinline__ int tuple_status(const SweepArgs& a, const Tuple& q, double T,
                                            const LargeSmem& sm) {
  int st = a.lstat[q.e];
  // the guard first: a rejected sweep may also show a zero pivot or a T out
  // of range (the whole-slice sweep, whose ksum stays 0, never rejects)
  if (st == RGF_TUPLE_OK && ill_conditioned(sm.ksum, sm.ksum_c)) st = RGF_TUPLE_ILL_CONDITIONED;
  if (st == RGF_TUPLE_OK && sm.flag) st = RGF_TUPLE_SINGULAR;
  if (st == RGF_TUPLE_OK && !isfinite(T)) st = RGF_TUPLE_NONFINITE;
  if (st == RGF_TUPLE_OK && !t_in_range(T, a.P)) st = RGF_TUPLE_OUT_OF_RANGE;
  return st;
}

// Forward sweep that stores the restart state (g_h, G1_h) after every
// `stride` half-slices into ck[1..] (the state at h = 0 is rebuilt from the
// leads). Leaves g_{H-1} in Kb[(H-1) & 1] and G1_{H-1} in G1b[(H-1) & 1].
__device__ __forceinline__ void large_forward_ckpt(const SweepArgs& a, const Tuple& q,
                                                   cx<double>* const (&Kb)[2],
                                                   cx<double>* const (&G1b)[2], cx<double>* X,
                                                   cx<double>* Xp, cx<double>* ck,
                                                   cx<double> (&A)[BS][BC], LargeSmem& sm) {
  const int H = 2 * a.L;
  for (int h = 0; h < H; ++h) {
    large_step(a, q, h, Kb[(h + 1) & 1], Kb[h & 1], G1b[(h + 1) & 1], G1b[h & 1], X, Xp, A, sm);
    if ((h + 1) % a.stride == 0 && h + 1 < H) {
      cx<double>* c = ck + (size_t)((h + 1) / a.stride) * 2 * FULL;
      for (size_t i = threadIdx.x; i < FULL; i += BW * 64) {
        stg(c + i, ldg(Kb[h & 1] + i));
        stg(c + FULL + i, ldg(G1b[h & 1] + i));
      }
      __syncthreads();
    }
  }
}

// Recompute (g_h, G1_h) for h0 <= h < h1 into the segment buffer sg (pairs
// of full matrices) from restart state sgi (from the leads for sgi = 0).
__device__ __forceinline__ void large_recompute(const SweepArgs& a, const Tuple& q, int sgi,
                                                int h0, int h1, const cx<double>* ck,
                                                cx<double>* sg, cx<double>* X, cx<double>* Xp,
                                                cx<double> (&A)[BS][BC], LargeSmem& sm) {
  for (int h = h0; h < h1; ++h) {
    const int j = h - h0;
    const cx<double>* Kp = (j == 0) ? ck + (size_t)sgi * 2 * FULL : sg + (size_t)(j - 1) * 2 * FULL;
    cx<double>* Ko = sg + (size_t)j * 2 * FULL;
    large_step(a, q, h, Kp, Ko, Kp + FULL, Ko + FULL, X, Xp, A, sm);
  }
}

__global__ __launch_bounds__(BW * 64, 2) void rgf_fwd_large_kernel(SweepArgs a) {
  __shared__ LargeSmem sm;
  cx<double>* slot = a.slots + (size_t)blockIdx.x * a.slot_mats * (BP * BP);
  cx<double>* K = slot;  // g_h in place: M_h is built from it before it is rewritten
  cx<double>* G1b[2] = {slot + FULL, slot + 2 * FULL};
  cx<double>* X = slot + 3 * FULL;
  cx<double>* Y = slot + 4 * FULL;
  cx<double>* Xp = slot + 5 * FULL;
  const int H = 2 * a.L;

  for (int64_t tau = blockIdx.x; tau < a.ntuples; tau += gridDim.x) {
    const Tuple q = make_tuple_(a, tau);
    if (threadIdx.x == 0) {
      sm.flag = 0;
      sm.ksum = 0.0;
      sm.ksum_c = 0.0;
    }
    __syncthreads();
    cx<double> A[BS][BC];
    for (int h = 0; h < H; ++h)
      large_step(a, q, h, K, K, G1b[(h + 1) & 1], G1b[h & 1], X, Xp, A, sm);
    const double T = large_trace(a, q, G1b[(H - 1) & 1], Y, nullptr, sm, a.tchan != nullptr);
    const int st = tuple_status(a, q, T, sm);
    if (threadIdx.x == 0) {
      a.T_out[tau] = (st == RGF_TUPLE_OK) ? T : __builtin_nan("");
      if (a.status) a.status[tau] = st;
      // the whole-slice sweep recomputes the tuples the guard rejected
      if (a.fb_flags) a.fb_flags[tau] = (st == RGF_TUPLE_ILL_CONDITIONED) ? 1 : 0;
    }
    if (a.tchan) {  // T_p = d_p sum_q d_q |S_pq|^2 (block_sum's barriers order rowacc)
      for (int p = threadIdx.x; p < a.P; p += BW * 64)
        a.tchan[tau * a.P + p] =
            (st == RGF_TUPLE_OK) ? -2.0 * q.sig[p].im * sm.rowacc[p] : __builtin_nan("");
    }
    __syncthreads();
  }
}

// Gradient of T with respect to every on-site energy: the reverse sweep of
// rgf_adjoint.hip (Dyson's equation, Eq. (3), cut between half-slices),
//   Z_h = g_h (C_h Z_{h+1}),  Q_h = G1_h^T + g_h (C_h Q_{h+1}),
//   dT/d eps_{h,a} = 2 Re sum_c Z_h[a][c] Q_h[a][c],
// with Z_last = g_last Phi_R (D S^dagger D) Phi_L^T, on workspace-resident
// matrices (Z and Q row-major, ping-pong: the blocked products read all of
// Z_{h+1} while writing Z_h). Restart states (g_h, G1_h) are stored every
// `stride` half-slices and each segment is recomputed before it is walked
// back.
__global__ __launch_bounds__(BW * 64, 2) void rgf_grad_large_kernel(SweepArgs a) {
  __shared__ LargeSmem sm;
  cx<double>* slot = a.slots + (size_t)blockIdx.x * a.slot_mats * (BP * BP);
  cx<double>* const Kb[2] = {slot, slot + FULL};
  cx<double>* const G1b[2] = {slot + 2 * FULL, slot + 3 * FULL};
  cx<double>* X = slot + 4 * FULL;
  cx<double>* Y = slot + 5 * FULL;
  cx<double>* Sb = slot + 6 * FULL;
  cx<double>* Zb[2] = {slot + 7 * FULL, slot + 8 * FULL};
  cx<double>* Qb[2] = {slot + 9 * FULL, slot + 10 * FULL};
  cx<double>* Xp = slot + 11 * FULL;
  cx<double>* ck = a.ckpt + (size_t)blockIdx.x * a.n_ckpt * 2 * FULL;
  cx<double>* sg = a.seg + (size_t)blockIdx.x * a.stride * 2 * FULL;
  const int H = 2 * a.L;
  const int n1 = half_size(a.N, half_parity(0, a.parity));
  const int nlast = half_size(a.N, half_parity(H - 1, a.parity));
  const double* phiL = a.phi;
  const double* phiR = a.phi + (size_t)a.P * LD;

  for (int64_t tau = blockIdx.x; tau < a.ntuples; tau += gridDim.x) {
    const Tuple q = make_tuple_(a, tau);
    if (threadIdx.x == 0) {
      sm.flag = 0;
      sm.ksum = 0.0;
      sm.ksum_c = 0.0;
    }
    __syncthreads();
    cx<double> A[BS][BC];

    large_forward_ckpt(a, q, Kb, G1b, X, Xp, ck, A, sm);
    const cx<double>* Klast = Kb[(H - 1) & 1];
    const double T = large_trace(a, q, G1b[(H - 1) & 1], Y, Sb, sm);
    const int st = tuple_status(a, q, T, sm);
    if (threadIdx.x == 0) {
      a.T_out[tau] = (st == RGF_TUPLE_OK) ? T : __builtin_nan("");
      if (a.status) a.status[tau] = st;
    }
    const double wt = a.dL_dT[tau];
    if (st != RGF_TUPLE_OK || wt == 0.0) {
      __syncthreads();
      continue;
    }

    // ---- Z_last = g_last Phi_R R Phi_L^T with R = D S^dagger D (R[k][p] =
    // d_k conj(S[p][k]) d_p): V = g_last Phi_R -> Y, V2 = V R -> X,
    // Z_last = V2 Phi_L^T -> Z (row-major)
    for (int r0 = 0; r0 < nlast; r0 += BP)
      for (int c0 = 0; c0 < a.P; c0 += BP) {
        auto fa = [&](int r, int k) -> cx<double> {
          return ldg(Klast + (size_t)k * LD + r0 + r);
        };
        auto fb = [&](int k, int c) -> cx<double> {
          return mk(phiR[(size_t)(c0 + c) * LD + k], 0.0);
        };
        auto epi = [&](int r, int c, cx<double> v, bool ok) {
          if (ok) stg(Y + (size_t)(c0 + c) * LD + r0 + r, v);
        };
        gemm_mfma<BW, BP>(min(BP, nlast - r0), min(BP, a.P - c0), nlast, fa, fb, epi);
      }
    __syncthreads();
    for (int r0 = 0; r0 < nlast; r0 += BP)
      for (int c0 = 0; c0 < a.P; c0 += BP) {
        auto fa = [&](int r, int k) -> cx<double> { return ldg(Y + (size_t)k * LD + r0 + r); };
        auto fb = [&](int k, int c) -> cx<double> {
          const cx<double> sv = ldg(Sb + (size_t)k * LD + c0 + c);  // S[c0 + c][k]
          const double f = 4.0 * q.sig[k].im * q.sig[c0 + c].im;    // d_k d_p
          return mk(f * sv.re, -f * sv.im);
        };
        auto epi = [&](int r, int c, cx<double> v, bool ok) {
          if (ok) stg(X + (size_t)(c0 + c) * LD + r0 + r, v);
        };
        gemm_mfma<BW, BP>(min(BP, nlast - r0), min(BP, a.P - c0), a.P, fa, fb, epi);
      }
    __syncthreads();
    int cz = 0;
    for (int r0 = 0; r0 < nlast; r0 += BP)
      for (int c0 = 0; c0 < n1; c0 += BP) {
        auto fa = [&](int r, int k) -> cx<double> { return ldg(X + (size_t)k * LD + r0 + r); };
        auto fb = [&](int k, int c) -> cx<double> {
          return mk(phiL[(size_t)k * LD + c0 + c], 0.0);
        };
        auto epi = [&](int r, int c, cx<double> v, bool ok) {
          if (ok) stg(Zb[0] + (size_t)(r0 + r) * LD + c0 + c, v);
        };
        gemm_mfma<BW, BP>(min(BP, nlast - r0), min(BP, n1 - c0), a.P, fa, fb, epi);
      }
    __syncthreads();

    // ---- backward over segments
    const int nseg = (H + a.stride - 1) / a.stride;
    for (int sgi = nseg - 1; sgi >= 0; --sgi) {
      const int h0 = sgi * a.stride;
      const int h1 = min(H, h0 + a.stride);
      large_recompute(a, q, sgi, h0, h1, ck, sg, X, Xp, A, sm);
      for (int h = h1 - 1; h >= h0; --h) {
        const cx<double>* gh = sg + (size_t)(h - h0) * 2 * FULL;
        const cx<double>* G1h = gh + FULL;
        const int e = half_parity(h, a.parity);
        const int n = half_size(a.N, e);
        for (int i = threadIdx.x; i < NR; i += BW * 64) sm.rowacc[i] = 0.0;
        __syncthreads();
        if (h < H - 1) {
          const int en = half_parity(h + 1, a.parity);
          const int nn = half_size(a.N, en);
          const double t = a.t;
          const cx<double>* Zo = Zb[cz];
          cx<double>* Zn = Zb[cz ^ 1];
          const cx<double>* Qo = Qb[cz];
          cx<double>* Qn = Qb[cz ^ 1];
          // (C_h X)[k][c]: h even (L_i -> R_i): t (X[k + 1 - eR][c] + X[k - eR][c]);
          //                h odd  (R_i -> L_{i+1}): t X[k][c]
          auto capply = [&](const cx<double>* Xm, int k, int c) -> cx<double> {
            if (h & 1) return cscale(ldg(Xm + (size_t)k * LD + c), t);
            const int b0 = k + 1 - en, b1 = k - en;
            cx<double> acc = mk(0.0, 0.0);
            if (b0 >= 0 && b0 < nn) acc = ldg(Xm + (size_t)b0 * LD + c);
            if (b1 >= 0 && b1 < nn) acc = cadd(acc, ldg(Xm + (size_t)b1 * LD + c));
            return cscale(acc, t);
          };
          for (int r0 = 0; r0 < n; r0 += BP)
            for (int c0 = 0; c0 < n1; c0 += BP) {
              auto fa = [&](int r, int k) -> cx<double> {
                return ldg(gh + (size_t)k * LD + r0 + r);
              };
              auto fb = [&](int k, int c) -> cx<double> { return capply(Zo, k, c0 + c); };
              auto epi = [&](int r, int c, cx<double> v, bool ok) {
                if (ok) stg(Zn + (size_t)(r0 + r) * LD + c0 + c, v);
              };
              gemm_mfma<BW, BP>(min(BP, n - r0), min(BP, n1 - c0), n, fa, fb, epi);
            }
          __syncthreads();
          for (int r0 = 0; r0 < n; r0 += BP)
            for (int c0 = 0; c0 < n1; c0 += BP) {
              auto fa = [&](int r, int k) -> cx<double> {
                return ldg(gh + (size_t)k * LD + r0 + r);
              };
              auto fb = [&](int k, int c) -> cx<double> { return capply(Qo, k, c0 + c); };
              auto epi = [&](int r, int c, cx<double> v, bool ok) {
                double part = 0.0;
                if (ok) {
                  const size_t o = (size_t)(r0 + r) * LD + c0 + c;
                  v = cadd(v, ldg(G1h + o));  // G1_h^T[r][c] = G1_h[c][r]
                  const cx<double> z = ldg(Zn + o);
                  part = z.re * v.re - z.im * v.im;
                  stg(Qn + o, v);
                }
                part += __shfl_xor(part, 1);
                part += __shfl_xor(part, 2);
                part += __shfl_xor(part, 4);
                part += __shfl_xor(part, 8);
                if ((lane_id() & 15) == 0 && r0 + r < n) atomicAdd(&sm.rowacc[r0 + r], part);
              };
              gemm_mfma<BW, BP>(min(BP, n - r0), min(BP, n1 - c0), n, fa, fb, epi);
            }
          cz ^= 1;
        } else {
          // last half-slice: Z = Z_last, Q = G1^T
          for (int i = threadIdx.x; i < n * n1; i += BW * 64) {
            const int r = i / n1, c = i - r * n1;
            const size_t o = (size_t)r * LD + c;
            const cx<double> v = ldg(G1h + o);
            const cx<double> z = ldg(Zb[cz] + o);
            stg(Qb[cz] + o, v);
            atomicAdd(&sm.rowacc[r], z.re * v.re - z.im * v.im);
          }
        }
        __syncthreads();
        if (threadIdx.x < n) {
          const int i = h >> 1;
          const int k = half_row(threadIdx.x, e);
          atomicAdd(a.dL_deps + (q.r * (int64_t)a.L + i) * a.N + k,
                    2.0 * wt * sm.rowacc[threadIdx.x]);
        }
        __syncthreads();
      }
    }
  }
}

// Local density of states -Im G_ss / pi of every site (rgf_ldos.hip's
// backward sweep of the diagonal blocks, Dyson's equation cut between
// half-slices):
//   F_{H-1} = g_{H-1},   F_h = g_h + g_h V,   V = (C_h F_{h+1} C_h^T) g_h,
// on workspace-resident matrices. V is formed from all of F_{h+1} before
// F_h overwrites it, so one F buffer serves (row-major; F and g symmetric).
__global__ __launch_bounds__(BW * 64, 2) void rgf_ldos_large_kernel(SweepArgs a) {
  constexpr double kInvPi = 0.31830988618379067154;
  __shared__ LargeSmem sm;
  cx<double>* slot = a.slots + (size_t)blockIdx.x * a.slot_mats * (BP * BP);
  cx<double>* const Kb[2] = {slot, slot + FULL};
  cx<double>* const G1b[2] = {slot + 2 * FULL, slot + 3 * FULL};
  cx<double>* X = slot + 4 * FULL;
  cx<double>* Y = slot + 5 * FULL;
  cx<double>* F = slot + 7 * FULL;
  cx<double>* V = slot + 9 * FULL;
  cx<double>* Xp = slot + 11 * FULL;
  cx<double>* ck = a.ckpt + (size_t)blockIdx.x * a.n_ckpt * 2 * FULL;
  cx<double>* sg = a.seg + (size_t)blockIdx.x * a.stride * 2 * FULL;
  const int H = 2 * a.L;

  for (int64_t tau = blockIdx.x; tau < a.ntuples; tau += gridDim.x) {
    const Tuple q = make_tuple_(a, tau);
    if (threadIdx.x == 0) {
      sm.flag = 0;
      sm.ksum = 0.0;
      sm.ksum_c = 0.0;
    }
    __syncthreads();
    cx<double> A[BS][BC];
    double* out = a.ldos + tau * (int64_t)a.L * a.N;  // [L][N] of this tuple

    large_forward_ckpt(a, q, Kb, G1b, X, Xp, ck, A, sm);
    const cx<double>* Klast = Kb[(H - 1) & 1];
    const double T = large_trace(a, q, G1b[(H - 1) & 1], Y, nullptr, sm);
    const int st = tuple_status(a, q, T, sm);
    if (threadIdx.x == 0) {
      if (a.T_out) a.T_out[tau] = (st == RGF_TUPLE_OK) ? T : __builtin_nan("");
      if (a.status) a.status[tau] = st;
    }
    if (st != RGF_TUPLE_OK) {
      for (int64_t i = threadIdx.x; i < (int64_t)a.L * a.N; i += BW * 64)
        out[i] = __builtin_nan("");
      __syncthreads();
      continue;
    }

    // ---- last half-slice: F = g_{H-1}
    {
      const int e = half_parity(H - 1, a.parity);
      const int n = half_size(a.N, e);
      for (int i = threadIdx.x; i < n * n; i += BW * 64) {
        const int r = i / n, c = i - r * n;
        stg(F + (size_t)r * LD + c, ldg(Klast + (size_t)r * LD + c));
      }
      if (threadIdx.x < n)
        out[(int64_t)((H - 1) >> 1) * a.N + half_row(threadIdx.x, e)] =
            -ldg(Klast + (size_t)threadIdx.x * LD + threadIdx.x).im * kInvPi;
      __syncthreads();
    }

    // ---- backward over segments
    const int nseg = (H + a.stride - 1) / a.stride;
    for (int sgi = nseg - 1; sgi >= 0; --sgi) {
      const int h0 = sgi * a.stride;
      const int h1 = min(H, h0 + a.stride);
      large_recompute(a, q, sgi, h0, h1, ck, sg, X, Xp, A, sm);
      for (int h = min(h1, H - 1) - 1; h >= h0; --h) {
        const cx<double>* gh = sg + (size_t)(h - h0) * 2 * FULL;
        const int e = half_parity(h, a.parity);
        const int n = half_size(a.N, e);
        const int en = half_parity(h + 1, a.parity);
        const int nn = half_size(a.N, en);
        const double t2 = a.t * a.t;
        const bool odd = (h & 1) != 0;
        // rows b of half-slice h+1 that row k of half-slice h bonds to:
        // h odd (R_i -> L_{i+1}): b = k; h even (L_i -> R_i): k + 1 - eR, k - eR
        auto nb0 = [&](int k) { return odd ? k : k + 1 - en; };
        auto nb1 = [&](int k) { return odd ? -1 : k - en; };
        // W[r][k] = t^2 sum_{b ~ r, b' ~ k} F[b][b']
        auto fa_w = [&](int r, int k) -> cx<double> {
          const int rb[2] = {nb0(r), nb1(r)};
          const int kb2[2] = {nb0(k), nb1(k)};
          cx<double> acc = mk(0.0, 0.0);
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            if (kb2[u] < 0 || kb2[u] >= nn) continue;
#pragma unroll
            for (int v = 0; v < 2; ++v) {
              if (rb[v] < 0 || rb[v] >= nn) continue;
              acc = cadd(acc, ldg(F + (size_t)kb2[u] * LD + rb[v]));
            }
          }
          return cscale(acc, t2);
        };
        for (int r0 = 0; r0 < n; r0 += BP)
          for (int c0 = 0; c0 < n; c0 += BP) {
            auto fa = [&](int r, int k) -> cx<double> { return fa_w(r0 + r, k); };
            auto fb = [&](int k, int c) -> cx<double> {
              return ldg(gh + (size_t)k * LD + c0 + c);
            };
            auto epi = [&](int r, int c, cx<double> v, bool ok) {
              if (ok) stg(V + (size_t)(r0 + r) * LD + c0 + c, v);
            };
            gemm_mfma<BW, BP>(min(BP, n - r0), min(BP, n - c0), n, fa, fb, epi);
          }
        __syncthreads();
        for (int r0 = 0; r0 < n; r0 += BP)
          for (int c0 = 0; c0 < n; c0 += BP) {
            auto fa = [&](int r, int k) -> cx<double> {
              return ldg(gh + (size_t)k * LD + r0 + r);
            };
            auto fb = [&](int k, int c) -> cx<double> {
              return ldg(V + (size_t)k * LD + c0 + c);
            };
            auto epi = [&](int r, int c, cx<double> v, bool ok) {
              if (!ok) return;
              const int rr = r0 + r, cc = c0 + c;
              v = cadd(v, ldg(gh + (size_t)rr * LD + cc));
              stg(F + (size_t)rr * LD + cc, v);
              if (rr == cc) out[(int64_t)(h >> 1) * a.N + half_row(rr, e)] = -v.im * kInvPi;
            };
            gemm_mfma<BW, BP>(min(BP, n - r0), min(BP, n - c0), n, fa, fb, epi);
          }
        __syncthreads();
      }
    }
  }
}


// ---------------------------------------------------------------- accuracy fallback
// The whole-slice form of the recursion (Eqs. (4)-(5) with the full N x N
// slice) for the tuples the half-slice guard rejected. The carried state is
// the same as on the half-slice chain -- g of the rows R_i that bond to the
// next slice and G1 = G_{1i} on (L_1, R_i) -- but each slice is inverted as
// a whole, with partial pivoting across both row classes:
//   M_i = z - H_i - t^2 g_{i-1} on L_i x L_i   (- Sigma_L at i = 1, - Sigma_R at i = L),
//   W = M_i^{-1},   g_i = W[R_i, R_i],   G1_i = t G1_{i-1} W[L_i, R_i]   (G1_1 = W[L_1, R_1]).
// The diagonal of M_i carries the intra-slice bonds, so no block divides by
// the bare z - eps of one sublattice. Costs about (8 + 1) N^3 flops per
// slice instead of 4 N^3; it runs only on flagged tuples.

// Entry (r, c) of M_i, r, c < N.
__device__ __forceinline__ cx<double> m_whole_entry(const SweepArgs& a, const Tuple& q, int i,
                                                    const cx<double>* K, int r, int c) {
  const int eL = half_parity(2 * (i - 1), a.parity);
  if (q.eps_r && (is_vacancy(q.eps_r[(int64_t)(i - 1) * a.N + r]) ||
                  is_vacancy(q.eps_r[(int64_t)(i - 1) * a.N + c])))
    return mk((r == c) ? 1.0 : 0.0, 0.0);  // a vacancy's row and column: the identity's
  cx<double> v = mk(0.0, 0.0);
  if (r == c) v = mk(q.z.re - (q.eps_r ? q.eps_r[(int64_t)(i - 1) * a.N + r] : 0.0), q.z.im);
  if (r == c + 1 || c == r + 1) v.re -= a.t;
  const bool rl = (r & 1) == eL, cl = (c & 1) == eL;
  // row k of a row class has local index k >> 1 (k = 2 a + parity of the class)
  if (rl && cl && i > 1)
    v = cadd(v, cscale(ldg(K + (size_t)(c >> 1) * LD + (r >> 1)), -(a.t * a.t)));
  const int pld = a.phi_ld;
  const double* ph = (rl && cl && i == 1)         ? a.phi
                     : (!rl && !cl && i == a.L) ? a.phi + (size_t)a.P * pld
                                                : nullptr;
  if (ph) {
    for (int p = 0; p < a.P; ++p) {
      const double f = ph[(size_t)p * pld + (r >> 1)] * ph[(size_t)p * pld + (c >> 1)];
      v.re = fma(-f, q.sig[p].re, v.re);
      v.im = fma(-f, q.sig[p].im, v.im);
    }
  }
  return v;
}

// M_i into X (column-major, leading dimension LDX); returns the thread's
// largest |re| + |im| (NaN if any entry is NaN).
template <int LDX>
__device__ __forceinline__ double build_M_whole(const SweepArgs& a, const Tuple& q, int i,
                                                const cx<double>* K, cx<double>* X) {
  const int N = a.N;
  double mx = 0.0;
  for (int idx = threadIdx.x; idx < N * N; idx += BW * 64) {
    const int c = idx / N, r = idx - c * N;
    const cx<double> v = m_whole_entry(a, q, i, K, r, c);
    const double m1 = cabs1(v);
    mx = (m1 > mx || m1 != m1) ? m1 : mx;
    stg(X + (size_t)c * LDX + r, v);
  }
  return mx;
}

// Complex elements of one workgroup's buffers: g and G1 x 2 at leading
// dimension LD (at most 256 rows), M_i and its inverse at LDX, the refined
// columns (LDX x LDX/2), staged rows.
template <int LDX>
constexpr size_t whole_slot_elems() {
  return 3 * FULL + 2 * (size_t)LDX * LDX + (size_t)LDX * (LDX / 2) + (size_t)BP * BP;
}

template <int RS, int RC, int LDX>
__global__ __launch_bounds__(BW * 64, 2) void rgf_whole_kernel(SweepArgs a) {
  __shared__ LargeSmem sm;
  constexpr size_t FX = (size_t)LDX * LDX;
  cx<double>* slot = a.slots + (size_t)blockIdx.x * whole_slot_elems<LDX>();
  cx<double>* K = slot;
  cx<double>* G1b[2] = {slot + FULL, slot + 2 * FULL};
  cx<double>* X = slot + 3 * FULL;
  cx<double>* W = X + FX;
  cx<double>* V = W + FX;            // refined columns R_i of M_i^{-1} (N x n_R, ld LDX)
  cx<double>* Xp = V + FX / 2;
  const int n1 = half_size(a.N, half_parity(0, a.parity));
  const int N = a.N;
  const double t = a.t;

  for (int64_t tau = blockIdx.x; tau < a.ntuples; tau += gridDim.x) {
    if (a.fb_flags[tau] == 0) continue;  // same word for every thread: uniform
    const Tuple q = make_tuple_(a, tau);
    if (threadIdx.x == 0) {
      sm.flag = 0;
      sm.ksum = 0.0;
      sm.ksum_c = 0.0;
    }
    __syncthreads();
    cx<double> A[RS][RC];
    int cur = 0;
    for (int i = 1; i <= a.L; ++i) {
      const double mx = block_max<BW>(build_M_whole<LDX>(a, q, i, K, X), sm.red);
      // ends on a barrier; vacancies get 0 on the diagonal of W, and the
      // Newton step below keeps their rows and columns of V at exactly 0
      (void)invert_panels<RS, RC, LDX>(N, pow2_scale(mx), X, Xp, W, A, sm,
                                       q.eps_r ? q.eps_r + (int64_t)(i - 1) * N : nullptr);
      const int eL = half_parity(2 * (i - 1), a.parity), eR = eL ^ 1;
      const int nLi = half_size(N, eL), nRi = half_size(N, eR);
      // One Newton step on the columns R_i of the inverse (Gauss-Jordan
      // alone loses digits when M_i mixes entries of very different size,
      // e.g. lead self-energies of nearly decoupled modes near E = 0):
      //   Res = E_R - M_i W[:, R_i] -> X,   V = W[:, R_i] + W Res.
      for (int r0 = 0; r0 < N; r0 += BP)
        for (int c0 = 0; c0 < nRi; c0 += BP) {
          auto fa = [&](int r, int k) -> cx<double> { return m_whole_entry(a, q, i, K, r0 + r, k); };
          auto fb = [&](int k, int c) -> cx<double> {
            return ldg(W + (size_t)(2 * (c0 + c) + eR) * LDX + k);
          };
          auto epi = [&](int r, int c, cx<double> v, bool ok) {
            if (!ok) return;
            const double one = (r0 + r == 2 * (c0 + c) + eR) ? 1.0 : 0.0;
            stg(X + (size_t)(c0 + c) * LDX + r0 + r, mk(one - v.re, -v.im));
          };
          gemm_mfma<BW, BP>(min(BP, N - r0), min(BP, nRi - c0), N, fa, fb, epi);
        }
      __syncthreads();
      for (int r0 = 0; r0 < N; r0 += BP)
        for (int c0 = 0; c0 < nRi; c0 += BP) {
          auto fa = [&](int r, int k) -> cx<double> { return ldg(W + (size_t)k * LDX + r0 + r); };
          auto fb = [&](int k, int c) -> cx<double> { return ldg(X + (size_t)(c0 + c) * LDX + k); };
          auto epi = [&](int r, int c, cx<double> v, bool ok) {
            if (!ok) return;
            const cx<double> w0 = ldg(W + (size_t)(2 * (c0 + c) + eR) * LDX + r0 + r);
            stg(V + (size_t)(c0 + c) * LDX + r0 + r, cadd(w0, v));
          };
          gemm_mfma<BW, BP>(min(BP, N - r0), min(BP, nRi - c0), N, fa, fb, epi);
        }
      __syncthreads();
      cx<double>* G1o = G1b[cur ^ 1];
      if (i == 1) {
        for (int idx = threadIdx.x; idx < n1 * nRi; idx += BW * 64) {
          const int c = idx / n1, r = idx - c * n1;
          stg(G1o + (size_t)c * LD + r, ldg(V + (size_t)c * LDX + 2 * r + eL));
        }
      } else {
        const cx<double>* G1i = G1b[cur];
        for (int r0 = 0; r0 < n1; r0 += BP)
          for (int c0 = 0; c0 < nRi; c0 += BP) {
            auto fa = [&](int r, int k) -> cx<double> {
              return cscale(ldg(G1i + (size_t)k * LD + r0 + r), t);
            };
            auto fb = [&](int k, int c) -> cx<double> {
              return ldg(V + (size_t)(c0 + c) * LDX + 2 * k + eL);
            };
            auto epi = [&](int r, int c, cx<double> v, bool ok) {
              if (ok) stg(G1o + (size_t)(c0 + c) * LD + r0 + r, v);
            };
            gemm_mfma<BW, BP>(min(BP, n1 - r0), min(BP, nRi - c0), nLi, fa, fb, epi);
          }
      }
      // g_i = V[R_i, :] -> K (K, read by the residual above, is free now)
      for (int idx = threadIdx.x; idx < nRi * nRi; idx += BW * 64) {
        const int c = idx / nRi, r = idx - c * nRi;
        stg(K + (size_t)c * LD + r, ldg(V + (size_t)c * LDX + 2 * r + eR));
      }
      __syncthreads();
      cur ^= 1;
    }
    const double T = large_trace(a, q, G1b[cur], X, nullptr, sm, a.tchan != nullptr);
    const int st = tuple_status(a, q, T, sm);
    if (threadIdx.x == 0) {
      a.T_out[tau] = (st == RGF_TUPLE_OK) ? T : __builtin_nan("");
      if (a.status) a.status[tau] = st;
    }
    if (a.tchan) {
      for (int p = threadIdx.x; p < a.P; p += BW * 64)
        a.tchan[tau * a.P + p] =
            (st == RGF_TUPLE_OK) ? -2.0 * q.sig[p].im * sm.rowacc[p] : __builtin_nan("");
    }
    __syncthreads();
  }
}

}  // namespace

const void* large_kernel_ptr(bool grad) {
  return grad ? (const void*)rgf_grad_large_kernel : (const void*)rgf_fwd_large_kernel;
}

TileCfg large_block_tile() { return TileCfg{-1, BW, BS, BC}; }

int large_slot_blocks(bool grad) { return grad ? kGradSlotBlocks : kSlotBlocks; }

static SweepArgs large_args(const Plan& p, const double* E, const double* eps, double* T_out,
                            int32_t* status_out, char* ws) {
  SweepArgs a;
  memset(&a, 0, sizeof(a));
  a.N = p.N;
  a.L = p.L;
  a.parity = p.parity;
  a.P = p.P;
  a.t = p.t;
  a.eta = p.eta;
  a.E = E;
  a.nE = p.nE;
  a.eps = eps;
  a.nreal = p.nreal;
  a.sigma = reinterpret_cast<const cx<double>*>(ws + p.off_sigma);
  a.phi = reinterpret_cast<const double*>(ws + p.off_phi);
  a.lstat = reinterpret_cast<const int32_t*>(ws + p.off_lstat);
  a.T_out = T_out;
  a.status = status_out;
  a.slots = reinterpret_cast<cx<double>*>(ws + p.off_slots);
  a.slot_mats = p.slot_mats;
  a.ntuples = p.ntuples;
  a.phi_ld = LD;
  return a;
}

hipError_t launch_forward_large(const Plan& p, const double* E, const double* eps,
                                double* T_out, int32_t* status_out, char* ws, hipStream_t s,
                                double* tchan) {
  if (p.ntuples == 0) return hipSuccess;
  hipError_t err = launch_lead(p, E, ws, s);
  if (err != hipSuccess) return err;
  SweepArgs a = large_args(p, E, eps, T_out, status_out, ws);
  a.tchan = tchan;
  a.fb_flags = p.fb_grid > 0 ? reinterpret_cast<int32_t*>(ws + p.off_flags) : nullptr;
  hipLaunchKernelGGL(rgf_fwd_large_kernel, dim3(p.grid), dim3(BW * 64), 0, s, a);
  err = hipGetLastError();
  if (err != hipSuccess || !a.fb_flags) return err;
  return launch_whole_fallback(p, a, ws, s);
}

hipError_t launch_grad_large(const Plan& p, const double* E, const double* eps,
                             const double* dL_dT, double* T_out, double* dL_deps,
                             int32_t* status_out, char* ws, hipStream_t s) {
  if (p.ntuples == 0) return hipSuccess;
  hipError_t err = launch_lead(p, E, ws, s);
  if (err != hipSuccess) return err;
  SweepArgs a = large_args(p, E, eps, T_out, status_out, ws);
  a.dL_dT = dL_dT;
  a.dL_deps = dL_deps;
  a.ckpt = reinterpret_cast<cx<double>*>(ws + p.off_ckpt);
  a.seg = reinterpret_cast<cx<double>*>(ws + p.off_seg);
  a.stride = (int)p.ckpt_stride;
  a.n_ckpt = (int)p.n_ckpt;
  hipLaunchKernelGGL(rgf_grad_large_kernel, dim3(p.grid), dim3(BW * 64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_ldos_large(const Plan& p, const double* E, const double* eps, double* ldos,
                             double* T_out, int32_t* status_out, char* ws, hipStream_t s) {
  if (p.ntuples == 0) return hipSuccess;
  hipError_t err = launch_lead(p, E, ws, s);
  if (err != hipSuccess) return err;
  SweepArgs a = large_args(p, E, eps, T_out, status_out, ws);
  a.ckpt = reinterpret_cast<cx<double>*>(ws + p.off_ckpt);
  a.seg = reinterpret_cast<cx<double>*>(ws + p.off_seg);
  a.stride = (int)p.ckpt_stride;
  a.n_ckpt = (int)p.n_ckpt;
  a.ldos = ldos;
  hipLaunchKernelGGL(rgf_ldos_large_kernel, dim3(p.grid), dim3(BW * 64), 0, s, a);
  return hipGetLastError();
}


size_t whole_slot_bytes(int N) {
  return 16 * (N <= LD ? whole_slot_elems<LD>() : whole_slot_elems<NRMAX>());
}

hipError_t launch_whole_fallback(const Plan& p, const SweepArgs& fwd, char* ws, hipStream_t s) {
  if (p.fb_grid <= 0 || p.ntuples == 0) return hipSuccess;
  SweepArgs a = fwd;
  a.slots = reinterpret_cast<cx<double>*>(ws + p.off_slots);  // the sweep's slots, now free
  if (p.N <= LD)
    hipLaunchKernelGGL((rgf_whole_kernel<BS, BC, LD>), dim3(p.fb_grid), dim3(BW * 64), 0, s, a);
  else
    hipLaunchKernelGGL((rgf_whole_kernel<WS, WC, NRMAX>), dim3(p.fb_grid), dim3(BW * 64), 0, s,
                       a);
  return hipGetLastError();
}

}  // namespace rgf
