// rgf_sweep.hpp -- one half-slice step of the recursion and the conductance
// trace, shared by the forward kernel and the adjoint kernel.
//
// Per half-slice h (Eq. (4)-(5) of the paper on the half-slice chain):
//   M_h  = z - diag(eps_h) - C_{h-1}^T g_{h-1} C_{h-1}   (- Sigma_L at h = 0,
//                                                         - Sigma_R at h = 2L-1)
//   g_h  = M_h^{-1}                                       (Gauss-Jordan, in registers)
//   G1_h = G1_{h-1} C_{h-1} g_h                            (GEMM, in registers)
// with C = t*I between R_{i-1} and L_i, and C = B_i (the t-weighted adjacency
// of the zigzag chain) between L_i and R_i, so C^T g C is t^2 g or a
// four-point stencil of g. G1 is the block of the left-connected Green's
// function between L_1 and the current half-slice; after the last half-slice
// it is the block G_{1L} of the full Green's function (Eq. (1)).
//
// Precision of the inversion (template TJ):
//   double                 FP64 Gauss-Jordan;
//   float, REFINE = false  FP32 Gauss-Jordan (single-precision study);
//   float, REFINE = true   FP32 Gauss-Jordan, then Newton steps in FP64,
//                          g <- g (2I - M g) with M regenerated in FP64, until
//                          the residual reaches rounding; half-slices whose
//                          FP32 start does not converge are redone in FP64.
// G1, the lead self-energies and the trace are FP64 in every mode.

#pragma once

#include "rgf_engine.hpp"
#include "rgf_internal.hpp"
#include "rgf_mfma.hpp"
#include "rgf_mgj.hpp"

namespace rgf {

constexpr int KC = 4;

struct SweepArgs {
  int N, L, parity, P;
  double t, eta;
  const double* E;
  int64_t nE;
  const double* eps;  // [nreal][L][N] or null
  int64_t nreal;
  const cx<double>* sigma;  // [nE][P]
  const double* phi;        // [2][P][NP]
  const int32_t* lstat;     // [nE]
  double* T_out;            // [nreal][nE]
  int32_t* status;          // [nreal][nE] or null
  cx<double>* slots;        // [grid][slot_mats][NP*NP]
  int slot_mats;
  int64_t ntuples;
  // adjoint only
  const double* dL_dT;      // [nreal][nE]
  double* dL_deps;          // [nreal][L][N]
  cx<double>* ckpt;         // [grid][n_ckpt][2][NP*NP]
  cx<double>* seg;          // [grid][stride][2][NP*NP]
  int stride, n_ckpt;
  // local density of states only
  double* ldos;             // [nreal][nE][L][N]
  // transmission per incoming lead channel, or null
  double* tchan;            // [nreal][nE][P]
  // tuples the half-slice recursion could not resolve accurately (1) and
  // that the whole-slice sweep recomputes, or null
  int32_t* fb_flags;        // [nreal][nE]
  int phi_ld;               // leading dimension of the lead mode tables
  // mixed mode: device counters of the refinement (refined half-slices,
  // Newton updates, FP64 re-inversions) that the forward kernels add to, or
  // null
  unsigned long long* refine_stats;
};

// Accuracy guard of the half-slice recursion. Each half-slice inversion
// contributes kappa_h = max|(f M_h)^{-1}| (f scales M_h to entries below 1,
// so kappa_h estimates the condition number in the max-entry norm).
// Cutting a slice between its two row classes leaves dangling bonds. When
// every on-site term of a half-slice lies within kChiralWindow |t| of E
// (pristine or nearly pristine rows: the sublattice-symmetric regime), their
// zero-energy states make the inverses grow like 1/E on a whole subspace at
// every step, and the rounding error of T reaches about 5e-3 u sum_h kappa_h
// (u = 2^-53); such half-slices add kappa_h to a separate sum. Isolated
// resonances of disordered rows raise kappa_h at a few steps only and cost
// far less accuracy (about 1e-4 u sum_h kappa_h measured). A tuple is handed
// to the whole-slice sweep (conductance) or flagged RGF_TUPLE_ILL_CONDITIONED
// (gradient, LDOS) when the sublattice-symmetric sum exceeds kIllCondChiral
// or the total exceeds kIllCondAll.
constexpr double kChiralWindow = 0.01;
constexpr double kIllCondChiral = 1e9;
constexpr double kIllCondAll = 1e11;

// True if a tuple's accumulated condition estimates reject it.
__device__ __forceinline__ bool ill_conditioned(double ksum_all, double ksum_chiral) {
  return !(ksum_all <= kIllCondAll) || !(ksum_chiral <= kIllCondChiral);
}

template <int NW, int S, int C>
struct SweepSmem {
  static constexpr int NP = NW * C;
  cx<double> colbuf[2 * (NP + 1)];  // column and 1/pivot, double-buffered; also cx<float>
  cx<double> wbuf[NW * NP];    // also used as cx<float>[2*NW*NP]
  cx<double> As[2 * KC * NP];
  cx<double> Bs[2 * KC * NP];
  int pivrow[NP];
  int pinv[NP];
  double red[NW * 2];
  double rowacc[NP];
  double kred[NW];   // per-wave kappa of the latest inversion
  double ksum;       // running sum of kappa_h over the forward sweep
  double ksum_c;     // the same over the sublattice-symmetric half-slices
  int flag;
  // refinement counts of this workgroup (thread 0): refined half-slices,
  // Newton updates, FP64 re-inversions; the forward kernels zero them at
  // their start and add them to SweepArgs::refine_stats at their end
  unsigned rf[3];
};

// Adds the workgroup's refinement counts to the device counters (thread 0).
template <typename Smem>
__device__ __forceinline__ void flush_refine_stats(const SweepArgs& a, const Smem& sm) {
  if (threadIdx.x == 0 && a.refine_stats) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
      if (sm.rf[i]) atomicAdd(a.refine_stats + i, (unsigned long long)sm.rf[i]);
  }
}

// Largest |re| + |im| of a register tile across the wave (from the high 32
// bits of the magnitudes, so it is a lower bound within 2^-20).
template <typename T, int S, int C>
__device__ __forceinline__ double tile_absmax_wave(const cx<T> (&A)[S][C]) {
  uint32_t b = 0u;
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int j = 0; j < C; ++j) b = max(b, mag_hi(cabs1(A[s][j])));
  b = wave_max_u32(b);
  if constexpr (sizeof(T) == sizeof(double))
    return __longlong_as_double((long long)((uint64_t)b << 32));
  else
    return (double)__uint_as_float(b);
}

// Eq. (2) for unitary scattering bounds T by the number of open channels,
// at most the P lead modes; a value outside [0, P] (beyond rounding) means
// the recursion lost its accuracy and the tuple is flagged.
__device__ __forceinline__ bool t_in_range(double T, int P) {
  return T >= -1e-6 && T <= (double)P + 1e-6;
}

// Per-tuple constants. hs, he: the first and the last half-slice of the
// sweep (0 and 2L - 1 for the whole chain; a segment's ends when the chain
// is solved in segments, whose coupling to the left is then left out). The
// mode-space self-energy Phi diag(sigma) Phi^T is added at both: from phi_s
// and phi_e, or, where these are null, from the lead tables (left lead at
// hs, right lead at he). g1: whether the sweep forms the running product G1.
struct Tuple {
  int64_t r, e, idx;
  cx<double> z;
  const cx<double>* sig;
  const double* eps_r;
  const double* phi_s;
  const double* phi_e;
  int hs, he;
  bool g1;
};

__device__ __forceinline__ Tuple make_tuple_(const SweepArgs& a, int64_t tau) {
  Tuple q;
  q.idx = tau;
  q.r = tau / a.nE;
  q.e = tau - q.r * a.nE;
  q.z = mk(a.E[q.e], a.eta);
  q.sig = a.sigma + q.e * a.P;
  q.eps_r = a.eps ? a.eps + q.r * (int64_t)a.L * a.N : nullptr;
  q.phi_s = q.phi_e = nullptr;
  q.hs = 0;
  q.he = 2 * a.L - 1;
  q.g1 = true;
  return q;
}

// A -= Phi diag(sigma) Phi^T on the n x n block (lead self-energy), as P
// rank-1 updates: phi[p][.] holds mode p on the interface rows.
template <typename T, int NW, int S, int C>
__device__ __forceinline__ void sub_mode_sum(cx<T> (&A)[S][C], const double* phi,
                                             const cx<double>* sig, int P, int n) {
  constexpr int NP = NW * C;
  const int lane = lane_id(), w = wave_id();
  phi = opaque_uniform(phi);
#pragma unroll 1
  for (int p = 0; p < P; ++p) {
    const double* ph = phi + (size_t)p * NP;
    const cx<double> sp = sig[p];
    double fr[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int r = lane + 64 * s;
      fr[s] = (r < n) ? ph[r] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int c = w * C + j;
      const double fc = (c < n) ? ph[c] : 0.0;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const double f = fr[s] * fc;
        A[s][j].re = (T)fma(-f, sp.re, (double)A[s][j].re);
        A[s][j].im = (T)fma(-f, sp.im, (double)A[s][j].im);
      }
    }
  }
}

// Assemble M_h into the register tile (padded with the identity).
//   L half (h even, h > hs): M = z - eps - t^2 K           (K = g of R_{i-1})
//   R half (h odd):         M = z - eps - t^2 B'^T K B'    (K = g of L_i)
// where (B'^T K B')[r][c] = sum of K over the neighbour rows of r and the
// neighbour columns of c; the column sums go through the wave's LDS scratch.
// Sums are formed in FP64 and rounded once to T.
// Returns (wave-uniform) the high word of max_k |E - eps_{h,k}| over the
// rows present, for the accuracy guard, with bit 31 set if the half-slice
// has a vacancy.
template <typename T, int NW, int S, int C>
__device__ __forceinline__ uint32_t build_M(cx<T> (&A)[S][C], const SweepArgs& a,
                                            const Tuple& q, int h, const cx<double>* K,
                                            cx<double>* wbuf) {
  constexpr int NP = NW * C;
  const int lane = lane_id(), w = wave_id();
  const bool rhalf = (h & 1) != 0;
  const int e = half_parity(h, a.parity);
  const int n = half_size(a.N, e);
  const int nL = half_size(a.N, e ^ 1);  // L half of the same slice (R half only)
  const double mt2 = -(a.t * a.t);
  const double* eps_slice = q.eps_r ? q.eps_r + (int64_t)(h >> 1) * a.N : nullptr;
  K = opaque_uniform(K);
  if (eps_slice) eps_slice = opaque_uniform(eps_slice);
  double dre[S];  // E - eps of the lane's rows: -inf at a vacancy (eps = +inf)
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int r = lane + 64 * s;
    dre[s] = (r < n) ? q.z.re - (eps_slice ? eps_slice[half_row(r, e)] : 0.0) : 1.0;
  }
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int c = w * C + j;
    if (!rhalf) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int r = lane + 64 * s;
        cx<double> v = mk(0.0, 0.0);
        if (h > q.hs && r < n && c < n) v = cscale(ldg(K + (size_t)c * NP + r), mt2);
        if (r == c) v = cadd(v, mk(dre[s], r < n ? q.z.im : 0.0));
        A[s][j] = mk<T>((T)v.re, (T)v.im);
      }
      if ((j & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    } else {
      const int c0 = nb_lo(c, e), c1 = nb_hi(c, e);
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int r = lane + 64 * s;
        cx<double> cs = mk(0.0, 0.0);
        if (c < n && r < nL) {
          if (c0 >= 0) cs = ldg(K + (size_t)c0 * NP + r);
          if (c1 < nL) cs = cadd(cs, ldg(K + (size_t)c1 * NP + r));
        }
        if (r < NP) wbuf[r] = cs;
      }
      wave_sync_lds();
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int r = lane + 64 * s;
        cx<double> v = mk(0.0, 0.0);
        if (r < n && c < n) {
          const int r0 = nb_lo(r, e), r1 = nb_hi(r, e);
          if (r0 >= 0) v = wbuf[r0];
          if (r1 < nL) v = cadd(v, wbuf[r1]);
          v = cscale(v, mt2);
        }
        if (r == c) v = cadd(v, mk(dre[s], r < n ? q.z.im : 0.0));
        A[s][j] = mk<T>((T)v.re, (T)v.im);
      }
      wave_sync_lds();
    }
  }
  if (h == q.hs) sub_mode_sum<T, NW, S, C>(A, q.phi_s ? q.phi_s : a.phi, q.sig, a.P, n);
  if (h == q.he)
    sub_mode_sum<T, NW, S, C>(A, q.phi_e ? q.phi_e : a.phi + (size_t)a.P * NP, q.sig, a.P, n);
  // vacancies: their rows and columns become the identity's, so the inverse
  // is that of the lattice without them (the caller zeroes their own
  // diagonal entries of the inverse)
  bool vl = false;
#pragma unroll
  for (int s = 0; s < S; ++s) vl = vl || isinf(dre[s]);
  const bool anyv = __builtin_amdgcn_ballot_w64(vl) != 0;
  if (anyv) {
    // the wave's vacant columns as a mask (bit j: column w C + j)
    const int cl = w * C + lane;
    const uint64_t cm = __builtin_amdgcn_ballot_w64(lane < C && cl < n &&
                                                    is_vacancy(eps_slice[half_row(cl, e)]));
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int c = w * C + j;
      const bool vc = ((cm >> j) & 1u) != 0u;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int r = lane + 64 * s;
        if (isinf(dre[s]) || vc) A[s][j] = mk<T>((r == c) ? T(1) : T(0), T(0));
      }
    }
  }
  uint32_t dk = 0u;
#pragma unroll
  for (int s = 0; s < S; ++s)
    if (lane + 64 * s < n && !isinf(dre[s])) dk = max(dk, mag_hi(fabs(dre[s])));
  // bit 31 (never set in the high word of a magnitude) flags a vacancy
  dk = wave_max_u32(dk);
  return anyv ? (dk | 0x80000000u) : dk;
}

// One entry of M_h in FP64 (for the refinement residual), r, c < NP.
template <int NP>
__device__ __forceinline__ cx<double> m_entry(const SweepArgs& a, const Tuple& q, int h,
                                              const cx<double>* K, int r, int c) {
  const int e = half_parity(h, a.parity);
  const int n = half_size(a.N, e);
  if (r >= n || c >= n) return mk((r == c) ? 1.0 : 0.0, 0.0);
  const double* eps_slice = q.eps_r ? q.eps_r + (int64_t)(h >> 1) * a.N : nullptr;
  if (eps_slice && (is_vacancy(eps_slice[half_row(r, e)]) || is_vacancy(eps_slice[half_row(c, e)])))
    return mk((r == c) ? 1.0 : 0.0, 0.0);  // vacancy: identity row and column
  cx<double> v = mk(0.0, 0.0);
  if (r == c) v = mk(q.z.re - (eps_slice ? eps_slice[half_row(r, e)] : 0.0), q.z.im);
  const double mt2 = -(a.t * a.t);
  if (!(h & 1)) {
    if (h > q.hs) v = cadd(v, cscale(ldg(K + (size_t)c * NP + r), mt2));
  } else {
    const int nL = half_size(a.N, e ^ 1);
    const int r0 = nb_lo(r, e), r1 = nb_hi(r, e), c0 = nb_lo(c, e), c1 = nb_hi(c, e);
    cx<double> acc = mk(0.0, 0.0);
    if (r0 >= 0 && c0 >= 0) acc = cadd(acc, ldg(K + (size_t)c0 * NP + r0));
    if (r0 >= 0 && c1 < nL) acc = cadd(acc, ldg(K + (size_t)c1 * NP + r0));
    if (r1 < nL && c0 >= 0) acc = cadd(acc, ldg(K + (size_t)c0 * NP + r1));
    if (r1 < nL && c1 < nL) acc = cadd(acc, ldg(K + (size_t)c1 * NP + r1));
    v = cadd(v, cscale(acc, mt2));
  }
  const double* phi = nullptr;
  if (h == q.hs) phi = q.phi_s ? q.phi_s : a.phi;
  if (h == q.he) phi = q.phi_e ? q.phi_e : a.phi + (size_t)a.P * NP;
  if (phi) {
    for (int p = 0; p < a.P; ++p) {
      const double f = phi[(size_t)p * NP + r] * phi[(size_t)p * NP + c];
      v.re = fma(-f, q.sig[p].re, v.re);
      v.im = fma(-f, q.sig[p].im, v.im);
    }
  }
  return v;
}

// Zeroes the diagonal entries of g_h (in K, and in K2 if non-null) at the
// vacant rows of half-slice h: M_h holds the identity's row and column
// there, so the inverse holds 1 where the removed site's Green's function
// is 0. Block-wide; the caller orders it between barriers.
template <int NP>
__device__ __forceinline__ void zero_vacant_diag(const SweepArgs& a, const Tuple& q, int h,
                                                 cx<double>* K, cx<double>* K2) {
  const int e = half_parity(h, a.parity);
  const int n = half_size(a.N, e);
  const double* eps_slice = q.eps_r + (int64_t)(h >> 1) * a.N;
  for (int r = threadIdx.x; r < n; r += blockDim.x)
    if (is_vacancy(eps_slice[half_row(r, e)])) {
      stg(K + (size_t)r * NP + r, mk(0.0, 0.0));
      if (K2) stg(K2 + (size_t)r * NP + r, mk(0.0, 0.0));
    }
}

// One half-slice step: reads g_{h-1} from Kprev and G1_{h-1} from G1, writes
// g_h to Kout and G1_h to G1 (in place). Kprev != Kout when REFINE (the
// residual regenerates M_h from Kprev after Kout holds the FP32 inverse);
// Rbuf (NP x NP) is the refinement scratch. A is the caller's FP64 register
// tile (reused as GEMM accumulator); AJ the inversion tile.
template <typename TJ, bool REFINE, int NW, int S, int C>
__device__ __forceinline__ void half_step(const SweepArgs& a, const Tuple& q, int h,
                                          const cx<double>* Kprev, cx<double>* Kout,
                                          const cx<double>* G1in, cx<double>* G1out,
                                          cx<double>* Rbuf, cx<double> (&A)[S][C],
                                          SweepSmem<NW, S, C>& sm) {
  constexpr int NP = NW * C;
  const int w = wave_id();
  const int e = half_parity(h, a.parity);
  const int n = half_size(a.N, e);
  const int n1 = half_size(a.N, half_parity(q.hs, a.parity));
  uint32_t dkey;  // high word of max_k |E - eps_{h,k}| | vacancy bit (wave-uniform)
  if constexpr (sizeof(TJ) == sizeof(double)) {
    dkey = build_M<double, NW, S, C>(A, a, q, h, Kprev, sm.wbuf + w * NP);
    const double f = tile_scale<double, NW, S, C>(A, reinterpret_cast<uint32_t*>(sm.red));
    scale_regs(A, f);
    gj_invert<double, NW, S, C>(A, n, sm.colbuf, sm.pivrow, sm.pinv, &sm.flag);
    {
      const double km = tile_absmax_wave(A);
      if (lane_id() == 0) sm.kred[w] = km;
    }
    // (a vacancy's diagonal entry is zeroed by the store)
    store_unpermuted<double, double, NW, S, C>(
        A, n, f, sm.wbuf, sm.pivrow, sm.pinv, Kout, h == q.hs ? G1out : nullptr,
        (dkey >> 31) ? q.eps_r + (int64_t)(h >> 1) * a.N : nullptr, e);
  } else {
    cx<float> AJ[S][C];
    dkey = build_M<float, NW, S, C>(AJ, a, q, h, Kprev, sm.wbuf + w * NP);
    const float f = tile_scale<float, NW, S, C>(AJ, reinterpret_cast<uint32_t*>(sm.red));
    scale_regs(AJ, f);
    gj_invert<float, NW, S, C>(AJ, n, reinterpret_cast<cx<float>*>(sm.colbuf), sm.pivrow,
                               sm.pinv, &sm.flag);
    {
      const double km = tile_absmax_wave(AJ);
      if (lane_id() == 0) sm.kred[w] = km;
    }
    // without refinement the store zeroes a vacancy's diagonal entry; the
    // refinement keeps the identity's 1 there until it has converged
    store_unpermuted<float, double, NW, S, C>(
        AJ, n, f, reinterpret_cast<cx<float>*>(sm.wbuf), sm.pivrow, sm.pinv, Kout,
        (h == q.hs && !REFINE) ? G1out : nullptr,
        (!REFINE && (dkey >> 31)) ? q.eps_r + (int64_t)(h >> 1) * a.N : nullptr, e);
  }
  [[maybe_unused]] const bool vac = (dkey >> 31) != 0;  // block-uniform: every wave holds every row
  dkey &= 0x7FFFFFFFu;
  __syncthreads();
  if (threadIdx.x == 0) {  // the next write of kred follows two more barriers
    double km = sm.kred[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) km = max(km, sm.kred[i]);
    sm.ksum += km;
    if (dkey < mag_hi(kChiralWindow * fabs(a.t))) sm.ksum_c += km;
  }
  if constexpr (REFINE) {
    // Newton's iteration for the inverse in FP64 from the FP32 start g0:
    //   R_k = I - M g_k,  g_{k+1} = g_k (I + R_k),  R_{k+1} = R_k^2,
    // with M regenerated in FP64 from Kprev. It converges when the spectral
    // radius of R_0 is below 1; n max|R_0| bounds the infinity norm, so a
    // start with n max|R_0| >= 1/2 (kappa ~ 1/u_32 near resonances of
    // disordered ribbons) is not used, and neither is one whose residual
    // fails to shrink at a later step or that has not converged after four
    // steps: such a half-slice is inverted again by the FP64 Gauss-Jordan.
    const int lane = lane_id();
    bool converged = false;
    double rprev = 0.0;
    unsigned upd = 0;
    for (int it = 0; it < 4; ++it) {
      {
        const Tuple& qq = q;
        auto fa = [&](int r, int k) -> cx<double> { return m_entry<NP>(a, qq, h, Kprev, r, k); };
        auto fb = [&](int k, int c) -> cx<double> {
          return (c < n) ? ldg(Kout + (size_t)c * NP + k) : mk(0.0, 0.0);
        };
        gemm_regs<double, NW, S, C, KC>(A, n, fa, fb, sm.As, sm.Bs);
      }
      double lmax = 0.0;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int r = lane + 64 * s;
#pragma unroll
        for (int j = 0; j < C; ++j) {
          const int c = w * C + j;
          const cx<double> d = mk(((r == c) ? 1.0 : 0.0) - A[s][j].re, -A[s][j].im);
          if (r < n && c < n) {
            const double m1 = cabs1(d);
            lmax = (m1 > lmax || m1 != m1) ? m1 : lmax;
          }
          A[s][j] = mk(((r == c) ? 1.0 : 0.0) + d.re, d.im);   // I + R_k
        }
      }
      const double rmax = block_max<NW>(lmax, sm.red);
      if (it == 0 ? !((double)n * rmax < 0.5) : !(rmax < rprev)) break;  // not converging
      if (!(rmax > 1e-15)) {   // at rounding level already
        converged = true;
        break;
      }
      store_regs<double, double, NW, S, C>(A, n, n, Rbuf);
      __syncthreads();
      auto fa = [&](int r, int k) -> cx<double> {
        return (r < n) ? ldg(Kout + (size_t)k * NP + r) : mk(0.0, 0.0);
      };
      auto fb = [&](int k, int c) -> cx<double> {
        return (c < n) ? ldg(Rbuf + (size_t)c * NP + k) : mk(0.0, 0.0);
      };
      gemm_regs<double, NW, S, C, KC>(A, n, fa, fb, sm.As, sm.Bs);
      store_regs<double, double, NW, S, C>(A, n, n, Kout);
      __syncthreads();
      ++upd;
      if (rmax < 1e-8) {   // the next residual is below n rmax^2 < n * 1e-16
        converged = true;
        break;
      }
      rprev = rmax;
    }
    const bool fallback = !converged;
    if (threadIdx.x == 0) {
      sm.rf[0] += 1u;
      sm.rf[1] += upd;
      sm.rf[2] += fallback ? 1u : 0u;
    }
    if (fallback) {
      build_M<double, NW, S, C>(A, a, q, h, Kprev, sm.wbuf + w * NP);
      const double f = tile_scale<double, NW, S, C>(A, reinterpret_cast<uint32_t*>(sm.red));
      scale_regs(A, f);
      gj_invert<double, NW, S, C>(A, n, sm.colbuf, sm.pivrow, sm.pinv, &sm.flag);
      store_unpermuted<double, double, NW, S, C>(A, n, f, sm.wbuf, sm.pivrow, sm.pinv, Kout,
                                                 nullptr);
      __syncthreads();
    }
    if (vac) {
      zero_vacant_diag<NP>(a, q, h, Kout, nullptr);
      __syncthreads();
    }
    if (h == q.hs) {
      for (int i = threadIdx.x; i < NP * NP; i += NW * 64) stg(G1out + i, ldg(Kout + i));
      __syncthreads();
    }
  }
  if (h > q.hs && q.g1) {
    // G1_h = (G1_{h-1} C_{h-1}) g_h on the matrix cores; g_h is complex
    // symmetric, so it is read transposed (rows contiguous)
    const double t = a.t;
    const cx<double>* G1r = opaque_uniform(G1in);
    const cx<double>* Kg = opaque_uniform(Kout);
    cx<double>* G1w = opaque_uniform(G1out);
    auto fb = [&](int k, int c) -> cx<double> { return ldg(Kg + (size_t)k * NP + c); };
    auto epi = [&](int r, int c, cx<double> v, bool ok) {
      if (ok) stg(G1w + (size_t)c * NP + r, v);
    };
    if (!(h & 1)) {
      auto fa = [&](int r, int k) -> cx<double> {
        return cscale(ldg(G1r + (size_t)k * NP + r), t);
      };
      gemm_mfma<NW, NP>(n1, n, n, fa, fb, epi);
    } else {
      const int nL = half_size(a.N, e ^ 1);
      auto fa = [&](int r, int k) -> cx<double> {
        const int k0 = nb_lo(k, e), k1 = nb_hi(k, e);
        cx<double> acc = mk(0.0, 0.0);
        if (k0 >= 0) acc = ldg(G1r + (size_t)k0 * NP + r);
        if (k1 < nL) acc = cadd(acc, ldg(G1r + (size_t)k1 * NP + r));
        return cscale(acc, t);
      };
      gemm_mfma<NW, NP>(n1, n, n, fa, fb, epi);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------
// The half-slice step with the matrix-core inversion of rgf_mgj.hpp (8
// waves, n <= 128; the G1 product and the refinement on the matrix cores).

// M_h in the accumulator layout of wave w's tile column (rgf_mgj.hpp),
// padded with the identity; every entry is formed in FP64 and rounded once
// to T. K (g of the previous half-slice) is complex symmetric, so entry
// (r, c) reads K[r][c] with the 16 lanes of a row group on 16 consecutive
// columns (coalesced). Returns (block-uniform) the high word of
// max_k |E - eps_{h,k}| over the rows present, for the accuracy guard, with
// bit 31 set if the half-slice has a vacancy.
// If Mout is non-null, M_h is also stored there in FP64, row-major
// (Mout[r NP + c]; M_h is complex symmetric, so it reads column-major too).
template <typename T>
__device__ __forceinline__ uint32_t mgj_build(MgjTile<T>& D, const SweepArgs& a, const Tuple& q,
                                              int h, const cx<double>* K,
                                              cx<double>* Mout = nullptr) {
  constexpr int NP = MG_NP;
  // lane and wave made opaque so that the per-entry row / column offsets
  // are recomputed here instead of being hoisted out of the slice loop
  // (32 entries x up to four offsets would stay live for the whole sweep)
  int lane = lane_id(), w = wave_id();
  asm volatile("" : "+v"(lane));
  asm volatile("" : "+s"(w));
  const int li = lane & 15, lk = lane >> 4;
  const bool rhalf = (h & 1) != 0;
  const int e = half_parity(h, a.parity);
  const int n = half_size(a.N, e);
  const int nL = half_size(a.N, e ^ 1);
  const double mt2 = -(a.t * a.t);
  const double* eps_slice = q.eps_r ? q.eps_r + (int64_t)(h >> 1) * a.N : nullptr;
  const double* ph = (h == q.hs)   ? (q.phi_s ? q.phi_s : a.phi)
                     : (h == q.he) ? (q.phi_e ? q.phi_e : a.phi + (size_t)a.P * NP)
                                   : nullptr;
  K = opaque_uniform(K);
  const int c = 16 * w + li;
  const int c0 = nb_lo(c, e), c1 = nb_hi(c, e);
  // max |E - eps| over the rows present (rows lane and lane + 64 of every
  // wave: block-uniform) and the vacancies as a 128-bit row mask in scalar
  // registers (word i: rows 32 i .. 32 i + 31)
  uint32_t dk = 0u, vm[4];
  {
    const int l0 = lane_id();
    bool v0 = false, v1 = false;
    if (l0 < n) {
      const double ev = eps_slice ? eps_slice[half_row(l0, e)] : 0.0;
      v0 = is_vacancy(ev);
      if (!v0) dk = mag_hi(fabs(q.z.re - ev));
    }
    if (l0 + 64 < n) {
      const double ev = eps_slice ? eps_slice[half_row(l0 + 64, e)] : 0.0;
      v1 = is_vacancy(ev);
      if (!v1) dk = max(dk, mag_hi(fabs(q.z.re - ev)));
    }
    const uint64_t b0 = __builtin_amdgcn_ballot_w64(v0), b1 = __builtin_amdgcn_ballot_w64(v1);
    vm[0] = (uint32_t)b0;
    vm[1] = (uint32_t)(b0 >> 32);
    vm[2] = (uint32_t)b1;
    vm[3] = (uint32_t)(b1 >> 32);
  }
  dk = wave_max_u32(dk);
  const bool anyv = (vm[0] | vm[1] | vm[2] | vm[3]) != 0u;
  // column c = 16 w + li lies in word w / 2 (wave-uniform)
  const uint32_t vmc = (w >> 1) == 0 ? vm[0] : (w >> 1) == 1 ? vm[1] : (w >> 1) == 2 ? vm[2] : vm[3];
  const bool vc = ((vmc >> (c & 31)) & 1u) != 0u;
#pragma unroll
  for (int I = 0; I < MG_TI; ++I)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * I + mgj_row<T>(v, lk);   // in word I / 2
      cx<double> x = mk((r == c) ? 1.0 : 0.0, 0.0);
      if (r < n && c < n) {
        x = mk(0.0, 0.0);
        if (h > q.hs) {
          if (!rhalf) {
            x = cscale(ldg(K + (size_t)r * NP + c), mt2);
          } else {
            const int r0 = nb_lo(r, e), r1 = nb_hi(r, e);
            cx<double> acc = mk(0.0, 0.0);
            if (r0 >= 0) {
              if (c0 >= 0) acc = cadd(acc, ldg(K + (size_t)r0 * NP + c0));
              if (c1 < nL) acc = cadd(acc, ldg(K + (size_t)r0 * NP + c1));
            }
            if (r1 < nL) {
              if (c0 >= 0) acc = cadd(acc, ldg(K + (size_t)r1 * NP + c0));
              if (c1 < nL) acc = cadd(acc, ldg(K + (size_t)r1 * NP + c1));
            }
            x = cscale(acc, mt2);
          }
        }
        if (r == c) {
          const double d = q.z.re - (eps_slice ? eps_slice[half_row(r, e)] : 0.0);
          x = cadd(x, mk(d, q.z.im));
        }
        if (ph) {  // lead self-energy on the first and the last half-slice
          for (int p = 0; p < a.P; ++p) {
            const double f = ph[(size_t)p * NP + r] * ph[(size_t)p * NP + c];
            x.re = fma(-f, q.sig[p].re, x.re);
            x.im = fma(-f, q.sig[p].im, x.im);
          }
        }
      }
      // a vacancy's row and column are the identity's
      if (anyv && (vc || ((vm[I >> 1] >> (r & 31)) & 1u))) x = mk((r == c) ? 1.0 : 0.0, 0.0);
      mgj_set(D, I, v, mk<T>((T)x.re, (T)x.im));
      if (Mout) stg(Mout + (size_t)r * NP + c, x);
      // bound the loads in flight (register pressure)
      if ((v & 1) == 1) __builtin_amdgcn_sched_barrier(0);
    }
  return anyv ? (dk | 0x80000000u) : dk;
}

// g = M_h^{-1} into Kout by the matrix-core Gauss-Jordan in precision T
// (and into K2 if non-null); records kappa_h for the guard in sm.kred.
template <typename T, int NW, int S, int C>
__device__ __forceinline__ uint32_t mgj_inverse_to(const SweepArgs& a, const Tuple& q, int h,
                                                   const cx<double>* Kprev, cx<double>* Kout,
                                                   cx<double>* K2, SweepSmem<NW, S, C>& sm,
                                                   MgjSmem<T>& ms, cx<double>* Mout = nullptr) {
  constexpr bool F64 = sizeof(T) == sizeof(double);
  const int n = half_size(a.N, half_parity(h, a.parity));
  MgjTile<T> D;
  const uint32_t dkey = mgj_build<T>(D, a, q, h, Kprev, Mout);
  const double f = mgj_pow2_scale(mgj_absmax(D, ms), F64 ? -1022 : -126);
  mgj_scale(D, (T)f);
  mgj_invert(D, n, ms, &sm.flag);
  {
    uint32_t b = 0u;
#pragma unroll
    for (int I = 0; I < MG_TI; ++I)
#pragma unroll
      for (int v = 0; v < 4; ++v) b = max(b, mag_hi(cabs1(mgj_get(D, I, v))));
    b = wave_max_u32(b);
    if (lane_id() == 0)
      sm.kred[wave_id()] = F64 ? __longlong_as_double((long long)((uint64_t)b << 32))
                               : (double)__uint_as_float(b);
  }
  mgj_store<T, double>(D, n, f, ms, Kout, K2);
  return dkey;
}

template <typename TJ, bool REFINE>
__device__ __forceinline__ void half_step_mgj(const SweepArgs& a, const Tuple& q, int h,
                                              const cx<double>* Kprev, cx<double>* Kout,
                                              const cx<double>* G1in, cx<double>* G1out,
                                              cx<double>* Rbuf, cx<double>* Mbuf,
                                              SweepSmem<8, 2, 16>& sm, MgjSmem<double>& ms64) {
  constexpr int NW = 8, NP = MG_NP;
  static_assert(NP == 8 * 16, "matrix-core tile is the (8, 2, 16) tiling");
  const int e = half_parity(h, a.parity);
  const int n = half_size(a.N, e);
  const int n1 = half_size(a.N, half_parity(q.hs, a.parity));
  uint32_t dkey;
  if constexpr (sizeof(TJ) == sizeof(double))
    dkey = mgj_inverse_to<double>(a, q, h, Kprev, Kout, h == q.hs ? G1out : nullptr, sm, ms64);
  else
    dkey = mgj_inverse_to<float>(a, q, h, Kprev, Kout, (h == q.hs && !REFINE) ? G1out : nullptr, sm,
                                 *reinterpret_cast<MgjSmem<float>*>(&ms64),
                                 REFINE ? Mbuf : nullptr);
  const bool vac = (dkey >> 31) != 0;  // block-uniform
  dkey &= 0x7FFFFFFFu;
  __syncthreads();
  if (threadIdx.x == 0) {  // kred is written again only after further barriers
    double km = sm.kred[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) km = max(km, sm.kred[i]);
    sm.ksum += km;
    if (dkey < mag_hi(kChiralWindow * fabs(a.t))) sm.ksum_c += km;
  }
  if (!REFINE && vac) {
    zero_vacant_diag<NP>(a, q, h, Kout, h == q.hs ? G1out : nullptr);
    __syncthreads();
  }
  if constexpr (REFINE) {
    // Newton's iteration in FP64 on the matrix cores from the FP32 start:
    //   R_k = I - M g_k,  g_{k+1} = g_k (I + R_k);
    // the start is used only if n max|R_0| < 1/2 (the infinity norm bound
    // keeps the spectral radius of R_0 below 1), the residual must shrink
    // at every step and converge within four; otherwise the half-slice is
    // inverted again by the FP64 Gauss-Jordan.
    bool converged = false;
    double rprev = 0.0;
    unsigned upd = 0;
    for (int it = 0; it < 4; ++it) {
      double lmax = 0.0;
      {
        // M_h as stored by the build (FP64, complex symmetric)
        auto fa = [&](int r, int k) -> cx<double> { return ldg(Mbuf + (size_t)k * NP + r); };
        auto fb = [&](int k, int c) -> cx<double> { return ldg(Kout + (size_t)c * NP + k); };
        auto epi = [&](int r, int c, cx<double> v, bool ok) {
          if (!ok) return;
          const cx<double> d = mk(((r == c) ? 1.0 : 0.0) - v.re, -v.im);
          const double m1 = cabs1(d);
          lmax = (m1 > lmax || m1 != m1) ? m1 : lmax;
          stg(Rbuf + (size_t)c * NP + r, mk(((r == c) ? 1.0 : 0.0) + d.re, d.im));  // I + R_k
        };
        gemm_mfma<NW, NP>(n, n, n, fa, fb, epi);
      }
      const double rmax = block_max<NW>(lmax, sm.red);
      if (it == 0 ? !((double)n * rmax < 0.5) : !(rmax < rprev)) break;  // not converging
      if (!(rmax > 1e-15)) {  // at rounding level already
        converged = true;
        break;
      }
      {
        auto fa = [&](int r, int k) -> cx<double> { return ldg(Kout + (size_t)k * NP + r); };
        auto fb = [&](int k, int c) -> cx<double> { return ldg(Rbuf + (size_t)c * NP + k); };
        auto epi = [&](int r, int c, cx<double> v, bool ok) {
          if (ok) stg(Kout + (size_t)c * NP + r, v);
        };
        gemm_mfma<NW, NP>(n, n, n, fa, fb, epi);
      }
      __syncthreads();
      ++upd;
      if (rmax < 1e-8) {  // the next residual is below n rmax^2 < n * 1e-16
        converged = true;
        break;
      }
      rprev = rmax;
    }
    if (threadIdx.x == 0) {
      sm.rf[0] += 1u;
      sm.rf[1] += upd;
      sm.rf[2] += converged ? 0u : 1u;
    }
    if (!converged) {
      (void)mgj_inverse_to<double>(a, q, h, Kprev, Kout, nullptr, sm, ms64);
      __syncthreads();
    }
    if (vac) {
      zero_vacant_diag<NP>(a, q, h, Kout, nullptr);
      __syncthreads();
    }
    if (h == q.hs) {
      for (int i = threadIdx.x; i < NP * NP; i += NW * 64) stg(G1out + i, ldg(Kout + i));
      __syncthreads();
    }
  }
  if (h > q.hs && q.g1) {
    // G1_h = (G1_{h-1} C_{h-1}) g_h on the matrix cores (g_h read transposed)
    const double t = a.t;
    const cx<double>* G1r = opaque_uniform(G1in);
    const cx<double>* Kg = opaque_uniform(Kout);
    cx<double>* G1w = opaque_uniform(G1out);
    auto fb = [&](int k, int c) -> cx<double> { return ldg(Kg + (size_t)k * NP + c); };
    auto epi = [&](int r, int c, cx<double> v, bool ok) {
      if (ok) stg(G1w + (size_t)c * NP + r, v);
    };
    if (!(h & 1)) {
      auto fa = [&](int r, int k) -> cx<double> {
        return cscale(ldg(G1r + (size_t)k * NP + r), t);
      };
      gemm_mfma<NW, NP>(n1, n, n, fa, fb, epi);
    } else {
      const int nL = half_size(a.N, e ^ 1);
      auto fa = [&](int r, int k) -> cx<double> {
        const int k0 = nb_lo(k, e), k1 = nb_hi(k, e);
        cx<double> acc = mk(0.0, 0.0);
        if (k0 >= 0) acc = ldg(G1r + (size_t)k0 * NP + r);
        if (k1 < nL) acc = cadd(acc, ldg(G1r + (size_t)k1 * NP + r));
        return cscale(acc, t);
      };
      gemm_mfma<NW, NP>(n1, n, n, fa, fb, epi);
    }
    __syncthreads();
  }
}

// Conductance from G = G_{1L} in Gbuf: X = G Phi_R -> Xbuf (n1 x P), then
// S = Phi_L^T X in registers; returns T = sum_{p,q} d_p d_q |S_pq|^2 (every
// thread). S is left in A (rows p, columns q) for callers that need it.
// With chan set, the channel sums sum_q d_q |S_pq|^2 are left in
// sm.rowacc[p] (the transmission of incoming channel p is d_p times that).
template <int NW, int S, int C>
__device__ __forceinline__ double trace_T(const SweepArgs& a, const Tuple& q,
                                          const cx<double>* Gbuf, cx<double>* Xbuf,
                                          cx<double> (&A)[S][C], SweepSmem<NW, S, C>& sm,
                                          bool chan = false) {
  constexpr int NP = NW * C;
  const int lane = lane_id(), w = wave_id();
  const int n1 = half_size(a.N, half_parity(0, a.parity));
  const int nlast = half_size(a.N, half_parity(2 * a.L - 1, a.parity));
  const double* phiL = a.phi;
  const double* phiR = a.phi + (size_t)a.P * NP;
  {
    auto fa = [&](int r, int k) -> cx<double> {
      return (r < n1) ? ldg(Gbuf + (size_t)k * NP + r) : mk(0.0, 0.0);
    };
    auto fb = [&](int k, int c) -> cx<double> {
      return (c < a.P) ? mk(phiR[(size_t)c * NP + k], 0.0) : mk(0.0, 0.0);
    };
    gemm_regs<double, NW, S, C, KC>(A, nlast, fa, fb, sm.As, sm.Bs);
    store_regs<double, double, NW, S, C>(A, n1, a.P, Xbuf);
    if (chan)
      for (int i = threadIdx.x; i < NP; i += NW * 64) sm.rowacc[i] = 0.0;
    __syncthreads();
  }
  double part = 0.0;
  {
    auto fa = [&](int r, int k) -> cx<double> {
      return (r < a.P) ? mk(phiL[(size_t)r * NP + k], 0.0) : mk(0.0, 0.0);
    };
    auto fb = [&](int k, int c) -> cx<double> {
      return (c < a.P) ? ldg(Xbuf + (size_t)c * NP + k) : mk(0.0, 0.0);
    };
    gemm_regs<double, NW, S, C, KC>(A, n1, fa, fb, sm.As, sm.Bs);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int p = lane + 64 * s;
      if (p >= a.P) continue;
      double row = 0.0;
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const int qq = w * C + j;
        if (qq < a.P) {
          const double dq = -2.0 * q.sig[qq].im;
          row += dq * (A[s][j].re * A[s][j].re + A[s][j].im * A[s][j].im);
        }
      }
      part += -2.0 * q.sig[p].im * row;
      if (chan) atomicAdd(&sm.rowacc[p], row);
    }
  }
  return block_sum<NW>(part, sm.red);
}

// Forward sweep over all half-slices that also stores the restart state
// (g_h, G1_h) after every `stride` half-slices into ck[1..] (the state at
// h = 0 is rebuilt from the leads, so ck[0] stays unused). Used by the
// reverse sweeps, which recompute each segment from its checkpoint. Leaves
// g_{H-1} in kb[(H-1) & 1] and G1_{H-1} in gbuf.
template <typename TJ, bool REFINE, int NW, int S, int C>
__device__ __forceinline__ void forward_with_checkpoints(const SweepArgs& a, const Tuple& q,
                                                         cx<double>* const (&kb)[2],
                                                         cx<double>* gbuf, cx<double>* rbuf,
                                                         cx<double>* ck, cx<double> (&A)[S][C],
                                                         SweepSmem<NW, S, C>& sm) {
  constexpr int NP = NW * C;
  constexpr size_t MAT = (size_t)NP * NP;
  const int H = 2 * a.L;
  for (int h = 0; h < H; ++h) {
    half_step<TJ, REFINE, NW, S, C>(a, q, h, kb[(h + 1) & 1], kb[h & 1], gbuf, gbuf, rbuf, A,
                                    sm);
    if ((h + 1) % a.stride == 0 && h + 1 < H) {
      cx<double>* c = ck + (size_t)((h + 1) / a.stride) * 2 * MAT;
      for (size_t i = threadIdx.x; i < MAT; i += NW * 64) {
        stg(c + i, ldg(kb[h & 1] + i));
        stg(c + MAT + i, ldg(gbuf + i));
      }
      __syncthreads();
    }
  }
}

// Recompute g_h, G1_h for h0 <= h < h1 into the segment buffer sg (pairs of
// matrices), starting from checkpoint sgi (or from the leads for sgi = 0).
template <typename TJ, bool REFINE, int NW, int S, int C>
__device__ __forceinline__ void recompute_segment(const SweepArgs& a, const Tuple& q, int sgi,
                                                  int h0, int h1, cx<double>* ck, cx<double>* sg,
                                                  cx<double>* rbuf, cx<double> (&A)[S][C],
                                                  SweepSmem<NW, S, C>& sm) {
  constexpr size_t MAT = (size_t)NW * C * NW * C;
  for (int h = h0; h < h1; ++h) {
    const int j = h - h0;
    const cx<double>* Kp = (j == 0) ? ck + (size_t)sgi * 2 * MAT : sg + (size_t)(j - 1) * 2 * MAT;
    const cx<double>* Gp = Kp + MAT;
    cx<double>* Ko = sg + (size_t)j * 2 * MAT;
    half_step<TJ, REFINE, NW, S, C>(a, q, h, Kp, Ko, Gp, Ko + MAT, rbuf, A, sm);
  }
}

}  // namespace rgf
