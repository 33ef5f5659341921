// rgf_ldos.hip -- local density of states of every device site,
//   rho_s(E) = -Im G_ss(E) / pi,
// the spectral density behind the charge density that the paper lists
// among the quantities the Green's function gives (G from Eq. (1)).
//
// The diagonal blocks of G follow from Dyson's equation (Eq. (3)) cut
// between half-slices h and h+1 of the half-slice chain:
//   F_{H-1} = g_{H-1},    F_h = g_h + g_h (C_h F_{h+1} C_h^T) g_h,
// with g_h the left-connected Green's functions of the forward sweep and C_h
// the coupling from half-slice h to h+1 (t * I, or the t-weighted zigzag
// adjacency). The forward sweep stores restart states every `stride`
// half-slices; the backward sweep recomputes each segment from its
// checkpoint, exactly as the adjoint does. Per backward half-slice:
//   V   = W g_h,        W = C_h F_{h+1} C_h^T  (a stencil of F_{h+1}, formed
//                                              while loading the operand)
//   F_h = g_h + g_h V  (the diagonal is written out in the epilogue)
// two n^3 complex GEMMs on the matrix cores. g_h and F_h are complex
// symmetric, so each is read in whichever order is contiguous.

#include <string.h>

#include "rgf_sweep.hpp"

namespace rgf {

namespace {

template <typename TJ, bool REFINE, int NW, int S, int C>
__global__ __launch_bounds__(NW * 64) void rgf_ldos_kernel(SweepArgs a) {
  constexpr int NP = NW * C;
  constexpr size_t MAT = (size_t)NP * NP;
  constexpr double kInvPi = 0.31830988618379067154;
  __shared__ SweepSmem<NW, S, C> sm;
  // slot: K0, G1, R, K1, F, V, X
  cx<double>* slot = a.slots + (size_t)blockIdx.x * a.slot_mats * MAT;
  cx<double>* const kb[2] = {slot, REFINE ? slot + 3 * MAT : slot};
  cx<double>* gbuf = slot + MAT;
  cx<double>* rbuf = slot + 2 * MAT;
  cx<double>* fbuf = slot + 4 * MAT;
  cx<double>* vbuf = slot + 5 * MAT;
  cx<double>* xbuf = slot + 6 * MAT;
  cx<double>* ck = a.ckpt + (size_t)blockIdx.x * a.n_ckpt * 2 * MAT;
  cx<double>* sg = a.seg + (size_t)blockIdx.x * a.stride * 2 * MAT;
  const int H = 2 * a.L;

  for (int64_t tau = blockIdx.x; tau < a.ntuples; tau += gridDim.x) {
    const Tuple q = make_tuple_(a, tau);
    if (threadIdx.x == 0) {
      sm.flag = 0;
      sm.ksum = 0.0;
      sm.ksum_c = 0.0;
    }
    __syncthreads();
    cx<double> A[S][C];
    double* out = a.ldos + tau * (int64_t)a.L * a.N;  // [L][N] of this tuple

    forward_with_checkpoints<TJ, REFINE, NW, S, C>(a, q, kb, gbuf, rbuf, ck, A, sm);
    const cx<double>* Klast = kb[(H - 1) & 1];
    const double T = trace_T<NW, S, C>(a, q, gbuf, xbuf, A, sm);
    int st = a.lstat[q.e];
    // the guard first: a rejected sweep may also show a zero pivot or a T
    // out of range (no whole-slice form of this sweep)
    if ((sizeof(TJ) == sizeof(double) || REFINE) && st == RGF_TUPLE_OK &&
        ill_conditioned(sm.ksum, sm.ksum_c))
      st = RGF_TUPLE_ILL_CONDITIONED;
    if (st == RGF_TUPLE_OK && sm.flag) st = RGF_TUPLE_SINGULAR;
    if (st == RGF_TUPLE_OK && !isfinite(T)) st = RGF_TUPLE_NONFINITE;
    if (st == RGF_TUPLE_OK && !t_in_range(T, a.P)) st = RGF_TUPLE_OUT_OF_RANGE;
    if (threadIdx.x == 0) {
      if (a.T_out) a.T_out[tau] = (st == RGF_TUPLE_OK) ? T : __builtin_nan("");
      if (a.status) a.status[tau] = st;
    }
    if (st != RGF_TUPLE_OK) {
      for (int64_t i = threadIdx.x; i < (int64_t)a.L * a.N; i += NW * 64)
        out[i] = __builtin_nan("");
      __syncthreads();
      continue;
    }

    // ---- last half-slice: F = g_{H-1}
    {
      const int e = half_parity(H - 1, a.parity);
      const int n = half_size(a.N, e);
      for (int i = threadIdx.x; i < n * n; i += NW * 64) {
        const int r = i / n, c = i - r * n;
        stg(fbuf + (size_t)r * NP + c, ldg(Klast + (size_t)r * NP + c));
      }
      if (threadIdx.x < n)
        out[(int64_t)((H - 1) >> 1) * a.N + half_row(threadIdx.x, e)] =
            -ldg(Klast + (size_t)threadIdx.x * NP + threadIdx.x).im * kInvPi;
      __syncthreads();
    }

    // ---- backward over segments
    const int nseg = (H + a.stride - 1) / a.stride;
    for (int sgi = nseg - 1; sgi >= 0; --sgi) {
      const int h0 = sgi * a.stride;
      const int h1 = min(H, h0 + a.stride);
      recompute_segment<TJ, REFINE, NW, S, C>(a, q, sgi, h0, h1, ck, sg, rbuf, A, sm);
      for (int h = min(h1, H - 1) - 1; h >= h0; --h) {
        const cx<double>* gh = opaque_uniform(sg + (size_t)(h - h0) * 2 * MAT);
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
              acc = cadd(acc, ldg(fbuf + (size_t)kb2[u] * NP + rb[v]));
            }
          }
          return cscale(acc, t2);
        };
        {
          auto fb = [&](int k, int c) -> cx<double> { return ldg(gh + (size_t)k * NP + c); };
          auto epi = [&](int r, int c, cx<double> v, bool ok) {
            if (ok) stg(vbuf + (size_t)r * NP + c, v);
          };
          gemm_mfma<NW, NP>(n, n, n, fa_w, fb, epi);
        }
        __syncthreads();
        {
          auto fa = [&](int r, int k) -> cx<double> { return ldg(gh + (size_t)k * NP + r); };
          auto fb = [&](int k, int c) -> cx<double> { return ldg(vbuf + (size_t)k * NP + c); };
          auto epi = [&](int r, int c, cx<double> v, bool ok) {
            if (!ok) return;
            v = cadd(v, ldg(gh + (size_t)r * NP + c));
            stg(fbuf + (size_t)r * NP + c, v);
            if (r == c) out[(int64_t)(h >> 1) * a.N + half_row(r, e)] = -v.im * kInvPi;
          };
          gemm_mfma<NW, NP>(n, n, n, fa, fb, epi);
        }
        __syncthreads();
      }
    }
  }
}

using LdosKernel = void (*)(SweepArgs);

struct LdosEntry {
  int NW, S, C;
  LdosKernel k[3];
};

#define RGF_LDOS_ENTRY(NW, S, C)                                             \
  {                                                                          \
    NW, S, C, {                                                              \
      rgf_ldos_kernel<double, false, NW, S, C>,                              \
          rgf_ldos_kernel<float, true, NW, S, C>,                            \
          rgf_ldos_kernel<float, false, NW, S, C>                            \
    }                                                                        \
  }

// same order as the forward table (indexed by TileCfg::id)
const LdosEntry kLdos[] = {
    RGF_LDOS_ENTRY(1, 1, 8),  RGF_LDOS_ENTRY(1, 1, 16), RGF_LDOS_ENTRY(2, 1, 16),
    RGF_LDOS_ENTRY(4, 1, 12), RGF_LDOS_ENTRY(4, 1, 15), RGF_LDOS_ENTRY(4, 1, 16),
    RGF_LDOS_ENTRY(8, 1, 8),  RGF_LDOS_ENTRY(8, 2, 12), RGF_LDOS_ENTRY(8, 2, 15),
    RGF_LDOS_ENTRY(8, 2, 16),
};

}  // namespace

hipError_t launch_ldos(const Plan& p, const double* E, const double* eps, double* ldos,
                       double* T_out, int32_t* status_out, char* ws, hipStream_t s) {
  if (p.ntuples == 0) return hipSuccess;
  hipError_t err = launch_lead(p, E, ws, s);
  if (err != hipSuccess) return err;
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
  a.ckpt = reinterpret_cast<cx<double>*>(ws + p.off_ckpt);
  a.seg = reinterpret_cast<cx<double>*>(ws + p.off_seg);
  a.stride = (int)p.ckpt_stride;
  a.n_ckpt = (int)p.n_ckpt;
  a.ldos = ldos;
  const LdosEntry& f = kLdos[p.tile.id];
  if (f.NW != p.tile.NW || f.S != p.tile.S || f.C != p.tile.C) return hipErrorInvalidValue;
  hipLaunchKernelGGL(f.k[p.precision], dim3(p.grid), dim3(f.NW * 64), 0, s, a);
  return hipGetLastError();
}

}  // namespace rgf
