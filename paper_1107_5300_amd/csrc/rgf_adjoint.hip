// rgf_adjoint.hip -- gradient of the conductance with respect to every
// on-site energy, by a backward sweep over the half-slice chain.
//
// From Eq. (1), dG/d eps_s = G E_ss G, so Eq. (2) gives
//   dT/d eps_s = 2 Re[ G[s, R_L] B G[L_1, s] ],   B = Gamma_R G_{1L}^dagger Gamma_L.
// With the left-connected g_h and G1_h of the forward sweep and C_h the
// coupling from half-slice h to h+1, Dyson's equation (Eq. (3)) cut between
// h and h+1 gives the full-system blocks
//   G[h, last]  = g_h C_h G[h+1, last],          G[last, last] = g_last
//   G[h, first] = G1_h^T + g_h C_h G[h+1, first], G[last, first] = G1_last^T
// (g and G are complex symmetric). Carrying Z_h = G[h, last] B instead of
// G[h, last]:
//   Z_h = g_h (C_h Z_{h+1}),  Q_h = G1_h^T + g_h (C_h Q_{h+1}),
//   dT/d eps_{h,a} = 2 Re sum_c Z_h[a][c] Q_h[a][c].
// The kernel accumulates w * dT/d eps into dL_deps (w = dL/dT of the tuple)
// with FP64 atomics, so energies of one realization sum in any order.
//
// Memory: the forward sweep stores its restart state (g, G1) every `stride`
// half-slices; the backward sweep walks the segments from the last one,
// recomputing each segment's g_h and G1_h from its checkpoint into a segment
// buffer and then stepping Z and Q back through it. Per tuple this needs
// O((2L/stride + stride) NP^2) complex128, and about three forward sweeps of
// arithmetic.

#include <string.h>

#include "rgf_sweep.hpp"

namespace rgf {

namespace {

template <typename TJ, bool REFINE, int NW, int S, int C>
__global__ __launch_bounds__(NW * 64) void rgf_grad_kernel(SweepArgs a) {
  constexpr int NP = NW * C;
  constexpr size_t MAT = (size_t)NP * NP;
  __shared__ SweepSmem<NW, S, C> sm;
  const int lane = lane_id(), w = wave_id();
  // slot: K0, G1, R, K1, Z, Q, X
  cx<double>* slot = a.slots + (size_t)blockIdx.x * a.slot_mats * MAT;
  cx<double>* const kb[2] = {slot, REFINE ? slot + 3 * MAT : slot};
  cx<double>* gbuf = slot + MAT;
  cx<double>* rbuf = slot + 2 * MAT;
  cx<double>* zbuf = slot + 4 * MAT;
  cx<double>* qbuf = slot + 5 * MAT;
  cx<double>* xbuf = slot + 6 * MAT;
  cx<double>* ck = a.ckpt + (size_t)blockIdx.x * a.n_ckpt * 2 * MAT;
  cx<double>* sg = a.seg + (size_t)blockIdx.x * a.stride * 2 * MAT;
  const int H = 2 * a.L;
  const int n1 = half_size(a.N, half_parity(0, a.parity));
  const int nlast = half_size(a.N, half_parity(H - 1, a.parity));
  const double* phiL = a.phi;
  const double* phiR = a.phi + (size_t)a.P * NP;

  for (int64_t tau = blockIdx.x; tau < a.ntuples; tau += gridDim.x) {
    const Tuple q = make_tuple_(a, tau);
    if (threadIdx.x == 0) {
      sm.flag = 0;
      sm.ksum = 0.0;
      sm.ksum_c = 0.0;
    }
    __syncthreads();
    cx<double> A[S][C];

    // ---- forward sweep with checkpoints of (g_h, G1_h) after every stride
    forward_with_checkpoints<TJ, REFINE, NW, S, C>(a, q, kb, gbuf, rbuf, ck, A, sm);
    cx<double>* Klast = kb[(H - 1) & 1];
    const double T = trace_T<NW, S, C>(a, q, gbuf, xbuf, A, sm);  // S = Phi_L^T G Phi_R in A
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
      a.T_out[tau] = (st == RGF_TUPLE_OK) ? T : __builtin_nan("");
      if (a.status) a.status[tau] = st;
    }
    const double wt = a.dL_dT[tau];
    if (st != RGF_TUPLE_OK || wt == 0.0) {
      __syncthreads();
      continue;
    }

    // ---- Y = D S^dagger D (P x P) -> rbuf;  Y[q][p] = d_q conj(S[p][q]) d_p
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int p = lane + 64 * s;
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const int qq = w * C + j;
        if (p < a.P && qq < a.P) {
          const double f = 4.0 * q.sig[p].im * q.sig[qq].im;  // d_p d_q
          stg(rbuf + (size_t)p * NP + qq, mk(f * A[s][j].re, -f * A[s][j].im));
        }
      }
    }
    __syncthreads();
    // V = g_last Phi_R (nlast x P) -> xbuf
    {
      auto fa = [&](int r, int k) -> cx<double> {
        return (r < nlast) ? ldg(Klast + (size_t)k * NP + r) : mk(0.0, 0.0);
      };
      auto fb = [&](int k, int c) -> cx<double> {
        return (c < a.P) ? mk(phiR[(size_t)c * NP + k], 0.0) : mk(0.0, 0.0);
      };
      gemm_regs<double, NW, S, C, KC>(A, nlast, fa, fb, sm.As, sm.Bs);
      store_regs<double, double, NW, S, C>(A, nlast, a.P, xbuf);
      __syncthreads();
    }
    // V2 = V Y (nlast x P) -> zbuf
    {
      auto fa = [&](int r, int k) -> cx<double> {
        return (r < nlast) ? ldg(xbuf + (size_t)k * NP + r) : mk(0.0, 0.0);
      };
      auto fb = [&](int k, int c) -> cx<double> {
        return (c < a.P) ? ldg(rbuf + (size_t)c * NP + k) : mk(0.0, 0.0);
      };
      gemm_regs<double, NW, S, C, KC>(A, a.P, fa, fb, sm.As, sm.Bs);
      store_regs<double, double, NW, S, C>(A, nlast, a.P, zbuf);
      __syncthreads();
    }
    // Z_last = V2 Phi_L^T (nlast x n1) -> xbuf, then -> zbuf
    {
      auto fa = [&](int r, int k) -> cx<double> {
        return (r < nlast) ? ldg(zbuf + (size_t)k * NP + r) : mk(0.0, 0.0);
      };
      auto fb = [&](int k, int c) -> cx<double> {
        return (c < n1) ? mk(phiL[(size_t)k * NP + c], 0.0) : mk(0.0, 0.0);
      };
      gemm_regs<double, NW, S, C, KC>(A, a.P, fa, fb, sm.As, sm.Bs);
      store_regs_rowmajor<double, double, NW, S, C>(A, nlast, n1, zbuf);
      __syncthreads();
    }

    // ---- backward over segments
    const int nseg = (H + a.stride - 1) / a.stride;
    for (int sgi = nseg - 1; sgi >= 0; --sgi) {
      const int h0 = sgi * a.stride;
      const int h1 = min(H, h0 + a.stride);
      // recompute g_h, G1_h of the segment into sg
      recompute_segment<TJ, REFINE, NW, S, C>(a, q, sgi, h0, h1, ck, sg, rbuf, A, sm);
      // step Z and Q back through the segment; both are kept row-major
      // (X[r][c] at r*NP + c), so the matrix-core GEMMs read C_h X along rows
      // and write their results with contiguous columns
      for (int h = h1 - 1; h >= h0; --h) {
        const cx<double>* gh = opaque_uniform(sg + (size_t)(h - h0) * 2 * MAT);
        const cx<double>* G1h = gh + MAT;
        const int e = half_parity(h, a.parity);
        const int n = half_size(a.N, e);
        if (threadIdx.x < NP) sm.rowacc[threadIdx.x] = 0.0;
        if (h < H - 1) {
          const int en = half_parity(h + 1, a.parity);
          const int nn = half_size(a.N, en);
          const double t = a.t;
          // (C_h X)[k][c]: h even (L_i -> R_i): t * (X[k + 1 - eR][c] + X[k - eR][c]);
          //                h odd  (R_i -> L_{i+1}): t * X[k][c]
          auto capply = [&](const cx<double>* X, int k, int c) -> cx<double> {
            if (h & 1) return cscale(ldg(X + (size_t)k * NP + c), t);
            const int b0 = k + 1 - en, b1 = k - en;
            cx<double> acc = mk(0.0, 0.0);
            if (b0 >= 0 && b0 < nn) acc = ldg(X + (size_t)b0 * NP + c);
            if (b1 >= 0 && b1 < nn) acc = cadd(acc, ldg(X + (size_t)b1 * NP + c));
            return cscale(acc, t);
          };
          auto fa = [&](int r, int k) -> cx<double> { return ldg(gh + (size_t)k * NP + r); };
          // Z_h = g_h (C_h Z_{h+1}), in place
          {
            auto fb = [&](int k, int c) -> cx<double> { return capply(zbuf, k, c); };
            auto epi = [&](int r, int c, cx<double> v, bool ok) {
              if (ok) stg(zbuf + (size_t)r * NP + c, v);
            };
            gemm_mfma<NW, NP>(n, n1, n, fa, fb, epi);
          }
          // Q_h = G1_h^T + g_h (C_h Q_{h+1}), in place, and the row sums
          // sum_c Re(Z_h[a][c] Q_h[a][c]) (16 columns per row group, then LDS)
          {
            auto fb = [&](int k, int c) -> cx<double> { return capply(qbuf, k, c); };
            auto epi = [&](int r, int c, cx<double> v, bool ok) {
              double part = 0.0;
              if (ok) {
                v = cadd(v, ldg(G1h + (size_t)r * NP + c));  // G1_h^T[r][c] = G1_h[c][r]
                const cx<double> z = ldg(zbuf + (size_t)r * NP + c);
                part = z.re * v.re - z.im * v.im;
                stg(qbuf + (size_t)r * NP + c, v);
              }
              part += __shfl_xor(part, 1);
              part += __shfl_xor(part, 2);
              part += __shfl_xor(part, 4);
              part += __shfl_xor(part, 8);
              if ((lane_id() & 15) == 0 && r < n) atomicAdd(&sm.rowacc[r], part);
            };
            gemm_mfma<NW, NP>(n, n1, n, fa, fb, epi);
          }
        } else {
          // last half-slice: Z = Z_last (already in zbuf), Q = G1^T
          __syncthreads();
          for (int i = threadIdx.x; i < n * n1; i += NW * 64) {
            const int r = i / n1, c = i - r * n1;
            const cx<double> v = ldg(G1h + (size_t)r * NP + c);
            const cx<double> z = ldg(zbuf + (size_t)r * NP + c);
            stg(qbuf + (size_t)r * NP + c, v);
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

__global__ void fill_zero_kernel(double* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0.0;
}

using GradKernel = void (*)(SweepArgs);

struct GradEntry {
  int NW, S, C;
  GradKernel k[3];
};

#define RGF_GRAD_ENTRY(NW, S, C)                                             \
  {                                                                          \
    NW, S, C, {                                                              \
      rgf_grad_kernel<double, false, NW, S, C>,                              \
          rgf_grad_kernel<float, true, NW, S, C>,                            \
          rgf_grad_kernel<float, false, NW, S, C>                            \
    }                                                                        \
  }

const GradEntry kGrad[] = {
    RGF_GRAD_ENTRY(1, 1, 8),  RGF_GRAD_ENTRY(1, 1, 16), RGF_GRAD_ENTRY(2, 1, 16),
    RGF_GRAD_ENTRY(4, 1, 12), RGF_GRAD_ENTRY(4, 1, 15), RGF_GRAD_ENTRY(4, 1, 16),
    RGF_GRAD_ENTRY(8, 1, 8),  RGF_GRAD_ENTRY(8, 2, 12), RGF_GRAD_ENTRY(8, 2, 15), RGF_GRAD_ENTRY(8, 2, 16),
};

}  // namespace

const void* grad_kernel_ptr(const TileCfg& t, int precision) {
  return (const void*)kGrad[t.id].k[precision];
}

hipError_t launch_grad(const Plan& p, const double* E, const double* eps, const double* dL_dT,
                       double* T_out, double* dL_deps, int32_t* status_out, char* ws,
                       hipStream_t s) {
  const int64_t ng = p.nreal * (int64_t)p.L * p.N;
  if (ng > 0) {
    int64_t blocks = (ng + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, dL_deps, ng);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  if (p.large) return launch_grad_large(p, E, eps, dL_dT, T_out, dL_deps, status_out, ws, s);
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
  a.dL_dT = dL_dT;
  a.dL_deps = dL_deps;
  a.ckpt = reinterpret_cast<cx<double>*>(ws + p.off_ckpt);
  a.seg = reinterpret_cast<cx<double>*>(ws + p.off_seg);
  a.stride = (int)p.ckpt_stride;
  a.n_ckpt = (int)p.n_ckpt;
  const GradEntry& f = kGrad[p.tile.id];
  hipLaunchKernelGGL(f.k[p.precision], dim3(p.grid), dim3(f.NW * 64), 0, s, a);
  return hipGetLastError();
}

}  // namespace rgf
