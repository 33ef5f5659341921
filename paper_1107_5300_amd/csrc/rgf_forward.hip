// rgf_forward.hip -- forward RGF sweep and conductance trace (FP64).
//
// One persistent workgroup walks the 2L half-slices of one (realization,
// energy) tuple at a time (the recursion is serial in the ribbon length) and
// takes the next tuple when done; tuples are independent.
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
// Conductance (Eq. (2)) with Gamma_{L,R} = Phi_{L,R} diag(d) Phi_{L,R}^T,
// d_p = -2 Im sigma_p (lead modes, see rgf_lead.hip):
//   T = Tr[Gamma_L G Gamma_R G^dagger] = sum_{p,q} d_p d_q |(Phi_L^T G Phi_R)_{pq}|^2.
//
// Per-slot global scratch: K (the latest g_h) and G1, each NP x NP complex128,
// column-major with ld = NP; both stay L2/MALL-resident while the slot runs.

#include "rgf_engine.hpp"
#include "rgf_internal.hpp"

namespace rgf {

namespace {

constexpr int KC = 8;

struct FwdArgs {
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
  cx<double>* slots;        // [grid][2][NP*NP]
  int64_t ntuples;
};

template <int NW, int S, int C>
struct FwdSmem {
  static constexpr int NP = NW * C;
  cx<double> colbuf[2 * NP];
  cx<double> wbuf[NW * NP];
  cx<double> As[KC * NP];
  cx<double> Bs[KC * NP];
  int pivrow[NP];
  int pinv[NP];
  double red[NW];
  int flag;
};

// A -= Phi diag(sigma) Phi^T on the n x n block (lead self-energy), as P
// rank-1 updates: phi[p][.] holds mode p on the interface rows.
template <int NW, int S, int C>
__device__ __forceinline__ void sub_mode_sum(cx<double> (&A)[S][C], const double* phi,
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
        A[s][j].re = fma(-f, sp.re, A[s][j].re);
        A[s][j].im = fma(-f, sp.im, A[s][j].im);
      }
    }
  }
}

// Assemble M_h into the register tile (padded with the identity).
//   L half (h even, h > 0): M = z - eps - t^2 K            (K = g of R_{i-1})
//   R half (h odd):         M = z - eps - t^2 B'^T K B'    (K = g of L_i)
// where (B'^T K B')[r][c] = sum of K over the neighbour rows of r and the
// neighbour columns of c; the column sums go through the wave's LDS scratch.
template <int NW, int S, int C>
__device__ __forceinline__ void build_M(cx<double> (&A)[S][C], const FwdArgs& a, int h,
                                        const double* eps_slice, cx<double> z,
                                        const cx<double>* K, const cx<double>* sig,
                                        cx<double>* wbuf) {
  constexpr int NP = NW * C;
  const int lane = lane_id(), w = wave_id();
  const bool rhalf = (h & 1) != 0;
  const int e = half_parity(h, a.parity);
  const int n = half_size(a.N, e);
  const int nL = half_size(a.N, e ^ 1);  // L half of the same slice (R half only)
  const double mt2 = -(a.t * a.t);
  K = opaque_uniform(K);
  if (eps_slice) eps_slice = opaque_uniform(eps_slice);
  double dre[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int r = lane + 64 * s;
    dre[s] = (r < n) ? z.re - (eps_slice ? eps_slice[half_row(r, e)] : 0.0) : 1.0;
  }
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int c = w * C + j;
    if (!rhalf) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int r = lane + 64 * s;
        cx<double> v = mk(0.0, 0.0);
        if (h > 0 && r < n && c < n) v = cscale(ldg(K + (size_t)c * NP + r), mt2);
        if (r == c) v = cadd(v, mk(dre[s], r < n ? z.im : 0.0));
        A[s][j] = v;
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
        if (r == c) v = cadd(v, mk(dre[s], r < n ? z.im : 0.0));
        A[s][j] = v;
      }
      wave_sync_lds();
    }
  }
  if (h == 0) sub_mode_sum<NW, S, C>(A, a.phi, sig, a.P, n);
  if (h == 2 * a.L - 1) sub_mode_sum<NW, S, C>(A, a.phi + (size_t)a.P * NP, sig, a.P, n);
}

template <int NW, int S, int C>
__global__ __launch_bounds__(NW * 64) void rgf_fwd_kernel(FwdArgs a) {
  constexpr int NP = NW * C;
  __shared__ FwdSmem<NW, S, C> sm;
  const int lane = lane_id(), w = wave_id();
  cx<double>* kbuf = a.slots + (size_t)blockIdx.x * 2 * NP * NP;
  cx<double>* gbuf = kbuf + (size_t)NP * NP;
  const int n1 = half_size(a.N, half_parity(0, a.parity));
  const int nlast = half_size(a.N, half_parity(2 * a.L - 1, a.parity));
  const double* phiL = a.phi;
  const double* phiR = a.phi + (size_t)a.P * NP;

  for (int64_t tau = blockIdx.x; tau < a.ntuples; tau += gridDim.x) {
    const int64_t rr = tau / a.nE, ee = tau - rr * a.nE;
    const cx<double> z = mk(a.E[ee], a.eta);
    const cx<double>* sig = a.sigma + ee * a.P;
    const double* eps_r = a.eps ? a.eps + rr * (int64_t)a.L * a.N : nullptr;
    if (threadIdx.x == 0) sm.flag = 0;
    __syncthreads();
    cx<double> A[S][C];

    for (int h = 0; h < 2 * a.L; ++h) {
      const int e = half_parity(h, a.parity);
      const int n = half_size(a.N, e);
      const double* eps_slice = eps_r ? eps_r + (int64_t)(h >> 1) * a.N : nullptr;
      build_M<NW, S, C>(A, a, h, eps_slice, z, kbuf, sig, sm.wbuf + w * NP);
      __syncthreads();
      gj_invert<double, NW, S, C>(A, n, sm.colbuf, sm.wbuf, sm.pivrow, sm.pinv, &sm.flag);
      store_unpermuted<double, double, NW, S, C>(A, n, sm.wbuf, sm.pivrow, sm.pinv, kbuf,
                                                 h == 0 ? gbuf : nullptr);
      __syncthreads();
      if (h > 0) {
        const double t = a.t;
        auto fb = [&](int k, int c) -> cx<double> {
          return (c < n) ? ldg(kbuf + (size_t)c * NP + k) : mk(0.0, 0.0);
        };
        if (!(h & 1)) {
          auto fa = [&](int r, int k) -> cx<double> {
            return (r < n1) ? cscale(ldg(gbuf + (size_t)k * NP + r), t) : mk(0.0, 0.0);
          };
          gemm_regs<double, NW, S, C, KC>(A, n, fa, fb, sm.As, sm.Bs);
        } else {
          const int nL = half_size(a.N, e ^ 1);
          auto fa = [&](int r, int k) -> cx<double> {
            if (r >= n1) return mk(0.0, 0.0);
            const int k0 = nb_lo(k, e), k1 = nb_hi(k, e);
            cx<double> acc = mk(0.0, 0.0);
            if (k0 >= 0) acc = ldg(gbuf + (size_t)k0 * NP + r);
            if (k1 < nL) acc = cadd(acc, ldg(gbuf + (size_t)k1 * NP + r));
            return cscale(acc, t);
          };
          gemm_regs<double, NW, S, C, KC>(A, n, fa, fb, sm.As, sm.Bs);
        }
        store_regs<double, double, NW, S, C>(A, n1, n, gbuf);
        __syncthreads();
      }
    }

    // ---- trace: X = G Phi_R (n1 x P), then S = Phi_L^T X (P x P)
    {
      auto fa = [&](int r, int k) -> cx<double> {
        return (r < n1) ? ldg(gbuf + (size_t)k * NP + r) : mk(0.0, 0.0);
      };
      auto fb = [&](int k, int c) -> cx<double> {
        return (c < a.P) ? mk(phiR[(size_t)c * NP + k], 0.0) : mk(0.0, 0.0);
      };
      gemm_regs<double, NW, S, C, KC>(A, nlast, fa, fb, sm.As, sm.Bs);
      store_regs<double, double, NW, S, C>(A, n1, a.P, kbuf);
      __syncthreads();
    }
    double part = 0.0;
    {
      auto fa = [&](int r, int k) -> cx<double> {
        return (r < a.P) ? mk(phiL[(size_t)r * NP + k], 0.0) : mk(0.0, 0.0);
      };
      auto fb = [&](int k, int c) -> cx<double> {
        return (c < a.P) ? ldg(kbuf + (size_t)c * NP + k) : mk(0.0, 0.0);
      };
      gemm_regs<double, NW, S, C, KC>(A, n1, fa, fb, sm.As, sm.Bs);
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int p = lane + 64 * s;
        if (p >= a.P) continue;
        const double dp = -2.0 * sig[p].im;
#pragma unroll
        for (int j = 0; j < C; ++j) {
          const int q = w * C + j;
          if (q < a.P) {
            const double dq = -2.0 * sig[q].im;
            part += dp * dq * (A[s][j].re * A[s][j].re + A[s][j].im * A[s][j].im);
          }
        }
      }
    }
    const double T = block_sum<NW>(part, sm.red);
    if (threadIdx.x == 0) {
      int st = a.lstat[ee];
      if (st == RGF_TUPLE_OK && sm.flag) st = RGF_TUPLE_SINGULAR;
      if (st == RGF_TUPLE_OK && !isfinite(T)) st = RGF_TUPLE_NONFINITE;
      a.T_out[tau] = (st == RGF_TUPLE_OK) ? T : __builtin_nan("");
      if (a.status) a.status[tau] = st;
    }
    __syncthreads();
  }
}

using FwdKernel = void (*)(FwdArgs);

struct FwdEntry {
  int NW, S, C;
  FwdKernel k;
};

const FwdEntry kFwd[] = {
    {1, 1, 8, rgf_fwd_kernel<1, 1, 8>},    {1, 1, 16, rgf_fwd_kernel<1, 1, 16>},
    {2, 1, 16, rgf_fwd_kernel<2, 1, 16>},  {4, 1, 12, rgf_fwd_kernel<4, 1, 12>},
    {4, 1, 15, rgf_fwd_kernel<4, 1, 15>},  {4, 1, 16, rgf_fwd_kernel<4, 1, 16>},
    {8, 2, 12, rgf_fwd_kernel<8, 2, 12>},  {8, 2, 15, rgf_fwd_kernel<8, 2, 15>},
    {8, 2, 16, rgf_fwd_kernel<8, 2, 16>},
};

}  // namespace

bool pick_tile(int n, int precision, TileCfg* out) {
  (void)precision;
  for (int i = 0; i < (int)(sizeof(kFwd) / sizeof(kFwd[0])); ++i) {
    const FwdEntry& f = kFwd[i];
    if (f.NW * f.C >= n && 64 * f.S >= f.NW * f.C) {
      *out = TileCfg{i, f.NW, f.S, f.C};
      return true;
    }
  }
  return false;
}

int persistent_grid(const TileCfg& t, int64_t ntuples, int precision, bool grad) {
  (void)precision;
  (void)grad;
  int dev = 0, ncu = 256, occ = 1;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
    int o = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, (const void*)kFwd[t.id].k,
                                                     t.threads(), 0) == hipSuccess &&
        o > 0)
      occ = o;
  } else {
    (void)hipGetLastError();
  }
  int64_t g = (int64_t)ncu * occ;
  if (g > ntuples) g = ntuples;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t launch_forward(const Plan& p, const double* E, const double* eps, double* T_out,
                          int32_t* status_out, char* ws, hipStream_t s) {
  if (p.ntuples == 0) return hipSuccess;
  hipError_t err = launch_lead(p, E, ws, s);
  if (err != hipSuccess) return err;
  FwdArgs a;
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
  a.ntuples = p.ntuples;
  const FwdEntry& f = kFwd[p.tile.id];
  hipLaunchKernelGGL(f.k, dim3(p.grid), dim3(f.NW * 64), 0, s, a);
  return hipGetLastError();
}

}  // namespace rgf
