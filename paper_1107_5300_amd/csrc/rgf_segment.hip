// rgf_segment.hip -- the conductance recursion split along the ribbon length
// (parallel in L) for batches too small to fill the chip.
//
// The paper notes that parallelising the transport calculation needs a
// modification of the recursion, Eqs. (4)-(5) (timing discussion). Here the
// chain of 2L half-slices is cut into G segments of whole slices,
// half-slices [a_k, b_k] (a_k even: the L class of a slice; b_k odd: the R
// class of the segment's last slice), and each segment is solved on its
// own, every (tuple, segment) pair on a workgroup of its own.
//
// An isolated segment is a closed system whose Green's function has poles
// within eta of the real axis; solving it alone and joining would amplify
// rounding near every one of them. So each segment is closed at both ends
// by the self-energy Lambda of a semi-infinite pristine ribbon (the lead's,
// Phi diag(sigma) Phi^T; it depends only on the row class of the end, the
// two classes of N rows), which makes it an open system like the device
// between its leads. At the first and the last half-slice of the ribbon
// this is the true lead self-energy; at every cut the join takes it out
// again.
//
//   forward item (k):  the left-connected sweep of Eqs. (4)-(5) over the
//     closed segment, giving its corner blocks Rbb = G^k[b, b] (the last g)
//     and Rab = G^k[a, b] (the running product G1, Eq. (5));
//   backward item (k >= 1): the same sweep over the reversed segment (the
//     reversed ribbon is an armchair ribbon of parity (parity + L) mod 2
//     with the slices in reverse order), whose last g is Raa = G^k[a, a].
//
// The join (one workgroup per tuple) runs left to right. The joined part
// has the corners Lfb = G[first, b], Lbb = G[b, b] (b = b_{k-1}, closed by
// Lambda); the cut's row classes agree, so one Lambda serves both sides and
// the bond is t I. Dyson's equation (Eq. (3)) with the perturbation
// [[Lambda, -t], [-t, Lambda]] on (b, a_k) gives, by block elimination,
//   Q    = (I + Lambda Lbb)^{-1}
//   S    = I + Lambda Raa - t^2 Lbb Q Raa
//   Y    = S^{-1} (Lambda Rab - t^2 Lbb Q Rab)
//   Lfb' = t Lfb Q (Rab - Raa Y)
//   Lbb' = Rbb - Rab^T Y                    (Rba = Rab^T: G is complex symmetric)
// (with Lambda = 0 this is Lfb' = t Lfb (I - t^2 Raa Lbb)^{-1} Rab). After
// the last segment Lfb = G_{1L} and Eq. (2) gives T, as in the sequential
// sweep. Each item costs one segment sweep (the backward one without the G1
// products); a join costs about six half-slice steps. The accuracy guard
// sums the condition estimates of every inversion of the tuple; rejected
// tuples are recomputed by the whole-slice sweep, as in rgf_conductance.

#include <string.h>

#include "rgf_sweep.hpp"

namespace rgf {

namespace {

// One launch's view of the segment decomposition.
struct SegArgs {
  int G;                   // segments per tuple: segment k holds slices [k L / G, (k + 1) L / G)
  const double* phi2;      // [2][P][NP] mode tables of the two row classes (class 0, class 1)
  cx<double>* mats;        // [ntuples][G][3][NP*NP]: Rab, Rbb, Raa of each segment
  cx<double>* scratch;     // [join grid][6][NP*NP]: the join's work matrices
  double* kap;             // [ntuples][2G] (ksum, ksum_c) of each item, forward then backward
  int* flag;               // [ntuples][2G] exact-zero pivot seen by the item
  int64_t nitems;          // ntuples * (2G - 1)
};

__device__ __forceinline__ int seg_bound(const SegArgs& g, int L, int k) {
  return (int)((int64_t)k * L / g.G);
}

__device__ __forceinline__ cx<double>* seg_mat(const SegArgs& g, int64_t tau, int k, int which,
                                               size_t MAT) {
  return g.mats + ((size_t)tau * g.G + k) * 3 * MAT + (size_t)which * MAT;
}

// Item j of a tuple: j < G forward segment j, else backward segment j - G + 1.
template <int NW, int S, int C>
__global__ __launch_bounds__(NW * 64, NW >= 8 ? 2 : 3) void rgf_seg_sweep_kernel(
    SweepArgs a, SweepArgs ar, SegArgs g) {
  constexpr int NP = NW * C;
  constexpr size_t MAT = (size_t)NP * NP;
  __shared__ SweepSmem<NW, S, C> sm;
  const int H = 2 * a.L;
  const int per = 2 * g.G - 1;
  for (int64_t it = blockIdx.x; it < g.nitems; it += gridDim.x) {
    const int64_t tau = it / per;
    const int j = (int)(it - tau * per);
    const bool fwd = j < g.G;
    const int k = fwd ? j : j - g.G + 1;
    const int a_k = 2 * seg_bound(g, a.L, k), b_k = 2 * seg_bound(g, a.L, k + 1) - 1;
    const SweepArgs& A = fwd ? a : ar;
    Tuple q = make_tuple_(A, tau);
    q.hs = fwd ? a_k : H - 1 - b_k;
    q.he = fwd ? b_k : H - 1 - a_k;
    q.g1 = fwd;
    // both ends closed by the pristine self-energy of their row class
    q.phi_s = g.phi2 + (size_t)half_parity(q.hs, A.parity) * A.P * NP;
    q.phi_e = g.phi2 + (size_t)half_parity(q.he, A.parity) * A.P * NP;
    const int h1 = q.he;
    cx<double>* K = seg_mat(g, tau, k, fwd ? 1 : 2, MAT);
    cx<double>* G1 = fwd ? seg_mat(g, tau, k, 0, MAT) : nullptr;
    if (threadIdx.x == 0) {
      sm.flag = 0;
      sm.ksum = 0.0;
      sm.ksum_c = 0.0;
    }
    __syncthreads();
    cx<double> R[S][C];
    for (int h = q.hs; h <= h1; ++h)
      half_step<double, false, NW, S, C>(A, q, h, K, K, G1, G1, nullptr, R, sm);
    if (threadIdx.x == 0) {
      const int slot = fwd ? k : g.G + k;
      g.kap[(tau * 2 * g.G + slot) * 2] = sm.ksum;
      g.kap[(tau * 2 * g.G + slot) * 2 + 1] = sm.ksum_c;
      g.flag[tau * 2 * g.G + slot] = sm.flag;
    }
    __syncthreads();
  }
}

// W = X^{-1} for the n x n matrix X (column-major, leading dimension NP) in
// place, by the register Gauss-Jordan; returns max|(f X)^{-1}| (every
// thread), the condition estimate of the guard.
template <int NW, int S, int C>
__device__ __forceinline__ double invert_in_place(cx<double>* X, int n, cx<double> (&R)[S][C],
                                                  SweepSmem<NW, S, C>& sm) {
  constexpr int NP = NW * C;
  const int lane = lane_id(), w = wave_id();
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int c = w * C + j;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int r = lane + 64 * s;
      R[s][j] = (r < n && c < n) ? ldg(X + (size_t)c * NP + r) : mk((r == c) ? 1.0 : 0.0, 0.0);
    }
  }
  const double f = tile_scale<double, NW, S, C>(R, reinterpret_cast<uint32_t*>(sm.red));
  scale_regs(R, f);
  __syncthreads();  // every wave has read X before the inverse overwrites it
  gj_invert<double, NW, S, C>(R, n, sm.colbuf, sm.pivrow, sm.pinv, &sm.flag);
  const double km = tile_absmax_wave(R);
  store_unpermuted<double, double, NW, S, C>(R, n, f, sm.wbuf, sm.pivrow, sm.pinv, X, nullptr);
  if (lane == 0) sm.kred[w] = km;
  __syncthreads();
  double kap = sm.kred[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) kap = max(kap, sm.kred[i]);
  __syncthreads();  // kred is rewritten by the next inversion
  return kap;
}

// Join the segments of each tuple (one workgroup per tuple) and evaluate
// Eq. (2); flags the tuples the guard rejects for the whole-slice sweep.
template <int NW, int S, int C>
__global__ __launch_bounds__(NW * 64, NW >= 8 ? 2 : 3) void rgf_seg_join_kernel(
    SweepArgs a, SweepArgs ar, SegArgs g) {
  constexpr int NP = NW * C;
  constexpr size_t MAT = (size_t)NP * NP;
  __shared__ SweepSmem<NW, S, C> sm;
  const double t = a.t, t2 = a.t * a.t;
  const int n1 = half_size(a.N, half_parity(0, a.parity));
  cx<double>* X = g.scratch + (size_t)blockIdx.x * 6 * MAT;
  cx<double>* Lam = X;             // Lambda, later Y
  cx<double>* Qb = X + MAT;        // I + Lambda Lbb, then Q
  cx<double>* QRaa = X + 2 * MAT;  // Q Raa
  cx<double>* QRab = X + 3 * MAT;  // Q Rab, then Rab - Raa Y
  cx<double>* Sb = X + 4 * MAT;    // Lbb Q Raa, then S, then S^{-1}
  cx<double>* Rh = X + 5 * MAT;    // the right-hand side of Y
  auto delta = [](int r, int c) { return (r == c) ? 1.0 : 0.0; };
  for (int64_t tau = blockIdx.x; tau < a.ntuples; tau += gridDim.x) {
    const Tuple q = make_tuple_(a, tau);
    cx<double>* Lfb = seg_mat(g, tau, 0, 0, MAT);
    cx<double>* Lbb = seg_mat(g, tau, 0, 1, MAT);
    cx<double> R[S][C];
    double ksum = 0.0, ksum_c = 0.0;
    int flag = 0;
    for (int i = 0; i < 2 * g.G; ++i) {
      if (i == g.G) continue;  // segment 0 has no backward item
      ksum += g.kap[(tau * 2 * g.G + i) * 2];
      ksum_c += g.kap[(tau * 2 * g.G + i) * 2 + 1];
      flag |= g.flag[tau * 2 * g.G + i];
    }
    if (threadIdx.x == 0) sm.flag = 0;
    __syncthreads();
    for (int k = 1; k < g.G; ++k) {
      const cx<double>* Rab = seg_mat(g, tau, k, 0, MAT);
      const cx<double>* Rbb = seg_mat(g, tau, k, 1, MAT);
      const cx<double>* Raa = seg_mat(g, tau, k, 2, MAT);
      const int ha = 2 * seg_bound(g, a.L, k), hb = 2 * seg_bound(g, a.L, k + 1) - 1;
      const int ea = half_parity(ha, a.parity);
      const int n = half_size(a.N, ea);   // rows of b_{k-1} and a_k (the same class)
      const int nb = half_size(a.N, half_parity(hb, a.parity));
      const double* ph = g.phi2 + (size_t)ea * a.P * NP;
      // Lambda = Phi diag(sigma) Phi^T of the cut's row class
      {
        auto fa = [&](int r, int p) -> cx<double> { return cscale(q.sig[p], ph[(size_t)p * NP + r]); };
        auto fb = [&](int p, int c) -> cx<double> { return mk(ph[(size_t)p * NP + c], 0.0); };
        auto epi = [&](int r, int c, cx<double> v, bool ok) {
          if (ok) stg(Lam + (size_t)c * NP + r, v);
        };
        gemm_mfma<NW, NP>(n, n, a.P, fa, fb, epi);
      }
      __syncthreads();
      auto mul = [&](const cx<double>* A_, const cx<double>* B_, int nr, int nc, int nk,
                     auto epi) {
        auto fa = [&](int r, int kk) -> cx<double> { return ldg(A_ + (size_t)kk * NP + r); };
        auto fb = [&](int kk, int c) -> cx<double> { return ldg(B_ + (size_t)c * NP + kk); };
        gemm_mfma<NW, NP>(nr, nc, nk, fa, fb, epi);
        __syncthreads();
      };
      // Q = (I + Lambda Lbb)^{-1}
      mul(Lam, Lbb, n, n, n, [&](int r, int c, cx<double> v, bool ok) {
        if (ok) stg(Qb + (size_t)c * NP + r, mk(delta(r, c) + v.re, v.im));
      });
      ksum += invert_in_place<NW, S, C>(Qb, n, R, sm);
      // Q Raa, Q Rab
      mul(Qb, Raa, n, n, n, [&](int r, int c, cx<double> v, bool ok) {
        if (ok) stg(QRaa + (size_t)c * NP + r, v);
      });
      mul(Qb, Rab, n, nb, n, [&](int r, int c, cx<double> v, bool ok) {
        if (ok) stg(QRab + (size_t)c * NP + r, v);
      });
      // S = I + Lambda Raa - t^2 Lbb (Q Raa)
      mul(Lbb, QRaa, n, n, n, [&](int r, int c, cx<double> v, bool ok) {
        if (ok) stg(Sb + (size_t)c * NP + r, v);
      });
      mul(Lam, Raa, n, n, n, [&](int r, int c, cx<double> v, bool ok) {
        if (!ok) return;
        const cx<double> w = ldg(Sb + (size_t)c * NP + r);
        stg(Sb + (size_t)c * NP + r, mk(delta(r, c) + v.re - t2 * w.re, v.im - t2 * w.im));
      });
      ksum += invert_in_place<NW, S, C>(Sb, n, R, sm);
      // right-hand side Lambda Rab - t^2 Lbb (Q Rab)
      mul(Lbb, QRab, n, nb, n, [&](int r, int c, cx<double> v, bool ok) {
        if (ok) stg(Rh + (size_t)c * NP + r, v);
      });
      mul(Lam, Rab, n, nb, n, [&](int r, int c, cx<double> v, bool ok) {
        if (!ok) return;
        const cx<double> w = ldg(Rh + (size_t)c * NP + r);
        stg(Rh + (size_t)c * NP + r, mk(v.re - t2 * w.re, v.im - t2 * w.im));
      });
      // Y = S^{-1} (right-hand side), into Lambda's buffer
      mul(Sb, Rh, n, nb, n, [&](int r, int c, cx<double> v, bool ok) {
        if (ok) stg(Lam + (size_t)c * NP + r, v);
      });
      // Lbb' = Rbb - Rab^T Y (Lbb is not read again in this step)
      {
        auto fa = [&](int r, int kk) -> cx<double> { return ldg(Rab + (size_t)r * NP + kk); };
        auto fb = [&](int kk, int c) -> cx<double> { return ldg(Lam + (size_t)c * NP + kk); };
        auto epi = [&](int r, int c, cx<double> v, bool ok) {
          if (ok) stg(Lbb + (size_t)c * NP + r, csub(ldg(Rbb + (size_t)c * NP + r), v));
        };
        gemm_mfma<NW, NP>(nb, nb, n, fa, fb, epi);
        __syncthreads();
      }
      // Z = Q Rab - Q Raa Y (in place), then Lfb' = t Lfb Z
      mul(QRaa, Lam, n, nb, n, [&](int r, int c, cx<double> v, bool ok) {
        if (ok) stg(QRab + (size_t)c * NP + r, csub(ldg(QRab + (size_t)c * NP + r), v));
      });
      mul(Lfb, QRab, n1, nb, n, [&](int r, int c, cx<double> v, bool ok) {
        if (ok) stg(Lfb + (size_t)c * NP + r, cscale(v, t));
      });
    }
    // Eq. (2) from G_{1L} = Lfb (the trace's scratch: Lambda's buffer)
    const double T = trace_T<NW, S, C>(a, q, Lfb, Lam, R, sm);
    if (threadIdx.x == 0) {
      int st = a.lstat[q.e];
      if (st == RGF_TUPLE_OK && ill_conditioned(ksum, ksum_c)) st = RGF_TUPLE_ILL_CONDITIONED;
      if (st == RGF_TUPLE_OK && (flag || sm.flag)) st = RGF_TUPLE_SINGULAR;
      if (st == RGF_TUPLE_OK && !isfinite(T)) st = RGF_TUPLE_NONFINITE;
      if (st == RGF_TUPLE_OK && !t_in_range(T, a.P)) st = RGF_TUPLE_OUT_OF_RANGE;
      a.T_out[tau] = (st == RGF_TUPLE_OK) ? T : __builtin_nan("");
      if (a.status) a.status[tau] = st;
      if (a.fb_flags) a.fb_flags[tau] = (st == RGF_TUPLE_ILL_CONDITIONED) ? 1 : 0;
    }
    __syncthreads();
  }
}

// Reverse the slice order of the on-site energies: out[r][L-1-i][k] = in[r][i][k].
__global__ void reverse_slices_kernel(const double* in, double* out, int64_t nreal, int L,
                                      int N) {
  const int64_t total = nreal * (int64_t)L * N;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = x / ((int64_t)L * N);
    const int64_t rem = x - r * L * N;
    const int i = (int)(rem / N), k = (int)(rem - (int64_t)i * N);
    out[(r * L + (L - 1 - i)) * N + k] = in[x];
  }
}

struct SegEntry {
  int NW, S, C;
  void (*sweep)(SweepArgs, SweepArgs, SegArgs);
  void (*join)(SweepArgs, SweepArgs, SegArgs);
};

#define RGF_SEG_ENTRY(NW, S, C) \
  { NW, S, C, rgf_seg_sweep_kernel<NW, S, C>, rgf_seg_join_kernel<NW, S, C> }

const SegEntry kSeg[] = {
    RGF_SEG_ENTRY(1, 1, 8),  RGF_SEG_ENTRY(1, 1, 16), RGF_SEG_ENTRY(2, 1, 16),
    RGF_SEG_ENTRY(4, 1, 12), RGF_SEG_ENTRY(4, 1, 15), RGF_SEG_ENTRY(4, 1, 16),
    RGF_SEG_ENTRY(8, 1, 8),  RGF_SEG_ENTRY(8, 2, 12), RGF_SEG_ENTRY(8, 2, 15),
    RGF_SEG_ENTRY(8, 2, 16),
};

const SegEntry* seg_entry(const TileCfg& t) {
  for (const SegEntry& e : kSeg)
    if (e.NW == t.NW && e.S == t.S && e.C == t.C) return &e;
  return nullptr;
}

SweepArgs base_args(const Plan& p, const double* E, const double* eps, double* T_out,
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
  a.phi_ld = p.phi_ld;
  return a;
}

}  // namespace

bool seg_supported(const TileCfg& t) { return seg_entry(t) != nullptr; }

const void* seg_sweep_kernel(const TileCfg& t) {
  const SegEntry* e = seg_entry(t);
  return e ? reinterpret_cast<const void*>(e->sweep) : nullptr;
}

hipError_t launch_segments(const SegPlan& sp, const double* E, const double* eps,
                           double* T_out, int32_t* status_out, char* ws, hipStream_t s) {
  const Plan& p = sp.fwd;
  if (p.ntuples == 0) return hipSuccess;
  const SegEntry* f = seg_entry(p.tile);
  if (!f) return hipErrorInvalidValue;
  char* wx = ws + sp.off_aux;  // mode tables of both row classes (and their sigma)
  hipError_t err = launch_lead(p, E, ws, s);
  if (err == hipSuccess) err = launch_lead(sp.aux, E, wx, s);
  if (err != hipSuccess) return err;
  double* eps_rev = nullptr;
  if (eps) {
    eps_rev = reinterpret_cast<double*>(ws + sp.off_eps_rev);
    const int64_t total = p.nreal * (int64_t)p.L * p.N;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(reverse_slices_kernel, dim3(blocks), dim3(256), 0, s, eps, eps_rev,
                       p.nreal, p.L, p.N);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  SweepArgs a = base_args(p, E, eps, T_out, status_out, ws);
  a.fb_flags = p.fb_grid > 0 ? reinterpret_cast<int32_t*>(ws + p.off_flags) : nullptr;
  // the reversed ribbon: parity (parity + L) mod 2, slices reversed
  SweepArgs ar = base_args(sp.aux, E, eps_rev, nullptr, nullptr, wx);
  ar.L = p.L;
  ar.parity = (p.parity + p.L) & 1;
  ar.nreal = p.nreal;
  ar.ntuples = p.ntuples;
  SegArgs g;
  g.G = sp.G;
  g.phi2 = reinterpret_cast<const double*>(wx + sp.aux.off_phi);
  g.mats = reinterpret_cast<cx<double>*>(ws + sp.off_mats);
  g.scratch = reinterpret_cast<cx<double>*>(ws + sp.off_scratch);
  g.kap = reinterpret_cast<double*>(ws + sp.off_kap);
  g.flag = reinterpret_cast<int*>(ws + sp.off_flag);
  g.nitems = p.ntuples * (2 * (int64_t)sp.G - 1);
  hipLaunchKernelGGL(f->sweep, dim3(sp.sweep_grid), dim3(f->NW * 64), 0, s, a, ar, g);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  hipLaunchKernelGGL(f->join, dim3(sp.join_grid), dim3(f->NW * 64), 0, s, a, ar, g);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  if (!a.fb_flags) return hipSuccess;
  return launch_whole_fallback(p, a, ws, s);
}

}  // namespace rgf
