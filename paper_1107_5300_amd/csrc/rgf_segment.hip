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
// The joins run as a tree: at level l (l = 1, 2, ...) the part made of
// segments [j 2^l, j 2^l + 2^(l-1)) merges with the part that follows it,
// every (tuple, pair) on a workgroup of its own, so a tuple's G segments
// are joined in ceil(log2 G) levels. A part has the corners Paa, Pab, Pbb
// of its Green's function (Pba = Pab^T: G is complex symmetric) with both
// ends closed by Lambda. At the cut between P's last half-slice b and Q's
// first a the row classes agree, so one Lambda serves both sides and the
// bond is t I. Dyson's equation (Eq. (3)) with the perturbation
// [[Lambda, -t], [-t, Lambda]] on (b, a), solved by block elimination:
//   Q1   = (I + Lambda Pbb)^{-1},   S = I + Lambda Qaa - t^2 Pbb Q1 Qaa
//   Y    = S^{-1} (Lambda Qab - t^2 Pbb Q1 Qab)
//   Rab  = t Pab Q1 (Qab - Qaa Y),  Rbb = Qbb - Qab^T Y
//   Y2   = S^{-1} t (Pbb Q1 Lambda Pba - Pba)
//   Raa  = Paa - Pab Q1 (Lambda Pba + t Qaa Y2)     (not for the leftmost part)
// (with Lambda = 0, Rab = t Pab (I - t^2 Qaa Pbb)^{-1} Qab). After the last
// level the part of all segments has Rab = G_{1L}, and Eq. (2) gives T as in
// the sequential sweep. Each item costs one segment sweep (the backward one
// without the G1 products); a merge costs about eight half-slice steps. The
// accuracy guard sums the condition estimates of every inversion of the
// tuple; rejected tuples are recomputed by the whole-slice sweep, as in
// rgf_conductance.

#include <string.h>

#include "rgf_segplan.hpp"
#include "rgf_sweep.hpp"

namespace rgf {

namespace {

// One launch's view of the segment decomposition.
struct SegArgs {
  int G;                   // segments per tuple: segment k holds slices [k L / G, (k + 1) L / G)
  const double* phi2;      // [2][P][NP] mode tables of the two row classes (class 0, class 1)
  cx<double>* mats;        // [ntuples][G][3][NP*NP]: Rab, Rbb, Raa of each segment (of each
                           // part after the merges, at the part's first segment)
  cx<double>* scratch;     // [merge grid][8][NP*NP]: a merge's work matrices
  double* kap;             // [ntuples][3G][2] (ksum, ksum_c): forward items, backward items,
                           // merges (by the first segment of the right part)
  int* flag;               // [ntuples][3G] exact-zero pivot seen by the item
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
      g.kap[(tau * 3 * g.G + slot) * 2] = sm.ksum;
      g.kap[(tau * 3 * g.G + slot) * 2 + 1] = sm.ksum_c;
      g.flag[tau * 3 * g.G + slot] = sm.flag;
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

// Level `level` of the tree of joins: item (tuple, j) merges the part that
// starts at segment j 2^level with the one at j 2^level + 2^(level-1),
// writing the merged corners over the left part's.
template <int NW, int S, int C>
__global__ __launch_bounds__(NW * 64, NW >= 8 ? 2 : 3) void rgf_seg_merge_kernel(
    SweepArgs a, SegArgs g, int level) {
  constexpr int NP = NW * C;
  constexpr size_t MAT = (size_t)NP * NP;
  __shared__ SweepSmem<NW, S, C> sm;
  const double t = a.t, t2 = a.t * a.t;
  const int half = 1 << (level - 1), span = 2 * half;
  const int npairs = (g.G - half + span - 1) / span;   // pairs whose right part exists
  cx<double>* X = g.scratch + (size_t)blockIdx.x * 8 * MAT;
  cx<double>* Lam = X;              // Lambda
  cx<double>* Q1 = X + MAT;         // I + Lambda Pbb, then Q1
  cx<double>* Q1Qaa = X + 2 * MAT;
  cx<double>* Zb = X + 3 * MAT;     // Q1 Qab, then Z = Q1 Qab - Q1 Qaa Y
  cx<double>* Sb = X + 4 * MAT;     // Pbb Q1 Qaa, then S, then S^{-1}
  cx<double>* Yb = X + 5 * MAT;     // Pbb Q1 Qab, then the right-hand side, then Y
  cx<double>* U = X + 6 * MAT;      // Lambda Pba, then Lambda Pba + t Qaa Y2
  cx<double>* V = X + 7 * MAT;      // Q1 Lambda Pba, then the right-hand side of Y2, Y2, Q1 (..)
  auto delta = [](int r, int c) { return (r == c) ? 1.0 : 0.0; };
  for (int64_t it = blockIdx.x; it < a.ntuples * (int64_t)npairs; it += gridDim.x) {
    const int64_t tau = it / npairs;
    const int left = (int)(it - tau * npairs) * span, right = left + half;
    const int qend = min(right + half, g.G);        // Q holds segments [right, qend)
    const Tuple q = make_tuple_(a, tau);
    cx<double>* Pab = seg_mat(g, tau, left, 0, MAT);
    cx<double>* Pbb = seg_mat(g, tau, left, 1, MAT);
    cx<double>* Paa = seg_mat(g, tau, left, 2, MAT);
    const cx<double>* Qab = seg_mat(g, tau, right, 0, MAT);
    const cx<double>* Qbb = seg_mat(g, tau, right, 1, MAT);
    const cx<double>* Qaa = seg_mat(g, tau, right, 2, MAT);
    const int ha = 2 * seg_bound(g, a.L, right);
    const int ec = half_parity(ha, a.parity);
    const int n = half_size(a.N, ec);      // rows at the cut (both sides)
    const int npa = half_size(a.N, half_parity(2 * seg_bound(g, a.L, left), a.parity));
    const int nqb = half_size(a.N, half_parity(2 * seg_bound(g, a.L, qend) - 1, a.parity));
    const double* ph = g.phi2 + (size_t)ec * a.P * NP;
    cx<double> R[S][C];
    if (threadIdx.x == 0) sm.flag = 0;
    __syncthreads();
    auto mul = [&](const cx<double>* A_, const cx<double>* B_, int nr, int nc, int nk,
                   auto epi) {
      auto fa = [&](int r, int kk) -> cx<double> { return ldg(A_ + (size_t)kk * NP + r); };
      auto fb = [&](int kk, int c) -> cx<double> { return ldg(B_ + (size_t)c * NP + kk); };
      gemm_mfma<NW, NP>(nr, nc, nk, fa, fb, epi);
      __syncthreads();
    };
    auto put = [](cx<double>* D) {
      return [D](int r, int c, cx<double> v, bool ok) {
        if (ok) stg(D + (size_t)c * NP + r, v);
      };
    };
    // Lambda = Phi diag(sigma) Phi^T of the cut's row class
    {
      auto fa = [&](int r, int p) -> cx<double> { return cscale(q.sig[p], ph[(size_t)p * NP + r]); };
      auto fb = [&](int p, int c) -> cx<double> { return mk(ph[(size_t)p * NP + c], 0.0); };
      gemm_mfma<NW, NP>(n, n, a.P, fa, fb, put(Lam));
      __syncthreads();
    }
    double ksum = 0.0;
    // Q1 = (I + Lambda Pbb)^{-1}
    mul(Lam, Pbb, n, n, n, [&](int r, int c, cx<double> v, bool ok) {
      if (ok) stg(Q1 + (size_t)c * NP + r, mk(delta(r, c) + v.re, v.im));
    });
    ksum += invert_in_place<NW, S, C>(Q1, n, R, sm);
    mul(Q1, Qaa, n, n, n, put(Q1Qaa));
    mul(Q1, Qab, n, nqb, n, put(Zb));
    // S = I + Lambda Qaa - t^2 Pbb Q1 Qaa, inverted
    mul(Pbb, Q1Qaa, n, n, n, put(Sb));
    mul(Lam, Qaa, n, n, n, [&](int r, int c, cx<double> v, bool ok) {
      if (!ok) return;
      const cx<double> w = ldg(Sb + (size_t)c * NP + r);
      stg(Sb + (size_t)c * NP + r, mk(delta(r, c) + v.re - t2 * w.re, v.im - t2 * w.im));
    });
    ksum += invert_in_place<NW, S, C>(Sb, n, R, sm);
    // Y = S^{-1} (Lambda Qab - t^2 Pbb Q1 Qab)
    mul(Pbb, Zb, n, nqb, n, put(Yb));
    mul(Lam, Qab, n, nqb, n, [&](int r, int c, cx<double> v, bool ok) {
      if (!ok) return;
      const cx<double> w = ldg(Yb + (size_t)c * NP + r);
      stg(Yb + (size_t)c * NP + r, mk(v.re - t2 * w.re, v.im - t2 * w.im));
    });
    mul(Sb, Yb, n, nqb, n, put(Yb));
    if (left > 0) {
      // Raa = Paa - Pab Q1 (Lambda Pba + t Qaa Y2),
      // Y2 = S^{-1} t (Pbb Q1 Lambda Pba - Pba)
      {
        auto fa = [&](int r, int kk) -> cx<double> { return ldg(Lam + (size_t)kk * NP + r); };
        auto fb = [&](int kk, int c) -> cx<double> { return ldg(Pab + (size_t)kk * NP + c); };
        gemm_mfma<NW, NP>(n, npa, n, fa, fb, put(U));   // Lambda Pba (Pba[k][c] = Pab[c][k])
        __syncthreads();
      }
      mul(Q1, U, n, npa, n, put(V));
      mul(Pbb, V, n, npa, n, [&](int r, int c, cx<double> v, bool ok) {
        if (!ok) return;
        const cx<double> pba = ldg(Pab + (size_t)r * NP + c);   // Pba[r][c]
        stg(V + (size_t)c * NP + r, mk(t * (v.re - pba.re), t * (v.im - pba.im)));
      });
      mul(Sb, V, n, npa, n, put(V));                             // Y2
      mul(Qaa, V, n, npa, n, [&](int r, int c, cx<double> v, bool ok) {
        if (ok) stg(U + (size_t)c * NP + r, cadd(ldg(U + (size_t)c * NP + r), cscale(v, t)));
      });
      mul(Q1, U, n, npa, n, put(V));
      mul(Pab, V, npa, npa, n, [&](int r, int c, cx<double> v, bool ok) {
        if (ok) stg(Paa + (size_t)c * NP + r, csub(ldg(Paa + (size_t)c * NP + r), v));
      });
    }
    // Z = Q1 Qab - Q1 Qaa Y, then Rbb = Qbb - Qab^T Y (over Pbb), Rab = t Pab Z (over Pab)
    mul(Q1Qaa, Yb, n, nqb, n, [&](int r, int c, cx<double> v, bool ok) {
      if (ok) stg(Zb + (size_t)c * NP + r, csub(ldg(Zb + (size_t)c * NP + r), v));
    });
    {
      auto fa = [&](int r, int kk) -> cx<double> { return ldg(Qab + (size_t)r * NP + kk); };
      auto fb = [&](int kk, int c) -> cx<double> { return ldg(Yb + (size_t)c * NP + kk); };
      auto epi = [&](int r, int c, cx<double> v, bool ok) {
        if (ok) stg(Pbb + (size_t)c * NP + r, csub(ldg(Qbb + (size_t)c * NP + r), v));
      };
      gemm_mfma<NW, NP>(nqb, nqb, n, fa, fb, epi);
      __syncthreads();
    }
    mul(Pab, Zb, npa, nqb, n, [&](int r, int c, cx<double> v, bool ok) {
      if (ok) stg(Pab + (size_t)c * NP + r, cscale(v, t));
    });
    if (threadIdx.x == 0) {
      g.kap[(tau * 3 * g.G + 2 * g.G + right) * 2] = ksum;
      g.kap[(tau * 3 * g.G + 2 * g.G + right) * 2 + 1] = 0.0;
      g.flag[tau * 3 * g.G + 2 * g.G + right] = sm.flag;
    }
    __syncthreads();
  }
}

// Eq. (2) from the merged part (one workgroup per tuple) and the status of
// the tuple; flags the tuples the guard rejects for the whole-slice sweep.
template <int NW, int S, int C>
__global__ __launch_bounds__(NW * 64, NW >= 8 ? 2 : 3) void rgf_seg_join_kernel(
    SweepArgs a, SweepArgs ar, SegArgs g) {
  constexpr int NP = NW * C;
  constexpr size_t MAT = (size_t)NP * NP;
  __shared__ SweepSmem<NW, S, C> sm;
  for (int64_t tau = blockIdx.x; tau < a.ntuples; tau += gridDim.x) {
    const Tuple q = make_tuple_(a, tau);
    cx<double> R[S][C];
    double ksum = 0.0, ksum_c = 0.0;
    int flag = 0;
    for (int i = 0; i < 3 * g.G; ++i) {
      if (i == g.G || i == 2 * g.G) continue;  // no backward item for segment 0, no merge at 0
      ksum += g.kap[(tau * 3 * g.G + i) * 2];
      ksum_c += g.kap[(tau * 3 * g.G + i) * 2 + 1];
      flag |= g.flag[tau * 3 * g.G + i];
    }
    // G_{1L} = Rab of the part of all segments (the trace's scratch: its Rbb)
    const double T = trace_T<NW, S, C>(a, q, seg_mat(g, tau, 0, 0, MAT),
                                       seg_mat(g, tau, 0, 1, MAT), R, sm);
    if (threadIdx.x == 0) {
      int st = a.lstat[q.e];
      if (st == RGF_TUPLE_OK && ill_conditioned(ksum, ksum_c)) st = RGF_TUPLE_ILL_CONDITIONED;
      if (st == RGF_TUPLE_OK && flag) st = RGF_TUPLE_SINGULAR;
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
  void (*merge)(SweepArgs, SegArgs, int);
  void (*join)(SweepArgs, SweepArgs, SegArgs);
};

#define RGF_SEG_ENTRY(NW, S, C)                                                 \
  {                                                                             \
    NW, S, C, rgf_seg_sweep_kernel<NW, S, C>, rgf_seg_merge_kernel<NW, S, C>,   \
        rgf_seg_join_kernel<NW, S, C>                                           \
  }

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
  for (int level = 1; (1 << (level - 1)) < sp.G; ++level) {
    const int half = 1 << (level - 1);
    const int64_t items = p.ntuples * (int64_t)((sp.G - half + 2 * half - 1) / (2 * half));
    const int grid = (int)std::min<int64_t>(items, sp.merge_grid);
    hipLaunchKernelGGL(f->merge, dim3(grid), dim3(f->NW * 64), 0, s, a, g, level);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  hipLaunchKernelGGL(f->join, dim3(sp.join_grid), dim3(f->NW * 64), 0, s, a, ar, g);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  if (!a.fb_flags) return hipSuccess;
  return launch_whole_fallback(p, a, ws, s);
}

}  // namespace rgf
