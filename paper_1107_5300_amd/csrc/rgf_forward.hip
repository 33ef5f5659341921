// rgf_forward.hip -- forward RGF sweep and conductance trace.
//
// One persistent workgroup walks the 2L half-slices of one (realization,
// energy) tuple at a time (the recursion is serial in the ribbon length) and
// takes the next tuple when done; tuples are independent. The half-slice
// step and the trace live in rgf_sweep.hpp.
//
// Per-slot global scratch (column-major, ld = NP, complex128): K (the latest
// g_h) and G1; the refined mode adds a second K (ping-pong) and the residual.
// A slot stays L2/MALL-resident while its workgroup runs.

#include <string.h>

#include "rgf_sweep.hpp"

namespace rgf {

namespace {

// Register budget: an 8-wave workgroup holds two waves per SIMD (one
// workgroup per compute unit); narrower tilings ask for three waves per SIMD
// (two with the refinement's extra tiles) so that several workgroups share a
// compute unit and hide each other's barrier and memory latency.
// CHAN: also write the transmission per incoming lead channel (a.tchan).
template <typename TJ, bool REFINE, int NW, int S, int C, bool CHAN = false>
__global__ __launch_bounds__(NW * 64, NW >= 8 ? 2 : (REFINE ? 2 : 3)) void rgf_fwd_kernel(
    SweepArgs a) {
  constexpr int NP = NW * C;
  // the accuracy guard covers the FP64 and mixed modes (not the FP32 study)
  constexpr bool GUARD = sizeof(TJ) == sizeof(double) || REFINE;
  __shared__ SweepSmem<NW, S, C> sm;
  cx<double>* slot = a.slots + (size_t)blockIdx.x * a.slot_mats * NP * NP;
  cx<double>* kb[2] = {slot, REFINE ? slot + (size_t)3 * NP * NP : slot};
  cx<double>* gbuf = slot + (size_t)NP * NP;
  cx<double>* rbuf = slot + (size_t)2 * NP * NP;
  if (threadIdx.x == 0) sm.rf[0] = sm.rf[1] = sm.rf[2] = 0u;

  for (int64_t tau = blockIdx.x; tau < a.ntuples; tau += gridDim.x) {
    const Tuple q = make_tuple_(a, tau);
    if (threadIdx.x == 0) {
      sm.flag = 0;
      sm.ksum = 0.0;
      sm.ksum_c = 0.0;
    }
    __syncthreads();
    cx<double> A[S][C];
    for (int h = 0; h < 2 * a.L; ++h) {
      half_step<TJ, REFINE, NW, S, C>(a, q, h, kb[(h + 1) & 1], kb[h & 1], gbuf, gbuf, rbuf,
                                      A, sm);
    }
    const double T = trace_T<NW, S, C>(a, q, gbuf, rbuf, A, sm, CHAN);
    if (CHAN || threadIdx.x == 0) {
      int st = a.lstat[q.e];
      // the guard first: a rejected sweep may also show a zero pivot or a T
      // out of range, and the whole-slice sweep recomputes it
      if (GUARD && st == RGF_TUPLE_OK && ill_conditioned(sm.ksum, sm.ksum_c))
        st = RGF_TUPLE_ILL_CONDITIONED;
      if (st == RGF_TUPLE_OK && sm.flag) st = RGF_TUPLE_SINGULAR;
      if (st == RGF_TUPLE_OK && !isfinite(T)) st = RGF_TUPLE_NONFINITE;
      if (st == RGF_TUPLE_OK && !t_in_range(T, a.P)) st = RGF_TUPLE_OUT_OF_RANGE;
      if (threadIdx.x == 0) {
        a.T_out[tau] = (st == RGF_TUPLE_OK) ? T : __builtin_nan("");
        if (a.status) a.status[tau] = st;
        // the whole-slice sweep recomputes the tuples the guard rejected
        if (a.fb_flags) a.fb_flags[tau] = (st == RGF_TUPLE_ILL_CONDITIONED) ? 1 : 0;
      }
      if constexpr (CHAN) {  // T_p = d_p sum_q d_q |S_pq|^2 (block_sum's barriers order rowacc)
        for (int p = threadIdx.x; p < a.P; p += NW * 64)
          a.tchan[tau * a.P + p] =
              (st == RGF_TUPLE_OK) ? -2.0 * q.sig[p].im * sm.rowacc[p] : __builtin_nan("");
      }
    }
    __syncthreads();
  }
  if constexpr (REFINE) flush_refine_stats(a, sm);
}

// The sweep with the matrix-core Gauss-Jordan (rgf_mgj.hpp) for half-slices
// of up to 128 rows: one 8-wave workgroup per compute unit, the (8, 2, 16)
// tiling for the trace.
template <typename TJ, bool REFINE>
__global__ __launch_bounds__(512, 1) void rgf_fwd_mgj_kernel(SweepArgs a) {
  constexpr int NW = 8, S = 2, C = 16, NP = NW * C;
  __shared__ SweepSmem<NW, S, C> sm;
  __shared__ MgjSmem<double> ms;  // the FP32 inversion uses it as MgjSmem<float>
  cx<double>* slot = a.slots + (size_t)blockIdx.x * a.slot_mats * NP * NP;
  cx<double>* kb[2] = {slot, REFINE ? slot + (size_t)3 * NP * NP : slot};
  cx<double>* gbuf = slot + (size_t)NP * NP;
  cx<double>* rbuf = slot + (size_t)2 * NP * NP;
  cx<double>* mbuf = REFINE ? slot + (size_t)4 * NP * NP : nullptr;  // M_h in FP64
  if (threadIdx.x == 0) sm.rf[0] = sm.rf[1] = sm.rf[2] = 0u;

  for (int64_t tau = blockIdx.x; tau < a.ntuples; tau += gridDim.x) {
    const Tuple q = make_tuple_(a, tau);
    if (threadIdx.x == 0) {
      sm.flag = 0;
      sm.ksum = 0.0;
      sm.ksum_c = 0.0;
    }
    __syncthreads();
    for (int h = 0; h < 2 * a.L; ++h)
      half_step_mgj<TJ, REFINE>(a, q, h, kb[(h + 1) & 1], kb[h & 1], gbuf, gbuf, rbuf, mbuf, sm,
                                ms);
    cx<double> A[S][C];
    const double T = trace_T<NW, S, C>(a, q, gbuf, rbuf, A, sm);
    if (threadIdx.x == 0) {
      int st = a.lstat[q.e];
      if (st == RGF_TUPLE_OK && ill_conditioned(sm.ksum, sm.ksum_c))
        st = RGF_TUPLE_ILL_CONDITIONED;
      if (st == RGF_TUPLE_OK && sm.flag) st = RGF_TUPLE_SINGULAR;
      if (st == RGF_TUPLE_OK && !isfinite(T)) st = RGF_TUPLE_NONFINITE;
      if (st == RGF_TUPLE_OK && !t_in_range(T, a.P)) st = RGF_TUPLE_OUT_OF_RANGE;
      a.T_out[tau] = (st == RGF_TUPLE_OK) ? T : __builtin_nan("");
      if (a.status) a.status[tau] = st;
      if (a.fb_flags) a.fb_flags[tau] = (st == RGF_TUPLE_ILL_CONDITIONED) ? 1 : 0;
    }
    __syncthreads();
  }
  if constexpr (REFINE) flush_refine_stats(a, sm);
}

using FwdKernel = void (*)(SweepArgs);

struct FwdEntry {
  int NW, S, C;
  FwdKernel k[3];  // by precision: FP64, MIXED, FP32
  FwdKernel chan;  // FP64 with the per-channel transmission
  bool mgj;        // matrix-core Gauss-Jordan (FP64 and mixed)
};

#define RGF_FWD_ENTRY(NW, S, C)                                              \
  {                                                                          \
    NW, S, C,                                                                \
        {rgf_fwd_kernel<double, false, NW, S, C>,                            \
         rgf_fwd_kernel<float, true, NW, S, C>,                              \
         rgf_fwd_kernel<float, false, NW, S, C>},                            \
        rgf_fwd_kernel<double, false, NW, S, C, true>, false                 \
  }

const FwdEntry kFwd[] = {
    RGF_FWD_ENTRY(1, 1, 8),  RGF_FWD_ENTRY(1, 1, 16), RGF_FWD_ENTRY(2, 1, 16),
    RGF_FWD_ENTRY(4, 1, 12), RGF_FWD_ENTRY(4, 1, 15), RGF_FWD_ENTRY(4, 1, 16),
    RGF_FWD_ENTRY(8, 1, 8),  RGF_FWD_ENTRY(8, 2, 12), RGF_FWD_ENTRY(8, 2, 15), RGF_FWD_ENTRY(8, 2, 16),
    // matrix-core Gauss-Jordan for 96 < n <= 128 (the FP32 study mode and the
    // per-channel transmission keep the register tiling's kernels)
    {8, 2, 16,
     {rgf_fwd_mgj_kernel<double, false>, rgf_fwd_mgj_kernel<float, true>,
      rgf_fwd_kernel<float, false, 8, 2, 16>},
     rgf_fwd_kernel<double, false, 8, 2, 16, true>, true},
};

}  // namespace

int slot_matrices(int precision, bool grad) {
  // forward: K, G1, residual/trace scratch (+ second K and M_h when
  // refining); adjoint adds Z, Q and one more scratch
  if (grad) return 7;
  return precision == RGF_PREC_MIXED ? 5 : 3;
}

int tile_count() { return (int)(sizeof(kFwd) / sizeof(kFwd[0])); }

TileCfg tile_at(int i) { return TileCfg{i, kFwd[i].NW, kFwd[i].S, kFwd[i].C, kFwd[i].mgj}; }

bool pick_tile(int n, int precision, TileCfg* out) {
  int tid = 0, per_cu = 0;
  if (tuned_choice(n, precision, &tid, &per_cu)) {
    *out = tile_at(tid);
    return true;
  }
  // mixed precision above 96 rows: the matrix-core Gauss-Jordan in FP32 (it
  // pads to 128 rows); FP64 and the FP32 study keep the smallest register
  // tiling that holds n (in FP64 the register elimination is faster: the
  // blocked version's serial panel eliminations set its pace)
  const bool mgj = n > 96 && n <= kTileMaxRows && precision == RGF_PREC_MIXED;
  for (int i = 0; i < (int)(sizeof(kFwd) / sizeof(kFwd[0])); ++i) {
    const FwdEntry& f = kFwd[i];
    if (f.mgj == mgj && f.NW * f.C >= n && 64 * f.S >= f.NW * f.C) {
      *out = tile_at(i);
      return true;
    }
  }
  return false;
}

const void* fwd_kernel_ptr(const TileCfg& t, int precision) {
  return (const void*)kFwd[t.id].k[precision];
}

hipError_t launch_forward(const Plan& p, const double* E, const double* eps, double* T_out,
                          int32_t* status_out, char* ws, hipStream_t s, double* tchan) {
  if (p.large) return launch_forward_large(p, E, eps, T_out, status_out, ws, s, tchan);
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
  a.tchan = tchan;
  a.phi_ld = p.phi_ld;
  a.fb_flags = p.fb_grid > 0 ? reinterpret_cast<int32_t*>(ws + p.off_flags) : nullptr;
  a.refine_stats = p.precision == RGF_PREC_MIXED ? device_refine_stats() : nullptr;
  const FwdEntry& f = kFwd[p.tile.id];
  if (tchan && p.precision != RGF_PREC_FP64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(tchan ? f.chan : f.k[p.precision], dim3(p.grid), dim3(f.NW * 64), 0, s, a);
  err = hipGetLastError();
  if (err != hipSuccess || !a.fb_flags) return err;
  return launch_whole_fallback(p, a, ws, s);
}

}  // namespace rgf
