// rgf_mfma.hpp -- FP64 complex GEMM on the CDNA matrix cores: the update of
// the running propagator G1_h = (G1_{h-1} C_{h-1}) g_h and the reverse
// sweep's products g_h (C_h Z_{h+1}), g_h (C_h Q_{h+1}).
//
// v_mfma_f64_16x16x4f64 computes D = A B + D for a 16 x 4 block A, a 4 x 16
// block B and a 16 x 16 block D, one double per lane for A and B and four
// for D. Lane layout (lane l of 64, measured on gfx950):
//   A: lane l holds A[l % 16][l / 16]
//   B: lane l holds B[l / 16][l % 16]
//   D: lane l, element v holds D[4 v + l / 16][l % 16]
// A complex product takes four real ones per k-step:
//   Re += a.re b.re + (-a.im) b.im,   Im += a.re b.im + a.im b.re.
//
// The FP64 matrix rate equals the FP64 vector rate on this chip; the gain
// over a vector GEMM is that the operands reach the lanes in their natural
// layout (no broadcast of one operand to all 64 lanes through LDS) and one
// instruction does 1024 multiply-adds.

#pragma once

#include "rgf_engine.hpp"

namespace rgf {

typedef double mf64x4 __attribute__((ext_vector_type(4)));

// Arrangement of the waves of a workgroup over the output tiles: WR groups
// of rows times WC groups of columns.
template <int NW>
struct WaveGrid;
template <>
struct WaveGrid<1> {
  static constexpr int WR = 1, WC = 1;
};
template <>
struct WaveGrid<2> {
  static constexpr int WR = 2, WC = 1;
};
template <>
struct WaveGrid<4> {
  static constexpr int WR = 2, WC = 2;
};
template <>
struct WaveGrid<8> {
  static constexpr int WR = 4, WC = 2;
};

template <int TR, int TC>
__device__ __forceinline__ void mfma_complex_step(mf64x4 (&accr)[TR][TC], mf64x4 (&acci)[TR][TC],
                                                  const cx<double> (&a)[TR],
                                                  const cx<double> (&b)[TC]) {
  // first the re*re and re*im products of every tile, then the im parts, so
  // that consecutive instructions never wait on each other's accumulator
#pragma unroll
  for (int i = 0; i < TR; ++i)
#pragma unroll
    for (int j = 0; j < TC; ++j) {
      accr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].re, b[j].re, accr[i][j], 0, 0, 0);
      acci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].re, b[j].im, acci[i][j], 0, 0, 0);
    }
#pragma unroll
  for (int i = 0; i < TR; ++i) {
    const double nim = -a[i].im;
#pragma unroll
    for (int j = 0; j < TC; ++j) {
      accr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(nim, b[j].im, accr[i][j], 0, 0, 0);
      acci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].im, b[j].re, acci[i][j], 0, 0, 0);
    }
  }
}

// D[r][c] = sum_{k < nk} fa(r, k) * fb(k, c)   for r < nr, c < nc, handed to
// epi(r, c, D[r][c], valid) after a workgroup barrier (so the epilogue may
// write memory that fa or fb read). The epilogue runs on every lane of a
// wave whose block intersects the output, with valid = (r < nr && c < nc),
// so it may reduce across lanes. fa is called for r < nr, k < nk and fb for
// k < nk, c < nc only; each is called with 16 consecutive rows (fa) or
// columns (fb) across the lanes of a row group, so loads that are
// contiguous in that index coalesce. Operands are loaded one k-step ahead.
// In the epilogue the 16 lanes l % 16 = 0..15 of a row group hold 16
// consecutive columns of one row (lane l, element v: row 4 v + l / 16).
template <int NW, int NP, typename FA, typename FB, typename EPI>
__device__ __forceinline__ void gemm_mfma(int nr, int nc, int nk, FA fa, FB fb, EPI epi) {
  constexpr int PT = (NP + 15) / 16;
  constexpr int WR = WaveGrid<NW>::WR, WC = WaveGrid<NW>::WC;
  constexpr int TR = (PT + WR - 1) / WR, TC = (PT + WC - 1) / WC;
  const int lane = lane_id(), w = wave_id();
  const int li = lane & 15, lk = lane >> 4;
  const int r0 = (w / WC) * TR * 16, c0 = (w % WC) * TC * 16;
  mf64x4 accr[TR][TC], acci[TR][TC];
#pragma unroll
  for (int i = 0; i < TR; ++i)
#pragma unroll
    for (int j = 0; j < TC; ++j) {
      accr[i][j] = (mf64x4){0.0, 0.0, 0.0, 0.0};
      acci[i][j] = (mf64x4){0.0, 0.0, 0.0, 0.0};
    }
  auto load = [&](int ks, cx<double> (&a)[TR], cx<double> (&b)[TC]) {
    const int k = ks * 4 + lk;
#pragma unroll
    for (int i = 0; i < TR; ++i) {
      const int r = r0 + i * 16 + li;
      a[i] = (r < nr && k < nk) ? fa(r, k) : mk(0.0, 0.0);
    }
#pragma unroll
    for (int j = 0; j < TC; ++j) {
      const int c = c0 + j * 16 + li;
      b[j] = (c < nc && k < nk) ? fb(k, c) : mk(0.0, 0.0);
    }
  };
  if (r0 < nr && c0 < nc) {
    const int nks = (nk + 3) >> 2;
    cx<double> a0[TR], b0[TC], a1[TR], b1[TC];
    if (nks > 0) load(0, a0, b0);
    for (int ks = 0; ks < nks; ks += 2) {
      if (ks + 1 < nks) load(ks + 1, a1, b1);
      mfma_complex_step<TR, TC>(accr, acci, a0, b0);
      if (ks + 2 < nks) load(ks + 2, a0, b0);
      if (ks + 1 < nks) mfma_complex_step<TR, TC>(accr, acci, a1, b1);
    }
  }
  __syncthreads();
  if (r0 < nr && c0 < nc) {
#pragma unroll
    for (int i = 0; i < TR; ++i)
#pragma unroll
      for (int j = 0; j < TC; ++j) {
        const int c = c0 + j * 16 + li;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = r0 + i * 16 + 4 * v + lk;
          epi(r, c, mk(accr[i][j][v], acci[i][j][v]), r < nr && c < nc);
        }
      }
  }
}

}  // namespace rgf
