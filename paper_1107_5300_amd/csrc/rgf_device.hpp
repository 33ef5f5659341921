// rgf_device.hpp -- device-side building blocks of the RGF kernels (gfx950).
//
// Geometry of the half-slice chain used by every kernel.
//
// The ribbon model has slices i = 1..L of N atoms; slice i bonds to slice
// i+1 through rows k with (k + i + parity) even (set R_i), and within a slice
// the transverse zigzag chain bonds k <-> k+1. Since k and k+1 always have
// opposite parity, every intra-slice bond joins the other row set
// L_i = {k : (k + i - 1 + parity) even} to R_i, and R_i is the row set that
// slice i+1 calls L_{i+1}. The atoms therefore form a chain of 2L
// "half-slices" L_1, R_1, L_2, R_2, ..., L_L, R_L with no bonds inside a
// half-slice (its block of E - H is diagonal), the bidiagonal block
// B_i = t * adjacency(L_i, R_i) between L_i and R_i, and t times the identity
// between R_{i-1} and L_i (same rows k). Dyson's equation (Eq. (3)) applied
// at each half-slice boundary is Eq. (4)-(5) of the paper on this finer
// partition: every step inverts an n x n complex symmetric matrix, n ~ N/2.
//
// Local index a of a half-slice with row parity e maps to row k = 2a + e;
// the set holds (N + 1 - e) / 2 rows.

#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rgf {

template <typename T>
struct cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) {
  cx<T> r;
  r.re = a;
  r.im = b;
  return r;
}

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) {
  return mk<T>(a.re + b.re, a.im + b.im);
}

template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) {
  return mk<T>(a.re - b.re, a.im - b.im);
}

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return mk<T>(fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re));
}

template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) {
  return mk<T>(a.re * s, a.im * s);
}

// acc + a * b
template <typename T>
__device__ __forceinline__ cx<T> cfma(cx<T> a, cx<T> b, cx<T> acc) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
  return acc;
}

// acc - a * b
template <typename T>
__device__ __forceinline__ cx<T> cfms(cx<T> a, cx<T> b, cx<T> acc) {
  acc.re = fma(-a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(-a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
  return acc;
}

// 1 / b by Smith's method (R. L. Smith, "Algorithm 116: Complex division",
// Comm. ACM 5 (1962) 435), which avoids overflow of |b|^2.
template <typename T>
__device__ __forceinline__ cx<T> crcp(cx<T> b) {
  T c = b.re, d = b.im;
  if (fabs(c) >= fabs(d)) {
    T r = d / c;
    T den = c + d * r;
    return mk<T>(T(1) / den, -r / den);
  } else {
    T r = c / d;
    T den = c * r + d;
    return mk<T>(r / den, T(-1) / den);
  }
}

// 1/b = conj(b) / |b|^2 with one division, for arguments of moderate
// magnitude (the pivots of a tile scaled to entries below 1): |b|^2 cannot
// overflow there, and it underflows only for pivots so small that the
// inversion has no accurate digits left (the result is then infinite and
// the tuple reports a non-finite conductance).
template <typename T>
__device__ __forceinline__ cx<T> crcp_scaled(cx<T> b) {
  const T inv = T(1) / fma(b.re, b.re, b.im * b.im);
  return mk<T>(b.re * inv, -b.im * inv);
}

// |re| + |im|: the pivot magnitude of LAPACK-style complex pivoting.
template <typename T>
__device__ __forceinline__ T cabs1(cx<T> a) {
  return fabs(a.re) + fabs(a.im);
}

template <typename T>
__device__ __forceinline__ bool cfinite(cx<T> a) {
  return isfinite(a.re) && isfinite(a.im);
}

// ----------------------------------------------------------------------------
// Half-slice geometry.
// ----------------------------------------------------------------------------

// Row parity e of half-slice h = 0..2L-1 (h even: L_{h/2+1}, h odd: R_{h/2+1}).
__device__ __host__ __forceinline__ int half_parity(int h, int parity) {
  // slice i = h/2 + 1; L_i: k = (i - 1 + parity) mod 2, R_i: k = (i + parity) mod 2,
  // i.e. the sequence e, 1-e, 1-e, e, e, 1-e, ... with e = parity.
  return (((h + 1) >> 1) + parity) & 1;
}

__device__ __host__ __forceinline__ int half_size(int N, int e) {
  return (N + 1 - e) >> 1;
}

__device__ __host__ __forceinline__ int half_row(int a, int e) { return 2 * a + e; }

// A vacancy (a site removed from the lattice) is marked by the on-site
// energy +inf: that limit decouples the site, so its row and column of
// every Green's function vanish and the rest is that of the lattice without
// it. The kernels replace its row and column of M by the identity's and
// zero its diagonal entry of g.
__device__ __host__ __forceinline__ bool is_vacancy(double eps) {
  return eps == __builtin_huge_val();
}

// Neighbours in L_i of row b of R_i (R_i parity eR): local a = b - 1 + eR and
// a = b + eR, each valid only inside [0, nL).
__device__ __forceinline__ int nb_lo(int b, int eR) { return b - 1 + eR; }
__device__ __forceinline__ int nb_hi(int b, int eR) { return b + eR; }

// ----------------------------------------------------------------------------
// Global-memory complex loads/stores (16 B / 8 B vector accesses).
// ----------------------------------------------------------------------------

__device__ __forceinline__ cx<double> ldg(const cx<double>* p) {
  double2 v = *reinterpret_cast<const double2*>(p);
  return mk<double>(v.x, v.y);
}
__device__ __forceinline__ void stg(cx<double>* p, cx<double> a) {
  *reinterpret_cast<double2*>(p) = make_double2(a.re, a.im);
}
__device__ __forceinline__ cx<float> ldg(const cx<float>* p) {
  float2 v = *reinterpret_cast<const float2*>(p);
  return mk<float>(v.x, v.y);
}
__device__ __forceinline__ void stg(cx<float>* p, cx<float> a) {
  *reinterpret_cast<float2*>(p) = make_float2(a.re, a.im);
}

}  // namespace rgf
