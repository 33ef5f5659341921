// rgf_lead.hip -- lead self-energies by Sancho-Rubio decimation, FP64.
//
// The paper computes the lead self-energies at the first and the last slice
// separately from the recursion (method section, and the timing discussion
// that excludes them). Here they come from the decimation of M. P. Lopez
// Sancho, J. M. Lopez Sancho and J. Rubio, J. Phys. F 15 (1985) 851, applied
// to the decoupled transverse modes of the pristine lead:
//
//   * the slice Hamiltonian t * (k <-> k+1 chain) has eigenvectors
//     phi_p(k) = sqrt(2/(N+1)) sin(p pi (k+1)/(N+1)), p = 1..N;
//   * the longitudinal bonds t * diag([(k + i + parity) even]) equal
//     t (1 + s_i J) / 2 with J = diag((-1)^k), and J phi_p = phi_{N+1-p};
//   * so each pair (p, N+1-p) is a separate two-orbital chain; in the basis
//     (phi_p +/- phi_{N+1-p})/sqrt(2) it is a single chain with alternating
//     hoppings e_p = 2t cos(p pi/(N+1)) and t and zero on-site energy. For
//     odd N the middle mode p = (N+1)/2 pairs with itself (e = 0).
//
// Both leads present the same chain to the device (surface site, then the e
// bond, then t, ...), so one surface Green's function g_p per mode serves
// both. With w_p = 2 for pairs and 1 for the middle mode,
//   Sigma_L[a][b] = sum_p phi_p(k_a) phi_p(k_b) * sigma_p,  sigma_p = w_p t^2 g_p,
// on the slice-1 rows that bond to the lead, and the same with the slice-L
// rows for Sigma_R. Gamma = i(Sigma - Sigma^dagger) = Phi diag(-2 Im sigma) Phi^T.
//
// One thread decimates one (energy, mode): 2 x 2 complex algebra in FP64.

#include "rgf_device.hpp"
#include "rgf_internal.hpp"

namespace rgf {

namespace {

struct m2 {
  cx<double> a, b, c, d;  // [[a, b], [c, d]]
};

__device__ __forceinline__ m2 mmul(const m2& x, const m2& y) {
  m2 r;
  r.a = cfma(x.a, y.a, cmul(x.b, y.c));
  r.b = cfma(x.a, y.b, cmul(x.b, y.d));
  r.c = cfma(x.c, y.a, cmul(x.d, y.c));
  r.d = cfma(x.c, y.b, cmul(x.d, y.d));
  return r;
}

__device__ __forceinline__ m2 madd(const m2& x, const m2& y) {
  return m2{cadd(x.a, y.a), cadd(x.b, y.b), cadd(x.c, y.c), cadd(x.d, y.d)};
}

// (z I - x)^{-1}
__device__ __forceinline__ m2 resolvent(cx<double> z, const m2& x) {
  cx<double> a = csub(z, x.a), d = csub(z, x.d);
  cx<double> b = mk(-x.b.re, -x.b.im), c = mk(-x.c.re, -x.c.im);
  cx<double> det = csub(cmul(a, d), cmul(b, c));
  cx<double> id = crcp(det);
  return m2{cmul(d, id), cmul(mk(-b.re, -b.im), id), cmul(mk(-c.re, -c.im), id),
            cmul(a, id)};
}

__device__ __forceinline__ double mmax(const m2& x) {
  return fmax(fmax(cabs1(x.a), cabs1(x.b)), fmax(cabs1(x.c), cabs1(x.d)));
}

// Principal square root (branch cut on the negative real axis), from the
// half-angle formulas: sqrt(a) = sqrt((|a| + re)/2) + i sign(im) sqrt((|a| - re)/2),
// with the smaller component taken as im / (2 * larger) to avoid cancellation.
__device__ __forceinline__ cx<double> csqrt_principal(cx<double> a) {
  const double m = hypot(a.re, a.im);
  if (m == 0.0) return mk(0.0, 0.0);
  if (a.re >= 0.0) {
    const double x = sqrt(0.5 * (m + a.re));
    return mk(x, a.im / (2.0 * x));
  }
  const double y = copysign(sqrt(0.5 * (m - a.re)), a.im);
  return mk(a.im / (2.0 * y), y);
}

// One block per energy; threads loop over the modes. method 0: decimation;
// method 1: closed form (mode matching): the surface Green's function of the
// chain s0 -e- s1 -t- s0' -e- ... solves g = 1 / (z - e^2 / (z - t^2 g)), i.e.
//   z t^2 g^2 - (z^2 + t^2 - e^2) g + z = 0,
// whose roots are the two Bloch solutions; the retarded one is the root whose
// layer-to-layer amplitude |e t g / (z - t^2 g)| is below 1 (decaying or
// outgoing for eta > 0). For e = 0 the surface site is isolated: g = 1/z.
__global__ void lead_modes_kernel(int N, int P, double t, double eta,
                                  const double* __restrict__ E,
                                  cx<double>* __restrict__ sigma,
                                  int32_t* __restrict__ lstat, int method) {
  const int64_t e = blockIdx.x;
  const cx<double> z = mk(E[e], eta);
  const cx<double> zero = mk(0.0, 0.0);
  int bad = RGF_TUPLE_OK;
  for (int p = threadIdx.x + 1; p <= P; p += blockDim.x) {
    bool middle = (N & 1) && (p == P);
    // e_p = 2t cos(p pi/(N+1)); the middle mode of odd N has cos = 0 exactly
    double ep = middle ? 0.0 : 2.0 * t * cospi((double)p / (double)(N + 1));
    double wp = middle ? 1.0 : 2.0;
    if (method == 1) {
      cx<double> g;
      if (ep == 0.0) {
        g = crcp(z);
      } else {
        const cx<double> z2 = cmul(z, z);
        const cx<double> b = mk(z2.re + t * t - ep * ep, z2.im);
        const cx<double> disc = csub(cmul(b, b), cscale(z2, 4.0 * t * t));
        const cx<double> sq = csqrt_principal(disc);
        const cx<double> den = crcp(cscale(z, 2.0 * t * t));
        const cx<double> g1 = cmul(cadd(b, sq), den), g2 = cmul(csub(b, sq), den);
        const cx<double> d1 = csub(z, cscale(g1, t * t)), d2 = csub(z, cscale(g2, t * t));
        const double l1 = hypot(g1.re, g1.im) / hypot(d1.re, d1.im);
        const double l2 = hypot(g2.re, g2.im) / hypot(d2.re, d2.im);
        g = (l1 <= l2) ? g1 : g2;
      }
      const cx<double> sg = cscale(g, wp * t * t);
      sigma[e * P + (p - 1)] = sg;
      if (!cfinite(sg)) bad = max(bad, (int)RGF_TUPLE_NONFINITE);
      continue;
    }
    // principal layer: sites (s0, s1) joined by e_p; s1 -> s0 of the next layer by t
    m2 h00{zero, mk(ep, 0.0), mk(ep, 0.0), zero};
    m2 alpha{zero, zero, mk(t, 0.0), zero};   // H_{layer, next}
    m2 beta{zero, mk(t, 0.0), zero, zero};    // H_{next, layer}
    m2 es = h00, eb = h00;
    const double tol = 1e-15 * fmax(fmax(fabs(t), fabs(ep)), 1.0);
    const int maxit = 200;
    bool ok = false;
    for (int it = 0; it < maxit; ++it) {
      m2 g = resolvent(z, eb);
      m2 ag = mmul(alpha, g), bg = mmul(beta, g);
      m2 agb = mmul(ag, beta), bga = mmul(bg, alpha);
      es = madd(es, agb);
      eb = madd(eb, madd(agb, bga));
      alpha = mmul(ag, alpha);
      beta = mmul(bg, beta);
      if (fmax(mmax(alpha), mmax(beta)) < tol) {
        ok = true;
        break;
      }
    }
    m2 gs = resolvent(z, es);
    cx<double> g = gs.a;
    if (ep != 0.0) {
      // The surface Green's function solves z t^2 g^2 - (z^2 + t^2 - e^2) g + z = 0,
      // whose two roots multiply to 1/t^2. When the layer's Bloch phase is
      // commensurate with the doubling (e.g. e = t at E = +-|t|) the
      // decimation can settle on the advanced root; keep the root whose
      // layer-to-layer amplitude |e t g / (z - t^2 g)| decays.
      const cx<double> g2 = crcp(cscale(g, t * t));
      const cx<double> d1 = csub(z, cscale(g, t * t)), d2 = csub(z, cscale(g2, t * t));
      const double l1 = fabs(ep * t) * hypot(g.re, g.im) / hypot(d1.re, d1.im);
      const double l2 = fabs(ep * t) * hypot(g2.re, g2.im) / hypot(d2.re, d2.im);
      if (l2 < l1) g = g2;
      // Near such phases the decimation also stagnates at ~eta accuracy;
      // polish the selected root with Newton steps on the same quadratic.
      const cx<double> qa = cscale(z, t * t);
      const cx<double> qb = mk(-(z.re * z.re - z.im * z.im + t * t - ep * ep), -2.0 * z.re * z.im);
      for (int it = 0; it < 3; ++it) {
        const cx<double> f = cadd(cmul(cadd(cmul(qa, g), qb), g), z);   // (qa g + qb) g + z
        const cx<double> df = cadd(cscale(cmul(qa, g), 2.0), qb);       // 2 qa g + qb
        g = csub(g, cmul(f, crcp(df)));
      }
    }
    cx<double> sg = cscale(g, wp * t * t);
    sigma[e * P + (p - 1)] = sg;
    if (!ok) bad = max(bad, (int)RGF_TUPLE_NO_CONVERGENCE);
    else if (!cfinite(sg)) bad = max(bad, (int)RGF_TUPLE_NONFINITE);
  }
  __shared__ int worst;
  if (threadIdx.x == 0) worst = RGF_TUPLE_OK;
  __syncthreads();
  if (bad != RGF_TUPLE_OK) atomicMax(&worst, bad);
  __syncthreads();
  if (threadIdx.x == 0) lstat[e] = worst;
}

// phi tables: phiL[p][a] = phi_{p+1}(k_a) on the slice-1 interface rows,
// phiR[p][b] on the slice-L interface rows; zero for padded rows.
__global__ void phi_kernel(int N, int L, int parity, int P, int ld,
                           double* __restrict__ phi) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  int total = 2 * P * ld;
  if (idx >= total) return;
  int side = idx / (P * ld);
  int rem = idx % (P * ld);
  int p = rem / ld + 1;
  int a = rem % ld;
  // slice-1 interface = L_1 (half-slice 0); slice-L interface = R_L (2L-1)
  int e = side == 0 ? half_parity(0, parity) : half_parity(2 * L - 1, parity);
  int n = half_size(N, e);
  double v = 0.0;
  if (a < n) {
    int k = half_row(a, e);
    long m = ((long)p * (long)(k + 1)) % (2 * (long)(N + 1));
    v = sqrt(2.0 / (double)(N + 1)) * sinpi((double)m / (double)(N + 1));
  }
  phi[idx] = v;
}

// Dense export of Sigma_L / Sigma_R (interleaved re, im) from the mode sums.
__global__ void export_sigma_kernel(int P, int ld, int nl, int nr, int64_t nE,
                                    const cx<double>* __restrict__ sigma,
                                    const double* __restrict__ phi,
                                    double* __restrict__ sl, double* __restrict__ sr) {
  int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t per = (int64_t)nl * nl + (int64_t)nr * nr;
  if (gid >= nE * per) return;
  int64_t e = gid / per;
  int64_t rem = gid % per;
  const double* ph = phi;
  int n = nl;
  double* out = sl;
  if (rem >= (int64_t)nl * nl) {
    rem -= (int64_t)nl * nl;
    ph = phi + (size_t)P * ld;
    n = nr;
    out = sr;
  }
  int a = (int)(rem / n), b = (int)(rem % n);
  cx<double> acc = mk(0.0, 0.0);
  for (int p = 0; p < P; ++p) {
    double f = ph[p * ld + a] * ph[p * ld + b];
    cx<double> s = sigma[e * P + p];
    acc.re = fma(f, s.re, acc.re);
    acc.im = fma(f, s.im, acc.im);
  }
  if (out) {
    int64_t o = (e * (int64_t)n * n + rem) * 2;
    out[o] = acc.re;
    out[o + 1] = acc.im;
  }
}

}  // namespace

hipError_t launch_lead(const Plan& p, const double* E, char* ws, hipStream_t s, int method) {
  auto* sigma = reinterpret_cast<cx<double>*>(ws + p.off_sigma);
  auto* phi = reinterpret_cast<double*>(ws + p.off_phi);
  auto* lstat = reinterpret_cast<int32_t*>(ws + p.off_lstat);
  const int ld = p.phi_ld;
  if (p.nE > 0) {
    hipLaunchKernelGGL(lead_modes_kernel, dim3((unsigned)p.nE), dim3(128), 0, s, p.N,
                       p.P, p.t, p.eta, E, sigma, lstat, method);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  int n2 = 2 * p.P * ld;
  hipLaunchKernelGGL(phi_kernel, dim3((n2 + 255) / 256), dim3(256), 0, s, p.N, p.L,
                     p.parity, p.P, ld, phi);
  return hipGetLastError();
}

hipError_t launch_export_sigma(const Plan& p, const double* E, double* sl, double* sr,
                               int32_t* lstat_out, char* ws, hipStream_t s) {
  hipError_t err = launch_lead(p, E, ws, s);
  if (err != hipSuccess) return err;
  int nl = half_size(p.N, half_parity(0, p.parity));
  int nr = half_size(p.N, half_parity(2 * p.L - 1, p.parity));
  int64_t total = p.nE * ((int64_t)nl * nl + (int64_t)nr * nr);
  if (total > 0) {
    hipLaunchKernelGGL(export_sigma_kernel, dim3((unsigned)((total + 255) / 256)),
                       dim3(256), 0, s, p.P, p.phi_ld, nl, nr, p.nE,
                       reinterpret_cast<const cx<double>*>(ws + p.off_sigma),
                       reinterpret_cast<const double*>(ws + p.off_phi), sl, sr);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  if (lstat_out && p.nE > 0)
    err = hipMemcpyAsync(lstat_out, ws + p.off_lstat, p.nE * sizeof(int32_t),
                         hipMemcpyDeviceToDevice, s);
  return err;
}

}  // namespace rgf

namespace rgf {

hipError_t launch_lead_modes(const Plan& p, const double* E, int method, double* sigma_out,
                             int32_t* lstat_out, char* ws, hipStream_t s) {
  hipError_t err = launch_lead(p, E, ws, s, method);
  if (err != hipSuccess || p.nE == 0) return err;
  if (sigma_out)
    err = hipMemcpyAsync(sigma_out, ws + p.off_sigma, (size_t)p.nE * p.P * 16,
                         hipMemcpyDeviceToDevice, s);
  if (err == hipSuccess && lstat_out)
    err = hipMemcpyAsync(lstat_out, ws + p.off_lstat, p.nE * sizeof(int32_t),
                         hipMemcpyDeviceToDevice, s);
  return err;
}

}  // namespace rgf
