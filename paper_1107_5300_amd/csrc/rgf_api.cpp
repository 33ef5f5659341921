// rgf_api.cpp -- the C ABI of librgf: argument validation, workspace planning
// and dispatch to the launchers. No device memory is allocated here; all
// scratch comes from the caller's workspace.

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>

#include "rgf_internal.hpp"

namespace rgf {

namespace {
thread_local std::string g_last_error;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}
}  // namespace

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

static int validate_desc(const rgf_ribbon_desc* d) {
  if (!d) return fail(RGF_ERR_INVALID_ARG, "desc is NULL");
  if (d->struct_size != sizeof(rgf_ribbon_desc))
    return fail(RGF_ERR_INVALID_ARG, "desc->struct_size is %u, expected %zu",
                d->struct_size, sizeof(rgf_ribbon_desc));
  if (d->width_n < 2 || d->width_n > RGF_MAX_WIDTH)
    return fail(d->width_n > RGF_MAX_WIDTH ? RGF_ERR_UNSUPPORTED : RGF_ERR_INVALID_ARG,
                "width_n = %d outside [2, %d]", d->width_n, RGF_MAX_WIDTH);
  if (d->length_l < 1 || d->length_l > (1 << 24))
    return fail(RGF_ERR_INVALID_ARG, "length_l = %d outside [1, 2^24]", d->length_l);
  if (d->parity != 0 && d->parity != 1)
    return fail(RGF_ERR_INVALID_ARG, "parity = %d, expected 0 or 1", d->parity);
  if (!isfinite(d->hopping_ev) || d->hopping_ev == 0.0)
    return fail(RGF_ERR_INVALID_ARG, "hopping_ev = %g must be finite and non-zero",
                d->hopping_ev);
  if (!isfinite(d->eta_ev) || !(d->eta_ev > 0.0))
    return fail(RGF_ERR_INVALID_ARG, "eta_ev = %g must be finite and > 0", d->eta_ev);
  return RGF_OK;
}

int make_plan(const rgf_ribbon_desc* d, int64_t nE, int64_t nreal, int precision,
              int want_grad, int64_t ckpt_stride, Plan* p) {
  int st = validate_desc(d);
  if (st != RGF_OK) return st;
  if (nE < 0) return fail(RGF_ERR_INVALID_ARG, "n_energies = %lld < 0", (long long)nE);
  if (nreal < 1) return fail(RGF_ERR_INVALID_ARG, "n_real = %lld < 1", (long long)nreal);
  if (precision != RGF_PREC_FP64 && precision != RGF_PREC_MIXED &&
      precision != RGF_PREC_FP32)
    return fail(RGF_ERR_INVALID_ARG, "precision = %d unknown", precision);
  if (ckpt_stride < 0)
    return fail(RGF_ERR_INVALID_ARG, "ckpt_stride = %lld < 0", (long long)ckpt_stride);
  Plan q;
  memset(&q, 0, sizeof(q));
  q.N = d->width_n;
  q.L = d->length_l;
  q.parity = d->parity;
  q.t = d->hopping_ev;
  q.eta = d->eta_ev;
  q.P = lead_modes(q.N);
  q.n1 = (q.N + 1 - (q.parity & 1)) / 2;
  q.nmax = (q.N + 1) / 2;
  q.nE = nE;
  q.nreal = nreal;
  q.ntuples = nE * nreal;
  q.precision = precision;
  q.want_grad = want_grad != 0;
  if (!pick_tile(q.nmax, precision, &q.tile))
    return fail(RGF_ERR_UNSUPPORTED, "width_n = %d exceeds the register tiling", q.N);
  const int NP = q.tile.NP();
  q.grid = persistent_grid(q.tile, std::max<int64_t>(q.ntuples, 1), precision, q.want_grad);
  q.slot_elems = (int64_t)NP * NP;
  q.slot_mats = slot_matrices(precision, q.want_grad);
  size_t off = 0;
  q.off_sigma = off;
  off = align_up(off + (size_t)nE * q.P * 16, 256);
  q.off_phi = off;
  off = align_up(off + (size_t)2 * q.P * NP * 8, 256);
  q.off_lstat = off;
  off = align_up(off + (size_t)nE * 4, 256);
  q.off_status = off;
  q.off_slots = off;
  off = align_up(off + (size_t)q.grid * q.slot_mats * q.slot_elems * 16, 256);
  q.off_ckpt = q.off_seg = off;
  if (q.want_grad) {
    const int64_t H = 2 * (int64_t)q.L;
    int64_t stride = ckpt_stride;
    if (stride == 0) {
      stride = 1;
      while (stride * stride < H) ++stride;
    }
    if (stride > H) stride = H;
    q.ckpt_stride = stride;
    q.n_ckpt = (H + stride - 1) / stride;
    q.off_ckpt = off;
    off = align_up(off + (size_t)q.grid * q.n_ckpt * 2 * q.slot_elems * 16, 256);
    q.off_seg = off;
    off = align_up(off + (size_t)q.grid * stride * 2 * q.slot_elems * 16, 256);
  }
  q.total = off;
  *p = q;
  return RGF_OK;
}

int persistent_grid(const TileCfg& t, int64_t ntuples, int precision, bool grad) {
  int dev = 0, ncu = 256, occ = 1;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
    const void* k = grad ? grad_kernel_ptr(t, precision) : fwd_kernel_ptr(t, precision);
    int o = 0;
    if (k && hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, k, t.threads(), 0) == hipSuccess &&
        o > 0)
      occ = o;
    else
      (void)hipGetLastError();
  } else {
    (void)hipGetLastError();
  }
  int64_t g = (int64_t)ncu * occ;
  if (g > ntuples) g = ntuples;
  if (g < 1) g = 1;
  return (int)g;
}

static int check_ws(const Plan& p, void* ws, size_t bytes) {
  if (bytes < p.total)
    return fail(RGF_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", bytes, p.total);
  if (p.total > 0 && !ws) return fail(RGF_ERR_INVALID_ARG, "workspace is NULL");
  if (((uintptr_t)ws) % 256 != 0)
    return fail(RGF_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  return RGF_OK;
}

static int hip_fail(hipError_t e) {
  return fail(RGF_ERR_HIP, "HIP error %d: %s", (int)e, hipGetErrorString(e));
}

}  // namespace rgf

using namespace rgf;

extern "C" {

size_t rgf_workspace_bytes(const rgf_ribbon_desc* desc, int64_t n_energies, int64_t n_real,
                           int precision, int want_grad, int64_t ckpt_stride) {
  Plan p;
  if (make_plan(desc, n_energies, n_real, precision, want_grad, ckpt_stride, &p) != RGF_OK)
    return 0;
  return std::max<size_t>(p.total, 256);
}

int rgf_conductance(const rgf_ribbon_desc* desc, const double* energies_ev,
                    int64_t n_energies, const double* onsite_eps_ev, int64_t n_real,
                    int precision, double* T_out, int32_t* status_out, void* workspace,
                    size_t workspace_bytes, void* hip_stream) {
  Plan p;
  int st = make_plan(desc, n_energies, n_real, precision, 0, 0, &p);
  if (st != RGF_OK) return st;
  if (n_energies == 0) return RGF_OK;
  if (!energies_ev) return fail(RGF_ERR_INVALID_ARG, "energies_ev is NULL");
  if (!T_out) return fail(RGF_ERR_INVALID_ARG, "T_out is NULL");
  st = check_ws(p, workspace, workspace_bytes);
  if (st != RGF_OK) return st;
  hipError_t e = launch_forward(p, energies_ev, onsite_eps_ev, T_out, status_out,
                                (char*)workspace, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e);
  return RGF_OK;
}

int rgf_grad(const rgf_ribbon_desc* desc, const double* energies_ev, int64_t n_energies,
             const double* onsite_eps_ev, int64_t n_real, int precision,
             const double* dL_dT, double* T_out, double* dL_deps, int64_t ckpt_stride,
             int32_t* status_out, void* workspace, size_t workspace_bytes,
             void* hip_stream) {
  Plan p;
  int st = make_plan(desc, n_energies, n_real, precision, 1, ckpt_stride, &p);
  if (st != RGF_OK) return st;
  if (!dL_deps) return fail(RGF_ERR_INVALID_ARG, "dL_deps is NULL");
  if (n_energies > 0) {
    if (!energies_ev) return fail(RGF_ERR_INVALID_ARG, "energies_ev is NULL");
    if (!T_out) return fail(RGF_ERR_INVALID_ARG, "T_out is NULL");
    if (!dL_dT) return fail(RGF_ERR_INVALID_ARG, "dL_dT is NULL");
  }
  st = check_ws(p, workspace, workspace_bytes);
  if (st != RGF_OK) return st;
  hipError_t e = launch_grad(p, energies_ev, onsite_eps_ev, dL_dT, T_out, dL_deps, status_out,
                             (char*)workspace, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e);
  return RGF_OK;
}

size_t rgf_batched_workspace_bytes(const rgf_ribbon_desc* descs, int32_t n_desc,
                                   int64_t n_energies, int64_t n_real, int precision) {
  (void)descs;
  (void)n_desc;
  (void)n_energies;
  (void)n_real;
  (void)precision;
  fail(RGF_ERR_UNSUPPORTED, "batched ribbons are not available in this build");
  return 0;
}

int rgf_conductance_batched(const rgf_ribbon_desc* descs, int32_t n_desc,
                            const int64_t* eps_offsets, const int64_t* T_offsets,
                            const double* energies_ev, int64_t n_energies,
                            const double* onsite_eps_ev, int64_t n_real, int precision,
                            double* T_out, int32_t* status_out, void* workspace,
                            size_t workspace_bytes, void* hip_stream) {
  (void)descs;
  (void)n_desc;
  (void)eps_offsets;
  (void)T_offsets;
  (void)energies_ev;
  (void)n_energies;
  (void)onsite_eps_ev;
  (void)n_real;
  (void)precision;
  (void)T_out;
  (void)status_out;
  (void)workspace;
  (void)workspace_bytes;
  (void)hip_stream;
  return fail(RGF_ERR_UNSUPPORTED, "batched ribbons are not available in this build");
}

int rgf_lead_self_energy(const rgf_ribbon_desc* desc, const double* energies_ev,
                         int64_t n_energies, double* sigma_l_out, double* sigma_r_out,
                         int32_t* lead_status_out, int32_t* nl_out, int32_t* nr_out,
                         void* workspace, size_t workspace_bytes, void* hip_stream) {
  Plan p;
  int st = make_plan(desc, n_energies, 1, RGF_PREC_FP64, 0, 0, &p);
  if (st != RGF_OK) return st;
  // slice-1 lead rows: (k + parity) even; slice-L rows: (k + L + parity) even
  const int eL = p.parity & 1;
  const int eR = (p.L + p.parity) & 1;
  if (nl_out) *nl_out = (p.N + 1 - eL) / 2;
  if (nr_out) *nr_out = (p.N + 1 - eR) / 2;
  if (!sigma_l_out && !sigma_r_out && !lead_status_out) return RGF_OK;
  if (n_energies == 0) return RGF_OK;
  if (!energies_ev) return fail(RGF_ERR_INVALID_ARG, "energies_ev is NULL");
  st = check_ws(p, workspace, workspace_bytes);
  if (st != RGF_OK) return st;
  hipError_t e = launch_export_sigma(p, energies_ev, sigma_l_out, sigma_r_out,
                                     lead_status_out, (char*)workspace,
                                     (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e);
  return RGF_OK;
}

const char* rgf_status_string(int status) {
  switch (status) {
    case RGF_OK: return "RGF_OK";
    case RGF_ERR_INVALID_ARG: return "RGF_ERR_INVALID_ARG";
    case RGF_ERR_HIP: return "RGF_ERR_HIP";
    case RGF_ERR_WORKSPACE: return "RGF_ERR_WORKSPACE";
    case RGF_ERR_UNSUPPORTED: return "RGF_ERR_UNSUPPORTED";
    default: return "RGF_UNKNOWN_STATUS";
  }
}

const char* rgf_last_error_message(void) { return g_last_error.c_str(); }

int rgf_version(int* major, int* minor) {
  if (major) *major = RGF_ABI_VERSION_MAJOR;
  if (minor) *minor = RGF_ABI_VERSION_MINOR;
  return RGF_OK;
}

}  // extern "C"
