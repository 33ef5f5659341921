// rgf_api.cpp -- the C ABI of librgf: argument validation, workspace planning
// and dispatch to the launchers. No device memory is allocated here; all
// scratch comes from the caller's workspace.

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "rgf_internal.hpp"
#include "rgf_segplan.hpp"

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
              int want_grad, int64_t ckpt_stride, Plan* p, int grid_cap) {
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
  q.large = q.nmax > kTileMaxRows;
  if (q.large) {
    // half-slices wider than one register tile: blocked inversion, FP64
    // conductance only
    if (precision != RGF_PREC_FP64)
      return fail(RGF_ERR_UNSUPPORTED,
                  "width_n = %d: half-slices above %d rows run in FP64 only", q.N,
                  kTileMaxRows);
    q.tile = large_block_tile();
  } else if (!pick_tile(q.nmax, precision, &q.tile)) {
    return fail(RGF_ERR_UNSUPPORTED, "width_n = %d exceeds the register tiling", q.N);
  }
  if (!q.large && q.want_grad && q.tile.mgj) {
    // the gradient and LDOS sweeps keep the register tiling: the smallest
    // one that holds n
    for (int i = 0; i < tile_count(); ++i) {
      const TileCfg c = tile_at(i);
      if (!c.mgj && c.NP() >= q.nmax && 64 * c.S >= c.NP()) {
        q.tile = c;
        break;
      }
    }
  }
  if (!q.large && q.want_grad && q.ntuples <= device_cu_count()) {
    // Fewer tuples than compute units: each workgroup runs one tuple at a
    // time and the sweep is latency-bound, so prefer the tiling with the
    // most waves per tuple among those that pad n by at most a quarter.
    TileCfg best = q.tile;
    for (int i = 0; i < tile_count(); ++i) {
      const TileCfg c = tile_at(i);
      const int np = c.NP();
      if (c.mgj || np < q.nmax || 64 * c.S < np || 4 * np > 5 * q.nmax + 32) continue;
      if (c.NW > best.NW || (c.NW == best.NW && np < best.NP())) best = c;
    }
    q.tile = best;
  }
  const int NP = q.tile.NP();
  if (q.large) {
    q.grid = persistent_grid_large(std::max<int64_t>(q.ntuples, 1), q.want_grad);
    q.slot_elems = (int64_t)kTileMaxRows * kTileMaxRows;
    q.slot_mats = large_slot_blocks(q.want_grad);
    q.mat_elems = (int64_t)kLargeLd * kLargeLd;
    q.phi_ld = kLargeLd;
  } else {
    int tid = 0, per_cu = 0;
    if (!q.want_grad && tuned_choice(q.nmax, precision, &tid, &per_cu)) q.per_cu = per_cu;
    q.grid = persistent_grid(q.tile, std::max<int64_t>(q.ntuples, 1), precision, q.want_grad,
                             q.per_cu);
    q.slot_elems = (int64_t)NP * NP;
    q.slot_mats = slot_matrices(precision, q.want_grad);
    q.mat_elems = q.slot_elems;
    q.phi_ld = NP;
  }
  if (grid_cap > 0 && q.grid > grid_cap) q.grid = grid_cap;
  size_t off = 0;
  q.off_sigma = off;
  off = align_up(off + (size_t)nE * q.P * 16, 256);
  q.off_phi = off;
  off = align_up(off + (size_t)2 * q.P * q.phi_ld * 8, 256);
  q.off_lstat = off;
  off = align_up(off + (size_t)nE * 4, 256);
  const bool fallback = !q.want_grad && precision != RGF_PREC_FP32;
  q.off_flags = off;
  if (fallback) off = align_up(off + (size_t)q.ntuples * 4, 256);
  q.off_status = off;
  q.off_slots = off;
  const size_t slots_bytes = (size_t)q.grid * q.slot_mats * q.slot_elems * 16;
  off = align_up(off + slots_bytes, 256);
  if (fallback) {
    // the whole-slice workgroups reuse the slot region after the sweep; at
    // least one of them fits
    const size_t fb_slot = whole_slot_bytes(q.N);
    int64_t g = (int64_t)(slots_bytes / fb_slot);
    g = std::min<int64_t>(g, std::min<int64_t>(std::max<int64_t>(q.ntuples, 1), device_cu_count()));
    q.fb_grid = (int)std::max<int64_t>(g, 1);
    off = std::max(off, align_up(q.off_slots + (size_t)q.fb_grid * fb_slot, 256));
  }
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
    off = align_up(off + (size_t)q.grid * q.n_ckpt * 2 * q.mat_elems * 16, 256);
    q.off_seg = off;
    off = align_up(off + (size_t)q.grid * stride * 2 * q.mat_elems * 16, 256);
  }
  q.total = off;
  *p = q;
  return RGF_OK;
}

namespace {
std::mutex g_tune_mu;
std::map<std::pair<int, int>, std::pair<int, int>> g_tuned;  // (n, prec) -> (tile, per_cu)
}  // namespace

bool tuned_choice(int n, int precision, int* tile_id, int* per_cu) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find({n, precision});
  if (it == g_tuned.end()) return false;
  *tile_id = it->second.first;
  *per_cu = it->second.second;
  return true;
}

void set_tuned_choice(int n, int precision, int tile_id, int per_cu) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[{n, precision}] = {tile_id, per_cu};
}

// Device properties and kernel occupancies are queried once per device
// (plans are made on every call, twice per torch call).
namespace {
struct DeviceInfo {
  int ncu = 0;
  std::map<std::pair<const void*, int>, int> occupancy;  // (kernel, threads) -> blocks per CU
};
std::mutex g_dev_mu;
std::map<int, DeviceInfo> g_dev;

bool current_device(int* dev) {
  if (hipGetDevice(dev) == hipSuccess) return true;
  (void)hipGetLastError();
  return false;
}

// Blocks of `threads` threads of kernel k per CU on the current device (1 if
// unknown).
int kernel_occupancy(const void* k, int threads) {
  int dev = 0;
  if (!k || !current_device(&dev)) return 1;
  std::lock_guard<std::mutex> lk(g_dev_mu);
  auto& m = g_dev[dev].occupancy;
  auto it = m.find({k, threads});
  if (it != m.end()) return it->second;
  int o = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, k, threads, 0) != hipSuccess || o < 1) {
    (void)hipGetLastError();
    return 1;  // not cached: a later call may succeed
  }
  m[{k, threads}] = o;
  return o;
}
}  // namespace

// Counters of the mixed mode's refinement, one copy per device: refined
// half-slices, Newton updates, FP64 re-inversions (rgf_refine_stats).
__device__ unsigned long long g_refine_stats[3];

namespace {
std::map<int, unsigned long long*> g_refine_ptr;  // device -> address of g_refine_stats
}  // namespace

unsigned long long* device_refine_stats() {
  int dev = 0;
  if (!current_device(&dev)) return nullptr;
  std::lock_guard<std::mutex> lk(g_dev_mu);
  auto it = g_refine_ptr.find(dev);
  if (it != g_refine_ptr.end()) return it->second;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(g_refine_stats)) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;  // not cached: a later call may succeed
  }
  auto* c = static_cast<unsigned long long*>(ptr);
  g_refine_ptr[dev] = c;
  return c;
}

int device_cu_count() {
  int dev = 0;
  if (!current_device(&dev)) return 256;
  std::lock_guard<std::mutex> lk(g_dev_mu);
  DeviceInfo& d = g_dev[dev];
  if (d.ncu == 0) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
      (void)hipGetLastError();
      return 256;
    }
    d.ncu = prop.multiProcessorCount;
  }
  return d.ncu;
}

int persistent_grid(const TileCfg& t, int64_t ntuples, int precision, bool grad, int per_cu) {
  const int ncu = device_cu_count();
  const void* k = grad ? grad_kernel_ptr(t, precision) : fwd_kernel_ptr(t, precision);
  int occ = kernel_occupancy(k, t.threads());
  if (per_cu > 0 && per_cu < occ) occ = per_cu;
  int64_t g = (int64_t)ncu * occ;
  if (g > ntuples) g = ntuples;
  if (g < 1) g = 1;
  return (int)g;
}

int persistent_grid_large(int64_t ntuples, bool grad) {
  const int ncu = device_cu_count();
  const int occ = kernel_occupancy(large_kernel_ptr(grad), large_block_tile().threads());
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

// ------------------------------------------------------- segments (in L)

int make_seg_plan(const rgf_ribbon_desc* d, int64_t nE, int64_t nreal, int n_segments,
                  SegPlan* sp) {
  if (n_segments < 0) return fail(RGF_ERR_INVALID_ARG, "n_segments = %d < 0", n_segments);
  SegPlan q;
  memset(&q, 0, sizeof(q));
  // the ribbon's own plan: lead tables, and flags and slots for the
  // whole-slice recomputation of rejected tuples (one slot per tuple at most)
  int st = make_plan(d, nE, nreal, RGF_PREC_FP64, 0, 0, &q.fwd);
  if (st != RGF_OK) return st;
  if (q.fwd.large)
    return fail(RGF_ERR_UNSUPPORTED,
                "width_n = %d: the segment sweep holds half-slices of up to %d rows",
                d->width_n, kTileMaxRows);
  if (!seg_supported(q.fwd.tile))
    return fail(RGF_ERR_UNSUPPORTED, "no segment kernel for width_n = %d", d->width_n);
  // the mode tables of both row classes: the leads of a ribbon of the same
  // width, odd length and parity 0 (left lead on class 0, right lead on
  // class 1); sigma is the same for every lead of this width
  rgf_ribbon_desc da = *d;
  da.parity = 0;
  da.length_l = d->length_l | 1;
  st = make_plan(&da, nE, nreal, RGF_PREC_FP64, 0, 0, &q.aux);
  if (st != RGF_OK) return st;
  if (q.aux.phi_ld != q.fwd.phi_ld)  // both plans pick the tile by the width alone
    return fail(RGF_ERR_UNSUPPORTED, "width_n = %d: lead tables of different layouts",
                d->width_n);
  const int NP = q.fwd.tile.NP();
  const int64_t nt = q.fwd.ntuples;
  const int ncu = device_cu_count();
  const int occ = kernel_occupancy(seg_sweep_kernel(q.fwd.tile), q.fwd.tile.threads());
  const int64_t cap = (int64_t)ncu * occ;
  int64_t G = n_segments;
  // automatic: the most segments whose nt (2G - 1) items fit the slots at
  // once (a tuple's latency is about 2L/G half-slice steps of its segments
  // plus 8 per level of the ceil(log2 G) levels of joins), at least two
  // slices each
  if (G == 0) {
    G = nt > 0 ? (cap / std::max<int64_t>(nt, 1) + 1) / 2 : 1;
    G = std::min<int64_t>(G, std::max<int64_t>(1, d->length_l / 2));
  }
  G = std::max<int64_t>(1, std::min<int64_t>({G, (int64_t)d->length_l, 1024}));
  q.G = (int)G;
  const int64_t nitems = nt * (2 * G - 1);
  q.sweep_grid = (int)std::max<int64_t>(1, std::min(cap, nitems));
  q.merge_grid = (int)std::max<int64_t>(1, std::min(cap, nt * (G / 2)));
  q.join_grid = (int)std::max<int64_t>(1, std::min(cap, nt));
  // lead tables of the reversed ribbon: the part of its plan before the flags
  size_t off = align_up(q.fwd.total, 256);
  q.off_aux = off;
  off = align_up(off + q.aux.off_flags, 256);
  q.off_eps_rev = off;
  off = align_up(off + (size_t)nreal * d->length_l * d->width_n * 8, 256);
  q.off_mats = off;
  off = align_up(off + (size_t)nt * G * 3 * NP * NP * 16, 256);
  q.off_scratch = off;
  off = align_up(off + (size_t)q.merge_grid * 8 * NP * NP * 16, 256);
  q.off_kap = off;
  off = align_up(off + (size_t)nt * 3 * G * 2 * 8, 256);
  q.off_flag = off;
  off = align_up(off + (size_t)nt * 3 * G * 4, 256);
  q.total = off;
  *sp = q;
  return RGF_OK;
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

size_t rgf_segments_workspace_bytes(const rgf_ribbon_desc* desc, int64_t n_energies,
                                    int64_t n_real, int32_t n_segments) {
  SegPlan sp;
  if (make_seg_plan(desc, n_energies, n_real, n_segments, &sp) != RGF_OK) return 0;
  return std::max<size_t>(sp.total, 256);
}

int rgf_conductance_segments(const rgf_ribbon_desc* desc, const double* energies_ev,
                             int64_t n_energies, const double* onsite_eps_ev, int64_t n_real,
                             int32_t n_segments, double* T_out, int32_t* status_out,
                             int32_t* segments_out, void* workspace, size_t workspace_bytes,
                             void* hip_stream) {
  SegPlan sp;
  int st = make_seg_plan(desc, n_energies, n_real, n_segments, &sp);
  if (st != RGF_OK) return st;
  if (segments_out) *segments_out = sp.G;
  if (n_energies == 0) return RGF_OK;
  if (!energies_ev) return fail(RGF_ERR_INVALID_ARG, "energies_ev is NULL");
  if (!T_out) return fail(RGF_ERR_INVALID_ARG, "T_out is NULL");
  if (workspace_bytes < sp.total)
    return fail(RGF_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", workspace_bytes,
                sp.total);
  if (!workspace || ((uintptr_t)workspace) % 256 != 0)
    return fail(RGF_ERR_INVALID_ARG, "workspace must be non-NULL and 256-byte aligned");
  hipError_t e = launch_segments(sp, energies_ev, onsite_eps_ev, T_out, status_out,
                                 (char*)workspace, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e);
  return RGF_OK;
}

int rgf_channel_transmission(const rgf_ribbon_desc* desc, const double* energies_ev,
                             int64_t n_energies, const double* onsite_eps_ev, int64_t n_real,
                             int precision, double* T_channel_out, double* T_out,
                             int32_t* status_out, void* workspace, size_t workspace_bytes,
                             void* hip_stream) {
  Plan p;
  int st = make_plan(desc, n_energies, n_real, precision, 0, 0, &p);
  if (st != RGF_OK) return st;
  if (precision != RGF_PREC_FP64)
    return fail(RGF_ERR_UNSUPPORTED, "the per-channel transmission runs in FP64 only");
  if (n_energies == 0) return RGF_OK;
  if (!energies_ev) return fail(RGF_ERR_INVALID_ARG, "energies_ev is NULL");
  if (!T_channel_out) return fail(RGF_ERR_INVALID_ARG, "T_channel_out is NULL");
  if (!T_out) return fail(RGF_ERR_INVALID_ARG, "T_out is NULL");
  st = check_ws(p, workspace, workspace_bytes);
  if (st != RGF_OK) return st;
  hipError_t e = launch_forward(p, energies_ev, onsite_eps_ev, T_out, status_out,
                                (char*)workspace, (hipStream_t)hip_stream, T_channel_out);
  if (e != hipSuccess) return hip_fail(e);
  return RGF_OK;
}

int rgf_lead_modes(const rgf_ribbon_desc* desc, const double* energies_ev, int64_t n_energies,
                   int method, double* sigma_modes_out, int32_t* lead_status_out,
                   int32_t* n_modes_out, void* workspace, size_t workspace_bytes,
                   void* hip_stream) {
  if (method != 0 && method != 1)
    return fail(RGF_ERR_INVALID_ARG, "method = %d, expected 0 or 1", method);
  Plan p;
  int st = make_plan(desc, n_energies, 1, RGF_PREC_FP64, 0, 0, &p);
  if (st != RGF_OK) return st;
  if (n_modes_out) *n_modes_out = p.P;
  if (!sigma_modes_out && !lead_status_out) return RGF_OK;
  if (n_energies == 0) return RGF_OK;
  if (!energies_ev) return fail(RGF_ERR_INVALID_ARG, "energies_ev is NULL");
  st = check_ws(p, workspace, workspace_bytes);
  if (st != RGF_OK) return st;
  hipError_t e = launch_lead_modes(p, energies_ev, method, sigma_modes_out, lead_status_out,
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

int rgf_ldos(const rgf_ribbon_desc* desc, const double* energies_ev, int64_t n_energies,
             const double* onsite_eps_ev, int64_t n_real, int precision, double* ldos_out,
             double* T_out, int64_t ckpt_stride, int32_t* status_out, void* workspace,
             size_t workspace_bytes, void* hip_stream) {
  Plan p;
  int st = make_plan(desc, n_energies, n_real, precision, 1, ckpt_stride, &p);
  if (st != RGF_OK) return st;
  if (n_energies > 0) {
    if (!energies_ev) return fail(RGF_ERR_INVALID_ARG, "energies_ev is NULL");
    if (!ldos_out) return fail(RGF_ERR_INVALID_ARG, "ldos_out is NULL");
  }
  st = check_ws(p, workspace, workspace_bytes);
  if (st != RGF_OK) return st;
  hipError_t e = (p.large ? launch_ldos_large : launch_ldos)(
      p, energies_ev, onsite_eps_ev, ldos_out, T_out, status_out, (char*)workspace,
      (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e);
  return RGF_OK;
}

// Ribbons of several widths in one call: one persistent launch per ribbon
// on the caller's stream, most expensive (N^3 L) first; the workspace is
// reused from one launch to the next (stream order), so it is sized by the
// largest plan. The whole sequence can be captured into a hipGraph.
// Plans of a batched call. When every ribbon has enough tuples to fill the
// GPU by itself, the ribbons run one after another, each on the whole GPU,
// sharing one workspace (*concurrent = false): running them side by side
// then only fragments the compute units (a CU holding a narrow ribbon's
// workgroups cannot take a whole 8-wave workgroup of a wide one; measured
// 1.85x slower on the widths 60/120/240 workload). Otherwise every ribbon gets
// a share of the persistent workgroups proportional to its work and its own
// workspace part at base[d], and they run concurrently.
static int batched_plans(const rgf_ribbon_desc* descs, int32_t n_desc, int64_t n_energies,
                         int64_t n_real, int precision, Plan* plans, size_t* base,
                         size_t* bytes, bool* concurrent) {
  if (!descs) return fail(RGF_ERR_INVALID_ARG, "descs is NULL");
  if (n_desc < 1 || n_desc > 64)
    return fail(RGF_ERR_INVALID_ARG, "n_desc = %d outside [1, 64]", n_desc);
  double cost[64], total = 0.0;
  bool all_fill = true;
  for (int d = 0; d < n_desc; ++d) {
    int st = make_plan(&descs[d], n_energies, n_real, precision, 0, 0, &plans[d]);
    if (st != RGF_OK) {
      std::string m = rgf_last_error_message();
      return fail(st, "descs[%d]: %s", d, m.c_str());
    }
    const double n = plans[d].nmax;
    cost[d] = n * n * n * plans[d].L * (double)std::max<int64_t>(plans[d].ntuples, 1);
    total += cost[d];
    const int64_t slots = plans[d].large
                              ? persistent_grid_large(INT64_MAX, false)
                              : persistent_grid(plans[d].tile, INT64_MAX, precision, false,
                                                plans[d].per_cu);
    if (plans[d].ntuples < slots) all_fill = false;
  }
  *concurrent = n_desc > 1 && !all_fill;
  size_t off = 0, mx = 0;
  for (int d = 0; d < n_desc; ++d) {
    if (*concurrent) {
      const int cap = std::max(1, (int)ceil(plans[d].grid * cost[d] / total));
      int st = make_plan(&descs[d], n_energies, n_real, precision, 0, 0, &plans[d], cap);
      if (st != RGF_OK) return st;
      base[d] = off;
      off = align_up(off + plans[d].total, 256);
    } else {
      base[d] = 0;
      mx = std::max(mx, plans[d].total);
    }
  }
  *bytes = std::max<size_t>(*concurrent ? off : mx, 256);
  return RGF_OK;
}

size_t rgf_batched_workspace_bytes(const rgf_ribbon_desc* descs, int32_t n_desc,
                                   int64_t n_energies, int64_t n_real, int precision) {
  Plan plans[64];
  size_t base[64], bytes = 0;
  bool conc = false;
  if (batched_plans(descs, n_desc, n_energies, n_real, precision, plans, base, &bytes, &conc) !=
      RGF_OK)
    return 0;
  return bytes;
}

namespace {
// Streams the batched call forks onto (default priority, non-blocking), with
// the events of the fork and the joins; one set per device, used under a
// lock for the whole enqueue so that concurrent calls do not interleave
// their records and waits.
constexpr int kBatchStreams = 7;
struct BatchPool {
  bool ok = false;
  hipStream_t st[kBatchStreams];
  hipEvent_t fork, join[kBatchStreams];
};
std::mutex g_pool_mu;
std::map<int, BatchPool> g_pool;

BatchPool* batch_pool() {
  int dev = 0;
  if (!current_device(&dev)) return nullptr;
  BatchPool& p = g_pool[dev];
  if (p.ok) return &p;
  for (int i = 0; i < kBatchStreams; ++i)
    if (hipStreamCreateWithFlags(&p.st[i], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p.join[i], hipEventDisableTiming) != hipSuccess)
      return nullptr;
  if (hipEventCreateWithFlags(&p.fork, hipEventDisableTiming) != hipSuccess) return nullptr;
  p.ok = true;
  return &p;
}
}  // namespace

int rgf_conductance_batched(const rgf_ribbon_desc* descs, int32_t n_desc,
                            const int64_t* eps_offsets, const int64_t* T_offsets,
                            const double* energies_ev, int64_t n_energies,
                            const double* onsite_eps_ev, int64_t n_real, int precision,
                            double* T_out, int32_t* status_out, void* workspace,
                            size_t workspace_bytes, void* hip_stream) {
  Plan plans[64];
  size_t base[64], bytes = 0;
  bool concurrent = false;
  int st = batched_plans(descs, n_desc, n_energies, n_real, precision, plans, base, &bytes,
                         &concurrent);
  if (st != RGF_OK) return st;
  if (n_energies == 0) return RGF_OK;
  if (!energies_ev) return fail(RGF_ERR_INVALID_ARG, "energies_ev is NULL");
  if (!T_out) return fail(RGF_ERR_INVALID_ARG, "T_out is NULL");
  if (!T_offsets) return fail(RGF_ERR_INVALID_ARG, "T_offsets is NULL");
  if (onsite_eps_ev && !eps_offsets) return fail(RGF_ERR_INVALID_ARG, "eps_offsets is NULL");
  for (int d = 0; d < n_desc; ++d) {
    if (T_offsets[d] < 0 || (onsite_eps_ev && eps_offsets[d] < 0))
      return fail(RGF_ERR_INVALID_ARG, "negative offset for descs[%d]", d);
  }
  if (workspace_bytes < bytes)
    return fail(RGF_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", workspace_bytes, bytes);
  if (!workspace || ((uintptr_t)workspace) % 256 != 0)
    return fail(RGF_ERR_INVALID_ARG, "workspace must be non-NULL and 256-byte aligned");
  int order[64];
  for (int d = 0; d < n_desc; ++d) order[d] = d;
  std::stable_sort(order, order + n_desc, [&](int x, int y) {
    const double cx = (double)plans[x].nmax * plans[x].nmax * plans[x].nmax * plans[x].L;
    const double cy = (double)plans[y].nmax * plans[y].nmax * plans[y].nmax * plans[y].L;
    return cx > cy;
  });
  hipStream_t s = (hipStream_t)hip_stream;
  auto launch = [&](int d, hipStream_t on) {
    const double* eps = onsite_eps_ev ? onsite_eps_ev + eps_offsets[d] : nullptr;
    return launch_forward(plans[d], energies_ev, eps, T_out + T_offsets[d],
                          status_out ? status_out + T_offsets[d] : nullptr,
                          (char*)workspace + base[d], on);
  };
  if (!concurrent) {  // one after another on the caller's stream, each on the whole GPU
    for (int i = 0; i < n_desc; ++i) {
      hipError_t e = launch(order[i], s);
      if (e != hipSuccess) return hip_fail(e);
    }
    return RGF_OK;
  }
  std::lock_guard<std::mutex> lk(g_pool_mu);
  BatchPool* pool = batch_pool();
  if (!pool) {
    (void)hipGetLastError();
    return fail(RGF_ERR_HIP, "could not create the batched call's streams");
  }
  // fork: the other ribbons' streams wait for the work queued on s so far
  hipError_t e = hipEventRecord(pool->fork, s);
  const int used = std::min(n_desc - 1, kBatchStreams);
  for (int j = 0; e == hipSuccess && j < used; ++j)
    e = hipStreamWaitEvent(pool->st[j], pool->fork, 0);
  // the costliest ribbon on s, the others round-robin on the pool's streams
  for (int i = 0; e == hipSuccess && i < n_desc; ++i)
    e = launch(order[i], i == 0 ? s : pool->st[(i - 1) % kBatchStreams]);
  // join: s waits for every forked stream (also after a failed launch, so
  // that no stream is left forked from a capture)
  for (int j = 0; j < used; ++j) {
    hipError_t r = hipEventRecord(pool->join[j], pool->st[j]);
    if (r == hipSuccess) r = hipStreamWaitEvent(s, pool->join[j], 0);
    if (e == hipSuccess) e = r;
  }
  return e == hipSuccess ? RGF_OK : hip_fail(e);
}

// ---------------------------------------------------------------- autotuner

namespace {
constexpr int kTuneL = 8;

struct TuneShape {
  int64_t nE;
};

int tune_plan(const rgf_ribbon_desc* desc, int precision, rgf_ribbon_desc* dd,
              TuneShape* ts) {
  int st = validate_desc(desc);
  if (st != RGF_OK) return st;
  *dd = *desc;
  dd->length_l = std::min(desc->length_l, kTuneL);
  ts->nE = (int64_t)device_cu_count() * 4;  // enough tuples for every grid size tried
  if ((desc->width_n + 1) / 2 > kTileMaxRows && precision != RGF_PREC_FP64)
    return fail(RGF_ERR_UNSUPPORTED, "width_n = %d: half-slices above %d rows run in FP64 only",
                desc->width_n, kTileMaxRows);
  return RGF_OK;
}

size_t tune_bytes_for(const rgf_ribbon_desc* dd, int64_t nE, int precision) {
  // energies + T of the trial sweep, then the largest plan over all candidate
  // tilings at their full persistent grid
  const int n = (dd->width_n + 1) / 2;
  const int P = lead_modes(dd->width_n);
  const int mats = slot_matrices(precision, false);
  size_t mx = 0;
  for (int i = 0; i < tile_count(); ++i) {
    const TileCfg t = tile_at(i);
    if (t.NP() < n || 64 * t.S < t.NP()) continue;
    const size_t NP = (size_t)t.NP();
    const bool fallback = precision != RGF_PREC_FP32;  // flags + whole-slice slots
    const size_t head = align_up((size_t)nE * P * 16, 256) + align_up(2 * (size_t)P * NP * 8, 256) +
                        align_up((size_t)nE * 4, 256) +
                        (fallback ? align_up((size_t)nE * 4, 256) : 0);
    size_t slots = (size_t)persistent_grid(t, nE, precision, false) * mats * NP * NP * 16;
    if (fallback) slots = std::max(slots, whole_slot_bytes(dd->width_n));
    mx = std::max(mx, head + align_up(slots, 256));
  }
  return align_up((size_t)nE * 16, 256) + mx;
}
}  // namespace

size_t rgf_autotune_workspace_bytes(const rgf_ribbon_desc* desc, int precision) {
  rgf_ribbon_desc dd;
  TuneShape ts;
  if (tune_plan(desc, precision, &dd, &ts) != RGF_OK) return 0;
  if (precision < 0 || precision > 2) {
    fail(RGF_ERR_INVALID_ARG, "precision = %d unknown", precision);
    return 0;
  }
  return tune_bytes_for(&dd, ts.nE, precision);
}

int rgf_autotune(const rgf_ribbon_desc* desc, int precision, void* workspace,
                 size_t workspace_bytes, void* hip_stream, int32_t* chosen_out) {
  rgf_ribbon_desc dd;
  TuneShape ts;
  int st = tune_plan(desc, precision, &dd, &ts);
  if (st != RGF_OK) return st;
  if (precision < 0 || precision > 2)
    return fail(RGF_ERR_INVALID_ARG, "precision = %d unknown", precision);
  const size_t need = tune_bytes_for(&dd, ts.nE, precision);
  if (workspace_bytes < need)
    return fail(RGF_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", workspace_bytes, need);
  if (!workspace || ((uintptr_t)workspace) % 256 != 0)
    return fail(RGF_ERR_INVALID_ARG, "workspace must be non-NULL and 256-byte aligned");
  if ((dd.width_n + 1) / 2 > kTileMaxRows) {
    // one blocked kernel serves every width above the register tilings:
    // nothing to choose
    if (chosen_out) {
      const TileCfg t = large_block_tile();
      *chosen_out = t.NW * 10000 + t.S * 1000 + t.C * 10;
    }
    return RGF_OK;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  char* base = (char*)workspace;
  double* E = (double*)base;
  double* T = E + ts.nE;
  char* ws = base + align_up((size_t)ts.nE * 16, 256);
  const size_t ws_bytes = workspace_bytes - (size_t)(ws - base);
  std::vector<double> hE((size_t)ts.nE);
  for (int64_t i = 0; i < ts.nE; ++i)
    hE[(size_t)i] = dd.hopping_ev * (-0.9 + 1.8 * (double)i / (double)(ts.nE - 1 + (ts.nE == 1)));
  hipError_t he = hipMemcpyAsync(E, hE.data(), (size_t)ts.nE * 8, hipMemcpyHostToDevice, s);
  if (he != hipSuccess) return hip_fail(he);
  const int n = (dd.width_n + 1) / 2;
  hipEvent_t e0, e1;
  if ((he = hipEventCreate(&e0)) != hipSuccess) return hip_fail(he);
  if ((he = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(he);
  }
  float best = 1e30f;
  int best_tile = -1, best_pc = 0;
  for (int i = 0; i < tile_count(); ++i) {
    TileCfg t = tile_at(i);
    if (t.NP() < n || 64 * t.S < t.NP()) continue;
    for (int pc : {0, 1}) {
      set_tuned_choice(n, precision, i, pc);
      Plan p;
      if (make_plan(&dd, ts.nE, 1, precision, 0, 0, &p) != RGF_OK) continue;
      if (p.total > ws_bytes) continue;
      float ms_best = 1e30f;
      for (int rep = 0; rep < 3 && he == hipSuccess; ++rep) {
        he = hipEventRecord(e0, s);
        if (he == hipSuccess) he = launch_forward(p, E, nullptr, T, nullptr, ws, s);
        if (he == hipSuccess) he = hipEventRecord(e1, s);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) ms_best = std::min(ms_best, ms);  // first run warms up
      }
      if (he != hipSuccess) break;
      if (ms_best < best) {
        best = ms_best;
        best_tile = i;
        best_pc = pc;
      }
      // one slot per CU is already the occupancy limit: nothing else to try
      if (pc == 0 && persistent_grid(t, 1 << 30, precision, false, 1) ==
                         persistent_grid(t, 1 << 30, precision, false, 0))
        break;
    }
    if (he != hipSuccess) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (he != hipSuccess) return hip_fail(he);
  if (best_tile < 0) return fail(RGF_ERR_UNSUPPORTED, "no register tiling holds width %d", dd.width_n);
  set_tuned_choice(n, precision, best_tile, best_pc);
  if (chosen_out) {
    TileCfg t = tile_at(best_tile);
    *chosen_out = (t.mgj ? 100000 : 0) + t.NW * 10000 + t.S * 1000 + t.C * 10 + best_pc;
  }
  return RGF_OK;
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

int rgf_refine_stats(uint64_t* counts_out, int reset, void* hip_stream) {
  if (!counts_out) return fail(RGF_ERR_INVALID_ARG, "counts_out is NULL");
  unsigned long long* c = device_refine_stats();
  if (!c) return fail(RGF_ERR_HIP, "no device counters (no current HIP device)");
  hipError_t e = hipStreamSynchronize((hipStream_t)hip_stream);
  if (e == hipSuccess) e = hipMemcpy(counts_out, c, 3 * sizeof(uint64_t), hipMemcpyDeviceToHost);
  if (e == hipSuccess && reset) {
    static const uint64_t zeros[3] = {0, 0, 0};
    e = hipMemcpy(c, zeros, sizeof(zeros), hipMemcpyHostToDevice);
  }
  return e == hipSuccess ? RGF_OK : hip_fail(e);
}

int rgf_version(int* major, int* minor) {
  if (major) *major = RGF_ABI_VERSION_MAJOR;
  if (minor) *minor = RGF_ABI_VERSION_MINOR;
  return RGF_OK;
}

}  // extern "C"
