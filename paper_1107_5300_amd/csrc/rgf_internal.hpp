// rgf_internal.hpp -- host-side plan shared by the C ABI and the launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/rgf.h"

namespace rgf {

// Register tiling of one workgroup: NW waves; lane l owns rows l + 64 s
// (s < S) and wave w owns columns w*C .. w*C + C - 1 of every n x n matrix
// of the half-slice recursion, padded to NP = NW*C with the identity.
struct TileCfg {
  int id;  // index into the kernel table of a launcher
  int NW, S, C;
  bool mgj = false;  // forward sweep with the matrix-core Gauss-Jordan (same NW, S, C)
  int NP() const { return NW * C; }
  int threads() const { return NW * 64; }
};

// Pick the smallest register tiling whose padded size NP holds n rows.
// Returns false if n exceeds the largest tiling.
bool pick_tile(int n, int precision, TileCfg* out);

// All tilings (in table order) and the table size.
int tile_count();
int device_cu_count();
TileCfg tile_at(int i);

// Autotuned choice for (n, precision): tile id and slots per CU (0 = not tuned).
bool tuned_choice(int n, int precision, int* tile_id, int* per_cu);
void set_tuned_choice(int n, int precision, int tile_id, int per_cu);

// Number of transverse modes of the lead (mode pairs plus the middle mode of
// odd N).
inline int lead_modes(int N) { return (N + 1) / 2; }

// Half-slices wider than the widest register tiling (n > kTileMaxRows) take
// the blocked path of rgf_large.hip: matrices in the workspace with leading
// dimension kLargeLd, inverted by panels, FP64 forward only.
constexpr int kTileMaxRows = 128;
constexpr int kLargeLd = 256;

// Byte layout of one call's workspace.
struct Plan {
  int N, L, parity, P, n1, nmax;
  double t, eta;
  int64_t nE, nreal, ntuples;
  int precision;
  TileCfg tile;
  int grid;           // persistent workgroups
  int per_cu;         // forced slots per CU (0 = occupancy limit)
  int64_t slot_elems; // complex elements of one matrix buffer (NP*NP)
  int64_t mat_elems;  // complex elements of one stored restart matrix
  int slot_mats;      // matrix buffers per slot
  // byte offsets
  size_t off_sigma, off_phi, off_lstat, off_status, off_slots, off_ckpt, off_seg,
      total;
  int64_t ckpt_stride, n_ckpt;
  bool want_grad;
  bool large;   // blocked path (n > kTileMaxRows)
  int phi_ld;   // leading dimension of the lead mode tables
  // accuracy fallback of the conductance sweeps: per-tuple flags (int32)
  // and the whole-slice workgroups, whose buffers reuse the slot region
  size_t off_flags;
  int fb_grid;  // 0: no fallback (gradient, LDOS, FP32 study mode)
};

// The current device's counters of the mixed mode's refinement (device
// address of three 64-bit counters, see rgf_refine_stats), or null.
unsigned long long* device_refine_stats();

// Fill the plan; returns RGF_OK or an error code (with message set).
// grid_cap > 0 limits the persistent grid (fewer slots, a smaller workspace).
int make_plan(const rgf_ribbon_desc* d, int64_t nE, int64_t nreal, int precision,
              int want_grad, int64_t ckpt_stride, Plan* p, int grid_cap = 0);

void set_error(const char* fmt, ...);

// Launchers (enqueue only; return hipError_t).
// method 0: Sancho-Rubio decimation per transverse mode; 1: the closed-form
// root of each mode chain's surface equation (mode matching).
hipError_t launch_lead(const Plan& p, const double* E, char* ws, hipStream_t s,
                       int method = 0);
// tchan (optional): transmission per incoming lead channel, [nreal][nE][P].
hipError_t launch_forward(const Plan& p, const double* E, const double* eps,
                          double* T_out, int32_t* status_out, char* ws,
                          hipStream_t s, double* tchan = nullptr);
// Per-mode lead self-energies sigma_p ([nE][P] complex128 as (re, im)) by
// either method, and the lead status.
hipError_t launch_lead_modes(const Plan& p, const double* E, int method, double* sigma_out,
                             int32_t* lstat_out, char* ws, hipStream_t s);
hipError_t launch_export_sigma(const Plan& p, const double* E, double* sl,
                               double* sr, int32_t* lstat_out, char* ws,
                               hipStream_t s);
hipError_t launch_grad(const Plan& p, const double* E, const double* eps,
                       const double* dL_dT, double* T_out, double* dL_deps,
                       int32_t* status_out, char* ws, hipStream_t s);

// Persistent grid size for a tile config on the current device.
int persistent_grid(const TileCfg& t, int64_t ntuples, int precision, bool grad,
                    int per_cu = 0);
// The same for the blocked wide-half-slice kernels.
int persistent_grid_large(int64_t ntuples, bool grad);

// Kernel entry of the forward sweep / adjoint for a tile and precision.
const void* fwd_kernel_ptr(const TileCfg& t, int precision);
hipError_t launch_ldos(const Plan& p, const double* E, const double* eps, double* ldos,
                       double* T_out, int32_t* status_out, char* ws, hipStream_t s);
const void* grad_kernel_ptr(const TileCfg& t, int precision);

// Matrix buffers (NP x NP complex128) per persistent slot.
int slot_matrices(int precision, bool grad);

struct SweepArgs;
// Whole-slice recursion for the tuples flagged by a conductance sweep whose
// arguments are `fwd` (launched after it on the same stream), and the bytes
// one of its workgroups needs for width N.
hipError_t launch_whole_fallback(const Plan& p, const SweepArgs& fwd, char* ws, hipStream_t s);
size_t whole_slot_bytes(int N);

// Blocked forward sweep, gradient and local density of states for
// kTileMaxRows < n <= kLargeLd (FP64).
hipError_t launch_forward_large(const Plan& p, const double* E, const double* eps,
                                double* T_out, int32_t* status_out, char* ws, hipStream_t s,
                                double* tchan);
hipError_t launch_grad_large(const Plan& p, const double* E, const double* eps,
                             const double* dL_dT, double* T_out, double* dL_deps,
                             int32_t* status_out, char* ws, hipStream_t s);
hipError_t launch_ldos_large(const Plan& p, const double* E, const double* eps, double* ldos,
                             double* T_out, int32_t* status_out, char* ws, hipStream_t s);
const void* large_kernel_ptr(bool grad);
// Register tiling of the blocked kernels' elimination panels (id -1: not a
// table entry), and their buffers per slot in units of kTileMaxRows^2
// complex128.
TileCfg large_block_tile();
int large_slot_blocks(bool grad);

}  // namespace rgf
