// rgf_segplan.hpp -- host-side plan of the conductance recursion split
// along the ribbon length (csrc/rgf_segment.hip), shared by the entry point
// and the launcher.

#pragma once

#include "rgf_internal.hpp"

namespace rgf {

// The conductance recursion split along the length (parallel in L,
// csrc/rgf_segment.hip). fwd: the ribbon's plan (its lead tables, the
// accuracy fallback's flags and slots); aux: the plan of a pristine ribbon
// of the same width and odd length, parity 0, whose lead tables (at
// off_aux) hold the mode tables of both row classes. Per tuple G segments,
// each with three NP x NP matrices at off_mats; a merge's eight work
// matrices per workgroup at off_scratch; per item and merge (ksum, ksum_c)
// and a flag at off_kap / off_flag; the reversed on-site energies at
// off_eps_rev.
struct SegPlan {
  Plan fwd, aux;
  int G;
  int sweep_grid, merge_grid, join_grid;
  size_t off_aux, off_eps_rev, off_mats, off_scratch, off_kap, off_flag, total;
};
int make_seg_plan(const rgf_ribbon_desc* d, int64_t nE, int64_t nreal, int n_segments,
                  SegPlan* sp);
hipError_t launch_segments(const SegPlan& sp, const double* E, const double* eps,
                           double* T_out, int32_t* status_out, char* ws, hipStream_t s);
// Whether the segment kernels exist for a register tiling, and the kernel
// entry of the segment sweep (for occupancy queries).
bool seg_supported(const TileCfg& t);
const void* seg_sweep_kernel(const TileCfg& t);

}  // namespace rgf
