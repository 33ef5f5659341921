// rgf_noalloc.hip -- the conductance sweep for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops): the
// same kernels as rgf_conductance, with the workspace in a fixed device
// array of this library instead of a caller buffer.
//
// `scratch` below is a device variable. In host code its name is only a
// host-side stand-in: its device address differs per GPU and is obtained
// once per device with hipGetSymbolAddress, then kept in g_scratch[dev]; the
// kernels receive that address, exactly as they receive a caller workspace.

#include <algorithm>
#include <mutex>

#include "rgf_internal.hpp"

namespace rgf {

namespace {

constexpr size_t kScratchBytes = (size_t)RGF_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size must keep the 256-byte workspace alignment");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices];  // device address of `scratch` on each device (null: not resolved)

// Device address of the scratch array on the current device, resolved on the
// first call for that device.
int scratch_on_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    set_error("hipGetDevice failed: %s", hipGetErrorString(e));
    return RGF_ERR_HIP;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device ordinal %d outside [0, %d)", dev, kMaxDevices);
    return RGF_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error("hipGetSymbolAddress(scratch) on device %d failed: %s", dev,
                hipGetErrorString(e));
      return RGF_ERR_HIP;
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return RGF_OK;
}

}  // namespace

}  // namespace rgf

using namespace rgf;

extern "C" int rgf_conductance_noalloc(const rgf_ribbon_desc* desc, const double* energies_ev,
                                       int64_t n_energies, const double* onsite_eps_ev,
                                       int64_t n_real, int precision, double* T_out,
                                       int32_t* status_out, void* hip_stream) {
  Plan p;
  int st = make_plan(desc, n_energies, n_real, precision, 0, 0, &p);
  if (st != RGF_OK) return st;
  if (n_energies == 0) return RGF_OK;
  if (!energies_ev) {
    set_error("energies_ev is NULL");
    return RGF_ERR_INVALID_ARG;
  }
  if (!T_out) {
    set_error("T_out is NULL");
    return RGF_ERR_INVALID_ARG;
  }
  if (p.total > kScratchBytes) {
    // fewer persistent workgroups (each needs its own slot) until it fits
    const size_t slot = (size_t)p.slot_mats * (size_t)p.slot_elems * 16;
    const size_t head = p.off_slots;
    const int64_t cap = head < kScratchBytes ? (int64_t)((kScratchBytes - head) / slot) : 0;
    if (cap < 1) {
      set_error("the call needs %zu bytes of scratch for its lead tables and one slot; the "
                "fixed scratch holds %zu (use rgf_conductance with a workspace)",
                head + slot, kScratchBytes);
      return RGF_ERR_WORKSPACE;
    }
    st = make_plan(desc, n_energies, n_real, precision, 0, 0, &p,
                   (int)std::min<int64_t>(cap, 1 << 30));
    if (st != RGF_OK) return st;
    if (p.total > kScratchBytes) {
      set_error("scratch plan of %zu bytes exceeds the fixed %zu", p.total, kScratchBytes);
      return RGF_ERR_WORKSPACE;
    }
  }
  void* ws = nullptr;
  st = scratch_on_current_device(&ws);
  if (st != RGF_OK) return st;
  hipError_t e = launch_forward(p, energies_ev, onsite_eps_ev, T_out, status_out, (char*)ws,
                                (hipStream_t)hip_stream);
  if (e != hipSuccess) {
    set_error("HIP error %d: %s", (int)e, hipGetErrorString(e));
    return RGF_ERR_HIP;
  }
  return RGF_OK;
}
