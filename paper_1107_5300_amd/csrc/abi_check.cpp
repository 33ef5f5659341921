// abi_check.cpp -- host-only driver of librgf's argument validation and
// workspace planning, built with AddressSanitizer and UndefinedBehaviorSanitizer
// on the host side (paper_1107_5300_amd/build.py: build_abi_check). It calls
// every entry point with invalid and valid arguments that must be rejected
// or planned before anything is enqueued, so it runs without a GPU. Exit
// status 0 when every check holds; sanitizer reports abort the process.

#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "../../include/rgf.h"

static int g_fail = 0;

#define CHECK(cond)                                                     \
  do {                                                                  \
    if (!(cond)) {                                                      \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      g_fail = 1;                                                       \
    }                                                                   \
  } while (0)

static rgf_ribbon_desc desc(int N, int L, int parity = 0) {
  rgf_ribbon_desc d;
  memset(&d, 0, sizeof(d));
  d.struct_size = sizeof(d);
  d.width_n = N;
  d.length_l = L;
  d.parity = parity;
  d.hopping_ev = -2.7;
  d.eta_ev = 1e-8;
  return d;
}

int main() {
  void* const fake = (void*)(uintptr_t)4096;  // never dereferenced: rejected earlier
  double* const fd = (double*)fake;
  // descriptors
  rgf_ribbon_desc bad = desc(20, 10);
  bad.struct_size = 8;
  CHECK(rgf_conductance(&bad, fd, 4, nullptr, 1, 0, fd, nullptr, nullptr, 0, nullptr) ==
        RGF_ERR_INVALID_ARG);
  CHECK(strlen(rgf_last_error_message()) > 0);
  CHECK(rgf_conductance(nullptr, fd, 4, nullptr, 1, 0, fd, nullptr, nullptr, 0, nullptr) ==
        RGF_ERR_INVALID_ARG);
  for (int N : {1, 513, 100000}) {
    rgf_ribbon_desc d = desc(N, 10);
    CHECK(rgf_workspace_bytes(&d, 4, 1, 0, 0, 0) == 0);
  }
  rgf_ribbon_desc d = desc(20, 10);
  d.eta_ev = -1.0;
  CHECK(rgf_workspace_bytes(&d, 4, 1, 0, 0, 0) == 0);
  d = desc(20, 10);
  d.hopping_ev = 0.0;
  CHECK(rgf_workspace_bytes(&d, 4, 1, 0, 0, 0) == 0);
  // workspace planning over widths, precisions, gradients and strides
  for (int N : {2, 3, 20, 61, 120, 200, 240, 256, 257, 480, 512})
    for (int prec : {0, 1, 2})
      for (int grad : {0, 1})
        for (int stride : {0, 1, 7}) {
          rgf_ribbon_desc w = desc(N, 9, N % 2);
          const size_t b = rgf_workspace_bytes(&w, 17, 3, prec, grad, stride);
          const bool wide = N > RGF_TILE_MAX_WIDTH;
          CHECK((b > 0) == (!wide || prec == RGF_PREC_FP64));
        }
  // null pointers, undersized and misaligned workspaces
  rgf_ribbon_desc g = desc(24, 6);
  const size_t need = rgf_workspace_bytes(&g, 4, 1, 0, 0, 0);
  CHECK(need > 0);
  CHECK(rgf_conductance(&g, nullptr, 4, nullptr, 1, 0, fd, nullptr, fake, need, nullptr) ==
        RGF_ERR_INVALID_ARG);
  CHECK(rgf_conductance(&g, fd, 4, nullptr, 1, 0, fd, nullptr, fake, need - 1, nullptr) ==
        RGF_ERR_WORKSPACE);
  CHECK(rgf_conductance(&g, fd, 4, nullptr, 1, 0, fd, nullptr, (char*)fake + 8, need, nullptr) ==
        RGF_ERR_INVALID_ARG);
  CHECK(rgf_conductance(&g, fd, -1, nullptr, 1, 0, fd, nullptr, fake, need, nullptr) ==
        RGF_ERR_INVALID_ARG);
  CHECK(rgf_conductance(&g, fd, 4, nullptr, 0, 0, fd, nullptr, fake, need, nullptr) ==
        RGF_ERR_INVALID_ARG);
  CHECK(rgf_conductance(&g, nullptr, 0, nullptr, 1, 0, nullptr, nullptr, nullptr, 0, nullptr) ==
        RGF_OK);
  CHECK(rgf_channel_transmission(&g, fd, 4, nullptr, 1, 1, fd, fd, nullptr, fake, need,
                                 nullptr) == RGF_ERR_UNSUPPORTED);
  CHECK(rgf_grad(&g, fd, 4, fd, 1, 0, nullptr, fd, fd, 0, nullptr, fake, need, nullptr) ==
        RGF_ERR_INVALID_ARG);
  CHECK(rgf_ldos(&g, fd, 4, nullptr, 1, 0, nullptr, nullptr, 0, nullptr, fake, need, nullptr) ==
        RGF_ERR_INVALID_ARG);
  // the no-allocation entry point: oversized lead tables are refused
  rgf_ribbon_desc big = desc(240, 10);
  CHECK(rgf_conductance_noalloc(&big, fd, ((int64_t)192 << 20) / (120 * 16) + 1, nullptr, 1, 0,
                                fd, nullptr, nullptr) == RGF_ERR_WORKSPACE);
  // batched plans
  rgf_ribbon_desc ds[3] = {desc(60, 5), desc(120, 5), desc(240, 5)};
  CHECK(rgf_batched_workspace_bytes(ds, 3, 8, 2, 1) > 0);
  CHECK(rgf_batched_workspace_bytes(ds, 0, 8, 2, 1) == 0);
  CHECK(rgf_batched_workspace_bytes(ds, 65, 8, 2, 1) == 0);
  int64_t offs[3] = {0, -5, 10};
  CHECK(rgf_conductance_batched(ds, 3, offs, offs, fd, 8, fd, 2, 0, fd, nullptr, fake,
                                (size_t)1 << 40, nullptr) == RGF_ERR_INVALID_ARG);
  // size queries
  int32_t nl = 0, nr = 0, P = 0;
  rgf_ribbon_desc s7 = desc(7, 3);
  CHECK(rgf_lead_self_energy(&s7, nullptr, 0, nullptr, nullptr, nullptr, &nl, &nr, nullptr, 0,
                             nullptr) == RGF_OK);
  CHECK(nl == 4 && nr == 3);
  CHECK(rgf_lead_modes(&s7, nullptr, 0, 0, nullptr, nullptr, &P, nullptr, 0, nullptr) == RGF_OK);
  CHECK(P == 4);
  CHECK(rgf_lead_modes(&s7, nullptr, 0, 2, nullptr, nullptr, &P, nullptr, 0, nullptr) ==
        RGF_ERR_INVALID_ARG);
  // autotuner sizing
  rgf_ribbon_desc t = desc(480, 20);
  CHECK(rgf_autotune_workspace_bytes(&t, 0) > 0);
  CHECK(rgf_autotune_workspace_bytes(&t, 1) == 0);
  CHECK(rgf_refine_stats(nullptr, 0, nullptr) == RGF_ERR_INVALID_ARG);
  // segments along the length: argument errors before anything is enqueued
  rgf_ribbon_desc sg = desc(60, 40);
  CHECK(rgf_segments_workspace_bytes(&sg, 4, 1, -1) == 0);
  CHECK(rgf_segments_workspace_bytes(&t, 4, 1, 0) == 0);   /* N = 480: unsupported */
  CHECK(rgf_conductance_segments(&sg, nullptr, 4, nullptr, 1, 4, nullptr, nullptr, nullptr,
                                 nullptr, 0, nullptr) != RGF_OK);
  int a = 0, b = 0;
  CHECK(rgf_version(&a, &b) == RGF_OK && a == RGF_ABI_VERSION_MAJOR);
  CHECK(strcmp(rgf_status_string(RGF_ERR_WORKSPACE), "RGF_ERR_WORKSPACE") == 0);
  printf(g_fail ? "abi_check: FAILED\n" : "abi_check: ok\n");
  return g_fail;
}
