"""rgf_conductance_noalloc: the conductance sweep in the library's fixed
device scratch (no workspace argument, nothing allocated by the call),
checked through the C ABI against rgf_conductance on the same inputs."""

import ctypes
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBP = os.path.join(ROOT, "paper_1107_5300_amd", "librgf.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIBP), reason="librgf.so not built")


def test_noalloc_rejects_oversized_calls_before_enqueue():
    """Lead tables that alone exceed the fixed scratch are refused with
    RGF_ERR_WORKSPACE before any HIP call (runs without a GPU)."""
    from paper_1107_5300_amd import _lib as L
    lib = L.lib()
    d = L.make_desc(240, 10)
    # sigma alone: n_E * 120 modes * 16 bytes > 192 MiB
    nE = (192 << 20) // (120 * 16) + 1
    rc = lib.rgf_conductance_noalloc(ctypes.byref(d), ctypes.c_void_p(256), nE, None, 1, 0,
                                     ctypes.c_void_p(256), None, None)
    assert rc == L.RGF_ERR_WORKSPACE
    assert b"scratch" in lib.rgf_last_error_message()
    # argument errors as for rgf_conductance
    assert lib.rgf_conductance_noalloc(ctypes.byref(d), None, 4, None, 1, 0,
                                       ctypes.c_void_p(256), None, None) == L.RGF_ERR_INVALID_ARG
    assert lib.rgf_conductance_noalloc(ctypes.byref(d), ctypes.c_void_p(256), 4, None, 1, 0,
                                       None, None, None) == L.RGF_ERR_INVALID_ARG
    assert lib.rgf_conductance_noalloc(ctypes.byref(d), None, 0, None, 1, 0, None, None,
                                       None) == L.RGF_OK


def _call_both(lib, L, torch, N, Lc, nE, R, precision, seed):
    import rgf_workloads as W
    dev = torch.device("cuda:0")
    d = L.make_desc(N, Lc, 0, W.T_HOP, W.ETA)
    Es = torch.tensor(np.linspace(-0.45, 0.43, nE) * abs(W.T_HOP), device=dev)
    eps = torch.tensor(np.stack([W.disorder(Lc, N, 0.5, r=seed + r) for r in range(R)]),
                       device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # reference: rgf_conductance with a caller workspace
    nbytes = lib.rgf_workspace_bytes(ctypes.byref(d), nE, R, precision, 0, 0)
    assert nbytes > 0
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    T0 = torch.full((R, nE), -1.0, dtype=torch.float64, device=dev)
    s0 = torch.full((R, nE), -7, dtype=torch.int32, device=dev)
    L.check(lib.rgf_conductance(ctypes.byref(d), ctypes.c_void_p(Es.data_ptr()), nE,
                                ctypes.c_void_p(eps.data_ptr()), R, precision,
                                ctypes.c_void_p(T0.data_ptr()), ctypes.c_void_p(s0.data_ptr()),
                                ctypes.c_void_p(ws.data_ptr()), nbytes, stream))
    T1 = torch.full((R, nE), -1.0, dtype=torch.float64, device=dev)
    s1 = torch.full((R, nE), -7, dtype=torch.int32, device=dev)
    L.check(lib.rgf_conductance_noalloc(ctypes.byref(d), ctypes.c_void_p(Es.data_ptr()), nE,
                                        ctypes.c_void_p(eps.data_ptr()), R, precision,
                                        ctypes.c_void_p(T1.data_ptr()),
                                        ctypes.c_void_p(s1.data_ptr()), stream))
    torch.cuda.synchronize()
    return T0.cpu().numpy(), s0.cpu().numpy(), T1.cpu().numpy(), s1.cpu().numpy()


@pytest.mark.gpu
def test_noalloc_matches_workspace_call_twice():
    """Two calls in a row, the second smaller, each equal to rgf_conductance
    on the same inputs. The first (N = 480: 5.5 MB per workgroup slot) needs
    more slots than the fixed scratch holds, so it runs on a reduced
    persistent grid; every tuple's arithmetic is the same, so the results
    agree bit for bit."""
    import torch
    from paper_1107_5300_amd import _lib as L
    lib = L.lib()
    print("noalloc case 1: N=480 L=4 nE=48 R=1 fp64", flush=True)
    T0, s0, T1, s1 = _call_both(lib, L, torch, 480, 4, 48, 1, L.RGF_PREC_FP64, 60)
    assert (s0 == 0).all() and (s1 == 0).all()
    assert np.array_equal(T0, T1), np.abs(T0 - T1).max()
    print("noalloc case 2: N=60 L=30 nE=20 R=2 fp64", flush=True)
    T0, s0, T1, s1 = _call_both(lib, L, torch, 60, 30, 20, 2, L.RGF_PREC_FP64, 70)
    assert (s0 == 0).all() and (s1 == 0).all()
    assert np.array_equal(T0, T1), np.abs(T0 - T1).max()


@pytest.mark.gpu
def test_noalloc_mixed_precision_reduced_grid():
    """Mixed precision at N = 240 needs four matrices per slot, so the fixed
    scratch holds fewer slots than compute units; results equal the
    workspace call's."""
    import torch
    from paper_1107_5300_amd import _lib as L
    lib = L.lib()
    print("noalloc case 3: N=240 L=6 nE=300 R=1 mixed", flush=True)
    T0, s0, T1, s1 = _call_both(lib, L, torch, 240, 6, 300, 1, L.RGF_PREC_MIXED, 80)
    assert (s0 == s1).all()
    assert np.array_equal(T0, T1), np.nanmax(np.abs(T0 - T1))
