"""Python/torch binding of librgf (argument marshalling only).

Every numeric step runs in the HIP kernels of librgf.so; torch provides
device memory (the call's workspace and outputs) and the stream. Inputs must
be float64 tensors on the current CUDA (HIP) device.
"""

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as _L

PRECISIONS = {"fp64": _L.RGF_PREC_FP64, "mixed": _L.RGF_PREC_MIXED, "fp32": _L.RGF_PREC_FP32}


@dataclass(frozen=True)
class Ribbon:
    """Armchair ribbon: N atoms per slice, L slices, hopping t and broadening
    eta in eV; slice i bonds rows (k + i + parity) even to slice i+1."""
    N: int
    L: int
    parity: int = 0
    t: float = -2.7
    eta: float = 1e-8

    def desc(self):
        return _L.make_desc(self.N, self.L, self.parity, self.t, self.eta)


def _prec(p):
    if isinstance(p, str):
        return PRECISIONS[p]
    return int(p)


def _vp(x):
    return None if x is None else ctypes.c_void_p(x.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(x, name, shape=None):
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if x.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU")
    if x.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(x.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(x.shape)}, expected {tuple(shape)}")


class Workspace:
    """Device scratch for librgf calls, grown on demand (torch allocator)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes, device):
        nbytes = max(int(nbytes), 256)
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        return self.buf


_default_ws = {}


def _workspace(ws, nbytes, device):
    """The caller's Workspace, or a default one per (device, stream). A call
    under graph capture must bring its own Workspace: the graph keeps the
    buffer's address, and a later eager call that grew the default buffer
    would free it."""
    if ws is None:
        stream = torch.cuda.current_stream(device)
        if torch.cuda.is_current_stream_capturing():
            raise RuntimeError("calls under graph capture need a dedicated Workspace "
                               "(pass workspace=Workspace())")
        ws = _default_ws.setdefault((device.index, stream.cuda_stream), Workspace())
    return ws.get(nbytes, device)


def workspace_bytes(ribbon, n_energies, n_real=1, precision="fp64", want_grad=False,
                    ckpt_stride=0):
    d = ribbon.desc()
    n = _L.lib().rgf_workspace_bytes(ctypes.byref(d), int(n_energies), int(n_real),
                                     _prec(precision), int(bool(want_grad)), int(ckpt_stride))
    if n == 0:
        msg = _L.lib().rgf_last_error_message().decode(errors="replace")
        raise _L.RGFError(_L.RGF_ERR_INVALID_ARG, msg)
    return n


def conductance(ribbon, energies, eps=None, n_real=1, precision="fp64", workspace=None,
                return_status=False, out=None):
    """T[r, e] in units of 2e^2/h (Eq. (2) of the paper) for each disorder
    realization r (eps[r] of shape [L, N], or pristine if eps is None) and
    energy e. Asynchronous on the current stream."""
    _need(energies, "energies")
    nE = energies.numel()
    dev = energies.device
    if eps is not None:
        if eps.dim() == 2:
            eps = eps.unsqueeze(0)
        _need(eps, "eps", (eps.shape[0], ribbon.L, ribbon.N))
        n_real = eps.shape[0]
    d = ribbon.desc()
    L = _L.lib()
    prec = _prec(precision)
    nbytes = L.rgf_workspace_bytes(ctypes.byref(d), nE, int(n_real), prec, 0, 0)
    if nbytes == 0:
        msg = L.rgf_last_error_message().decode(errors="replace")
        raise _L.RGFError(_L.RGF_ERR_INVALID_ARG, msg)
    ws = _workspace(workspace, nbytes, dev)
    T = out if out is not None else torch.empty((int(n_real), nE), dtype=torch.float64, device=dev)
    st = torch.empty((int(n_real), nE), dtype=torch.int32, device=dev)
    _L.check(L.rgf_conductance(ctypes.byref(d), _vp(energies), nE, _vp(eps), int(n_real), prec,
                               _vp(T), _vp(st), _vp(ws), ws.numel(), _stream()))
    if return_status:
        return T, st
    return T


def conductance_noalloc(ribbon, energies, eps=None, n_real=1, precision="fp64",
                        return_status=False, out=None, status_out=None):
    """The conductance of `conductance`, computed in the library's fixed
    device scratch instead of a torch workspace (no allocation inside the
    library call; pass `out` and `status_out` to allocate nothing at all).
    Calls that overlap on one GPU share that scratch and must not run
    concurrently."""
    _need(energies, "energies")
    nE = energies.numel()
    dev = energies.device
    if eps is not None:
        if eps.dim() == 2:
            eps = eps.unsqueeze(0)
        _need(eps, "eps", (eps.shape[0], ribbon.L, ribbon.N))
        n_real = eps.shape[0]
    d = ribbon.desc()
    T = out if out is not None else torch.empty((int(n_real), nE), dtype=torch.float64, device=dev)
    st = status_out if status_out is not None else torch.empty((int(n_real), nE),
                                                               dtype=torch.int32, device=dev)
    _L.check(_L.lib().rgf_conductance_noalloc(ctypes.byref(d), _vp(energies), nE, _vp(eps),
                                              int(n_real), _prec(precision), _vp(T), _vp(st),
                                              _stream()))
    if return_status:
        return T, st
    return T


def conductance_segments(ribbon, energies, eps=None, n_real=1, n_segments=0, workspace=None,
                         return_status=False, return_segments=False, out=None):
    """The conductance of `conductance` (FP64) with each tuple's recursion
    split into segments along the ribbon length, solved on separate
    workgroups and joined (librgf rgf_conductance_segments): for batches of
    tuples too small to fill the GPU. n_segments = 0 picks the count."""
    _need(energies, "energies")
    nE = energies.numel()
    dev = energies.device
    if eps is not None:
        if eps.dim() == 2:
            eps = eps.unsqueeze(0)
        _need(eps, "eps", (eps.shape[0], ribbon.L, ribbon.N))
        n_real = eps.shape[0]
    d = ribbon.desc()
    L = _L.lib()
    nbytes = L.rgf_segments_workspace_bytes(ctypes.byref(d), nE, int(n_real), int(n_segments))
    if nbytes == 0:
        msg = L.rgf_last_error_message().decode(errors="replace")
        raise _L.RGFError(_L.RGF_ERR_INVALID_ARG, msg)
    ws = _workspace(workspace, nbytes, dev)
    T = out if out is not None else torch.empty((int(n_real), nE), dtype=torch.float64, device=dev)
    st = torch.empty((int(n_real), nE), dtype=torch.int32, device=dev)
    G = ctypes.c_int32()
    _L.check(L.rgf_conductance_segments(ctypes.byref(d), _vp(energies), nE, _vp(eps),
                                        int(n_real), int(n_segments), _vp(T), _vp(st),
                                        ctypes.byref(G), _vp(ws), ws.numel(), _stream()))
    res = (T,)
    if return_status:
        res += (st,)
    if return_segments:
        res += (G.value,)
    return res[0] if len(res) == 1 else res


def conductance_batched(ribbons, energies, eps_list=None, n_real=1, precision="fp64",
                        workspace=None, return_status=False):
    """Several ribbons (e.g. mixed widths) sharing one energy grid and one
    realization count, in one librgf call. eps_list[d] is [R, L_d, N_d] (or
    None for pristine ribbons); returns a list of T [R, nE] tensors."""
    _need(energies, "energies")
    nE = energies.numel()
    dev = energies.device
    nd = len(ribbons)
    descs = (_L.RibbonDesc * nd)(*[r.desc() for r in ribbons])
    if eps_list is not None:
        eps_list = [e.unsqueeze(0) if e.dim() == 2 else e for e in eps_list]
        n_real = eps_list[0].shape[0]
        for d, (r, e) in enumerate(zip(ribbons, eps_list)):
            _need(e, f"eps_list[{d}]", (n_real, r.L, r.N))
        flat = torch.cat([e.reshape(-1) for e in eps_list])
        offs = [0]
        for e in eps_list[:-1]:
            offs.append(offs[-1] + e.numel())
        eps_off = (ctypes.c_int64 * nd)(*offs)
    else:
        flat, eps_off = None, None
    T = torch.empty((nd, int(n_real), nE), dtype=torch.float64, device=dev)
    st = torch.empty((nd, int(n_real), nE), dtype=torch.int32, device=dev)
    T_off = (ctypes.c_int64 * nd)(*[d * int(n_real) * nE for d in range(nd)])
    L = _L.lib()
    prec = _prec(precision)
    nbytes = L.rgf_batched_workspace_bytes(descs, nd, nE, int(n_real), prec)
    if nbytes == 0:
        msg = L.rgf_last_error_message().decode(errors="replace")
        raise _L.RGFError(_L.RGF_ERR_INVALID_ARG, msg)
    ws = _workspace(workspace, nbytes, dev)
    eps_off_p = None if eps_off is None else ctypes.cast(eps_off, ctypes.c_void_p)
    T_off_p = ctypes.cast(T_off, ctypes.c_void_p)
    _L.check(L.rgf_conductance_batched(descs, nd, eps_off_p, T_off_p, _vp(energies), nE, _vp(flat),
                                       int(n_real), prec, _vp(T), _vp(st), _vp(ws), ws.numel(),
                                       _stream()))
    out = [T[d] for d in range(nd)]
    if return_status:
        return out, [st[d] for d in range(nd)]
    return out


def grad(ribbon, energies, eps, dL_dT, precision="fp64", ckpt_stride=0, workspace=None,
         return_status=False):
    """(T [R, nE], dL/deps [R, L, N]) for L = sum dL_dT * T: the vector-Jacobian
    product of the conductance with respect to every on-site energy, by the
    adjoint sweep of librgf (checkpoint stride in half-slices, 0 = automatic)."""
    _need(energies, "energies")
    nE = energies.numel()
    dev = energies.device
    if eps.dim() == 2:
        eps = eps.unsqueeze(0)
    _need(eps, "eps", (eps.shape[0], ribbon.L, ribbon.N))
    R = eps.shape[0]
    _need(dL_dT, "dL_dT", (R, nE))
    d = ribbon.desc()
    L = _L.lib()
    prec = _prec(precision)
    nbytes = L.rgf_workspace_bytes(ctypes.byref(d), nE, R, prec, 1, int(ckpt_stride))
    if nbytes == 0:
        msg = L.rgf_last_error_message().decode(errors="replace")
        raise _L.RGFError(_L.RGF_ERR_INVALID_ARG, msg)
    ws = _workspace(workspace, nbytes, dev)
    T = torch.empty((R, nE), dtype=torch.float64, device=dev)
    g = torch.empty((R, ribbon.L, ribbon.N), dtype=torch.float64, device=dev)
    st = torch.empty((R, nE), dtype=torch.int32, device=dev)
    _L.check(L.rgf_grad(ctypes.byref(d), _vp(energies), nE, _vp(eps), R, prec, _vp(dL_dT),
                        _vp(T), _vp(g), int(ckpt_stride), _vp(st), _vp(ws), ws.numel(),
                        _stream()))
    if return_status:
        return T, g, st
    return T, g


def ldos(ribbon, energies, eps=None, n_real=1, precision="fp64", ckpt_stride=0,
         workspace=None, return_T=False, return_status=False):
    """Local density of states -Im G_ss(E)/pi of every site: [R, nE, L, N]
    (states per eV per site), by the forward sweep and the backward sweep of
    the diagonal blocks in librgf."""
    _need(energies, "energies")
    nE = energies.numel()
    dev = energies.device
    if eps is not None:
        if eps.dim() == 2:
            eps = eps.unsqueeze(0)
        _need(eps, "eps", (eps.shape[0], ribbon.L, ribbon.N))
        n_real = eps.shape[0]
    d = ribbon.desc()
    L = _L.lib()
    prec = _prec(precision)
    nbytes = L.rgf_workspace_bytes(ctypes.byref(d), nE, int(n_real), prec, 1, int(ckpt_stride))
    if nbytes == 0:
        msg = L.rgf_last_error_message().decode(errors="replace")
        raise _L.RGFError(_L.RGF_ERR_INVALID_ARG, msg)
    ws = _workspace(workspace, nbytes, dev)
    out = torch.empty((int(n_real), nE, ribbon.L, ribbon.N), dtype=torch.float64, device=dev)
    T = torch.empty((int(n_real), nE), dtype=torch.float64, device=dev)
    st = torch.empty((int(n_real), nE), dtype=torch.int32, device=dev)
    _L.check(L.rgf_ldos(ctypes.byref(d), _vp(energies), nE, _vp(eps), int(n_real), prec,
                        _vp(out), _vp(T), int(ckpt_stride), _vp(st), _vp(ws), ws.numel(),
                        _stream()))
    res = (out,)
    if return_T:
        res += (T,)
    if return_status:
        res += (st,)
    return res[0] if len(res) == 1 else res


class RGFConductance(torch.autograd.Function):
    """T = RGFConductance.apply(eps, energies, ribbon, precision): conductance
    [R, nE] with a backward pass through the adjoint sweep (no gradient with
    respect to the energies)."""

    @staticmethod
    def forward(ctx, eps, energies, ribbon, precision="fp64"):
        ctx.save_for_backward(eps, energies)
        ctx.ribbon = ribbon
        ctx.precision = precision
        return conductance(ribbon, energies, eps, precision=precision)

    @staticmethod
    def backward(ctx, grad_T):
        eps, energies = ctx.saved_tensors
        _, g = grad(ctx.ribbon, energies, eps.contiguous(), grad_T.contiguous(),
                    precision=ctx.precision)
        if eps.dim() == 2:
            g = g[0]
        return g, None, None, None


def lead_self_energy(ribbon, energies, workspace=None):
    """(Sigma_L [nE, nl, nl], Sigma_R [nE, nr, nr], status [nE]) as complex128,
    restricted to the slice-1 / slice-L rows that bond to the leads."""
    _need(energies, "energies")
    nE = energies.numel()
    dev = energies.device
    d = ribbon.desc()
    L = _L.lib()
    nl = ctypes.c_int32()
    nr = ctypes.c_int32()
    _L.check(L.rgf_lead_self_energy(ctypes.byref(d), None, 0, None, None, None,
                                    ctypes.byref(nl), ctypes.byref(nr), None, 0, None))
    nbytes = L.rgf_workspace_bytes(ctypes.byref(d), nE, 1, 0, 0, 0)
    ws = _workspace(workspace, nbytes, dev)
    sl = torch.empty((nE, nl.value, nl.value, 2), dtype=torch.float64, device=dev)
    sr = torch.empty((nE, nr.value, nr.value, 2), dtype=torch.float64, device=dev)
    st = torch.empty((nE,), dtype=torch.int32, device=dev)
    _L.check(L.rgf_lead_self_energy(ctypes.byref(d), _vp(energies), nE, _vp(sl), _vp(sr),
                                    _vp(st), None, None, _vp(ws), ws.numel(), _stream()))
    return torch.view_as_complex(sl), torch.view_as_complex(sr), st


def channel_transmission(ribbon, energies, eps=None, n_real=1, precision="fp64",
                         workspace=None, return_status=False):
    """(T_channel [R, nE, P], T [R, nE]): the conductance split over the
    incoming channels (transverse mode chains) of the left lead; the sum over
    the last axis is T."""
    _need(energies, "energies")
    nE = energies.numel()
    dev = energies.device
    if eps is not None:
        if eps.dim() == 2:
            eps = eps.unsqueeze(0)
        _need(eps, "eps", (eps.shape[0], ribbon.L, ribbon.N))
        n_real = eps.shape[0]
    d = ribbon.desc()
    L = _L.lib()
    prec = _prec(precision)
    P = ctypes.c_int32()
    _L.check(L.rgf_lead_modes(ctypes.byref(d), None, 0, 0, None, None, ctypes.byref(P), None, 0,
                              None))
    nbytes = L.rgf_workspace_bytes(ctypes.byref(d), nE, int(n_real), prec, 0, 0)
    if nbytes == 0:
        msg = L.rgf_last_error_message().decode(errors="replace")
        raise _L.RGFError(_L.RGF_ERR_INVALID_ARG, msg)
    ws = _workspace(workspace, nbytes, dev)
    tc = torch.empty((int(n_real), nE, P.value), dtype=torch.float64, device=dev)
    T = torch.empty((int(n_real), nE), dtype=torch.float64, device=dev)
    st = torch.empty((int(n_real), nE), dtype=torch.int32, device=dev)
    _L.check(L.rgf_channel_transmission(ctypes.byref(d), _vp(energies), nE, _vp(eps),
                                        int(n_real), prec, _vp(tc), _vp(T), _vp(st), _vp(ws),
                                        ws.numel(), _stream()))
    if return_status:
        return tc, T, st
    return tc, T


LEAD_METHODS = {"decimation": 0, "mode_matching": 1}


def lead_modes(ribbon, energies, method="decimation", workspace=None):
    """(sigma [nE, P] complex128, status [nE]): the per-mode lead
    self-energies, by Sancho-Rubio decimation or by closed-form mode
    matching."""
    _need(energies, "energies")
    if method not in LEAD_METHODS:
        raise ValueError(f"method must be one of {sorted(LEAD_METHODS)}")
    nE = energies.numel()
    dev = energies.device
    d = ribbon.desc()
    L = _L.lib()
    P = ctypes.c_int32()
    _L.check(L.rgf_lead_modes(ctypes.byref(d), None, 0, 0, None, None, ctypes.byref(P), None, 0,
                              None))
    nbytes = L.rgf_workspace_bytes(ctypes.byref(d), nE, 1, 0, 0, 0)
    ws = _workspace(workspace, nbytes, dev)
    sig = torch.empty((nE, P.value, 2), dtype=torch.float64, device=dev)
    st = torch.empty((nE,), dtype=torch.int32, device=dev)
    _L.check(L.rgf_lead_modes(ctypes.byref(d), _vp(energies), nE, LEAD_METHODS[method], _vp(sig),
                              _vp(st), None, _vp(ws), ws.numel(), _stream()))
    return torch.view_as_complex(sig), st


def autotune(ribbon, precision="fp64", device=None):
    """Time the register tilings for this width on the device and keep the
    fastest for later calls (process-wide). Returns (NW, S, C, slots_per_cu)."""
    dev = device or torch.device("cuda", torch.cuda.current_device())
    d = ribbon.desc()
    L = _L.lib()
    prec = _prec(precision)
    nbytes = L.rgf_autotune_workspace_bytes(ctypes.byref(d), prec)
    if nbytes == 0:
        msg = L.rgf_last_error_message().decode(errors="replace")
        raise _L.RGFError(_L.RGF_ERR_INVALID_ARG, msg)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    chosen = ctypes.c_int32()
    _L.check(L.rgf_autotune(ctypes.byref(d), prec, _vp(ws), ws.numel(), _stream(),
                            ctypes.byref(chosen)))
    c = chosen.value
    return TileChoice(c % 100000 // 10000, (c // 1000) % 10, (c // 10) % 100, c % 10,
                      mgj=c >= 100000)


class TileChoice(tuple):
    """(NW, S, C, slots_per_cu) of the autotuner's choice; .mgj is True for
    the forward sweep with the matrix-core Gauss-Jordan."""

    def __new__(cls, NW, S, C, per_cu, mgj=False):
        t = super().__new__(cls, (NW, S, C, per_cu))
        t.mgj = bool(mgj)
        return t


def refine_stats(reset=False):
    """Counters of the mixed mode's refinement on the current device (librgf
    rgf_refine_stats): {"refined", "newton_updates", "fp64_reinversions"}
    summed over the forward sweeps since the last reset; waits for the
    current stream."""
    c = (ctypes.c_uint64 * 3)()
    _L.check(_L.lib().rgf_refine_stats(c, 1 if reset else 0, _stream()))
    return {"refined": int(c[0]), "newton_updates": int(c[1]), "fp64_reinversions": int(c[2])}


def version():
    a, b = ctypes.c_int(), ctypes.c_int()
    _L.lib().rgf_version(ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value
