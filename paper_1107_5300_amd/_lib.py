"""ctypes loader for librgf.so (argument marshalling only).

The shared library is the HIP build in this directory. torch is imported
first so that librgf binds to the HIP runtime torch already loaded (both
carry the soname libamdhip64.so.7). There is no fallback: a missing or
unloadable library raises.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librgf.so")

RGF_OK = 0
RGF_ERR_INVALID_ARG = -1
RGF_ERR_HIP = -2
RGF_ERR_WORKSPACE = -3
RGF_ERR_UNSUPPORTED = -4

RGF_PREC_FP64 = 0
RGF_PREC_MIXED = 1
RGF_PREC_FP32 = 2

TUPLE_OK = 0
TUPLE_NO_CONVERGENCE = 1
TUPLE_SINGULAR = 2
TUPLE_NONFINITE = 3
TUPLE_OUT_OF_RANGE = 4
TUPLE_ILL_CONDITIONED = 5

# every symbol declared in include/rgf.h
EXPORTED = (
    "rgf_workspace_bytes",
    "rgf_conductance",
    "rgf_grad",
    "rgf_ldos",
    "rgf_channel_transmission",
    "rgf_lead_modes",
    "rgf_batched_workspace_bytes",
    "rgf_conductance_batched",
    "rgf_conductance_noalloc",
    "rgf_segments_workspace_bytes",
    "rgf_conductance_segments",
    "rgf_lead_self_energy",
    "rgf_autotune_workspace_bytes",
    "rgf_autotune",
    "rgf_refine_stats",
    "rgf_status_string",
    "rgf_last_error_message",
    "rgf_version",
)


class RibbonDesc(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("width_n", ctypes.c_int32),
        ("length_l", ctypes.c_int32),
        ("parity", ctypes.c_int32),
        ("hopping_ev", ctypes.c_double),
        ("eta_ev", ctypes.c_double),
    ]


class RGFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_int = ctypes.c_int
_sz = ctypes.c_size_t
_pdesc = ctypes.POINTER(RibbonDesc)


def _declare(lib):
    lib.rgf_workspace_bytes.restype = _sz
    lib.rgf_workspace_bytes.argtypes = [_pdesc, _i64, _i64, _int, _int, _i64]
    lib.rgf_conductance.restype = _int
    lib.rgf_conductance.argtypes = [_pdesc, _vp, _i64, _vp, _i64, _int, _vp, _vp, _vp, _sz, _vp]
    lib.rgf_grad.restype = _int
    lib.rgf_grad.argtypes = [_pdesc, _vp, _i64, _vp, _i64, _int, _vp, _vp, _vp, _i64, _vp,
                             _vp, _sz, _vp]
    lib.rgf_ldos.restype = _int
    lib.rgf_ldos.argtypes = [_pdesc, _vp, _i64, _vp, _i64, _int, _vp, _vp, _i64, _vp, _vp, _sz,
                             _vp]
    lib.rgf_channel_transmission.restype = _int
    lib.rgf_channel_transmission.argtypes = [_pdesc, _vp, _i64, _vp, _i64, _int, _vp, _vp, _vp,
                                             _vp, _sz, _vp]
    lib.rgf_lead_modes.restype = _int
    lib.rgf_lead_modes.argtypes = [_pdesc, _vp, _i64, _int, _vp, _vp, ctypes.POINTER(_i32), _vp,
                                   _sz, _vp]
    lib.rgf_batched_workspace_bytes.restype = _sz
    lib.rgf_batched_workspace_bytes.argtypes = [_pdesc, _i32, _i64, _i64, _int]
    lib.rgf_conductance_batched.restype = _int
    lib.rgf_conductance_batched.argtypes = [_pdesc, _i32, _vp, _vp, _vp, _i64, _vp, _i64, _int,
                                            _vp, _vp, _vp, _sz, _vp]
    lib.rgf_conductance_noalloc.restype = _int
    lib.rgf_conductance_noalloc.argtypes = [_pdesc, _vp, _i64, _vp, _i64, _int, _vp, _vp, _vp]
    lib.rgf_segments_workspace_bytes.restype = _sz
    lib.rgf_segments_workspace_bytes.argtypes = [_pdesc, _i64, _i64, _i32]
    lib.rgf_conductance_segments.restype = _int
    lib.rgf_conductance_segments.argtypes = [_pdesc, _vp, _i64, _vp, _i64, _i32, _vp, _vp,
                                             ctypes.POINTER(_i32), _vp, _sz, _vp]
    lib.rgf_lead_self_energy.restype = _int
    lib.rgf_lead_self_energy.argtypes = [_pdesc, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _sz,
                                         _vp]
    lib.rgf_autotune_workspace_bytes.restype = _sz
    lib.rgf_autotune_workspace_bytes.argtypes = [_pdesc, _int]
    lib.rgf_autotune.restype = _int
    lib.rgf_autotune.argtypes = [_pdesc, _int, _vp, _sz, _vp, ctypes.POINTER(_i32)]
    lib.rgf_refine_stats.restype = _int
    lib.rgf_refine_stats.argtypes = [ctypes.POINTER(ctypes.c_uint64), _int, _vp]
    lib.rgf_status_string.restype = ctypes.c_char_p
    lib.rgf_status_string.argtypes = [_int]
    lib.rgf_last_error_message.restype = ctypes.c_char_p
    lib.rgf_last_error_message.argtypes = []
    lib.rgf_version.restype = _int
    lib.rgf_version.argtypes = [ctypes.POINTER(_int), ctypes.POINTER(_int)]


def lib():
    """The loaded librgf (raises if it is not built)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (binds the HIP runtime torch ships)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_1107_5300_amd.build` (hipcc, gfx950)")
        handle = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)
        _declare(handle)
        _lib = handle
    return _lib


def check(code):
    if code != RGF_OK:
        L = lib()
        msg = L.rgf_last_error_message().decode(errors="replace")
        raise RGFError(code, f"{L.rgf_status_string(code).decode()}: {msg}")


def make_desc(N, L, parity=0, t=-2.7, eta=1e-8):
    d = RibbonDesc()
    d.struct_size = ctypes.sizeof(RibbonDesc)
    d.width_n = int(N)
    d.length_l = int(L)
    d.parity = int(parity)
    d.hopping_ev = float(t)
    d.eta_ev = float(eta)
    return d
