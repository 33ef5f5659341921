"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/rgf.h, and rejects bad arguments
before anything is enqueued."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rgf.h")
LIBP = os.path.join(ROOT, "paper_1107_5300_amd", "librgf.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIBP), reason="librgf.so not built")


def _header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rgf_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    from paper_1107_5300_amd import _lib as L
    lib = L.lib()
    names = _header_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(L.EXPORTED) == names


def test_version_and_strings():
    from paper_1107_5300_amd import _lib as L
    lib = L.lib()
    a, b = ctypes.c_int(), ctypes.c_int()
    assert lib.rgf_version(ctypes.byref(a), ctypes.byref(b)) == 0
    assert (a.value, b.value) == (1, 3)
    assert lib.rgf_status_string(-1) == b"RGF_ERR_INVALID_ARG"
    assert lib.rgf_status_string(-3) == b"RGF_ERR_WORKSPACE"


@pytest.mark.parametrize("field,value,code", [
    ("width_n", 1, -1), ("width_n", 100000, -4), ("width_n", 513, -4),
    ("length_l", 0, -1), ("parity", 2, -1),
    ("hopping_ev", 0.0, -1), ("hopping_ev", float("nan"), -1), ("eta_ev", 0.0, -1),
    ("eta_ev", -1e-8, -1), ("eta_ev", float("inf"), -1), ("struct_size", 8, -1),
])
def test_invalid_descriptor(field, value, code):
    from paper_1107_5300_amd import _lib as L
    lib = L.lib()
    d = L.make_desc(20, 10)
    setattr(d, field, value)
    rc = lib.rgf_conductance(ctypes.byref(d), ctypes.c_void_p(16), 4, None, 1, 0,
                             ctypes.c_void_p(16), None, None, 0, None)
    assert rc == code
    assert len(lib.rgf_last_error_message()) > 0
    assert lib.rgf_workspace_bytes(ctypes.byref(d), 4, 1, 0, 0, 0) == 0


def test_null_pointers_and_small_workspace():
    from paper_1107_5300_amd import _lib as L
    lib = L.lib()
    d = L.make_desc(20, 10)
    need = lib.rgf_workspace_bytes(ctypes.byref(d), 4, 1, 0, 0, 0)
    assert need > 0
    # NULL energies
    assert lib.rgf_conductance(ctypes.byref(d), None, 4, None, 1, 0, ctypes.c_void_p(256),
                               None, ctypes.c_void_p(256), need, None) == -1
    # NULL T_out
    assert lib.rgf_conductance(ctypes.byref(d), ctypes.c_void_p(256), 4, None, 1, 0, None,
                               None, ctypes.c_void_p(256), need, None) == -1
    # workspace too small
    assert lib.rgf_conductance(ctypes.byref(d), ctypes.c_void_p(256), 4, None, 1, 0,
                               ctypes.c_void_p(256), None, ctypes.c_void_p(256), need - 1,
                               None) == -3
    assert b"workspace" in lib.rgf_last_error_message()
    # misaligned workspace
    assert lib.rgf_conductance(ctypes.byref(d), ctypes.c_void_p(256), 4, None, 1, 0,
                               ctypes.c_void_p(256), None, ctypes.c_void_p(264), need,
                               None) == -1
    # bad counts / precision
    assert lib.rgf_conductance(ctypes.byref(d), ctypes.c_void_p(256), -1, None, 1, 0,
                               ctypes.c_void_p(256), None, ctypes.c_void_p(256), need,
                               None) == -1
    assert lib.rgf_conductance(ctypes.byref(d), ctypes.c_void_p(256), 4, None, 0, 0,
                               ctypes.c_void_p(256), None, ctypes.c_void_p(256), need,
                               None) == -1
    assert lib.rgf_conductance(ctypes.byref(d), ctypes.c_void_p(256), 4, None, 1, 7,
                               ctypes.c_void_p(256), None, ctypes.c_void_p(256), need,
                               None) == -1
    # zero energies is a no-op
    assert lib.rgf_conductance(ctypes.byref(d), None, 0, None, 1, 0, None, None, None, 0,
                               None) == 0


def test_lead_sizes_query():
    from paper_1107_5300_amd import _lib as L
    lib = L.lib()
    for N, Lc, par, nl, nr in [(20, 10, 0, 10, 10), (7, 3, 0, 4, 3), (7, 4, 0, 4, 4),
                               (7, 4, 1, 3, 3), (7, 3, 1, 3, 4)]:
        d = L.make_desc(N, Lc, par)
        a, b = ctypes.c_int32(), ctypes.c_int32()
        assert lib.rgf_lead_self_energy(ctypes.byref(d), None, 0, None, None, None,
                                        ctypes.byref(a), ctypes.byref(b), None, 0, None) == 0
        assert (a.value, b.value) == (nl, nr), (N, Lc, par)


def test_forward_kernels_use_no_scratch():
    """The forward sweep kernels keep their register tiles in registers: a
    kernel that needs scratch memory (a spilled or dynamically indexed tile)
    is several times slower. Reads the resource report the build writes."""
    from paper_1107_5300_amd import _lib as L
    path = os.path.join(os.path.dirname(L.LIB_PATH), "_build", "kernel_resources.txt")
    if not os.path.exists(path):
        pytest.skip("no resource report (library not built in this tree)")
    with open(path) as fh:
        rows = [ln.rstrip("\n").split("\t") for ln in fh][1:]
    fwd = [r for r in rows if "rgf_fwd_kernel<" in r[0] and "true" not in r[0]]
    assert len(fwd) >= 20, "report lists too few forward kernels"
    bad = [(r[0], r[3], r[4]) for r in fwd if r[3] != "0" or r[4] != "0"]
    assert not bad, f"forward kernels with scratch / VGPR spills: {bad}"


def test_gradient_and_ldos_kernel_spills_bounded():
    """The FP64 gradient and LDOS kernels: no scratch in any tiling but the
    8-wave two-slot ones, where the spill stays under 64 registers (in the
    compiled code most reloads sit outside the sweep loops; the rest are at
    most 8 per half-slice beside 128 to 192 matrix instructions)."""
    from paper_1107_5300_amd import _lib as L
    path = os.path.join(os.path.dirname(L.LIB_PATH), "_build", "kernel_resources.txt")
    if not os.path.exists(path):
        pytest.skip("no resource report (library not built in this tree)")
    with open(path) as fh:
        rows = [ln.rstrip("\n").split("\t") for ln in fh][1:]
    ks = [r for r in rows if ("rgf_grad_kernel<double" in r[0] or "rgf_ldos_kernel<double" in r[0])]
    assert len(ks) >= 20, "report lists too few gradient / LDOS kernels"
    for r in ks:
        two_slot = ", 8, 2," in r[0]
        if not two_slot:
            assert r[3] == "0" and r[4] == "0", r
        else:
            assert int(r[4]) <= 64 and int(r[3]) <= 256, r


def test_widest_supported_and_first_unsupported_width():
    """N = 512 is the widest ribbon (two blocks of at most 128 rows per
    half-slice); N = 513 reports RGF_ERR_UNSUPPORTED before anything is
    enqueued."""
    from paper_1107_5300_amd import _lib as L
    lib = L.lib()
    for N in (256, 257, 480, 512):
        ok = L.make_desc(N, 4)
        assert lib.rgf_workspace_bytes(ctypes.byref(ok), 4, 1, 0, 0, 0) > 0, N
    d = L.make_desc(513, 4)
    assert lib.rgf_workspace_bytes(ctypes.byref(d), 4, 1, 0, 0, 0) == 0
    rc = lib.rgf_conductance(ctypes.byref(d), ctypes.c_void_p(16), 4, None, 1, 0,
                             ctypes.c_void_p(16), None, ctypes.c_void_p(256), 1 << 30, None)
    assert rc == L.RGF_ERR_UNSUPPORTED
    assert b"outside [2, 512]" in lib.rgf_last_error_message()


@pytest.mark.parametrize("N", [257, 480, 512])
def test_wide_ribbons_fp64_only(N):
    """Half-slices above 128 rows are inverted by panels in FP64: every entry
    point plans with RGF_PREC_FP64, while the FP32 modes report
    RGF_ERR_UNSUPPORTED before anything is enqueued. N = 256 supports every
    entry point and precision."""
    from paper_1107_5300_amd import _lib as L
    lib = L.lib()
    d = L.make_desc(N, 4)
    for prec in (1, 2):
        for grad in (0, 1):
            assert lib.rgf_workspace_bytes(ctypes.byref(d), 4, 1, prec, grad, 0) == 0
            assert b"FP64 only" in lib.rgf_last_error_message()
    assert lib.rgf_workspace_bytes(ctypes.byref(d), 4, 1, 0, 1, 0) > 0
    rc = lib.rgf_ldos(ctypes.byref(d), ctypes.c_void_p(16), 4, None, 1, 1,
                      ctypes.c_void_p(16), None, 0, None, None, 0, None)
    assert rc == L.RGF_ERR_UNSUPPORTED
    assert b"FP64 only" in lib.rgf_last_error_message()
    rc = lib.rgf_ldos(ctypes.byref(d), ctypes.c_void_p(16), 4, None, 1, 0,
                      ctypes.c_void_p(16), None, 0, None, None, 0, None)
    assert rc == L.RGF_ERR_WORKSPACE   # FP64 plans; the NULL workspace is too small
    rc = lib.rgf_grad(ctypes.byref(d), ctypes.c_void_p(16), 4, None, 1, 1,
                      ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16), 0, None,
                      None, 0, None)
    assert rc == L.RGF_ERR_UNSUPPORTED
    rc = lib.rgf_conductance(ctypes.byref(d), ctypes.c_void_p(16), 4, None, 1, 1,
                             ctypes.c_void_p(16), None, ctypes.c_void_p(256), 1 << 30, None)
    assert rc == L.RGF_ERR_UNSUPPORTED
    narrow = L.make_desc(256, 4)
    for prec in (0, 1, 2):
        for grad in (0, 1):
            assert lib.rgf_workspace_bytes(ctypes.byref(narrow), 4, 1, prec, grad, 0) > 0


def test_wide_gradient_workspace_layout():
    """The wide gradient's workspace: 45 blocks of 128 x 128 complex128 per
    slot plus, per slot, two 256 x 256 restart matrices per checkpoint and
    per segment entry (stride s, ceil(2L/s) checkpoints)."""
    from paper_1107_5300_amd import _lib as L
    lib = L.lib()
    d = L.make_desc(480, 8)
    full = 256 * 256 * 16
    for stride, nck in ((4, 4), (16, 1)):
        one = lib.rgf_workspace_bytes(ctypes.byref(d), 1, 1, 0, 1, stride)
        two = lib.rgf_workspace_bytes(ctypes.byref(d), 1, 2, 0, 1, stride)  # two tuples
        per_slot = 45 * 128 * 128 * 16 + (nck + stride) * 2 * full
        assert per_slot <= two - one <= per_slot + 3 * 256, (stride, two - one, per_slot)


def test_wide_ribbon_workspace_scales_with_grid():
    """The blocked path's workspace: lead tables with leading dimension 256
    plus 21 blocks of 128 x 128 complex128 per persistent slot (five 256 x 256
    matrices and the staged pivot rows; the grid is at most the tuple
    count), and at least one slot of the whole-slice accuracy fallback
    (three 256 x 256 and two 512 x 512 matrices, the refined 512 x 256
    columns and staged rows), which
    reuses the slot region."""
    from paper_1107_5300_amd import _lib as L
    lib = L.lib()
    d = L.make_desc(480, 4)
    slot = 21 * 128 * 128 * 16
    whole = (3 * 256 * 256 + 2 * 512 * 512 + 512 * 256 + 128 * 128) * 16
    one = lib.rgf_workspace_bytes(ctypes.byref(d), 1, 1, 0, 0, 0)
    assert one >= whole + 2 * 240 * 256 * 8
    three = lib.rgf_workspace_bytes(ctypes.byref(d), 3, 1, 0, 0, 0)
    four = lib.rgf_workspace_bytes(ctypes.byref(d), 4, 1, 0, 0, 0)
    assert three >= 3 * slot and four - three >= slot
    # the FP64 gradient has no fallback: no whole-slice slot
    g1 = lib.rgf_workspace_bytes(ctypes.byref(d), 1, 1, 0, 1, 0)
    assert g1 > 0


def test_channel_transmission_and_lead_modes_arguments():
    """rgf_channel_transmission runs in FP64 only; rgf_lead_modes reports the
    number of modes P = ceil(N/2) with NULL outputs and rejects an unknown
    method, all before anything is enqueued."""
    from paper_1107_5300_amd import _lib as L
    lib = L.lib()
    d = L.make_desc(21, 5)
    P = ctypes.c_int32()
    assert lib.rgf_lead_modes(ctypes.byref(d), None, 0, 1, None, None, ctypes.byref(P), None,
                              0, None) == 0
    assert P.value == 11
    assert lib.rgf_lead_modes(ctypes.byref(d), ctypes.c_void_p(16), 2, 2, ctypes.c_void_p(16),
                              None, None, ctypes.c_void_p(256), 1 << 20, None) == -1
    for prec in (1, 2):
        rc = lib.rgf_channel_transmission(ctypes.byref(d), ctypes.c_void_p(16), 4, None, 1, prec,
                                          ctypes.c_void_p(16), ctypes.c_void_p(16), None,
                                          ctypes.c_void_p(256), 1 << 30, None)
        assert rc == L.RGF_ERR_UNSUPPORTED
    rc = lib.rgf_channel_transmission(ctypes.byref(d), ctypes.c_void_p(16), 4, None, 1, 0,
                                      None, ctypes.c_void_p(16), None, ctypes.c_void_p(256),
                                      1 << 30, None)
    assert rc == -1 and b"T_channel_out" in lib.rgf_last_error_message()


def test_autotune_wide_widths():
    """Above N = 256 the autotuner has one configuration: FP64 needs no tuning
    workspace beyond the trial buffers, and FP32 modes are rejected."""
    from paper_1107_5300_amd import _lib as L
    lib = L.lib()
    d = L.make_desc(480, 8)
    assert lib.rgf_autotune_workspace_bytes(ctypes.byref(d), 0) > 0
    for prec in (1, 2):
        assert lib.rgf_autotune_workspace_bytes(ctypes.byref(d), prec) == 0
        assert b"FP64 only" in lib.rgf_last_error_message()


def test_validation_layer_under_sanitizers():
    """The host validation and planning code (rgf_api.cpp, rgf_noalloc.hip)
    rebuilt with AddressSanitizer and UndefinedBehaviorSanitizer on the host
    side and driven through every entry point's error and planning paths by
    csrc/abi_check.cpp (no GPU needed). Leak checking is off: the HIP
    runtime keeps allocations until exit."""
    import shutil
    import subprocess
    if shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc not available")
    from paper_1107_5300_amd import build as B
    exe = B.build_abi_check()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, env=env,
                       timeout=300)
    out = r.stdout.decode(errors="replace")
    assert r.returncode == 0, out[-3000:]
    assert "abi_check: ok" in out
    assert "runtime error" not in out and "AddressSanitizer" not in out
