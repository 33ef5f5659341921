"""GPU parity of ribbons wider than N = 256 (half-slices above 128 rows,
inverted by the panel Gauss-Jordan in the workspace) through the C ABI.

Stored oracle values (tests/golden/make_wide_golden.py, oracle/ only) for
widths 257..512, the full-size N = 480, L = 8000 ribbon on sampled energies,
and the gradient dT/deps and the local density of states of every site at
N = 257 and 480; closed-form and
invariant checks (quantised pristine conductance, T(t) = T(-t),
0 <= T <= M(E)) at any size. Bars as for the narrow path: 1e-9 relative on
short ribbons (gradients 1e-8 relative to max(1, max|dT/deps|)), 1e-6
absolute at full size.
"""

import os
import sys

import numpy as np
import pytest

import oracle as O
import rgf_workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL_SMALL = 1e-9


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1107_5300_amd as P
    P.version()
    return P


def _gpu_T(P, N, L, parity, t, Es, eps=None):
    import torch
    rib = P.Ribbon(N, L, parity, t, W.ETA)
    E = torch.tensor(np.asarray(Es, dtype=np.float64), device="cuda")
    ep = None if eps is None else torch.tensor(np.asarray(eps), device="cuda")
    T, st = P.conductance(rib, E, ep, return_status=True)
    torch.cuda.synchronize()
    return T.cpu().numpy(), st.cpu().numpy()


def _wide_rows():
    rows = np.loadtxt(os.path.join(HERE, "golden", "wide_ribbons.txt"))
    return [tuple(r) for r in np.atleast_2d(rows)]


@pytest.mark.parametrize("row", _wide_rows(), ids=lambda r: f"N{int(r[0])}_r{int(r[4])}_E{r[5]:.3f}")
def test_wide_ribbons_match_oracle(P, row):
    N, L, parity, w, r, E, want = row
    N, L, parity, r = int(N), int(L), int(parity), int(r)
    _say("wide", N, L, parity, r, E)
    eps = W.disorder(L, N, w, r=r)
    got, st = _gpu_T(P, N, L, parity, W.T_HOP, [E], eps[None])
    assert st[0, 0] == 0
    assert abs(got[0, 0] - want) <= TOL_SMALL * max(1.0, abs(want)), (got[0, 0], want)


@pytest.mark.parametrize("L,parity", [(1, 0), (2, 1)])
def test_shortest_wide_ribbons(P, L, parity):
    """L = 1 (both lead self-energies on the one slice) and L = 2 at
    N = 258, against the oracle run here (its lead decimation at this width
    takes seconds)."""
    N = 258
    E = -0.27 * abs(W.T_HOP)
    eps = W.disorder(L, N, 0.5, r=30 + L)
    _say("shortest wide", N, L, parity)
    got, st = _gpu_T(P, N, L, parity, W.T_HOP, [E], eps[None])
    assert st[0, 0] == 0
    want = O.transmission(N, L, W.T_HOP, W.ETA, E, eps, parity)
    assert abs(got[0, 0] - want) <= TOL_SMALL * max(1.0, abs(want)), (got[0, 0], want)


def test_realizations_and_energies_in_one_launch(P):
    """Both N = 480 realizations and both stored energies in one call (one
    tuple per workgroup), against the same stored values."""
    rows = [r for r in _wide_rows() if int(r[0]) == 480]
    Es = sorted({r[5] for r in rows})
    reals = sorted({int(r[4]) for r in rows})
    L = int(rows[0][1])
    eps = np.stack([W.disorder(L, 480, 0.5, r=r) for r in reals])
    _say("wide batch", len(reals), len(Es))
    got, st = _gpu_T(P, 480, L, 0, W.T_HOP, Es, eps)
    assert (st == 0).all()
    for N, L_, par, w, r, E, want in rows:
        i, j = reals.index(int(r)), Es.index(E)
        assert abs(got[i, j] - want) <= TOL_SMALL * max(1.0, abs(want))


def _away_from_edges(N, xs, t):
    """Energies of the grid at least 2e-4 |t| from every subband edge
    |1 -+ 2 cos(p pi/(N+1))| |t| (where M(E) jumps)."""
    p = np.arange(1, N // 2 + 1)
    c = np.cos(p * np.pi / (N + 1))
    edges = np.concatenate([np.abs(1 - 2 * c), 1 + 2 * c])
    return [x * abs(t) for x in xs if np.abs(edges - abs(x)).min() > 2e-4]


@pytest.mark.parametrize("N,parity", [(480, 0), (301, 1), (512, 0)])
def test_pristine_wide_ribbon_is_quantised(P, N, parity):
    """A pristine ribbon transmits every open channel: T = M(E). The grid
    skips E = 0 (see test_pristine_gap_evanescent for the gap)."""
    Es = _away_from_edges(N, np.linspace(-0.3, 0.3, 40), W.T_HOP)
    _say("pristine wide", N, parity, len(Es))
    got, st = _gpu_T(P, N, 5, parity, W.T_HOP, Es)
    assert (st == 0).all()
    M = np.array([O.open_channels(N, E, W.T_HOP) for E in Es])
    assert np.abs(got[0] - M).max() <= 1e-4, np.abs(got[0] - M).max()


def test_pristine_gap_evanescent(P):
    """Inside the subband gap of a pristine semiconducting ribbon no lead
    mode propagates: M(E) = 0, so 0 <= T <= M(E) leaves |T| at rounding
    level. Entries of M_h then span many orders of magnitude and an
    elimination without pivoting across the whole half-slice returns
    garbage; this pins the pivoted panel inversion."""
    N = 480
    gap = 0.003769 * abs(W.T_HOP)  # half-gap of N = 480
    Es = [0.25 * gap, -0.5 * gap, 0.8 * gap]
    assert all(O.open_channels(N, E, W.T_HOP) == 0 for E in Es)
    for L in (4, 9):
        _say("pristine gap", N, L)
        got, st = _gpu_T(P, N, L, L % 2, W.T_HOP, Es)
        assert (st == 0).all()
        assert np.abs(got).max() <= 1e-9, got


def test_zero_energy_pristine_wide_exact(P):
    """E = 0 exactly in a pristine N = 480 ribbon (in its gap, M(0) = 0): the
    accuracy guard hands the tuple to the whole-slice sweep (480 x 480
    inversions); status OK and |T| at rounding level (the stored oracle
    values at E = 0 are in tests/test_gpu_accuracy_guard.py)."""
    got, st = _gpu_T(P, 480, 4, 0, W.T_HOP, [0.0])
    assert st[0, 0] == 0, st
    assert abs(got[0, 0]) <= 1e-9, got


def test_invariants_wide_disordered(P):
    """0 <= T <= M(E) and T(t) = T(-t) on a disordered N = 480 ribbon."""
    N, L = 480, 40
    eps = W.disorder(L, N, 0.5, r=7)
    Es = np.linspace(-0.3, 0.3, 12) * abs(W.T_HOP)
    _say("wide invariants", N, L)
    a, sa = _gpu_T(P, N, L, 0, W.T_HOP, Es, eps[None])
    b, sb = _gpu_T(P, N, L, 0, -W.T_HOP, Es, eps[None])
    assert (sa == 0).all() and (sb == 0).all()
    M = np.array([O.open_channels(N, E, W.T_HOP) for E in Es])
    assert (a[0] >= -1e-12).all() and (a[0] <= M + 1e-9).all()
    assert np.abs(a - b).max() <= 1e-9


def test_graph_capture_replays_wide(P):
    """The N = 300 conductance call captured in a graph and replayed several
    times, with eager work between replays, matches the eager result."""
    import torch
    N, L = 300, 4
    _say("wide graph capture")
    Es = torch.tensor(np.linspace(-0.3, 0.3, 6) * abs(W.T_HOP), device="cuda")
    eps = torch.tensor(W.disorder_batch(L, N, 0.5, 2), device="cuda")
    rib = P.Ribbon(N, L, 0, W.T_HOP, W.ETA)
    ws = P.Workspace()
    out = torch.empty((2, 6), dtype=torch.float64, device="cuda")
    ref = P.conductance(rib, Es, eps, workspace=ws).clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        P.conductance(rib, Es, eps, workspace=ws, out=out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        P.conductance(rib, Es, eps, workspace=ws, out=out)
    for k in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), k
        P.conductance(rib, Es * 0.5, eps, workspace=ws)
        torch.cuda.synchronize()


def test_nan_energy_sets_status_wide(P):
    got, st = _gpu_T(P, 300, 3, 0, W.T_HOP, [0.3, float("nan")])
    assert st[0, 0] == 0 and np.isfinite(got[0, 0])
    assert st[0, 1] != 0 and np.isnan(got[0, 1])


def test_batched_with_wide_and_narrow_ribbons(P):
    """A wide and two narrow ribbons in one batched call equal single calls."""
    import torch
    widths = [(60, 4), (480, 3), (130, 5)]
    Es = np.array([-0.2, 0.15]) * abs(W.T_HOP)
    _say("batched wide", widths)
    ribs = [P.Ribbon(N, L, 0, W.T_HOP, W.ETA) for N, L in widths]
    eps = [W.disorder_batch(L, N, 0.5, 2) for N, L in widths]
    out, st = P.conductance_batched(ribs, torch.tensor(Es, device="cuda"),
                                    [torch.tensor(e, device="cuda") for e in eps],
                                    return_status=True)
    torch.cuda.synchronize()
    for d, (N, L) in enumerate(widths):
        assert (st[d].cpu().numpy() == 0).all()
        one, _ = _gpu_T(P, N, L, 0, W.T_HOP, Es, eps[d])
        assert np.abs(out[d].cpu().numpy() - one).max() <= 1e-12


def test_lead_self_energy_wide_properties(P):
    """Sigma_L, Sigma_R at N = 480: complex symmetric, Gamma = -2 Im Sigma
    positive semidefinite with rank = open channels (one per propagating
    mode pair), through the same lead tables the blocked sweep reads."""
    import torch
    N, L = 480, 6
    E = 0.137 * abs(W.T_HOP)
    rib = P.Ribbon(N, L, 0, W.T_HOP, W.ETA)
    sl, sr, st = P.lead_self_energy(rib, torch.tensor([E], dtype=torch.float64,
                                                      device="cuda"))
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    for s in (sl[0].cpu().numpy(), sr[0].cpu().numpy()):
        assert s.shape == (240, 240)
        assert np.abs(s - s.T).max() <= 1e-12 * np.abs(s).max()
        gam = -2.0 * s.imag
        ev = np.linalg.eigvalsh(0.5 * (gam + gam.T))
        assert ev.min() >= -1e-9 * ev.max()
        assert int((ev > 1e-6 * ev.max()).sum()) == O.open_channels(N, E, W.T_HOP)


def test_autotune_wide_is_fixed(P):
    rib = P.Ribbon(480, 4, 0, W.T_HOP, W.ETA)
    NW, S, C, per_cu = P.autotune(rib)
    assert (NW, S, C, per_cu) == (8, 4, 8, 0)


def test_large_n480_full_length_sampled(P):
    """N = 480, L = 8000 disordered ribbon (the paper's widest workload) on
    the stored sampled energies, 1e-6 against the oracle."""
    rows = np.atleast_2d(np.loadtxt(os.path.join(HERE, "golden", "large_n480_sampled.txt")))
    cfg = W.WORKLOADS["large_n480"]
    N, L = cfg["N"][0], cfg["L"]
    Es_all = W.energies("large_n480")
    eps = W.disorder(L, N, cfg["w"], r=0)
    js = [int(r[0]) for r in rows]
    _say("large_n480 sampled", N, L, js)
    got, st = _gpu_T(P, N, L, 0, W.T_HOP, Es_all[js], eps[None])
    assert (st == 0).all()
    for k, (j, E, want) in enumerate(rows):
        assert E == Es_all[int(j)]
        _say("  oracle E index", int(j), want, got[0, k])
        assert abs(got[0, k] - want) <= 1e-6


# ------------------------------------------------------------------ gradients

def _grad_rows():
    path = os.path.join(HERE, "golden", "wide_grad.txt")
    out, cur = [], None
    with open(path) as fh:
        for ln in fh:
            if ln.startswith("#"):
                continue
            f = ln.split()
            if f[0] == "ribbon":
                cur = dict(N=int(f[1]), L=int(f[2]), parity=int(f[3]), w=float(f[4]),
                           r=int(f[5]), E=float(f[6]), T=float(f[7]))
                cur["g"] = np.zeros((cur["L"], cur["N"]))
                out.append(cur)
            else:
                cur["g"][int(f[0]), int(f[1])] = float(f[2])
    return out


def _grad(P, N, L, parity, Es, eps, w, stride=0):
    import torch
    t = lambda x: torch.tensor(np.asarray(x, dtype=np.float64), device="cuda")
    T, g, st = P.grad(P.Ribbon(N, L, parity, W.T_HOP, W.ETA), t(Es), t(eps), t(w),
                      ckpt_stride=stride, return_status=True)
    torch.cuda.synchronize()
    return T.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("k", [0, 1])
def test_wide_grad_matches_oracle(P, k):
    """dT/deps of every site against the oracle's forward-backward gradient."""
    c = _grad_rows()[k]
    N, L = c["N"], c["L"]
    _say("wide grad", N, L, c["parity"])
    eps = W.disorder(L, N, c["w"], r=c["r"])
    T, g, st = _grad(P, N, L, c["parity"], [c["E"]], eps[None], [[1.0]])
    assert (st == 0).all()
    assert abs(T[0, 0] - c["T"]) <= 1e-9 * max(1.0, abs(c["T"]))
    scale = max(1.0, np.abs(c["g"]).max())
    assert np.abs(g[0] - c["g"]).max() <= 1e-8 * scale, np.abs(g[0] - c["g"]).max()


def test_wide_grad_strides_and_weights(P):
    """Checkpoint strides give the same gradient; several energies and
    realizations in one call give the weighted sum of single-energy calls."""
    N, L = 300, 5
    eps = W.disorder_batch(L, N, 0.5, 2)
    Es = np.array([-0.31, 0.27]) * abs(W.T_HOP)
    w = np.array([[0.7, -1.3], [2.0, 0.4]])
    _say("wide grad strides", N, L)
    T0, g0, st = _grad(P, N, L, 0, Es, eps, w)
    assert (st == 0).all()
    for stride in (1, 3, 10):
        T1, g1, _ = _grad(P, N, L, 0, Es, eps, w, stride=stride)
        assert np.abs(g1 - g0).max() <= 1e-12 * max(1.0, np.abs(g0).max())
        assert np.abs(T1 - T0).max() <= 1e-13 * max(1.0, np.abs(T0).max())
    want = np.zeros_like(g0)
    for r in range(2):
        for j in range(2):
            _, gj, _ = _grad(P, N, L, 0, [Es[j]], eps[r:r + 1], [[1.0]])
            want[r] += w[r, j] * gj[0]
    assert np.abs(g0 - want).max() <= 1e-12 * max(1.0, np.abs(want).max())


def test_wide_grad_finite_differences(P):
    """N = 480: the gradient against central differences of the GPU
    forward sweep (h = 1e-6 |t|) on seeded sites."""
    N, L = 480, 4
    eps = W.disorder(L, N, 0.5, r=77)
    E = 0.21 * abs(W.T_HOP)
    _, g, st = _grad(P, N, L, 0, [E], eps[None], [[1.0]])
    assert (st == 0).all()
    h = 1e-6 * abs(W.T_HOP)
    sites = W.fd_sites(L, N, count=8, seed=5)
    batch = []
    for i, k in sites:
        for sgn in (1.0, -1.0):
            e2 = eps.copy()
            e2[i, k] += sgn * h
            batch.append(e2)
    _say("wide grad fd", len(sites))
    Tfd, st2 = _gpu_T(P, N, L, 0, W.T_HOP, [E], np.stack(batch))
    assert (st2 == 0).all()
    for n_, (i, k) in enumerate(sites):
        fd = (Tfd[2 * n_, 0] - Tfd[2 * n_ + 1, 0]) / (2 * h)
        assert abs(fd - g[0, i, k]) <= 1e-6 + 1e-4 * abs(g[0, i, k]), (i, k, fd, g[0, i, k])


# ------------------------------------------------------------------ LDOS

def _ldos_rows():
    out, cur = [], None
    with open(os.path.join(HERE, "golden", "wide_ldos.txt")) as fh:
        for ln in fh:
            if ln.startswith("#"):
                continue
            f = ln.split()
            if f[0] == "ribbon":
                cur = dict(N=int(f[1]), L=int(f[2]), parity=int(f[3]), w=float(f[4]),
                           r=int(f[5]), E=float(f[6]))
                cur["rho"] = np.zeros((cur["L"], cur["N"]))
                out.append(cur)
            else:
                cur["rho"][int(f[0]), int(f[1])] = float(f[2])
    return out


def _ldos(P, N, L, parity, Es, eps=None, stride=0):
    import torch
    rib = P.Ribbon(N, L, parity, W.T_HOP, W.ETA)
    E = torch.tensor(np.asarray(Es, dtype=np.float64), device="cuda")
    ep = None if eps is None else torch.tensor(np.asarray(eps), device="cuda")
    rho, T, st = P.ldos(rib, E, ep, ckpt_stride=stride, return_T=True, return_status=True)
    torch.cuda.synchronize()
    return rho.cpu().numpy(), T.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("k", [0, 1])
def test_wide_ldos_matches_oracle(P, k):
    """-Im G_ss/pi of every site against the oracle, 1e-9 relative to
    max(1, max rho)."""
    c = _ldos_rows()[k]
    N, L = c["N"], c["L"]
    _say("wide ldos", N, L, c["parity"])
    eps = W.disorder(L, N, c["w"], r=c["r"])
    rho, _, st = _ldos(P, N, L, c["parity"], [c["E"]], eps[None])
    assert (st == 0).all()
    scale = max(1.0, np.abs(c["rho"]).max())
    assert np.abs(rho[0, 0] - c["rho"]).max() <= 1e-9 * scale


def test_wide_ldos_pristine_period_and_strides(P):
    """A pristine N = 480 ribbon between identical leads is a piece of the
    infinite ribbon: the LDOS repeats every two slices (the bond pattern's
    period) and is non-negative; checkpoint strides agree; T equals the
    conductance call's."""
    N, L = 480, 6
    Es = np.array([0.137, -0.21]) * abs(W.T_HOP)
    _say("wide ldos pristine", N, L)
    rho, T, st = _ldos(P, N, L, 0, Es)
    assert (st == 0).all()
    scale = np.abs(rho).max()
    assert (rho >= -1e-9 * scale).all()
    for i in range(L - 2):
        assert np.abs(rho[0, :, i] - rho[0, :, i + 2]).max() <= 1e-8 * scale
    for stride in (1, 5):
        r2, _, _ = _ldos(P, N, L, 0, Es, stride=stride)
        assert np.abs(r2 - rho).max() <= 1e-12 * scale
    T2, _ = _gpu_T(P, N, L, 0, W.T_HOP, Es)
    assert np.abs(T - T2).max() <= 1e-12 * max(1.0, np.abs(T2).max())
