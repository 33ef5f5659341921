"""GPU parity of lattice defects: vacancies (on-site energy +inf, the site
removed from the lattice) and edge roughness (vacancies confined to the two
edge rows), against the oracle, whose own vacancy handling is pinned to the
brute-force inverse with the sites deleted (test_oracle_defects.py).

Every kernel family sees them: the register Gauss-Jordan (narrow ribbons,
FP64 and mixed), the matrix-core Gauss-Jordan (mixed, half-slices of
97..128 rows), the panel Gauss-Jordan (N > 256), the whole-slice fallback
near E = 0, and the gradient and LDOS sweeps, whose outputs at a vacancy
are exactly 0. Bars as for disordered ribbons: 1e-9 relative for FP64
conductances, 1e-8 for mixed precision and for gradients (relative to
max(1, max|dT/deps|)), 1e-9 absolute for the LDOS.
"""

import os
import sys

import numpy as np
import pytest

import oracle as O
import rgf_workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-9
HERE = os.path.dirname(os.path.abspath(__file__))


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


def _t(x):
    import torch
    return torch.tensor(np.asarray(x, dtype=np.float64), device="cuda")


def _T(P, N, L, parity, Es, eps, precision="fp64", t=W.T_HOP):
    import torch
    T, st = P.conductance(P.Ribbon(N, L, parity, t, W.ETA), _t(Es), _t(eps),
                          precision=precision, return_status=True)
    torch.cuda.synchronize()
    return T.cpu().numpy(), st.cpu().numpy()


def _case(seed, n_max=40, l_max=12):
    rng = np.random.default_rng(77000 + seed)
    N = int(rng.integers(3, n_max + 1))
    L = int(rng.integers(1, l_max + 1))
    parity = int(rng.integers(0, 2))
    w = float(rng.choice([0.0, 0.2, 0.5]))
    eps = W.vacancies(W.disorder(L, N, w, r=seed), float(rng.choice([0.03, 0.1, 0.2])), seed)
    E = float(rng.uniform(-0.9, 0.9) * abs(W.T_HOP))
    return N, L, parity, eps, E


def _check_T(got, eps, N, L, parity, Es, tol, t=W.T_HOP):
    for j, E in enumerate(Es):
        sig = O.lead_self_energies(N, L, t, W.ETA, E, parity)
        for r in range(eps.shape[0]):
            want = O.transmission(N, L, t, W.ETA, E, eps[r], parity, sigmas=sig)
            assert abs(got[r, j] - want) <= tol * max(1.0, abs(want)), (r, E, got[r, j], want)


@pytest.mark.parametrize("seed", range(16))
def test_vacancies_small_ribbons_fp64(P, seed):
    N, L, parity, eps, E = _case(seed)
    Es = [E, 0.37 * abs(W.T_HOP), -0.62 * abs(W.T_HOP)]
    _say("vacancies fp64", seed, N, L, parity, int(np.isinf(eps).sum()))
    got, st = _T(P, N, L, parity, Es, eps[None])
    assert (st == 0).all(), st
    _check_T(got, eps[None], N, L, parity, Es, TOL)


@pytest.mark.parametrize("seed", range(8))
def test_vacancies_small_ribbons_mixed(P, seed):
    N, L, parity, eps, E = _case(100 + seed)
    Es = [E, -0.29 * abs(W.T_HOP)]
    _say("vacancies mixed", seed, N, L, parity)
    got, st = _T(P, N, L, parity, Es, eps[None], "mixed")
    assert (st == 0).all(), st
    _check_T(got, eps[None], N, L, parity, Es, 1e-8)


@pytest.mark.parametrize("N,precision", [(61, "fp64"), (120, "fp64"), (240, "fp64"),
                                         (200, "mixed"), (240, "mixed"), (90, "mixed")])
def test_vacancies_across_tilings(P, N, precision):
    """Every register tiling (FP64), the matrix-core Gauss-Jordan (mixed,
    N = 193..256) and the register path of the mixed mode (N = 90), with
    several realizations in one launch."""
    L, R = 9, 3
    eps = np.stack([W.vacancies(W.disorder(L, N, 0.3, r=40 + r), 0.05, 60 + r) for r in range(R)])
    Es = np.array([-0.45, 0.08, 0.36]) * abs(W.T_HOP)
    _say("vacancies tilings", N, precision)
    got, st = _T(P, N, L, 0, Es, eps, precision)
    assert (st == 0).all(), st
    _check_T(got, eps, N, L, 0, Es, TOL if precision == "fp64" else 1e-8)


def _golden():
    """tests/golden/defects_wide.txt (make_defects_golden.py, oracle/ only)."""
    T, grad, ldos, cur = [], None, None, None
    with open(os.path.join(HERE, "golden", "defects_wide.txt")) as fh:
        for ln in fh:
            if ln.startswith("#"):
                continue
            f = ln.split()
            if f[0] in ("T", "grad", "ldos"):
                c = dict(N=int(f[1]), L=int(f[2]), parity=int(f[3]), w=float(f[4]),
                         r=int(f[5]), d=float(f[6]), s=int(f[7]), E=float(f[8]))
                if f[0] == "T":
                    c["T"] = float(f[9])
                    T.append(c)
                    continue
                if f[0] == "grad":
                    c["T"] = float(f[9])
                    grad = c
                else:
                    ldos = c
                cur = c
                c["a"] = np.zeros((c["L"], c["N"]))
            else:
                cur["a"][int(f[0]), int(f[1])] = float(f[2])
    return T, grad, ldos


def _geps(c):
    return W.vacancies(W.disorder(c["L"], c["N"], c["w"], r=c["r"]), c["d"], c["s"])


@pytest.mark.parametrize("k", range(6))
def test_vacancies_wide_ribbons(P, k):
    """Half-slices above 128 rows (the panel Gauss-Jordan), and a pristine
    metallic N = 290 ribbon with a few vacancies near E = 0 (the
    whole-slice fallback of wide ribbons), against the stored oracle."""
    c = _golden()[0][k]
    N, L, parity = c["N"], c["L"], c["parity"]
    eps = _geps(c)
    assert np.isinf(eps).any()
    _say("vacancies wide", N, L, parity, c["E"])
    got, st = _T(P, N, L, parity, [c["E"]], eps[None])
    assert (st == 0).all(), st
    want = c["T"]
    # in a gap T is rounding noise of order 1e-9 in the oracle's wide leads
    tol = 1e-8 if O.open_channels(N, c["E"], W.T_HOP) == 0 else TOL * max(1.0, abs(want))
    assert abs(got[0, 0] - want) <= tol, (got[0, 0], want)


@pytest.mark.parametrize("N,parity", [(14, 0), (23, 1), (58, 0)])
def test_edge_roughness(P, N, parity):
    """Vacancies confined to the two edge rows (edge roughness), long
    ribbon: the oracle's value."""
    L = 60
    eps = W.vacancies(np.zeros((L, N)), 0.3, 3, rows=(0, N - 1))
    Es = [0.1 * abs(W.T_HOP), 0.42 * abs(W.T_HOP), -0.77 * abs(W.T_HOP)]
    _say("edge roughness", N, parity, int(np.isinf(eps).sum()))
    got, st = _T(P, N, L, parity, Es, eps[None])
    assert (st == 0).all(), st
    _check_T(got, eps[None], N, L, parity, Es, TOL)


def test_cut_slice_blocks_transport(P):
    """A slice with every site removed disconnects the leads: T = 0 (the
    Green's function between the ends vanishes identically), and a slice
    with one site left conducts no more than one channel."""
    N, L = 12, 8
    eps = np.zeros((2, L, N))
    eps[0, 3, :] = np.inf
    eps[1, 3, :] = np.inf
    eps[1, 3, 5] = 0.0
    Es = [0.2 * abs(W.T_HOP), 0.6 * abs(W.T_HOP)]
    _say("cut slice")
    got, st = _T(P, N, L, 0, Es, eps)
    assert (st == 0).all(), st
    assert (got[0] == 0.0).all(), got[0]
    assert (got[1] <= 1.0 + 1e-12).all() and (got[1] >= -1e-12).all()
    _check_T(got, eps, N, L, 0, Es, TOL)


@pytest.mark.parametrize("L", [1, 2])
def test_vacancies_at_the_lead_interfaces(P, L):
    """Vacancies in the first and last slice (the sites the leads couple
    to), down to a one-slice device."""
    N = 16
    eps = np.zeros((L, N))
    eps[0, [0, 5, 6]] = np.inf
    eps[L - 1, [3, 15]] = np.inf
    Es = [0.15 * abs(W.T_HOP), -0.55 * abs(W.T_HOP)]
    for parity in (0, 1):
        _say("lead interface vacancies", L, parity)
        got, st = _T(P, N, L, parity, Es, eps[None])
        assert (st == 0).all(), st
        _check_T(got, eps[None], N, L, parity, Es, TOL)


def test_vacancies_near_zero_energy_take_the_fallback(P):
    """A nearly pristine metallic ribbon with a few vacancies near E = 0,
    where the half-slice recursion alone loses digits: equal to the oracle
    (the whole-slice fallback removes the sites the same way)."""
    N, L = 20, 40
    eps = W.vacancies(np.zeros((L, N)), 0.01, 21)
    assert np.isinf(eps).any()
    Es = [2e-7, 1e-6, 1e-5, 1e-4]
    _say("vacancies near zero")
    got, st = _T(P, N, L, 0, Es, eps[None])
    assert (st == 0).all(), st
    _check_T(got, eps[None], N, L, 0, Es, TOL)
    got, st = _T(P, N, L, 0, Es, eps[None], "mixed")
    assert (st == 0).all(), st
    _check_T(got, eps[None], N, L, 0, Es, TOL)


def _grad(P, N, L, parity, Es, eps, w, precision="fp64"):
    import torch
    T, g, st = P.grad(P.Ribbon(N, L, parity, W.T_HOP, W.ETA), _t(Es), _t(eps), _t(w),
                      precision=precision, return_status=True)
    torch.cuda.synchronize()
    return T.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("seed,N,precision", [(0, 9, "fp64"), (1, 17, "fp64"), (2, 30, "fp64"),
                                              (3, 140, "fp64"), (4, 21, "mixed")])
def test_vacancy_gradient_vs_oracle(P, seed, N, precision):
    """dT/deps with vacancies: equal to the oracle's, exactly 0 at every
    vacancy (register path; N = 140 on the widest narrow tiling)."""
    L = 7
    eps = W.vacancies(W.disorder(L, N, 0.3, r=seed), 0.08, 500 + seed)
    rng = np.random.default_rng(seed)
    Es = np.array([0.27, -0.48]) * abs(W.T_HOP)
    w = rng.normal(size=(1, len(Es)))
    _say("vacancy grad", seed, N, precision)
    T, g, st = _grad(P, N, L, seed & 1, Es, eps[None], w, precision)
    assert (st == 0).all(), st
    want = np.zeros((L, N))
    for j, E in enumerate(Es):
        Tj, dj = O.transmission_grad(N, L, W.T_HOP, W.ETA, E, eps, seed & 1)
        assert abs(T[0, j] - Tj) <= TOL * max(1.0, abs(Tj))
        want += w[0, j] * dj
    assert (g[0][np.isinf(eps)] == 0.0).all()
    assert np.abs(g[0] - want).max() <= 1e-8 * max(1.0, np.abs(want).max())


def test_wide_vacancy_gradient_and_ldos(P):
    """N = 270 gradient and N = 262 LDOS (panel path) with vacancies against
    the stored oracle; exactly 0 at the vacancies."""
    import torch
    _, cg, cl = _golden()
    eps = _geps(cg)
    _say("wide vacancy grad", cg["N"], cg["L"])
    T, g, st = _grad(P, cg["N"], cg["L"], cg["parity"], [cg["E"]], eps[None], [[1.0]])
    assert (st == 0).all(), st
    assert abs(T[0, 0] - cg["T"]) <= TOL * max(1.0, abs(cg["T"]))
    assert (g[0][np.isinf(eps)] == 0.0).all()
    assert np.abs(g[0] - cg["a"]).max() <= 1e-8 * max(1.0, np.abs(cg["a"]).max())
    eps = _geps(cl)
    _say("wide vacancy ldos", cl["N"], cl["L"])
    rho, st = P.ldos(P.Ribbon(cl["N"], cl["L"], cl["parity"], W.T_HOP, W.ETA), _t([cl["E"]]),
                     _t(eps[None]), return_status=True)
    torch.cuda.synchronize()
    rho, st = rho.cpu().numpy(), st.cpu().numpy()
    assert (st == 0).all(), st
    assert (rho[0, 0][np.isinf(eps)] == 0.0).all()
    assert np.abs(rho[0, 0] - cl["a"]).max() <= 1e-9


@pytest.mark.parametrize("N", [11, 64, 150])
def test_vacancy_ldos_vs_oracle(P, N):
    """LDOS with vacancies: the oracle's at every site, exactly 0 at the
    vacancies."""
    import torch
    L = 6
    eps = W.vacancies(W.disorder(L, N, 0.25, r=N), 0.1, N)
    Es = [0.33 * abs(W.T_HOP)]
    _say("vacancy ldos", N)
    rho, T, st = P.ldos(P.Ribbon(N, L, 0, W.T_HOP, W.ETA), _t(Es), _t(eps[None]),
                        return_T=True, return_status=True)
    torch.cuda.synchronize()
    rho, st = rho.cpu().numpy(), st.cpu().numpy()
    assert (st == 0).all(), st
    want = O.ldos(N, L, W.T_HOP, W.ETA, Es[0], eps, 0)
    assert (rho[0, 0][np.isinf(eps)] == 0.0).all()
    assert np.abs(rho[0, 0] - want).max() <= 1e-9, np.abs(rho[0, 0] - want).max()


def test_vacancy_channels_batched_and_noalloc(P):
    """Per-channel transmission sums to T with vacancies; the batched and
    the no-allocation entry points equal the workspace call bit for bit."""
    import torch
    N, L = 26, 15
    eps = W.vacancies(W.disorder(L, N, 0.2, r=3), 0.06, 3)
    Es = _t(np.array([0.12, 0.51]) * abs(W.T_HOP))
    rib = P.Ribbon(N, L, 1, W.T_HOP, W.ETA)
    _say("vacancy channels batched noalloc")
    ep = _t(eps[None])
    tc, Tc, stc = P.channel_transmission(rib, Es, ep, return_status=True)
    T1, st1 = P.conductance(rib, Es, ep, return_status=True)
    T2, st2 = P.conductance_noalloc(rib, Es, ep, return_status=True)
    outs, sts = P.conductance_batched([rib], Es, [ep], return_status=True)
    torch.cuda.synchronize()
    for s in (stc, st1, st2, sts[0]):
        assert (s.cpu() == 0).all()
    assert torch.equal(T2.cpu(), T1.cpu()) and torch.equal(outs[0].cpu(), T1.cpu())
    assert np.abs(tc.cpu().numpy().sum(-1) - T1.cpu().numpy()).max() <= 1e-9
    _check_T(T1.cpu().numpy(), eps[None], N, L, 1, Es.cpu().numpy(), TOL)
