"""GPU parity of the local density of states (rgf_ldos through the C ABI)
against the oracle's ldos (pinned in tests/test_oracle_ldos.py).

rho_s(E) = -Im G_ss(E)/pi in states per eV per site. Bars: FP64 within
1e-9 relative to max(1, max|rho|) on small and medium ribbons (both sides
FP64, different elimination orders); mixed precision within 1e-7 of FP64.
"""

import sys

import numpy as np
import pytest

import oracle as O
import rgf_workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-9


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1107_5300_amd as P
    P.version()  # loads librgf.so or raises
    return P


def _gpu(P, N, L, parity, t, Es, eps=None, precision="fp64", eta=W.ETA, ckpt_stride=0):
    import torch
    rib = P.Ribbon(N, L, parity, t, eta)
    E = torch.tensor(np.asarray(Es, dtype=np.float64), device="cuda")
    ep = None if eps is None else torch.tensor(np.asarray(eps)[None] if np.ndim(eps) == 2
                                               else np.asarray(eps), device="cuda")
    rho, T, st = P.ldos(rib, E, ep, precision=precision, ckpt_stride=ckpt_stride,
                        return_T=True, return_status=True)
    torch.cuda.synchronize()
    return rho.cpu().numpy(), T.cpu().numpy(), st.cpu().numpy()


def _close(a, b, tol=TOL):
    scale = max(1.0, float(np.abs(b).max()))
    err = float(np.abs(a - b).max())
    assert err <= tol * scale, (err, scale)
    return err


@pytest.mark.parametrize("x", [0.05, 0.6, 1.3, 1.9])
def test_chain_closed_form(P, x):
    """N = 2 pristine ribbon = infinite 1D chain: rho = 1/(pi sqrt(4t^2 - E^2))."""
    t = W.T_HOP
    E = x * abs(t)
    _say("chain", x)
    rho, _, st = _gpu(P, 2, 9, 0, t, [E], eta=1e-12)
    assert (st == 0).all()
    want = 1.0 / (np.pi * np.sqrt(4 * t * t - E * E))
    np.testing.assert_allclose(rho[0, 0], want, rtol=1e-9)


@pytest.mark.parametrize("seed", range(24))
def test_random_small_ribbons(P, seed):
    N, L, parity, t, eps, E = W.random_case(seed)
    _say("random", seed, N, L, parity)
    rho, T, st = _gpu(P, N, L, parity, t, [E], eps)
    assert (st == 0).all()
    _close(rho[0, 0], O.ldos(N, L, t, W.ETA, E, eps, parity))
    assert abs(T[0, 0] - O.transmission(N, L, t, W.ETA, E, eps, parity)) <= 1e-9 * max(1.0, T[0, 0])


@pytest.mark.parametrize("N", [16, 30, 59, 64, 100, 121, 160, 240])
def test_widths_span_tiles(P, N):
    L = 6
    eps = W.disorder(L, N, 0.5, r=3)
    Es = [-0.37 * abs(W.T_HOP), 0.21 * abs(W.T_HOP)]
    _say("width", N)
    rho, _, st = _gpu(P, N, L, 0, W.T_HOP, Es, eps)
    assert (st == 0).all()
    for j, E in enumerate(Es):
        _close(rho[0, j], O.ldos(N, L, W.T_HOP, W.ETA, E, eps, 0))


def test_medium_ribbon_and_realizations(P):
    N, L, R = 60, 40, 3
    eps = W.disorder_batch(L, N, 0.5, R)
    Es = np.array([-0.45, 0.05, 0.33]) * abs(W.T_HOP)
    _say("medium", N, L, R)
    rho, _, st = _gpu(P, N, L, 1, W.T_HOP, Es, eps)
    assert (st == 0).all()
    assert rho.shape == (R, 3, L, N)
    for r in range(R):
        for j, E in enumerate(Es):
            _close(rho[r, j], O.ldos(N, L, W.T_HOP, W.ETA, E, eps[r], 1))


def test_checkpoint_strides_agree(P):
    N, L = 24, 13
    eps = W.disorder(L, N, 0.4, r=5)
    Es = [0.3 * abs(W.T_HOP)]
    ref, _, _ = _gpu(P, N, L, 0, W.T_HOP, Es, eps)
    for s in (1, 3, 7, 26):
        _say("stride", s)
        got, _, st = _gpu(P, N, L, 0, W.T_HOP, Es, eps, ckpt_stride=s)
        assert (st == 0).all()
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * max(1.0, np.abs(ref).max()))


def test_mixed_precision_vs_oracle(P):
    """Mixed-precision LDOS of every site against the oracle (as FP64)."""
    N, L = 120, 30
    eps = W.disorder(L, N, 0.5, r=1)
    Es = np.array([-0.4, 0.12]) * abs(W.T_HOP)
    _say("mixed", N, L)
    b, _, sb = _gpu(P, N, L, 0, W.T_HOP, Es, eps, precision="mixed")
    assert (sb == 0).all()
    for j, E in enumerate(Es):
        _close(b[0, j], O.ldos(N, L, W.T_HOP, W.ETA, E, eps, 0))


@pytest.mark.parametrize("seed", range(4))
def test_mixed_small_ribbons_vs_oracle(P, seed):
    N, L, parity, t, eps, E = W.random_case(7300 + seed, n_max=20, l_max=9)
    _say("mixed small", seed, N, L, parity)
    Es = [E, 0.38 * abs(t)]
    rho, _, st = _gpu(P, N, L, parity, t, Es, eps, precision="mixed")
    assert (st == 0).all()
    for j, Ej in enumerate(Es):
        _close(rho[0, j], O.ldos(N, L, t, W.ETA, Ej, eps, parity))


def test_nan_energy_sets_status(P):
    rho, T, st = _gpu(P, 10, 5, 0, W.T_HOP, [0.3, float("nan")])
    assert st[0, 0] == 0 and st[0, 1] != 0
    assert np.isnan(rho[0, 1]).all() and np.isnan(T[0, 1])
    assert np.isfinite(rho[0, 0]).all()


def test_non_negative_at_scale(P):
    N, L = 240, 200
    eps = W.disorder(L, N, 0.5, r=0)
    Es = np.linspace(-0.5, 0.5, 8) * abs(W.T_HOP)
    _say("scale", N, L)
    rho, _, st = _gpu(P, N, L, 0, W.T_HOP, Es, eps)
    assert (st == 0).all()
    assert (rho >= -1e-9 * np.abs(rho).max()).all()
