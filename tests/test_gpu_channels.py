"""GPU parity of the per-channel transmission (rgf_channel_transmission) and
of the two lead methods (rgf_lead_modes: decimation and mode matching),
through the C ABI, against the oracle.

Channels: the oracle splits Eq. (2) over the eigenvectors of its dense
Gamma_L; the library over its transverse mode chains. The two sets are the
same channels (evanescent modes included: their broadening is of order eta,
not zero, and a few carry T_p ~ 1e-6), so the sorted lists of channel
transmissions agree. Bars: 1e-9 absolute per channel on short
ribbons (both FP64), sum over channels = T to 1e-12 relative.
"""

import sys

import numpy as np
import pytest

import oracle as O
import rgf_workloads as W

pytestmark = pytest.mark.gpu


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


def _chan(P, N, L, parity, t, Es, eps=None):
    import torch
    rib = P.Ribbon(N, L, parity, t, W.ETA)
    tc, T, st = P.channel_transmission(rib, _t(Es), None if eps is None else _t(eps),
                                       return_status=True)
    torch.cuda.synchronize()
    return tc.cpu().numpy(), T.cpu().numpy(), st.cpu().numpy()


def _compare(gpu_tp, oracle_ti, tol=1e-9):
    g = np.sort(gpu_tp)[::-1]
    o = np.sort(oracle_ti)[::-1]
    k = min(len(o), len(g))
    assert np.abs(g[:k] - o[:k]).max(initial=0.0) <= tol, (g[:k], o[:k])
    assert np.abs(g[k:]).max(initial=0.0) <= tol and np.abs(o[k:]).max(initial=0.0) <= tol


# ------------------------------------------------------------------ leads

@pytest.mark.parametrize("N", [2, 7, 20, 21, 60, 240, 480])
def test_lead_methods_agree(P, N):
    """Decimation and closed-form mode matching give the same sigma_p."""
    xs = np.array([-1.0, -0.83, -0.2, 0.013, 0.37, 0.91, 1.0, 1.7, -2.4])
    if N % 2 == 1:
        xs = xs[np.abs(np.abs(xs) - 1.0) > 1e-3]   # flat band of odd N at |E| = |t|
    Es = xs * abs(W.T_HOP)
    rib = P.Ribbon(N, 4, 0, W.T_HOP, W.ETA)
    _say("lead methods", N)
    s0, st0 = P.lead_modes(rib, _t(Es), "decimation")
    s1, st1 = P.lead_modes(rib, _t(Es), "mode_matching")
    s0, s1 = s0.cpu().numpy(), s1.cpu().numpy()
    assert (st0.cpu().numpy() == 0).all() and (st1.cpu().numpy() == 0).all()
    assert s0.shape == (len(Es), (N + 1) // 2)
    err = np.abs(s0 - s1).max() / max(1.0, np.abs(s0).max())
    assert err <= 1e-9, err
    assert (s1.imag <= 1e-12).all()   # retarded: Im sigma <= 0


@pytest.mark.parametrize("N,parity", [(7, 0), (20, 0), (21, 1)])
def test_mode_matching_dense_sigma_matches_oracle(P, N, parity):
    """Sigma_L = Phi diag(sigma_p) Phi^T from the mode-matching sigma_p, with
    the textbook transverse modes of the zigzag chain, against the oracle's
    dense lead self-energy (its own decimation of the two-slice cell)."""
    L = 4
    Es = np.array([-0.83, 0.37, 1.7]) * abs(W.T_HOP)
    rib = P.Ribbon(N, L, parity, W.T_HOP, W.ETA)
    sig, st = P.lead_modes(rib, _t(Es), "mode_matching")
    sig = sig.cpu().numpy()
    rows = np.arange(parity % 2, N, 2)
    p = np.arange(1, (N + 1) // 2 + 1)
    phi = np.sqrt(2.0 / (N + 1)) * np.sin(np.outer(p, rows + 1) * np.pi / (N + 1))
    for j, E in enumerate(Es):
        dense = phi.T @ np.diag(sig[j]) @ phi
        ol, _ = O.lead_self_energies(N, L, W.T_HOP, W.ETA, E, parity)
        want = ol[np.ix_(rows, rows)]
        assert np.abs(dense - want).max() <= 1e-9 * max(1.0, np.abs(want).max())


# ------------------------------------------------------------------ channels

@pytest.mark.parametrize("seed", range(16))
def test_channels_small_vs_oracle(P, seed):
    N, L, parity, t, eps, E = W.random_case(6100 + seed, n_max=14, l_max=8)
    _say("channels small", seed, N, L, parity)
    tc, T, st = _chan(P, N, L, parity, t, [E], eps[None])
    assert st[0, 0] == 0
    assert abs(tc[0, 0].sum() - T[0, 0]) <= 1e-12 * max(1.0, T[0, 0])
    _, ti = O.channel_transmission(N, L, t, W.ETA, E, eps, parity, rel_tol=1e-14)
    _compare(tc[0, 0], ti)


@pytest.mark.parametrize("N", [20, 60, 121])
def test_channels_pristine_transmit_fully(P, N):
    Es = np.array([-0.47, 0.33, 0.88]) * abs(W.T_HOP)
    _say("channels pristine", N)
    tc, T, st = _chan(P, N, 5, 0, W.T_HOP, Es)
    assert (st == 0).all()
    for j, E in enumerate(Es):
        M = O.open_channels(N, E, W.T_HOP)
        g = np.sort(tc[0, j])[::-1]
        assert np.abs(g[:M] - 1.0).max(initial=0.0) <= 1e-5
        assert np.abs(g[M:]).max(initial=0.0) <= 1e-6


def test_channels_medium_disordered(P):
    N, L = 120, 40
    eps = W.disorder(L, N, 0.5, r=9)
    Es = np.array([-0.3, 0.21]) * abs(W.T_HOP)
    _say("channels medium", N, L)
    tc, T, st = _chan(P, N, L, 0, W.T_HOP, Es, eps[None])
    assert (st == 0).all()
    for j, E in enumerate(Es):
        _, ti = O.channel_transmission(N, L, W.T_HOP, W.ETA, E, eps, 0, rel_tol=1e-14)
        _compare(tc[0, j], ti)
        assert ((tc[0, j] >= -1e-12) & (tc[0, j] <= 1 + 1e-9)).all()


def test_channels_wide_pristine_and_sum(P):
    """N = 480 (panel path): full transmission of the M(E) open channels of a
    pristine ribbon; a disordered one sums to T."""
    N = 480
    Es = np.array([0.137, -0.21]) * abs(W.T_HOP)
    _say("channels wide", N)
    tc, T, st = _chan(P, N, 4, 0, W.T_HOP, Es)
    assert (st == 0).all()
    for j, E in enumerate(Es):
        M = O.open_channels(N, E, W.T_HOP)
        g = np.sort(tc[0, j])[::-1]
        assert np.abs(g[:M] - 1.0).max() <= 1e-5 and np.abs(g[M:]).max() <= 1e-6
    eps = W.disorder(4, N, 0.5, r=3)
    tc, T, st = _chan(P, N, 4, 0, W.T_HOP, Es, eps[None])
    assert (st == 0).all()
    assert np.abs(tc[0].sum(axis=1) - T[0]).max() <= 1e-12 * max(1.0, np.abs(T).max())
    assert ((tc >= -1e-12) & (tc <= 1 + 1e-9)).all()


def test_channels_wide_vs_oracle(P):
    """N = 258 (panel path), L = 2, disordered: the channel list against the
    oracle's eigen-decomposition of its dense Gamma_L, run here (its lead
    decimation at this width takes seconds)."""
    N, L = 258, 2
    eps = W.disorder(L, N, 0.5, r=58)
    E = 0.31 * abs(W.T_HOP)
    _say("channels wide oracle", N, L)
    tc, T, st = _chan(P, N, L, 1, W.T_HOP, [E], eps[None])
    assert st[0, 0] == 0
    _, ti = O.channel_transmission(N, L, W.T_HOP, W.ETA, E, eps, 1, rel_tol=1e-14)
    _compare(tc[0, 0], ti)
    assert abs(tc[0, 0].sum() - T[0, 0]) <= 1e-12 * max(1.0, T[0, 0])


def test_channels_nan_status(P):
    tc, T, st = _chan(P, 10, 5, 0, W.T_HOP, [0.3, float("nan")])
    assert st[0, 0] == 0 and st[0, 1] != 0
    assert np.isfinite(tc[0, 0]).all() and np.isnan(tc[0, 1]).all()
