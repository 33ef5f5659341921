"""Pins of the oracle's per-channel transmission (CPU only).

The channels are the eigenvectors of Gamma_L with a non-zero eigenvalue
(Eq. (2) split over them). Pins from outside the function:
  * a pristine ribbon is one piece of the infinite ribbon: every open channel
    is transmitted fully, T_i = 1, and there are M(E) of them (the closed-form
    subband count);
  * unitarity bounds each channel, 0 <= T_i <= 1, for disordered ribbons;
  * the channels sum to the brute-force conductance of the full inverse;
  * the recursion's G_{1L} and the full inverse give the same channels.
A dropped Gamma_R, a transposed G or a wrong sign of Gamma fails one of these.
"""

import numpy as np
import pytest

import oracle as O
import rgf_workloads as W

T_HOP, ETA = W.T_HOP, W.ETA


@pytest.mark.parametrize("N,E", [(6, 0.8), (9, -1.3), (12, 0.47), (20, 0.9), (21, -2.1)])
def test_pristine_channels_transmit_fully(N, E):
    g, Ti = O.channel_transmission_bf(N, 4, T_HOP, ETA, E)
    M = O.open_channels(N, E, T_HOP)
    assert len(Ti) == M
    assert np.abs(Ti - 1.0).max() <= 1e-5


@pytest.mark.parametrize("seed", range(12))
def test_disordered_channels_bounded_and_sum(seed):
    N, L, parity, t, eps, E = W.random_case(5200 + seed, n_max=10, l_max=6)
    g, Ti = O.channel_transmission_bf(N, L, t, ETA, E, eps, parity)
    assert (Ti >= -1e-10).all() and (Ti <= 1 + 1e-9).all()
    T = O.transmission_bf(N, L, t, ETA, E, eps, parity)
    assert abs(Ti.sum() - T) <= 1e-9 * max(1.0, T)


@pytest.mark.parametrize("seed", range(8))
def test_recursion_equals_full_inverse(seed):
    N, L, parity, t, eps, E = W.random_case(5300 + seed, n_max=10, l_max=6)
    sig = O.lead_self_energies(N, L, t, ETA, E, parity)
    g1, T1 = O.channel_transmission(N, L, t, ETA, E, eps, parity, sigmas=sig)
    g2, T2 = O.channel_transmission_bf(N, L, t, ETA, E, eps, parity, sigmas=sig)
    np.testing.assert_allclose(g1, g2, rtol=1e-12)
    np.testing.assert_allclose(T1, T2, rtol=0, atol=1e-9)


def test_planted_transpose_is_caught():
    """Using G^T G^dagger-style products instead of G Gamma_R G^dagger breaks
    the pristine pin: a mutation check on the CPU."""
    N, L, E = 12, 4, 0.47
    sig = O.lead_self_energies(N, L, T_HOP, ETA, E, 0)
    _, G = O.transmission(N, L, T_HOP, ETA, E, None, 0, sigmas=sig, return_g=True)
    gl, gr = 1j * (sig[0] - sig[0].conj().T), 1j * (sig[1] - sig[1].conj().T)
    w, Ti = O.rgf_oracle._channel_split(gl, gr, G, 1e-6)
    wb, Tb = O.rgf_oracle._channel_split(gl, np.eye(N), G, 1e-6)   # Gamma_R dropped
    assert np.abs(Ti - 1).max() <= 1e-5
    assert np.abs(Tb - 1).max() > 1e-2
