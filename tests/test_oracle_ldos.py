"""Pins of the oracle's local density of states (CPU only).

rho_s(E) = -Im G_ss(E) / pi with G the full Green's function of Eq. (1).
  * ldos_bf (the definition, from the full inverse) against the closed form
    of the infinite 1D chain: the N = 2 armchair ribbon is a single chain
    with hopping t, and with pristine leads on both sides every device site
    has rho = 1 / (pi sqrt(4 t^2 - E^2)) inside the band.
  * ldos (forward sweep + backward recursion of the diagonal blocks) against
    ldos_bf on small random ribbons, both parities, either sign of t.
  * non-negativity.
"""

import numpy as np
import pytest

import oracle as O
import oracle.rgf_oracle as R
import rgf_workloads as W

T = W.T_HOP


def _chain(E, t=T):
    return 1.0 / (np.pi * np.sqrt(4.0 * t * t - E * E))


@pytest.mark.parametrize("x", [0.05, 0.4, 1.1, 1.9])
@pytest.mark.parametrize("fn", ["ldos_bf", "ldos"])
def test_chain_closed_form(fn, x):
    E = x * abs(T)
    r = getattr(O, fn)(2, 7, T, 1e-12, E)
    np.testing.assert_allclose(r, _chain(E), rtol=1e-8, atol=0)


@pytest.mark.parametrize("seed", range(16))
def test_recursion_matches_brute_force(seed):
    N, L, parity, t, eps, E = W.random_case(seed)
    a = O.ldos(N, L, t, W.ETA, E, eps, parity)
    b = O.ldos_bf(N, L, t, W.ETA, E, eps, parity)
    assert a.shape == (L, N)
    np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-12 * max(1.0, np.abs(b).max()))


@pytest.mark.parametrize("seed", range(6))
def test_non_negative(seed):
    N, L, parity, t, eps, E = W.random_case(seed + 100)
    assert (O.ldos(N, L, t, W.ETA, E, eps, parity) >= -1e-12).all()


def test_pristine_ribbon_is_translation_invariant():
    """With ideal leads on both sides a pristine device is a piece of the
    infinite ribbon: every slice has the same LDOS profile, positive inside
    the band."""
    N, L = 12, 9
    E = 0.9 * abs(T)
    r = O.ldos(N, L, T, 1e-10, E)
    assert (r > 0).all()
    np.testing.assert_allclose(r, np.broadcast_to(r[0], r.shape), rtol=1e-8)


def test_mutated_bond_is_caught(monkeypatch):
    """A dropped transverse bond (a plausible indexing mistake) breaks the
    chain closed form."""
    orig = R.slice_hamiltonian

    def sh(N, t, eps_row=None):
        H = orig(N, t, eps_row)
        H[N - 2, N - 1] = H[N - 1, N - 2] = 0.0
        return H
    monkeypatch.setattr(R, "slice_hamiltonian", sh)
    E = 0.4 * abs(T)
    r = R.ldos(2, 7, T, 1e-12, E)
    assert not np.allclose(r, _chain(E), rtol=1e-6)
