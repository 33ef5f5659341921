"""Mutation check of the oracle's pins (CPU only).

Each case plants one plausible mistake in the oracle (a dropped bond, a
flipped parity, a wrong sign, a missing self-energy, the advanced instead of
the retarded lead, a lost factor) and checks that the independent pins of
tests/test_oracle_pins.py (closed forms, brute force, finite differences)
reject the mutated oracle, while the unmodified oracle passes them.
"""

import numpy as np
import pytest

import oracle as O
import oracle.rgf_oracle as R
import rgf_workloads as W

from test_oracle_pins import _sigma_closed_form

T = W.T_HOP
ETA = W.ETA


def _battery():
    """A few pins from test_oracle_pins, as booleans."""
    ok = []
    # (1) recursion == brute force on small disordered ribbons
    for seed in (3, 11, 29):
        N, L, parity, t, eps, E = W.random_case(seed)
        a = O.transmission(N, L, t, ETA, E, eps, parity)
        b = O.transmission_bf(N, L, t, ETA, E, eps, parity)
        ok.append(abs(a - b) <= 1e-9 * max(1.0, abs(b)))
    # (2) pristine quantisation T = M(E)
    for x in (-0.62, 0.31, 0.9):
        E = x * abs(T)
        Tq = O.transmission(12, 9, T, ETA, E)
        ok.append(abs(Tq - O.open_channels(12, E, T)) <= 1e-4)
    # (3) lead self-energy == closed-form mode chains on the interface rows
    for (N, parity, L, x) in ((6, 1, 2, 0.8), (7, 0, 4, 0.4)):
        E = x * abs(T)
        sl, sr = O.lead_self_energies(N, L, T, ETA, E, parity)
        ks, S = _sigma_closed_form(N, T, ETA, E, interface_even=(parity % 2 == 0))
        ok.append(np.abs(sl[np.ix_(ks, ks)] - S).max() <= 1e-10 * np.abs(S).max())
        ks, S = _sigma_closed_form(N, T, ETA, E, interface_even=((L + parity) % 2 == 0))
        ok.append(np.abs(sr[np.ix_(ks, ks)] - S).max() <= 1e-10 * np.abs(S).max())
    # (4) 1D chain with one impurity
    eps = np.zeros((6, 2))
    eps[2, 1] = 0.5 * abs(T)
    Ee = 0.3 * abs(T)
    want = (4 * T * T - Ee * Ee) / (4 * T * T - Ee * Ee + (0.5 * abs(T)) ** 2)
    ok.append(abs(O.transmission(2, 6, T, 1e-12, Ee, eps, 0) - want) <= 1e-8)
    # (5) gradient recursion vs central finite differences of the brute force
    N, L, parity, t = 6, 4, 0, T
    eps = W.disorder(L, N, 0.4, r=8)
    E = 0.9 * abs(T)
    _, d = O.transmission_grad(N, L, t, ETA, E, eps, parity)
    assert np.abs(d).max() > 1e-2
    h = 1e-6 * abs(t)
    i, k = np.unravel_index(np.argmax(np.abs(d)), d.shape)
    ep = eps.copy(); ep[i, k] += h
    em = eps.copy(); em[i, k] -= h
    fd = (O.transmission_bf(N, L, t, ETA, E, ep, parity)
          - O.transmission_bf(N, L, t, ETA, E, em, parity)) / (2 * h)
    ok.append(abs(fd - d[i, k]) <= 1e-6 + 1e-4 * abs(fd))
    return all(ok)


def test_unmodified_oracle_passes():
    assert _battery()


def _mut_dropped_bond(monkeypatch):
    orig = R.slice_hamiltonian

    def sh(N, t, eps_row=None):
        H = orig(N, t, eps_row)
        if N > 2:
            H[N - 2, N - 1] = H[N - 1, N - 2] = 0.0
        return H
    monkeypatch.setattr(R, "slice_hamiltonian", sh)


def _mut_parity(monkeypatch):
    monkeypatch.setattr(R, "coupling_mask",
                        lambda N, i, parity=0: ((np.arange(N) + i + parity + 1) % 2) == 0)


def _mut_gamma_missing_i(monkeypatch):
    monkeypatch.setattr(R, "_gamma", lambda sig: sig - sig.conj().T)


def _mut_dyson_sign(monkeypatch):
    orig_inv = np.linalg.inv
    # z - H + U^T g U instead of z - H - U^T g U: flip the coupling term by
    # negating t in the diagonal coupling used by the recursion only
    orig_cd = R.coupling_diag
    state = {"in_rec": False}
    orig_tr = R.transmission

    def tr(*a, **k):
        state["in_rec"] = True
        try:
            return orig_tr(*a, **k)
        finally:
            state["in_rec"] = False

    def cd(N, t, i, parity=0):
        v = orig_cd(N, t, i, parity)
        return v * (1j if state["in_rec"] else 1.0)   # u^2 -> -u^2
    monkeypatch.setattr(R, "coupling_diag", cd)
    monkeypatch.setattr(R, "transmission", tr)
    monkeypatch.setattr(O, "transmission", tr)
    del orig_inv


def _mut_missing_sigma_r(monkeypatch):
    orig = R.lead_self_energies

    def lse(*a, **k):
        out = orig(*a, **k)
        if isinstance(out, tuple) and len(out) == 2:
            return out[0], np.zeros_like(out[1])
        return out
    monkeypatch.setattr(R, "lead_self_energies", lse)
    monkeypatch.setattr(O, "lead_self_energies", lse)


def _mut_advanced_lead(monkeypatch):
    orig = R.surface_gf_modes
    monkeypatch.setattr(R, "surface_gf_modes",
                        lambda z, h00, h01: orig(np.conj(z), h00, h01))


def _mut_grad_factor(monkeypatch):
    orig = R.transmission_grad

    def tg(*a, **k):
        Tv, d = orig(*a, **k)
        return Tv, 0.5 * d
    monkeypatch.setattr(R, "transmission_grad", tg)
    monkeypatch.setattr(O, "transmission_grad", tg)


def _mut_g1_without_coupling(monkeypatch):
    orig_cd = R.coupling_diag
    orig_tr = R.transmission
    calls = {"n": 0}

    def tr(N, L, t, eta, E, eps=None, parity=0, sigmas=None, return_g=False):
        # same sweep, but G1 advanced without the hopping block
        z = complex(E, eta)
        if sigmas is None:
            sigmas = R.lead_self_energies(N, L, t, eta, E, parity)
        sig_l, sig_r = sigmas
        Hs = R._device_slices(N, L, t, eps)
        eye = np.eye(N, dtype=np.complex128)
        A = z * eye - Hs[0] - sig_l - (sig_r if L == 1 else 0)
        g = np.linalg.inv(A)
        G1 = g
        for j in range(2, L + 1):
            u = orig_cd(N, t, j - 1, parity)
            A = z * eye - Hs[j - 1] - u[:, None] * g * u[None, :]
            if j == L:
                A = A - sig_r
            g = np.linalg.inv(A)
            G1 = G1 @ g
        calls["n"] += 1
        return np.real(np.trace(R._gamma(sig_l) @ G1 @ R._gamma(sig_r) @ G1.conj().T))
    monkeypatch.setattr(R, "transmission", tr)
    monkeypatch.setattr(O, "transmission", tr)
    del orig_tr


MUTATIONS = {
    "dropped transverse bond": _mut_dropped_bond,
    "flipped bond parity": _mut_parity,
    "Gamma without the factor i": _mut_gamma_missing_i,
    "wrong sign of the Dyson term": _mut_dyson_sign,
    "missing Sigma_R": _mut_missing_sigma_r,
    "advanced lead Green's function": _mut_advanced_lead,
    "gradient off by a factor": _mut_grad_factor,
    "G_1i update without the hopping block": _mut_g1_without_coupling,
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_reject_mutation(monkeypatch, name):
    MUTATIONS[name](monkeypatch)
    try:
        passed = _battery()
    except (AssertionError, ArithmeticError, np.linalg.LinAlgError, ValueError):
        passed = False
    assert not passed, f"the pins did not notice: {name}"
