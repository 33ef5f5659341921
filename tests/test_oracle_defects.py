"""Oracle pins for lattice defects (vacancies and edge roughness).

A vacancy is a site with on-site energy +inf: the atom is removed. The
oracle's recursion decouples such sites; these tests pin it to things
outside itself: the brute-force inverse with the sites deleted from the
matrix, the large-but-finite on-site energy limit, the left-to-right /
right-to-left symmetry, the transverse mirror of even ribbons, and a
planted mistake that the pins must reject.
"""

import numpy as np
import pytest

import oracle as O
import rgf_workloads as W

T = W.T_HOP
ETA = W.ETA


def _case(seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(3, 11))
    L = int(rng.integers(1, 7))
    parity = int(rng.integers(0, 2))
    w = float(rng.choice([0.0, 0.3, 0.5]))
    eps = W.vacancies(W.disorder(L, N, w, r=seed), float(rng.choice([0.1, 0.25])), seed)
    E = float(rng.uniform(-0.9, 0.9) * abs(T))
    return N, L, parity, eps, E


@pytest.mark.parametrize("seed", range(30))
def test_vacancies_recursion_equals_deleted_brute_force(seed):
    N, L, parity, eps, E = _case(seed)
    sig = O.lead_self_energies(N, L, T, ETA, E, parity)
    a = O.transmission(N, L, T, ETA, E, eps, parity, sigmas=sig)
    b = O.transmission_bf(N, L, T, ETA, E, eps, parity, sigmas=sig)
    assert abs(a - b) <= 1e-10 * max(1.0, abs(b)), (a, b)
    c = O.transmission_rl(N, L, T, ETA, E, eps, parity, sigmas=sig)
    assert abs(a - c) <= 1e-10 * max(1.0, abs(a))
    assert -1e-12 <= a <= O.open_channels(N, E, T) + 1e-9


@pytest.mark.parametrize("seed", range(6))
def test_vacancy_is_the_infinite_onsite_limit(seed):
    """T(eps_s = X) -> T(vacancy) as X grows, with the t^2/X rate of a
    decoupling site."""
    N, L, parity, eps, E = _case(100 + seed)
    if not np.isinf(eps).any():
        eps[0, 0] = np.inf
    base = O.transmission(N, L, T, ETA, E, eps, parity)
    d = [abs(O.transmission(N, L, T, ETA, E, np.where(np.isinf(eps), X, eps), parity) - base)
         for X in (1e6, 1e9)]
    assert d[1] <= 1e-7 * max(1.0, abs(base))
    assert d[1] <= 1e-2 * d[0] + 1e-13


@pytest.mark.parametrize("seed", range(6))
def test_mirror_of_even_ribbon_with_vacancies(seed):
    """For even N the transverse mirror k -> N-1-k maps the bond pattern of
    parity p onto parity 1-p: T is unchanged with the defects mirrored."""
    rng = np.random.default_rng(seed)
    N, L = 2 * int(rng.integers(2, 6)), int(rng.integers(2, 6))
    eps = W.vacancies(W.disorder(L, N, 0.4, r=seed), 0.2, 50 + seed)
    E = float(rng.uniform(-0.8, 0.8) * abs(T))
    a = O.transmission(N, L, T, ETA, E, eps, 0)
    b = O.transmission(N, L, T, ETA, E, eps[:, ::-1].copy(), 1)
    assert abs(a - b) <= 1e-10 * max(1.0, abs(a))


@pytest.mark.parametrize("seed", range(6))
def test_vacancy_gradient_and_ldos_against_deleted_brute_force(seed):
    N, L, parity, eps, E = _case(200 + seed)
    vac = np.isinf(eps)
    Ta, ga = O.transmission_grad(N, L, T, ETA, E, eps, parity)
    Tb, gb = O.transmission_grad_bf(N, L, T, ETA, E, eps, parity)
    assert abs(Ta - Tb) <= 1e-10 * max(1.0, abs(Tb))
    assert np.abs(ga - gb).max() <= 1e-9 * max(1.0, np.abs(gb).max())
    assert (ga[vac] == 0.0).all()
    la = O.ldos(N, L, T, ETA, E, eps, parity)
    lb = O.ldos_bf(N, L, T, ETA, E, eps, parity)
    assert np.abs(la - lb).max() <= 1e-9 * max(1.0, np.abs(lb).max())
    assert (la[vac] == 0.0).all()


def test_edge_roughness_generator_and_fully_vacant_slice():
    """Edge roughness removes only edge atoms; a slice whose atoms are all
    removed cuts the ribbon (T = 0)."""
    eps = W.vacancies(np.zeros((40, 12)), 0.3, 5, rows=(0, 11))
    vac = np.isinf(eps)
    assert vac.any() and not vac[:, 1:11].any()
    cut = np.zeros((4, 6))
    cut[2, :] = np.inf
    assert abs(O.transmission(6, 4, T, ETA, 0.31 * abs(T), cut, 0)) <= 1e-14


def test_planted_mistake_is_rejected(monkeypatch):
    """Leaving the removed site's own Green's-function entry at 1 (instead of
    0) couples it back through its neighbours: the deleted brute force
    tells the difference."""
    good = O.rgf_oracle._slice_inverse

    def wrong(A, vac):
        if vac is None or not vac.any():
            return np.linalg.inv(A)
        idx = np.nonzero(vac)[0]
        A = A.copy()
        A[idx, :] = 0.0
        A[:, idx] = 0.0
        A[idx, idx] = 1.0
        return np.linalg.inv(A)          # missing: g[idx, idx] = 0

    N, L, parity, E = 8, 4, 0, 0.42 * abs(T)
    eps = np.zeros((L, N))
    eps[1, 0] = np.inf                   # row 0 of slice 2 bonds to slice 3
    want = O.transmission_bf(N, L, T, ETA, E, eps, parity)
    assert good is not wrong
    assert abs(O.transmission(N, L, T, ETA, E, eps, parity) - want) <= 1e-10
    monkeypatch.setattr(O.rgf_oracle, "_slice_inverse", wrong)
    assert abs(O.transmission(N, L, T, ETA, E, eps, parity) - want) > 1e-6
