"""Pins of the CPU oracle against what the physics and mathematics fix.

None of these re-types the oracle's own formulas: each compares the oracle
with an independent route (the brute-force definition of Eq. (1)-(2), closed
forms of the pristine armchair ribbon, band counting, a 1D scattering
formula, finite differences, exact symmetries of a bipartite lattice).
"""

import numpy as np
import pytest

import oracle as O
import rgf_workloads as W

T = W.T_HOP
ETA = W.ETA


# ---------------------------------------------------------------- helpers

def _unit_cell_bloch(N, t, parity, theta):
    """Bloch Hamiltonian of the two-slice lead cell, built from the model
    definition (zigzag-chain slices, alternating longitudinal bonds)."""
    H0 = np.diag(np.full(N - 1, t), 1) + np.diag(np.full(N - 1, t), -1)
    k = np.arange(N)
    U0 = np.diag(np.where((k + parity) % 2 == 0, t, 0.0))
    U1 = np.diag(np.where((k + 1 + parity) % 2 == 0, t, 0.0))
    Z = np.zeros((N, N))
    h00 = np.block([[H0, U0], [U0.T, H0]])
    h01 = np.block([[Z, Z], [U1, Z]])          # slice 1 -> slice 0 of next cell
    return h00 + h01 * np.exp(1j * theta) + h01.T * np.exp(-1j * theta)


def _bands(N, t, parity, n_theta):
    th = np.linspace(-np.pi, np.pi, n_theta, endpoint=False)
    return np.array([np.linalg.eigvalsh(_unit_cell_bloch(N, t, parity, x)) for x in th])


def _ssh_surface_g(z, e, t):
    """Closed-form surface Green's function of the semi-infinite chain
    s0 -e- s1 -t- s2 -e- s3 ... (zero on-site): g = 1/(z - e^2/(z - t^2 g)).
    Of the two roots the retarded one has the decaying Bloch factor
    |lambda| = |e t g g'| < 1 with g' = 1/(z - t^2 g)."""
    if e == 0.0:
        return 1.0 / z          # the surface site is cut off from the chain
    a = z * t * t
    b = -(z * z + t * t - e * e)
    c = z
    disc = np.sqrt(b * b - 4 * a * c + 0j)
    roots = [(-b + disc) / (2 * a), (-b - disc) / (2 * a)]
    best = None
    for g in roots:
        gp = 1.0 / (z - t * t * g)
        lam = abs(e * t * g * gp)
        if best is None or lam < best[0]:
            best = (lam, g)
    return best[1]


def _sigma_closed_form(N, t, eta, E, interface_even):
    """t^2 * sum over transverse modes of phi_p phi_p^T * weight * g_p on the
    interface rows (k of one parity), from the mode decomposition of the
    pristine lead; weight 2 for the mode pairs (p, N+1-p), 1 for the
    self-paired middle mode of odd N."""
    z = complex(E, eta)
    ks = np.arange(0 if interface_even else 1, N, 2)
    P = (N + 1) // 2
    S = np.zeros((len(ks), len(ks)), dtype=complex)
    for p in range(1, P + 1):
        phi = np.sqrt(2.0 / (N + 1)) * np.sin(p * np.pi * (ks + 1) / (N + 1))
        e = 0.0 if (N % 2 == 1 and p == P) else 2 * t * np.cos(p * np.pi / (N + 1))
        w = 1.0 if (N % 2 == 1 and p == P) else 2.0
        S += t * t * w * _ssh_surface_g(z, e, t) * np.outer(phi, phi)
    return ks, S


# ---------------------------------------------------------------- recursion vs definition

@pytest.mark.parametrize("seed", range(40))
def test_rgf_equals_bruteforce(seed):
    """Eqs. (4)-(5) reproduce Eq. (1)+(2) computed by a dense inverse."""
    N, L, parity, t, eps, E = W.random_case(seed)
    a = O.transmission(N, L, t, ETA, E, eps, parity)
    b = O.transmission_bf(N, L, t, ETA, E, eps, parity)
    assert abs(a - b) <= 1e-9 * max(1.0, abs(b))


@pytest.mark.parametrize("seed", range(20))
def test_t_lr_equals_t_rl(seed):
    N, L, parity, t, eps, E = W.random_case(100 + seed)
    a = O.transmission(N, L, t, ETA, E, eps, parity)
    b = O.transmission_rl(N, L, t, ETA, E, eps, parity)
    assert abs(a - b) <= 1e-10 * max(1.0, abs(a))


@pytest.mark.parametrize("seed", range(20))
def test_bounds_zero_to_channels(seed):
    N, L, parity, t, eps, E = W.random_case(200 + seed)
    a = O.transmission(N, L, t, ETA, E, eps, parity)
    assert -1e-12 <= a <= O.open_channels(N, E, t) + 1e-9


@pytest.mark.parametrize("seed", range(10))
def test_hopping_sign_symmetry(seed):
    """Bipartite lattice: flipping the sign of t is a gauge change."""
    N, L, parity, t, eps, E = W.random_case(300 + seed)
    a = O.transmission(N, L, t, ETA, E, eps, parity)
    b = O.transmission(N, L, -t, ETA, E, eps, parity)
    assert abs(a - b) <= 1e-12 * max(1.0, abs(a))


@pytest.mark.parametrize("seed", range(10))
def test_particle_hole_symmetry(seed):
    """Sublattice sign flip maps H -> -H: T(E; eps) = T(-E; -eps)."""
    N, L, parity, t, eps, E = W.random_case(400 + seed)
    a = O.transmission(N, L, t, ETA, E, eps, parity)
    b = O.transmission(N, L, t, ETA, -E, -eps, parity)
    assert abs(a - b) <= 1e-11 * max(1.0, abs(a))


# ---------------------------------------------------------------- closed forms

def test_pristine_quantised_config1():
    """Pristine ribbon: T(E) equals the number of open subbands M(E); the
    deviation is the absorption of eta over the length (bound ~ L*eta)."""
    N, L = 20, 50
    Es = W.energies("pristine_n20")
    Ts = O.transmission_sweep(N, L, T, ETA, Es)
    Ms = np.array([O.open_channels(N, E, T) for E in Es])
    assert np.abs(Ts - Ms).max() <= 1e-4
    assert set(Ms.tolist()) >= {1, 3, 10}


def test_pristine_quantised_small_eta():
    N, L = 20, 50
    Es = W.energies("pristine_n20")[::7]
    Ts = O.transmission_sweep(N, L, T, 1e-10, Es)
    Ms = np.array([O.open_channels(N, E, T) for E in Es])
    assert np.abs(Ts - Ms).max() <= 1e-6


def _propagating_count(N, t, parity, E):
    """Right-moving Bloch states of the two-slice lead cell at real energy E:
    half the number of unimodular solutions lambda of the quadratic
    eigenproblem (E - h00 - lambda h01 - h01^T / lambda) psi = 0."""
    import scipy.linalg as sla
    H0 = np.diag(np.full(N - 1, t), 1) + np.diag(np.full(N - 1, t), -1)
    k = np.arange(N)
    U0 = np.diag(np.where((k + parity) % 2 == 0, t, 0.0))
    U1 = np.diag(np.where((k + 1 + parity) % 2 == 0, t, 0.0))
    Z = np.zeros((N, N))
    h00 = np.block([[H0, U0], [U0.T, H0]])
    h01 = np.block([[Z, Z], [U1, Z]])
    n = 2 * N
    I = np.eye(n)
    A = np.block([[np.zeros((n, n)), I], [-h01.T, E * I - h00]])
    B = np.block([[I, np.zeros((n, n))], [np.zeros((n, n)), h01]])
    lam = sla.eig(A, B, right=False)
    lam = lam[np.isfinite(lam)]
    unimodular = np.sum(np.abs(np.abs(lam) - 1.0) < 1e-7)
    assert unimodular % 2 == 0
    return unimodular // 2


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 20, 21])
def test_open_channels_vs_bloch_states(N):
    """M(E) closed form == number of right-moving Bloch states of the lead."""
    p = np.arange(1, N // 2 + 1)
    c = np.cos(p * np.pi / (N + 1))
    edges = np.concatenate([np.abs(1 - 2 * c), 1 + 2 * c, [1.0]]) * abs(T)
    checked = 0
    for x in np.linspace(0.013, 2.95, 37):
        E = x * abs(T)
        if np.min(np.abs(np.abs(E) - edges)) < 0.02 * abs(T):
            continue
        assert O.open_channels(N, E, T) == _propagating_count(N, T, N % 2, E), (N, x)
        checked += 1
    assert checked >= 5


@pytest.mark.parametrize("N", [20, 60, 120, 240, 61, 62])
def test_half_gap_vs_bands(N):
    bands = _bands(N, T, 0, 2)          # theta = -pi and 0: band extrema
    emin = np.min(np.abs(bands))
    assert abs(emin - O.half_gap(N, T)) <= 1e-9


def test_half_gap_values():
    g = [O.half_gap(N, T) / abs(T) for N in (60, 120, 240, 480)]
    assert np.allclose(g, [0.02959, 0.01495, 0.007517, 0.003769], atol=2e-5)
    assert O.half_gap(20, T) < 1e-12        # N = 2 mod 3: metallic


SIGMA_CASES = [
    (4, 0, 3, 0.37), (5, 0, 3, 0.41), (5, 1, 4, -0.22), (6, 1, 2, 0.8),
    (7, 0, 4, 1.3), (8, 0, 5, -0.05), (11, 1, 3, 0.6), (20, 0, 50, 0.33),
    (20, 0, 50, 1.0), (20, 1, 7, -1.0),            # commensurate Bloch phase (cos = 1/2 mode)
    (60, 0, 7, -0.83), (60, 1, 8, 0.91), (61, 0, 5, 0.013),
]


def _check_sigma(N, parity, L, E, method, tol):
    E = E * abs(T)
    sl, sr = O.lead_self_energies(N, L, T, ETA, E, parity, method=method)
    # Sigma_L lives on rows of slice 1 with (k + parity) even
    ks, S = _sigma_closed_form(N, T, ETA, E, interface_even=(parity % 2 == 0))
    assert np.abs(sl[np.ix_(ks, ks)] - S).max() <= tol * np.abs(S).max()
    off = sl.copy()
    off[np.ix_(ks, ks)] = 0
    assert np.abs(off).max() == 0.0
    # Sigma_R lives on rows of slice L with (k + L + parity) even
    ks, S = _sigma_closed_form(N, T, ETA, E, interface_even=((L + parity) % 2 == 0))
    assert np.abs(sr[np.ix_(ks, ks)] - S).max() <= tol * np.abs(S).max()


@pytest.mark.parametrize("N,parity,L,E", SIGMA_CASES)
def test_sigma_matches_mode_closed_form(N, parity, L, E):
    """Lead self-energies (Bloch-mode eigenproblem) == closed-form surface
    Green's functions of the decoupled transverse-mode chains, assembled on
    the interface rows."""
    _check_sigma(N, parity, L, E, "modes", 1e-12)


def test_sigma_wide_lead_closed_form():
    _check_sigma(240, 0, 2000, -0.2, "modes", 1e-12)


@pytest.mark.parametrize("N,parity,L,E", [c for c in SIGMA_CASES if c[0] <= 20 and abs(c[3]) != 1.0])
def test_sigma_decimation_route_closed_form(N, parity, L, E):
    """The Sancho-Rubio route agrees on narrow leads away from commensurate
    Bloch phases (it loses digits on wide leads)."""
    _check_sigma(N, parity, L, E, "decimation", 1e-10)


@pytest.mark.parametrize("E", [0.1, 0.5, 1.7])
def test_surface_gf_fixed_point_and_sign(E):
    N, L = 8, 4
    sl, sr, info = O.lead_self_energies(N, L, T, ETA, E * abs(T), 0, return_info=True)
    z = complex(E * abs(T), ETA)
    for g, (h00, h01) in zip(info["g_surf"], info["cells"]):
        rhs = np.linalg.inv(z * np.eye(2 * N) - h00 - h01 @ g @ h01.T)
        assert np.abs(g - rhs).max() <= 1e-10 * np.abs(g).max()
    for s in (sl, sr):
        gam = 1j * (s - s.conj().T)
        assert np.linalg.eigvalsh(gam).min() >= -1e-12


@pytest.mark.parametrize("eps0,E", [(0.5, 0.3), (1.2, -1.1), (-0.8, 1.9)])
def test_chain_single_impurity(eps0, E):
    """N = 2 is a uniform 1D chain; one impurity eps0 gives
    T = (4t^2 - E^2) / (4t^2 - E^2 + eps0^2)."""
    L = 6
    eps = np.zeros((L, 2))
    eps[2, 1] = eps0 * abs(T)
    Ee = E * abs(T)
    got = O.transmission(2, L, T, 1e-12, Ee, eps, 0)
    want = (4 * T * T - Ee * Ee) / (4 * T * T - Ee * Ee + (eps0 * abs(T)) ** 2)
    assert abs(got - want) <= 1e-8
    assert abs(O.transmission(2, L, T, 1e-12, Ee, None, 0) - 1.0) <= 1e-8


def test_in_gap_decay_rate():
    """Inside the gap T(L) ~ exp(-2 kappa L), with kappa the slowest decay of
    the evanescent lead modes: for the mode chain with hoppings t and
    e = 2t cos(p pi/(N+1)), E^2 = t^2 (1 + 4c^2 - 4c cosh(kappa))."""
    N = 60
    E = 0.5 * O.half_gap(N, T)
    t80 = O.transmission(N, 80, T, ETA, E)
    t160 = O.transmission(N, 160, T, ETA, E)
    slope = np.log(t160 / t80) / 80
    p = np.arange(1, N // 2 + 1)
    c = np.cos(p * np.pi / (N + 1))
    kappa = np.arccosh((1 + 4 * c * c - (E / T) ** 2) / (4 * c)).min()
    assert abs(slope + 2 * kappa) <= 1e-3 * 2 * kappa


# ---------------------------------------------------------------- gradient

@pytest.mark.parametrize("seed", range(4))
def test_gradient_bf_vs_finite_differences(seed):
    N, L, parity, t, eps, E = W.random_case(500 + seed, n_max=6, l_max=4)
    _, d = O.transmission_grad_bf(N, L, t, ETA, E, eps, parity)
    h = 1e-6 * abs(t)
    for (i, k) in [(0, 0), (L - 1, N - 1), (L // 2, N // 2)]:
        ep = eps.copy(); ep[i, k] += h
        em = eps.copy(); em[i, k] -= h
        fd = (O.transmission_bf(N, L, t, ETA, E, ep, parity)
              - O.transmission_bf(N, L, t, ETA, E, em, parity)) / (2 * h)
        assert abs(fd - d[i, k]) <= 1e-6 + 1e-4 * abs(fd)


@pytest.mark.parametrize("seed", range(12))
def test_gradient_recursion_vs_bf(seed):
    N, L, parity, t, eps, E = W.random_case(600 + seed)
    T1, d1 = O.transmission_grad(N, L, t, ETA, E, eps, parity)
    T2, d2 = O.transmission_grad_bf(N, L, t, ETA, E, eps, parity)
    assert abs(T1 - T2) <= 1e-9 * max(1, abs(T2))
    assert np.abs(d1 - d2).max() <= 1e-8 * max(1.0, np.abs(d2).max())


def test_gradient_sums_to_energy_derivative():
    """The sum of the gradient over all device sites equals the derivative of
    T under a uniform shift of every device on-site energy."""
    N, L = 6, 4
    eps = W.disorder(L, N, 0.4, r=3)
    E = 0.6 * abs(T)
    _, d = O.transmission_grad(N, L, T, ETA, E, eps)
    h = 1e-6
    tp = O.transmission(N, L, T, ETA, E, eps + h)
    tm = O.transmission(N, L, T, ETA, E, eps - h)
    assert abs(d.sum() - (tp - tm) / (2 * h)) <= 1e-6
