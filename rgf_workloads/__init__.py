"""Seeded synthetic inputs for the armchair-ribbon RGF workloads.

This module only draws numbers and lays out grids: it holds none of the
method's arithmetic. The oracle (CPU) and the HIP library consume the same
float64 arrays produced here, so random numbers are drawn exactly once.

Workloads (all with t = -2.7 eV, eta = 1e-8 eV, parity 0):
  pristine_n20     N=20,  L=50,   1 realization (no disorder), 64 energies
                   linspace(-1, 1)|t|
  disorder_n240    N=240, L=2000, 1 realization, U[-0.5, 0.5]|t|, 256 energies
                   linspace(-0.5, 0.5)|t|
  batched_mixed    N in {60, 120, 240}, L=1000, 16 realizations,
                   U[-0.5, 0.5]|t|, 4096 energies: 512 midpoints of
                   (-0.05, 0.05)|t| and 1792 midpoints on each of
                   [-1, -0.05]|t| and [0.05, 1]|t|
  adjoint_n120     N=120, L=500, 1 realization, U[-0.3, 0.3]|t|, 128 energies
                   linspace(-0.5, 0.5)|t|; 100 finite-difference sites
  large_n480       N=480, L=8000, 1 realization, U[-0.5, 0.5]|t|, 1024 energies
                   linspace(-0.3, 0.3)|t|

Disorder of realization r: numpy default_rng(11075300 + r).uniform(-w|t|,
w|t|, size=(L, N)) in float64. An even number of linspace points and the
midpoint grids never hit E = 0 exactly.
"""

import numpy as np

T_HOP = -2.7
ETA = 1e-8
SEED_BASE = 11075300

WORKLOADS = {
    "pristine_n20": dict(N=[20], L=50, n_real=1, w=0.0, n_E=64),
    "disorder_n240": dict(N=[240], L=2000, n_real=1, w=0.5, n_E=256),
    "batched_mixed": dict(N=[60, 120, 240], L=1000, n_real=16, w=0.5, n_E=4096),
    "adjoint_n120": dict(N=[120], L=500, n_real=1, w=0.3, n_E=128),
    "large_n480": dict(N=[480], L=8000, n_real=1, w=0.5, n_E=1024),
}


def midpoints(a, b, n):
    """n midpoints of n equal sub-intervals of [a, b]."""
    h = (b - a) / n
    return a + h * (np.arange(n) + 0.5)


def energies(name, t=T_HOP):
    """Energy grid of a workload, in eV (float64)."""
    at = abs(t)
    if name == "pristine_n20":
        x = np.linspace(-1.0, 1.0, 64)
    elif name == "disorder_n240":
        x = np.linspace(-0.5, 0.5, 256)
    elif name == "batched_mixed":
        x = np.concatenate([
            midpoints(-1.0, -0.05, 1792),
            midpoints(-0.05, 0.05, 512),
            midpoints(0.05, 1.0, 1792),
        ])
    elif name == "adjoint_n120":
        x = np.linspace(-0.5, 0.5, 128)
    elif name == "large_n480":
        x = np.linspace(-0.3, 0.3, 1024)
    else:
        raise KeyError(name)
    return (x * at).astype(np.float64)


def disorder(L, N, w, r=0, t=T_HOP):
    """On-site energies [L, N] of realization r, uniform in [-w|t|, w|t|]."""
    if w == 0.0:
        return np.zeros((L, N), dtype=np.float64)
    rng = np.random.default_rng(SEED_BASE + r)
    return rng.uniform(-w * abs(t), w * abs(t), size=(L, N)).astype(np.float64)


def disorder_batch(L, N, w, n_real, t=T_HOP):
    """[n_real, L, N] stack of disorder realizations 0..n_real-1."""
    return np.stack([disorder(L, N, w, r, t) for r in range(n_real)])


def vacancies(eps, density, seed, rows=None):
    """eps with a seeded random fraction `density` of its sites removed
    (on-site energy +inf, the library's vacancy marker). rows: the
    transverse rows eligible (all if None); rows=(0, N-1) gives edge
    roughness. Returns a new float64 array."""
    eps = np.array(eps, dtype=np.float64, copy=True)
    L, N = eps.shape
    rng = np.random.default_rng(SEED_BASE + 7919 * (seed + 1))
    mask = rng.random((L, N)) < density
    if rows is not None:
        keep = np.zeros(N, dtype=bool)
        keep[list(rows)] = True
        mask &= keep[None, :]
    eps[mask] = np.inf
    return eps


def fd_sites(L, N, count=100, seed=4):
    """Sites (i, k) for finite-difference gradient checks, without replacement."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(L * N, size=count, replace=False)
    return np.stack([flat // N, flat % N], axis=1)


def random_case(seed, n_max=10, l_max=7):
    """A small random ribbon for parity tests: (N, L, parity, t, eps, E)."""
    rng = np.random.default_rng(seed)
    N = int(rng.integers(2, n_max + 1))
    L = int(rng.integers(1, l_max + 1))
    parity = int(rng.integers(0, 2))
    t = T_HOP if rng.random() < 0.5 else -T_HOP
    w = float(rng.choice([0.0, 0.3, 0.5, 1.0]))
    eps = rng.uniform(-w * abs(t), w * abs(t), size=(L, N)) if w > 0 else np.zeros((L, N))
    E = float(rng.uniform(-0.95, 0.95) * abs(t))
    return N, L, parity, t, eps.astype(np.float64), E
