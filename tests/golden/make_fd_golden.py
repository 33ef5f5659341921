"""Write tests/golden/fd_adjoint_n120.txt: central finite differences of the
oracle's conductance with respect to single on-site energies, on the
adjoint workload's ribbon (N = 120, L = 500, disorder U[-0.3, 0.3]|t|,
realization 0) at 100 seeded sites and three energies of its grid.

  fd = (T(eps + h e_s) - T(eps - h e_s)) / (2 h),   h = 1e-6 |t|,

each T from oracle.transmission (the lead self-energies depend only on E and
are computed once per energy). The energies are grid points 17, 70 and 101
(E/|t| = -0.366, 0.051, 0.295), at least 3.9e-3 |t| from every subband edge
of N = 120, where T is smooth in eps. The oracle's own rounding (~1e-13 in T
at this length) contributes ~4e-8 to each difference quotient.

Run from the repository root:  python tests/golden/make_fd_golden.py
(about ten minutes on eight cores).
"""

import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
ENERGY_INDICES = (17, 70, 101)
H_REL = 1e-6


def _init():
    sys.path.insert(0, ROOT)


def _fd_task(args):
    import numpy as np
    import oracle as O
    import rgf_workloads as W
    j, sites = args
    cfg = W.WORKLOADS["adjoint_n120"]
    N, L = cfg["N"][0], cfg["L"]
    E = float(W.energies("adjoint_n120")[j])
    eps = W.disorder(L, N, cfg["w"], r=0)
    h = H_REL * abs(W.T_HOP)
    sig = O.lead_self_energies(N, L, W.T_HOP, W.ETA, E, 0)
    out = []
    for i, k in sites:
        ep = eps.copy()
        ep[i, k] += h
        em = eps.copy()
        em[i, k] -= h
        tp = O.transmission(N, L, W.T_HOP, W.ETA, E, ep, 0, sigmas=sig)
        tm = O.transmission(N, L, W.T_HOP, W.ETA, E, em, 0, sigmas=sig)
        out.append((j, E, int(i), int(k), (tp - tm) / (2 * h)))
    return out


def main():
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    sys.path.insert(0, ROOT)
    import rgf_workloads as W
    cfg = W.WORKLOADS["adjoint_n120"]
    sites = W.fd_sites(cfg["L"], cfg["N"][0], 100, seed=4)
    chunks = [(j, sites[c:c + 10]) for j in ENERGY_INDICES for c in range(0, len(sites), 10)]
    with mp.get_context("spawn").Pool(8, initializer=_init) as pool:
        res = pool.map(_fd_task, chunks)
    with open(os.path.join(HERE, "fd_adjoint_n120.txt"), "w") as f:
        f.write("# central differences of oracle.transmission, h = 1e-6 |t|, on the adjoint\n")
        f.write("# workload ribbon (N=120, L=500, disorder U[-0.3,0.3]|t| realization 0,\n")
        f.write("# t=-2.7 eV, eta=1e-8 eV), sites rgf_workloads.fd_sites(500, 120, 100, 4)\n")
        f.write("# columns: j E_eV i k dT/deps_ik ((2e^2/h)/eV)\n")
        for rows in res:
            for j, E, i, k, d in rows:
                f.write(f"{j} {E:.17e} {i} {k} {d:.17e}\n")


if __name__ == "__main__":
    main()
