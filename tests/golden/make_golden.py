"""Write the stored oracle values under tests/golden/.

The paper prints no numeric conductance values (its figures are curves), so
these fixtures are regression values of the CPU oracle, written by this
script from oracle/ only. Each file states the workload it covers.

Run from the repository root:  python tests/golden/make_golden.py
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O          # noqa: E402
import rgf_workloads as W   # noqa: E402


def main():
    # pristine N=20, L=50 ribbon, 64 energies: quantised steps (Fig. 3 of the
    # paper describes this step-like G(E) of an ideal ribbon)
    Es = W.energies("pristine_n20")
    Ts = O.transmission_sweep(20, 50, W.T_HOP, W.ETA, Es)
    Ms = [O.open_channels(20, E, W.T_HOP) for E in Es]
    with open(os.path.join(HERE, "pristine_n20.txt"), "w") as f:
        f.write("# pristine armchair ribbon N=20 L=50 t=-2.7 eV eta=1e-8 eV parity=0\n")
        f.write("# columns: E_eV  T_oracle(2e^2/h)  M(E)\n")
        for E, T, M in zip(Es, Ts, Ms):
            f.write(f"{E:.17e} {T:.17e} {M:d}\n")
    # small disordered ribbons (seeded), both parities, odd and even N
    with open(os.path.join(HERE, "small_disorder.txt"), "w") as f:
        f.write("# random_case(seed) ribbons from rgf_workloads, eta=1e-8 eV\n")
        f.write("# columns: seed N L parity t E_eV T_oracle\n")
        for seed in range(1000, 1024):
            N, L, parity, t, eps, E = W.random_case(seed, n_max=24, l_max=30)
            T = O.transmission(N, L, t, W.ETA, E, eps, parity)
            f.write(f"{seed} {N} {L} {parity} {t:.17e} {E:.17e} {T:.17e}\n")


if __name__ == "__main__":
    main()
