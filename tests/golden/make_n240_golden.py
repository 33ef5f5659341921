"""Write tests/golden/n240_sampled.txt: the oracle's conductance of the
N = 240, L = 2000 disordered ribbon (disorder U[-0.5, 0.5]|t|, realization
0) at eight energies of its 256-point grid, four of them within 0.05 |t| of
the charge-neutrality point, where single precision loses accuracy.

Each value is oracle.transmission (whole-slice recursion, eigenproblem
leads), about 15 s per energy on one core; stored once so that the GPU tests
can hold both the FP64 and the mixed-precision sweep to them.

Run from the repository root:  python tests/golden/make_n240_golden.py
"""

import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
# grid indices: 118, 124, 131, 137 have |E| < 0.05 |t|
INDICES = (20, 60, 118, 124, 131, 137, 190, 240)


def _init():
    sys.path.insert(0, ROOT)


def _task(j):
    import oracle as O
    import rgf_workloads as W
    cfg = W.WORKLOADS["disorder_n240"]
    N, L = cfg["N"][0], cfg["L"]
    E = float(W.energies("disorder_n240")[j])
    eps = W.disorder(L, N, cfg["w"], r=0)
    return j, E, O.transmission(N, L, W.T_HOP, W.ETA, E, eps, 0)


def main():
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    with mp.get_context("spawn").Pool(8, initializer=_init) as pool:
        res = pool.map(_task, INDICES)
    with open(os.path.join(HERE, "n240_sampled.txt"), "w") as f:
        f.write("# N=240 L=2000 parity 0, disorder U[-0.5,0.5]|t| realization 0, t=-2.7 eV,\n")
        f.write("# eta=1e-8 eV; energies rgf_workloads.energies('disorder_n240')[j];\n")
        f.write("# T from oracle.transmission. columns: j E_eV T_oracle(2e^2/h)\n")
        for j, E, T in res:
            f.write(f"{j} {E:.17e} {T:.17e}\n")


if __name__ == "__main__":
    main()
