"""Write tests/golden/near_zero.txt: the oracle's conductance of pristine
ribbons wider than N = 256 at and near E = 0, where the GPU's half-slice
recursion hands the tuple to its whole-slice form.

The oracle's lead self-energies (the Bloch-mode eigenproblem of the
two-slice lead cell) take tens of seconds per energy at these widths, too
slow to run inside the GPU tests, so the values are written once, by this
script, from oracle/ only.

Run from the repository root:  python tests/golden/make_near_zero_golden.py
"""

import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))

# (N, L, parity, E_eV): pristine ribbons, t = -2.7 eV, eta = 1e-8 eV.
# 480 and 301 are semiconducting (E = 0 in the gap); 482 = 2 (mod 3) is
# metallic (one open channel at E = 0).
CASES = [
    (480, 4, 0, 0.0),
    (480, 5, 1, 0.0),
    (480, 4, 0, 1e-6),
    (301, 3, 0, 0.0),
    (482, 4, 0, 1e-6),
    (482, 3, 1, 1e-5),
]


def _task(case):
    import oracle as O
    N, L, parity, E = case
    return case, O.transmission(N, L, -2.7, 1e-8, E, None, parity)


def main():
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    sys.path.insert(0, ROOT)
    ctx = mp.get_context("spawn")
    with ctx.Pool(6, initializer=sys.path.insert, initargs=(0, ROOT)) as pool:
        res = pool.map(_task, CASES)
    with open(os.path.join(HERE, "near_zero.txt"), "w") as f:
        f.write("# pristine ribbons near E = 0, t=-2.7 eV, eta=1e-8 eV; T from\n")
        f.write("# oracle.transmission (whole-slice recursion, eigenproblem leads)\n")
        f.write("# columns: N L parity E_eV T_oracle(2e^2/h)\n")
        for (N, L, parity, E), T in res:
            f.write(f"{N} {L} {parity} {E:.17e} {T:.17e}\n")


if __name__ == "__main__":
    main()
