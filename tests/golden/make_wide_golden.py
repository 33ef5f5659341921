"""Write the stored oracle values for ribbons wider than N = 256 under
tests/golden/ (wide_ribbons.txt, large_n480_sampled.txt, wide_grad.txt,
wide_ldos.txt).

The oracle's lead self-energies (the Bloch-mode eigenproblem of the
960-site lead cell) take tens of seconds per energy at N = 480 and its sweep
about five minutes for L = 8000, too slow to run inside
the GPU tests, so these values are written once, by this script, from
oracle/ and the seeded input generators only. Each line names its ribbon,
disorder realization and energy; the disorder is regenerated from the seed
by rgf_workloads.disorder.

Run from the repository root:  python tests/golden/make_wide_golden.py
(about twenty minutes on eight cores); with the argument `grad` or `ldos`
it writes only wide_grad.txt or wide_ldos.txt.
"""

import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))

# (N, L, parity, x = E/|t|, [(w, r), ...]): widths on both sides of the
# register-tile limit (257, 258), odd widths and both parities, the paper's
# widest ribbon (480) with two realizations, and the widest supported (512).
WIDE = [
    (257, 5, 0, -0.31, [(0.5, 257)]),
    (257, 5, 0, 0.45, [(0.5, 257)]),
    (258, 4, 1, 0.024, [(0.5, 258)]),
    (301, 3, 0, -0.2, [(0.3, 301)]),
    (479, 3, 1, 0.3, [(0.5, 479)]),
    (480, 6, 0, -0.21, [(0.5, 480), (0.5, 481)]),
    (480, 6, 0, 0.137, [(0.5, 480), (0.5, 481)]),
    (512, 3, 1, -0.12, [(0.5, 512)]),
]
# sampled energies (indices into the workload's grid) of the full-size
# N = 480, L = 8000 ribbon, realization 0
LARGE_SAMPLES = [100, 700]
# gradients dT/deps of every site: (N, L, parity, x = E/|t|, w, r)
GRAD = [
    (257, 3, 1, 0.41, 0.5, 2570),
    (480, 4, 0, -0.137, 0.5, 4800),
]


def _wide_task(case):
    import oracle as O
    import rgf_workloads as W
    N, L, parity, x, reals = case
    E = x * abs(W.T_HOP)
    sig = O.lead_self_energies(N, L, W.T_HOP, W.ETA, E, parity)
    out = []
    for w, r in reals:
        eps = W.disorder(L, N, w, r=r)
        T = O.transmission(N, L, W.T_HOP, W.ETA, E, eps, parity, sigmas=sig)
        out.append((N, L, parity, w, r, E, T))
    return out


def _large_task(j):
    import oracle as O
    import rgf_workloads as W
    cfg = W.WORKLOADS["large_n480"]
    N, L = cfg["N"][0], cfg["L"]
    E = W.energies("large_n480")[j]
    eps = W.disorder(L, N, cfg["w"], r=0)
    return j, E, O.transmission(N, L, W.T_HOP, W.ETA, E, eps, 0)


# local density of states of every site: (N, L, parity, x = E/|t|, w, r)
LDOS = [
    (257, 3, 0, -0.23, 0.5, 2571),
    (480, 4, 1, 0.18, 0.5, 4801),
]


def _ldos_task(case):
    import oracle as O
    import rgf_workloads as W
    N, L, parity, x, w, r = case
    E = x * abs(W.T_HOP)
    eps = W.disorder(L, N, w, r=r)
    return case, E, O.ldos(N, L, W.T_HOP, W.ETA, E, eps, parity)


def write_ldos(res):
    with open(os.path.join(HERE, "wide_ldos.txt"), "w") as f:
        f.write("# -Im G_ss/pi of every site of ribbons wider than N = 256, t=-2.7 eV,\n")
        f.write("# eta=1e-8 eV; disorder rgf_workloads.disorder(L, N, w, r); from\n")
        f.write("# oracle.ldos. A header line per ribbon:\n")
        f.write("# ribbon N L parity w r E_eV, then L*N lines: i k rho_ik (1/eV)\n")
        for (N, L, parity, x, w, r), E, rho in res:
            f.write(f"ribbon {N} {L} {parity} {w} {r} {E:.17e}\n")
            for i in range(L):
                for k in range(N):
                    f.write(f"{i} {k} {rho[i, k]:.17e}\n")


def _grad_task(case):
    import oracle as O
    import rgf_workloads as W
    N, L, parity, x, w, r = case
    E = x * abs(W.T_HOP)
    eps = W.disorder(L, N, w, r=r)
    T, g = O.transmission_grad(N, L, W.T_HOP, W.ETA, E, eps, parity)
    return case, E, T, g


def write_grad(res):
    with open(os.path.join(HERE, "wide_grad.txt"), "w") as f:
        f.write("# dT/deps of every site of ribbons wider than N = 256, t=-2.7 eV,\n")
        f.write("# eta=1e-8 eV; disorder rgf_workloads.disorder(L, N, w, r); from\n")
        f.write("# oracle.transmission_grad. A header line per ribbon:\n")
        f.write("# ribbon N L parity w r E_eV T_oracle, then L*N lines: i k dT/deps_ik\n")
        for (N, L, parity, x, w, r), E, T, g in res:
            f.write(f"ribbon {N} {L} {parity} {w} {r} {E:.17e} {T:.17e}\n")
            for i in range(L):
                for k in range(N):
                    f.write(f"{i} {k} {g[i, k]:.17e}\n")


def main():
    if sys.argv[1:] in (["grad"], ["ldos"]):   # one file only
        os.environ["OMP_NUM_THREADS"] = "4"
        sys.path.insert(0, ROOT)
        ctx = mp.get_context("spawn")
        with ctx.Pool(2, initializer=sys.path.insert, initargs=(0, ROOT)) as pool:
            if sys.argv[1] == "grad":
                write_grad(pool.map(_grad_task, GRAD))
            else:
                write_ldos(pool.map(_ldos_task, LDOS))
        return
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    os.environ["MKL_NUM_THREADS"] = "1"
    sys.path.insert(0, ROOT)
    ctx = mp.get_context("spawn")
    with ctx.Pool(8, initializer=sys.path.insert, initargs=(0, ROOT)) as pool:
        large = pool.map_async(_large_task, LARGE_SAMPLES)
        grad = pool.map_async(_grad_task, GRAD)
        ldos = pool.map_async(_ldos_task, LDOS)
        wide = pool.map(_wide_task, WIDE)
        large = large.get()
        write_grad(grad.get())
        write_ldos(ldos.get())
        pool.close()
        pool.join()
    with open(os.path.join(HERE, "wide_ribbons.txt"), "w") as f:
        f.write("# ribbons wider than N = 256, t=-2.7 eV, eta=1e-8 eV; disorder\n")
        f.write("# rgf_workloads.disorder(L, N, w, r); T from oracle.transmission\n")
        f.write("# columns: N L parity w r E_eV T_oracle(2e^2/h)\n")
        for rows in wide:
            for N, L, parity, w, r, E, T in rows:
                f.write(f"{N} {L} {parity} {w} {r} {E:.17e} {T:.17e}\n")
    with open(os.path.join(HERE, "large_n480_sampled.txt"), "w") as f:
        f.write("# N=480 L=8000 parity 0, disorder U[-0.5,0.5]|t| realization 0,\n")
        f.write("# energies rgf_workloads.energies('large_n480')[j]; T from oracle.transmission\n")
        f.write("# columns: j E_eV T_oracle(2e^2/h)\n")
        for j, E, T in large:
            f.write(f"{j} {E:.17e} {T:.17e}\n")


if __name__ == "__main__":
    main()
