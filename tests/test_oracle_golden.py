"""The oracle reproduces its stored regression values (tests/golden/)."""

import os

import numpy as np

import oracle as O
import rgf_workloads as W

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_pristine_n20_golden():
    d = np.loadtxt(os.path.join(GOLD, "pristine_n20.txt"))
    Ts = O.transmission_sweep(20, 50, W.T_HOP, W.ETA, d[:, 0])
    assert np.abs(Ts - d[:, 1]).max() <= 1e-11
    assert np.abs(d[:, 1] - d[:, 2]).max() <= 1e-4


def test_small_disorder_golden():
    rows = np.loadtxt(os.path.join(GOLD, "small_disorder.txt"))
    for row in rows:
        seed = int(row[0])
        N, L, parity, t, eps, E = W.random_case(seed, n_max=24, l_max=30)
        assert (N, L, parity) == (int(row[1]), int(row[2]), int(row[3]))
        T = O.transmission(N, L, t, W.ETA, E, eps, parity)
        assert abs(T - row[6]) <= 1e-11 * max(1.0, abs(row[6]))
