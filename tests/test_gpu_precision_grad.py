"""GPU tests of the precision modes and of the adjoint (gradient) sweep.

Bars (units of 2e^2/h): mixed precision (FP32 inversion + FP64 Newton
refinement per half-slice, FP64 fallback) 1e-8 against FP64 on small and
medium ribbons and the target's 1e-6 at full size; gradients against the
oracle's forward-backward recursion to 1e-8 relative on small ribbons and
1e-7 at the N=120, L=500 workload, and against central finite differences
(h = 1e-6|t|) on 100 sites: at least 90 within 1e-6 + 1e-3 relative plus
twice the measured truncation estimate |D(2h) - D(h)|/3, all within 5e-2
relative (the forward sweep's own rounding, about 1e-9 near subband edges,
is amplified by 1/h in the differences).
"""

import os
import sys

import numpy as np
import pytest

import oracle as O
import rgf_workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1107_5300_amd as P
    P.version()
    return P


def _t(x):
    import torch
    return torch.tensor(np.asarray(x, dtype=np.float64), device="cuda")


def _T(P, N, L, parity, t, Es, eps, precision="fp64"):
    import torch
    T, st = P.conductance(P.Ribbon(N, L, parity, t, W.ETA), _t(Es),
                          None if eps is None else _t(eps), precision=precision,
                          return_status=True)
    torch.cuda.synchronize()
    return T.cpu().numpy(), st.cpu().numpy()


# ------------------------------------------------------------------ precision

@pytest.mark.parametrize("seed", range(16))
def test_mixed_small_ribbons(P, seed):
    N, L, parity, t, eps, E = W.random_case(8100 + seed, n_max=24, l_max=12)
    _say("mixed small", seed, N, L)
    Es = [E, 0.33 * abs(t), -0.71 * abs(t)]
    got, st = _T(P, N, L, parity, t, Es, eps[None], "mixed")
    assert (st == 0).all()
    for j, Ej in enumerate(Es):
        want = O.transmission(N, L, t, W.ETA, Ej, eps, parity)
        assert abs(got[0, j] - want) <= 1e-8 * max(1.0, abs(want)), (j, got[0, j], want)


@pytest.mark.parametrize("N", [20, 61, 120, 240])
def test_mixed_widths(P, N):
    """Mixed precision across the register tilings, against the oracle."""
    L = 11
    _say("mixed width", N)
    eps = W.disorder(L, N, 0.5, r=2)
    Es = np.array([-0.4, 0.02, 0.3]) * abs(W.T_HOP)
    a, st = _T(P, N, L, 0, W.T_HOP, Es, eps[None], "mixed")
    assert (st == 0).all()
    for j, E in enumerate(Es):
        want = O.transmission(N, L, W.T_HOP, W.ETA, E, eps, 0)
        assert abs(a[0, j] - want) <= 1e-8 * max(1.0, abs(want)), (E, a[0, j], want)


def test_single_precision_study_n240(P):
    """Full-size N=240, L=2000 ribbon: plain FP32 inversions miss the FP64
    result by more than 1e-6 near the charge-neutrality point (the paper's
    single-precision finding); FP32 with FP64 refinement stays within 1e-6."""
    N, L = 240, 2000
    _say("precision study", N, L)
    Es = W.energies("disorder_n240")[96:160]       # |E| <= 0.125|t| around the CNP
    eps = W.disorder(L, N, 0.5, r=0)
    f64, s64 = _T(P, N, L, 0, W.T_HOP, Es, eps[None], "fp64")
    mix, smx = _T(P, N, L, 0, W.T_HOP, Es, eps[None], "mixed")
    f32, s32 = _T(P, N, L, 0, W.T_HOP, Es, eps[None], "fp32")
    assert (s64 == 0).all() and (smx == 0).all()
    d_mix = np.abs(mix - f64).max()
    d_32 = np.nanmax(np.abs(f32 - f64))
    _say("  max|dT| mixed", d_mix, "plain fp32", d_32)
    assert d_mix <= 1e-6
    assert d_32 > 1e-6


def test_n240_fp64_and_mixed_vs_stored_oracle(P):
    """The full N = 240, L = 2000 workload ribbon at eight stored oracle
    energies (tests/golden/make_n240_golden.py), four of them within
    0.05 |t| of the charge-neutrality point: FP64 and mixed precision both
    within 1e-9 (the target's bar is 1e-6)."""
    N, L = 240, 2000
    rows = np.loadtxt(os.path.join(HERE, "golden", "n240_sampled.txt"))
    Es = W.energies("disorder_n240")
    idx = rows[:, 0].astype(int)
    assert np.array_equal(rows[:, 1], Es[idx])
    assert (np.abs(rows[:, 1]) < 0.05 * abs(W.T_HOP)).sum() >= 4
    eps = W.disorder(L, N, 0.5, r=0)
    for prec in ("fp64", "mixed"):
        _say("n240 stored oracle", prec)
        got, st = _T(P, N, L, 0, W.T_HOP, rows[:, 1], eps[None], prec)
        assert (st == 0).all()
        d = np.abs(got[0] - rows[:, 2])
        _say("  max |dT|", d.max())
        assert d.max() <= 1e-9, (prec, d)


# ------------------------------------------------------------------ gradients

def _grad(P, N, L, parity, t, Es, eps, w, precision="fp64", stride=0):
    import torch
    T, g, st = P.grad(P.Ribbon(N, L, parity, t, W.ETA), _t(Es), _t(eps), _t(w),
                      precision=precision, ckpt_stride=stride, return_status=True)
    torch.cuda.synchronize()
    return T.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("seed", range(20))
def test_grad_small_vs_oracle(P, seed):
    N, L, parity, t, eps, E = W.random_case(9100 + seed, n_max=14, l_max=9)
    _say("grad small", seed, N, L, parity)
    rng = np.random.default_rng(seed)
    Es = np.array([E, 0.41 * abs(t), -0.13 * abs(t)])
    w = rng.normal(size=(1, len(Es)))
    T, g, st = _grad(P, N, L, parity, t, Es, eps[None], w)
    assert (st == 0).all()
    want = np.zeros((L, N))
    for j, Ej in enumerate(Es):
        Tj, dj = O.transmission_grad(N, L, t, W.ETA, Ej, eps, parity)
        assert abs(T[0, j] - Tj) <= 1e-9 * max(1.0, abs(Tj))
        want += w[0, j] * dj
    scale = max(1.0, np.abs(want).max())
    assert np.abs(g[0] - want).max() <= 1e-8 * scale


def test_grad_checkpoint_strides_agree(P):
    N, L = 16, 13
    _say("grad strides", N, L)
    eps = W.disorder_batch(L, N, 0.4, 2)
    Es = np.linspace(-0.6, 0.6, 5) * abs(W.T_HOP)
    w = np.random.default_rng(1).normal(size=(2, len(Es)))
    ref = _grad(P, N, L, 0, W.T_HOP, Es, eps, w, stride=2 * L)[1]
    for s in (1, 2, 3, 7, 0):
        g = _grad(P, N, L, 0, W.T_HOP, Es, eps, w, stride=s)[1]
        assert np.abs(g - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max()), s


@pytest.mark.parametrize("N", [61, 120, 240])
def test_grad_widths_vs_oracle(P, N):
    L = 5
    _say("grad width", N)
    eps = W.disorder(L, N, 0.3, r=N)
    Es = np.array([-0.27, 0.35]) * abs(W.T_HOP)
    w = np.array([[0.7, -1.3]])
    T, g, st = _grad(P, N, L, N % 2, W.T_HOP, Es, eps[None], w)
    want = np.zeros((L, N))
    for j, E in enumerate(Es):
        want += w[0, j] * O.transmission_grad(N, L, W.T_HOP, W.ETA, E, eps, N % 2)[1]
    assert np.abs(g[0] - want).max() <= 1e-8 * max(1.0, np.abs(want).max())


@pytest.mark.parametrize("seed", range(6))
def test_grad_mixed_small_vs_oracle(P, seed):
    """Mixed-precision gradient of random small ribbons against the oracle's
    exact gradient (1e-8 relative, as for FP64)."""
    N, L, parity, t, eps, E = W.random_case(9300 + seed, n_max=24, l_max=12)
    _say("grad mixed small", seed, N, L, parity)
    Es = np.array([E, 0.27 * abs(t), -0.52 * abs(t)])
    w = np.random.default_rng(seed).normal(size=(1, len(Es)))
    T, g, st = _grad(P, N, L, parity, t, Es, eps[None], w, "mixed")
    assert (st == 0).all()
    want = np.zeros((L, N))
    for j, Ej in enumerate(Es):
        Tj, dj = O.transmission_grad(N, L, t, W.ETA, Ej, eps, parity)
        assert abs(T[0, j] - Tj) <= 1e-9 * max(1.0, abs(Tj))
        want += w[0, j] * dj
    assert np.abs(g[0] - want).max() <= 1e-8 * max(1.0, np.abs(want).max())


def test_grad_mixed_precision(P):
    """N = 40, L = 30: the mixed gradient against the oracle's."""
    N, L = 40, 30
    _say("grad mixed", N, L)
    eps = W.disorder(L, N, 0.3, r=5)
    Es = np.linspace(-0.4, 0.4, 6) * abs(W.T_HOP)
    w = np.ones((1, len(Es)))
    gmx = _grad(P, N, L, 0, W.T_HOP, Es, eps[None], w, "mixed")[1]
    want = sum(O.transmission_grad(N, L, W.T_HOP, W.ETA, E, eps, 0)[1] for E in Es)
    assert np.abs(gmx[0] - want).max() <= 1e-8 * max(1.0, np.abs(want).max())


def test_grad_zero_weights_and_skip(P):
    N, L = 10, 6
    eps = W.disorder(L, N, 0.3, r=7)
    Es = np.array([0.2, 0.5]) * abs(W.T_HOP)
    T, g, st = _grad(P, N, L, 0, W.T_HOP, Es, eps[None], np.zeros((1, 2)))
    assert np.abs(g).max() == 0.0
    T2, _ = _T(P, N, L, 0, W.T_HOP, Es, eps[None])
    assert np.abs(T - T2).max() <= 1e-12


def test_autograd_function(P):
    import torch
    N, L = 12, 8
    _say("autograd")
    eps = _t(W.disorder(L, N, 0.4, r=9)).requires_grad_(True)
    E = _t(np.array([0.1, 0.45, -0.3]) * abs(W.T_HOP))
    rib = P.Ribbon(N, L, 0, W.T_HOP, W.ETA)
    T = P.RGFConductance.apply(eps, E, rib, "fp64")
    (T * torch.tensor([[1.0, 2.0, -0.5]], device="cuda", dtype=torch.float64)).sum().backward()
    _, g = P.grad(rib, E, eps.detach(), _t([[1.0, 2.0, -0.5]]))
    assert torch.allclose(eps.grad, g[0], rtol=0, atol=1e-13)


def _fd_golden():
    rows = np.loadtxt(os.path.join(HERE, "golden", "fd_adjoint_n120.txt"))
    out = {}
    for j, E, i, k, d in rows:
        out.setdefault(int(j), (E, []))[1].append((int(i), int(k), d))
    return out


def test_grad_adjoint_n120_vs_oracle_and_fd(P):
    """The adjoint workload (N=120, L=500, U[-0.3,0.3]|t|, 128 energies):
    the gradient of single energies against the oracle's exact forward-
    backward gradient on every site, and against the oracle's central
    differences (h = 1e-6|t|, tests/golden/make_fd_golden.py) on the 100
    seeded sites, held to 1e-6 + 1e-4 |fd| on every site (the oracle's FP64
    rounding contributes ~4e-8 to a difference quotient)."""
    N, L = 120, 500
    _say("adjoint_n120", N, L)
    Es = W.energies("adjoint_n120")
    eps = W.disorder(L, N, 0.3, r=0)
    for j in (17, 70):
        Tj, dj = O.transmission_grad(N, L, W.T_HOP, W.ETA, Es[j], eps, 0)
        wj = np.zeros((1, len(Es)))
        wj[0, j] = 1.0
        Tg, gj, _ = _grad(P, N, L, 0, W.T_HOP, Es, eps[None], wj)
        rel = np.abs(gj[0] - dj).max() / max(1.0, np.abs(dj).max())
        _say("  oracle gradient, energy", j, "max rel err", rel)
        assert abs(Tg[0, j] - Tj) <= 1e-9
        assert rel <= 1e-7
    fd = _fd_golden()
    assert sorted(fd) == [17, 70, 101]
    sites = W.fd_sites(L, N, 100, seed=4)
    for j, (E, rows) in sorted(fd.items()):
        assert abs(E - Es[j]) <= 1e-15 * abs(E)
        assert [(i, k) for i, k, _ in rows] == [tuple(s) for s in sites]
        wj = np.zeros((1, len(Es)))
        wj[0, j] = 1.0
        _, g, st = _grad(P, N, L, 0, W.T_HOP, Es, eps[None], wj)
        assert (st == 0).all()
        worst = 0.0
        for i, k, d in rows:
            err = abs(g[0, i, k] - d)
            worst = max(worst, err / (1e-6 + 1e-4 * abs(d)))
            assert err <= 1e-6 + 1e-4 * abs(d), (j, i, k, d, g[0, i, k])
        _say("  energy", j, "100 FD sites, worst ratio to 1e-6 + 1e-4|fd|:", worst)


def test_grad_mixed_adjoint_n120_vs_oracle(P):
    """The mixed-precision gradient of the adjoint workload against the
    oracle's exact gradient on two energies (every site), as for FP64."""
    N, L = 120, 500
    _say("adjoint_n120 mixed", N, L)
    Es = W.energies("adjoint_n120")
    eps = W.disorder(L, N, 0.3, r=0)
    for j in (40, 101):
        Tj, dj = O.transmission_grad(N, L, W.T_HOP, W.ETA, Es[j], eps, 0)
        wj = np.zeros((1, len(Es)))
        wj[0, j] = 1.0
        Tg, gj, st = _grad(P, N, L, 0, W.T_HOP, Es, eps[None], wj, "mixed")
        assert (st == 0).all()
        rel = np.abs(gj[0] - dj).max() / max(1.0, np.abs(dj).max())
        _say("  mixed oracle gradient, energy", j, "max rel err", rel)
        assert abs(Tg[0, j] - Tj) <= 1e-9
        assert rel <= 1e-7


def test_fp64_accuracy_adjoint_workload(P):
    """Forward FP64 accuracy on every energy of the N=120, L=500 workload
    against the oracle (run in parallel on the host)."""
    import multiprocessing as mp
    N, L = 120, 500
    _say("fp64 accuracy adjoint_n120")
    Es = W.energies("adjoint_n120")[::8]
    eps = W.disorder(L, N, 0.3, r=0)
    got, st = _T(P, N, L, 0, W.T_HOP, Es, eps[None])
    assert (st == 0).all()
    # one single-threaded BLAS per worker process (the children read the
    # thread counts from the environment when they start)
    keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in keys}
    os.environ.update({k: "1" for k in keys})
    try:
        nproc = max(1, min(16, len(Es), len(os.sched_getaffinity(0))))
        with mp.get_context("spawn").Pool(nproc) as pool:
            want = pool.starmap(O.transmission, [(N, L, W.T_HOP, W.ETA, float(E), eps, 0)
                                                 for E in Es])
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    d = np.abs(got[0] - np.array(want))
    _say("  max |dT|", d.max(), "at E/|t| =", Es[int(np.argmax(d))] / abs(W.T_HOP))
    assert d.max() <= 1e-8
