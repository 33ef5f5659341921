"""GPU parity of the conductance recursion split along the ribbon length
(rgf_conductance_segments): each tuple's slices cut into G segments closed
by the pristine lead self-energy, each solved on its own workgroup (the
left-connected sweep and, from the second segment on, the sweep of the
reversed segment), joined by Dyson's equation.

Against the oracle (1e-9 relative, as for the sequential sweep) on random
small ribbons with every segment count from 1 to L, both parities and odd
widths; against rgf_conductance on every register tiling (1e-9 relative per
tuple: the same quantity by a different order of operations); pristine
ribbons; vacancies; the accuracy guard's whole-slice recomputation near
E = 0; the automatic segment count for small batches; graph capture.
"""

import sys

import numpy as np
import pytest

import oracle as O
import rgf_workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-9


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


def _seg(P, N, L, parity, Es, eps, G, t=W.T_HOP):
    import torch
    T, st, g = P.conductance_segments(P.Ribbon(N, L, parity, t, W.ETA), _t(Es),
                                      None if eps is None else _t(eps), n_segments=G,
                                      return_status=True, return_segments=True)
    torch.cuda.synchronize()
    return T.cpu().numpy(), st.cpu().numpy(), g


def _seq(P, N, L, parity, Es, eps, t=W.T_HOP):
    import torch
    T, st = P.conductance(P.Ribbon(N, L, parity, t, W.ETA), _t(Es),
                          None if eps is None else _t(eps), return_status=True)
    torch.cuda.synchronize()
    return T.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("seed", range(12))
def test_small_ribbons_every_segment_count_vs_oracle(P, seed):
    N, L, parity, t, eps, E = W.random_case(5300 + seed, n_max=12, l_max=7)
    Es = [E, 0.41 * abs(t), -0.23 * abs(t)]
    want = [O.transmission(N, L, t, W.ETA, x, eps, parity) for x in Es]
    for G in range(1, L + 1):
        _say("segments small", seed, N, L, parity, G)
        got, st, g = _seg(P, N, L, parity, Es, eps[None], G, t)
        assert g == G
        assert (st == 0).all(), st
        for j in range(len(Es)):
            assert abs(got[0, j] - want[j]) <= TOL * max(1.0, abs(want[j])), (G, j, got[0, j],
                                                                             want[j])


@pytest.mark.parametrize("N,L,G", [(8, 9, 3), (16, 12, 4), (30, 10, 5), (45, 8, 3), (60, 9, 9),
                                   (90, 7, 2), (120, 8, 4), (200, 6, 3), (240, 8, 8),
                                   (256, 5, 2)])
def test_every_tiling_equals_sequential_sweep(P, N, L, G):
    """Several realizations and energies in one call, both parities: equal
    to rgf_conductance to 1e-9 relative, and to the oracle on one tuple."""
    R = 2
    eps = np.stack([W.disorder(L, N, 0.4, r=70 + r) for r in range(R)])
    Es = np.array([-0.52, -0.07, 0.19, 0.44]) * abs(W.T_HOP)
    for parity in (0, 1):
        _say("segments tiling", N, L, G, parity)
        got, st, g = _seg(P, N, L, parity, Es, eps, G)
        ref, st0 = _seq(P, N, L, parity, Es, eps)
        assert g == G and (st == 0).all() and (st0 == 0).all()
        assert (np.abs(got - ref) <= TOL * np.maximum(1.0, np.abs(ref))).all(), \
            np.abs(got - ref).max()
        want = O.transmission(N, L, W.T_HOP, W.ETA, Es[2], eps[1], parity)
        assert abs(got[1, 2] - want) <= TOL * max(1.0, abs(want))


@pytest.mark.parametrize("N", [20, 21, 60])
def test_pristine_ribbons(P, N):
    """Pristine ribbons, where an isolated segment would have sharp
    resonances: the oracle's T to 1e-9, and within 1e-4 of the number of
    open channels (the broadening eta absorbs a little over 80 slices, most
    near subband edges, where the group velocity is small)."""
    L, G = 80, 8
    Es = np.array([0.05, 0.31, 0.62, -0.44]) * abs(W.T_HOP)
    _say("segments pristine", N)
    got, st, _ = _seg(P, N, L, 0, Es, None, G)
    assert (st == 0).all()
    for j, E in enumerate(Es):
        want = O.transmission(N, L, W.T_HOP, W.ETA, E, None, 0)
        assert abs(got[0, j] - want) <= TOL * max(1.0, want), (E, got[0, j], want)
        assert abs(got[0, j] - O.open_channels(N, E, W.T_HOP)) <= 1e-4


def test_vacancies_in_segments(P):
    """Vacancies, including a fully removed slice at a segment boundary
    (T = 0 exactly) and vacancies at the segment ends."""
    N, L, G = 18, 12, 4
    eps = W.vacancies(W.disorder(L, N, 0.2, r=4), 0.1, 4)
    cut = np.zeros((L, N))
    cut[3, :] = np.inf    # the first slice of segment 1 (slices 0..2 | 3..5 | ...)
    cut2 = np.zeros((L, N))
    cut2[2, [0, 4, 9]] = np.inf
    cut2[3, [1, 5, 17]] = np.inf
    Es = np.array([0.21, -0.38]) * abs(W.T_HOP)
    _say("segments vacancies")
    got, st, _ = _seg(P, N, L, 1, Es, np.stack([eps, cut, cut2]), G)
    assert (st == 0).all(), st
    assert (got[1] == 0.0).all(), got[1]
    for r, e in enumerate((eps, cut, cut2)):
        for j, E in enumerate(Es):
            want = O.transmission(N, L, W.T_HOP, W.ETA, E, e, 1)
            assert abs(got[r, j] - want) <= TOL * max(1.0, abs(want)), (r, E)


def test_near_zero_energy_recomputed(P):
    """Pristine metallic N = 20 near E = 0: the guard sends the tuples to
    the whole-slice sweep; the oracle's value, status OK."""
    N, L, G = 20, 40, 5
    Es = [2e-7, 1e-6, 1e-4, 0.3 * abs(W.T_HOP)]
    _say("segments near zero")
    got, st, _ = _seg(P, N, L, 0, Es, None, G)
    assert (st == 0).all(), st
    for j, E in enumerate(Es):
        want = O.transmission(N, L, W.T_HOP, W.ETA, E, None, 0)
        assert abs(got[0, j] - want) <= TOL * max(1.0, abs(want)), (E, got[0, j], want)


def test_automatic_segment_count_for_small_batches(P):
    """Four tuples of a long N = 120 ribbon: the automatic count splits
    each tuple (G > 1) and the result equals the sequential sweep; a batch
    that fills the GPU by itself gets G = 1."""
    N, L = 120, 300
    eps = W.disorder(L, N, 0.5, r=8)[None]
    Es = np.array([-0.33, -0.02, 0.12, 0.47]) * abs(W.T_HOP)
    _say("segments auto")
    got, st, g = _seg(P, N, L, 0, Es, eps, 0)
    ref, _ = _seq(P, N, L, 0, Es, eps)
    assert g > 1 and (st == 0).all()
    assert (np.abs(got - ref) <= TOL * np.maximum(1.0, np.abs(ref))).all(), np.abs(got - ref).max()
    import torch
    many = torch.tensor(np.linspace(-0.5, 0.5, 2048) * abs(W.T_HOP), device="cuda")
    nb = P.conductance_segments(P.Ribbon(N, 4, 0, W.T_HOP, W.ETA), many, None,
                                return_segments=True)[1]
    assert nb == 1


def test_graph_capture_replays(P):
    """The segmented call captured in a HIP graph: every replay, with eager
    work in between, equals the eager call."""
    import torch
    N, L, G = 40, 24, 6
    rib = P.Ribbon(N, L, 0, W.T_HOP, W.ETA)
    Es = _t(np.array([-0.4, 0.1, 0.35]) * abs(W.T_HOP))
    eps = _t(W.disorder_batch(L, N, 0.5, 2))
    ws = P.Workspace()
    out = torch.empty((2, 3), dtype=torch.float64, device="cuda")
    _say("segments graph capture")
    ref = P.conductance_segments(rib, Es, eps, n_segments=G, workspace=ws).clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        P.conductance_segments(rib, Es, eps, n_segments=G, workspace=ws, out=out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        P.conductance_segments(rib, Es, eps, n_segments=G, workspace=ws, out=out)
    for k in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), k
        P.conductance_segments(rib, Es * 0.5, eps, n_segments=G, workspace=ws)
        torch.cuda.synchronize()


def test_wide_ribbons_rejected(P):
    import torch
    with pytest.raises(Exception):
        P.conductance_segments(P.Ribbon(300, 4, 0, W.T_HOP, W.ETA),
                               torch.zeros(2, dtype=torch.float64, device="cuda"))
