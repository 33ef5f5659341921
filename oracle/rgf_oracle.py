"""FP64 CPU oracle: armchair graphene ribbon conductance by the recursive
Green's function method.

TEST INFRASTRUCTURE ONLY (see the package docstring). Plain numpy, complex128,
dense matrices, no structure tricks and no blocking beyond what the equations
state. Nothing here is shared with the HIP library.

Model (paper: model paragraph and Fig. 1(a); readings listed in the design doc):
  * slice i = 1..L holds N atoms, one p orbital each, indexed k = 0..N-1 along
    the transverse zigzag chain of an armchair ribbon;
  * slice Hamiltonian H_i = diag(eps_i) + t * (k <-> k+1 path adjacency);
  * slice i couples to slice i+1 through the diagonal block
    U_i = t * diag([(k + i + parity) even]), so consecutive slices alternate
    which half of the chain carries the longitudinal bonds;
  * two semi-infinite pristine leads (eps = 0, same N, same parity rule) are
    attached to slice 1 and slice L;
  * z = E + i*eta is used in the leads and in the device alike.

All energies and t, eta, eps are in eV; the conductance is in units of 2e^2/h.
"""

import numpy as np

__all__ = [
    "coupling_mask",
    "slice_hamiltonian",
    "coupling",
    "coupling_diag",
    "sancho_rubio",
    "surface_gf_modes",
    "lead_self_energies",
    "transmission",
    "transmission_rl",
    "transmission_bf",
    "transmission_grad",
    "transmission_grad_bf",
    "ldos",
    "ldos_bf",
    "channel_transmission",
    "channel_transmission_bf",
    "open_channels",
    "half_gap",
    "transmission_sweep",
]


# --------------------------------------------------------------------------
# Model: the slice Hamiltonian and the inter-slice hopping (model paragraph;
# Fig. 1(a): armchair edges, one p orbital per carbon atom).
# --------------------------------------------------------------------------

def coupling_mask(N, i, parity=0):
    """Boolean vector: rows k of slice i that bond to slice i+1."""
    k = np.arange(N)
    return ((k + i + parity) % 2) == 0


def slice_hamiltonian(N, t, eps_row=None):
    """H_i = diag(eps) + t * path adjacency (the transverse zigzag chain)."""
    H = np.zeros((N, N), dtype=np.complex128)
    if eps_row is not None:
        H[np.arange(N), np.arange(N)] = np.asarray(eps_row, dtype=np.float64)
    for k in range(N - 1):
        H[k, k + 1] = t
        H[k + 1, k] = t
    return H


def coupling(N, t, i, parity=0):
    """U_i = H_{i,i+1}: hopping block from slice i to slice i+1."""
    return np.diag(coupling_diag(N, t, i, parity)).astype(np.complex128)


def coupling_diag(N, t, i, parity=0):
    """Diagonal of U_i (U_i is diagonal: each row bonds straight ahead or not)."""
    return np.where(coupling_mask(N, i, parity), t, 0.0)


# --------------------------------------------------------------------------
# Leads: the paper obtains the lead self-energies at slices 1 and M from an
# eigenproblem, separately from the recursion (method section). The default
# here is that route (Bloch modes of the lead); Sancho-Rubio decimation
# (M. P. Lopez Sancho, J. M. Lopez Sancho, J. Rubio, J. Phys. F 15 (1985) 851)
# is kept as a second route to the same retarded surface Green's function.
# --------------------------------------------------------------------------

def sancho_rubio(z, h00, h01, tol=1e-15, maxit=200):
    """Surface Green's function of a semi-infinite stack of identical layers.

    h00: Hamiltonian of one layer; h01: hopping from the surface layer to the
    next layer deeper in the stack (the reverse hopping is h01^T since H is
    real symmetric). Returns (g_surf, iterations, converged).
    """
    n = h00.shape[0]
    eye = np.eye(n, dtype=np.complex128)
    eps_s = h00.astype(np.complex128).copy()
    eps_b = h00.astype(np.complex128).copy()
    alpha = h01.astype(np.complex128).copy()
    beta = h01.T.astype(np.complex128).copy()
    scale = max(np.abs(h01).max(), np.abs(h00).max(), 1.0)
    it = 0
    converged = False
    while it < maxit:
        g = np.linalg.inv(z * eye - eps_b)
        agb = alpha @ g @ beta
        bga = beta @ g @ alpha
        eps_s = eps_s + agb
        eps_b = eps_b + agb + bga
        alpha = alpha @ g @ alpha
        beta = beta @ g @ beta
        it += 1
        if max(np.abs(alpha).max(), np.abs(beta).max()) < tol * scale:
            converged = True
            break
    return np.linalg.inv(z * eye - eps_s), it, converged


def surface_gf_modes(z, h00, h01):
    """Surface Green's function of a semi-infinite stack of identical layers
    from its Bloch modes: the eigenproblem route of the paper's method section
    (mode matching as in T. Ando, Phys. Rev. B 44 (1991) 8017).

    Bloch solutions psi_{n+1} = lam psi_n of
    (z - h00 - lam h01 - h01^T / lam) psi = 0 come from the linear pencil
    A v = lam B v, v = (psi, lam psi). With eta > 0 exactly m = dim(h00) of
    them decay into the stack (|lam| < 1; lam = 0 for the null space of
    h01^T). With U their eigenvectors and F = U diag(lam) U^{-1} the layer-
    to-layer transfer, the surface layer obeys
    g_surf = (z - h00 - h01 F)^{-1}.
    """
    import scipy.linalg as sla
    m = h00.shape[0]
    I = np.eye(m)
    Z = np.zeros((m, m))
    A = np.block([[Z, I], [-h01.T, z * I - h00]])
    B = np.block([[I, Z], [Z, h01]])
    lam, V = sla.eig(A, B)
    sel = np.nonzero(np.isfinite(lam) & (np.abs(lam) < 1.0))[0]
    if len(sel) != m:
        raise ArithmeticError(f"{len(sel)} decaying modes for a layer of {m} sites")
    U = V[:m, sel]
    F = U @ np.diag(lam[sel]) @ np.linalg.inv(U)
    return np.linalg.inv(z * I - h00 - h01 @ F)


def _lead_cells(N, t, L, parity):
    """Two-slice principal layers of the left and right leads.

    Left lead: surface cell (slice -1, slice 0); the next cell deeper is
    (slice -3, slice -2) and the only bond between them is slice -1 <-> -2.
    Right lead: surface cell (slice L+1, slice L+2); next cell (L+3, L+4),
    bonded through slice L+2 <-> L+3.
    """
    H0 = slice_hamiltonian(N, t)
    Z = np.zeros((N, N), dtype=np.complex128)
    # left
    Um1 = coupling(N, t, -1, parity)
    Um2 = coupling(N, t, -2, parity)
    h00_l = np.block([[H0, Um1], [Um1.T, H0]])
    h01_l = np.block([[Z, Um2.T], [Z, Z]])  # row: slice -1, column: slice -2
    # right
    Up1 = coupling(N, t, L + 1, parity)
    Up2 = coupling(N, t, L + 2, parity)
    h00_r = np.block([[H0, Up1], [Up1.T, H0]])
    h01_r = np.block([[Z, Z], [Up2, Z]])  # row: slice L+2, column: slice L+3
    return (h00_l, h01_l), (h00_r, h01_r)


def lead_self_energies(N, L, t, eta, E, parity=0, tol=1e-15, maxit=200,
                       return_info=False, method="modes"):
    """Sigma_L (acts on slice 1) and Sigma_R (acts on slice L), N x N each.

    Sigma_L = H_{1,0} g_L H_{0,1} = U_0^T g_L[0,0] U_0,
    Sigma_R = H_{L,L+1} g_R H_{L+1,L} = U_L g_R[L+1,L+1] U_L^T.
    method = "modes": Bloch-mode eigenproblem (surface_gf_modes), the default;
    method = "decimation": Sancho-Rubio on the dense two-slice cell (loses
    digits for wide leads and can settle on the advanced solution when the
    cell's Bloch phase is commensurate; kept as a cross-check).
    """
    z = complex(E, eta)
    (h00_l, h01_l), (h00_r, h01_r) = _lead_cells(N, t, L, parity)
    if method == "modes":
        gl, itl, okl = surface_gf_modes(z, h00_l, h01_l), 0, True
        gr, itr, okr = surface_gf_modes(z, h00_r, h01_r), 0, True
    else:
        gl, itl, okl = sancho_rubio(z, h00_l, h01_l, tol, maxit)
        gr, itr, okr = sancho_rubio(z, h00_r, h01_r, tol, maxit)
    g0 = gl[N:, N:]        # slice 0 block of the left surface cell
    gLp1 = gr[:N, :N]      # slice L+1 block of the right surface cell
    U0 = coupling(N, t, 0, parity)
    UL = coupling(N, t, L, parity)
    sig_l = U0.T @ g0 @ U0
    sig_r = UL @ gLp1 @ UL.T
    if not return_info:
        return sig_l, sig_r
    info = {
        "iterations": (itl, itr),
        "converged": (okl, okr),
        "g_surf": (gl, gr),
        "cells": ((h00_l, h01_l), (h00_r, h01_r)),
    }
    return sig_l, sig_r, info


def _gamma(sig):
    """Broadening Gamma = i (Sigma - Sigma^dagger) (Eq. (2) and its reference)."""
    return 1j * (sig - sig.conj().T)


# --------------------------------------------------------------------------
# Recursive Green's function (Eqs. (3)-(5)).
#
# Eq. (4) is used in its algebraically identical form
#   g_jj = (E - H_j - Sigma^l g_{j-1,j-1} Sigma^r)^{-1},
# with Sigma^l = H_{j,j-1} = U_{j-1}^T and Sigma^r = H_{j-1,j} = U_{j-1} the
# inter-slice hopping blocks, and Eq. (5) as the running product
#   G_{1j} = G_{1,j-1} Sigma^r g_jj.
# The lead self-energies enter at the first and the last slice; after the last
# slice G_{1L} is the block of the full Green's function of Eq. (1) that
# Eq. (2) needs.
# --------------------------------------------------------------------------

def _device_slices(N, L, t, eps):
    """Slice Hamiltonians H_1..H_L; a vacant site (on-site energy +inf, see
    _vacancies) gets 0 here, its row and column are decoupled by
    _slice_inverse."""
    if eps is None:
        eps = np.zeros((L, N))
    eps = np.asarray(eps, dtype=np.float64)
    assert eps.shape == (L, N)
    eps = np.where(np.isposinf(eps), 0.0, eps)
    return [slice_hamiltonian(N, t, eps[i]) for i in range(L)]


# --------------------------------------------------------------------------
# Lattice defects (the paper's simulation flow starts from generating atomic
# defects; its model paragraph names lattice defects beside disorder). A
# vacancy removes an atom: on-site energy +inf, the limit in which the site
# decouples from every bond and from the leads.
# --------------------------------------------------------------------------

def _vacancies(N, L, eps):
    """Boolean [L, N]: the sites removed from the lattice (eps = +inf)."""
    if eps is None:
        return np.zeros((L, N), dtype=bool)
    return np.isposinf(np.asarray(eps, dtype=np.float64))


def _slice_inverse(A, vac):
    """A^{-1} for the lattice without the vacant sites (boolean mask vac):
    their rows and columns of A are replaced by the identity's, so the
    inverse is block diagonal, and their own diagonal entries are then set
    to zero -- the Green's function of the lattice with the sites removed,
    embedded with zero rows and columns."""
    if vac is None or not vac.any():
        return np.linalg.inv(A)
    idx = np.nonzero(vac)[0]
    A = A.copy()
    A[idx, :] = 0.0
    A[:, idx] = 0.0
    A[idx, idx] = 1.0
    g = np.linalg.inv(A)
    g[idx, idx] = 0.0
    return g


def transmission(N, L, t, eta, E, eps=None, parity=0, sigmas=None,
                 return_g=False):
    """T(E) = Re Tr[Gamma_L G_1L Gamma_R G_1L^dagger] by the left-to-right sweep."""
    z = complex(E, eta)
    if sigmas is None:
        sigmas = lead_self_energies(N, L, t, eta, E, parity)
    sig_l, sig_r = sigmas
    Hs = _device_slices(N, L, t, eps)
    vac = _vacancies(N, L, eps)
    eye = np.eye(N, dtype=np.complex128)
    # slice 1
    A = z * eye - Hs[0] - sig_l
    if L == 1:
        A = A - sig_r
    g = _slice_inverse(A, vac[0])
    G1 = g
    for j in range(2, L + 1):
        u = coupling_diag(N, t, j - 1, parity)     # H_{j-1,j} = diag(u)
        # U^T g U and G1 U with U = diag(u), written as row/column scalings
        A = z * eye - Hs[j - 1] - u[:, None] * g * u[None, :]
        if j == L:
            A = A - sig_r
        g = _slice_inverse(A, vac[j - 1])
        G1 = (G1 * u[None, :]) @ g
    T = np.real(np.trace(_gamma(sig_l) @ G1 @ _gamma(sig_r) @ G1.conj().T))
    if return_g:
        return T, G1
    return T


def transmission_rl(N, L, t, eta, E, eps=None, parity=0, sigmas=None):
    """T_RL = Re Tr[Gamma_R G_L1 Gamma_L G_L1^dagger] by the right-to-left sweep.

    Same Dyson recursion run from slice L down to slice 1; equals T_LR for a
    two-terminal system (self-check).
    """
    z = complex(E, eta)
    if sigmas is None:
        sigmas = lead_self_energies(N, L, t, eta, E, parity)
    sig_l, sig_r = sigmas
    Hs = _device_slices(N, L, t, eps)
    vac = _vacancies(N, L, eps)
    eye = np.eye(N, dtype=np.complex128)
    A = z * eye - Hs[L - 1] - sig_r
    if L == 1:
        A = A - sig_l
    g = _slice_inverse(A, vac[L - 1])
    GL = g                                       # G_{L,j} (right-connected)
    for j in range(L - 1, 0, -1):
        U = coupling(N, t, j, parity)            # H_{j,j+1}
        A = z * eye - Hs[j - 1] - U @ g @ U.T
        if j == 1:
            A = A - sig_l
        g = _slice_inverse(A, vac[j - 1])
        GL = GL @ U.T @ g
    return np.real(np.trace(_gamma(sig_r) @ GL @ _gamma(sig_l) @ GL.conj().T))


def _full_matrix(N, L, t, eta, E, eps, parity, sigmas):
    """z - H - Sigma_L - Sigma_R over all N*L device sites (Eq. (1))."""
    z = complex(E, eta)
    Hs = _device_slices(N, L, t, eps)
    M = np.zeros((N * L, N * L), dtype=np.complex128)
    for i in range(L):
        M[i * N:(i + 1) * N, i * N:(i + 1) * N] = z * np.eye(N) - Hs[i]
        if i + 1 < L:
            U = coupling(N, t, i + 1, parity)
            M[i * N:(i + 1) * N, (i + 1) * N:(i + 2) * N] = -U
            M[(i + 1) * N:(i + 2) * N, i * N:(i + 1) * N] = -U.T
    sig_l, sig_r = sigmas
    M[:N, :N] -= sig_l
    M[(L - 1) * N:, (L - 1) * N:] -= sig_r
    return M


def transmission_bf(N, L, t, eta, E, eps=None, parity=0, sigmas=None):
    """Brute force: invert the full device matrix, then Eq. (2). Vacant
    sites (eps = +inf) are deleted from the matrix, and from the lead
    couplings, before the inversion."""
    if sigmas is None:
        sigmas = lead_self_energies(N, L, t, eta, E, parity)
    sig_l, sig_r = sigmas
    M = _full_matrix(N, L, t, eta, E, eps, parity, sigmas)
    keep = ~_vacancies(N, L, eps).reshape(-1)
    first, last = keep.copy(), keep.copy()
    first[N:] = False                      # kept sites of slice 1
    last[:(L - 1) * N] = False             # kept sites of slice L
    G = np.linalg.inv(M[np.ix_(keep, keep)])
    cols = np.cumsum(keep) - 1             # position of a kept site in G
    G1L = G[np.ix_(cols[first], cols[last])]
    kl, kr = first[:N], last[(L - 1) * N:]
    gl = _gamma(sig_l)[np.ix_(kl, kl)]
    gr = _gamma(sig_r)[np.ix_(kr, kr)]
    return np.real(np.trace(gl @ G1L @ gr @ G1L.conj().T))


# --------------------------------------------------------------------------
# Gradient dT/d eps_{i,k}.
#
# From Eq. (1): dG/d eps_s = G E_ss G, so Eq. (2) gives
#   dT/d eps_s = 2 Re[ G[s, slice L] B G[slice 1, s] ],  B = Gamma_R G_1L^dag Gamma_L.
# --------------------------------------------------------------------------

def _kept_inverse(N, L, t, eta, E, eps, parity, sigmas):
    """(G over the kept sites, kept mask [L*N], position of each kept site
    in G): the full device matrix with vacant sites deleted, inverted."""
    M = _full_matrix(N, L, t, eta, E, eps, parity, sigmas)
    keep = ~_vacancies(N, L, eps).reshape(-1)
    return np.linalg.inv(M[np.ix_(keep, keep)]), keep, np.cumsum(keep) - 1


def transmission_grad_bf(N, L, t, eta, E, eps=None, parity=0, sigmas=None):
    """(T, dT/deps [L, N]) from the full inverse (tiny ribbons only); vacant
    sites are deleted and get a zero derivative."""
    if sigmas is None:
        sigmas = lead_self_energies(N, L, t, eta, E, parity)
    sig_l, sig_r = sigmas
    G, keep, pos = _kept_inverse(N, L, t, eta, E, eps, parity, sigmas)
    first = keep.copy()
    first[N:] = False
    last = keep.copy()
    last[:(L - 1) * N] = False
    kl, kr = first[:N], last[(L - 1) * N:]
    G1L = G[np.ix_(pos[first], pos[last])]
    gl = _gamma(sig_l)[np.ix_(kl, kl)]
    gr = _gamma(sig_r)[np.ix_(kr, kr)]
    T = np.real(np.trace(gl @ G1L @ gr @ G1L.conj().T))
    B = gr @ G1L.conj().T @ gl
    right = G[:, pos[last]]          # G[s, slice L]
    left = G[pos[first], :]          # G[slice 1, s]
    d = np.zeros(N * L)
    d[keep] = 2.0 * np.real(np.einsum("sa,ab,bs->s", right, B, left))
    return T, d.reshape(L, N)


def transmission_grad(N, L, t, eta, E, eps=None, parity=0, sigmas=None):
    """(T, dT/deps [L, N]) by a forward and a backward Dyson sweep.

    Forward (left-connected, Eq. (4)-(5) form): g_i, the running
    G1_i = g_{1,i} and the column block g_{i,1}.
    Backward (Eq. (3) with the cut between slices i and i+1, both orders):
      F_{i,L} = g_i U_i F_{i+1,L},          F_{L,L} = g_L
      F_{i,1} = g_{i,1} + g_i U_i F_{i+1,1}, F_{L,1} = g_{L,1}
      F_{1,i} = G1_i + F_{1,i+1} U_i^T g_i, F_{1,L} = G1_L
    where F is the full-system Green's function.
    """
    z = complex(E, eta)
    if sigmas is None:
        sigmas = lead_self_energies(N, L, t, eta, E, parity)
    sig_l, sig_r = sigmas
    Hs = _device_slices(N, L, t, eps)
    vac = _vacancies(N, L, eps)
    eye = np.eye(N, dtype=np.complex128)
    gs, G1s = [], []
    A = z * eye - Hs[0] - sig_l
    if L == 1:
        A = A - sig_r
    g = _slice_inverse(A, vac[0])
    gs.append(g)
    G1s.append(g)
    for j in range(2, L + 1):
        U = coupling(N, t, j - 1, parity)
        A = z * eye - Hs[j - 1] - U.T @ g @ U
        if j == L:
            A = A - sig_r
        g = _slice_inverse(A, vac[j - 1])
        gs.append(g)
        G1s.append(G1s[-1] @ U @ g)
    G1L = G1s[-1]
    gl, gr = _gamma(sig_l), _gamma(sig_r)
    T = np.real(np.trace(gl @ G1L @ gr @ G1L.conj().T))
    B = gr @ G1L.conj().T @ gl
    d = np.zeros((L, N))
    FiL = gs[-1]                    # F_{L,L}
    F1i = G1L                       # F_{1,L}
    d[L - 1] = 2.0 * np.real(np.einsum("ka,ab,bk->k", FiL, B, F1i))
    for i in range(L - 1, 0, -1):   # slice i (1-based), python index i-1
        U = coupling(N, t, i, parity)
        FiL = gs[i - 1] @ U @ FiL
        F1i = G1s[i - 1] + F1i @ U.T @ gs[i - 1]
        d[i - 1] = 2.0 * np.real(np.einsum("ka,ab,bk->k", FiL, B, F1i))
    return T, d


# --------------------------------------------------------------------------
# Local density of states rho_s(E) = -Im G_ss(E) / pi: the diagonal of the
# full Green's function G of Eq. (1) (the paper lists the charge density
# among what the Green's function gives; the LDOS at energy E is its
# spectral density).
# --------------------------------------------------------------------------

def ldos_bf(N, L, t, eta, E, eps=None, parity=0, sigmas=None):
    """-Im diag(G) / pi as [L, N], from the full inverse (tiny ribbons only);
    vacant sites are deleted and get zero."""
    if sigmas is None:
        sigmas = lead_self_energies(N, L, t, eta, E, parity)
    G, keep, _ = _kept_inverse(N, L, t, eta, E, eps, parity, sigmas)
    out = np.zeros(N * L)
    out[keep] = -np.imag(np.diag(G)) / np.pi
    return out.reshape(L, N)


def ldos(N, L, t, eta, E, eps=None, parity=0, sigmas=None):
    """-Im diag(G) / pi as [L, N] by the forward sweep of the left-connected
    g_i (Eq. (4) form) and the backward recursion for the diagonal blocks of
    the full Green's function, Dyson's equation (Eq. (3)) cut between slices
    i and i+1:
      F_{L,L} = g_L,   F_{i,i} = g_i + g_i U_i F_{i+1,i+1} U_i^T g_i.
    """
    z = complex(E, eta)
    if sigmas is None:
        sigmas = lead_self_energies(N, L, t, eta, E, parity)
    sig_l, sig_r = sigmas
    Hs = _device_slices(N, L, t, eps)
    vac = _vacancies(N, L, eps)
    eye = np.eye(N, dtype=np.complex128)
    gs = []
    A = z * eye - Hs[0] - sig_l
    if L == 1:
        A = A - sig_r
    g = _slice_inverse(A, vac[0])
    gs.append(g)
    for j in range(2, L + 1):
        U = coupling(N, t, j - 1, parity)
        A = z * eye - Hs[j - 1] - U.T @ g @ U
        if j == L:
            A = A - sig_r
        g = _slice_inverse(A, vac[j - 1])
        gs.append(g)
    out = np.empty((L, N))
    F = gs[-1]
    out[L - 1] = -np.imag(np.diag(F)) / np.pi
    for i in range(L - 1, 0, -1):   # slice i (1-based), python index i-1
        U = coupling(N, t, i, parity)
        gi = gs[i - 1]
        F = gi + gi @ U @ F @ U.T @ gi
        out[i - 1] = -np.imag(np.diag(F)) / np.pi
    return out


# --------------------------------------------------------------------------
# Transmission per incoming lead channel. Gamma_L is real symmetric and
# positive semidefinite; its eigenvectors u_i with gamma_i > 0 are the
# incoming channels of the left lead, and Eq. (2) splits as
#   T = Tr[Gamma_L G Gamma_R G^dagger] = sum_i gamma_i u_i^T G Gamma_R G^dagger u_i.
# --------------------------------------------------------------------------

def _channel_split(gl, gr, G, rel_tol):
    """(gamma_i, T_i) for the eigenpairs of Gamma_L with gamma_i above
    rel_tol * max gamma, in decreasing gamma."""
    gl = np.real(0.5 * (gl + gl.conj().T))
    w, U = np.linalg.eigh(gl)
    keep = w > rel_tol * max(w.max(), 0.0)
    w, U = w[keep][::-1], U[:, keep][:, ::-1]
    M = G @ gr @ G.conj().T
    Ti = np.array([w[i] * np.real(U[:, i] @ M @ U[:, i]) for i in range(len(w))])
    return w, Ti


def channel_transmission(N, L, t, eta, E, eps=None, parity=0, sigmas=None, rel_tol=1e-6):
    """(gamma_i, T_i) of the left lead's incoming channels (eigenpairs of
    Gamma_L whose gamma_i exceeds rel_tol * max gamma; evanescent modes have
    gamma of order eta), G = G_{1L} from the recursion. sum_i T_i = T."""
    if sigmas is None:
        sigmas = lead_self_energies(N, L, t, eta, E, parity)
    _, G = transmission(N, L, t, eta, E, eps, parity, sigmas, return_g=True)
    return _channel_split(_gamma(sigmas[0]), _gamma(sigmas[1]), G, rel_tol)


def channel_transmission_bf(N, L, t, eta, E, eps=None, parity=0, sigmas=None, rel_tol=1e-6):
    """channel_transmission with G_{1L} from the full inverse (tiny ribbons)."""
    if sigmas is None:
        sigmas = lead_self_energies(N, L, t, eta, E, parity)
    Gf = np.linalg.inv(_full_matrix(N, L, t, eta, E, eps, parity, sigmas))
    return _channel_split(_gamma(sigmas[0]), _gamma(sigmas[1]), Gf[:N, (L - 1) * N:], rel_tol)


# --------------------------------------------------------------------------
# Closed forms for the pristine armchair ribbon.
# --------------------------------------------------------------------------

def open_channels(N, E, t):
    """Number of propagating channels M(E) in the pristine lead.

    Transverse modes p and N+1-p of the zigzag chain pair up; each pair is a
    chain with alternating hoppings |t| and 2|t|cos(p pi/(N+1)), whose band
    covers |1 - 2c_p| < |E|/|t| < 1 + 2c_p and carries one right-moving state.
    A metallic ribbon (N = 2 mod 3) has one channel at E = 0.
    """
    x = abs(E) / abs(t)
    p = np.arange(1, N // 2 + 1)
    c = np.cos(p * np.pi / (N + 1))
    m = int(np.sum((np.abs(1.0 - 2.0 * c) < x) & (x < 1.0 + 2.0 * c)))
    if x == 0.0 and N % 3 == 2:
        m += 1
    return m


def half_gap(N, t):
    """Half of the band gap around E = 0 of the pristine ribbon, in eV."""
    p = np.arange(1, N // 2 + 1)
    return abs(t) * float(np.min(np.abs(1.0 - 2.0 * np.cos(p * np.pi / (N + 1)))))


# --------------------------------------------------------------------------
# Convenience: an energy sweep sharing the lead self-energies per energy.
# --------------------------------------------------------------------------

def transmission_sweep(N, L, t, eta, energies, eps=None, parity=0):
    """T for each energy (one realization), by transmission()."""
    out = np.empty(len(energies))
    for j, E in enumerate(energies):
        out[j] = transmission(N, L, t, eta, float(E), eps, parity)
    return out
