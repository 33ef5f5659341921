"""Plain FP64 CPU oracle for the RGF conductance of armchair graphene ribbons.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import this
package: only the test-suite, the smoke check and the benchmark's CPU
baseline leg use it. It shares no code with the HIP library and the HIP
library never calls it.

Paper: S. Ihnatsenka, "Computation of electron quantum transport in graphene
nanoribbons using GPU", Comput. Phys. Commun. 183 (2012) 543 (arXiv:1107.5300).

Every function is written from the paper's equations (Eq. (1) the Green's
function, Eq. (2) the conductance, Eq. (3) Dyson's equation, Eqs. (4)-(5) the
slice recursion) plus the textbook definitions the paper defers to
(broadening Gamma = i(Sigma - Sigma^dagger); the lead surface Green's
function from the Bloch-mode eigenproblem, or from Sancho-Rubio decimation).

Parity status per function (see the pins in tests/test_oracle_*.py):
  transmission_bf        pinned: closed forms (quantised pristine T, 1D chain
                         impurity), symmetries, bounds
  transmission           pinned: == transmission_bf on tiny ribbons
  lead_self_energies     pinned: closed-form surface GF of the decoupled
                         transverse-mode chains (both routes: Bloch-mode
                         eigenproblem, default, and Sancho-Rubio), fixed-point
                         residual, sign of Im Sigma
  open_channels          pinned: Bloch band counting of the lead unit cell
  half_gap               pinned: band-structure minimum over a dense k grid
  transmission_grad_bf   pinned: central finite differences
  transmission_grad      pinned: == transmission_grad_bf on tiny ribbons
  ldos_bf                pinned: closed-form LDOS of the infinite 1D chain
                         (the N = 2 ribbon), non-negativity
  ldos                   pinned: == ldos_bf on tiny ribbons
  channel_transmission_bf
                         pinned: pristine ribbons transmit every open channel
                         fully (T_i = 1, M(E) channels), 0 <= T_i <= 1, sum
                         T_i = transmission_bf
  channel_transmission   pinned: == channel_transmission_bf on tiny ribbons
"""

from .rgf_oracle import (  # noqa: F401
    coupling_mask,
    slice_hamiltonian,
    coupling,
    coupling_diag,
    sancho_rubio,
    surface_gf_modes,
    lead_self_energies,
    transmission,
    transmission_rl,
    ldos,
    ldos_bf,
    channel_transmission,
    channel_transmission_bf,
    transmission_bf,
    transmission_grad,
    transmission_grad_bf,
    open_channels,
    half_gap,
    transmission_sweep,
)
