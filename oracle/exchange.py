"""Static (exchange) part of the self-energy (oracle, test infrastructure).

Sec. 2 states that the static part uses the same MT-MT expression as Eq. (8) with the screening
part of the interaction replaced by the bare one, W~(tau) -> V, and the Green's function replaced
by -G(beta).  With G^R(beta) read at the last grid point (beta^-):

    Sigma_x^R_ab = -sum C^I_aa' (-G^R_a'b'(beta)) V^R_IJ C^J_bb' = +sum C^I_aa' G^R_a'b'(beta) V^R_IJ C^J_bb'.

exchange_r applies the oracle's Eq. (8) with that replacement; exchange_k is the k-space form
(the q-convolution of the oracle's Eq. (3) structure with the same replacement).

Parity status: pinned in the tests by the one-orbital, one-function closed form
Sigma_x = C^2 G(beta) V (its sign in particular), by a local V (Sigma_x only at R = 0, one
matrix sandwich per atom), and by the agreement of the R- and k-space forms under the lattice sum.
"""
from .self_energy import self_energy_k, self_energy_r


def exchange_r(GR, VR, spec, C):
    """Sigma_x^R [N_R][No][No] from G^R(tau) [n_tau][N_R][No][No] (last tau = beta^-) and V^R [N_R][Np][Np]."""
    return self_energy_r(-GR[-1:], VR[None], spec, C)[0]


def exchange_k(Gk, VR, spec, C):
    """Sigma_x(k) [N_k][No][No] from G(k, tau) and V^R, by the k-space convolution."""
    return self_energy_k(-Gk[-1:], VR[None], spec, C)[0]
