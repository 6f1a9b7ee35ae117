"""One cycle of the self-consistent GW loop (oracle, test infrastructure).

Sec. 2, Eqs. (1)-(4): from G(k, tau) the cycle forms the polarizability, screens the bare
interaction, forms the self-energy (correlation from W~, exchange from V) and solves the Dyson
equation for the next G, with the chemical potential moved so that the electron count stays at its
target.  Every step is one of the oracle's own functions, in this order:

    G^R(tau)        = k_to_r(G(k, tau))
    P^q(tau)        = polarizability_q(G(k, tau))                     (Eq. (1), time domain)
    P(q, i nu)      = filon_matrix(tau, bosonic) P^q(tau)
    W~(q, i nu)     = screened_interaction(V, P)                       (Eq. (2))
    W~(q, tau)      = omega_to_tau_matrix(tau, bosonic) W~(q, i nu)
    Sigma_c(k, tau) = self_energy_k(G(k, tau), k_to_r(W~(q, tau)))    (Eq. (3), time domain)
    Sigma_c(k, i w) = filon_matrix(tau, fermionic) Sigma_c(k, tau)
    Sigma_x(k)      = r_to_k(exchange_r(G^R, V^R))
    mu              = update_mu(...)  (unless given)                   (Sec. 4)
    G(k, i w)       = green_dyson(H, mu, w, Sigma_c, Sigma_x)          (Eq. (4))
    G(k, tau)       = green_tau(G(k, i w), H, mu, ...)

with n_omega = n_tau frequencies throughout.  Parity status: each step is pinned on its own in
the tests; the chain itself is the definition written out.
"""
import numpy as np

from .dyson import omega_to_tau_matrix, screened_interaction
from .exchange import exchange_r
from .fourier import k_to_r, r_to_k
from .green import green_dyson, green_tau, update_mu
from .matsubara import apply_tau_to_omega, bosonic_frequencies, fermionic_frequencies, filon_matrix
from .polarizability import polarizability_q
from .self_energy import self_energy_k


def cycle(Gk, spec, C, Hk, V, taus, n_target, mu=None, mu_lo=None, mu_hi=None, tol=1e-10, max_iter=200):
    """One cycle from G(k, tau) [n_tau][N_k][N_orb][N_orb]; V [N_k][N_pb][N_pb] the bare interaction.
    With mu given the Dyson step uses it (no search).  Returns (G(k, tau), mu, parts) with parts the
    intermediate results (P(q, i nu), W~(q, tau), Sigma_c(k, i w), Sigma_x(k), G(k, i w))."""
    nt, beta, g = spec.n_tau, spec.beta, spec.spin
    omb, omf = bosonic_frequencies(nt, beta), fermionic_frequencies(nt, beta)
    GR = k_to_r(Gk, spec.mesh)
    Pw = apply_tau_to_omega(filon_matrix(taus, omb), polarizability_q(Gk, spec, C, g))
    Wt = apply_tau_to_omega(omega_to_tau_matrix(taus, omb), screened_interaction(V, Pw))
    Sc = apply_tau_to_omega(filon_matrix(taus, omf), self_energy_k(Gk, k_to_r(Wt, spec.mesh), spec, C))
    VR = k_to_r(np.asarray(V)[None], spec.mesh)[0]
    Sx = r_to_k(exchange_r(GR, VR, spec, C)[None], spec.mesh)[0]
    if mu is None:
        mu, _ = update_mu(Hk, beta, nt, g, n_target, mu_lo, mu_hi, tol, max_iter, Sc, Sx)
    Gw = green_dyson(Hk, mu, omf, Sigma=Sc, Sigma_x=Sx)
    return green_tau(Gw, Hk, mu, beta, taus, Sigma_x=Sx), mu, dict(P=Pw, W=Wt, Sigma_c=Sc, Sigma_x=Sx, G_w=Gw)


def run(Gk, spec, C, Hk, V, taus, n_target, mu0, cycles, mix=0.5, tol=1e-10, max_iter=200):
    """`cycles` cycles from G(k, tau) = Gk with the next input mix G_new + (1 - mix) G_in and the mu
    search bracketed by mu -+ 1 around the previous one.  Returns the list of (G(k, tau), mu)."""
    G, mu, out = np.asarray(Gk), mu0, []
    for _ in range(cycles):
        Gn, mu, _ = cycle(G, spec, C, Hk, V, taus, n_target, mu_lo=mu - 1.0, mu_hi=mu + 1.0, tol=tol,
                          max_iter=max_iter)
        G = mix * Gn + (1.0 - mix) * G
        out.append((G, mu))
    return out
