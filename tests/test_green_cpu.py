"""Pins of the Green's-function Dyson oracle, Eq. (4)."""
import numpy as np

import oracle
import synthcell as sc
from oracle.green import green_dyson, fermionic_points
from tests import cells


def _band_g0(b, omegas):
    # G0 = U diag(1 / (i w + mu - eps)) U^H from the eigen-decomposition of H(k)
    return np.einsum("kab,mkb,kcb->mkac", b.U, 1.0 / (1j * omegas[:, None, None] + b.mu - b.eps[None]),
                     np.conj(b.U))


def test_free_green_function_is_band_form():
    spec = cells.two_species()
    hop, b, Gk, C = cells.inputs(spec)
    Hk = sc.hamiltonian_k(spec, hop)
    om = fermionic_points(5, spec.beta)
    G = green_dyson(Hk, b.mu, om)
    assert np.max(np.abs(G - _band_g0(b, om))) < 1e-12 * np.max(np.abs(G))


def test_scalar_form():
    G = green_dyson(np.array([[[0.3]]]), 0.1, np.array([0.7]), Sigma=np.array([[[[0.05 - 0.2j]]]]),
                    Sigma_x=np.array([[[-0.4]]]))
    assert abs(G[0, 0, 0, 0] - 1.0 / (0.7j + 0.1 - 0.3 + 0.4 - (0.05 - 0.2j))) < 1e-15


def test_dyson_identity_with_band_g0():
    spec = cells.two_species()
    hop, b, Gk, C = cells.inputs(spec)
    Hk = sc.hamiltonian_k(spec, hop)
    om = fermionic_points(4, spec.beta)
    rng = np.random.default_rng(21)
    n = spec.N_orb
    S = 0.1 * (rng.standard_normal((4, spec.N_R, n, n)) + 1j * rng.standard_normal((4, spec.N_R, n, n)))
    Sx = 0.1 * rng.standard_normal((spec.N_R, n, n))
    G = green_dyson(Hk, b.mu, om, Sigma=S, Sigma_x=Sx)
    G0 = _band_g0(b, om)
    rhs = G0 + np.einsum("mkab,mkbc,mkcd->mkad", G0, S + Sx[None], G)
    assert np.max(np.abs(G - rhs)) < 1e-10 * np.max(np.abs(G))


def test_high_frequency_tail():
    spec = cells.tiny()
    hop, b, Gk, C = cells.inputs(spec)
    Hk = sc.hamiltonian_k(spec, hop)
    w = 1e6
    G = green_dyson(Hk, b.mu, np.array([w]))
    tail = 1j * w * G[0]
    assert np.max(np.abs(tail - np.eye(spec.N_orb)[None])) < 1e-5


def test_matsubara_transform_of_band_green_function():
    # int_0^beta exp(i w tau) G(tau) dtau with G(tau) = -(1 - f(x)) exp(-x tau), x = eps - mu,
    # equals 1 / (i w - x) for fermionic w: the free Dyson solution, band by band
    beta, x = 7.0, np.array([-0.8, 0.05, 1.3])
    om = fermionic_points(3, beta)
    f = sc.fermi(x, beta)
    for w in om:
        exact = -(1.0 - f) * (np.exp((1j * w - x) * beta) - 1.0) / (1j * w - x)
        G = green_dyson(np.diag(x)[None].astype(complex), 0.0, np.array([w]))[0, 0]
        assert np.max(np.abs(np.diag(G) - exact)) < 1e-12 * np.max(np.abs(exact))


def test_count_converges_to_fermi_sum():
    from oracle.green import density_omega
    spec = cells.tiny(complex_hopping=True)
    hop, b, Gk, C = cells.inputs(spec)
    Hk = sc.hamiltonian_k(spec, hop)
    mu = b.mu + 0.3
    exact = spec.spin * sc.fermi(b.eps - mu, spec.beta).sum() / spec.N_R
    err = []
    for n_om in (16, 64, 256):
        G = green_dyson(Hk, mu, fermionic_points(n_om, spec.beta))
        err.append(abs(density_omega(G, Hk, mu, spec.beta, spec.spin) - exact))
    # the first dropped tail term falls as n_omega^-3: each fourfold step gains well over 20x
    assert err[2] < 2e-5 * exact and err[1] < err[0] / 20 and err[2] < err[1] / 20


def test_update_mu_reaches_band_chemical_potential():
    import pytest
    from oracle.green import update_mu
    spec = cells.tiny(complex_hopping=True)
    hop, b, Gk, C = cells.inputs(spec)
    Hk = sc.hamiltonian_k(spec, hop)
    target = spec.spin * spec.N_orb / 2.0
    mu, n = update_mu(Hk, spec.beta, 64, spec.spin, target, b.mu - 1.0, b.mu + 1.0, 1e-10, 80)
    assert abs(n - target) <= 1e-10 and abs(mu - b.mu) < 1e-4
    with pytest.raises(ValueError):
        update_mu(Hk, spec.beta, 64, spec.spin, target, b.mu + 0.5, b.mu + 1.0, 1e-10, 80)
