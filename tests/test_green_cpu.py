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


def test_tail_transforms_against_brute_force_matsubara_sums():
    """The closed forms green_tau uses for the two tails: (1/beta) sum over all fermionic n of
    exp(-i w_n tau) / (i w_n) = -1/2 and of exp(-i w_n tau) / (i w_n)^2 = (2 tau - beta) / 4 on
    0 < tau < beta, checked by direct symmetric sums; and green_tau returns exactly those forms
    for a G made of the tails alone, at any number of frequencies."""
    from oracle.green import green_tau
    beta = 3.0
    n = np.arange(-400000, 400000)
    w = (2 * n + 1) * np.pi / beta
    for t in (0.3, 1.1, 2.6):
        s1 = np.sum(np.exp(-1j * w * t) / (1j * w)).real / beta
        s2 = np.sum(np.exp(-1j * w * t) / (1j * w) ** 2).real / beta
        assert abs(s1 + 0.5) < 2e-5 and abs(s2 - (2 * t - beta) / 4) < 2e-6
    rng = np.random.default_rng(4)
    c2 = rng.standard_normal((2, 3, 3)) + 1j * rng.standard_normal((2, 3, 3))
    c2 = c2 + np.conj(np.swapaxes(c2, -1, -2))
    Hk, mu = c2 + 0.4 * np.eye(3)[None], 0.4
    for n_om in (1, 7):
        om = fermionic_points(n_om, beta)
        Gw = np.eye(3)[None, None] / (1j * om[:, None, None, None]) + c2[None] / (1j * om[:, None, None, None]) ** 2
        taus = np.array([0.0, 0.7, 2.2, beta])
        Gt = green_tau(Gw, Hk, mu, beta, taus)
        ex = -0.5 * np.eye(3)[None, None] + c2[None] * ((2 * taus - beta) / 4)[:, None, None, None]
        assert np.max(np.abs(Gt - ex)) < 1e-13


def test_green_tau_converges_to_the_band_green_function():
    """For the free Dyson solution the sum converges to -U (1 - f) e^{-x tau} U^+ on the whole grid
    (end points 0+ and beta- included), faster than the third power of the frequency count."""
    from oracle.green import green_tau
    spec = cells.tiny(complex_hopping=True, beta=10.0)
    hop, b, Gk, C = cells.inputs(spec)
    Hk = sc.hamiltonian_k(spec, hop)
    err = []
    for n_om in (50, 200, 800):
        Gw = green_dyson(Hk, b.mu, fermionic_points(n_om, spec.beta))
        err.append(np.max(np.abs(green_tau(Gw, Hk, b.mu, spec.beta, sc.tau_grid(spec)) - Gk)))
    assert err[0] / err[1] > 30 and err[1] / err[2] > 30 and err[2] < 1e-8


def test_green_tau_count_at_beta_equals_the_tail_summed_count():
    """-g / N_k sum_k Tr G(k, beta^-) of the reconstruction is the Matsubara count of density_omega,
    for a G with a causal self-energy and a static part (an identity of the two formulas)."""
    from oracle.green import density_omega, green_tau
    spec = cells.two_species()
    hop, b, Gk, C = cells.inputs(spec)
    Hk = sc.hamiltonian_k(spec, hop)
    rng = np.random.default_rng(8)
    n, n_om = spec.N_orb, 12
    X = rng.standard_normal((spec.N_R, n, n)) + 1j * rng.standard_normal((spec.N_R, n, n))
    om = fermionic_points(n_om, spec.beta)
    S = 0.2 * (X @ np.conj(np.swapaxes(X, -1, -2)) / n)[None] / (1j * om[:, None, None, None] - 0.3)
    Y = rng.standard_normal((spec.N_R, n, n))
    Sx = (0.1 * (Y + np.swapaxes(Y, -1, -2))).astype(np.complex128)
    mu = b.mu + 0.1
    Gw = green_dyson(Hk, mu, om, Sigma=S, Sigma_x=Sx)
    Gt = green_tau(Gw, Hk, mu, spec.beta, [spec.beta], Sigma_x=Sx)
    n_tau = -spec.spin / spec.N_R * np.einsum("kaa->", Gt[0]).real
    assert abs(n_tau - density_omega(Gw, Hk, mu, spec.beta, spec.spin, Sx)) < 1e-11 * n_tau
