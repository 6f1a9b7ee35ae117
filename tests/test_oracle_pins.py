"""Pins of the FP64 oracle against mathematics independent of it (CPU only).

Each test checks the oracle against something it does not compute itself:
brute-force supercell diagonalisation, band-basis closed forms, sum rules,
exact integrals, or an identity (Hermiticity, tau-mirror, convolution theorem)
that a plausible slip (dropped term, wrong sign, swapped index, transposed
operand, missing 1/N_k) would break.
"""
import numpy as np
import pytest

import oracle
import synthcell as sc
from oracle.lattice import k_minus_q_index, minus_index
from tests import cells


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# --------------------------------------------------------------------------
# lattice sums
# --------------------------------------------------------------------------
@pytest.mark.parametrize("mk", ["tiny", "two_species"])
def test_k_to_r_matches_bruteforce_supercell(mk):
    spec = cells.tiny(complex_hopping=True) if mk == "tiny" else cells.two_species()
    hop, b, Gk, C = cells.inputs(spec)
    GR = oracle.k_to_r(Gk, spec.mesh)
    taus = sc.tau_grid(spec)
    GRb = oracle.bruteforce.green_R(hop, spec.mesh, spec.N_orb, spec.beta, taus)
    assert relmax(GR, GRb) < 1e-12


def test_r_to_k_single_translation_closed_form():
    mesh = (3, 2, 2)
    NR = 12
    M = sc.random_complex((4, 5), seed=1)
    FR = np.zeros((NR, 4, 5), dtype=np.complex128)
    R0 = 7
    FR[R0] = M
    Fk = oracle.r_to_k(FR, mesh)
    pts = oracle.mesh_points(mesh)
    for k in range(NR):
        ph = np.exp(-2j * np.pi * np.sum(pts[k] * pts[R0] / np.array(mesh)))
        assert np.allclose(Fk[k], ph * M, atol=1e-14)
    back = oracle.k_to_r(Fk, mesh)
    assert relmax(back, FR) < 1e-14


# --------------------------------------------------------------------------
# Green's function input: invariants (pins the generator with the oracle sums)
# --------------------------------------------------------------------------
def test_green_jump_hermiticity_density():
    spec = cells.two_species()
    hop, b, Gk, C = cells.inputs(spec)
    GR = oracle.k_to_r(Gk, spec.mesh)
    mR = minus_index(spec.mesh)
    jump = GR[0] + GR[-1]
    expect = np.zeros_like(jump)
    expect[0] = -np.eye(spec.N_orb)
    assert np.max(np.abs(jump - expect)) < 1e-13
    for R in range(spec.N_R):
        assert np.max(np.abs(GR[:, mR[R]] - np.conj(np.transpose(GR[:, R], (0, 2, 1))))) < 1e-14
    n = oracle.electron_count(GR[-1, 0], spec.spin)
    assert abs(n - spec.spin * spec.N_orb / 2.0) < 1e-9


# --------------------------------------------------------------------------
# polarizability
# --------------------------------------------------------------------------
def _band_P(spec, b, C, g, taus_idx, qs):
    """P^q_IJ(tau) = -(g/N_k) sum_k sum_nn' g(x_n^k, tau) g(x_n'^{k-q}, beta - tau) M^I_nn' conj(M^J_nn')."""
    Nk = spec.N_R
    kmq = k_minus_q_index(spec.mesh)
    taus = sc.tau_grid(spec)
    x = b.eps - b.mu
    orb_off, pb_off = spec.orb_off, spec.pb_off

    def gfac(xx, t):
        return np.where(xx >= 0, np.exp(-np.abs(xx) * t) / (1 + np.exp(-np.abs(xx) * spec.beta)),
                        np.exp(np.minimum(xx, 0) * (spec.beta - t)) / (1 + np.exp(np.minimum(xx, 0) * spec.beta)))

    out = np.zeros((len(taus_idx), len(qs), spec.N_pb, spec.N_pb), dtype=np.complex128)
    for iq, q in enumerate(qs):
        for k in range(Nk):
            U1, U2 = b.U[k], b.U[kmq[k, q]]
            M = np.zeros((spec.N_pb, spec.N_orb, spec.N_orb), dtype=np.complex128)
            for A in range(spec.n_atoms):
                s = spec.species[A]
                rows = slice(orb_off[A], orb_off[A + 1])
                M[pb_off[A]:pb_off[A + 1]] = np.einsum("Iab,an,bm->Inm", C[s], U1[rows], np.conj(U2[rows]))
            for it, ti in enumerate(taus_idx):
                t = taus[ti]
                w = np.outer(gfac(x[k], t), gfac(x[kmq[k, q]], spec.beta - t))
                out[it, iq] += np.einsum("nm,Inm,Jnm->IJ", w, M, np.conj(M))
    return -g / Nk * out


@pytest.mark.parametrize("mk", ["tiny", "two_species"])
def test_polarizability_band_closed_form(mk):
    spec = cells.tiny(complex_hopping=True) if mk == "tiny" else cells.two_species()
    hop, b, Gk, C = cells.inputs(spec)
    taus_idx = [0, 3, spec.n_tau - 1]
    qs = list(range(spec.N_R))
    P = oracle.polarizability_q(Gk, spec, C, spec.spin, taus=taus_idx, qs=qs)
    Pb = _band_P(spec, b, C, spec.spin, taus_idx, qs)
    assert relmax(P, Pb) < 1e-12


def test_polarizability_single_level():
    lat = np.eye(3) * 3.0
    spec = sc.CellSpec("one", lat, np.zeros((1, 3)), np.zeros(1, dtype=np.int64), (1,), (1,), (1, 1, 1),
                       6, 10.0)
    x, beta, g = 0.137, spec.beta, 2.0
    f = 1.0 / (1.0 + np.exp(beta * x))
    taus = sc.tau_grid(spec)
    Gk = (-(1 - f) * np.exp(-x * taus)).reshape(6, 1, 1, 1).astype(np.complex128)
    C = [np.ones((1, 1, 1))]
    P = oracle.polarizability_q(Gk, spec, C, g)
    assert np.allclose(P.ravel(), -g * f * (1 - f), rtol=1e-13, atol=0)


@pytest.mark.parametrize("mk", ["tiny", "two_species"])
def test_polarizability_convolution_theorem_bruteforce(mk):
    """k-space convolution, back-transformed, equals Eq. (5) on the brute-force G^R."""
    spec = cells.tiny() if mk == "tiny" else cells.two_species()
    hop, b, Gk, C = cells.inputs(spec)
    taus_idx = [1, spec.n_tau - 2]
    Pq = oracle.polarizability_q(Gk, spec, C, spec.spin, taus=taus_idx)
    PR_from_q = oracle.k_to_r(Pq, spec.mesh)
    GRb = oracle.bruteforce.green_R(hop, spec.mesh, spec.N_orb, spec.beta, sc.tau_grid(spec))
    PR = oracle.polarizability_r(GRb, spec, C, spec.spin, taus=taus_idx)
    assert relmax(PR_from_q, PR) < 1e-12


def test_polarizability_hermitian_and_mirror():
    spec = cells.two_species()
    hop, b, Gk, C = cells.inputs(spec)
    GR = oracle.k_to_r(Gk, spec.mesh)
    PR = oracle.polarizability_r(GR, spec, C, spec.spin)
    mR = minus_index(spec.mesh)
    nt = spec.n_tau
    for R in range(spec.N_R):
        herm = np.conj(np.transpose(PR[:, R], (0, 2, 1)))
        assert relmax(PR[:, mR[R]], herm) < 1e-13
        mirror = np.transpose(PR[::-1, mR[R]], (0, 2, 1))  # P^{-R}_JI(beta - tau)
        assert relmax(PR[:, R], mirror) < 1e-13
    # block routine agrees with the full one
    blk = oracle.polarizability_r_block(GR, spec, C, spec.spin, 2, 3, 1, 2)
    assert relmax(blk, PR[2, 3][spec.pb_off[1]:spec.pb_off[2], spec.pb_off[2]:spec.pb_off[3]]) < 1e-13


# --------------------------------------------------------------------------
# self-energy
# --------------------------------------------------------------------------
def test_self_energy_local_interaction():
    """W^R_IJ = w delta_R0 delta_IJ: Sigma^k = -w sum_I C^I G^{R=0}_AA C^I for every k."""
    spec = cells.two_species()
    hop, b, Gk, C = cells.inputs(spec)
    w = 0.73
    WR = np.zeros((spec.n_tau, spec.N_R, spec.N_pb, spec.N_pb), dtype=np.complex128)
    WR[:, 0] = w * np.eye(spec.N_pb)
    S = oracle.self_energy_k(Gk, WR, spec, C, taus=[2])
    GR = oracle.bruteforce.green_R(hop, spec.mesh, spec.N_orb, spec.beta, sc.tau_grid(spec))
    expect = np.zeros((spec.N_orb, spec.N_orb), dtype=np.complex128)
    for A in range(spec.n_atoms):
        o = slice(spec.orb_off[A], spec.orb_off[A + 1])
        CA = C[spec.species[A]]
        expect[o, o] = -w * np.einsum("Iab,bc,Icd->ad", CA, GR[2, 0][o, o], CA)
    for k in range(spec.N_R):
        assert relmax(S[0, k], expect) < 1e-12


def test_self_energy_rank_one_single_translation():
    """W^R_IJ(tau) = u_I v_J delta_{R,R0}: Sigma^R_AB = -delta_{R,R0} U_A G^{R0}_AB V_B."""
    spec = cells.two_species()
    hop, b, Gk, C = cells.inputs(spec)
    rng = np.random.default_rng(3)
    u = rng.standard_normal(spec.N_pb) + 0.3j * rng.standard_normal(spec.N_pb)
    v = rng.standard_normal(spec.N_pb) - 0.2j * rng.standard_normal(spec.N_pb)
    R0 = 4
    WR = np.zeros((spec.n_tau, spec.N_R, spec.N_pb, spec.N_pb), dtype=np.complex128)
    WR[:, R0] = np.outer(u, v)
    t = 5
    Sk = oracle.self_energy_k(Gk, WR, spec, C, taus=[t])
    SR = oracle.k_to_r(Sk, spec.mesh)[0]
    GR = oracle.bruteforce.green_R(hop, spec.mesh, spec.N_orb, spec.beta, sc.tau_grid(spec))
    for R in range(spec.N_R):
        exp = np.zeros((spec.N_orb, spec.N_orb), dtype=np.complex128)
        if R == R0:
            for A in range(spec.n_atoms):
                for B in range(spec.n_atoms):
                    oa = slice(spec.orb_off[A], spec.orb_off[A + 1])
                    ob = slice(spec.orb_off[B], spec.orb_off[B + 1])
                    UA = np.einsum("I,Iab->ab", u[spec.pb_off[A]:spec.pb_off[A + 1]], C[spec.species[A]])
                    VB = np.einsum("J,Jab->ab", v[spec.pb_off[B]:spec.pb_off[B + 1]], C[spec.species[B]])
                    exp[oa, ob] = -UA @ GR[t, R0][oa, ob] @ VB.T
        assert np.max(np.abs(SR[R] - exp)) < 1e-12 * max(1.0, np.max(np.abs(exp)))


def test_self_energy_convolution_theorem_and_hermitian():
    spec = cells.two_species()
    hop, b, Gk, C = cells.inputs(spec)
    WR = sc.w_tensor(spec)
    taus_idx = [0, 4]
    Sk = oracle.self_energy_k(Gk, WR, spec, C, taus=taus_idx)
    for it in range(2):
        for k in range(spec.N_R):
            assert relmax(Sk[it, k], np.conj(Sk[it, k].T)) < 1e-13
    GRb = oracle.bruteforce.green_R(hop, spec.mesh, spec.N_orb, spec.beta, sc.tau_grid(spec))
    SR = oracle.self_energy_r(GRb, WR, spec, C, taus=taus_idx)
    assert relmax(oracle.k_to_r(Sk, spec.mesh), SR) < 1e-12
    blk = oracle.self_energy_r_block(GRb, WR[4, 3][spec.pb_off[0]:spec.pb_off[1], spec.pb_off[1]:spec.pb_off[2]],
                                     spec, C, 4, 3, 0, 1)
    assert relmax(blk, SR[1, 3][spec.orb_off[0]:spec.orb_off[1], spec.orb_off[1]:spec.orb_off[2]]) < 1e-13


# --------------------------------------------------------------------------
# tau -> Matsubara
# --------------------------------------------------------------------------
def test_filon_zero_frequency_is_trapezoid():
    tau = np.sort(np.concatenate([[0.0, 7.0], np.random.default_rng(1).uniform(0, 7.0, 9)]))
    T = oracle.filon_matrix(tau, [0.0])
    F = np.cos(tau) + tau ** 2
    assert abs(T[0] @ F - np.trapezoid(F, tau)) < 1e-13


def test_filon_exact_for_linear_functions():
    beta = 9.0
    tau = np.sort(np.concatenate([[0.0, beta], np.random.default_rng(2).uniform(0, beta, 13)]))
    for w in oracle.fermionic_frequencies(5, beta).tolist() + oracle.bosonic_frequencies(4, beta).tolist():
        a, c = 0.7 - 0.2j, -1.3 + 0.4j
        F = a + c * tau
        T = oracle.filon_matrix(tau, [w])
        if w == 0:
            exact = a * beta + c * beta ** 2 / 2
        else:
            e = np.exp(1j * w * beta)
            exact = a * (e - 1) / (1j * w) + c * (beta * e / (1j * w) + (e - 1) / w ** 2)
        assert abs(T[0] @ F - exact) < 1e-12 * max(1.0, abs(exact))


def test_filon_second_order_convergence():
    beta, x = 10.0, 0.8
    w = oracle.fermionic_frequencies(3, beta)
    exact = (np.exp((1j * w - x) * beta) - 1) / (1j * w - x)
    errs = []
    for n in (41, 81, 161):
        tau = beta * np.arange(n) / (n - 1)
        T = oracle.filon_matrix(tau, w)
        errs.append(np.max(np.abs(T @ np.exp(-x * tau) - exact)))
    assert errs[0] / errs[1] > 3.8 and errs[1] / errs[2] > 3.8


def test_filon_lindhard_tiny():
    """T applied to the oracle P^q(tau) approaches the Lindhard P^q(i nu) as h^2."""
    errs = []
    for n_tau in (101, 201):
        spec = cells.tiny(n_tau=n_tau, beta=4.0)
        hop, b, Gk, C = cells.inputs(spec)
        q = 3
        Pq = oracle.polarizability_q(Gk, spec, C, spec.spin, qs=[q])[:, 0]  # [tau][I][J]
        nu = oracle.bosonic_frequencies(4, spec.beta)
        Pw = oracle.apply_tau_to_omega(oracle.filon_matrix(sc.tau_grid(spec), nu), Pq)
        kmq = k_minus_q_index(spec.mesh)
        x = b.eps - b.mu
        f = sc.fermi(x, spec.beta)
        ex = np.zeros_like(Pw)
        for k in range(spec.N_R):
            k2 = kmq[k, q]
            M = np.zeros((spec.N_pb, spec.N_orb, spec.N_orb), dtype=np.complex128)
            for A in range(spec.n_atoms):
                rows = slice(spec.orb_off[A], spec.orb_off[A + 1])
                M[spec.pb_off[A]:spec.pb_off[A + 1]] = np.einsum("Iab,an,bm->Inm", C[0], b.U[k][rows],
                                                                np.conj(b.U[k2][rows]))
            for m, v in enumerate(nu):
                d = x[k][:, None] - x[k2][None, :]
                num = f[k][:, None] - f[k2][None, :]
                with np.errstate(divide="ignore", invalid="ignore"):
                    fac = num / (1j * v - d)
                if v == 0:
                    deg = np.abs(d) < 1e-12
                    fac = np.where(deg, spec.beta * f[k][:, None] * (1 - f[k][:, None]), fac)
                ex[m] += np.einsum("nm,Inm,Jnm->IJ", fac, M, np.conj(M))
        ex *= -spec.spin / spec.N_R
        errs.append(np.max(np.abs(Pw - ex)) / np.max(np.abs(ex)))
    assert errs[0] < 1e-3
    assert errs[0] / errs[1] > 3.5


def test_electron_count_sign_and_spin():
    spec = cells.tiny()
    hop, b, Gk, C = cells.inputs(spec)
    GR = oracle.k_to_r(Gk, spec.mesh)
    assert abs(oracle.electron_count(GR[-1, 0], 2.0) - spec.N_orb) < 1e-9
    assert abs(oracle.electron_count(GR[-1, 0], 1.0) - spec.N_orb / 2) < 1e-9


def test_filon_fermionic_resolvent_tiny():
    """T at the oracle's fermionic frequencies, applied to the band G(k, tau) of the tiny cell,
    approaches the resolvent G(k, i w_n) = U (i w_n - (eps - mu))^-1 U^+ as h^2.  The closed form
    needs exp(i w_n beta) = -1 (for other w the integral of -(1 - f) exp(-x tau) is
    (1 - f)(1 - exp(-x beta)) / (i w - x) times a phase), so it pins the frequency set with T."""
    errs = []
    for n_tau in (101, 201):
        spec = cells.tiny(n_tau=n_tau, beta=4.0, complex_hopping=True)
        hop, b, Gk, C = cells.inputs(spec)
        w = oracle.fermionic_frequencies(5, spec.beta)
        Gw = oracle.apply_tau_to_omega(oracle.filon_matrix(sc.tau_grid(spec), w), Gk)  # [m][k][a][b]
        x = b.eps - b.mu
        ex = np.einsum("kan,mkn,kbn->mkab", b.U, 1.0 / (1j * w[:, None, None] - x[None]), np.conj(b.U))
        errs.append(relmax(Gw, ex))
    assert errs[0] < 1e-3
    assert errs[0] / errs[1] > 3.5


def test_bosonic_frequencies_annihilate_constants():
    """A tau-independent function integrates to beta F at nu_0 and to zero at every other bosonic
    frequency (exp(i nu_m beta) = 1); T is exact on constants, so this holds to rounding."""
    beta = 6.5
    tau = beta * np.arange(9) / 8
    nu = oracle.bosonic_frequencies(6, beta)
    Fw = oracle.filon_matrix(tau, nu) @ np.full(9, 0.3 - 0.1j)
    assert abs(Fw[0] - beta * (0.3 - 0.1j)) < 1e-13
    assert np.max(np.abs(Fw[1:])) < 1e-13
    assert np.all(np.diff(nu) > 0) and nu[0] == 0.0
