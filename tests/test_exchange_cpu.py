"""Pins of the static (exchange) self-energy oracle: Eq. (8) with W~ -> V, G(tau) -> -G(beta)."""
import numpy as np

import oracle
import synthcell as sc
from tests import cells


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _one_function_cell():
    return sc.CellSpec("one", 3.0 * np.eye(3), np.zeros((1, 3)), np.array([0]), (1,), (1,), (2, 1, 1), 4, 10.0,
                       config_id=12, request_id=0, complex_hopping=False)


def test_one_orbital_one_function_closed_form():
    spec = _one_function_cell()
    c = 0.8
    C = [np.array([[[c]]])]
    rng = np.random.default_rng(11)
    GR = rng.standard_normal((4, 2, 1, 1)) + 1j * rng.standard_normal((4, 2, 1, 1))
    VR = rng.standard_normal((2, 1, 1)) + 1j * rng.standard_normal((2, 1, 1))
    Sx = oracle.exchange_r(GR, VR, spec, C)
    for R in range(2):
        assert abs(Sx[R, 0, 0] - c * c * GR[-1, R, 0, 0] * VR[R, 0, 0]) < 1e-15   # + sign: -(-G(beta))


def test_local_interaction_only_at_origin():
    spec = cells.two_species()
    hop, b, Gk, C = cells.inputs(spec)
    v = 0.61
    VR = np.zeros((spec.N_R, spec.N_pb, spec.N_pb), dtype=np.complex128)
    VR[0] = v * np.eye(spec.N_pb)
    GRb = oracle.bruteforce.green_R(hop, spec.mesh, spec.N_orb, spec.beta, sc.tau_grid(spec))
    Sx = oracle.exchange_r(GRb, VR, spec, C)
    assert np.max(np.abs(Sx[1:])) == 0.0
    expect = np.zeros((spec.N_orb, spec.N_orb), dtype=np.complex128)
    for A in range(spec.n_atoms):
        o = slice(spec.orb_off[A], spec.orb_off[A + 1])
        CA = C[spec.species[A]]
        expect[o, o] = v * np.einsum("Iab,bc,Icd->ad", CA, GRb[-1, 0][o, o], CA)
    assert relmax(Sx[0], expect) < 1e-12


def test_real_and_momentum_space_forms_agree():
    spec = cells.two_species()
    hop, b, Gk, C = cells.inputs(spec)
    A = sc.w_amplitude(spec)
    sR, _ = sc.w_factors(spec)
    VR = (sR[:, None, None] * A[None]).astype(np.complex128)
    Sk = oracle.exchange_k(Gk, VR, spec, C)
    GRb = oracle.bruteforce.green_R(hop, spec.mesh, spec.N_orb, spec.beta, sc.tau_grid(spec))
    SR = oracle.exchange_r(GRb, VR, spec, C)
    assert relmax(oracle.k_to_r(Sk[None], spec.mesh)[0], SR) < 1e-12
    for k in range(spec.N_R):
        assert relmax(Sk[k], np.conj(Sk[k].T)) < 1e-13
