"""Pins of the interstitial-block oracle (Eqs. (6), (7), (9), (10))."""
import numpy as np

import synthcell as sc
from oracle.interstitial import polarizability_int, self_energy_int
from oracle.lattice import minus_index
from tests import cells


def _blocks(spec, n_g, seed, n_prod=False):
    no = spec.N_pb if n_prod else spec.N_orb
    sh = (spec.n_tau, spec.N_R)
    return (sc.random_complex(sh + (no, n_g), seed), sc.random_complex(sh + (n_g, no), seed + 1),
            sc.random_complex(sh + (n_g, n_g), seed + 2))


def test_int_int_hadamard_forms():
    spec = cells.two_species()
    C = sc.coefficients(spec)
    og, go, gg = _blocks(spec, 5, 10)
    pg, gp, pgg = polarizability_int(og, go, gg, spec, C, 2.0)
    mR = minus_index(spec.mesh)
    nt = spec.n_tau
    for t in range(nt):
        for R in range(spec.N_R):
            assert np.max(np.abs(pgg[t, R] + 2.0 * gg[t, R] * gg[nt - 1 - t, mR[R]].T)) < 1e-13
    wpg, wgp, wgg = _blocks(spec, 5, 20, n_prod=True)
    sog, sgo, sgg = self_energy_int(og, go, gg, wpg, wgp, wgg, spec, C)
    assert np.max(np.abs(sgg + gg * wgg)) < 1e-13


def test_one_orbital_mt_int_closed_form():
    spec = sc.CellSpec("one", 3.0 * np.eye(3), np.zeros((1, 3)), np.array([0]), (1,), (1,), (2, 1, 1), 4, 10.0,
                       config_id=12)
    c = 0.7
    C = [np.array([[[c]]])]
    og, go, gg = _blocks(spec, 3, 30)
    pg, gp, pgg = polarizability_int(og, go, gg, spec, C, 2.0)
    mR = minus_index(spec.mesh)
    for t in range(4):
        for R in range(2):
            want = -2.0 * c * og[t, R, 0, :] * go[3 - t, mR[R], :, 0]
            assert np.max(np.abs(pg[t, R, 0, :] - want)) < 1e-14
    wpg, wgp, wgg = _blocks(spec, 3, 40, n_prod=True)
    sog, sgo, sgg = self_energy_int(og, go, gg, wpg, wgp, wgg, spec, C)
    assert np.max(np.abs(sog[:, :, 0, :] + c * og[:, :, 0, :] * wpg[:, :, 0, :])) < 1e-14
    assert np.max(np.abs(sgo[:, :, :, 0] + c * go[:, :, :, 0] * wgp[:, :, :, 0])) < 1e-14


def test_mixed_blocks_obey_the_tau_mirror():
    spec = cells.two_species()
    C = sc.coefficients(spec)
    og, go, gg = _blocks(spec, 4, 50)
    pg, gp, _ = polarizability_int(og, go, gg, spec, C, 2.0)
    mR = minus_index(spec.mesh)
    nt = spec.n_tau
    for t in range(nt):
        for R in range(spec.N_R):
            assert np.max(np.abs(gp[t, R] - pg[nt - 1 - t, mR[R]].T)) < 1e-13 * np.max(np.abs(gp))
