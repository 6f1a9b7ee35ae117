"""Pins of the real-space cutoff planner of the oracle (Sec. 2, Figs. 1 and 2), CPU only.

The planner is checked against counts that do not come from it: on a simple cubic lattice
(one atom, a = 1) the lattice points within distance r of the origin are 1, 7, 19, 27, 33
for r = 0.5, 1, sqrt 2, sqrt 3, 2 (shells of 1, 6, 12, 8, 6 points); the tier split follows
the shells; a mesh of 2 along an axis puts two images of the pair at distance 1 inside a
sphere of radius 1 and must be refused; and the kept list is closed under the exchange
(R, A, B) -> (-R, B, A) with the tiers exchanged too.
"""
import numpy as np
import pytest

import oracle
import synthcell as sc
from oracle.lattice import minus_index


@pytest.mark.parametrize("r,count", [(0.5, 1), (1.0, 7), (1.5, 19), (1.8, 27), (2.05, 33)])
def test_simple_cubic_shell_counts(r, count):
    p = oracle.plan_pairs(np.eye(3), np.zeros((1, 3)), [0], [20], (5, 5, 5), min(r, 1.2), r, [[10, 5]])
    assert len(p) == count


def test_simple_cubic_tiers_follow_the_shells():
    p = oracle.plan_pairs(np.eye(3), np.zeros((1, 3)), [0], [20], (5, 5, 5), 1.2, 1.8, [[10, 5]])
    m = p[:, 3]
    # same atom, same cell: all 20 functions; 6 neighbours at 1 <= r_b: 10; 12 + 8 at sqrt 2, sqrt 3: 5
    assert (np.count_nonzero(m == 20), np.count_nonzero(m == 10), np.count_nonzero(m == 5)) == (1, 6, 20)
    assert np.array_equal(p[:, 3], p[:, 4])
    assert p[m == 20][0, 0] == 0


def test_coarse_mesh_is_refused():
    with pytest.raises(ValueError):
        oracle.plan_pairs(np.eye(3), np.zeros((1, 3)), [0], [20], (2, 2, 2), 1.0, 1.0, [[10, 5]])


@pytest.mark.parametrize("kind", ["si8", "si24"])
def test_list_is_closed_under_mirror_and_counts_three_shells(kind):
    spec = sc.serving_cell(kind, 16, 0)
    p = oracle.plan_pairs(spec.lattice, spec.positions, spec.species, spec.n_pb, spec.mesh, 2.5, 4.6,
                          [[60, 16]])
    mi = minus_index(spec.mesh)
    keep = {tuple(r) for r in p.tolist()}
    for R, A, B, mA, mB in p.tolist():
        assert (int(mi[R]), B, A, mB, mA) in keep
    # diamond Si: 4 neighbours at 2.35 A, 12 at 3.84 A, 12 at 4.50 A within 4.6 A, plus the atom itself
    assert len(p) == 29 * spec.n_atoms
    assert np.count_nonzero(p[:, 3] == 60) == 5 * spec.n_atoms


def _truncated(spec, C, m_of_species):
    """The same cell with the basis of species s cut to its first m_of_species[s] functions."""
    t = sc.CellSpec(spec.name + "_cut", spec.lattice, spec.positions, spec.species, spec.n_orb,
                    tuple(int(m) for m in m_of_species), spec.mesh, spec.n_tau, spec.beta, spec.spin,
                    spec.config_id, spec.request_id, spec.complex_hopping)
    return t, [np.asarray(C[s])[:m] for s, m in enumerate(m_of_species)]


def _two_species():
    from tests import cells
    spec = cells.two_species(n_pb=(7, 6))
    hop, b, Gk, C = cells.inputs(spec)
    return spec, oracle.k_to_r(Gk, spec.mesh), C


@pytest.mark.parametrize("t,R,A,B", [(1, 2, 0, 1), (5, 0, 2, 2), (0, 3, 1, 0)])
def test_cut_blocks_equal_blocks_of_the_truncated_basis(t, R, A, B):
    """A block kept in a reduced basis is the block of the cell whose product basis holds only the
    first mA / mB functions (zero outside them), for P and Sigma: truncating the basis restricts
    Eqs. (5) and (8), it does not change the kept entries."""
    spec, GR, C = _two_species()
    mA, mB = 4, 3
    sA, sB = spec.species[A], spec.species[B]
    m_cut = [spec.n_pb[0], spec.n_pb[1]]
    m_cut[sA], m_cut[sB] = mA, mB
    if sA == sB:
        mB = mA
        m_cut[sA] = mA
    tspec, tC = _truncated(spec, C, m_cut)
    Pc = oracle.polarizability_r_block_cut(GR, spec, C, spec.spin, t, R, A, B, mA, mB)
    Pt = oracle.polarizability_r_block(GR, tspec, tC, spec.spin, t, R, A, B)
    assert Pc.shape == (spec.n_pb[sA], spec.n_pb[sB])
    assert np.max(np.abs(Pc[:mA, :mB] - Pt)) <= 1e-14 * np.max(np.abs(Pt))
    assert not np.any(Pc[mA:, :]) and not np.any(Pc[:, mB:])
    W = sc.random_complex((spec.n_pb[sA], spec.n_pb[sB]), seed=17)
    Sc = oracle.self_energy_r_block_cut(GR, W, spec, C, t, R, A, B, mA, mB)
    St = oracle.self_energy_r_block(GR, W[:mA, :mB], tspec, tC, t, R, A, B)
    assert np.max(np.abs(Sc - St)) <= 1e-14 * np.max(np.abs(St))


def test_cut_blocks_one_orbital_closed_form():
    """One orbital per atom, C^I = c_I: P^R_IJ(tau) = -g c_I c_J G^R_AB(tau) G^{-R}_BA(beta - tau) for
    I < mA, J < mB and zero elsewhere; Sigma^R_AB(tau) = -G^R_AB(tau) sum_{I < mA, J < mB} c_I W_IJ c_J."""
    lat = np.diag([2.0, 2.1, 2.2])
    pos = np.array([[0.0, 0.0, 0.0], [0.9, 1.0, 1.1]])
    spec = sc.CellSpec("one_orb", lat, pos, np.array([0, 0]), (1,), (5,), (2, 1, 1), 4, 3.0)
    rng = np.random.default_rng(5)
    GR = rng.standard_normal((4, 2, 2, 2)) + 1j * rng.standard_normal((4, 2, 2, 2))
    c = rng.standard_normal(5)
    C = [c.reshape(5, 1, 1)]
    t, R, A, B, mA, mB = 1, 1, 0, 1, 3, 3
    mR = minus_index(spec.mesh)[R]
    P = oracle.polarizability_r_block_cut(GR, spec, C, 2.0, t, R, A, B, mA, mB)
    ex = np.zeros((5, 5), dtype=np.complex128)
    ex[:mA, :mB] = -2.0 * np.outer(c[:mA], c[:mB]) * GR[t, R, A, B] * GR[3 - t, mR, B, A]
    assert np.max(np.abs(P - ex)) < 1e-14
    W = rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5))
    S = oracle.self_energy_r_block_cut(GR, W, spec, C, t, R, A, B, mA, mB)
    assert abs(S[0, 0] + GR[t, R, A, B] * (c[:mA] @ W[:mA, :mB] @ c[:mB])) < 1e-14
