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
