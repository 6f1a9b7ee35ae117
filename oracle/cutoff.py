"""Real-space cutoff and distance tiers of the product basis (test infrastructure).

Sec. 2 of the paper, with Figs. 1 and 2: a two-point function F^R_{r r'} is taken as zero
when the two arguments are farther apart than R_max; the product basis of the blocks that
remain is largest when both arguments sit on the same muffin-tin sphere, reduced when the
centres are at most the radius of sphere B apart, and smallest between that and the radius
of sphere C (= R_max).  The mesh of k points must be at least as fine as the number of
cells the sphere touches, so that no periodic image of a pair lies inside it.

Written independently of the product library: the search box for lattice images is bounded
with the smallest singular value of the lattice matrix.

Parity status: ``plan_pairs`` is pinned in the tests by closed-form shell counts on a simple
cubic lattice (1, 7, 19, 27, 33 points within radii 0.5, 1, sqrt 2, sqrt 3, 2), by the tier
split of those shells and by the rejection of a mesh that admits two images; the truncated
blocks are the dense oracle blocks (pinned elsewhere) with the functions outside the tier
set to zero, which is the definition itself.
"""
import itertools

import numpy as np

from .polarizability import polarizability_r_block
from .self_energy import self_energy_r_block


def plan_pairs(lattice, positions, species, n_pb, mesh, r_b, r_c, m_tier):
    """Kept blocks (R, A, B, mA, mB) in the order R, A, B.

    R is the mesh index (n1 * N2 + n2) * N3 + n3; the block couples atom A in cell R with
    atom B in cell 0 at the distance min over k of |(n + N k) . a + r_A - r_B|.  m_tier[s] =
    (m_B, m_C) for species s; A = B with R = 0 keeps all n_pb functions.  Raises ValueError
    when a pair has two images within r_c."""
    lat = np.asarray(lattice, dtype=np.float64)
    pos = np.asarray(positions, dtype=np.float64)
    mesh = np.asarray(mesh, dtype=np.int64)
    smin = np.linalg.svd(lat, compute_uv=False).min()
    diam = max(np.linalg.norm(pos[i] - pos[j]) for i in range(len(pos)) for j in range(len(pos)))
    K = [int(np.ceil((r_c + diam) / (mesh[i] * smin))) + 1 for i in range(3)]
    ks = np.array(list(itertools.product(*[range(-k, k + 1) for k in K])), dtype=np.float64)
    out = []
    for n1 in range(mesh[0]):
        for n2 in range(mesh[1]):
            for n3 in range(mesh[2]):
                R = (n1 * mesh[1] + n2) * mesh[2] + n3
                images = (np.array([n1, n2, n3], dtype=np.float64) + ks * mesh) @ lat
                for A in range(len(pos)):
                    for B in range(len(pos)):
                        d = np.linalg.norm(images + pos[A] - pos[B], axis=1)
                        if np.count_nonzero(d <= r_c) > 1:
                            raise ValueError("mesh too coarse for r_c: two images of a pair inside the sphere")
                        dmin = d.min()
                        if dmin > r_c:
                            continue
                        sA, sB = int(species[A]), int(species[B])
                        if A == B and R == 0:
                            mA, mB = n_pb[sA], n_pb[sB]
                        elif dmin <= r_b:
                            mA, mB = m_tier[sA][0], m_tier[sB][0]
                        else:
                            mA, mB = m_tier[sA][1], m_tier[sB][1]
                        out.append((R, A, B, int(mA), int(mB)))
    return np.array(out, dtype=np.int64).reshape(-1, 5)


def polarizability_r_block_cut(GR, spec, C, g, t, R, A, B, mA, mB):
    """Eq. (5) block of a kept pair in its truncated basis: P_IJ for I < mA, J < mB, zero
    elsewhere (P_IJ depends on C^I and C^J only, so truncation is a restriction)."""
    P = polarizability_r_block(GR, spec, C, g, t, R, A, B).copy()
    P[mA:, :] = 0
    P[:, mB:] = 0
    return P


def self_energy_r_block_cut(GR, Wblock, spec, C, t, R, A, B, mA, mB):
    """Eq. (8) block of a kept pair with W_IJ set to zero outside the truncated basis."""
    W = np.array(Wblock, dtype=np.complex128, copy=True)
    W[mA:, :] = 0
    W[:, mB:] = 0
    return self_energy_r_block(GR, W, spec, C, t, R, A, B)
