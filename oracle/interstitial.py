"""Interstitial (real-space grid) blocks of P and Sigma (oracle, test infrastructure).

Eqs. (6), (7), (9), (10): when one or both space arguments lie on interstitial grid points r, r',
the MT expressions keep their form with the product-basis coefficient of a grid point replaced by
a delta: a point carries one "orbital" (the value of G there) and one "product function" (the
product of two G values there).  So the oracle treats every grid point as a pseudo-atom with one
orbital, one product function and coefficient 1, appends them after the muffin-tin atoms, and
applies its own Eq. (5) and Eq. (8) to the extended matrices; the blocks with a grid index are
Eqs. (6), (7) (P) and (9), (10) (Sigma).  The second G of P is read as in Eq. (5) (G^{-R} with
swapped indices at beta - tau) and W is taken at the same tau as G.

Block layout (per tau and R): G_og [N_orb][n_g] = G^R_{tL; r'}, G_go [n_g][N_orb] = G^R_{r; tL},
G_gg [n_g][n_g]; P and W likewise with N_pb (P_pg, P_gp, P_gg); Sigma like G.

Parity status: pinned in the tests by the INT-INT closed forms (Hadamard products), the
one-orbital MT-INT closed form, and the tau-mirror identity P^R_{r; tK}(tau) = P^{-R}_{tK; r}(beta - tau)
between the two mixed blocks.
"""
from types import SimpleNamespace

import numpy as np

from .polarizability import polarizability_r
from .self_energy import self_energy_r


def extended(spec, C, n_g):
    """Layout of the cell with n_g grid pseudo-atoms appended, and the coefficients with the
    grid species (one orbital, one function, coefficient 1) appended."""
    norb = list(np.asarray(spec.atom_norb)) + [1] * n_g
    npb = list(np.asarray(spec.atom_npb)) + [1] * n_g
    species = list(np.asarray(spec.species)) + [spec.n_species] * n_g
    ns = SimpleNamespace(orb_off=np.concatenate([[0], np.cumsum(norb)]).astype(np.int64),
                         pb_off=np.concatenate([[0], np.cumsum(npb)]).astype(np.int64),
                         species=np.asarray(species), mesh=spec.mesh)
    return ns, list(C) + [np.ones((1, 1, 1))]


def _assemble(oo_shape, og, go, gg):
    nt, nr, no, ng = og.shape
    X = np.zeros((nt, nr, no + ng, no + ng), dtype=np.complex128)
    X[:, :, :no, no:] = og
    X[:, :, no:, :no] = go
    X[:, :, no:, no:] = gg
    return X


def polarizability_int(G_og, G_go, G_gg, spec, C, g, taus=None, Rs=None):
    """(P_pg, P_gp, P_gg) of Eqs. (6), (7) at the given tau and R indices (default all)."""
    n_g = G_gg.shape[-1]
    ns, Cx = extended(spec, C, n_g)
    P = polarizability_r(_assemble(None, G_og, G_go, G_gg), ns, Cx, g, taus, Rs)
    Np = spec.N_pb
    return P[:, :, :Np, Np:], P[:, :, Np:, :Np], P[:, :, Np:, Np:]


def self_energy_int(G_og, G_go, G_gg, W_pg, W_gp, W_gg, spec, C, taus=None, Rs=None):
    """(S_og, S_go, S_gg) of Eqs. (9), (10) at the given tau and R indices (default all)."""
    n_g = G_gg.shape[-1]
    ns, Cx = extended(spec, C, n_g)
    S = self_energy_r(_assemble(None, G_og, G_go, G_gg), _assemble(None, W_pg, W_gp, W_gg), ns, Cx, taus, Rs)
    No = spec.N_orb
    return S[:, :, :No, No:], S[:, :, No:, :No], S[:, :, No:, No:]
