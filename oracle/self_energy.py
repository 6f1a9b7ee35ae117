"""Self-energy (oracle, test infrastructure).

self_energy_k -- the plain k-space definition at fixed imaginary time (the
structure of Eq. (3) with the frequency convolution replaced by the product
at equal tau):

    Sigma^k_ab(tau) = -(1 / N_k) sum_q sum_{a',I in A; b',J in B}
                      C^I_aa' G^{k-q}_a'b'(tau) W^q_IJ(tau) C^J_bb',
    W^q = sum_R exp(-i q.R) W^R   (formed here by the oracle's own sum)

self_energy_r -- Eq. (8) (MT-MT) in real space, with the Green's function
carrying the summed orbital indices (a', b') and W at the same tau:

    Sigma^R_ab(tau) = -sum C^I_aa' G^R_a'b'(tau) W^R_IJ(tau) C^J_bb'

Pins (tests): a purely local W (W^R_IJ = w delta_R0 delta_IJ) reduces to one
matrix sandwich per atom; a rank-one single-R W reduces to a product of two
atom-local matrices with the brute-force supercell G^R; Hermiticity.
"""
import numpy as np

from .fourier import r_to_k
from .lattice import k_minus_q_index
from .polarizability import _layout, _species_groups


def _contract_S(X, Wm, spec, C):
    """sum_{a' b' I J} C^I_aa' X_a'b' Wm_IJ C^J_bb' over all atom pairs (no sign)."""
    orb_off, pb_off, species = _layout(spec)
    No = int(orb_off[-1])
    out = np.zeros((No, No), dtype=np.complex128)
    groups = _species_groups(spec)
    for sA, LA in groups.items():
        nA = int(orb_off[LA[0] + 1] - orb_off[LA[0]])
        mA = C[sA].shape[0]
        rowsA = np.concatenate([np.arange(orb_off[a], orb_off[a + 1]) for a in LA])
        prowsA = np.concatenate([np.arange(pb_off[a], pb_off[a + 1]) for a in LA])
        for sB, LB in groups.items():
            nB = int(orb_off[LB[0] + 1] - orb_off[LB[0]])
            mB = C[sB].shape[0]
            rowsB = np.concatenate([np.arange(orb_off[b], orb_off[b + 1]) for b in LB])
            prowsB = np.concatenate([np.arange(pb_off[b], pb_off[b + 1]) for b in LB])
            X4 = X[np.ix_(rowsA, rowsB)].reshape(len(LA), nA, len(LB), nB)
            W4 = Wm[np.ix_(prowsA, prowsB)].reshape(len(LA), mA, len(LB), mB)
            z = np.einsum("AIBJ,Jbc->AIBbc", W4, C[sB], optimize=True)
            t = np.einsum("AxBc,AIBbc->AIxBb", X4, z, optimize=True)
            s = np.einsum("Iax,AIxBb->AaBb", C[sA], t, optimize=True)
            out[np.ix_(rowsA, rowsB)] += s.reshape(len(LA) * nA, len(LB) * nB)
    return out


def self_energy_k(Gk, WR, spec, C, taus=None, ks=None):
    """Sigma^k(tau); returns [len(taus)][len(ks)][No][No].  WR: [N_tau][N_R][Np][Np]."""
    nt, Nk = Gk.shape[0], Gk.shape[1]
    taus = range(nt) if taus is None else taus
    ks = range(Nk) if ks is None else ks
    kmq = k_minus_q_index(spec.mesh)
    No = int(np.asarray(spec.orb_off)[-1])
    out = np.zeros((len(taus), len(ks), No, No), dtype=np.complex128)
    for it, t in enumerate(taus):
        Wq = r_to_k(WR[t], spec.mesh)  # [q][Np][Np]
        for ik, k in enumerate(ks):
            acc = np.zeros((No, No), dtype=np.complex128)
            for q in range(Nk):
                acc += _contract_S(Gk[t, kmq[k, q]], Wq[q], spec, C)
            out[it, ik] = -acc / Nk
    return out


def self_energy_r(GR, WR, spec, C, taus=None, Rs=None):
    """Eq. (8): Sigma^R(tau) = -C G^R(tau) W^R(tau) C blockwise; returns [taus][Rs][No][No]."""
    nt, NR = GR.shape[0], GR.shape[1]
    taus = range(nt) if taus is None else taus
    Rs = range(NR) if Rs is None else Rs
    No = int(np.asarray(spec.orb_off)[-1])
    out = np.zeros((len(taus), len(Rs), No, No), dtype=np.complex128)
    for it, t in enumerate(taus):
        for iR, R in enumerate(Rs):
            out[it, iR] = -_contract_S(GR[t, R], WR[t, R], spec, C)
    return out


def self_energy_r_block(GR, Wblock, spec, C, t, R, A, B):
    """One block Sigma^R_{a in A, b in B}(tau_t) of Eq. (8) as an explicit sum.

    Wblock is W^R_{I in A, J in B}(tau_t) (m_A x m_B).
    """
    orb_off, pb_off, species = _layout(spec)
    CA, CB = C[int(species[A])], C[int(species[B])]
    X = GR[t, R][orb_off[A]:orb_off[A + 1], orb_off[B]:orb_off[B + 1]]
    return -np.einsum("Iax,xy,IJ,Jby->ab", CA, X, Wblock, CB, optimize=True)
