"""Polarizability (oracle, test infrastructure).

polarizability_q -- the plain k-space definition at fixed imaginary time, i.e.
the structure of Eq. (1) with the frequency convolution replaced by the
product at (tau, beta - tau):

    P^q_IJ(tau) = -(g / N_k) sum_k sum_{a,b in A; c,d in B}
                  C^I_ab G^k_ac(tau) G^{k-q}_db(beta - tau) C^J_cd

polarizability_r -- Eq. (5) (MT-MT) read literally in real space, with the
second Green's function taken at -R with its indices exchanged:

    P^R_IJ(tau) = -g sum C^I_ab G^R_ac(tau) G^{-R}_db(beta - tau) C^J_cd

(I on atom A, J on atom B; a, b orbitals of A; c, d orbitals of B; g the spin
sum of Eq. (5)).  The two are related by the discrete convolution theorem on
the Born-von Karman torus.

Pins (tests): band-basis closed form of P^q(tau) from the eigenvectors of H(k);
single-level closed form P = -g f (1 - f); real-space Eq. (5) evaluated on the
brute-force supercell G^R; Hermiticity and the tau-mirror identity.
"""
import numpy as np

from .lattice import k_minus_q_index, minus_index


def _layout(spec):
    """(orb_off, pb_off, species) as plain arrays from any cell description."""
    return (np.asarray(spec.orb_off), np.asarray(spec.pb_off), np.asarray(spec.species))


def _pair_block(CA, CB, X4, Y4):
    """sum_{a,b,c,d} CA[I,a,b] X4[A,a,B,c] Y4[B,d,A,b] CB[J,c,d] -> [A,I,B,J]."""
    t1 = np.einsum("Iab,AaBc->AIbBc", CA, X4, optimize=True)
    t2 = np.einsum("AIbBc,BdAb->AIBcd", t1, Y4, optimize=True)
    return np.einsum("AIBcd,Jcd->AIBJ", t2, CB, optimize=True)


def _species_groups(spec):
    _, _, species = _layout(spec)
    groups = {}
    for at, s in enumerate(species):
        groups.setdefault(int(s), []).append(at)
    return groups


def _contract_P(X, Y, spec, C):
    """Real-space or k-space pair sum for one (X, Y) pair of full matrices.

    X[a, c] plays G(tau) with a on atom A, c on atom B; Y[d, b] plays
    G(beta - tau) with d on atom B, b on atom A.  Returns the N_pb x N_pb block
    matrix sum_{abcd} C^I_ab X_ac Y_db C^J_cd (no prefactor).
    """
    orb_off, pb_off, species = _layout(spec)
    Np = int(pb_off[-1])
    out = np.zeros((Np, Np), dtype=np.complex128)
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
            Y4 = Y[np.ix_(rowsB, rowsA)].reshape(len(LB), nB, len(LA), nA)
            blk = _pair_block(C[sA], C[sB], X4, Y4).reshape(len(LA) * mA, len(LB) * mB)
            out[np.ix_(prowsA, prowsB)] += blk
    return out


def polarizability_q(Gk, spec, C, g, taus=None, qs=None):
    """P^q(tau) for the requested tau and q indices; returns [len(taus)][len(qs)][Np][Np].

    Gk: [N_tau][N_k][N_orb][N_orb] complex.
    """
    nt, Nk = Gk.shape[0], Gk.shape[1]
    taus = range(nt) if taus is None else taus
    qs = range(Nk) if qs is None else qs
    kmq = k_minus_q_index(spec.mesh)
    Np = int(np.asarray(spec.pb_off)[-1])
    out = np.zeros((len(taus), len(qs), Np, Np), dtype=np.complex128)
    for it, t in enumerate(taus):
        tm = nt - 1 - t
        for iq, q in enumerate(qs):
            acc = np.zeros((Np, Np), dtype=np.complex128)
            for k in range(Nk):
                acc += _contract_P(Gk[t, k], Gk[tm, kmq[k, q]], spec, C)
            out[it, iq] = -g / Nk * acc
    return out


def polarizability_r(GR, spec, C, g, taus=None, Rs=None):
    """Eq. (5): P^R(tau) from G^R(tau) and G^{-R}(beta - tau); returns [taus][Rs][Np][Np]."""
    nt, NR = GR.shape[0], GR.shape[1]
    taus = range(nt) if taus is None else taus
    Rs = range(NR) if Rs is None else Rs
    mR = minus_index(spec.mesh)
    Np = int(np.asarray(spec.pb_off)[-1])
    out = np.zeros((len(taus), len(Rs), Np, Np), dtype=np.complex128)
    for it, t in enumerate(taus):
        for iR, R in enumerate(Rs):
            out[it, iR] = -g * _contract_P(GR[t, R], GR[nt - 1 - t, mR[R]], spec, C)
    return out


def polarizability_r_block(GR, spec, C, g, t, R, A, B):
    """One atom-pair block P^R_{I in A, J in B}(tau_t) of Eq. (5), written as explicit sums."""
    orb_off, pb_off, species = _layout(spec)
    nt = GR.shape[0]
    mR = minus_index(spec.mesh)
    CA, CB = C[int(species[A])], C[int(species[B])]
    X = GR[t, R][orb_off[A]:orb_off[A + 1], orb_off[B]:orb_off[B + 1]]
    Y = GR[nt - 1 - t, mR[R]][orb_off[B]:orb_off[B + 1], orb_off[A]:orb_off[A + 1]]
    return -g * np.einsum("Iab,ac,db,Jcd->IJ", CA, X, Y, CB, optimize=True)
