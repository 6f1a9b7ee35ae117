"""Lattice Fourier sums between k and R (oracle, test infrastructure).

Sec. 2 of the paper stores two-point functions as F^R_{rr'} = F_{R+r, r'} and
moves between R and k space around the P / Sigma evaluation.  Written here as
the plain dense sums over the mesh (no FFT):

    F^R = N_k^-1 sum_k exp(+i k.R) F(k)        (k_to_r)
    F(k) = sum_R exp(-i k.R) F^R               (r_to_k)

Pins: the brute-force supercell diagonalisation (G^R read off the supercell
Green's function directly, no Bloch theorem) and the round trip identity
r_to_k(k_to_r(F)) = F on random data, plus a single-R delta.
"""
import numpy as np

from .lattice import kr_phase


def k_to_r(Fk, mesh):
    """Fk: [..., N_k, rows, cols] with the k axis third from last."""
    E = kr_phase(mesh, +1.0)  # [k, R]
    Nk = E.shape[0]
    out = np.tensordot(E.T, np.moveaxis(Fk, -3, 0), axes=(1, 0)) / Nk  # [R, ..., rows, cols]
    return np.moveaxis(out, 0, -3)


def r_to_k(FR, mesh):
    E = kr_phase(mesh, -1.0)  # [k, R]
    out = np.tensordot(E, np.moveaxis(FR, -3, 0), axes=(1, 0))  # [k, ...]
    return np.moveaxis(out, 0, -3)
