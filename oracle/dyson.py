"""Screened interaction from the polarizability (oracle, test infrastructure).

Eq. (2) of the paper: at each momentum q and bosonic Matsubara frequency nu the screened
interaction solves W = V + V P W, with V the bare Coulomb matrix in the product basis.  The
self-energy of Eq. (8) uses only the screening part W~ = W - V (stated in Sec. 2, just before
the MT/INT formulae), so that is what is returned here:

    W~(q, nu) = (I - V(q) P(q, nu))^-1 V(q) - V(q).

The solve is a library primitive (numpy.linalg.solve, LU with partial pivoting, FP64).  No
symmetry of V or P is used.

The way back to imaginary time inverts the tau -> Matsubara matrix of ``matsubara.py``: with
as many frequencies as tau points it is square, and its inverse maps the frequency samples
back to the tau samples of the interpolant that has them as transform.

Parity status: pinned in the tests by closed forms: the scalar case v^2 p / (1 - v p); the
rank-one case P = -u u^H (Sherman-Morrison, W~ = -(V u)(V u)^H / (1 + u^H V u)); diagonal V and
P; P = 0; the Neumann series for a small V P; Hermiticity of W~ for Hermitian V and P.  The
inverse transform is pinned by T^-1 T = I and by recovering tau samples from frequencies.
"""
import numpy as np

from .matsubara import filon_matrix


def screened_interaction(V, P):
    """W~[m, q] = (I - V[q] P[m, q])^-1 V[q] - V[q].

    V: [N_k][n][n] complex; P: [n_omega][N_k][n][n] complex.  Returns complex128 of P's shape.
    """
    V = np.asarray(V, dtype=np.complex128)
    P = np.asarray(P, dtype=np.complex128)
    n_om, n_k, n, _ = P.shape
    eye = np.eye(n, dtype=np.complex128)
    out = np.empty_like(P)
    for m in range(n_om):
        for q in range(n_k):
            W = np.linalg.solve(eye - V[q] @ P[m, q], V[q])
            out[m, q] = W - V[q]
    return out


def omega_to_tau_matrix(tau, omegas):
    """The inverse of the tau -> Matsubara matrix (needs as many frequencies as tau points)."""
    T = filon_matrix(tau, omegas)
    if T.shape[0] != T.shape[1]:
        raise ValueError("the inverse transform needs n_omega == n_tau")
    return np.linalg.inv(T)
