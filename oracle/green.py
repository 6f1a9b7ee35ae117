"""Dyson equation for the Green's function (oracle, test infrastructure).

Eq. (4): G = G0 + G0 Sigma G at every (k, i w_n), with G0 the Hartree-level Green's function,
G0(k, i w_n)^-1 = (i w_n + mu) I - H(k).  Its solution, with the static (exchange) and the
frequency-dependent parts of the self-energy both included:

    G(k, i w_n) = [(i w_n + mu) I - H(k) - Sigma_x(k) - Sigma(k, i w_n)]^-1.

The inverse is a library primitive (numpy.linalg.inv, LU with partial pivoting, FP64).

Parity status: pinned in the tests by the band form of G0 (eigenvectors of H(k), Sigma = 0), by
the scalar form, by the Dyson identity G = G0 + G0 Sigma G with the band-form G0, by the
high-frequency tail i w G -> I, and by the exact Matsubara transform of the band G(tau).
"""
import numpy as np


def fermionic_points(n, beta):
    return (2.0 * np.arange(n) + 1.0) * np.pi / beta


def green_dyson(Hk, mu, omegas, Sigma=None, Sigma_x=None):
    """G[m, k] for H [N_k][n][n], frequencies omegas [n_omega], Sigma [n_omega][N_k][n][n] or None,
    Sigma_x [N_k][n][n] or None."""
    Hk = np.asarray(Hk, dtype=np.complex128)
    n_k, n, _ = Hk.shape
    eye = np.eye(n, dtype=np.complex128)
    out = np.empty((len(omegas), n_k, n, n), dtype=np.complex128)
    for m, w in enumerate(omegas):
        for k in range(n_k):
            A = (1j * w + mu) * eye - Hk[k]
            if Sigma_x is not None:
                A = A - Sigma_x[k]
            if Sigma is not None:
                A = A - Sigma[m, k]
            out[m, k] = np.linalg.inv(A)
    return out
