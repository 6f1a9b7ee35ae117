"""Brute-force supercell Green's function (oracle, test infrastructure).

Independent route to G^R(tau): build the Hamiltonian of the whole
Born-von Karman supercell (N_k * N_orb states) from the real-space hoppings,
diagonalise it directly (no Bloch theorem, no lattice Fourier sum), fix mu by
bisection on the full spectrum, and read G^R_ab(tau) = G_{(R,a),(0,b)}(tau)
off the supercell Green's function (the F^R definition of Sec. 2).
"""
import numpy as np

from .lattice import mesh_points


def supercell_hamiltonian(hop, mesh, n_orb):
    """H_{(R1,a),(R2,b)} = sum of H^R_ab over translations R = R1 - R2 modulo the mesh."""
    pts = mesh_points(mesh)
    N = np.array(mesh)
    NR = len(pts)
    Hs = np.zeros((NR * n_orb, NR * n_orb), dtype=np.complex128)
    for i1, R1 in enumerate(pts):
        for i2, R2 in enumerate(pts):
            d = (R1 - R2) % N
            blk = np.zeros((n_orb, n_orb), dtype=np.complex128)
            for R, h in hop.items():
                if np.all((np.array(R) - d) % N == 0):
                    blk += h
            Hs[i1 * n_orb:(i1 + 1) * n_orb, i2 * n_orb:(i2 + 1) * n_orb] = blk
    return 0.5 * (Hs + Hs.conj().T)


def _fermi(x, beta):
    return 0.5 * (1.0 - np.tanh(0.5 * beta * x))


def supercell_mu(eps, beta, n_target):
    lo, hi = eps.min() - 1.0, eps.max() + 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if _fermi(eps - mid, beta).sum() > n_target:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def green_R(hop, mesh, n_orb, beta, taus):
    """G^R(tau) for all R of the mesh, [len(taus)][N_R][n_orb][n_orb]."""
    Hs = supercell_hamiltonian(hop, mesh, n_orb)
    eps, V = np.linalg.eigh(Hs)
    NR = int(np.prod(mesh))
    mu = supercell_mu(eps, beta, NR * n_orb / 2.0)
    x = eps - mu
    out = np.empty((len(taus), NR, n_orb, n_orb), dtype=np.complex128)
    for it, t in enumerate(taus):
        # (1 - f(x)) exp(-x t) = exp(-x t) / (1 + exp(-x beta)), evaluated without overflow
        gx = np.where(x >= 0,
                      np.exp(-np.abs(x) * t) / (1.0 + np.exp(-np.abs(x) * beta)),
                      np.exp(np.minimum(x, 0) * (beta - t)) / (1.0 + np.exp(np.minimum(x, 0) * beta)))
        Gs = -(V * gx[None, :]) @ V.conj().T
        for R in range(NR):
            out[it, R] = Gs[R * n_orb:(R + 1) * n_orb, 0:n_orb]
    return out
