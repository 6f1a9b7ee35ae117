"""The self-consistent GW cycle on one cell, on the device (Sec. 2, Eqs. (1)-(4)).

Every step is a call of the library (argument marshalling only; the arithmetic runs in its
kernels), FP64 throughout, with n_omega = n_tau Matsubara points:

    G^R(tau)         gw_fourier_k2r                      G(k, tau) -> G^R(tau)
    P^R(tau)         gw_polarizability                   Eq. (5)
    P(q, i nu)       gw_drain (bosonic, parity +1)       R -> q, tau -> i nu
    W~(q, i nu)      gw_screened_interaction             Eq. (2), in place
    W~^R(tau)        gw_tau2omega (inverse matrix), gw_fourier_k2r
    Sigma_c^R(tau)   gw_self_energy                      Eq. (8)
    Sigma_c(k, i w)  gw_drain (fermionic, parity -1)
    Sigma_x(k)       gw_exchange, gw_fourier_r2k         static part (Sec. 2)
    mu, G(k, i w)    gw_update_mu (gw_green_dyson inside) Eq. (4), Sec. 4
    G(k, tau)        gw_green_tau, mixed with the previous iterate
    count            gw_density at beta^- of the new G(k, tau)

The G(k, tau) buffer is the state: each cycle reads it and leaves the next (mixed) iterate in it.
"""
from __future__ import annotations

import numpy as np

from . import (Cell, gw_density, gw_drain, gw_exchange, gw_fourier_k2r, gw_fourier_r2k, gw_green_dyson_workspace,
               gw_green_tau, gw_omega2tau_matrix, gw_polarizability, gw_screened_interaction,
               gw_screened_interaction_workspace, gw_self_energy, gw_tau2omega, gw_tau2omega_matrix, gw_update_mu,
               matsubara)


class SCGW:
    """Device buffers and one cycle of the loop for a cell.

    cell: a Cell; Hk: complex128 device [N_k][N_orb][N_orb]; V: complex128 device [N_k][N_pb][N_pb]
    (bare interaction, Hermitian positive definite); Gk: complex128 device [n_tau][N_k][N_orb][N_orb],
    the starting G(k, tau), updated in place by every cycle; n_target: the electron count to hold;
    mix: weight of the new iterate in G(k, tau) (1 = plain iteration)."""

    def __init__(self, cell: Cell, Hk, V, Gk, spin, n_target, mix=0.5):
        import torch
        self.torch = torch
        self.cell, self.Hk, self.Gk = cell, Hk, Gk
        self.spin, self.n_target, self.mix = float(spin), float(n_target), float(mix)
        nt, NR, No, Np = cell.n_tau, cell.N_R, cell.N_orb, cell.N_pb
        c128 = torch.complex128
        tau = cell.tau()
        nu = matsubara(nt, cell.beta, "bosonic")
        wf = matsubara(nt, cell.beta, "fermionic")
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        self.TB = dev(gw_tau2omega_matrix(tau, nu))
        self.TF = dev(gw_tau2omega_matrix(tau, wf))
        self.TBi = dev(gw_omega2tau_matrix(tau, nu))
        self.GR = torch.empty((nt, NR, No, No), dtype=c128, device="cuda")
        self.P = torch.empty((nt, NR, Np, Np), dtype=c128, device="cuda")
        self.S = torch.empty((nt, NR, No, No), dtype=c128, device="cuda")
        self.Gw = torch.empty((nt, NR, No, No), dtype=c128, device="cuda")
        # lattice sums run over all n_tau slices: the one-slice V and Sigma_x sit in slice 0 of
        # zero-filled buffers
        self.V = V
        self.VR = torch.zeros((nt, NR, Np, Np), dtype=c128, device="cuda")
        self.VR[0].copy_(V)
        gw_fourier_k2r(cell, self.VR, self.VR, basis=1)
        self.Sx = torch.zeros((nt, NR, No, No), dtype=c128, device="cuda")
        self.wwork = torch.empty(gw_screened_interaction_workspace(cell, nt * NR), dtype=torch.uint8, device="cuda")
        self.gwork = torch.empty(gw_green_dyson_workspace(cell, nt * NR), dtype=torch.uint8, device="cuda")
        self.info = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.n_dev = torch.zeros(1, dtype=torch.float64, device="cuda")

    def cycle(self, mu_lo, mu_hi, tol=1e-10, max_iter=200):
        """One cycle; returns (mu, Matsubara count at mu, count of the new G(k, tau) at beta^-,
        pivot report of the W step)."""
        c = self.cell
        gw_fourier_k2r(c, self.Gk, self.GR, basis=0)
        gw_polarizability(c, self.GR, self.P, self.spin)
        gw_drain(c, self.TB, self.P, self.P, basis=1, parity=1)
        gw_screened_interaction(c, self.V, self.P, self.P, self.wwork, info=self.info)
        gw_tau2omega(c, self.TBi, self.P, self.P, basis=1, parity=0)
        gw_fourier_k2r(c, self.P, self.P, basis=1)
        gw_self_energy(c, self.GR, self.P, self.S)
        gw_drain(c, self.TF, self.S, self.S, basis=0, parity=-1)
        gw_exchange(c, self.GR, self.VR[0], self.Sx[0])
        gw_fourier_r2k(c, self.Sx, self.Sx, basis=0)
        mu, n_w = gw_update_mu(c, self.Hk, self.Gw, self.gwork, self.n_dev, self.spin, self.n_target, mu_lo, mu_hi,
                               tol=tol, max_iter=max_iter, Sigma=self.S, Sigma_x=self.Sx[0])
        gw_green_tau(c, self.Gw, self.Hk, mu, self.Gk, Sigma_x=self.Sx[0], mix=self.mix)
        gw_density(c, self.Gk, self.spin, self.n_dev, space=1)
        self.torch.cuda.synchronize()
        return mu, n_w, float(self.n_dev.item()), int(self.info.item())
