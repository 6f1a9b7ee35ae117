"""Device-side materialisation of the serving requests' inputs (input data only).

For a request on a cell of the serving mix, the inputs of the path are G(k, tau) and
W(R, tau), built from the same seeded generators as the host versions in this package:

    G(k, tau_i) = -U diag(g(eps - mu, tau_i)) U^+,   g = (1 - f(x)) exp(-x tau) in the
                  overflow-free form (exponents kept <= 0);
    W^R_IJ(tau) = A_IJ exp(-|R|_min / 3 A) exp(-tau / 5).

Bands, coefficients and A are computed on the host once per cell kind; the per-request
materialisation runs on the caller's current stream (torch), so a serving loop can enqueue
it ahead of the path on a request's own stream.  Nothing here is part of the path itself.
"""
from __future__ import annotations

from typing import Dict

import numpy as np

from . import SERVING_NTAU, bands, coefficients, hoppings, serving_cell, tau_grid, w_amplitude, w_factors


class ServingInputs:
    """Cell descriptions and per-request device inputs of the serving mix."""

    def __init__(self):
        import torch
        self.torch = torch

    def spec(self, kind: str, n_tau: int):
        return serving_cell(kind, n_tau, 0)

    def kind_data(self, kind: str, complex_dtype) -> Dict:
        """Host work done once per kind: bands, C, A (device copies where used per request)."""
        torch = self.torch
        spec = serving_cell(kind, SERVING_NTAU[0], 0)
        b = bands(spec, hoppings(spec))
        U = torch.from_numpy(b.U).cuda()
        return {"C": coefficients(spec), "U": U, "Uh": U.conj().transpose(-1, -2).contiguous(),
                "x": torch.from_numpy(b.eps - b.mu).cuda(),
                "A": torch.from_numpy(w_amplitude(spec)).cuda().to(complex_dtype)}

    def cell_data(self, spec, complex_dtype) -> Dict:
        """Host work done once per (kind, n_tau): the tau grid and the W factors on the device."""
        torch = self.torch
        sR, et = w_factors(spec)
        return {"tau": torch.from_numpy(tau_grid(spec)).cuda(),
                "f": torch.from_numpy(et[:, None] * sR[None, :]).cuda().to(complex_dtype)}

    def materialize(self, kd: Dict, cd: Dict, spec, Gk, W) -> None:
        """Write G(k, tau) into Gk [n_tau][N_k][N_orb][N_orb] (complex128) and W(R, tau) into
        W [n_tau][N_R][N_pb][N_pb], on the current stream."""
        torch = self.torch
        x = kd["x"][None]
        tau = cd["tau"][:, None, None]
        xp, xn = x.clamp(min=0), x.clamp(max=0)
        gp = torch.exp(-xp * tau) / (1 + torch.exp(-xp * spec.beta))
        gn = torch.exp(xn * (spec.beta - tau)) / (1 + torch.exp(xn * spec.beta))
        mg = -torch.where(x >= 0, gp, gn)  # (n_tau, N_k, N_orb)
        step = max(1, 8 // max(1, spec.N_R // 8))
        for a in range(0, spec.n_tau, step):
            b = min(spec.n_tau, a + step)
            torch.matmul(kd["U"][None] * mg[a:b, :, None, :].to(torch.complex128), kd["Uh"][None], out=Gk[a:b])
        torch.mul(kd["A"][None, None], cd["f"][:, :, None, None], out=W)
