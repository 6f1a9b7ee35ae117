"""Electron count from the Green's function (oracle, test infrastructure).

The chemical-potential update of a GW iteration (Sec. 4) needs the electron
count; with G(tau) = -<T c(tau) c^+> the occupation is -G(beta^-), so

    n = -g sum_a G^{R=0}_aa(beta^-),   G^{R=0} = N_k^-1 sum_k G(k).

Pin (tests): with mu at half filling the count is g * N_orb / 2.
"""
import numpy as np


def electron_count(G_last_R0, g):
    """G_last_R0: the R = 0 block of G(beta^-) (N_orb x N_orb)."""
    return float(-g * np.real(np.trace(G_last_R0)))
