"""Imaginary time -> Matsubara frequency transform (oracle, test infrastructure).

The paper does all P / Sigma work at imaginary times tau in [0, beta] and moves
to Matsubara frequencies afterwards; its non-uniform grids and interpolation
transforms are defined in an earlier paper and not in this text (Appendix A).
The reading used here: F(i w_n) = int_0^beta exp(i w_n tau) F(tau) dtau with
F replaced by its piecewise-linear interpolant on the tau grid, integrated
exactly interval by interval (a Filon-type rule; the trapezoid rule at w = 0).

Frequencies: bosonic nu_m = 2 pi m / beta for P, fermionic
w_n = (2 n + 1) pi / beta for Sigma.

Pins (tests): row w = 0 equals the trapezoid weights; exact for F linear in
tau (closed-form integral); O(h^2) convergence to the exact Laplace-type
integral of exp(-x tau); the Lindhard form of P(i nu) from the band basis.
"""
import numpy as np


def bosonic_frequencies(n, beta):
    return 2.0 * np.pi * np.arange(n) / beta


def fermionic_frequencies(n, beta):
    return (2.0 * np.arange(n) + 1.0) * np.pi / beta


def _interval_weights(w, h):
    """Integrals over [0, h] of exp(i w s) (h - s) / h and of exp(i w s) s / h."""
    if w == 0.0:
        return h / 2.0, h / 2.0
    th = w * h
    e = np.exp(1j * th)
    right = e / (1j * w) + (e - 1.0) / (h * w * w)
    left = (e - 1.0) / (1j * w) - right
    return left, right


def filon_matrix(tau, omegas):
    """T[m, j] such that sum_j T[m, j] F(tau_j) = int exp(i w_m tau) F_lin(tau) dtau."""
    tau = np.asarray(tau, dtype=float)
    T = np.zeros((len(omegas), len(tau)), dtype=np.complex128)
    for m, w in enumerate(omegas):
        for j in range(len(tau) - 1):
            h = tau[j + 1] - tau[j]
            left, right = _interval_weights(float(w), h)
            ph = np.exp(1j * w * tau[j])
            T[m, j] += ph * left
            T[m, j + 1] += ph * right
    return T


def apply_tau_to_omega(T, F_tau):
    """F_omega[m, ...] = sum_j T[m, j] F_tau[j, ...]."""
    return np.tensordot(T, F_tau, axes=(1, 0))
