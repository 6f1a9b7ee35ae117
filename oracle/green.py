"""Dyson equation for the Green's function (oracle, test infrastructure).

Eq. (4): G = G0 + G0 Sigma G at every (k, i w_n), with G0 the Hartree-level Green's function,
G0(k, i w_n)^-1 = (i w_n + mu) I - H(k).  Its solution, with the static (exchange) and the
frequency-dependent parts of the self-energy both included:

    G(k, i w_n) = [(i w_n + mu) I - H(k) - Sigma_x(k) - Sigma(k, i w_n)]^-1.

The inverse is a library primitive (numpy.linalg.inv, LU with partial pivoting, FP64).

The chemical-potential update (Sec. 4) is the root of (electron count of the Dyson solution) minus
the target, by bisection.  The count is the Matsubara sum of Tr G over the frequencies kept, with
the 1 / (i w) and 1 / (i w)^2 tails of G summed in closed form (their coefficients are I and
H - mu + Sigma_x).

Parity status: pinned in the tests by the band form of G0 (eigenvectors of H(k), Sigma = 0), by
the scalar form, by the Dyson identity G = G0 + G0 Sigma G with the band-form G0, by the
high-frequency tail i w G -> I, and by the exact Matsubara transform of the band G(tau).  The
count is pinned by the Fermi sum of the band energies for Sigma = 0 (to the truncation error of
the third-order tail); the update by the count it reaches and by the band chemical potential for
Sigma = 0.
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


def tail_sum(n_omega, beta):
    """sum over m >= n_omega of 1 / w_m^2, w_m = (2 m + 1) pi / beta (closed form pi^2 / 8 minus the head)."""
    head = np.sum(1.0 / (2.0 * np.arange(n_omega) + 1.0) ** 2)
    return (beta / np.pi) ** 2 * (np.pi ** 2 / 8.0 - head)


def density_omega(G, Hk, mu, beta, g, Sigma_x=None):
    """Electron count from G at the first n_omega fermionic frequencies.

    n = (g / N_k) sum_k [ N_orb / 2 + (2 / beta) ( sum_{m < n_omega} Re Tr G(k, i w_m) - c2(k) S ) ],
    c2(k) = Re Tr (H(k) + Sigma_x(k)) - mu N_orb, S = sum_{m >= n_omega} 1 / w_m^2: the symmetric
    Matsubara sum of G plus its 1 / (i w) and 1 / (i w)^2 tails, whose coefficients are I and
    H - mu + Sigma_x."""
    G = np.asarray(G)
    n_om, n_k, n, _ = G.shape
    A = float(np.sum(np.real(np.einsum("mkaa->", G))))
    B = float(np.real(np.einsum("kaa->", Hk))) - mu * n * n_k
    if Sigma_x is not None:
        B += float(np.real(np.einsum("kaa->", Sigma_x)))
    return float(g / n_k * (n_k * n / 2.0 + 2.0 / beta * (A - B * tail_sum(n_om, beta))))


def update_mu(Hk, beta, n_omega, g, n_target, mu_lo, mu_hi, tol, max_iter, Sigma=None, Sigma_x=None):
    """Chemical potential (Sec. 4): the root in [mu_lo, mu_hi] of count(mu) - n_target, where count
    is the electron count of the Dyson solution of Eq. (4) at mu, found by plain bisection.

    The count rises with mu; the bracket must hold the target (ValueError otherwise).  Each step
    halves the bracket at its midpoint, solving Eq. (4) there; it stops when the count is within tol
    of the target or after max_iter halvings.  Returns (mu, count at mu)."""
    om = fermionic_points(n_omega, beta)

    def count(mu):
        return density_omega(green_dyson(Hk, mu, om, Sigma, Sigma_x), Hk, mu, beta, g, Sigma_x)

    lo, hi = float(mu_lo), float(mu_hi)
    if not (count(lo) <= n_target <= count(hi)):
        raise ValueError("the bracket does not hold the target count")
    mid, n_mid = lo, count(lo)
    for _ in range(max_iter):
        mid = 0.5 * (lo + hi)
        n_mid = count(mid)
        if abs(n_mid - n_target) <= tol:
            break
        if n_mid > n_target:
            hi = mid
        else:
            lo = mid
    return mid, n_mid


def green_tau(G_w, Hk, mu, beta, taus, Sigma_x=None):
    """G(k, tau) from G(k, i w_m), m < n_omega (the first fermionic frequencies): the inverse
    Matsubara sum (1 / beta) sum over all n of exp(-i w_n tau) G(i w_n), with the negative
    frequencies from G(-i w) = G(i w)^H and the tails I / (i w) and c2 / (i w)^2 (c2 = H - mu +
    Sigma_x) summed exactly: their transforms on 0 < tau < beta are -1/2 and (2 tau - beta) / 4.

        G(tau) = -I / 2 + c2 (2 tau - beta) / 4
                 + (1 / beta) sum_{m < n_omega} [exp(-i w_m tau) R_m + exp(i w_m tau) R_m^H],
        R_m = G(i w_m) - I / (i w_m) - c2 / (i w_m)^2.

    Parity status: pinned in the tests by the two tail transforms against brute-force symmetric
    Matsubara sums, by the band G(tau) (O(1 / n_omega^2) convergence to -(1 - f) e^{-x tau}), and
    by the count at beta^-, which equals density_omega."""
    G_w = np.asarray(G_w, dtype=np.complex128)
    n_om, n_k, n, _ = G_w.shape
    w = fermionic_points(n_om, beta)
    eye = np.eye(n)
    c2 = np.asarray(Hk, dtype=np.complex128) - mu * eye[None]
    if Sigma_x is not None:
        c2 = c2 + Sigma_x
    out = np.empty((len(taus), n_k, n, n), dtype=np.complex128)
    for i, t in enumerate(taus):
        acc = -0.5 * eye[None] + c2 * (2.0 * t - beta) / 4.0
        for m in range(n_om):
            R = G_w[m] - eye[None] / (1j * w[m]) - c2 / (1j * w[m]) ** 2
            ph = np.exp(-1j * w[m] * t) / beta
            acc = acc + ph * R + np.conj(ph) * np.conj(np.swapaxes(R, -1, -2))
        out[i] = acc
    return out
