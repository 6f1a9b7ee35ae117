"""Plain FP64 CPU oracle for the space-time P / Sigma path (test infrastructure).

This package is test infrastructure.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product library never
does, and it imports nothing from the product library.

It computes, slowly and by the plain definitions of Kutepov's paper:

* lattice Fourier sums between k and R (Sec. 2, the F^R definition and the
  R <-> k transforms of the new algorithm);
* the polarizability as a k-space convolution in imaginary time (the
  structure of Eq. (1) written at fixed tau), and in real space by Eq. (5);
* the self-energy as a k-space convolution (structure of Eq. (3)) and in real
  space by Eq. (8);
* the imaginary-time to Matsubara-frequency transform F(i w) = int_0^beta
  exp(i w tau) F(tau) dtau of the piecewise-linear interpolant of F;
* the electron count from G(R = 0, beta^-);
* the real-space cutoff and distance tiers of the product basis (Sec. 2, Figs. 1, 2);
* the screened interaction W~ = W - V from Eq. (2), and the inverse of the tau -> Matsubara
  matrix;
* the static (exchange) self-energy: Eq. (8) with W~ -> V and G(tau) -> -G(beta);
* the Dyson equation for G, Eq. (4), and the way back from Matsubara frequency to imaginary time
  for G with its high-frequency tails in closed form;
* one cycle of the self-consistent loop (Eqs. (1)-(4)) chained from the functions above;
* the interstitial-grid blocks of P and Sigma, Eqs. (6), (7), (9), (10).

Conventions (the paper leaves them open; the readings are the same as the
product library's documented ones):

* R and k run over the Born-von Karman mesh, index (n1 * N2 + n2) * N3 + n3;
  k = (j1 / N1, j2 / N2, j3 / N3) in reduced units, k.R = 2 pi sum_i j_i n_i / N_i;
* F^R_ab = F(a in cell R, b in cell 0);
  F(k) = sum_R exp(-i k.R) F^R,  F^R = N_k^-1 sum_k exp(+i k.R) F(k);
* tau_0 = 0+, tau_{N-1} = beta-, mirror(i) = N - 1 - i;
* the second Green's function of Eq. (5) is read as G^{-R}_{t'L''', tL''}(beta - tau);
* W enters Eq. (8) at the same tau as G.

Parity status of each function is recorded in its docstring.
"""
from .lattice import mesh_points, kr_phase, minus_index  # noqa: F401
from .fourier import k_to_r, r_to_k  # noqa: F401
from .polarizability import polarizability_q, polarizability_r, polarizability_r_block  # noqa: F401
from .self_energy import self_energy_k, self_energy_r, self_energy_r_block  # noqa: F401
from .matsubara import (  # noqa: F401
    bosonic_frequencies, fermionic_frequencies, filon_matrix, apply_tau_to_omega,
)
from .density import electron_count  # noqa: F401
from . import bruteforce  # noqa: F401
from .cutoff import plan_pairs, polarizability_r_block_cut, self_energy_r_block_cut  # noqa: F401
from .dyson import screened_interaction, omega_to_tau_matrix  # noqa: F401
from .exchange import exchange_r, exchange_k  # noqa: F401
from .green import green_dyson, green_tau  # noqa: F401
from . import scgw  # noqa: F401
from .interstitial import polarizability_int, self_energy_int  # noqa: F401
