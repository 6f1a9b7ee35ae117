/*
 * gwr.h -- C ABI of the space-time polarizability / self-energy library for
 * AMD Instinct MI355X (gfx950).
 *
 * The library evaluates the atom-pair-blocked real-space, imaginary-time
 * forms of the polarizability P (Eq. (5), MT-MT) and of the self-energy
 * Sigma (Eq. (8), MT-MT) of Kutepov's O(N) self-consistent GW method, and the
 * lattice (k <-> R) and Matsubara (tau -> i omega) transforms that feed and
 * drain them (Sec. 2: the F^R_{rr'} storage, the R <-> k transforms whose
 * cost is proportional to the number of pairs), the real-space cutoff with
 * distance-tiered product basis (Sec. 2, Figs. 1, 2), and the screened
 * interaction W of Eq. (2) that links P to Sigma.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - A cell has n_atoms atoms; atom A has species s(A), n_orb[s] orbitals and
 *    n_pb[s] product functions.  Orbitals and product functions occupy
 *    contiguous index ranges in atom order; N_orb and N_pb are their totals.
 *  - The Born-von Karman mesh N1 x N2 x N3 gives N_R = N_k = N1*N2*N3.  R and k
 *    are indexed (n1 * N2 + n2) * N3 + n3 with 0 <= n_i < N_i;
 *    k.R = 2 pi sum_i j_i n_i / N_i.  -R is taken modulo the mesh.
 *  - F^R_ab = F(a in cell R, b in cell 0);  F(k) = sum_R exp(-i k.R) F^R;
 *    F^R = N_k^-1 sum_k exp(+i k.R) F(k).
 *  - tau_i, i = 0 .. n_tau-1, is a grid on [0, beta] that is symmetric about
 *    beta/2; tau_0 stands for 0+ and tau_{n_tau-1} for beta-, and the mirror
 *    beta - tau_i is the index n_tau-1-i.
 *  - Tensors are dense, row-major and contiguous, complex numbers stored
 *    interleaved (re, im):
 *        G, Sigma  [n_tau][N_R][N_orb][N_orb]     ("orbital basis", basis = 0)
 *        P, W      [n_tau][N_R][N_pb][N_pb]       ("product basis", basis = 1)
 *    After a transform the leading axis may be frequency and the second k.
 *  - Every tensor pointer is a DEVICE pointer on the device that was current
 *    when the cell was created, allocated and owned by the caller.  The
 *    library never frees or retains it.
 *  - Validation is synchronous; on any error nothing is launched and the
 *    status says why (gw_last_error() gives detail, per thread).  Kernels are
 *    enqueued on `stream` (a hipStream_t; NULL is the null stream) and the
 *    call returns without synchronising.  Calls on different cells or
 *    streams may run concurrently; a cell is read-only after creation.
 */
#ifndef GWR_H
#define GWR_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GW_OK = 0,
  GW_ERR_ARG = -1,         /* null pointer, bad enum, non-symmetric C, aliasing ... */
  GW_ERR_SHAPE = -2,       /* sizes inconsistent or out of the supported range     */
  GW_ERR_NOMEM = -3,       /* device allocation failed during gw_cell_create       */
  GW_ERR_HIP = -4,         /* a HIP runtime call or kernel launch failed           */
  GW_ERR_UNSUPPORTED = -5  /* valid request this build does not implement          */
} gw_status;

/* Arithmetic of the P and Sigma contractions (Eqs. (5), (8)).
 *   GW_FP64   : G, W, P are complex128; FP64 MFMA; Sigma complex128.
 *   GW_FP32   : G, W, P are complex64; FP32 MFMA, FP32 accumulation;
 *               Sigma is accumulated over atom-orbital sums in FP64 and stored complex128.
 *   GW_BF16X3 : storage as GW_FP32; in both contractions each FP32 operand is split into
 *               bf16 hi + lo and the products hi*hi + hi*lo + lo*hi run on the BF16 matrix
 *               cores with FP32 accumulation (relative error a few 1e-6; Sigma's FP64
 *               orbital sums as for GW_FP32).  The split kernels cover species pairs of 9
 *               orbitals with 49..64 product functions on both atoms.  Other pairs run what
 *               GW_FP32 runs for them: the FP32 matrix-core kernels when both atoms have at
 *               most 9 orbitals and 64 product functions, else the plain vector-ALU kernels
 *               (FP32 operands, FP64 sums). */
typedef enum { GW_FP64 = 0, GW_FP32 = 1, GW_BF16X3 = 2 } gw_precision;

/* Storage type of a transform operand.  Transforms always compute in FP64. */
typedef enum { GW_C128 = 0, GW_C64 = 1 } gw_dtype;

typedef struct gw_cell gw_cell;

/* Create a cell description and upload its constants (product-basis
 * coefficients in every layout the kernels use) to the current device.
 *   species_of_atom[n_atoms] in [0, n_species);  n_orb[n_species], n_pb[n_species] >= 1;
 *   C: host FP64, species after species, each [n_pb[s]][n_orb[s]][n_orb[s]] holding
 *      <M_I | phi_a phi_b> (Eqs. (5), (8)); must be symmetric in (a, b) to 1e-12
 *      relative, else GW_ERR_ARG (the kernels fold that symmetry);
 *   mesh[3] >= 1 each; 2 <= n_tau <= 256; beta > 0;
 *   tau: host FP64 [n_tau], the imaginary-time grid on [0, beta] (Sec. 2: every function of
 *      tau lives on [0, beta]).  It must start at 0 (standing for 0+), end at beta (beta-),
 *      increase strictly and be symmetric about beta / 2: |tau_i + tau_{n_tau-1-i} - beta|
 *      <= 1e-12 beta for every i, as must |tau_0| and |tau_{n_tau-1} - beta|.  Otherwise
 *      GW_ERR_ARG before anything touches a device.  The mirror beta - tau_i is then the
 *      index n_tau-1-i, which the polarizability's tau mirror, the parity pairing of the
 *      drains and the beta^- slice of gw_density and gw_exchange rely on.  The grid is
 *      copied; any such grid works (uniform, or clustered at both ends).
 * Limits: n_orb <= 16, n_pb <= 128, N_R <= 64 (GW_ERR_SHAPE beyond).
 * On success *out owns device memory until gw_cell_destroy. */
gw_status gw_cell_create(gw_cell** out, int n_atoms, const int* species_of_atom, int n_species,
                         const int* n_orb, const int* n_pb, const double* C, const int* mesh,
                         int n_tau, double beta, const double* tau);
void gw_cell_destroy(gw_cell* cell);

/* The cell's tau grid, copied to the host buffer tau[n_tau].  GW_ERR_ARG for NULL. */
gw_status gw_cell_tau(const gw_cell* cell, double* tau);

/* Bytes of device scratch the path's calls (gw_fourier_k2r, gw_polarizability,
 * gw_self_energy, gw_fourier_r2k, gw_tau2omega, gw_drain, gw_density and the _pairs
 * variants) need for this cell at precision prec.  Every one of them keeps its temporaries
 * in registers and LDS, so the answer is 0 for every cell and precision; callers that
 * budget memory can rely on that.  The Dyson solves take their own workspace
 * (gw_screened_interaction_workspace, gw_green_dyson_workspace). */
size_t gw_workspace_bytes(const gw_cell* cell, gw_precision prec);

/* Totals of a cell (0 for a NULL cell). */
int gw_cell_n_orb_total(const gw_cell* cell);
int gw_cell_n_pb_total(const gw_cell* cell);
int gw_cell_n_R(const gw_cell* cell);

/* k -> R lattice sum (Sec. 2): out^R = N_k^-1 sum_k exp(+i k.R) in(k), per tau and
 * per matrix element; basis 0 (N_orb) or 1 (N_pb); in and out may be the same
 * pointer when in_type == out_type (in-place), otherwise they must not overlap. */
gw_status gw_fourier_k2r(const gw_cell* cell, const void* in, gw_dtype in_type, void* out,
                         gw_dtype out_type, int basis, void* stream);

/* R -> k lattice sum: out(k) = sum_R exp(-i k.R) in^R.  Same rules as gw_fourier_k2r. */
gw_status gw_fourier_r2k(const gw_cell* cell, const void* in, gw_dtype in_type, void* out,
                         gw_dtype out_type, int basis, void* stream);

/* Polarizability, Eq. (5) (MT-MT), for every (tau, R, A, B):
 *   P^R_IJ(tau) = -g sum_{a,b in A; c,d in B} C^I_ab G^R_ac(tau) G^{-R}_db(beta - tau) C^J_cd
 * GR: [n_tau][N_R][N_orb][N_orb], P: [n_tau][N_R][N_pb][N_pb], complex128 for GW_FP64,
 * complex64 otherwise; g = spin_factor (the spin sum of Eq. (5)).  Uses the identity
 * P^R_IJ(beta - tau) = P^{-R}_JI(tau) (symmetric C) to evaluate half the tau range. */
gw_status gw_polarizability(const gw_cell* cell, const void* GR, void* P, double spin_factor,
                            gw_precision prec, void* stream);

/* Self-energy, Eq. (8) (MT-MT), with W taken at the same tau as G:
 *   Sigma^R_ab(tau) = -sum_{a',I in A; b',J in B} C^I_aa' G^R_a'b'(tau) W^R_IJ(tau) C^J_bb'
 * GR, WR: complex128 for GW_FP64, complex64 otherwise; Sigma always complex128,
 * [n_tau][N_R][N_orb][N_orb]. */
gw_status gw_self_energy(const gw_cell* cell, const void* GR, const void* WR, void* Sigma,
                         gw_precision prec, void* stream);

/* Imaginary time -> Matsubara frequency along the leading axis:
 *   out[m][...] = sum_i T[m][i] in[i][...],  m < n_omega,
 * with T a DEVICE complex128 matrix [n_omega][n_tau] (see gw_tau2omega_matrix).
 * The trailing shape is [N_R][n][n] with n = N_orb (basis 0) or N_pb (basis 1).
 * parity declares the mirror symmetry of T about beta/2:
 *    0 : none assumed (any T);
 *   +1 : T[m][n_tau-1-i] == conj(T[m][i])   (bosonic frequencies on a symmetric grid);
 *   -1 : T[m][n_tau-1-i] == -conj(T[m][i])  (fermionic frequencies on a symmetric grid).
 * With parity != 0 the kernels may read only the columns i <= (n_tau-1)/2 of T and pair
 * each tau with its mirror (two real GEMMs instead of three); the result for a T that
 * lacks the declared symmetry is unspecified.  T must still hold all n_tau columns.
 * parity outside {-1, 0, +1} is GW_ERR_ARG.
 * FP64 arithmetic.  in == out is allowed when in_type == out_type. */
gw_status gw_tau2omega(const gw_cell* cell, const void* T, int n_omega, int parity, const void* in,
                       gw_dtype in_type, void* out, gw_dtype out_type, int basis, void* stream);

/* R -> k followed by tau -> Matsubara in one pass over HBM (product of the two
 * operators above; same argument rules, parity included).  For complex64 in and out with
 * parity +1 or -1 (the mixed paths' P drain), the paired, R -> k transformed columns are formed
 * in FP64 and held on chip as complex64 (the storage precision of in and out) before the FP64
 * tau contraction; the other cases stay FP64 throughout. */
gw_status gw_drain(const gw_cell* cell, const void* T, int n_omega, int parity, const void* in,
                   gw_dtype in_type, void* out, gw_dtype out_type, int basis, void* stream);

/* Electron count for the chemical-potential update (Sec. 4), one FP64 value written
 * to the DEVICE pointer n_dev:
 *   space = 0: G is G^R(tau), n = -g sum_a Re G^{R=0}_aa(beta^-)   (last tau, R = 0);
 *   space = 1: G is G(k, tau), n = -(g / N_k) sum_k sum_a Re G_aa(k, beta^-)
 *              (the same number: G^{R=0} is the k average).
 * G: [n_tau][N_R][N_orb][N_orb] in g_type storage; FP64 summation. */
gw_status gw_density(const gw_cell* cell, const void* G, gw_dtype g_type, int space, double spin_factor,
                     double* n_dev, void* stream);

/* Real-space cutoff and distance tiers of the product basis (Sec. 2, Figs. 1 and 2).
 * Plans the blocks (R, A, B) -- atom A in cell R, atom B in cell 0 -- that are kept:
 * those whose centre distance d = |R' . a + r_A - r_B|, minimised over the lattice vectors
 * R' equal to R modulo the mesh, is at most r_c (blocks farther apart are zero).  A kept
 * block's product basis depends on d: all functions of both atoms when A = B in the same
 * cell (R = 0); the first m_tier[2 s] functions of an atom of species s when 0 < d <= r_b;
 * the first m_tier[2 s + 1] when r_b < d <= r_c.
 *   lattice:   host [3][3], rows are the lattice vectors;
 *   positions: host [n_atoms][3], Cartesian, same length unit;
 *   m_tier:    host [n_species][2], each in [1, n_pb of the species].
 * GW_ERR_ARG for r_b < 0, r_c < r_b, non-finite input, a bad tier size, or a mesh so coarse
 * that some pair has two periodic images inside the sphere (the paper's k-mesh condition).
 * Set-up call: it allocates device memory for the list (held until gw_cell_destroy) and
 * replaces any earlier list of the cell; call it while no pair contraction of the cell is
 * in flight. */
gw_status gw_cell_set_pairs(gw_cell* cell, const double* lattice, const double* positions, double r_b,
                            double r_c, const int* m_tier);

/* The planned list: *n_pairs kept blocks and, when pairs != NULL, the first
 * min(n_pairs, capacity) of them as host int [.][5] = (R, A, B, mA, mB), with mA, mB the
 * product functions kept on atoms A and B.  GW_ERR_ARG without a list. */
gw_status gw_cell_pairs(const gw_cell* cell, long long* n_pairs, int* pairs, long long capacity);

/* Eq. (5) over the kept blocks only, every tau: P^R_IJ(tau) for I < mA, J < mB of each
 * listed (R, A, B), zero for the other (I, J) of that block.  Blocks outside the list are
 * not written: the caller zero-fills P once if it needs them.  Tensors, spin factor and
 * storage types as gw_polarizability.  The matrix-core kernels of gw_polarizability run over
 * the list where the block shape has one (precision as there); other shapes run plain
 * vector-ALU kernels (FP64 for GW_FP64, FP32 operands with FP64 sums otherwise).  GW_ERR_ARG
 * without a list. */
gw_status gw_polarizability_pairs(const gw_cell* cell, const void* GR, void* P, double spin_factor,
                                  gw_precision prec, void* stream);

/* Eq. (8) over the kept blocks only, every tau, with W^R_IJ taken as zero for I >= mA or
 * J >= mB of the block.  Sigma blocks outside the list are not written.  Tensors and storage
 * types as gw_self_energy; arithmetic as gw_polarizability_pairs. */
gw_status gw_self_energy_pairs(const gw_cell* cell, const void* GR, const void* WR, void* Sigma,
                               gw_precision prec, void* stream);

/* Packed storage of the kept blocks (Sec. 2: two-point functions stored only for the pairs
 * within R_max, each in the product basis of its distance tier).  A tau slice of a packed tensor
 * holds the kept (R, A, B) blocks of gw_cell_pairs one after the other, in that order, each as
 * its mA x mB kept functions row-major; *per_tau = sum over the kept blocks of mA mB (elements
 * per tau slice).  GW_ERR_ARG without a list. */
gw_status gw_cell_packed_size(const gw_cell* cell, long long* per_tau);

/* Eq. (5) over the kept blocks, written in the packed layout: P [n_tau][per_tau], the block
 * (R, A, B) holding P^R_IJ(tau) for I < mA, J < mB (the values gw_polarizability_pairs writes
 * there).  complex128 for GW_FP64, complex64 otherwise (GW_BF16X3 runs the FP32 matrix cores here).
 * GR as for gw_polarizability.  GW_ERR_ARG without a list or for overlapping tensors. */
gw_status gw_polarizability_packed(const gw_cell* cell, const void* GR, void* P, double spin_factor,
                                   gw_precision prec, void* stream);

/* Eq. (8) over the kept blocks with W^R(tau) read in the packed layout (W_IJ taken as zero beyond
 * a block's mA x mB functions, as in gw_self_energy_pairs); Sigma dense complex128
 * [n_tau][N_R][N_orb][N_orb], written on the kept blocks only.  Storage types as
 * gw_polarizability_packed. */
gw_status gw_self_energy_packed(const gw_cell* cell, const void* GR, const void* WR, void* Sigma,
                                gw_precision prec, void* stream);

/* R -> k of a packed tensor: out[t][q][pA + I][pB + J] = sum over the kept blocks (R, A, B) of
 * exp(-i q.R) F_(R,A,B)(t)[I][J], dense complex [n_tau][N_k][N_pb][N_pb] (every element written:
 * zero where no kept block has the function pair).  in: packed [n_tau][per_tau].  FP64
 * arithmetic; in and out must not overlap. */
gw_status gw_fourier_r2k_packed(const gw_cell* cell, const void* in, gw_dtype in_type, void* out,
                                gw_dtype out_type, void* stream);

/* k -> R into the packed layout: F_(R,A,B)(t)[I][J] = N_k^-1 sum_q exp(+i q.R) in[t][q][pA + I][pB + J]
 * for the kept blocks only.  in: dense [n_tau][N_k][N_pb][N_pb]; out: packed.  FP64 arithmetic. */
gw_status gw_fourier_k2r_packed(const gw_cell* cell, const void* in, gw_dtype in_type, void* out,
                                gw_dtype out_type, void* stream);

/* gw_fourier_r2k_packed into out, then gw_tau2omega in place on out (same T, n_omega and parity
 * rules): out[m][q][...] = sum_tau T[m][tau] (R -> k of the packed tensor)(tau).  out must hold
 * max(n_tau, n_omega) N_k N_pb^2 elements. */
gw_status gw_drain_packed(const gw_cell* cell, const void* T, int n_omega, int parity, const void* in,
                          gw_dtype in_type, void* out, gw_dtype out_type, void* stream);

/* Host helper: the FP64 matrix T[n_omega][n_tau] (complex, interleaved) that integrates
 * the piecewise-linear interpolant of F(tau) against exp(i omega_m tau) over [0, beta]
 * exactly (trapezoid rule at omega = 0).  tau: host, increasing; omega: host.
 * T_host: host buffer of 2*n_omega*n_tau doubles. */
gw_status gw_tau2omega_matrix(int n_tau, const double* tau, int n_omega, const double* omega,
                              double* T_host);

/* Interstitial-grid blocks of P, Eqs. (6), (7).  n_g real-space grid points per cell stand for
 * the interstitial region; a grid point enters as one "orbital" (the value of G there) and one
 * "product function" (the product of two G values there), so the MT coefficients remain only on
 * the muffin-tin side.  Per (tau, R), row-major, in `type` storage (complex128 or complex64):
 *   G_og [n_tau][N_R][N_orb][n_g] = G^R_{tL; r'},  G_go [n_tau][N_R][n_g][N_orb] = G^R_{r; tL},
 *   G_gg [n_tau][N_R][n_g][n_g];
 *   P_pg [n_tau][N_R][N_pb][n_g]: P^R_{tK; r'}(tau) = -g sum_{a,b in t} C^K_ab G^R_{a r'}(tau) G^{-R}_{r' b}(beta - tau)
 *   P_gp [n_tau][N_R][n_g][N_pb]: P^R_{r; tK}(tau) = -g sum_{c,d in t} G^R_{r c}(tau) G^{-R}_{d r}(beta - tau) C^K_cd
 *   P_gg [n_tau][N_R][n_g][n_g]:  P^R_{r r'}(tau) = -g G^R_{r r'}(tau) G^{-R}_{r' r}(beta - tau)
 * (the second G read as in Eq. (5)).  FP64 arithmetic; outputs must not overlap inputs or each
 * other.  Up to 8 species. */
gw_status gw_polarizability_int(const gw_cell* cell, int n_g, const void* G_og, const void* G_go, const void* G_gg,
                                void* P_pg, void* P_gp, void* P_gg, double spin_factor, gw_dtype type, void* stream);

/* Interstitial-grid blocks of Sigma, Eqs. (9), (10), W at the same tau as G; W blocks laid out
 * as the P blocks above, Sigma blocks as the G blocks but always complex128:
 *   S_og[tL][r'] = -sum_{I, a' in t} C^I_{L a'} G^R_{a' r'}(tau) W^R_{I r'}(tau)
 *   S_go[r][tL]  = -sum_{J, b' in t} G^R_{r b'}(tau) W^R_{r J}(tau) C^J_{L b'}
 *   S_gg[r][r']  = -G^R_{r r'}(tau) W^R_{r r'}(tau). */
gw_status gw_self_energy_int(const gw_cell* cell, int n_g, const void* G_og, const void* G_go, const void* G_gg,
                             const void* W_pg, const void* W_gp, const void* W_gg, void* S_og, void* S_go,
                             void* S_gg, gw_dtype type, void* stream);

/* Static (exchange) part of the self-energy (Sec. 2: the Eq. (8) expression with W~(tau)
 * replaced by the bare V and G(tau) by -G(beta)):
 *   Sigma_x^R_ab = + sum_{a',I in A; b',J in B} C^I_aa' G^R_a'b'(beta^-) V^R_IJ C^J_bb'
 * GR: [n_tau][N_R][N_orb][N_orb] as for gw_self_energy; only the last time point (beta^-) is read.
 * VR: [N_R][N_pb][N_pb] bare interaction in real space, same storage as GR (complex128 for
 *     GW_FP64, complex64 otherwise).  Sigma_x: complex128 [N_R][N_orb][N_orb], not overlapping
 *     the inputs.  Runs the self-energy kernels of the precision on that one time slice. */
gw_status gw_exchange(const gw_cell* cell, const void* GR, const void* VR, void* Sigma_x, gw_precision prec,
                      void* stream);

/* Screened interaction, Eq. (2): at every momentum q and bosonic frequency nu the solution of
 * W = V + V P W, returned as its screening part W~ = W - V (Sec. 2 splits W = V + W~; W~ is
 * what Eq. (8) takes):
 *   W~(q, nu) = (I - V(q) P(q, nu))^-1 V(q) - V(q) = (V(q)^-1 - P(q, nu))^-1 - V(q).
 *   V:  DEVICE complex128 [N_k][N_pb][N_pb], Hermitian positive definite (bare Coulomb);
 *   P:  DEVICE [n_omega][N_k][N_pb][N_pb] in p_type storage (the layout gw_drain leaves with
 *       basis 1); the Hermitian part of each P(q, nu) negative semidefinite (as at bosonic
 *       Matsubara frequencies), so that V^-1 - P has a positive definite Hermitian part: then
 *       every leading block is invertible and every pivot has a positive real part;
 *   W:  DEVICE, P's shape, w_type storage; may be P itself when p_type == w_type, else disjoint;
 *   prec: GW_FP64 runs both eliminations in FP64; GW_FP32 (and GW_BF16X3) in FP32 on complex64
 *       working copies (relative error about cond * 1e-7; the final W - V subtraction in FP64);
 *   work, work_size: DEVICE scratch of at least gw_screened_interaction_workspace(cell, 1, prec)
 *       bytes, owned by the caller and not retained; more lets more (q, nu) matrices be
 *       inverted per launch (up to the size for chunk = n_omega * N_k);
 *   info: NULL, or a DEVICE int set to 0, then to -(q + 1) if V(q) or to 1 + nu * N_k + q if
 *       V(q)^-1 - P(q, nu) met a pivot whose real part is not positive (one such matrix is
 *       named; the outputs are then not to be trusted).  Read it after the stream completes.
 * Both inverses are blocked Gauss-Jordan eliminations without pivoting, on the matrices
 * padded to a multiple of 64 with the identity.  Enqueued on `stream`. */
gw_status gw_screened_interaction(const gw_cell* cell, const void* V, const void* P, gw_dtype p_type, void* W,
                                  gw_dtype w_type, int n_omega, gw_precision prec, void* work, size_t work_size,
                                  int* info, void* stream);

/* Workspace bytes gw_screened_interaction needs to invert `chunk` (q, nu) matrices per launch
 * at precision prec: e * (Np^2 * (N_k + chunk) + 4096 * max(N_k, chunk)), Np = N_pb rounded up
 * to 64, e = 16 for GW_FP64 and 8 otherwise. */
gw_status gw_screened_interaction_workspace(const gw_cell* cell, int chunk, gw_precision prec, size_t* bytes);

/* Dyson equation for the Green's function, Eq. (4), with the Hartree-level G0^-1 = (i w + mu) - H:
 *   G(k, i w_m) = [(i w_m + mu) I - H(k) - Sigma_x(k) - Sigma(k, i w_m)]^-1,
 * at the first n_omega fermionic Matsubara frequencies w_m = (2 m + 1) pi / beta of the cell.
 *   Hk:      DEVICE complex128 [N_k][N_orb][N_orb] (one-electron Hamiltonian on the k mesh);
 *   Sigma:   DEVICE complex128 [n_omega][N_k][N_orb][N_orb] (the layout gw_drain leaves with
 *            basis 0), or NULL for none;  Sigma_x: DEVICE complex128 [N_k][N_orb][N_orb] or NULL;
 *   G:       DEVICE complex128 [n_omega][N_k][N_orb][N_orb]; may be Sigma itself, else disjoint;
 *   work:    DEVICE scratch of at least gw_green_dyson_workspace(cell, 1) bytes (more inverts
 *            more matrices per launch);
 *   info:    NULL or a DEVICE int: 0, or 1 + m * N_k + k of a matrix that met a pivot of
 *            -i A with non-positive real part (see below).
 * The inverse is the blocked FP64 Gauss-Jordan elimination of gw_screened_interaction applied
 * to -i A, whose Hermitian part w_m I - (Sigma - Sigma^H) / 2i is positive definite for a causal
 * self-energy, so no pivoting is needed; G = -i (-i A)^-1. */
gw_status gw_green_dyson(const gw_cell* cell, const void* Hk, double mu, int n_omega, const void* Sigma,
                         const void* Sigma_x, void* G, void* work, size_t work_size, int* info, void* stream);

/* gw_green_dyson without a workspace argument, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation).  Same
 * arguments, result and kernels as gw_green_dyson; the scratch is a static 64 MiB device array
 * inside the library (one per GPU, held until the process ends), so the call allocates nothing.
 * A cell one of whose padded matrices needs more than 64 MiB (16 (No^2 + 4096) bytes,
 * No = N_orb rounded up to 64, i.e. N_orb above 2040) is refused with GW_ERR_SHAPE before any
 * launch; smaller cells are solved 64 MiB / (16 (No^2 + 4096)) matrices per launch.  Every call
 * on one GPU uses that GPU's one array: calls that overlap in time on one GPU (on different
 * streams or host threads) race and give undefined results.  Nothing in the array needs to
 * start at zero (each launch writes what it reads); it keeps the last call's contents.
 * The first call on a GPU looks up the array's device address there (no allocation). */
gw_status gw_green_dyson_noalloc(const gw_cell* cell, const void* Hk, double mu, int n_omega, const void* Sigma,
                                 const void* Sigma_x, void* G, int* info, void* stream);

/* Workspace bytes of gw_green_dyson for `chunk` matrices per launch:
 * 16 * chunk * (No^2 + 4096), No = N_orb rounded up to 64. */
gw_status gw_green_dyson_workspace(const gw_cell* cell, int chunk, size_t* bytes);

/* Electron count (Sec. 4) from G at the first n_omega fermionic frequencies of the cell:
 *   n = (g / N_k) sum_k [ N_orb / 2 + (2 / beta) ( sum_{m < n_omega} Re Tr G(k, i w_m) - c2(k) S ) ],
 *   c2(k) = Re Tr (H(k) + Sigma_x(k)) - mu N_orb,  S = sum_{m >= n_omega} 1 / w_m^2,
 * i.e. the symmetric Matsubara sum of G with its 1 / (i w) and 1 / (i w)^2 tails (coefficients I
 * and H - mu + Sigma_x) summed in closed form.  G: DEVICE complex128 [n_omega][N_k][N_orb][N_orb]
 * (gw_green_dyson's output at this mu); Hk, Sigma_x (or NULL) as for gw_green_dyson; one FP64
 * value written to the DEVICE pointer n_dev. */
gw_status gw_density_omega(const gw_cell* cell, const void* G, int n_omega, const void* Hk, const void* Sigma_x,
                           double mu, double spin_factor, double* n_dev, void* stream);

/* Chemical-potential update (Sec. 4): Illinois regula falsi (a bracketing secant) on mu in
 * [mu_lo, mu_hi] (the count must rise through n_target there, else GW_ERR_ARG) until the
 * electron count of the Dyson solution (gw_green_dyson, then gw_density_omega) is within tol of
 * n_target, or max_iter steps.  G (not
 * Sigma), work and n_dev are the caller's scratch; on return G holds the solution at *mu_out and
 * *n_out its count.  Synchronous: waits on `stream` once per step.  The Dyson solves inside do
 * not report pivots; when Sigma may not be causal, check it first with gw_green_dyson's info. */
gw_status gw_update_mu(const gw_cell* cell, const void* Hk, const void* Sigma, const void* Sigma_x, int n_omega,
                       double spin_factor, double n_target, double mu_lo, double mu_hi, double tol, int max_iter,
                       void* G, void* work, size_t work_size, double* n_dev, double* mu_out, double* n_out,
                       void* stream);

/* Imaginary time from Matsubara frequency for the Green's function (the way back that closes the
 * Eqs. (1)-(4) cycle, Sec. 2): G(k, tau_i) on the cell's tau grid from G(k, i w_m) at the first
 * n_omega fermionic frequencies w_m = (2 m + 1) pi / beta,
 *   G(tau) = (1 / beta) sum over every fermionic w_n of exp(-i w_n tau) G(i w_n),
 * with the negative frequencies taken as G(k, -i w) = G(k, i w)^H (Hermitian H, Sigma_x and
 * Sigma(k, -i w) = Sigma(k, i w)^H) and the high-frequency tails I / (i w) + c2 / (i w)^2,
 * c2 = H(k) - mu + Sigma_x(k), summed in closed form (-I/2 and c2 (2 tau - beta) / 4):
 *   G(tau) = -I/2 + c2 (2 tau - beta) / 4
 *            + (1 / beta) sum_{m < n_omega} [e^{-i w_m tau} R_m + e^{+i w_m tau} R_m^H],
 *   R_m = G(i w_m) - I / (i w_m) - c2 / (i w_m)^2.
 * At tau = beta^- this gives exactly the count of gw_density_omega (-g / N_k sum_k Tr G(k, beta^-)).
 *   G:       DEVICE complex128 [n_omega][N_k][N_orb][N_orb] (gw_green_dyson's output at mu), n_omega <= 512;
 *   Hk:      DEVICE complex128 [N_k][N_orb][N_orb];  Sigma_x: same shape or NULL;
 *   mix:     in (0, 1]: G_tau <- mix G(tau) + (1 - mix) G_tau, the linear mixing of successive
 *            iterates of the self-consistent loop (G_tau is not read when mix = 1);
 *   G_tau:   DEVICE complex128 [n_tau][N_k][N_orb][N_orb], not overlapping the inputs.
 * FP64 arithmetic; enqueued on `stream`. */
gw_status gw_green_tau(const gw_cell* cell, const void* G, int n_omega, const void* Hk, const void* Sigma_x, double mu,
                       double mix, void* G_tau, void* stream);

/* Host helper: the inverse of gw_tau2omega_matrix(n_tau, tau, n_omega, omega) (needs
 * n_omega == n_tau), FP64 Gauss-Jordan with partial pivoting.  With it, gw_tau2omega (parity
 * 0, n_omega = n_tau) takes frequency samples back to the tau samples of the piecewise-linear
 * function whose transform they are.  Ti_host: 2 * n_tau * n_tau doubles.  GW_ERR_SHAPE when
 * n_omega != n_tau, GW_ERR_ARG for a singular matrix. */
gw_status gw_omega2tau_matrix(int n_tau, const double* tau, int n_omega, const double* omega, double* Ti_host);

const char* gw_status_string(gw_status s);
const char* gw_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GWR_H */
