"""Seeded synthetic cells: the inputs of the space-time P/Sigma path.

This module produces input data only.  It holds none of the arithmetic of the
path itself (no lattice sums of Green's functions, no polarizability or
self-energy, no Matsubara transform).  Both the HIP library and the CPU
oracle consume what it returns; neither is imported here.

What it builds, per cell (units: Hartree, Angstrom, beta in 1/Ha):

* geometry: lattice vectors, atom positions, species, orbitals n_s and
  product functions m_s per species, Born-von Karman mesh N1 x N2 x N3,
  uniform imaginary-time grid tau_i = beta * i / (N_tau - 1);
* a tight-binding Hamiltonian: onsite levels ~ U[-0.5, 0.5] Ha, hoppings
  h0 * xi * exp(-d / 2 A) with xi ~ U[-1, 1] for every orbital pair and every
  lattice translation with n_i in {-1, 0, 1}, d = |R + t_a - t_b|;
* the Green's function input G(k, tau) = -U diag(g(eps - mu, tau)) U^+ with
  mu at half filling, g in the overflow-free form of (1 - f) exp(-x tau);
* product-basis coefficients C^I_ab (real, symmetric in a, b; one set per
  species, as the atom-local vertices <M_K | phi_L phi_L''> of Eqs. (5), (8));
* the screened interaction W^R_IJ(tau) = A_IJ exp(-|R|_min / 3 A) exp(-tau / 5)
  with A = B B^T / N_pb + 0.5 I, B ~ N(0, 1).

Every random draw comes from numpy's PCG64 seeded with
SeedSequence([19110563, config_id, request_id]) and spawned sub-streams in a
fixed order (hoppings, coefficients, interaction, arrivals).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Sequence, Tuple

import numpy as np

ROOT_SEED = 19110563
H0_HOP = 0.25  # Ha, hopping scale


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------
@dataclass
class CellSpec:
    """A synthetic crystal: geometry, basis sizes, k-mesh and tau grid."""

    name: str
    lattice: np.ndarray  # (3, 3) rows are lattice vectors (A)
    positions: np.ndarray  # (N_at, 3) Cartesian (A)
    species: np.ndarray  # (N_at,) int species index
    n_orb: Tuple[int, ...]  # orbitals per species
    n_pb: Tuple[int, ...]  # product functions per species
    mesh: Tuple[int, int, int]
    n_tau: int
    beta: float
    spin: float = 2.0
    config_id: int = 0
    request_id: int = 0
    complex_hopping: bool = False

    @property
    def n_atoms(self) -> int:
        return int(len(self.species))

    @property
    def n_species(self) -> int:
        return len(self.n_orb)

    @property
    def atom_norb(self) -> np.ndarray:
        return np.array([self.n_orb[s] for s in self.species], dtype=np.int64)

    @property
    def atom_npb(self) -> np.ndarray:
        return np.array([self.n_pb[s] for s in self.species], dtype=np.int64)

    @property
    def N_orb(self) -> int:
        return int(self.atom_norb.sum())

    @property
    def N_pb(self) -> int:
        return int(self.atom_npb.sum())

    @property
    def N_R(self) -> int:
        return int(np.prod(self.mesh))

    @property
    def orb_off(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.atom_norb)]).astype(np.int64)

    @property
    def pb_off(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.atom_npb)]).astype(np.int64)

    @property
    def tau(self) -> np.ndarray:
        """The cell's imaginary-time grid (tau_grid)."""
        return tau_grid(self)

    def seed(self) -> np.random.SeedSequence:
        return np.random.SeedSequence([ROOT_SEED, self.config_id, self.request_id])


def _diamond_sites() -> np.ndarray:
    return np.array(
        [
            [0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0],
            [0.25, 0.25, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75], [0.75, 0.75, 0.25],
        ]
    )


def si_supercell(rep: Tuple[int, int, int], mesh, n_tau, beta, name, config_id, request_id=0,
                 n_orb=9, n_pb=60) -> CellSpec:
    """rep[0] x rep[1] x rep[2] copies of the 8-site conventional diamond cell (a = 5.431 A)."""
    a = 5.431
    frac = []
    for i in range(rep[0]):
        for j in range(rep[1]):
            for k in range(rep[2]):
                for s in _diamond_sites():
                    frac.append([(s[0] + i) / rep[0], (s[1] + j) / rep[1], (s[2] + k) / rep[2]])
    lat = np.diag([a * rep[0], a * rep[1], a * rep[2]])
    pos = np.array(frac) @ lat
    return CellSpec(name, lat, pos, np.zeros(len(pos), dtype=np.int64), (n_orb,), (n_pb,),
                    tuple(mesh), n_tau, beta, config_id=config_id, request_id=request_id)


def tiny_cell(config_id=1, request_id=0, n_tau=16, beta=50.0, mesh=(2, 2, 2),
              n_orb=4, n_pb=16) -> CellSpec:
    """Simple-cubic two-atom cell, a = 2.715 A (nearest neighbour 2.35 A)."""
    a = 2.715
    lat = np.diag([a, a, a])
    pos = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]]) @ lat
    return CellSpec("tiny2", lat, pos, np.zeros(2, dtype=np.int64), (n_orb,), (n_pb,),
                    tuple(mesh), n_tau, beta, config_id=config_id, request_id=request_id)


def oxide56(config_id=4, request_id=0, n_tau=64, beta=400.0) -> CellSpec:
    """Layered oxide-like cell: 8 transition-metal sites (16 orb, 100 pb), 48 light sites (9, 60)."""
    a, c = 7.56, 13.2
    lat = np.diag([a, a, c])
    tm, light = [], []
    for i in range(2):
        for j in range(2):
            for l in range(2):
                tm.append([i / 2, j / 2, l / 2])
    for i in range(2):
        for j in range(2):
            for l in range(2):
                light.append([(i + 0.5) / 2, j / 2, l / 2])  # in-plane bridges (x)
                light.append([i / 2, (j + 0.5) / 2, l / 2])  # in-plane bridges (y)
    for i in range(2):
        for j in range(2):
            for l in range(2):
                light.append([i / 2, j / 2, l / 2 + 0.18])  # apical above
                light.append([i / 2, j / 2, l / 2 - 0.18])  # apical below
    for i in range(2):
        for j in range(2):
            for l in range(2):
                light.append([(i + 0.5) / 2, (j + 0.5) / 2, l / 2 + 0.14])  # spacers
                light.append([(i + 0.5) / 2, (j + 0.5) / 2, l / 2 - 0.14])
    frac = np.array(tm + light) % 1.0
    pos = frac @ lat
    species = np.array([0] * len(tm) + [1] * len(light), dtype=np.int64)
    return CellSpec("oxide56", lat, pos, species, (16, 9), (100, 60), (2, 2, 1), n_tau, beta,
                    config_id=config_id, request_id=request_id)


def config(i: int, request_id: int = 0) -> CellSpec:
    """The four fixed workloads: 1 tiny, 2 Si8, 3 Si72, 4 oxide56."""
    if i == 1:
        return tiny_cell(1, request_id)
    if i == 2:
        return si_supercell((1, 1, 1), (4, 4, 4), 32, 100.0, "si8", 2, request_id)
    if i == 3:
        return si_supercell((3, 3, 1), (2, 2, 2), 48, 200.0, "si72", 3, request_id)
    if i == 4:
        return oxide56(4, request_id)
    raise ValueError(f"unknown config {i}")


def serving_cell(kind: str, n_tau: int, request_id: int) -> CellSpec:
    """Cells of the serving mix: tiny2, si8, si24, si40, si72."""
    if kind == "tiny2":
        return tiny_cell(5, request_id, n_tau=n_tau, beta=50.0)
    if kind == "si8":
        return si_supercell((1, 1, 1), (4, 4, 4), n_tau, 100.0, "si8", 5, request_id)
    if kind == "si24":
        return si_supercell((3, 1, 1), (2, 2, 2), n_tau, 200.0, "si24", 5, request_id)
    if kind == "si40":
        return si_supercell((5, 1, 1), (2, 2, 2), n_tau, 200.0, "si40", 5, request_id)
    if kind == "si72":
        return si_supercell((3, 3, 1), (2, 2, 2), n_tau, 200.0, "si72", 5, request_id)
    raise ValueError(kind)


SERVING_KINDS = ("tiny2", "si8", "si24", "si40", "si72")
SERVING_NTAU = (16, 24, 32, 40, 48)


# ----------------------------------------------------------------------------
# random streams
# ----------------------------------------------------------------------------
def _streams(spec: CellSpec) -> List[np.random.Generator]:
    kids = spec.seed().spawn(4)  # hoppings, coefficients, interaction, arrivals
    return [np.random.Generator(np.random.PCG64(k)) for k in kids]


# ----------------------------------------------------------------------------
# lattice bookkeeping (index order shared by every consumer)
# ----------------------------------------------------------------------------
def mesh_points(mesh) -> np.ndarray:
    """Integer triples (n1, n2, n3), index = (n1 * N2 + n2) * N3 + n3."""
    N1, N2, N3 = mesh
    g = np.array([[i, j, k] for i in range(N1) for j in range(N2) for k in range(N3)], dtype=np.int64)
    return g


def tau_grid(spec: CellSpec) -> np.ndarray:
    """Uniform grid on [0, beta]; tau_0 stands for 0+ and tau_{N-1} for beta-."""
    return spec.beta * np.arange(spec.n_tau) / (spec.n_tau - 1)


def min_image_length(spec: CellSpec, n: Sequence[int]) -> float:
    """Length of the shortest lattice vector equivalent to n modulo the mesh."""
    best = np.inf
    for s1 in (-1, 0, 1):
        for s2 in (-1, 0, 1):
            for s3 in (-1, 0, 1):
                m = np.array([n[0] + s1 * spec.mesh[0], n[1] + s2 * spec.mesh[1], n[2] + s3 * spec.mesh[2]])
                best = min(best, float(np.linalg.norm(m @ spec.lattice)))
    return best


# ----------------------------------------------------------------------------
# tight-binding Hamiltonian
# ----------------------------------------------------------------------------
def hoppings(spec: CellSpec) -> Dict[Tuple[int, int, int], np.ndarray]:
    """H^R_ab = <a in cell R | H | b in cell 0> for R in {-1,0,1}^3 (lattice units).

    H^{-R} = (H^R)^+ so that H(k) is Hermitian.
    """
    rng = _streams(spec)[0]
    No = spec.N_orb
    orb_atom = np.repeat(np.arange(spec.n_atoms), spec.atom_norb)
    pos_o = spec.positions[orb_atom]  # (No, 3)
    Rs = [(i, j, k) for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)]
    xi = {R: rng.uniform(-1.0, 1.0, size=(No, No)) for R in Rs}
    psi = {R: rng.uniform(-1.0, 1.0, size=(No, No)) for R in Rs} if spec.complex_hopping else None
    onsite = rng.uniform(-0.5, 0.5, size=No)
    H = {}
    for R in Rs:
        mR = (-R[0], -R[1], -R[2])
        Rc = np.array(R, dtype=float) @ spec.lattice
        d = np.linalg.norm(Rc[None, None, :] + pos_o[:, None, :] - pos_o[None, :, :], axis=-1)
        amp = 0.5 * (xi[R] + xi[mR].T)
        h = H0_HOP * np.exp(-d / 2.0) * amp
        if psi is not None:
            h = h + 1j * H0_HOP * np.exp(-d / 2.0) * 0.5 * (psi[R] - psi[mR].T)
        if R == (0, 0, 0):
            h = np.array(h)
            np.fill_diagonal(h, onsite)
        H[R] = h
    return H


def hamiltonian_k(spec: CellSpec, H: Dict[Tuple[int, int, int], np.ndarray]) -> np.ndarray:
    """H(k) = sum_R exp(-i k.R) H^R on the mesh; k = (j1/N1, j2/N2, j3/N3)."""
    ks = mesh_points(spec.mesh) / np.array(spec.mesh, dtype=float)
    Hk = np.zeros((spec.N_R, spec.N_orb, spec.N_orb), dtype=np.complex128)
    for R, h in H.items():
        ph = np.exp(-2j * np.pi * (ks @ np.array(R, dtype=float)))
        Hk += ph[:, None, None] * h[None]
    return 0.5 * (Hk + np.conj(np.transpose(Hk, (0, 2, 1))))


def fermi(x: np.ndarray, beta: float) -> np.ndarray:
    return 0.5 * (1.0 - np.tanh(0.5 * beta * x))


def chemical_potential(eps: np.ndarray, beta: float, n_target: float) -> float:
    """Bisection on sum f(eps - mu) / N_k = n_target (200 halvings)."""
    lo, hi = float(eps.min()) - 1.0, float(eps.max()) + 1.0
    nk = eps.shape[0]
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if fermi(eps - mid, beta).sum() / nk > n_target:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def _g_factor(x: np.ndarray, tau: float, beta: float) -> np.ndarray:
    """(1 - f(x)) exp(-x tau), written so that no exponent is positive."""
    out = np.empty_like(x)
    pos = x >= 0
    xp = x[pos]
    out[pos] = np.exp(-xp * tau) / (1.0 + np.exp(-xp * beta))
    xn = x[~pos]
    out[~pos] = np.exp(xn * (beta - tau)) / (1.0 + np.exp(xn * beta))
    return out


@dataclass
class Bands:
    eps: np.ndarray  # (N_k, N_orb)
    U: np.ndarray  # (N_k, N_orb, N_orb)
    mu: float


def bands(spec: CellSpec, H=None) -> Bands:
    if H is None:
        H = hoppings(spec)
    Hk = hamiltonian_k(spec, H)
    eps, U = np.linalg.eigh(Hk)
    mu = chemical_potential(eps, spec.beta, spec.N_orb / 2.0)
    return Bands(eps, U, mu)


def green_ktau(spec: CellSpec, b: Bands = None, dtype=np.complex128) -> np.ndarray:
    """Input G(k, tau_i), layout [tau][k][a][b]."""
    if b is None:
        b = bands(spec)
    taus = tau_grid(spec)
    x = b.eps - b.mu
    out = np.empty((spec.n_tau, spec.N_R, spec.N_orb, spec.N_orb), dtype=dtype)
    Uh = np.conj(np.transpose(b.U, (0, 2, 1)))
    for i, t in enumerate(taus):
        g = _g_factor(x, t, spec.beta)  # (N_k, N_orb)
        out[i] = -np.matmul(b.U * g[:, None, :], Uh)
    return out


# ----------------------------------------------------------------------------
# product basis coefficients
# ----------------------------------------------------------------------------
def coefficients(spec: CellSpec) -> List[np.ndarray]:
    """Per species C[I, a, b] (m x n x n), symmetric in (a, b), upper triangle ~ N(0, 1)."""
    rng = _streams(spec)[1]
    out = []
    for s in range(spec.n_species):
        m, n = spec.n_pb[s], spec.n_orb[s]
        raw = rng.standard_normal((m, n, n))
        up = np.triu(raw)
        C = up + np.transpose(np.triu(raw, 1), (0, 2, 1))
        out.append(np.ascontiguousarray(C))
    return out


# ----------------------------------------------------------------------------
# screened interaction
# ----------------------------------------------------------------------------
def w_amplitude(spec: CellSpec) -> np.ndarray:
    """A = B B^T / N_pb + 0.5 I (random SPD, N_pb x N_pb)."""
    rng = _streams(spec)[2]
    Np = spec.N_pb
    B = rng.standard_normal((Np, Np))
    A = B @ B.T / Np
    A[np.diag_indices(Np)] += 0.5
    return A


def w_factors(spec: CellSpec) -> Tuple[np.ndarray, np.ndarray]:
    """W^R_IJ(tau_i) = A_IJ * sR[R] * et[i]."""
    pts = mesh_points(spec.mesh)
    sR = np.array([np.exp(-min_image_length(spec, p) / 3.0) for p in pts])
    et = np.exp(-tau_grid(spec) / 5.0)
    return sR, et


def w_tensor(spec: CellSpec, A: np.ndarray = None, dtype=np.complex128) -> np.ndarray:
    """Full W, layout [tau][R][I][J] (small cells only)."""
    if A is None:
        A = w_amplitude(spec)
    sR, et = w_factors(spec)
    return (et[:, None, None, None] * sR[None, :, None, None] * A[None, None]).astype(dtype)


# ----------------------------------------------------------------------------
# serving request stream
# ----------------------------------------------------------------------------
@dataclass
class Request:
    request_id: int
    arrival: float  # seconds after the stream starts
    kind: str
    n_tau: int


def request_stream(n_requests: int, rate: float, seed_id: int = 5, burst: bool = False) -> List[Request]:
    """Poisson arrivals (rate per second); cell kind and N_tau drawn uniformly."""
    rng = _streams(CellSpec("stream", np.eye(3), np.zeros((1, 3)), np.zeros(1, dtype=np.int64),
                            (1,), (1,), (1, 1, 1), 2, 1.0, config_id=seed_id))[3]
    gaps = rng.exponential(1.0 / rate, size=n_requests) if rate > 0 else np.zeros(n_requests)
    kinds = rng.integers(0, len(SERVING_KINDS), size=n_requests)
    ntaus = rng.integers(0, len(SERVING_NTAU), size=n_requests)
    t = 0.0 if burst else np.cumsum(gaps)
    out = []
    for r in range(n_requests):
        arr = 0.0 if burst else float(t[r])
        out.append(Request(r, arr, SERVING_KINDS[kinds[r]], SERVING_NTAU[ntaus[r]]))
    return out


def random_complex(shape, seed: int, dtype=np.complex128) -> np.ndarray:
    """Plain seeded complex noise for kernel-level tests."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([ROOT_SEED, 99, seed])))
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(dtype)


def dyson_factors(n_k: int, n: int, n_omega: int, seed: int, scale: float = 0.5):
    """Seeded raw factors of the screened-interaction inputs: complex Gaussian B, X [n_k][n][n]
    and s [n_omega] = scale / (1 + m).  With them V(q) = B_q B_q^H / n + 0.5 I (Hermitian
    positive definite, a stand-in for the bare Coulomb matrix) and P(q, nu_m) =
    -s_m X_q X_q^H / n (Hermitian negative semidefinite and decaying over the frequency index,
    as a polarizability at bosonic frequencies is)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([ROOT_SEED, 71, seed])))
    B = rng.standard_normal((n_k, n, n)) + 1j * rng.standard_normal((n_k, n, n))
    X = rng.standard_normal((n_k, n, n)) + 1j * rng.standard_normal((n_k, n, n))
    s = scale / (1.0 + np.arange(n_omega, dtype=np.float64))
    return B, X, s


def dyson_inputs(n_k: int, n: int, n_omega: int, seed: int, scale: float = 0.5):
    """V [n_k][n][n], X [n_k][n][n] and s [n_omega] of dyson_factors, with V formed on the host
    (small cases)."""
    B, X, s = dyson_factors(n_k, n, n_omega, seed, scale)
    V = B @ np.conj(np.swapaxes(B, -1, -2)) / n
    V[:, np.arange(n), np.arange(n)] += 0.5
    return V, X, s
