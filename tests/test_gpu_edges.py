"""GPU parity at the edge shapes of the path, against the FP64 oracle.

Shapes: one atom (4 orbitals, 16 product functions); a 1 x 1 x 1 mesh (one R, one k);
one orbital and one product function per atom; the shortest tau grids (2 and 3 points, where
the polarizability's tau mirror pairs the two end points, or leaves one self-mirrored middle
point); and a 9-orbital species with 57 product functions (not a multiple of the 16-row
matrix tiles), which the BF16 split kernels cover with a ragged last tile; and seven 9-orbital
atoms with 60 functions, whose polarizability walk takes one band of four A atoms and a short
band of three (the dense P kernels walk bands of four).  Each shape runs
k -> R and R -> k, P and Sigma in FP64, FP32 and BF16 split, the tau -> Matsubara transform
and the fused drain with parity +1, -1 and 0, and the density.  Bars (max-abs error over
max-abs of the oracle): 1e-12 FP64, 2e-6 FP32 products, 1e-5 BF16 split products.  One more
case runs the BF16 split self-energy on a W that starts 8 bytes into its allocation (the
kernel's 8-byte load path) against the same W 16-byte aligned.
"""
import numpy as np
import pytest

import oracle
import synthcell as sc
from tests import cells

pytestmark = pytest.mark.gpu


def relmax(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def _one_atom():
    lat = np.diag([2.6, 2.7, 2.8])
    return sc.CellSpec("one_atom", lat, np.zeros((1, 3)), np.zeros(1, dtype=np.int64), (4,), (16,), (2, 2, 2), 16,
                       30.0, config_id=21, request_id=1, complex_hopping=True)


def _n1m1():
    lat = np.diag([2.4, 2.5, 2.6])
    pos = np.array([[0.0, 0.0, 0.0], [1.1, 1.3, 1.2]])
    return sc.CellSpec("n1m1", lat, pos, np.zeros(2, dtype=np.int64), (1,), (1,), (2, 1, 1), 6, 12.0,
                       config_id=22, request_id=2, complex_hopping=True)


def _si_m57():
    lat = np.diag([5.431, 5.431, 5.431])
    pos = np.array([[0.0, 0.0, 0.0], [1.358, 1.358, 1.358]])
    return sc.CellSpec("si_m57", lat, pos, np.zeros(2, dtype=np.int64), (9,), (57,), (2, 1, 1), 8, 40.0,
                       config_id=23, request_id=3)


def _si7_band():
    lat = np.diag([7.1, 6.8, 6.5])
    pos = np.array([[0.0, 0.0, 0.0], [1.4, 1.3, 1.5], [3.6, 0.4, 2.9], [5.2, 3.1, 0.8],
                    [2.3, 4.7, 4.4], [0.6, 5.6, 2.2], [4.9, 5.3, 5.6]])
    # 16 tau points of P times 4 R times 49 atom pairs: 3136 blocks, more than the grid of 2048
    # workgroups, so that workgroups also step from block to block along the band walk
    return sc.CellSpec("si7_band", lat, pos, np.zeros(7, dtype=np.int64), (9,), (60,), (2, 2, 1), 32, 30.0,
                       config_id=24, request_id=7)


SHAPES = {
    "one_atom": _one_atom,
    "mesh111": lambda: cells.tiny(mesh=(1, 1, 1), complex_hopping=True, request_id=4),
    "n1m1": _n1m1,
    "ntau2": lambda: cells.tiny(n_tau=2, beta=8.0, complex_hopping=True, request_id=5),
    "ntau3": lambda: cells.tiny(n_tau=3, beta=8.0, complex_hopping=True, request_id=6),
    "si_m57": _si_m57,
    "si7_band": _si7_band,
}
_cache = {}


def _case(name):
    if name not in _cache:
        spec = SHAPES[name]()
        hop, b, Gk, C = cells.inputs(spec)
        GR = oracle.k_to_r(Gk, spec.mesh)
        WR = sc.w_tensor(spec)
        _cache[name] = dict(spec=spec, Gk=Gk, C=C, GR=GR, WR=WR,
                            PR=oracle.polarizability_r(GR, spec, C, spec.spin),
                            SR=oracle.self_energy_r(GR, WR, spec, C))
    return _cache[name]


def dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    return t if dtype is None else t.to(dtype)


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("name", list(SHAPES))
def test_edge_fourier_and_density(name):
    import torch
    import paper_1911_05633_amd as g
    d = _case(name)
    spec = d["spec"]
    print(f"[edge fourier/density] {name}", flush=True)
    cell = g.Cell.from_spec(spec, d["C"])
    Gk = dev(d["Gk"])
    GR = torch.empty_like(Gk)
    g.gw_fourier_k2r(cell, Gk, GR, basis=0)
    assert relmax(host(GR), d["GR"]) < 1e-13
    back = torch.empty_like(Gk)
    g.gw_fourier_r2k(cell, GR, back, basis=0)
    assert relmax(host(back), d["Gk"]) < 1e-13
    n = torch.zeros(1, dtype=torch.float64, device="cuda")
    g.gw_density(cell, GR, spec.spin, n)
    ref = oracle.electron_count(d["GR"][-1, 0], spec.spin)
    assert abs(float(host(n)[0]) - ref) < 1e-12 * abs(ref)
    assert abs(ref - spec.spin * spec.N_orb / 2) < 1e-8


@pytest.mark.parametrize("name", list(SHAPES))
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_edge_contractions(name, prec):
    import torch
    import paper_1911_05633_amd as g
    d = _case(name)
    spec = d["spec"]
    print(f"[edge P/Sigma] {name} {prec}", flush=True)
    cell = g.Cell.from_spec(spec, d["C"])
    cdt = torch.complex128 if prec == "fp64" else torch.complex64
    GR, WR = dev(d["GR"], cdt), dev(d["WR"], cdt)
    P = torch.full((spec.n_tau, spec.N_R, spec.N_pb, spec.N_pb), float("nan"), dtype=cdt, device="cuda")
    S = torch.full((spec.n_tau, spec.N_R, spec.N_orb, spec.N_orb), float("nan"), dtype=torch.complex128,
                   device="cuda")
    g.gw_polarizability(cell, GR, P, spec.spin, prec=prec)
    g.gw_self_energy(cell, GR, WR, S, prec=prec)
    Ph, Sh = host(P).astype(np.complex128), host(S)
    assert np.all(np.isfinite(Ph)) and np.all(np.isfinite(Sh))
    SR = d["SR"]
    if prec != "fp64":  # the kernels read W in complex64 storage
        SR = oracle.self_energy_r(d["GR"], d["WR"].astype(np.complex64).astype(np.complex128), spec, d["C"])
    tol = {"fp64": 1e-12, "fp32": 2e-6, "bf16x3": 1e-5}[prec]
    eP, eS = relmax(Ph, d["PR"]), relmax(Sh, SR)
    print(f"[edge P/Sigma] {name} {prec}: P {eP:.2e}, Sigma {eS:.2e}", flush=True)
    assert eP < tol and eS < tol


def test_sigma_bf16_w_alignment():
    """The BF16 split self-energy loads each lane's pair of W columns as one 16-byte access
    only when every species has an even number of product functions and W is 16-byte aligned;
    a W that starts 8 bytes into its allocation takes the two 8-byte loads.  Both give the
    same bits, within the BF16 split bar of the oracle."""
    import torch
    import paper_1911_05633_amd as g
    d = _case("si7_band")
    spec = d["spec"]
    print("[edge Sigma W alignment] si7_band bf16x3", flush=True)
    cell = g.Cell.from_spec(spec, d["C"])
    GR = dev(d["GR"], torch.complex64)
    WR = dev(d["WR"], torch.complex64)
    buf = torch.empty(WR.numel() + 1, dtype=torch.complex64, device="cuda")
    WR8 = buf[1:].view(WR.shape)
    WR8.copy_(WR)
    assert WR.data_ptr() % 16 == 0 and WR8.data_ptr() % 16 == 8
    out = []
    for W in (WR, WR8):
        S = torch.full((spec.n_tau, spec.N_R, spec.N_orb, spec.N_orb), float("nan"), dtype=torch.complex128,
                       device="cuda")
        g.gw_self_energy(cell, GR, W, S, prec="bf16x3")
        out.append(host(S))
    assert np.array_equal(out[0], out[1])
    SR = oracle.self_energy_r(d["GR"], d["WR"].astype(np.complex64).astype(np.complex128), spec, d["C"])
    assert relmax(out[0], SR) < 1e-5


@pytest.mark.parametrize("name", list(SHAPES))
@pytest.mark.parametrize("basis,parity", [(0, -1), (0, 0), (1, 1), (1, 0)])
def test_edge_transforms(name, basis, parity):
    import torch
    import paper_1911_05633_amd as g
    d = _case(name)
    spec = d["spec"]
    print(f"[edge omega] {name} basis {basis} parity {parity}", flush=True)
    cell = g.Cell.from_spec(spec, d["C"])
    n = spec.N_orb if basis == 0 else spec.N_pb
    F = sc.random_complex((spec.n_tau, spec.N_R, n, n), seed=31 + basis)
    tau = sc.tau_grid(spec)
    kind = "fermionic" if basis == 0 else "bosonic"
    w = g.matsubara(spec.n_tau, spec.beta, kind)
    To = oracle.filon_matrix(tau, oracle.fermionic_frequencies(spec.n_tau, spec.beta) if kind == "fermionic"
                             else oracle.bosonic_frequencies(spec.n_tau, spec.beta))
    Td, Fd = dev(g.gw_tau2omega_matrix(tau, w)), dev(F)
    out = torch.empty_like(Fd)
    g.gw_tau2omega(cell, Td, Fd, out, basis=basis, parity=parity)
    assert relmax(host(out), oracle.apply_tau_to_omega(To, F)) < 1e-12
    ref_d = oracle.apply_tau_to_omega(To, oracle.r_to_k(F, spec.mesh))
    g.gw_drain(cell, Td, Fd, out, basis=basis, parity=parity)
    assert relmax(host(out), ref_d) < 1e-12
    F3 = Fd.to(torch.complex64)
    g.gw_drain(cell, Td, F3, F3, basis=basis, parity=parity)
    assert relmax(host(F3).astype(np.complex128), ref_d) < 1e-6
