"""GPU parity of the packed storage of the cutoff path (Sec. 2, Figs. 1 and 2) against the oracle.

A tau slice of a packed tensor holds the kept (R, A, B) blocks in the cell's list order, each as
its mA x mB kept functions.  gw_polarizability_packed must write the oracle's truncated blocks
there (every kept block, every tau); gw_self_energy_packed must read W there and give the
oracle's Sigma blocks; the lattice sums between the packed layout and dense k space must match
the oracle's r_to_k / k_to_r of the dense tensors the blocks stand for; the packed drain must
match the oracle's tau -> Matsubara of that R -> k.  FP64 bars 1e-12, complex64 storage 2e-6.
The packed slice is checked against the oracle planner's sum of mA mB.
"""
import numpy as np
import pytest

import oracle
import synthcell as sc
from tests import cells

pytestmark = pytest.mark.gpu

CASES = {
    "tiny": (lambda: cells.tiny(complex_hopping=True), 2.0, 2.6, [[10, 6]]),
    "two_species": (lambda: cells.two_species(), 1.0, 1.6, [[4, 2], [3, 1]]),
    "si8": (lambda: sc.config(2), 2.5, 4.6, [[40, 16]]),
}


def relmax(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


_cache = {}


def _setup(name):
    import paper_1911_05633_amd as g
    make, rb, rc, mt = CASES[name]
    spec = make()
    if name not in _cache:
        hop, b, Gk, C = cells.inputs(spec)
        plan = oracle.plan_pairs(spec.lattice, spec.positions, spec.species, spec.n_pb, spec.mesh, rb, rc, mt)
        _cache[name] = (C, oracle.k_to_r(Gk, spec.mesh), plan)
    C, GR, plan = _cache[name]
    cell = g.Cell.from_spec(spec, C)
    cell.set_pairs(spec.lattice, spec.positions, rb, rc, mt)
    return spec, C, GR, plan, cell


def _offsets(plan):
    sizes = plan[:, 3].astype(np.int64) * plan[:, 4]
    return np.concatenate([[0], np.cumsum(sizes)])


def _pack(dense, spec, plan):
    """Host packing of a dense [n_tau][N_R][N_pb][N_pb] tensor by the plan (layout only)."""
    off, po = _offsets(plan), np.asarray(spec.pb_off)
    out = np.zeros((dense.shape[0], off[-1]), dtype=dense.dtype)
    for b, (R, A, B, mA, mB) in enumerate(plan.tolist()):
        out[:, off[b]:off[b + 1]] = dense[:, R, po[A]:po[A] + mA, po[B]:po[B] + mB].reshape(dense.shape[0], -1)
    return out


def _unpack(pk, spec, plan):
    """The dense tensor a packed one stands for (zero outside the kept blocks' functions)."""
    off, po = _offsets(plan), np.asarray(spec.pb_off)
    out = np.zeros((pk.shape[0], spec.N_R, spec.N_pb, spec.N_pb), dtype=np.complex128)
    for b, (R, A, B, mA, mB) in enumerate(plan.tolist()):
        out[:, R, po[A]:po[A] + mA, po[B]:po[B] + mB] = pk[:, off[b]:off[b + 1]].reshape(-1, mA, mB)
    return out


def _taus(spec):
    return list(range(spec.n_tau)) if spec.n_tau <= 16 else [0, 3, spec.n_tau // 2, spec.n_tau - 1]


@pytest.mark.parametrize("name,prec", [("tiny", "fp64"), ("two_species", "fp64"), ("si8", "fp64"),
                                       ("two_species", "fp32"), ("si8", "fp32"), ("si8", "bf16x3")])
def test_packed_contractions(name, prec):
    import torch
    import paper_1911_05633_amd as g
    print(f"[packed P/Sigma] {name} {prec}", flush=True)
    spec, C, GR_h, plan, cell = _setup(name)
    off = _offsets(plan)
    assert cell.packed_elems() == off[-1]
    cdt = torch.complex128 if prec == "fp64" else torch.complex64
    GR = torch.from_numpy(np.ascontiguousarray(GR_h)).cuda().to(cdt)
    P = torch.full((spec.n_tau, off[-1]), float("nan"), dtype=cdt, device="cuda")
    g.gw_polarizability_packed(cell, GR, P, spec.spin, prec=prec)
    WR_h = sc.w_tensor(spec)
    Wpk_h = _pack(WR_h, spec, plan)
    S = torch.full((spec.n_tau, spec.N_R, spec.N_orb, spec.N_orb), float("nan"), dtype=torch.complex128,
                   device="cuda")
    g.gw_self_energy_packed(cell, GR, torch.from_numpy(Wpk_h).cuda().to(cdt), S, prec=prec)
    torch.cuda.synchronize()
    Ph, Sh = P.cpu().numpy().astype(np.complex128), S.cpu().numpy()
    assert np.all(np.isfinite(Ph))
    oo, po = np.asarray(spec.orb_off), np.asarray(spec.pb_off)
    cmpP, cmpS = [], []
    for b, (R, A, B, mA, mB) in enumerate(plan.tolist()):
        for t in _taus(spec):
            ref = oracle.polarizability_r_block_cut(GR_h, spec, C, spec.spin, t, R, A, B, mA, mB)[:mA, :mB]
            cmpP.append((Ph[t, off[b]:off[b + 1]].reshape(mA, mB), ref))
            Wb = WR_h[t, R, po[A]:po[A + 1], po[B]:po[B + 1]]
            if prec != "fp64":
                Wb = Wb.astype(np.complex64).astype(np.complex128)
            cmpS.append((Sh[t, R, oo[A]:oo[A + 1], oo[B]:oo[B + 1]],
                         oracle.self_energy_r_block_cut(GR_h, Wb, spec, C, t, R, A, B, mA, mB)))
    eP = max(float(np.max(np.abs(a - b))) for a, b in cmpP) / max(float(np.max(np.abs(b))) for _, b in cmpP)
    eS = max(float(np.max(np.abs(a - b))) for a, b in cmpS) / max(float(np.max(np.abs(b))) for _, b in cmpS)
    tol = 1e-12 if prec == "fp64" else 2e-6
    print(f"[packed P/Sigma] {name} {prec}: {len(plan)} blocks, {off[-1]} per tau, P {eP:.2e}, Sigma {eS:.2e}",
          flush=True)
    assert eP <= tol and eS <= tol


@pytest.mark.parametrize("name", ["tiny", "two_species", "si8"])
def test_packed_lattice_sums_and_drain(name):
    import torch
    import paper_1911_05633_amd as g
    print(f"[packed r2k/k2r/drain] {name}", flush=True)
    spec, C, GR_h, plan, cell = _setup(name)
    off = _offsets(plan)
    Fpk = sc.random_complex((spec.n_tau, off[-1]), seed=41)
    dense = _unpack(Fpk, spec, plan)
    Fk = torch.empty((spec.n_tau, spec.N_R, spec.N_pb, spec.N_pb), dtype=torch.complex128, device="cuda")
    Fd = torch.from_numpy(Fpk).cuda()
    g.gw_fourier_r2k_packed(cell, Fd, Fk)
    torch.cuda.synchronize()
    assert relmax(Fk.cpu().numpy(), oracle.r_to_k(dense, spec.mesh)) < 1e-12
    # k -> R of a dense k-space tensor, kept blocks only
    Gq = sc.random_complex((spec.n_tau, spec.N_R, spec.N_pb, spec.N_pb), seed=42)
    back = torch.full((spec.n_tau, off[-1]), float("nan"), dtype=torch.complex128, device="cuda")
    g.gw_fourier_k2r_packed(cell, torch.from_numpy(Gq).cuda(), back)
    torch.cuda.synchronize()
    assert relmax(back.cpu().numpy(), _pack(oracle.k_to_r(Gq, spec.mesh), spec, plan)) < 1e-12
    # complex64 packed in, complex128 out
    Fk2 = torch.empty_like(Fk)
    g.gw_fourier_r2k_packed(cell, Fd.to(torch.complex64), Fk2)
    torch.cuda.synchronize()
    assert relmax(Fk2.cpu().numpy(), oracle.r_to_k(dense, spec.mesh)) < 2e-7
    # drain: R -> k then tau -> Matsubara (bosonic, parity +1 and 0)
    tau = sc.tau_grid(spec)
    nu = g.matsubara(spec.n_tau, spec.beta, "bosonic")
    T = torch.from_numpy(g.gw_tau2omega_matrix(tau, nu)).cuda()
    ref = oracle.apply_tau_to_omega(oracle.filon_matrix(tau, oracle.bosonic_frequencies(spec.n_tau, spec.beta)),
                                    oracle.r_to_k(dense, spec.mesh))
    for par in (1, 0):
        out = torch.empty_like(Fk)
        g.gw_drain_packed(cell, T, Fd, out, parity=par)
        torch.cuda.synchronize()
        assert relmax(out.cpu().numpy(), ref) < 1e-12


def test_packed_equals_the_dense_list_path():
    """The packed blocks are the blocks gw_polarizability_pairs writes into the dense layout."""
    import torch
    import paper_1911_05633_amd as g
    spec, C, GR_h, plan, cell = _setup("two_species")
    off = _offsets(plan)
    GR = torch.from_numpy(np.ascontiguousarray(GR_h)).cuda()
    Pd = torch.zeros((spec.n_tau, spec.N_R, spec.N_pb, spec.N_pb), dtype=torch.complex128, device="cuda")
    g.gw_polarizability_pairs(cell, GR, Pd, spec.spin)
    Pp = torch.empty((spec.n_tau, off[-1]), dtype=torch.complex128, device="cuda")
    g.gw_polarizability_packed(cell, GR, Pp, spec.spin)
    torch.cuda.synchronize()
    assert relmax(Pp.cpu().numpy(), _pack(Pd.cpu().numpy(), spec, plan)) < 1e-13
