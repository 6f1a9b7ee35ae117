"""GPU parity of the real-space cutoff path (Sec. 2, Figs. 1 and 2) against the oracle.

gw_cell_set_pairs must plan exactly the oracle's kept blocks (integers, compared as sets).
gw_polarizability_pairs / gw_self_energy_pairs must reproduce the oracle's truncated blocks
for every kept (R, A, B) at the sampled tau points, and must leave every other block
untouched (the outputs start as NaN).  The matrix-core kernels walk the list for the shapes
they cover (the FP64 Sigma and other shapes use the plain kernels).  Bars: 1e-12 relative
(FP64), 2e-6 (complex64 storage, FP32 products), 1e-5 (BF16 split products), normwise over
the sample.  The coarse-mesh refusal and the call without a list
are checked as errors.
"""
import numpy as np
import pytest

import oracle
import synthcell as sc
from tests import cells

pytestmark = pytest.mark.gpu

CASES = {
    # name: (spec factory, r_b, r_c, m_tier per species)
    "tiny": (lambda: cells.tiny(complex_hopping=True), 2.0, 2.6, [[10, 6]]),
    "two_species": (lambda: cells.two_species(), 1.0, 1.6, [[4, 2], [3, 1]]),
    "si8": (lambda: sc.config(2), 2.5, 4.6, [[40, 16]]),
}


def relmax(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def _setup(name):
    import paper_1911_05633_amd as g
    make, rb, rc, mt = CASES[name]
    spec = make()
    hop, b, Gk, C = cells.inputs(spec)
    GR = oracle.k_to_r(Gk, spec.mesh)
    cell = g.Cell.from_spec(spec, C)
    n = cell.set_pairs(spec.lattice, spec.positions, rb, rc, mt)
    plan = oracle.plan_pairs(spec.lattice, spec.positions, spec.species, spec.n_pb, spec.mesh, rb, rc, mt)
    return spec, C, GR, cell, n, plan


@pytest.mark.parametrize("name", list(CASES))
def test_pair_plan_matches_oracle(name):
    print(f"[pairs plan] {name}", flush=True)
    spec, C, GR, cell, n, plan = _setup(name)
    got = {tuple(r) for r in cell.pairs().tolist()}
    want = {tuple(int(x) for x in r) for r in plan.tolist()}
    assert n == len(plan) and got == want


@pytest.mark.parametrize("name,prec", [("tiny", "fp64"), ("two_species", "fp64"), ("si8", "fp64"),
                                       ("tiny", "fp32"), ("two_species", "fp32"), ("si8", "fp32"),
                                       ("si8", "bf16x3")])
def test_contractions_over_pairs(name, prec):
    import torch
    import paper_1911_05633_amd as g
    print(f"[pairs P/Sigma] {name} {prec}", flush=True)
    spec, C, GR_h, cell, n, plan = _setup(name)
    cdt = torch.complex128 if prec == "fp64" else torch.complex64
    GR = torch.from_numpy(np.ascontiguousarray(GR_h)).cuda().to(cdt)
    WR_h = sc.w_tensor(spec)
    WR = torch.from_numpy(np.ascontiguousarray(WR_h)).cuda().to(cdt)
    P = torch.full((spec.n_tau, spec.N_R, spec.N_pb, spec.N_pb), float("nan"), dtype=cdt, device="cuda")
    S = torch.full((spec.n_tau, spec.N_R, spec.N_orb, spec.N_orb), float("nan"), dtype=torch.complex128,
                   device="cuda")
    g.gw_polarizability_pairs(cell, GR, P, spec.spin, prec=prec)
    g.gw_self_energy_pairs(cell, GR, WR, S, prec=prec)
    torch.cuda.synchronize()
    Ph, Sh = P.cpu().numpy(), S.cpu().numpy()
    po, oo = np.asarray(spec.pb_off), np.asarray(spec.orb_off)
    taus = list(range(spec.n_tau)) if spec.n_tau <= 16 else [0, 1, spec.n_tau // 2, spec.n_tau - 1]
    kept = np.zeros((spec.N_R, spec.n_atoms, spec.n_atoms), dtype=bool)
    cmpP, cmpS = [], []
    for R, A, B, mA, mB in plan.tolist():
        kept[R, A, B] = True
        for t in taus:
            cmpP.append((Ph[t, R, po[A]:po[A + 1], po[B]:po[B + 1]].astype(np.complex128),
                         oracle.polarizability_r_block_cut(GR_h, spec, C, spec.spin, t, R, A, B, mA, mB)))
            Wb = WR_h[t, R, po[A]:po[A + 1], po[B]:po[B + 1]]
            if prec != "fp64":
                Wb = Wb.astype(np.complex64).astype(np.complex128)  # the storage the kernel reads
            cmpS.append((Sh[t, R, oo[A]:oo[A + 1], oo[B]:oo[B + 1]],
                         oracle.self_energy_r_block_cut(GR_h, Wb, spec, C, t, R, A, B, mA, mB)))
    eP = max(float(np.max(np.abs(a - b))) for a, b in cmpP) / max(float(np.max(np.abs(b))) for _, b in cmpP)
    eS = max(float(np.max(np.abs(a - b))) for a, b in cmpS) / max(float(np.max(np.abs(b))) for _, b in cmpS)
    # blocks outside the list are not written
    for R in range(spec.N_R):
        for A in range(spec.n_atoms):
            for B in range(spec.n_atoms):
                pb = Ph[:, R, po[A]:po[A + 1], po[B]:po[B + 1]]
                sb = Sh[:, R, oo[A]:oo[A + 1], oo[B]:oo[B + 1]]
                if kept[R, A, B]:
                    assert np.all(np.isfinite(pb)) and np.all(np.isfinite(sb))
                else:
                    assert np.all(np.isnan(pb)) and np.all(np.isnan(sb))
    tol = {"fp64": 1e-12, "fp32": 2e-6, "bf16x3": 1e-5}[prec]
    print(f"[pairs P/Sigma] {name} {prec}: {n} blocks, P {eP:.2e}, Sigma {eS:.2e}", flush=True)
    assert eP <= tol and eS <= tol


def test_coarse_mesh_and_missing_list_are_errors():
    import torch
    import paper_1911_05633_amd as g
    spec = cells.tiny(mesh=(1, 1, 1))
    hop, b, Gk, C = cells.inputs(spec)
    cell = g.Cell.from_spec(spec, C)
    GR = torch.zeros((spec.n_tau, spec.N_R, spec.N_orb, spec.N_orb), dtype=torch.complex128, device="cuda")
    P = torch.zeros((spec.n_tau, spec.N_R, spec.N_pb, spec.N_pb), dtype=torch.complex128, device="cuda")
    with pytest.raises(g.GWError):
        g.gw_polarizability_pairs(cell, GR, P, 2.0)
    with pytest.raises(g.GWError):
        cell.set_pairs(spec.lattice, spec.positions, 1.0, 3.0, [[8, 4]])  # images 2.715 apart
    with pytest.raises(ValueError):
        oracle.plan_pairs(spec.lattice, spec.positions, spec.species, spec.n_pb, spec.mesh, 1.0, 3.0, [[8, 4]])


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_contractions_over_pairs_si24_sampled(prec):
    """24-atom diamond cell (3 x 1 x 1 of the 8-atom one) at r_c = 4.6 A: the plan equals the
    oracle's, and sampled kept blocks (tiers A, B and C) match the oracle's truncated blocks at
    three tau points while sampled blocks outside the list stay untouched (NaN)."""
    import torch
    import paper_1911_05633_amd as g
    print(f"[pairs si24] {prec}", flush=True)
    spec = sc.serving_cell("si24", 16, 3)
    hop, b, Gk, C = cells.inputs(spec)
    GR_h = oracle.k_to_r(Gk, spec.mesh)
    cell = g.Cell.from_spec(spec, C)
    mt = [[60, 16]]
    n = cell.set_pairs(spec.lattice, spec.positions, 2.5, 4.6, mt)
    plan = oracle.plan_pairs(spec.lattice, spec.positions, spec.species, spec.n_pb, spec.mesh, 2.5, 4.6, mt)
    assert n == len(plan) and {tuple(r) for r in cell.pairs().tolist()} == {tuple(int(x) for x in r) for r in
                                                                          plan.tolist()}
    cdt = torch.complex128 if prec == "fp64" else torch.complex64
    GR = torch.from_numpy(np.ascontiguousarray(GR_h)).cuda().to(cdt)
    WR_h = sc.w_tensor(spec)
    WR = torch.from_numpy(np.ascontiguousarray(WR_h)).cuda().to(cdt)
    P = torch.full((spec.n_tau, spec.N_R, spec.N_pb, spec.N_pb), float("nan"), dtype=cdt, device="cuda")
    S = torch.full((spec.n_tau, spec.N_R, spec.N_orb, spec.N_orb), float("nan"), dtype=torch.complex128,
                   device="cuda")
    g.gw_polarizability_pairs(cell, GR, P, spec.spin, prec=prec)
    g.gw_self_energy_pairs(cell, GR, WR, S, prec=prec)
    torch.cuda.synchronize()
    rng = np.random.default_rng(24)
    po, oo = np.asarray(spec.pb_off), np.asarray(spec.orb_off)
    tiers = [plan[plan[:, 3] == m] for m in (60, 16)]
    pick = np.concatenate([t[rng.choice(len(t), 12, replace=False)] for t in tiers])
    kept = {(int(r[0]), int(r[1]), int(r[2])) for r in plan}
    cmpP, cmpS = [], []
    for t in (0, 7, spec.n_tau - 1):
        Pt, St = P[t].cpu().numpy(), S[t].cpu().numpy()
        for R, A, B, mA, mB in pick.tolist():
            cmpP.append((Pt[R, po[A]:po[A + 1], po[B]:po[B + 1]].astype(np.complex128),
                         oracle.polarizability_r_block_cut(GR_h, spec, C, spec.spin, t, R, A, B, mA, mB)))
            Wb = WR_h[t, R, po[A]:po[A + 1], po[B]:po[B + 1]]
            if prec != "fp64":
                Wb = Wb.astype(np.complex64).astype(np.complex128)
            cmpS.append((St[R, oo[A]:oo[A + 1], oo[B]:oo[B + 1]],
                         oracle.self_energy_r_block_cut(GR_h, Wb, spec, C, t, R, A, B, mA, mB)))
        outside = 0
        while outside < 20:
            R, A, B = int(rng.integers(spec.N_R)), int(rng.integers(spec.n_atoms)), int(rng.integers(spec.n_atoms))
            if (R, A, B) in kept:
                continue
            outside += 1
            assert np.all(np.isnan(Pt[R, po[A]:po[A + 1], po[B]:po[B + 1]]))
            assert np.all(np.isnan(St[R, oo[A]:oo[A + 1], oo[B]:oo[B + 1]]))
    eP = max(float(np.max(np.abs(a - b))) for a, b in cmpP) / max(float(np.max(np.abs(b))) for _, b in cmpP)
    eS = max(float(np.max(np.abs(a - b))) for a, b in cmpS) / max(float(np.max(np.abs(b))) for _, b in cmpS)
    tol = {"fp64": 1e-12, "bf16x3": 1e-5}[prec]
    print(f"[pairs si24] {prec}: {n} blocks, P {eP:.2e}, Sigma {eS:.2e}", flush=True)
    assert eP <= tol and eS <= tol
