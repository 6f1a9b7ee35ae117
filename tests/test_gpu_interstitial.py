"""GPU parity of the interstitial-grid blocks of P and Sigma (Eqs. (6), (7), (9), (10)).

gw_polarizability_int / gw_self_energy_int against the oracle (grid points as unit pseudo-atoms
on top of Eqs. (5), (8)): every block at every tau and R for the two-species cell with 37 grid
points (ragged LDS tiles), sampled (tau, R) for the 8-atom Si cell with 64 grid points.  Bars:
1e-12 relative for complex128 storage, 1e-6 for complex64 storage (FP64 arithmetic on the
stored values).
"""
import numpy as np
import pytest

import synthcell as sc
from oracle.interstitial import polarizability_int, self_energy_int
from tests import cells

pytestmark = pytest.mark.gpu


def _blocks(spec, n_g, seed, rows):
    sh = (spec.n_tau, spec.N_R)
    return [sc.random_complex(sh + (rows, n_g), seed), sc.random_complex(sh + (n_g, rows), seed + 1),
            sc.random_complex(sh + (n_g, n_g), seed + 2)]


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("name,n_g,dtype", [("two_species", 37, "c128"), ("two_species", 37, "c64"),
                                            ("two_species", 1, "c128"), ("two_species", 257, "c128"),
                                            ("si8", 64, "c128"), ("oxide56", 48, "c128")])
def test_interstitial_blocks_match_oracle(name, n_g, dtype):
    import torch
    import paper_1911_05633_amd as g
    print(f"[interstitial] {name} n_g={n_g} {dtype}", flush=True)
    spec = {"two_species": cells.two_species, "si8": lambda: sc.config(2), "oxide56": lambda: sc.config(4)}[name]()
    C = sc.coefficients(spec)
    cell = g.Cell.from_spec(spec, C)
    G = _blocks(spec, n_g, 100, spec.N_orb)
    W = _blocks(spec, n_g, 200, spec.N_pb)
    npdt = np.complex128 if dtype == "c128" else np.complex64
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    G = [a.astype(npdt).astype(np.complex128) for a in G]
    W = [a.astype(npdt).astype(np.complex128) for a in W]
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(tdt).cuda()
    Gd, Wd = [dev(a) for a in G], [dev(a) for a in W]
    bl = (spec.n_tau, spec.N_R)
    P = [torch.empty(bl + (spec.N_pb, n_g), dtype=tdt, device="cuda"),
         torch.empty(bl + (n_g, spec.N_pb), dtype=tdt, device="cuda"),
         torch.empty(bl + (n_g, n_g), dtype=tdt, device="cuda")]
    S = [torch.empty(bl + (spec.N_orb, n_g), dtype=torch.complex128, device="cuda"),
         torch.empty(bl + (n_g, spec.N_orb), dtype=torch.complex128, device="cuda"),
         torch.empty(bl + (n_g, n_g), dtype=torch.complex128, device="cuda")]
    g.gw_polarizability_int(cell, *Gd, *P, spec.spin)
    g.gw_self_energy_int(cell, *Gd, *Wd, *S)
    torch.cuda.synchronize()
    taus, Rs = (None, None) if name == "two_species" else ([0, 17, spec.n_tau - 1], [0, 1, spec.N_R - 1])
    Pref = polarizability_int(*G, spec, C, spec.spin, taus, Rs)
    Sref = self_energy_int(*G, *W, spec, C, taus, Rs)
    tol = 1e-12 if dtype == "c128" else 1e-6
    ti = slice(None) if taus is None else taus
    Ri = slice(None) if Rs is None else Rs
    for got, ref in zip(P + S, list(Pref) + list(Sref)):
        a = got.cpu().numpy().astype(np.complex128)
        a = a[ti][:, Ri] if taus is not None else a
        assert _rel(a, ref) < tol


def test_interstitial_argument_errors():
    import torch
    import paper_1911_05633_amd as g
    print("[interstitial] errors", flush=True)
    spec = cells.two_species()
    C = sc.coefficients(spec)
    cell = g.Cell.from_spec(spec, C)
    n_g = 8
    Gd = [torch.from_numpy(a).cuda() for a in _blocks(spec, n_g, 1, spec.N_orb)]
    bl = (spec.n_tau, spec.N_R)
    P = [torch.empty(bl + (spec.N_pb, n_g), dtype=torch.complex128, device="cuda"),
         torch.empty(bl + (n_g, spec.N_pb), dtype=torch.complex128, device="cuda"),
         torch.empty(bl + (n_g, n_g), dtype=torch.complex128, device="cuda")]
    with pytest.raises(g.GWError):          # output aliasing an input
        g.gw_polarizability_int(cell, Gd[0], Gd[1], Gd[2], P[0], P[1], Gd[2])
    with pytest.raises(TypeError):          # mixed storage types
        g.gw_polarizability_int(cell, Gd[0], Gd[1], Gd[2].to(torch.complex64), *P)
