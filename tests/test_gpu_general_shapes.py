"""GPU parity of the general-shape matrix-core kernels (species of up to 16 orbitals and 128
product functions) against the FP64 oracle: the pairs outside the compact 9-orbital / 64-function
tiles, as in the layered oxide cell (16 / 100 beside 9 / 60), plus ragged shapes (11 / 77 and
13 / 90, 5 / 23) so that no size is a multiple of the 16-wide tiles.  Every block of every tau
and R is compared; FP64 at 1e-12, FP32 (and the BF16-split request, which runs the FP32
kernels on these shapes) at 2e-6 normwise.  The plain vector-ALU kernels run the same cells as
an on-device cross-check.
"""
import numpy as np
import pytest

import oracle
import synthcell as sc
from tests import cells

pytestmark = pytest.mark.gpu


def relmax(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def _cell(name):
    lat = np.array([[4.2, 0.0, 0.0], [0.3, 4.0, 0.0], [0.0, 0.2, 4.4]])
    if name == "oxide_like":  # heavy 16 / 100 and light 9 / 60 species
        pos = np.array([[0.0, 0.0, 0.0], [2.0, 2.1, 0.3], [0.4, 2.2, 2.0]])
        return sc.CellSpec(name, lat, pos, np.array([0, 1, 1]), (16, 9), (100, 60), (2, 1, 1), 6, 30.0,
                           config_id=31, request_id=1, complex_hopping=True)
    if name == "ragged":  # 11 / 77, 13 / 90 and 5 / 23
        pos = np.array([[0.0, 0.0, 0.0], [2.1, 1.9, 0.2], [0.3, 2.0, 2.2]])
        return sc.CellSpec(name, lat, pos, np.array([0, 1, 2]), (11, 13, 5), (77, 90, 23), (2, 2, 1), 5, 25.0,
                           config_id=32, request_id=2, complex_hopping=True)
    raise KeyError(name)


_cache = {}


def _case(name):
    if name not in _cache:
        spec = _cell(name)
        hop, b, Gk, C = cells.inputs(spec)
        GR = oracle.k_to_r(Gk, spec.mesh)
        WR = sc.w_tensor(spec)
        _cache[name] = dict(spec=spec, C=C, GR=GR, WR=WR, PR=oracle.polarizability_r(GR, spec, C, spec.spin),
                            SR=oracle.self_energy_r(GR, WR, spec, C))
    return _cache[name]


def _run(d, prec):
    import torch
    import paper_1911_05633_amd as g
    spec = d["spec"]
    cell = g.Cell.from_spec(spec, d["C"])
    cdt = torch.complex128 if prec == "fp64" else torch.complex64
    GR = torch.from_numpy(np.ascontiguousarray(d["GR"])).cuda().to(cdt)
    WR = torch.from_numpy(np.ascontiguousarray(d["WR"])).cuda().to(cdt)
    P = torch.full((spec.n_tau, spec.N_R, spec.N_pb, spec.N_pb), float("nan"), dtype=cdt, device="cuda")
    S = torch.full((spec.n_tau, spec.N_R, spec.N_orb, spec.N_orb), float("nan"), dtype=torch.complex128,
                   device="cuda")
    g.gw_polarizability(cell, GR, P, spec.spin, prec=prec)
    g.gw_self_energy(cell, GR, WR, S, prec=prec)
    torch.cuda.synchronize()
    return P.cpu().numpy().astype(np.complex128), S.cpu().numpy()


@pytest.mark.parametrize("name", ["oxide_like", "ragged"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_general_shapes_match_oracle(name, prec):
    print(f"[general shapes] {name} {prec}", flush=True)
    d = _case(name)
    P, S = _run(d, prec)
    assert np.all(np.isfinite(P)) and np.all(np.isfinite(S))
    SR = d["SR"]
    if prec != "fp64":
        spec = d["spec"]
        SR = oracle.self_energy_r(d["GR"], d["WR"].astype(np.complex64).astype(np.complex128), spec, d["C"])
    eP, eS = relmax(P, d["PR"]), relmax(S, SR)
    tol = 1e-12 if prec == "fp64" else 2e-6
    print(f"[general shapes] {name} {prec}: P {eP:.2e}, Sigma {eS:.2e}", flush=True)
    assert eP < tol and eS < tol


def test_general_shapes_match_plain_kernels(monkeypatch):
    print("[general shapes] matrix-core vs plain kernels", flush=True)
    d = _case("ragged")
    out = {}
    for mode in ("mfma", "generic"):
        if mode == "generic":
            monkeypatch.setenv("GWR_KERNELS", "generic")
        else:
            monkeypatch.delenv("GWR_KERNELS", raising=False)
        out[mode] = _run(d, "fp64")
    assert relmax(out["mfma"][0], out["generic"][0]) < 1e-13
    assert relmax(out["mfma"][1], out["generic"][1]) < 1e-13
