"""GPU parity of the static (exchange) self-energy against the oracle.

gw_exchange must equal oracle.exchange_r (Eq. (8) with W~ -> V and G(tau) -> -G(beta)) for every R:
1e-12 relative in FP64 (tiny and two-species cells, the 8-atom Si cell), 2e-6 with complex64
storage and FP32 products, 1e-5 with the BF16 split products (8-atom cell).  Only the last time
slice of G may be read: the other slices are NaN in the FP64 runs.
"""
import numpy as np
import pytest

import oracle
import synthcell as sc
from tests import cells

pytestmark = pytest.mark.gpu

CASES = {"tiny": lambda: cells.tiny(complex_hopping=True), "two_species": lambda: cells.two_species(),
         "si8": lambda: sc.config(2), "oxide56": lambda: sc.config(4)}


def _vr(spec):
    A = sc.w_amplitude(spec)
    sR, _ = sc.w_factors(spec)
    return np.ascontiguousarray((sR[:, None, None] * A[None]).astype(np.complex128))


@pytest.mark.parametrize("name,prec", [("tiny", "fp64"), ("two_species", "fp64"), ("si8", "fp64"),
                                       ("si8", "fp32"), ("si8", "bf16x3"), ("oxide56", "fp64"),
                                       ("oxide56", "bf16x3")])
def test_exchange_matches_oracle(name, prec):
    import torch
    import paper_1911_05633_amd as g
    print(f"[exchange] {name} {prec}", flush=True)
    spec = CASES[name]()
    hop, b, Gk, C = cells.inputs(spec)
    GR = np.ascontiguousarray(oracle.k_to_r(Gk, spec.mesh))
    VR = _vr(spec)
    cell = g.Cell.from_spec(spec, C)
    cdt = torch.complex128 if prec == "fp64" else torch.complex64
    GRd = torch.from_numpy(GR).to(cdt).cuda()
    if prec == "fp64":
        GRd[:-1] = float("nan")
    VRd = torch.from_numpy(VR).to(cdt).cuda()
    Sx = torch.empty((spec.N_R, spec.N_orb, spec.N_orb), dtype=torch.complex128, device="cuda")
    g.gw_exchange(cell, GRd, VRd, Sx, prec=prec)
    torch.cuda.synchronize()
    if prec == "fp64":
        ref = oracle.exchange_r(GR, VR, spec, C)
        tol = 1e-12
    else:
        ref = oracle.exchange_r(GR.astype(np.complex64).astype(np.complex128),
                                VR.astype(np.complex64).astype(np.complex128), spec, C)
        tol = 2e-6 if prec == "fp32" else 1e-5
    got = Sx.cpu().numpy()
    err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    assert err < tol, err
