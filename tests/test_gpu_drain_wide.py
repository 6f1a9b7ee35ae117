"""GPU parity of the wide-chunk paired drain (complex64 in and out, parity +1 / -1).

The drain with the tau mirror folded in runs, for complex64 storage, meshes of 2, 4 and 8
points, n_tau <= 64 and n_omega <= 64, on a kernel that moves 256 columns (256 / N_R elements
of every row) per chunk and holds the paired, R -> k transformed y in complex64 in LDS.  Each
case runs it and the two-stream ping-pong kernel (selected by GWR_DRAIN=pingpong) on the same
input, in place as the step does, and checks both against the oracle's r_to_k followed by the
Filon tau -> Matsubara matrix of Eqs. (5) and (8) on the complex64 values the kernels read.
Shapes give several chunks per workgroup, a ragged last chunk, odd n_tau (the self-mirrored
middle row), n_omega below and above n_tau (one to four 16-row m tiles; at n_tau = n_omega = 64
the kernel's y and A fill LDS exactly).  Bar: 1e-6 of the
largest output (complex64 storage; rounding y to complex64 adds about 1e-7).
"""
import os

import numpy as np
import pytest

import oracle
import synthcell as sc

pytestmark = pytest.mark.gpu


def relmax(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def _spec(mesh, n_tau, n_orb, n_pb, n_atoms, beta=30.0, rid=0):
    lat = np.diag([4.1, 4.3, 4.5])
    pos = np.array([[0.0, 0.0, 0.0], [1.6, 1.9, 2.1], [3.0, 0.7, 1.2]])[:n_atoms]
    return sc.CellSpec(f"dwide_{rid}", lat, pos, np.zeros(n_atoms, dtype=np.int64), (n_orb,), (n_pb,), tuple(mesh),
                       n_tau, beta, config_id=40, request_id=rid)


# (mesh, n_tau, n_orb per atom, n_pb per atom, atoms): product-basis columns N_pb^2 per R and
# orbital columns N_orb^2 per R, both ragged against the chunk width 256 / N_R
CASES = {
    "m8_t32": ((2, 2, 2), 32, 5, 81, 2),
    "m4_t47": ((2, 2, 1), 47, 7, 100, 3),
    "m2_t48": ((2, 1, 1), 48, 6, 100, 2),
    "m2_t5": ((2, 1, 1), 5, 3, 29, 2),
    "m8_t64": ((2, 2, 2), 64, 4, 70, 2),
    "m4_t61": ((2, 2, 1), 61, 5, 90, 2),
}


def _run(g, cell, Td, F, basis, parity, pingpong):
    import torch
    x = torch.from_numpy(F).cuda()
    if pingpong:
        os.environ["GWR_DRAIN"] = "pingpong"
    try:
        n_tau = cell.n_tau
        g.gw_drain(cell, Td, x[:n_tau], x, basis=basis, parity=parity)  # in place: in is out's first n_tau rows
        torch.cuda.synchronize()
    finally:
        os.environ.pop("GWR_DRAIN", None)
    return x.cpu().numpy()


@pytest.mark.parametrize("name", list(CASES))
# n_omega: None = n_tau, -1 = min(2 n_tau, 64) (more frequencies than tau points: the output rows
# outrun the input rows in place)
@pytest.mark.parametrize("basis,parity,n_omega",
                         [(1, 1, None), (1, 1, 19), (1, 1, -1), (0, -1, None), (0, -1, 3), (0, -1, -1)])
def test_drain_wide(name, basis, parity, n_omega):
    import torch
    import paper_1911_05633_amd as g
    mesh, n_tau, n_orb, n_pb, n_atoms = CASES[name]
    spec = _spec(mesh, n_tau, n_orb, n_pb, n_atoms, rid=len(name) + basis)
    print(f"[drain wide] {name} basis {basis} parity {parity} n_omega {n_omega}", flush=True)
    cell = g.Cell.from_spec(spec, sc.coefficients(spec))
    n = spec.N_orb if basis == 0 else spec.N_pb
    kind = "fermionic" if basis == 0 else "bosonic"
    tau = sc.tau_grid(spec)
    n_w = n_tau if n_omega is None else (min(2 * n_tau, 64) if n_omega < 0 else min(n_omega, n_tau))
    w = g.matsubara(n_w, spec.beta, kind)
    freqs = (oracle.fermionic_frequencies(n_w, spec.beta) if kind == "fermionic"
             else oracle.bosonic_frequencies(n_w, spec.beta))
    Td = torch.from_numpy(np.ascontiguousarray(g.gw_tau2omega_matrix(tau, w))).cuda()
    rows = max(n_tau, len(w))
    F = np.zeros((rows, spec.N_R, n, n), dtype=np.complex64)
    F[:n_tau] = sc.random_complex((n_tau, spec.N_R, n, n), seed=71 + basis)
    ref = oracle.apply_tau_to_omega(oracle.filon_matrix(tau, freqs),
                                    oracle.r_to_k(F[:n_tau].astype(np.complex128), spec.mesh))
    wd = _run(g, cell, Td, F, basis, parity, False)[:len(w)].astype(np.complex128)
    pp = _run(g, cell, Td, F, basis, parity, True)[:len(w)].astype(np.complex128)
    e_w, e_pp, e_x = relmax(wd, ref), relmax(pp, ref), relmax(wd, pp)
    print(f"    wide {e_w:.2e}  pingpong {e_pp:.2e}  wide vs pingpong {e_x:.2e}", flush=True)
    assert np.all(np.isfinite(wd))
    assert e_w < 1e-6 and e_pp < 1e-6 and e_x < 1e-6
