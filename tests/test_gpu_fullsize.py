"""Parity at the full workload sizes, in the launch configuration the benchmark times.

The 72-atom Si-like cell (the benchmark workload) and the 56-atom two-species oxide-like
cell run through the whole path (k -> R, P, Sigma, drains of both, electron count) on
the mixed and the plain FP64 paths.  The oracle cannot evaluate whole tensors of this
size in seconds, so it is checked on sampled outputs it computes one by one: atom-pair
blocks of P^R(tau) (Eq. (5)) and Sigma^R(tau) (Eq. (8)) at several (tau, R), and every
(Matsubara frequency, q) of the drained P and Sigma for one atom pair, built from the
oracle's blocks at all (tau, R).  Bars (normwise over the sample): 1e-5 mixed, 1e-10 FP64.
"""
import gc

import numpy as np
import pytest

import oracle
import synthcell as sc

pytestmark = pytest.mark.gpu


def _inputs(spec):
    hop = sc.hoppings(spec)
    b = sc.bands(spec, hop)
    Gk = sc.green_ktau(spec, b)
    C = sc.coefficients(spec)
    A = sc.w_amplitude(spec)
    sR, et = sc.w_factors(spec)
    return Gk, C, A, sR, et


def _sample_pairs(spec):
    na = spec.n_atoms
    sp = np.asarray(spec.species)
    pairs = [(0, 0), (0, na - 1), (na // 2, 5 % na), (na - 1, na - 1)]
    # one pair for every species pair present
    for s1 in range(spec.n_species):
        for s2 in range(spec.n_species):
            a = int(np.flatnonzero(sp == s1)[-1])
            b = int(np.flatnonzero(sp == s2)[0])
            pairs.append((a, b))
    return sorted(set(pairs))


def _err(pairs_of_arrays):
    num = max(float(np.max(np.abs(g - o))) for g, o in pairs_of_arrays)
    den = max(float(np.max(np.abs(o))) for _, o in pairs_of_arrays)
    return num / den


@pytest.mark.parametrize("cfg,prec", [(3, "fp32"), (3, "bf16x3"), (3, "fp64"), (4, "fp32"), (4, "fp64")])
def test_full_size_path_sampled(cfg, prec):
    import torch
    import paper_1911_05633_amd as g
    spec = sc.config(cfg)
    print(f"[full size] config {cfg} ({spec.name}) {prec}", flush=True)
    Gk_h, C, A, sR, et = _inputs(spec)
    nt, NR, No, Np = spec.n_tau, spec.N_R, spec.N_orb, spec.N_pb
    cdt = torch.complex128 if prec == "fp64" else torch.complex64  # bf16x3 stores complex64 too
    cell = g.Cell.from_spec(spec, C)
    Gk = torch.from_numpy(Gk_h).cuda()
    GR = torch.empty(Gk.shape, dtype=cdt, device="cuda")
    Ad = torch.from_numpy(A).cuda()
    W = torch.empty((nt, NR, Np, Np), dtype=cdt, device="cuda")
    for t in range(nt):
        for R in range(NR):
            W[t, R].copy_(Ad * float(sR[R] * et[t]))
    del Ad
    P = torch.empty((nt, NR, Np, Np), dtype=cdt, device="cuda")
    S = torch.empty((nt, NR, No, No), dtype=torch.complex128, device="cuda")
    n = torch.zeros(1, dtype=torch.float64, device="cuda")
    tau = sc.tau_grid(spec)
    nu = g.matsubara(nt, spec.beta, "bosonic")
    wf = g.matsubara(nt, spec.beta, "fermionic")
    TP, TS = torch.from_numpy(g.gw_tau2omega_matrix(tau, nu)).cuda(), torch.from_numpy(g.gw_tau2omega_matrix(tau, wf)).cuda()

    g.gw_fourier_k2r(cell, Gk, GR, basis=0)
    g.gw_polarizability(cell, GR, P, spec.spin, prec=prec)
    g.gw_self_energy(cell, GR, W, S, prec=prec)
    torch.cuda.synchronize()

    GR_o = oracle.k_to_r(Gk_h, spec.mesh)
    po, oo = np.asarray(spec.pb_off), np.asarray(spec.orb_off)
    pairs = _sample_pairs(spec)
    tRs = [(0, 0), (1, min(3, NR - 1)), (nt // 2, NR - 1), (nt - 1, NR // 2)]
    cmpP, cmpS = [], []
    for (Aa, Bb) in pairs:
        for (t, R) in tRs:
            pg = P[t, R, po[Aa]:po[Aa + 1], po[Bb]:po[Bb + 1]].cpu().numpy().astype(np.complex128)
            cmpP.append((pg, oracle.polarizability_r_block(GR_o, spec, C, spec.spin, t, R, Aa, Bb)))
            Wb = (et[t] * sR[R] * A[po[Aa]:po[Aa + 1], po[Bb]:po[Bb + 1]]).astype(np.complex128)
            sg = S[t, R, oo[Aa]:oo[Aa + 1], oo[Bb]:oo[Bb + 1]].cpu().numpy()
            cmpS.append((sg, oracle.self_energy_r_block(GR_o, Wb, spec, C, t, R, Aa, Bb)))
    eP, eS = _err(cmpP), _err(cmpS)

    # drains, then every (omega, q) of one atom pair against the oracle built from its blocks
    g.gw_drain(cell, TP, P, P, basis=1, parity=1)
    g.gw_drain(cell, TS, S, S, basis=0, parity=-1)
    if prec == "fp64":
        g.gw_density(cell, GR, spec.spin, n, space=0)
    else:
        g.gw_density(cell, Gk, spec.spin, n, space=1)
    torch.cuda.synchronize()
    Aa, Bb = pairs[len(pairs) // 2]
    Pblk = np.zeros((nt, NR, po[Aa + 1] - po[Aa], po[Bb + 1] - po[Bb]), dtype=np.complex128)
    Sblk = np.zeros((nt, NR, oo[Aa + 1] - oo[Aa], oo[Bb + 1] - oo[Bb]), dtype=np.complex128)
    for t in range(nt):
        for R in range(NR):
            Pblk[t, R] = oracle.polarizability_r_block(GR_o, spec, C, spec.spin, t, R, Aa, Bb)
            Wb = (et[t] * sR[R] * A[po[Aa]:po[Aa + 1], po[Bb]:po[Bb + 1]]).astype(np.complex128)
            Sblk[t, R] = oracle.self_energy_r_block(GR_o, Wb, spec, C, t, R, Aa, Bb)
    Pw = oracle.apply_tau_to_omega(oracle.filon_matrix(tau, oracle.bosonic_frequencies(nt, spec.beta)),
                                   oracle.r_to_k(Pblk, spec.mesh))
    Sw = oracle.apply_tau_to_omega(oracle.filon_matrix(tau, oracle.fermionic_frequencies(nt, spec.beta)),
                                   oracle.r_to_k(Sblk, spec.mesh))
    Pg = P[:, :, po[Aa]:po[Aa + 1], po[Bb]:po[Bb + 1]].cpu().numpy().astype(np.complex128)
    Sg = S[:, :, oo[Aa]:oo[Aa + 1], oo[Bb]:oo[Bb + 1]].cpu().numpy()
    ePw, eSw = _err([(Pg, Pw)]), _err([(Sg, Sw)])
    n_ref = oracle.electron_count(GR_o[-1, 0], spec.spin)
    en = abs(float(n.cpu()[0]) - n_ref) / n_ref
    print(f"[full size] config {cfg} {prec}: P(tau) {eP:.2e}, Sigma(tau) {eS:.2e}, P(q, i nu) {ePw:.2e}, "
          f"Sigma(k, i w) {eSw:.2e}, electron count {en:.1e} ({len(cmpP)} sampled blocks each)", flush=True)
    tol = 1e-10 if prec == "fp64" else 1e-5
    del P, S, W, GR, Gk
    gc.collect()
    torch.cuda.empty_cache()
    assert eP <= tol and eS <= tol and ePw <= tol and eSw <= tol
    assert en <= 1e-12
