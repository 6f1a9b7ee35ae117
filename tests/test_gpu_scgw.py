"""The self-consistent GW loop on the GPU (Sec. 2, Eqs. (1)-(4)) against the oracle, cycle by cycle.

Starting from the band G(k, tau), four cycles run on the device (paper_1911_05633_amd.scgw:
P, W~, Sigma_c, Sigma_x, the mu search with the Dyson solve, G(k, tau) back from the Matsubara
frequencies with its tails in closed form, mixed half and half with the previous iterate).  Each
cycle is compared with the oracle's cycle from the same input G(k, tau) at the mu the GPU found
(1e-9 normwise), that mu is checked to hold the target count by the oracle's own count, the new
G(k, tau) must hold it at beta^- (the count the next cycle starts from), and the change between
iterates must shrink.  An independent oracle run of the same four cycles (its own bisection for
mu) ends at the same mu and G(k, tau).  The bare interaction is a weak synthetic one (0.01 of a
random positive definite matrix), so that the self-energy stays causal.
"""
import numpy as np
import pytest

import oracle
import synthcell as sc
from oracle.green import density_omega
from tests import cells

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


CASES = {"tiny": lambda: cells.tiny(complex_hopping=True), "two_species": lambda: cells.two_species()}


@pytest.mark.parametrize("name", list(CASES))
def test_scgw_cycles_match_the_oracle(name):
    import torch
    import paper_1911_05633_amd as g
    from paper_1911_05633_amd.scgw import SCGW
    spec = CASES[name]()
    hop, b, Gk, C = cells.inputs(spec)
    Hk = sc.hamiltonian_k(spec, hop)
    V = 0.01 * sc.dyson_inputs(spec.N_R, spec.N_pb, 1, 9)[0]
    taus = sc.tau_grid(spec)
    target = spec.spin * spec.N_orb / 2.0
    cell = g.Cell.from_spec(spec, C)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    Gd = dev(Gk)
    loop = SCGW(cell, dev(Hk), dev(V), Gd, spec.spin, target, mix=0.5)
    G_prev, mu, steps = Gk.copy(), b.mu, []
    for c in range(4):
        print(f"[scgw] {name} cycle {c}", flush=True)
        mu_g, n_w, n_beta, info = loop.cycle(mu - 1.0, mu + 1.0)
        assert info == 0
        G_gpu = Gd.cpu().numpy()
        Gn, _, parts = oracle.scgw.cycle(G_prev, spec, C, Hk, V, taus, target, mu=mu_g)
        e = _rel(G_gpu, 0.5 * Gn + 0.5 * G_prev)
        n_or = density_omega(parts["G_w"], Hk, mu_g, spec.beta, spec.spin, parts["Sigma_x"])
        step = float(np.max(np.abs(G_gpu - G_prev)))
        print(f"[scgw] {name} cycle {c}: mu {mu_g:.10f}, count {n_w:.10f} (oracle {n_or:.10f}), "
              f"beta- {n_beta:.10f}, vs oracle {e:.2e}, step {step:.2e}", flush=True)
        assert e < 1e-9
        assert abs(n_w - target) <= 1e-9 and abs(n_or - target) < 1e-8 and abs(n_beta - target) < 1e-8
        steps.append(step)
        G_prev, mu = G_gpu, mu_g
    assert all(steps[i + 1] < steps[i] for i in range(len(steps) - 1))
    traj = oracle.scgw.run(Gk, spec, C, Hk, V, taus, target, b.mu, 4, mix=0.5)
    assert abs(traj[-1][1] - mu) < 1e-7 and _rel(G_prev, traj[-1][0]) < 1e-7
