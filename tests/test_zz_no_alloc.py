"""gw_green_dyson_noalloc (static device scratch, no allocation) against gw_green_dyson.

Two calls in a row on one GPU, the second on a smaller input, each compared with the entry point
that takes a caller workspace on the same inputs (bit-identical: the same kernels invert each
matrix independently) and with the oracle's Eq. (4) at 1e-10.  The first input (8-atom cell,
512 matrices of 72, padded to 128) needs three launches through the 64 MiB array, so the chunk
loop is exercised; the second (tiny cell) reuses the array with the first call's contents in it.
A cell whose one padded matrix exceeds the array is refused before any launch.
"""
import numpy as np
import pytest

import oracle
import synthcell as sc
from oracle.green import fermionic_points
from tests import cells

pytestmark = pytest.mark.gpu


def _sigma(spec, n_om, seed):
    """Causal one-pole Sigma(k, i w) = s X X^H / (i w - e) and a Hermitian static part."""
    rng = np.random.default_rng(seed)
    n = spec.N_orb
    X = rng.standard_normal((spec.N_R, n, n)) + 1j * rng.standard_normal((spec.N_R, n, n))
    XX = X @ np.conj(np.swapaxes(X, -1, -2)) / n
    om = fermionic_points(n_om, spec.beta)
    S = 0.2 * XX[None] / (1j * om[:, None, None, None] - 0.3)
    Y = rng.standard_normal((spec.N_R, n, n))
    return S, (0.1 * (Y + np.swapaxes(Y, -1, -2))).astype(np.complex128)


def _both(spec, n_om, seed):
    import torch
    import paper_1911_05633_amd as g
    hop, b, Gk, C = cells.inputs(spec)
    Hk = sc.hamiltonian_k(spec, hop)
    S, Sx = _sigma(spec, n_om, seed)
    cell = g.Cell.from_spec(spec, C)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    Hd, Sd, Sxd = dev(Hk), dev(S), dev(Sx)
    shape = (n_om, spec.N_R, spec.N_orb, spec.N_orb)
    G_ref = torch.empty(shape, dtype=torch.complex128, device="cuda")
    work = torch.empty(g.gw_green_dyson_workspace(cell, n_om * spec.N_R), dtype=torch.uint8, device="cuda")
    g.gw_green_dyson(cell, Hd, b.mu, G_ref, work, Sigma=Sd, Sigma_x=Sxd)
    G = torch.full(shape, float("nan"), dtype=torch.complex128, device="cuda")
    info = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    g.gw_green_dyson_noalloc(cell, Hd, b.mu, G, Sigma=Sd, Sigma_x=Sxd, info=info)
    torch.cuda.synchronize()
    ora = oracle.green_dyson(Hk, b.mu, fermionic_points(n_om, spec.beta), Sigma=S, Sigma_x=Sx)
    return G.cpu().numpy(), G_ref.cpu().numpy(), ora, int(info.item())


def test_noalloc_matches_workspace_entry_point_twice():
    import paper_1911_05633_amd as g
    runs = [("si8", sc.config(2), 8, 3), ("tiny", cells.tiny(complex_hopping=True), 3, 5)]
    per = [16 * (128 * 128 + 4096), 16 * (64 * 64 + 4096)]
    assert g.GREEN_NOALLOC_SCRATCH_BYTES // per[0] < 8 * 64  # the first call needs several launches
    for name, spec, n_om, seed in runs:
        print(f"[no-alloc] {name}: {n_om} frequencies x {spec.N_R} k of {spec.N_orb}", flush=True)
        G, G_ref, ora, info = _both(spec, n_om, seed)
        assert info == 0
        assert np.all(np.isfinite(G))
        assert np.array_equal(G, G_ref)
        assert np.max(np.abs(G - ora)) < 1e-10 * np.max(np.abs(ora))


def test_noalloc_refuses_a_cell_beyond_the_static_scratch():
    import torch
    import paper_1911_05633_amd as g
    print("[no-alloc] oversized cell is refused", flush=True)
    n_atoms = 128  # 128 atoms x 16 orbitals = 2048: one padded matrix needs 16 (2048^2 + 4096) > 64 MiB
    C = [np.ones((1, 16, 16))]
    cell = g.Cell([0] * n_atoms, [16], [1], C, (1, 1, 1), 2, 5.0, np.array([0.0, 5.0]))
    small = torch.zeros(4, dtype=torch.complex128, device="cuda")
    with pytest.raises(g.GWError, match="64 MiB"):
        g.lib.gw_green_dyson_noalloc  # noqa: B018 (exported)
        st = g.lib.gw_green_dyson_noalloc(cell.handle, small.data_ptr(), 0.0, 1, None, None, small.data_ptr(),
                                          None, None)
        g._check(st, "gw_green_dyson_noalloc")
    torch.cuda.synchronize()
