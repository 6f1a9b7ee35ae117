"""CPU-only checks of the C ABI: the library loads, exports every declared
symbol, validates arguments before touching a device, and its host-side
Matsubara matrix agrees with the oracle's (independent) construction."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "gwr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gw_[A-Za-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_1911_05633_amd as g
    names = declared_symbols()
    assert len(names) >= 14
    raw = ctypes.CDLL(g.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), n
    assert set(names) == set(g.SIGNATURES)


def test_validation_without_device():
    import paper_1911_05633_amd as g
    lib = g.lib
    assert lib.gw_polarizability(None, None, None, 2.0, 0, None) == g.GW_ERR_ARG
    assert lib.gw_self_energy(None, None, None, None, 0, None) == g.GW_ERR_ARG
    assert lib.gw_fourier_k2r(None, None, 0, None, 0, 0, None) == g.GW_ERR_ARG
    assert lib.gw_drain(None, None, 48, 0, None, 0, None, 0, 1, None) == g.GW_ERR_ARG
    assert lib.gw_tau2omega(None, None, 48, 1, None, 0, None, 0, 1, None) == g.GW_ERR_ARG
    assert lib.gw_density(None, None, 0, 0, 2.0, None, None) == g.GW_ERR_ARG
    h = ctypes.c_void_p()
    sp = np.zeros(2, dtype=np.int32)
    no = np.array([4], dtype=np.int32)
    npb = np.array([16], dtype=np.int32)
    mesh = np.array([2, 2, 2], dtype=np.int32)
    C = np.zeros(16 * 16, dtype=np.float64)
    tau8 = 10.0 * np.arange(8) / 7
    ip = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    # n_tau out of range, mesh entry 0, orbital count above the limit, bad species index
    assert lib.gw_cell_create(ctypes.byref(h), 2, ip(sp), 1, ip(no), ip(npb), dp(C), ip(mesh), 1, 10.0, dp(tau8)) == g.GW_ERR_SHAPE
    bad_mesh = np.array([2, 0, 2], dtype=np.int32)
    assert lib.gw_cell_create(ctypes.byref(h), 2, ip(sp), 1, ip(no), ip(npb), dp(C), ip(bad_mesh), 8, 10.0, dp(tau8)) == g.GW_ERR_SHAPE
    big = np.array([17], dtype=np.int32)
    assert lib.gw_cell_create(ctypes.byref(h), 2, ip(sp), 1, ip(big), ip(npb), dp(C), ip(mesh), 8, 10.0, dp(tau8)) == g.GW_ERR_SHAPE
    sp_bad = np.array([0, 3], dtype=np.int32)
    assert lib.gw_cell_create(ctypes.byref(h), 2, ip(sp_bad), 1, ip(no), ip(npb), dp(C), ip(mesh), 8, 10.0, dp(tau8)) == g.GW_ERR_ARG
    assert lib.gw_cell_create(ctypes.byref(h), 2, ip(sp), 1, ip(no), ip(npb), dp(C), ip(mesh), 8, -1.0, dp(tau8)) == g.GW_ERR_ARG
    assert b"beta" in lib.gw_last_error()


@pytest.mark.parametrize("kind", ["bosonic", "fermionic"])
def test_host_matsubara_matrix_matches_oracle(kind):
    import paper_1911_05633_amd as g
    beta, n = 200.0, 48
    tau = beta * np.arange(n) / (n - 1)
    w = g.matsubara(n, beta, kind)
    ref_w = oracle.bosonic_frequencies(n, beta) if kind == "bosonic" else oracle.fermionic_frequencies(n, beta)
    assert np.array_equal(w, ref_w)
    T = g.gw_tau2omega_matrix(tau, w)
    To = oracle.filon_matrix(tau, ref_w)
    assert np.max(np.abs(T - To)) / np.max(np.abs(To)) < 1e-12


def test_host_matsubara_matrix_nonuniform_grid():
    import paper_1911_05633_amd as g
    beta, n = 50.0, 33
    tau = 0.5 * beta * (1 - np.cos(np.pi * np.arange(n) / (n - 1)))
    w = oracle.fermionic_frequencies(20, beta)
    T = g.gw_tau2omega_matrix(tau, w)
    To = oracle.filon_matrix(tau, w)
    assert np.max(np.abs(T - To)) / np.max(np.abs(To)) < 1e-11
    with pytest.raises(g.GWError):
        g.gw_tau2omega_matrix(tau[::-1].copy(), w)


@pytest.mark.parametrize("kind,parity", [("bosonic", 1), ("fermionic", -1)])
@pytest.mark.parametrize("n", [48, 7, 2])
def test_host_matsubara_matrix_has_the_declared_mirror_parity(kind, parity, n):
    """T[m][n-1-i] = parity * conj(T[m][i]) on a grid symmetric about beta / 2 (the
    precondition of the two-GEMM drain), uniform and clustered grids alike."""
    import paper_1911_05633_amd as g
    beta = 100.0
    for tau in (beta * np.arange(n) / (n - 1), 0.5 * beta * (1 - np.cos(np.pi * np.arange(n) / (n - 1)))):
        T = g.gw_tau2omega_matrix(tau, g.matsubara(n + 3, beta, kind))
        mirror = parity * np.conj(T[:, ::-1])
        assert np.max(np.abs(T - mirror)) <= 1e-13 * np.max(np.abs(T))


def test_next_row_entry_points_reject_a_null_cell_without_device():
    import paper_1911_05633_amd as g
    lib = g.lib
    sz = ctypes.c_size_t()
    mu, n = ctypes.c_double(), ctypes.c_double()
    assert lib.gw_screened_interaction_workspace(None, 1, 0, ctypes.byref(sz)) == g.GW_ERR_ARG
    assert lib.gw_green_dyson_workspace(None, 1, ctypes.byref(sz)) == g.GW_ERR_ARG
    assert lib.gw_screened_interaction(None, None, None, 0, None, 0, 4, 0, None, 0, None, None) == g.GW_ERR_ARG
    assert lib.gw_green_dyson(None, None, 0.0, 4, None, None, None, None, 0, None, None) == g.GW_ERR_ARG
    assert lib.gw_density_omega(None, None, 4, None, None, 0.0, 2.0, None, None) == g.GW_ERR_ARG
    assert lib.gw_update_mu(None, None, None, None, 4, 2.0, 8.0, -1.0, 1.0, 1e-9, 10, None, None, 0, None,
                            ctypes.byref(mu), ctypes.byref(n), None) == g.GW_ERR_ARG
    assert lib.gw_exchange(None, None, None, None, 0, None) == g.GW_ERR_ARG
    assert lib.gw_polarizability_int(None, 8, None, None, None, None, None, None, 2.0, 0, None) == g.GW_ERR_ARG
    assert lib.gw_self_energy_int(None, 8, None, None, None, None, None, None, None, None, None, 0, None) == g.GW_ERR_ARG
    assert b"NULL" in lib.gw_last_error() or b"cell" in lib.gw_last_error()


def _create_args():
    import paper_1911_05633_amd as g
    sp = np.zeros(2, dtype=np.int32)
    no = np.array([4], dtype=np.int32)
    npb = np.array([16], dtype=np.int32)
    mesh = np.array([2, 2, 2], dtype=np.int32)
    C = np.zeros(16 * 16, dtype=np.float64)
    ip = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return g, (ip(sp), ip(no), ip(npb), dp(C), ip(mesh)), dp, (sp, no, npb, C, mesh)


@pytest.mark.parametrize("what", ["null", "start", "end", "order", "asymmetric", "nan"])
def test_cell_create_refuses_a_bad_tau_grid_before_any_device_call(what):
    """The tau grid must run from 0 to beta, increase and be symmetric about beta / 2: the
    polarizability's mirror and the drains' parity pairing read index n-1-i as beta - tau_i."""
    g, a, dp, keep = _create_args()
    beta, n = 10.0, 8
    tau = beta * np.arange(n) / (n - 1)
    if what == "start":
        tau[0] = 0.01
    elif what == "end":
        tau[-1] = beta - 0.01
    elif what == "order":
        tau[3], tau[4] = tau[4], tau[3]
    elif what == "asymmetric":
        tau[2] += 0.05  # increasing still, but no longer mirrored by tau[5]
    elif what == "nan":
        tau[2] = np.nan
    h = ctypes.c_void_p()
    ptr = None if what == "null" else dp(tau)
    assert g.lib.gw_cell_create(ctypes.byref(h), 2, a[0], 1, a[1], a[2], a[3], a[4], n, beta, ptr) == g.GW_ERR_ARG
    assert b"tau" in g.lib.gw_last_error()
    assert not h.value


@pytest.mark.parametrize("n", [2, 3, 48])
def test_cell_create_grid_checks_pass_symmetric_grids(n):
    """Uniform and clustered symmetric grids pass the tau checks: with them the call gets past the
    validation and fails only where it first needs a device (no GPU here), or succeeds on one."""
    g, a, dp, keep = _create_args()
    beta = 37.0
    for tau in (beta * np.arange(n) / (n - 1), 0.5 * beta * (1 - np.cos(np.pi * np.arange(n) / (n - 1)))):
        h = ctypes.c_void_p()
        st = g.lib.gw_cell_create(ctypes.byref(h), 2, a[0], 1, a[1], a[2], a[3], a[4], n, beta, dp(tau))
        assert st in (g.GW_OK, g.GW_ERR_HIP), g.lib.gw_last_error()
        if st == g.GW_OK:
            g.lib.gw_cell_destroy(h)
        else:
            assert b"tau" not in g.lib.gw_last_error()


def test_workspace_bytes_is_zero_for_the_path():
    """The path's calls keep their temporaries on chip: no scratch for any precision."""
    import paper_1911_05633_amd as g
    for p in (g.GW_FP64, g.GW_FP32, g.GW_BF16X3):
        assert g.lib.gw_workspace_bytes(None, p) == 0
    assert g.lib.gw_cell_tau(None, None) == g.GW_ERR_ARG
