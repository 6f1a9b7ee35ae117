"""Python binding of libgwr (space-time P / Sigma on MI355X).

Argument marshalling only: every call checks the tensors (device, dtype,
contiguity, element count against the cell), passes raw device pointers and
the current HIP stream to the C ABI declared in include/gwr.h, and turns a
non-zero status into GWError.  All arithmetic runs in the library's kernels.
If libgwr.so is missing the import of this module fails: there is no other
code path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgwr.so")

GW_OK, GW_ERR_ARG, GW_ERR_SHAPE, GW_ERR_NOMEM, GW_ERR_HIP, GW_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5
GW_FP64, GW_FP32, GW_BF16X3 = 0, 1, 2
GW_C128, GW_C64 = 0, 1
PRECISIONS = {"fp64": GW_FP64, "fp32": GW_FP32, "bf16x3": GW_BF16X3}

# every function the header declares, with its ctypes signature
_c_int, _c_double, _vp = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
_ip, _dp = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "gw_cell_create": (_c_int, [ctypes.POINTER(_vp), _c_int, _ip, _c_int, _ip, _ip, _dp, _ip, _c_int, _c_double,
                                _dp]),
    "gw_cell_tau": (_c_int, [_vp, _dp]),
    "gw_workspace_bytes": (ctypes.c_size_t, [_vp, _c_int]),
    "gw_cell_destroy": (None, [_vp]),
    "gw_cell_n_orb_total": (_c_int, [_vp]),
    "gw_cell_n_pb_total": (_c_int, [_vp]),
    "gw_cell_n_R": (_c_int, [_vp]),
    "gw_fourier_k2r": (_c_int, [_vp, _vp, _c_int, _vp, _c_int, _c_int, _vp]),
    "gw_fourier_r2k": (_c_int, [_vp, _vp, _c_int, _vp, _c_int, _c_int, _vp]),
    "gw_polarizability": (_c_int, [_vp, _vp, _vp, _c_double, _c_int, _vp]),
    "gw_self_energy": (_c_int, [_vp, _vp, _vp, _vp, _c_int, _vp]),
    "gw_tau2omega": (_c_int, [_vp, _vp, _c_int, _c_int, _vp, _c_int, _vp, _c_int, _c_int, _vp]),
    "gw_drain": (_c_int, [_vp, _vp, _c_int, _c_int, _vp, _c_int, _vp, _c_int, _c_int, _vp]),
    "gw_density": (_c_int, [_vp, _vp, _c_int, _c_int, _c_double, _vp, _vp]),
    "gw_tau2omega_matrix": (_c_int, [_c_int, _dp, _c_int, _dp, _dp]),
    "gw_cell_set_pairs": (_c_int, [_vp, _dp, _dp, _c_double, _c_double, _ip]),
    "gw_cell_pairs": (_c_int, [_vp, ctypes.POINTER(ctypes.c_longlong), _ip, ctypes.c_longlong]),
    "gw_polarizability_pairs": (_c_int, [_vp, _vp, _vp, _c_double, _c_int, _vp]),
    "gw_cell_packed_size": (_c_int, [_vp, ctypes.POINTER(ctypes.c_longlong)]),
    "gw_polarizability_packed": (_c_int, [_vp, _vp, _vp, _c_double, _c_int, _vp]),
    "gw_self_energy_packed": (_c_int, [_vp, _vp, _vp, _vp, _c_int, _vp]),
    "gw_fourier_r2k_packed": (_c_int, [_vp, _vp, _c_int, _vp, _c_int, _vp]),
    "gw_fourier_k2r_packed": (_c_int, [_vp, _vp, _c_int, _vp, _c_int, _vp]),
    "gw_drain_packed": (_c_int, [_vp, _vp, _c_int, _c_int, _vp, _c_int, _vp, _c_int, _vp]),
    "gw_self_energy_pairs": (_c_int, [_vp, _vp, _vp, _vp, _c_int, _vp]),
    "gw_polarizability_int": (_c_int, [_vp, _c_int, _vp, _vp, _vp, _vp, _vp, _vp, _c_double, _c_int, _vp]),
    "gw_self_energy_int": (_c_int, [_vp, _c_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _c_int, _vp]),
    "gw_exchange": (_c_int, [_vp, _vp, _vp, _vp, _c_int, _vp]),
    "gw_screened_interaction": (_c_int, [_vp, _vp, _vp, _c_int, _vp, _c_int, _c_int, _c_int, _vp, ctypes.c_size_t,
                                         _vp, _vp]),
    "gw_screened_interaction_workspace": (_c_int, [_vp, _c_int, _c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "gw_green_dyson": (_c_int, [_vp, _vp, _c_double, _c_int, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp, _vp]),
    "gw_green_dyson_workspace": (_c_int, [_vp, _c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "gw_green_dyson_noalloc": (_c_int, [_vp, _vp, _c_double, _c_int, _vp, _vp, _vp, _vp, _vp]),
    "gw_density_omega": (_c_int, [_vp, _vp, _c_int, _vp, _vp, _c_double, _c_double, _vp, _vp]),
    "gw_update_mu": (_c_int, [_vp, _vp, _vp, _vp, _c_int, _c_double, _c_double, _c_double, _c_double, _c_double,
                              _c_int, _vp, _vp, ctypes.c_size_t, _vp, _dp, _dp, _vp]),
    "gw_omega2tau_matrix": (_c_int, [_c_int, _dp, _c_int, _dp, _dp]),
    "gw_green_tau": (_c_int, [_vp, _vp, _c_int, _vp, _vp, _c_double, _c_double, _vp, _vp]),
    "gw_status_string": (ctypes.c_char_p, [_c_int]),
    "gw_last_error": (ctypes.c_char_p, []),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python paper_1911_05633_amd/build.py`")
    # Tensors handed to the library are device pointers of torch's HIP runtime, so the
    # library must bind to that same runtime: torch (which loads its own libamdhip64)
    # goes first, and libgwr's libamdhip64.so.7 dependency then resolves to it instead
    # of loading a second, separately initialised runtime from the system path.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


class GWError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = lib.gw_status_string(status).decode()
        detail = lib.gw_last_error().decode()
        super().__init__(f"{where}: {msg} ({detail})")


def _check(st, where):
    if st != GW_OK:
        raise GWError(st, where)


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.complex128:
        return GW_C128
    if t.dtype == torch.complex64:
        return GW_C64
    raise TypeError(f"expected complex128 or complex64, got {t.dtype}")


def _ptr(t, numel, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


class Cell:
    """Owns a gw_cell handle (constants on the current device)."""

    def __init__(self, species_of_atom, n_orb, n_pb, C, mesh, n_tau, beta, tau):
        species = np.ascontiguousarray(species_of_atom, dtype=np.int32)
        tau = np.ascontiguousarray(tau, dtype=np.float64)
        if tau.shape != (int(n_tau),):
            raise ValueError(f"tau must hold n_tau = {n_tau} points")
        n_orb = np.ascontiguousarray(n_orb, dtype=np.int32)
        n_pb = np.ascontiguousarray(n_pb, dtype=np.int32)
        Cflat = np.ascontiguousarray(np.concatenate([np.asarray(c, dtype=np.float64).ravel() for c in C]))
        mesh = np.ascontiguousarray(mesh, dtype=np.int32)
        h = ctypes.c_void_p()
        st = lib.gw_cell_create(ctypes.byref(h), len(species), species.ctypes.data_as(_ip), len(n_orb),
                                n_orb.ctypes.data_as(_ip), n_pb.ctypes.data_as(_ip), Cflat.ctypes.data_as(_dp),
                                mesh.ctypes.data_as(_ip), int(n_tau), float(beta), tau.ctypes.data_as(_dp))
        _check(st, "gw_cell_create")
        self.handle = h
        self.n_tau = int(n_tau)
        self.beta = float(beta)
        self.mesh = tuple(int(x) for x in mesh)
        self.N_orb = lib.gw_cell_n_orb_total(h)
        self.N_pb = lib.gw_cell_n_pb_total(h)
        self.N_R = lib.gw_cell_n_R(h)

    @classmethod
    def from_spec(cls, spec, C, tau=None):
        """A cell from a description with the attributes species, n_orb, n_pb, mesh, n_tau, beta and
        (unless tau is given) tau."""
        return cls(spec.species, spec.n_orb, spec.n_pb, C, spec.mesh, spec.n_tau, spec.beta,
                   spec.tau if tau is None else tau)

    def tau(self):
        """The cell's tau grid (host copy)."""
        out = np.zeros(self.n_tau, dtype=np.float64)
        _check(lib.gw_cell_tau(self.handle, out.ctypes.data_as(_dp)), "gw_cell_tau")
        return out

    def workspace_bytes(self, prec="fp64"):
        """Device scratch of the path's calls for this cell (gw_workspace_bytes)."""
        p = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        return int(lib.gw_workspace_bytes(self.handle, p))

    def n_basis(self, basis):
        return self.N_orb if basis == 0 else self.N_pb

    def elems(self, basis, lead=None):
        n = self.n_basis(basis)
        return (self.n_tau if lead is None else lead) * self.N_R * n * n

    def set_pairs(self, lattice, positions, r_b, r_c, m_tier):
        """Real-space cutoff and distance tiers (gw_cell_set_pairs); returns the number of
        kept (R, A, B) blocks."""
        lat = np.ascontiguousarray(lattice, dtype=np.float64).reshape(3, 3)
        pos = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1, 3)
        mt = np.ascontiguousarray(m_tier, dtype=np.int32).reshape(-1, 2)
        _check(lib.gw_cell_set_pairs(self.handle, lat.ctypes.data_as(_dp), pos.ctypes.data_as(_dp), float(r_b),
                                     float(r_c), mt.ctypes.data_as(_ip)), "gw_cell_set_pairs")
        return len(self.pairs())

    def packed_elems(self):
        """Elements per tau slice of the packed layout of the kept blocks."""
        n = ctypes.c_longlong()
        _check(lib.gw_cell_packed_size(self.handle, ctypes.byref(n)), "gw_cell_packed_size")
        return n.value

    def pairs(self):
        """The planned blocks as an int array [n][5] = (R, A, B, mA, mB)."""
        n = ctypes.c_longlong()
        _check(lib.gw_cell_pairs(self.handle, ctypes.byref(n), None, 0), "gw_cell_pairs")
        out = np.zeros((n.value, 5), dtype=np.int32)
        _check(lib.gw_cell_pairs(self.handle, ctypes.byref(n), out.ctypes.data_as(_ip), n.value), "gw_cell_pairs")
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib.gw_cell_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gw_fourier_k2r(cell, inp, out, basis=0):
    n = cell.elems(basis)
    _check(lib.gw_fourier_k2r(cell.handle, _ptr(inp, n, "in"), _dtype_code(inp), _ptr(out, n, "out"),
                              _dtype_code(out), basis, _stream()), "gw_fourier_k2r")


def gw_fourier_r2k(cell, inp, out, basis=0):
    n = cell.elems(basis)
    _check(lib.gw_fourier_r2k(cell.handle, _ptr(inp, n, "in"), _dtype_code(inp), _ptr(out, n, "out"),
                              _dtype_code(out), basis, _stream()), "gw_fourier_r2k")


def _prec(prec, t):
    if prec is None:
        return GW_FP64 if _dtype_code(t) == GW_C128 else GW_FP32
    return PRECISIONS[prec] if isinstance(prec, str) else int(prec)


def gw_polarizability(cell, GR, P, spin_factor=2.0, prec=None):
    p = _prec(prec, GR)
    want = GW_C128 if p == GW_FP64 else GW_C64
    if _dtype_code(GR) != want or _dtype_code(P) != want:
        raise TypeError("GR and P must be complex128 for fp64 and complex64 otherwise")
    _check(lib.gw_polarizability(cell.handle, _ptr(GR, cell.elems(0), "GR"), _ptr(P, cell.elems(1), "P"),
                                 float(spin_factor), p, _stream()), "gw_polarizability")


def gw_self_energy(cell, GR, WR, Sigma, prec=None):
    p = _prec(prec, GR)
    want = GW_C128 if p == GW_FP64 else GW_C64
    if _dtype_code(GR) != want or _dtype_code(WR) != want:
        raise TypeError("GR and WR must be complex128 for fp64 and complex64 otherwise")
    if _dtype_code(Sigma) != GW_C128:
        raise TypeError("Sigma is always complex128")
    _check(lib.gw_self_energy(cell.handle, _ptr(GR, cell.elems(0), "GR"), _ptr(WR, cell.elems(1), "WR"),
                              _ptr(Sigma, cell.elems(0), "Sigma"), p, _stream()), "gw_self_energy")


def gw_polarizability_pairs(cell, GR, P, spin_factor=2.0, prec=None):
    p = _prec(prec, GR)
    want = GW_C128 if p == GW_FP64 else GW_C64
    if _dtype_code(GR) != want or _dtype_code(P) != want:
        raise TypeError("GR and P must be complex128 for fp64 and complex64 otherwise")
    _check(lib.gw_polarizability_pairs(cell.handle, _ptr(GR, cell.elems(0), "GR"), _ptr(P, cell.elems(1), "P"),
                                       float(spin_factor), p, _stream()), "gw_polarizability_pairs")


def gw_self_energy_pairs(cell, GR, WR, Sigma, prec=None):
    p = _prec(prec, GR)
    want = GW_C128 if p == GW_FP64 else GW_C64
    if _dtype_code(GR) != want or _dtype_code(WR) != want:
        raise TypeError("GR and WR must be complex128 for fp64 and complex64 otherwise")
    if _dtype_code(Sigma) != GW_C128:
        raise TypeError("Sigma is always complex128")
    _check(lib.gw_self_energy_pairs(cell.handle, _ptr(GR, cell.elems(0), "GR"), _ptr(WR, cell.elems(1), "WR"),
                                    _ptr(Sigma, cell.elems(0), "Sigma"), p, _stream()), "gw_self_energy_pairs")


def gw_polarizability_packed(cell, GR, P, spin_factor=2.0, prec=None):
    """Eq. (5) over the kept blocks, P in the packed layout [n_tau][cell.packed_elems()]."""
    p = _prec(prec, GR)
    want = GW_C128 if p == GW_FP64 else GW_C64
    if _dtype_code(GR) != want or _dtype_code(P) != want:
        raise TypeError("GR and P must be complex128 for fp64 and complex64 otherwise")
    _check(lib.gw_polarizability_packed(cell.handle, _ptr(GR, cell.elems(0), "GR"),
                                        _ptr(P, cell.n_tau * cell.packed_elems(), "P"), float(spin_factor), p,
                                        _stream()), "gw_polarizability_packed")


def gw_self_energy_packed(cell, GR, WR, Sigma, prec=None):
    """Eq. (8) over the kept blocks with W in the packed layout; Sigma dense complex128."""
    p = _prec(prec, GR)
    want = GW_C128 if p == GW_FP64 else GW_C64
    if _dtype_code(GR) != want or _dtype_code(WR) != want:
        raise TypeError("GR and WR must be complex128 for fp64 and complex64 otherwise")
    if _dtype_code(Sigma) != GW_C128:
        raise TypeError("Sigma is always complex128")
    _check(lib.gw_self_energy_packed(cell.handle, _ptr(GR, cell.elems(0), "GR"),
                                     _ptr(WR, cell.n_tau * cell.packed_elems(), "WR"),
                                     _ptr(Sigma, cell.elems(0), "Sigma"), p, _stream()), "gw_self_energy_packed")


def gw_fourier_r2k_packed(cell, inp, out):
    """R -> k of a packed tensor into the dense k-space layout [n_tau][N_k][N_pb][N_pb]."""
    _check(lib.gw_fourier_r2k_packed(cell.handle, _ptr(inp, cell.n_tau * cell.packed_elems(), "in"),
                                     _dtype_code(inp), _ptr(out, cell.elems(1), "out"), _dtype_code(out),
                                     _stream()), "gw_fourier_r2k_packed")


def gw_fourier_k2r_packed(cell, inp, out):
    """k -> R of a dense k-space tensor into the packed layout (kept blocks only)."""
    _check(lib.gw_fourier_k2r_packed(cell.handle, _ptr(inp, cell.elems(1), "in"), _dtype_code(inp),
                                     _ptr(out, cell.n_tau * cell.packed_elems(), "out"), _dtype_code(out),
                                     _stream()), "gw_fourier_k2r_packed")


def gw_drain_packed(cell, T, inp, out, parity=0):
    """R -> k of a packed tensor, then tau -> Matsubara in place on out (max(n_tau, n_omega) rows)."""
    tp, n_omega = _T_ptr(cell, T)
    rows = max(cell.n_tau, n_omega)
    _check(lib.gw_drain_packed(cell.handle, tp, n_omega, int(parity),
                               _ptr(inp, cell.n_tau * cell.packed_elems(), "in"), _dtype_code(inp),
                               _ptr(out, cell.elems(1, rows), "out"), _dtype_code(out), _stream()),
           "gw_drain_packed")


def _T_ptr(cell, T):
    torch = _torch()
    if T.dtype != torch.complex128 or T.dim() != 2 or T.shape[1] != cell.n_tau:
        raise ValueError("T must be a complex128 device matrix [n_omega][n_tau]")
    return _ptr(T, T.numel(), "T"), int(T.shape[0])


def gw_tau2omega(cell, T, inp, out, basis=0, parity=0):
    """parity: 0 (general T), +1 (bosonic) or -1 (fermionic) mirror symmetry of T."""
    tp, n_omega = _T_ptr(cell, T)
    _check(lib.gw_tau2omega(cell.handle, tp, n_omega, int(parity), _ptr(inp, cell.elems(basis), "in"),
                            _dtype_code(inp),
                            _ptr(out, cell.elems(basis, n_omega) if out.data_ptr() != inp.data_ptr()
                                 else out.numel(), "out"),
                            _dtype_code(out), basis, _stream()), "gw_tau2omega")


def gw_drain(cell, T, inp, out, basis=1, parity=0):
    """parity: 0 (general T), +1 (bosonic) or -1 (fermionic) mirror symmetry of T."""
    tp, n_omega = _T_ptr(cell, T)
    _check(lib.gw_drain(cell.handle, tp, n_omega, int(parity), _ptr(inp, cell.elems(basis), "in"),
                        _dtype_code(inp),
                        _ptr(out, cell.elems(basis, n_omega) if out.data_ptr() != inp.data_ptr()
                             else out.numel(), "out"),
                        _dtype_code(out), basis, _stream()), "gw_drain")


def gw_density(cell, G, spin_factor, n_out, space=0):
    """space 0: G is G^R(tau); space 1: G is G(k, tau)."""
    torch = _torch()
    if n_out.dtype != torch.float64 or n_out.numel() != 1:
        raise ValueError("n_out must be a one-element float64 device tensor")
    _check(lib.gw_density(cell.handle, _ptr(G, cell.elems(0), "G"), _dtype_code(G), int(space),
                          float(spin_factor), _ptr(n_out, 1, "n_out"), _stream()), "gw_density")


def gw_tau2omega_matrix(tau, omega):
    """Host FP64 matrix T[n_omega][n_tau] (numpy complex128)."""
    tau = np.ascontiguousarray(tau, dtype=np.float64)
    omega = np.ascontiguousarray(omega, dtype=np.float64)
    out = np.zeros((len(omega), len(tau)), dtype=np.complex128)
    _check(lib.gw_tau2omega_matrix(len(tau), tau.ctypes.data_as(_dp), len(omega), omega.ctypes.data_as(_dp),
                                   out.ctypes.data_as(_dp)), "gw_tau2omega_matrix")
    return out


def _int_blocks(cell, n_g, tensors, rows, names):
    bl = cell.n_tau * cell.N_R
    code = _dtype_code(tensors[0])
    ptrs = []
    for t, r, name in zip(tensors, rows, names):
        if _dtype_code(t) != code:
            raise TypeError("all interstitial blocks must share one dtype")
        ptrs.append(_ptr(t, bl * r * n_g, name))
    return ptrs, code


def gw_polarizability_int(cell, G_og, G_go, G_gg, P_pg, P_gp, P_gg, spin_factor=2.0):
    """Interstitial blocks of P (Eqs. (6), (7)); n_g is read from G_gg's last axis."""
    n_g = int(G_gg.shape[-1])
    ptrs, code = _int_blocks(cell, n_g, [G_og, G_go, G_gg, P_pg, P_gp, P_gg],
                             [cell.N_orb, cell.N_orb, n_g, cell.N_pb, cell.N_pb, n_g],
                             ["G_og", "G_go", "G_gg", "P_pg", "P_gp", "P_gg"])
    _check(lib.gw_polarizability_int(cell.handle, n_g, *ptrs, float(spin_factor), code, _stream()),
           "gw_polarizability_int")


def gw_self_energy_int(cell, G_og, G_go, G_gg, W_pg, W_gp, W_gg, S_og, S_go, S_gg):
    """Interstitial blocks of Sigma (Eqs. (9), (10)); Sigma blocks complex128."""
    n_g = int(G_gg.shape[-1])
    ptrs, code = _int_blocks(cell, n_g, [G_og, G_go, G_gg, W_pg, W_gp, W_gg],
                             [cell.N_orb, cell.N_orb, n_g, cell.N_pb, cell.N_pb, n_g],
                             ["G_og", "G_go", "G_gg", "W_pg", "W_gp", "W_gg"])
    bl = cell.n_tau * cell.N_R
    outs = []
    for t, r, name in zip([S_og, S_go, S_gg], [cell.N_orb, cell.N_orb, n_g], ["S_og", "S_go", "S_gg"]):
        if _dtype_code(t) != GW_C128:
            raise TypeError("Sigma blocks are complex128")
        outs.append(_ptr(t, bl * r * n_g, name))
    _check(lib.gw_self_energy_int(cell.handle, n_g, *ptrs, *outs, code, _stream()), "gw_self_energy_int")


def gw_exchange(cell, GR, VR, Sigma_x, prec=None):
    """Static self-energy Sigma_x^R = + C G^R(beta^-) V^R C (Sigma_x: complex128 [N_R][N_orb][N_orb])."""
    p = _prec(prec, GR)
    want = GW_C128 if p == GW_FP64 else GW_C64
    if _dtype_code(GR) != want or _dtype_code(VR) != want:
        raise TypeError("GR and VR must be complex128 for fp64 and complex64 otherwise")
    if _dtype_code(Sigma_x) != GW_C128:
        raise TypeError("Sigma_x is always complex128")
    _check(lib.gw_exchange(cell.handle, _ptr(GR, cell.elems(0), "GR"), _ptr(VR, cell.elems(1, 1), "VR"),
                           _ptr(Sigma_x, cell.elems(0, 1), "Sigma_x"), p, _stream()), "gw_exchange")


def gw_screened_interaction_workspace(cell, chunk=1, prec="fp64"):
    """Workspace bytes for `chunk` (q, nu) matrices per launch at precision prec."""
    b = ctypes.c_size_t()
    p = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    _check(lib.gw_screened_interaction_workspace(cell.handle, int(chunk), p, ctypes.byref(b)),
           "gw_screened_interaction_workspace")
    return b.value


def gw_screened_interaction(cell, V, P, W, work, info=None, prec="fp64"):
    """W~(q, nu) = (I - V(q) P(q, nu))^-1 V(q) - V(q) for P of shape [n_omega][N_k][N_pb][N_pb].

    V: complex128 device [N_k][N_pb][N_pb]; work: a device tensor (any dtype) used as scratch;
    info: optional int32 device tensor of one element (see the header)."""
    torch = _torch()
    n = cell.N_pb
    per = cell.N_R * n * n
    if P.numel() % per or P.numel() == 0:
        raise ValueError("P must hold n_omega * N_k * N_pb^2 elements")
    n_omega = P.numel() // per
    if V.dtype != torch.complex128:
        raise TypeError("V must be complex128")
    if not work.is_cuda or not work.is_contiguous():
        raise ValueError("work must be a contiguous device tensor")
    ip = None
    if info is not None:
        if info.dtype != torch.int32 or info.numel() != 1:
            raise ValueError("info must be a one-element int32 device tensor")
        ip = _ptr(info, 1, "info")
    p = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    _check(lib.gw_screened_interaction(cell.handle, _ptr(V, per, "V"), _ptr(P, P.numel(), "P"), _dtype_code(P),
                                       _ptr(W, P.numel(), "W"), _dtype_code(W), n_omega, p,
                                       ctypes.c_void_p(work.data_ptr()), work.numel() * work.element_size(), ip,
                                       _stream()), "gw_screened_interaction")


def gw_green_dyson_workspace(cell, chunk=1):
    """Workspace bytes of gw_green_dyson for `chunk` (k, w) matrices per launch."""
    b = ctypes.c_size_t()
    _check(lib.gw_green_dyson_workspace(cell.handle, int(chunk), ctypes.byref(b)), "gw_green_dyson_workspace")
    return b.value


def gw_green_dyson(cell, Hk, mu, G, work, Sigma=None, Sigma_x=None, info=None):
    """G(k, i w_m) = [(i w_m + mu) - H(k) - Sigma_x(k) - Sigma(k, i w_m)]^-1; G: complex128
    [n_omega][N_k][N_orb][N_orb] (n_omega taken from its size)."""
    torch = _torch()
    per = cell.N_R * cell.N_orb * cell.N_orb
    if G.numel() % per or G.numel() == 0:
        raise ValueError("G must hold n_omega * N_k * N_orb^2 elements")
    n_omega = G.numel() // per
    for t, name in ((Hk, "Hk"), (G, "G"), (Sigma, "Sigma"), (Sigma_x, "Sigma_x")):
        if t is not None and t.dtype != torch.complex128:
            raise TypeError(f"{name} must be complex128")
    if not work.is_cuda or not work.is_contiguous():
        raise ValueError("work must be a contiguous device tensor")
    ip = None
    if info is not None:
        if info.dtype != torch.int32 or info.numel() != 1:
            raise ValueError("info must be a one-element int32 device tensor")
        ip = _ptr(info, 1, "info")
    _check(lib.gw_green_dyson(cell.handle, _ptr(Hk, per, "Hk"), float(mu), n_omega,
                              None if Sigma is None else _ptr(Sigma, G.numel(), "Sigma"),
                              None if Sigma_x is None else _ptr(Sigma_x, per, "Sigma_x"),
                              _ptr(G, G.numel(), "G"), ctypes.c_void_p(work.data_ptr()),
                              work.numel() * work.element_size(), ip, _stream()), "gw_green_dyson")


GREEN_NOALLOC_SCRATCH_BYTES = 64 << 20  # the library's static scratch of gw_green_dyson_noalloc


def gw_green_dyson_noalloc(cell, Hk, mu, G, Sigma=None, Sigma_x=None, info=None):
    """gw_green_dyson with the library's static device scratch instead of a workspace argument
    (for callers that cannot allocate); same arguments otherwise.  Calls that overlap in time
    on one GPU race."""
    torch = _torch()
    per = cell.N_R * cell.N_orb * cell.N_orb
    if G.numel() % per or G.numel() == 0:
        raise ValueError("G must hold n_omega * N_k * N_orb^2 elements")
    n_omega = G.numel() // per
    for t, name in ((Hk, "Hk"), (G, "G"), (Sigma, "Sigma"), (Sigma_x, "Sigma_x")):
        if t is not None and t.dtype != torch.complex128:
            raise TypeError(f"{name} must be complex128")
    ip = None
    if info is not None:
        if info.dtype != torch.int32 or info.numel() != 1:
            raise ValueError("info must be a one-element int32 device tensor")
        ip = _ptr(info, 1, "info")
    _check(lib.gw_green_dyson_noalloc(cell.handle, _ptr(Hk, per, "Hk"), float(mu), n_omega,
                                      None if Sigma is None else _ptr(Sigma, G.numel(), "Sigma"),
                                      None if Sigma_x is None else _ptr(Sigma_x, per, "Sigma_x"),
                                      _ptr(G, G.numel(), "G"), ip, _stream()), "gw_green_dyson_noalloc")


def gw_density_omega(cell, G, Hk, mu, spin_factor, n_out, Sigma_x=None):
    """Electron count of G at the first n_omega fermionic frequencies (written to n_out)."""
    per = cell.N_R * cell.N_orb * cell.N_orb
    n_omega = G.numel() // per
    _check(lib.gw_density_omega(cell.handle, _ptr(G, n_omega * per, "G"), n_omega, _ptr(Hk, per, "Hk"),
                                None if Sigma_x is None else _ptr(Sigma_x, per, "Sigma_x"), float(mu),
                                float(spin_factor), _ptr(n_out, 1, "n_out"), _stream()), "gw_density_omega")


def gw_update_mu(cell, Hk, G, work, n_dev, spin_factor, n_target, mu_lo, mu_hi, tol=1e-10, max_iter=100,
                 Sigma=None, Sigma_x=None):
    """Regula falsi (Illinois) on mu; returns (mu, count).  G: complex128 [n_omega][N_k][N_orb][N_orb]
    scratch that ends holding the Dyson solution at mu."""
    per = cell.N_R * cell.N_orb * cell.N_orb
    n_omega = G.numel() // per
    mu, n = ctypes.c_double(), ctypes.c_double()
    _check(lib.gw_update_mu(cell.handle, _ptr(Hk, per, "Hk"), None if Sigma is None else _ptr(Sigma, G.numel(), "Sigma"),
                            None if Sigma_x is None else _ptr(Sigma_x, per, "Sigma_x"), n_omega, float(spin_factor),
                            float(n_target), float(mu_lo), float(mu_hi), float(tol), int(max_iter),
                            _ptr(G, G.numel(), "G"), ctypes.c_void_p(work.data_ptr()),
                            work.numel() * work.element_size(), _ptr(n_dev, 1, "n_dev"), ctypes.byref(mu),
                            ctypes.byref(n), _stream()), "gw_update_mu")
    return mu.value, n.value


def gw_green_tau(cell, G, Hk, mu, G_tau, Sigma_x=None, mix=1.0):
    """G(k, tau) on the cell's grid from G(k, i w_m) (complex128 [n_omega][N_k][N_orb][N_orb]) by the
    Matsubara sum with the 1 / (i w) and 1 / (i w)^2 tails in closed form; G_tau: complex128
    [n_tau][N_k][N_orb][N_orb], set to mix G(tau) + (1 - mix) G_tau."""
    torch = _torch()
    per = cell.N_R * cell.N_orb * cell.N_orb
    if G.numel() % per or G.numel() == 0:
        raise ValueError("G must hold n_omega * N_k * N_orb^2 elements")
    for t, name in ((G, "G"), (Hk, "Hk"), (G_tau, "G_tau"), (Sigma_x, "Sigma_x")):
        if t is not None and t.dtype != torch.complex128:
            raise TypeError(f"{name} must be complex128")
    _check(lib.gw_green_tau(cell.handle, _ptr(G, G.numel(), "G"), G.numel() // per, _ptr(Hk, per, "Hk"),
                            None if Sigma_x is None else _ptr(Sigma_x, per, "Sigma_x"), float(mu), float(mix),
                            _ptr(G_tau, cell.n_tau * per, "G_tau"), _stream()), "gw_green_tau")


def gw_omega2tau_matrix(tau, omega):
    """Host FP64 inverse of gw_tau2omega_matrix(tau, omega) (numpy complex128 [n_tau][n_tau])."""
    tau = np.ascontiguousarray(tau, dtype=np.float64)
    omega = np.ascontiguousarray(omega, dtype=np.float64)
    out = np.zeros((len(tau), len(tau)), dtype=np.complex128)
    _check(lib.gw_omega2tau_matrix(len(tau), tau.ctypes.data_as(_dp), len(omega), omega.ctypes.data_as(_dp),
                                   out.ctypes.data_as(_dp)), "gw_omega2tau_matrix")
    return out


def matsubara(n, beta, kind):
    """First n Matsubara frequencies: bosonic 2 pi m / beta or fermionic (2m + 1) pi / beta."""
    m = np.arange(n, dtype=np.float64)
    return (2.0 * m if kind == "bosonic" else 2.0 * m + 1.0) * np.pi / beta
