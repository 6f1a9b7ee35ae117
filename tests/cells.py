"""Small cells used by the tests (built from the seeded input generators)."""
import numpy as np

import synthcell as sc


def tiny(n_tau=16, beta=50.0, mesh=(2, 2, 2), complex_hopping=False, request_id=0):
    s = sc.tiny_cell(1, request_id, n_tau=n_tau, beta=beta, mesh=mesh)
    s.complex_hopping = complex_hopping
    return s


def two_species(mesh=(3, 2, 1), n_tau=8, beta=20.0, complex_hopping=True, n_orb=(3, 2), n_pb=(5, 4),
                request_id=7):
    """Three atoms, two species, uneven blocks, odd mesh."""
    lat = np.array([[3.1, 0.0, 0.0], [0.4, 2.9, 0.0], [0.0, 0.3, 3.3]])
    pos = np.array([[0.0, 0.0, 0.0], [1.2, 1.1, 1.4], [2.0, 0.4, 2.5]])
    species = np.array([0, 1, 0], dtype=np.int64)
    return sc.CellSpec("two_species", lat, pos, species, tuple(n_orb), tuple(n_pb), tuple(mesh), n_tau,
                       beta, config_id=11, request_id=request_id, complex_hopping=complex_hopping)


def inputs(spec):
    hop = sc.hoppings(spec)
    b = sc.bands(spec, hop)
    Gk = sc.green_ktau(spec, b)
    C = sc.coefficients(spec)
    return hop, b, Gk, C
