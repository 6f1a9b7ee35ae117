"""Born-von Karman mesh bookkeeping for the oracle (test infrastructure).

The R-list of the paper (Sec. 2, the sphere R_max of Fig. 1) is taken to be
every translation of the k-mesh's supercell; -R is taken modulo the mesh.
"""
import numpy as np


def mesh_points(mesh):
    """All (n1, n2, n3) with 0 <= n_i < N_i, index (n1 * N2 + n2) * N3 + n3."""
    N1, N2, N3 = mesh
    out = []
    for a in range(N1):
        for b in range(N2):
            for c in range(N3):
                out.append((a, b, c))
    return np.array(out, dtype=np.int64)


def kr_phase(mesh, sign):
    """Matrix E[k, R] = exp(sign * 2 pi i sum_i j_i n_i / N_i)."""
    pts = mesh_points(mesh)
    frac = pts / np.array(mesh, dtype=float)  # k in reduced units
    arg = 2.0 * np.pi * (frac @ pts.T.astype(float))  # [k, R]
    return np.exp(sign * 1j * arg)


def minus_index(mesh):
    """Index of -R (mod mesh) for every R."""
    pts = mesh_points(mesh)
    N = np.array(mesh)
    neg = (-pts) % N
    return (neg[:, 0] * mesh[1] + neg[:, 1]) * mesh[2] + neg[:, 2]


def k_minus_q_index(mesh):
    """Table D[k, q] = index of k - q (mod mesh)."""
    pts = mesh_points(mesh)
    N = np.array(mesh)
    d = (pts[:, None, :] - pts[None, :, :]) % N
    return (d[..., 0] * mesh[1] + d[..., 1]) * mesh[2] + d[..., 2]
