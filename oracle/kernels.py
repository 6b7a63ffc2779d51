"""Dense pair kernels Phi_ij and G_ij = -grad_{x_i} Phi(x_i - x_j) (oracle, small N).

Open boundaries: Phi_ij = 1/|x_i - x_j| for i != j and Phi_ii = 0 (eq
nbody_periodic without box shifts; the primed sum drops i = j).
Periodic cube: Phi_ij = phi_EW(x_i - x_j), the Ewald sum over all box shifts
with tin-foil boundaries and a neutralising background; Phi_ii is the sum over
the self images only (eq nbody_periodic keeps i = j when n != 0).
"""
from __future__ import annotations

import numpy as np

from . import ewald


def open_dense(x):
    x = np.asarray(x, dtype=np.float64)
    d = x[:, None, :] - x[None, :, :]
    r2 = np.einsum("ijk,ijk->ij", d, d)
    np.fill_diagonal(r2, 1.0)
    rinv = 1.0 / np.sqrt(r2)
    np.fill_diagonal(rinv, 0.0)
    G = d * (rinv ** 3)[:, :, None]
    return rinv, G


def periodic_dense(x, L: float):
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    d = (x[:, None, :] - x[None, :, :]).reshape(-1, 3)
    phi, G = ewald.pair(d, L)
    return phi.reshape(n, n), G.reshape(n, n, 3)


def dense(sys_x, periodic: bool, L: float):
    return periodic_dense(sys_x, L) if periodic else open_dense(sys_x)
